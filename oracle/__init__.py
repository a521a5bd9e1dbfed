"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct CPU implementation of what the homomorphic
convolution / average-pooling path computes (RNS-CKKS arithmetic in
`ckks_oracle.c`, the layer schedule of the paper's Section 4 in
`he_layers.py`, and an FP64 slot simulator that runs the same schedule on
cleartext slot vectors).  Only `tests/`, `__graft_entry__.smoke()` and the
`cpu_baseline` leg of `bench.py` may import anything from this package.  It
shares no code with the GPU library in `paper_2306_09189_amd/`.

Parity unpinned: none of the functions here is left without a pin; the one
place where two correct implementations may legitimately differ -- the last
bit of a rounding in the encoder -- is pinned to the exact real value instead
(tests/test_oracle_encode.py).
"""
