"""MI355X (gfx950) library for homomorphic convolution and average pooling on
RNS-CKKS ciphertexts (arXiv 2306.09189, Section 4), behind the C ABI in
include/hecnn.h.  `hecnn` is the thin ctypes binding."""
from . import hecnn  # noqa: F401
