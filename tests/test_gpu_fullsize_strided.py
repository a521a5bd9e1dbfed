"""The benchmark's strided stage at the full ring (2N = 2^16, q_0 60-bit +
24 x 50-bit, 8 x 60-bit special primes, dnum = 3, scale 2^50), bit-exact with
the oracle, in every evaluation mode the benchmark can run.

An image of 32x32 channels at the benchmark's block size goes through a
3x3 stride-2 convolution into 64 channels: the unstrided output fills two
ciphertexts (Section 4.1, "With Image Shards"), each is downsampled by the
horizontal and vertical masked reductions (Section 4.2), the two are
consolidated into one and duplicated twice (Section 4.2, consolidation and
duplication).  The input has 8 channels (each held four times), so the
plan has 8 block offsets x 9 taps instead of the benchmark's 32 x 9: the
same kernels, launch shapes and output count, with a rotation-key set the
oracle can generate in about a minute.  The oracle's keys cover Q_3 and P
only (the input starts at level 3 and ends at level 0)."""
import numpy as np
import pytest

from checks import log, run_pipeline
from oracle import ckks
from oracle import he_layers as hl

pytestmark = pytest.mark.gpu

LOGN, L, Q0, QB, K, PB, DNUM, LS = 16, 24, 60, 50, 8, 60, 3, 50
LEVEL = 3


@pytest.fixture(scope="module")
def full_low():
    from paper_2306_09189_amd import hecnn
    log("2^16 context")
    ctx = hecnn.Context(LOGN, L, Q0, QB, K, PB, DNUM, LS, device=0)
    prm = ckks.Params(LOGN, [Q0] + [QB] * L, [PB] * K, DNUM)
    assert ctx.primes() == prm.mod
    ctx.keygen(2012)
    return ctx, prm, ckks.Oracle(prm, 2012, key_level=LEVEL)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("mode", [0, 2, 3])
def test_strided_two_shard_pipeline_bit_exact(full_low, mode):
    ctx, prm, o = full_low
    rng = np.random.default_rng(1012)
    x = rng.uniform(-1, 1, (8, 32, 32))
    w = rng.normal(0, 0.05, (64, 8, 3, 3))
    lay = hl.natural_layout(prm.N, 8, 32, 32)
    assert len(lay.shards) == 1 and lay.shards[0][:8] == [0, 0, 0, 0, 1, 1, 1, 1]
    log("strided 8 -> 64, mode %d" % mode)
    got = run_pipeline(ctx, prm, o, x, [("conv", w, 2)], LEVEL, seed=3012, mode=mode)
    assert got.shape == (64, 16, 16)
