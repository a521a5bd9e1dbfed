"""The allocation-free rotation (ckks_rotate_noalloc) against ckks_rotate,
through the C ABI on the GPU: bit for bit on two calls in a row, the second
with a smaller input (lower level, fewer limbs), at the full ring 2N = 2^16
(level 20, the benchmark's) and on a small ring; a rotation whose
temporaries exceed the scratch array is refused with HEC_EINVAL; a level
mismatch with HEC_ELEVEL; a missing key with HEC_ENOKEY."""
import numpy as np
import pytest

from checks import log

pytestmark = pytest.mark.gpu


def zeros_ct(ctx, level):
    coeff = np.zeros((2, level + 1, ctx.n), dtype=np.uint64)
    return ctx.ct_import(coeff, level, 1.0)


@pytest.mark.parametrize("logn,L,k,dnum,levels", [(16, 24, 8, 3, (20, 4)), (12, 6, 2, 3, (6, 2))])
def test_rotate_noalloc_matches_rotate(logn, L, k, dnum, levels):
    from paper_2306_09189_amd import hecnn
    qb = 50 if logn == 16 else 40
    ctx = hecnn.Context(logn, L, 60, qb, k, 60, dnum, qb, device=0)
    ctx.keygen(5)
    steps = [1, 3, -7]
    ctx.gen_rotation_keys(steps)
    rng = np.random.default_rng(logn)
    z = rng.uniform(-1, 1, ctx.N)
    for lvl in levels:
        log("logn %d level %d" % (logn, lvl))
        ct = ctx.encrypt(ctx.encode(z, lvl, 2.0 ** qb), seed=7, index=lvl)
        for s in steps + [0]:
            out = zeros_ct(ctx, lvl)
            ctx.rotate_noalloc(ct, s, out)
            ref = ctx.rotate(ct, s)
            assert (out.export() == ref.export()).all(), (lvl, s)
            assert out.info() == ref.info()
        assert np.abs(ctx.decrypt(out) - z).max() < 1e-6
    ct = ctx.encrypt(ctx.encode(z, levels[0], 2.0 ** qb), seed=8)
    with pytest.raises(hecnn.HecError) as e:
        ctx.rotate_noalloc(ct, 1, zeros_ct(ctx, levels[1]))
    assert e.value.status == hecnn.HEC_ELEVEL
    with pytest.raises(hecnn.HecError) as e:
        ctx.rotate_noalloc(ct, 2, zeros_ct(ctx, levels[0]))
    assert e.value.status == hecnn.HEC_ENOKEY


def test_rotate_noalloc_beyond_scratch():
    from paper_2306_09189_amd import hecnn
    # 2^16 with 31 ciphertext primes and 8 special primes: a rotation at level
    # 30 needs 288 limbs of 512 KiB (144 MiB) of temporaries
    ctx = hecnn.Context(16, 30, 60, 50, 8, 60, 3, 50, device=0)
    ctx.keygen(6)
    ctx.gen_rotation_keys([1])
    z = np.zeros(8)
    ct = ctx.encrypt(ctx.encode(z, 30, 2.0 ** 50), seed=1)
    with pytest.raises(hecnn.HecError) as e:
        ctx.rotate_noalloc(ct, 1, zeros_ct(ctx, 30))
    assert e.value.status == hecnn.HEC_EINVAL
    ct4 = ctx.encrypt(ctx.encode(z, 4, 2.0 ** 50), seed=1)
    out = zeros_ct(ctx, 4)
    ctx.rotate_noalloc(ct4, 1, out)
    assert (out.export() == ctx.rotate(ct4, 1).export()).all()
