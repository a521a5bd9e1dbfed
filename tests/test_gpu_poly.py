"""Ciphertext products, constants and the Chebyshev evaluator of the GPU
library vs the CPU oracle (MI355X, through the C ABI): bit-exact on a small
ring at several levels and degrees, decryption accuracy at n = 2^16."""
import sys

import numpy as np
import pytest
from numpy.polynomial import chebyshev as C

from oracle import ckks
from oracle import he_layers as hl

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gelu(x):
    return 0.5 * x * (1.0 + np.tanh(np.sqrt(2.0 / np.pi) * (x + 0.044715 * x ** 3)))


@pytest.fixture(scope="module")
def deep():
    from paper_2306_09189_amd import hecnn
    log("ctx logn=10 L=12 k=4 dnum=4")
    ctx = hecnn.Context(10, 12, 60, 40, 4, 60, 4, 40, device=0)
    prm = ckks.Params(10, [60] + [40] * 12, [60] * 4, 4)
    ctx.keygen(11)
    return ctx, prm, ckks.Oracle(prm, 11)


def enc_pair(ctx, o, lvl, seed, scale=2.0 ** 40):
    rng = np.random.default_rng(seed)
    z1, z2 = rng.uniform(-1, 1, o.p.N), rng.uniform(-1, 1, o.p.N)
    a = o.encrypt(o.encode(z1, lvl, scale), seed=seed)
    b = o.encrypt(o.encode(z2, lvl, scale), seed=seed + 100, index=1)
    return a, b, ctx.ct_import(a.data, lvl, a.scale), ctx.ct_import(b.data, lvl, b.scale)


@pytest.mark.parametrize("lvl", [12, 8, 5, 3, 0])
def test_mul_ct_bit_exact(deep, lvl):
    """Relinearized product: every digit count (beta = 4 .. 1), level 0 included."""
    ctx, prm, o = deep
    log("mul_ct level", lvl)
    a, b, ga, gb = enc_pair(ctx, o, lvl, 20 + lvl)
    ref = o.mul_ct(a, b)
    g = ctx.mul(ga, gb)
    assert g.level == lvl and g.scale == ref.scale
    assert (g.export() == ref.data).all()
    # a square (both operands the same handle)
    assert (ctx.mul(ga, ga).export() == o.mul_ct(a, a).data).all()


def test_mul_counts_one_keyswitch(deep):
    ctx, prm, o = deep
    a, b, ga, gb = enc_pair(ctx, o, 4, 3)
    k0 = ctx.keyswitch_count()
    ctx.mul(ga, gb)
    assert ctx.keyswitch_count() - k0 == 1


@pytest.mark.parametrize("value,pscale", [
    (1.5, None), (-0.3, None), (0.0, None), (1.0, 2.0 ** 40), (-1.0, 2.0 ** 40), (1e-9, 2.0 ** 40),
    (0.5, 3.0), (-0.5, 3.0), (2.5, 1.0), (-2.5, 1.0), (1e-300, 2.0 ** 40), (3.0e6, 2.0 ** 40)])
def test_constants_bit_exact(deep, value, pscale):
    """Constant products and sums, including exact ties (rounded away from zero),
    zero, subnormal-range products and constants near 2^62."""
    ctx, prm, o = deep
    lvl = 6
    a, b, ga, gb = enc_pair(ctx, o, lvl, 40)
    ps = float(prm.q[lvl]) if pscale is None else pscale
    ref = o.mul_const(a, value, ps)
    g = ctx.mul_const(ga, value, ps)
    assert g.scale == ref.scale and (g.export() == ref.data).all()
    ref = o.add_const(a, value)
    g = ctx.add_const(ga, value)
    assert g.scale == ref.scale and (g.export() == ref.data).all()


def test_constant_range_rejected(deep):
    from paper_2306_09189_amd import hecnn
    ctx, prm, o = deep
    a, b, ga, gb = enc_pair(ctx, o, 3, 41)
    with pytest.raises(hecnn.HecError):
        ctx.mul_const(ga, 2.0 ** 23, 2.0 ** 40)     # 2^63
    with pytest.raises(hecnn.HecError):
        ctx.mul_const(ga, float("nan"), 2.0 ** 40)
    g = ctx.mul_const(ga, 2.0 ** 21 - 1.0, 2.0 ** 40)  # just under 2^61
    assert (g.export() == o.mul_const(a, 2.0 ** 21 - 1.0, 2.0 ** 40).data).all()


def test_sub_drop_bit_exact(deep):
    ctx, prm, o = deep
    a, b, ga, gb = enc_pair(ctx, o, 7, 42)
    assert (ctx.sub(ga, gb).export() == o.sub(a, b).data).all()
    assert (ctx.drop(ga, 3).export() == o.drop_to(a, 3).data).all()
    assert (ctx.drop(ga, 7).export() == a.data).all()
    from paper_2306_09189_amd import hecnn
    with pytest.raises(hecnn.HecError):
        ctx.drop(ga, 8)


@pytest.mark.parametrize("deg", [1, 2, 3, 7, 16, 27, 59, 100])
def test_cheb_eval_bit_exact(deep, deg):
    """ChebEval on a GELU interpolant over [-8, 8]: every ciphertext bit equal to
    the oracle's, nominal scale and level equal, decryption within 1e-5 of FP64.
    Up to degree 63 the baby steps are 8 (leaf sums of at most 7 terms, one
    fused launch each); degree 100 takes 16 (sums of up to 15 terms, taken one
    constant product at a time)."""
    ctx, prm, o = deep
    a, b = -8.0, 8.0
    coef = C.chebinterpolate(lambda y: gelu((b - a) / 2 * y + (a + b) / 2), deg)
    if deg == 2:
        coef = np.array([0.25, 0.0, -0.5])     # only an even term: lin of a single T_2
    z = np.random.default_rng(deg).uniform(-6, 6, prm.N)
    ct = o.encrypt(o.encode(z, 12, 2.0 ** 40), seed=50 + deg)
    log("cheb deg", deg)
    ref = hl.ChebEval(hl.CkksBackend(o), ct, a, b).run(coef)
    g = ctx.cheb_eval(ctx.ct_import(ct.data, 12, ct.scale), coef, a, b)
    assert g.level == ref.level and g.scale == ref.scale
    assert (g.export() == ref.data).all()
    assert np.abs(ctx.decrypt(g) - hl.ref_cheb(z, coef, a, b)).max() < 1e-5


@pytest.mark.parametrize("deg,depth", [(59, 6), (27, 5)])
def test_cheb_eval_unit_interval_bit_exact(deep, deg, depth):
    """On [-1, 1] (map folded into the previous layer): the paper's depths, bits
    equal to the oracle's."""
    ctx, prm, o = deep
    coef = C.chebinterpolate(lambda y: gelu(8.0 * y), deg)
    z = np.random.default_rng(deg + 7).uniform(-1, 1, prm.N)
    ct = o.encrypt(o.encode(z, 12, 2.0 ** 40), seed=80 + deg)
    ref = hl.ChebEval(hl.CkksBackend(o), ct, -1.0, 1.0).run(coef)
    g = ctx.cheb_eval(ctx.ct_import(ct.data, 12, ct.scale), coef, -1.0, 1.0)
    assert 12 - g.level == depth and g.level == ref.level and g.scale == ref.scale
    assert (g.export() == ref.data).all()
    assert np.abs(ctx.decrypt(g) - hl.ref_cheb(z, coef, -1.0, 1.0)).max() < 1e-5


def test_cheb_eval_errors(deep):
    from paper_2306_09189_amd import hecnn
    ctx, prm, o = deep
    z = np.random.default_rng(5).uniform(-1, 1, prm.N)
    ct = o.encrypt(o.encode(z, 2, 2.0 ** 40), seed=60)
    g = ctx.ct_import(ct.data, 2, ct.scale)
    with pytest.raises(hecnn.HecError):          # degree 0
        ctx.cheb_eval(g, [1.0], -1.0, 1.0)
    with pytest.raises(hecnn.HecError):          # empty interval
        ctx.cheb_eval(g, [0.0, 1.0], 1.0, 1.0)
    with pytest.raises(hecnn.HecError):          # constant after division
        ctx.cheb_eval(g, [1.0, 0.0, 0.0], -1.0, 1.0)
    with pytest.raises(hecnn.HecError):          # degree 59 needs 7 levels
        ctx.cheb_eval(g, np.ones(60), -1.0, 1.0)


def test_image_cheb_eval_bit_exact(deep):
    """Every shard of a sharded image evaluated; bits equal to the oracle's per shard."""
    ctx, prm, o = deep
    x = np.random.default_rng(9).uniform(-6, 6, (4, 16, 16))
    img = ctx.image_encrypt(x, 12, 77)
    coef = C.chebinterpolate(lambda y: gelu(8.0 * y), 15)
    out = ctx.cheb_eval(img, coef, -8.0, 8.0)
    nsh = img.info()[-1]
    assert nsh >= 2 and out.info() == img.info()
    for u in range(nsh):
        lvl, sc = img.shard_info(u)
        ref = hl.ChebEval(hl.CkksBackend(o), ckks.Ct(img.shard_export(u), lvl, sc), -8.0, 8.0).run(coef)
        assert out.shard_info(u) == (ref.level, ref.scale)
        assert (out.shard_export(u) == ref.data).all(), u
    dec = out.decrypt()
    assert np.abs(dec - hl.ref_cheb(x, coef, -8.0, 8.0)).max() < 1e-5
