"""Ciphertext products with relinearization, constants and the Chebyshev
evaluator of the encrypted oracle (CPU only)."""
import numpy as np
import pytest
from numpy.polynomial import chebyshev as C

from oracle import ckks
from oracle import he_layers as hl


@pytest.fixture(scope="module")
def deep():
    p = ckks.Params(8, [60] + [40] * 12, [60, 60, 60, 60], 4)
    return p, ckks.Oracle(p, 9)


def gelu(x):
    return 0.5 * x * (1.0 + np.tanh(np.sqrt(2.0 / np.pi) * (x + 0.044715 * x ** 3)))


def test_mul_ct_relinearized(deep):
    """The relinearized product decrypts to z1 * z2, and c0 + c1 s differs from
    the unrelinearized d0 + d1 s + d2 s^2 by key-switching noise only (a wrong
    relinearization key or gadget would leave an error of the order of q)."""
    p, o = deep
    rng = np.random.default_rng(1)
    z1, z2 = rng.uniform(-1, 1, p.N), rng.uniform(-1, 1, p.N)
    lvl = 8
    a = o.encrypt(o.encode(z1, lvl, 2.0 ** 40), seed=1)
    b = o.encrypt(o.encode(z2, lvl, 2.0 ** 40), seed=2, index=1)
    c = o.mul_ct(a, b)
    assert c.scale == 2.0 ** 80 and c.level == lvl
    assert np.abs(o.decrypt(o.rescale(c)) - z1 * z2).max() < 1e-6
    qi = list(range(lvl + 1))
    s = o.limbs_of(o.s, lvl)
    d0 = o.mul_limbs(qi, a.data[0], b.data[0])
    d1 = o.add_limbs(qi, o.mul_limbs(qi, a.data[0], b.data[1]), o.mul_limbs(qi, a.data[1], b.data[0]))
    d2 = o.mul_limbs(qi, a.data[1], b.data[1])
    full = o.add_limbs(qi, o.add_limbs(qi, d0, o.mul_limbs(qi, d1, s)), o.mul_limbs(qi, d2, o.mul_limbs(qi, s, s)))
    relin = o.add_limbs(qi, c.data[0], o.mul_limbs(qi, c.data[1], s))
    diff = o.add_limbs(qi, relin, o.neg_limbs(qi, full))
    # centred residues of the difference in the first limb: small noise
    q0 = p.mod[0]
    dv = diff[0].astype(np.float64)
    dv = np.where(diff[0] > q0 // 2, dv - q0, dv)
    assert np.abs(dv).max() < 2.0 ** 40


def test_constants(deep):
    p, o = deep
    assert o.const_coeffs(0.5, 3.0)[0] == 2 and o.const_coeffs(-0.5, 3.0)[0] == -2
    assert o.const_coeffs(1.25, 4.0)[0] == 5 and (o.const_coeffs(1.25, 4.0)[1:] == 0).all()
    assert o.const_coeffs(1e-3, 2.0 ** 40)[0] == round(1e-3 * 2.0 ** 40)
    # the constant polynomial decodes to the constant in every slot
    z = o.decode(o.const_coeffs(0.375, 2.0 ** 30).astype(np.float64), 2.0 ** 30) \
        if hasattr(o, "decode") else None
    if z is not None:
        assert np.abs(np.asarray(z) - 0.375).max() < 1e-9
    z1 = np.random.default_rng(2).uniform(-1, 1, p.N)
    a = o.encrypt(o.encode(z1, 5, 2.0 ** 40), seed=3)
    assert np.abs(o.decrypt(o.add_const(a, -0.75)) - (z1 - 0.75)).max() < 1e-8
    m = o.rescale(o.mul_const(a, 1.5, float(p.q[5])))
    assert np.abs(o.decrypt(m) - 1.5 * z1).max() < 1e-8


def test_cheb_divide_identity():
    """p = q T_g + r at random points, for random coefficient vectors."""
    rng = np.random.default_rng(3)
    y = rng.uniform(-1, 1, 50)
    for d, g in ((59, 32), (27, 16), (11, 8), (8, 8), (15, 8)):
        c = rng.normal(0, 1, d + 1)
        q, r = hl.cheb_divide(c, g)
        Tg = C.chebval(y, [0] * g + [1])
        assert np.allclose(C.chebval(y, c), C.chebval(y, q) * Tg + C.chebval(y, r), atol=1e-9)
        assert len(r) == g and len(q) == d - g + 1
    assert hl.cheb_baby_size(59) == 8 and hl.cheb_baby_size(63) == 8 and hl.cheb_baby_size(64) == 16


@pytest.mark.parametrize("deg", [3, 7, 16, 59])
def test_cheb_eval_gelu(deep, deg):
    """Encrypted Chebyshev evaluation of a GELU interpolant on [-8, 8] within
    1e-5 of the same polynomial in FP64; nominal scales follow the table."""
    p, o = deep
    a, b = -8.0, 8.0
    coef = C.chebinterpolate(lambda y: gelu((b - a) / 2 * y + (a + b) / 2), deg)
    z = np.random.default_rng(deg).uniform(-6, 6, p.N)
    ct = o.encrypt(o.encode(z, 12, 2.0 ** 40), seed=4)
    ev = hl.ChebEval(hl.CkksBackend(o), ct, a, b)
    r = ev.run(coef)
    assert r.scale == ev.S[r.level]
    assert np.abs(o.decrypt(r) - hl.ref_cheb(z, coef, a, b)).max() < 1e-5
    if deg == 59:
        assert ct.level - r.level == 7      # six for the polynomial, one for the map onto [-1, 1]


@pytest.mark.parametrize("deg,depth", [(59, 6), (27, 5), (13, 4)])
def test_cheb_depth_on_unit_interval(deep, deg, depth):
    """On [-1, 1] (the map folded into the previous layer) the evaluation spends
    exactly the multiplicative depth the paper gives: 6 for degree 59, 5 for
    degree 27 (Appendix, Polynomial Approximation) -- ceil(log2(deg + 1)) --
    and stays within 1e-5 of the FP64 polynomial (GELU over [-8, 8] rescaled
    into the coefficients)."""
    p, o = deep
    coef = C.chebinterpolate(lambda y: gelu(8.0 * y), deg)
    z = np.random.default_rng(deg + 1).uniform(-0.9, 0.9, p.N)
    ct = o.encrypt(o.encode(z, 12, 2.0 ** 40), seed=5)
    ev = hl.ChebEval(hl.CkksBackend(o), ct, -1.0, 1.0)
    r = ev.run(coef)
    assert ct.level - r.level == depth
    assert r.scale == ev.S[r.level]
    assert np.abs(o.decrypt(r) - hl.ref_cheb(z, coef, -1.0, 1.0)).max() < 1e-5
