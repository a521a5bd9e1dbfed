"""Pins of the oracle's encoder/decoder (CPU only).

The encoding is the inverse canonical embedding on real slots: slot j of m(x)
is m(zeta^(5^j)), zeta = exp(i pi/n).  Pins:
* the FFT form equals the plain O(n N) definition, integer for integer;
* a constant slot vector encodes to the constant polynomial (closed form);
* a single unit slot encodes to (2s/n) cos(pi t/n) (closed form, +-1 where the
  exact value sits on a rounding boundary within double precision);
* decode(encode(z)) = z to within the rounding bound sqrt(n)/s;
* the Galois map x -> x^5 rotates the decoded slots left by one (the slot
  order and rotation direction).
"""
import math

import numpy as np
import pytest

from oracle import ckks


def enc(n, z, scale, direct=False):
    z = np.ascontiguousarray(z, dtype=np.float64)
    m = np.zeros(n, dtype=np.int64)
    f = ckks.lib().orc_encode_direct if direct else ckks.lib().orc_encode
    assert f(n, ckks.ptr(z, ckks.dblp), len(z), float(scale), ckks.ptr(m, ckks.i64p)) == 0
    return m


def dec(n, m, scale):
    m = np.ascontiguousarray(m, dtype=np.float64)
    z = np.zeros(n // 2)
    ckks.lib().orc_decode(n, ckks.ptr(m, ckks.dblp), float(scale), ckks.ptr(z, ckks.dblp))
    return z


@pytest.mark.parametrize("logn", [2, 4, 6, 8, 10])
def test_fft_equals_definition(logn):
    n = 1 << logn
    rng = np.random.default_rng(logn)
    for scale in (2.0 ** 20, 2.0 ** 40, 2.0 ** 50, float((1 << 50) - 12345)):
        z = rng.uniform(-1, 1, n // 2)
        assert (enc(n, z, scale) == enc(n, z, scale, direct=True)).all()
        z = (rng.uniform(0, 1, n // 2) < 0.3) * 0.37
        assert (enc(n, z, scale) == enc(n, z, scale, direct=True)).all()


def test_constant_and_unit_slots():
    n = 1 << 10
    s = 2.0 ** 40
    m = enc(n, np.full(n // 2, 0.625), s)
    assert m[0] == round(0.625 * s) and not m[1:].any()
    e0 = np.zeros(n // 2)
    e0[0] = 1.0
    m = enc(n, e0, s)
    ref = np.array([2 * s / n * math.cos(math.pi * t / n) for t in range(n)])
    assert np.abs(m - np.round(ref)).max() <= 1


@pytest.mark.parametrize("logn", [5, 10, 13])
def test_roundtrip(logn):
    n = 1 << logn
    z = np.random.default_rng(3).uniform(-1, 1, n // 2)
    s = 2.0 ** 40
    err = np.abs(dec(n, enc(n, z, s), s) - z).max()
    assert err < math.sqrt(n) / s * 4


def test_galois5_rotates_left():
    n = 1 << 8
    p = ckks.Params(8, [40], [], 1)
    q = p.q[0]
    z = np.random.default_rng(5).uniform(-1, 1, n // 2)
    s = 2.0 ** 30
    m = enc(n, z, s)
    res = np.zeros((1, n), dtype=np.uint64)
    pidx = ckks.u32arr([0])
    ckks.lib().orc_reduce_small(p.cref, ckks.ptr(m, ckks.i64p), ckks.ptr(pidx, ckks.u32p), 1, ckks.ptr(res))
    for g, shift in ((5, 1), (25, 2), (pow(5, n // 2 - 1, 2 * n), -1)):
        out = np.zeros_like(res)
        ckks.lib().orc_automorph(p.cref, ckks.ptr(pidx, ckks.u32p), 1, g, ckks.ptr(res), ckks.ptr(out))
        centered = np.array([int(v) if int(v) <= q // 2 else int(v) - q for v in out[0]], dtype=np.float64)
        assert np.abs(dec(n, centered, s) - np.roll(z, -shift)).max() < 1e-6


def test_automorph_definition():
    """sigma_g(a)(x) = a(x^g) mod x^n + 1, against substitution in Python."""
    n = 16
    p = ckks.Params(4, [30], [], 1)
    q = p.q[0]
    a = np.random.default_rng(0).integers(0, q, n, dtype=np.uint64)
    pidx = ckks.u32arr([0])
    for g in (3, 5, 7, 25, 31):
        out = np.zeros(n, dtype=np.uint64)
        ckks.lib().orc_automorph(p.cref, ckks.ptr(pidx, ckks.u32p), 1, g, ckks.ptr(a), ckks.ptr(out))
        ref = [0] * n
        for t in range(n):
            e = t * g % (2 * n)
            if e < n:
                ref[e] = (ref[e] + int(a[t])) % q
            else:
                ref[e - n] = (ref[e - n] - int(a[t])) % q
        assert [int(x) for x in out] == ref
