"""Bias addition, batch-norm folding and the conv -> bias -> GELU -> conv ->
pool block of the encrypted oracle (CPU only), against FP64."""
import numpy as np
import pytest
from numpy.polynomial import chebyshev as C

from oracle import ckks
from oracle import he_layers as hl


def gelu(x):
    return 0.5 * x * (1.0 + np.tanh(np.sqrt(2.0 / np.pi) * (x + 0.044715 * x ** 3)))


@pytest.fixture(scope="module")
def deep():
    p = ckks.Params(10, [60] + [40] * 12, [60] * 4, 4)
    return p, ckks.Oracle(p, 13)


def test_add_pt(deep):
    p, o = deep
    rng = np.random.default_rng(0)
    z1, z2 = rng.uniform(-1, 1, p.N), rng.uniform(-1, 1, p.N)
    ct = o.encrypt(o.encode(z1, 4, 2.0 ** 40), seed=1)
    r = o.add_pt(ct, o.encode(z2, 4, 2.0 ** 40))
    assert np.abs(o.decrypt(r) - (z1 + z2)).max() < 1e-7
    with pytest.raises(ValueError):
        o.add_pt(ct, o.encode(z2, 4, 2.0 ** 41))


def test_add_bias_layout():
    """The bias lands on the valid pixels of each channel's blocks only
    (slot simulator; duplicated and sharded layouts)."""
    for (C_, H, W, N) in ((3, 8, 8, 512), (8, 8, 8, 128), (2, 16, 16, 128)):
        lay = hl.natural_layout(N, C_, H, W)
        bias = np.arange(1, C_ + 1, dtype=np.float64)
        x = np.random.default_rng(1).normal(0, 1, (C_, H, W))
        sim = hl.SlotSim(N, [1.0] * 4)
        cts = [(v, 2, 1.0) for v in hl.pack(x, lay)]
        out = hl.add_bias(sim, cts, lay, bias)
        got = hl.unpack([v for v, _, _ in out], lay)
        assert np.allclose(got, x + bias[:, None, None])
        zero = hl.add_bias(sim, [(np.zeros(N), 2, 1.0) for _ in cts], lay, bias)
        expect = hl.pack(np.broadcast_to(bias[:, None, None], (C_, H, W)), lay)
        for (v, _, _), e in zip(zero, expect):
            assert (v == e).all()


def test_fold_bn_identity():
    """conv(x, w * gamma / d) + shift / d == (gamma conv(x, w) + shift) / d."""
    rng = np.random.default_rng(2)
    x, w = rng.normal(0, 1, (3, 8, 8)), rng.normal(0, 0.2, (4, 3, 3, 3))
    g, h = rng.uniform(0.5, 2, 4), rng.normal(0, 1, 4)
    wf, bf = hl.fold_bn(w, g, h, 7.0)
    lhs = hl.ref_conv2d(x, wf) + bf[:, None, None]
    rhs = (g[:, None, None] * hl.ref_conv2d(x, w) + h[:, None, None]) / 7.0
    assert np.allclose(lhs, rhs, atol=1e-12)


@pytest.mark.parametrize("lazy,bsgs", [(False, False), (True, False), (False, True)])
def test_basic_block(deep, lazy, bsgs):
    """Encrypted block (2 image shards, 4 -> 4 -> 4 channels, 16x16, GELU bound
    10 with the degree-59 interpolant) within 1e-4 of the FP64 block with the
    same polynomial, and within the polynomial's own error of the block with
    GELU itself; 10 levels spent (conv 1, GELU 6, conv 1, pool 2: downsampling
    and the merge of the two shards)."""
    p, o = deep
    rng = np.random.default_rng(3)
    Cc, H = 4, 16
    x = rng.uniform(-1, 1, (Cc, H, H))
    w1, w2 = rng.normal(0, 0.3, (Cc, Cc, 3, 3)), rng.normal(0, 0.3, (Cc, Cc, 3, 3))
    bn1 = (rng.uniform(0.5, 1.5, Cc), rng.normal(0, 0.5, Cc))
    bn2 = (rng.uniform(0.5, 1.5, Cc), rng.normal(0, 0.5, Cc))
    bound = 10.0
    coef = C.chebinterpolate(lambda y: gelu(bound * y), 59)
    lay = hl.natural_layout(p.N, Cc, H, H)
    assert len(lay.shards) == 2
    cts = [o.encrypt(o.encode(v, 12, 2.0 ** 40), seed=4, index=u) for u, v in enumerate(hl.pack(x, lay))]
    be = hl.CkksBackend(o)
    out, olay = hl.basic_block(be, cts, lay, w1, bn1, w2, bn2, bound, coef, lazy=lazy, bsgs=bsgs)
    assert len(out) == 1 and out[0].level == 2
    got = hl.unpack([o.decrypt(ct) for ct in out], olay)
    ref = hl.ref_basic_block(x, w1, bn1, w2, bn2, bound, coef)
    assert got.shape == ref.shape == (Cc, H // 2, H // 2)
    assert np.abs(got - ref).max() < 1e-4
    # the same block with GELU itself
    u = hl.ref_conv2d(x, w1) * bn1[0][:, None, None] + bn1[1][:, None, None]
    assert np.abs(u).max() < bound
    true = hl.ref_avgpool2x2(hl.ref_conv2d(gelu(u), w2) * bn2[0][:, None, None] + bn2[1][:, None, None])
    assert np.abs(got - true).max() < 1e-2
