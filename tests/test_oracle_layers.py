"""Encrypted oracle end to end (CPU only): decrypted homomorphic conv / pool
against direct FP64 conv2d / avg_pool2d, max abs error 1e-5, on small rings
and on the 2N = 2^13 workload (one 32x32x4 image, 3x3 conv 4->4, 2x2 pool)."""
import numpy as np
import pytest

from oracle import ckks
from oracle import he_layers as hl


def enc_image(o, x, lay, level, scale, seed):
    cts = []
    for u, v in enumerate(hl.pack(x, lay)):
        cts.append(o.encrypt(o.encode(v, level, scale), seed=seed, index=u))
    return cts


def dec_image(o, cts, lay):
    return hl.unpack([o.decrypt(c) for c in cts], lay)


@pytest.fixture(scope="module")
def small():
    p = ckks.Params(8, [60] + [40] * 6, [60, 60, 60], 3)   # P > every digit
    return p, ckks.Oracle(p, 5)


def test_conv_single_shard(small):
    p, o = small
    rng = np.random.default_rng(0)
    x = rng.uniform(-1, 1, (2, 8, 8))
    w = rng.normal(0, 0.1, (2, 2, 3, 3))
    lay = hl.natural_layout(p.N, 2, 8, 8)
    cts = enc_image(o, x, lay, 6, 2.0 ** 40, 11)
    outs, ol = hl.conv2d(hl.CkksBackend(o), cts, lay, w, pad=1)
    assert outs[0].level == 5 and outs[0].scale == 2.0 ** 40
    assert np.abs(dec_image(o, outs, ol) - hl.ref_conv2d(x, w, 1)).max() < 1e-5


def test_conv_image_shards_and_stride2(small):
    p, o = small
    rng = np.random.default_rng(1)
    x = rng.uniform(-1, 1, (4, 8, 8))     # 2 shards of 2 channels
    w = rng.normal(0, 0.1, (4, 4, 3, 3))
    lay = hl.natural_layout(p.N, 4, 8, 8)
    assert len(lay.shards) == 2
    cts = enc_image(o, x, lay, 6, 2.0 ** 40, 12)
    outs, ol = hl.conv2d(hl.CkksBackend(o), cts, lay, w, pad=1, stride=2)
    assert len(outs) == 1 and outs[0].level == 3
    assert np.abs(dec_image(o, outs, ol) - hl.ref_conv2d(x, w, 1, 2)).max() < 1e-5


def test_pool_separable_and_fused(small):
    p, o = small
    x = np.random.default_rng(2).uniform(-1, 1, (2, 8, 8))
    lay = hl.natural_layout(p.N, 2, 8, 8)
    for fused, lvl_out in ((False, 4), (True, 5)):
        cts = enc_image(o, x, lay, 6, 2.0 ** 40, 13)
        outs, ol = hl.avgpool2x2(hl.CkksBackend(o), cts, lay, fused=fused)
        assert outs[0].level == lvl_out
        assert np.abs(dec_image(o, outs, ol) - hl.ref_avgpool2x2(x)).max() < 1e-5


def test_channel_shards(small):
    """A 32x32 channel in 2^7-slot shards (8 shards per channel): conv (rows
    taken from neighbouring shards) then pooling (consolidation)."""
    p, o = small
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, (1, 32, 32))
    w = rng.normal(0, 0.2, (2, 1, 3, 3))
    lay = hl.natural_layout(p.N, 1, 32, 32)
    assert lay.kind == "channel" and len(lay.shards) == 8
    cts = enc_image(o, x, lay, 6, 2.0 ** 40, 14)
    be = hl.CkksBackend(o)
    c, cl = hl.conv2d(be, cts, lay, w, pad=1)
    ref = hl.ref_conv2d(x, w, 1)
    assert np.abs(dec_image(o, c, cl) - ref).max() < 1e-5
    pl_, pll = hl.avgpool2x2(be, c, cl)
    assert np.abs(dec_image(o, pl_, pll) - hl.ref_avgpool2x2(ref)).max() < 1e-5


@pytest.mark.slow
def test_ring_2e13_conv_pool():
    """2N = 2^13, 3 x 40-bit primes + one 60-bit special prime, scale 2^40: a
    3x3 conv 4->4 (level 2 -> 1) and the one-level pool (level 1 -> 0, masks at
    q/4 so the result is decryptable under the 40-bit q_0)."""
    p = ckks.Params(13, [40, 40, 40], [60], 3)
    o = ckks.Oracle(p, 2001)
    rng = np.random.default_rng(1001)
    x = rng.uniform(-1, 1, (4, 32, 32))
    w = rng.normal(0, 0.1, (4, 4, 3, 3))
    lay = hl.natural_layout(p.N, 4, 32, 32)
    be = hl.CkksBackend(o)
    cts = enc_image(o, x, lay, 2, 2.0 ** 40, 3001)
    c, cl = hl.conv2d(be, cts, lay, w, pad=1)
    ref_c = hl.ref_conv2d(x, w, 1)
    assert np.abs(dec_image(o, c, cl) - ref_c).max() < 1e-5
    pl_, pll = hl.avgpool2x2(be, c, cl)
    assert pl_[0].level == 0 and pl_[0].scale == 2.0 ** 38
    assert np.abs(dec_image(o, pl_, pll) - hl.ref_avgpool2x2(ref_c)).max() < 1e-5


def test_lazy_moddown_conv(small):
    """Lazy ModDown (products accumulated over Q*P, one ModDown per output
    shard) decrypts to the same convolution; with only zero rotations it is
    bit-identical to the per-rotation form (no key switch involved)."""
    p, o = small
    rng = np.random.default_rng(7)
    x = rng.uniform(-1, 1, (4, 8, 8))
    w = rng.normal(0, 0.1, (4, 4, 3, 3))
    lay = hl.natural_layout(p.N, 4, 8, 8)
    cts = enc_image(o, x, lay, 6, 2.0 ** 40, 15)
    be = hl.CkksBackend(o)
    a, al = hl.conv2d(be, cts, lay, w, pad=1, lazy=True)
    b, bl = hl.conv2d(be, cts, lay, w, pad=1, lazy=False)
    ref = hl.ref_conv2d(x, w, 1)
    ea = np.abs(dec_image(o, a, al) - ref).max()
    eb = np.abs(dec_image(o, b, bl) - ref).max()
    assert ea < 1e-5 and eb < 1e-5
    assert a[0].level == b[0].level and a[0].scale == b[0].scale
    assert not (a[0].data == b[0].data).all()     # different rounding, different bits
    # 1x1 kernel on a one-block-per-channel layout with a single channel: only the zero rotation
    x1 = rng.uniform(-1, 1, (1, 8, 8))
    w1 = rng.normal(0, 0.1, (1, 1, 1, 1))
    lay1 = hl.natural_layout(p.N, 1, 8, 8)
    c1 = enc_image(o, x1, lay1, 6, 2.0 ** 40, 16)
    la, _ = hl.conv2d(be, c1, lay1, w1, pad=0, lazy=True)
    lb, _ = hl.conv2d(be, c1, lay1, w1, pad=0, lazy=False)
    assert (la[0].data == lb[0].data).all()


def test_lazy_moddown_pooling(small):
    """Pooling and strided convolution with the masked rotation sums of the
    downsampling taken lazily (one ModDown per sum): same values within 1e-5,
    same levels and scales as the per-rotation form, other bits."""
    p, o = small
    rng = np.random.default_rng(8)
    be = hl.CkksBackend(o)
    x = rng.uniform(-1, 1, (4, 8, 8))
    lay = hl.natural_layout(p.N, 4, 8, 8)
    for fused, lvl_out in ((False, 4), (True, 5)):
        cts = enc_image(o, x, lay, 6, 2.0 ** 40, 17)
        a, al = hl.avgpool2x2(be, cts, lay, fused=fused, lazy=True)
        b, bl = hl.avgpool2x2(be, cts, lay, fused=fused, lazy=False)
        assert a[0].level == b[0].level == lvl_out and a[0].scale == b[0].scale
        assert al.shards == bl.shards
        ref = hl.ref_avgpool2x2(x)
        assert np.abs(dec_image(o, a, al) - ref).max() < 1e-5
        assert not (a[0].data == b[0].data).all()
    w = rng.normal(0, 0.1, (4, 4, 3, 3))
    cts = enc_image(o, x, lay, 6, 2.0 ** 40, 18)
    s, sl = hl.conv2d(be, cts, lay, w, pad=1, stride=2, lazy=True)
    assert s[0].level == 3
    assert np.abs(dec_image(o, s, sl) - hl.ref_conv2d(x, w, 1, 2)).max() < 1e-5


def test_lazy_moddown_channel_pooling(small):
    p, o = small
    rng = np.random.default_rng(9)
    be = hl.CkksBackend(o)
    x = rng.uniform(-1, 1, (1, 32, 32))
    lay = hl.natural_layout(p.N, 1, 32, 32)
    cts = enc_image(o, x, lay, 6, 2.0 ** 40, 19)
    a, al = hl.avgpool2x2(be, cts, lay, lazy=True)
    assert np.abs(dec_image(o, a, al) - hl.ref_avgpool2x2(x)).max() < 1e-5


def test_bsgs_conv(small):
    """Baby-step / giant-step convolution with double hoisting: the same
    convolution within 1e-5 (image shards, stride 2, channel shards), same
    level and scale; with only zero babies and zero giants (1x1 kernel, one
    channel per shard) it equals the lazy form bit for bit."""
    p, o = small
    rng = np.random.default_rng(10)
    be = hl.CkksBackend(o)
    x = rng.uniform(-1, 1, (4, 8, 8))
    w = rng.normal(0, 0.1, (4, 4, 3, 3))
    lay = hl.natural_layout(p.N, 4, 8, 8)
    cts = enc_image(o, x, lay, 6, 2.0 ** 40, 20)
    a, al = hl.conv2d(be, cts, lay, w, pad=1, bsgs=True)
    b, bl = hl.conv2d(be, cts, lay, w, pad=1, lazy=True)
    assert a[0].level == b[0].level and a[0].scale == b[0].scale and al.shards == bl.shards
    assert np.abs(dec_image(o, a, al) - hl.ref_conv2d(x, w, 1)).max() < 1e-5
    s, sl = hl.conv2d(be, cts, lay, w, pad=1, stride=2, bsgs=True)
    assert np.abs(dec_image(o, s, sl) - hl.ref_conv2d(x, w, 1, 2)).max() < 1e-5
    xc = rng.uniform(-1, 1, (1, 32, 32))
    wc = rng.normal(0, 0.2, (2, 1, 3, 3))
    lc = hl.natural_layout(p.N, 1, 32, 32)
    cc = enc_image(o, xc, lc, 6, 2.0 ** 40, 21)
    c, cl = hl.conv2d(be, cc, lc, wc, pad=1, bsgs=True)
    assert np.abs(dec_image(o, c, cl) - hl.ref_conv2d(xc, wc, 1)).max() < 1e-5
    x1 = rng.uniform(-1, 1, (1, 8, 8))
    w1 = rng.normal(0, 0.1, (1, 1, 1, 1))
    l1 = hl.natural_layout(p.N, 1, 8, 8)
    c1 = enc_image(o, x1, l1, 6, 2.0 ** 40, 22)
    za, _ = hl.conv2d(be, c1, l1, w1, pad=0, bsgs=True)
    zb, _ = hl.conv2d(be, c1, l1, w1, pad=0, lazy=True)
    assert (za[0].data == zb[0].data).all()


def test_bsgs_split_identity():
    """pt * rot_{b+g}(x) == rot_g(roll(pt, g) * rot_b(x)) on slot vectors, for
    every (amount, split) of a plan: the identity the giant steps rest on."""
    N = 256
    rng = np.random.default_rng(11)
    lay = hl.natural_layout(N, 4, 8, 8)
    w = rng.normal(0, 1, (4, 4, 3, 3))
    _, plan = hl.conv_plan_split(lay, w, 1)
    x = rng.normal(0, 1, N)
    rot = lambda v, a: np.roll(v, -a)   # slot j <- slot j + a
    for items in plan:
        for a, pts, (b, g) in items:
            assert (b + g - a) % N == 0 and b % lay.B == 0
            for vec in pts.values():
                assert np.allclose(vec * rot(x, a), rot(np.roll(vec, g) * rot(x, b), g))


def test_bsgs_split():
    assert hl.bsgs_split(list(range(16)), 1)[:6] == [(0, 0), (1, 0), (2, 0), (3, 0), (0, 4), (1, 4)]
    sp = hl.bsgs_split([24 * j for j in range(9)], 24)      # G = 3
    assert sp[4] == (24, 72) and sp[8] == (48, 144)
    for steps, unit in ((list(range(56)), 1), ([6 * j for j in (0, 2, 5, 7)], 6)):
        for a, (b, g) in zip(steps, hl.bsgs_split(steps, unit)):
            assert a == b + g and b % unit == 0 and g % unit == 0


def test_bsgs_pooling(small, monkeypatch):
    """Pooling (separable, fused, channel shards) with the masked rotation
    sums evaluated by baby and giant steps (threshold lowered so that the
    small shapes take that path)."""
    p, o = small
    monkeypatch.setattr(hl, "BSGS_MIN_STEPS", 2)
    rng = np.random.default_rng(12)
    be = hl.CkksBackend(o)
    x = rng.uniform(-1, 1, (4, 8, 8))
    lay = hl.natural_layout(p.N, 4, 8, 8)
    for fused, lvl_out in ((False, 4), (True, 5)):
        cts = enc_image(o, x, lay, 6, 2.0 ** 40, 23)
        a, al = hl.avgpool2x2(be, cts, lay, fused=fused, bsgs=True)
        b, _ = hl.avgpool2x2(be, cts, lay, fused=fused, lazy=True)
        assert a[0].level == lvl_out
        assert not (a[0].data == b[0].data).all()
        assert np.abs(dec_image(o, a, al) - hl.ref_avgpool2x2(x)).max() < 1e-5
    xc = rng.uniform(-1, 1, (1, 32, 32))
    lc = hl.natural_layout(p.N, 1, 32, 32)
    cc = enc_image(o, xc, lc, 6, 2.0 ** 40, 24)
    a, al = hl.avgpool2x2(be, cc, lc, bsgs=True)
    assert np.abs(dec_image(o, a, al) - hl.ref_avgpool2x2(xc)).max() < 1e-5


def test_bsgs_pooling_threshold(small):
    """Below BSGS_MIN_STEPS amounts the baby-step / giant-step mode pools
    exactly like the lazy mode."""
    p, o = small
    x = np.random.default_rng(13).uniform(-1, 1, (4, 8, 8))
    lay = hl.natural_layout(p.N, 4, 8, 8)
    be = hl.CkksBackend(o)
    cts = enc_image(o, x, lay, 6, 2.0 ** 40, 25)
    a, _ = hl.avgpool2x2(be, cts, lay, bsgs=True)
    b, _ = hl.avgpool2x2(be, cts, lay, lazy=True)
    assert (a[0].data == b[0].data).all()


def test_linear_and_pool_linear(small):
    """Linear (dot products by rotate-and-add over all slots, outputs masked
    into slots 0..O-1) and pool-linear, decrypted within 1e-5 of W @ x."""
    p, o = small
    rng = np.random.default_rng(14)
    be = hl.CkksBackend(o)
    x = rng.uniform(-1, 1, (4, 8, 8))
    lay = hl.natural_layout(p.N, 4, 8, 8)
    cts = enc_image(o, x, lay, 6, 2.0 ** 40, 26)
    for pool, O in ((False, 3), (True, 5)):
        W = rng.normal(0, 0.1, (O, 4) if pool else (O, 4 * 64))
        out = hl.linear(be, cts, lay, W, pool)
        assert out.level == 4 and out.scale == 2.0 ** 40
        got = o.decrypt(out)
        assert np.abs(got[:O] - hl.ref_linear(x, W, pool)).max() < 1e-5
        assert np.abs(got[O:]).max() < 1e-5


def test_basis_plaintext_pins(small):
    """Basis-mask plaintexts (a weight per block times the encoding of the
    tap's mask on that block at 2^s) against the exact encoding of the same
    slot vector: per coefficient within 1/2 + |w^|/2 + 2^(s-1) (rounding of
    the weight, of the basis polynomial and of the exact encoding; every mask
    coefficient of sigma^-1 is at most 1), and decoded within the triangle
    bound 2^(s-1)/scale + |w^| n / (2 scale) per block."""
    p, o = small
    rng = np.random.default_rng(31)
    lay = hl.natural_layout(p.N, 4, 4, 4)     # blocks of 16 slots, channels duplicated
    x = np.zeros((4, 4, 4))
    w = rng.normal(0, 0.3, (4, 4, 3, 3))
    out, plan = hl.conv_plan_split(lay, w, 1)
    s = 20
    be = hl.CkksBackend(o, basis=s)
    pscale = be.q(5)
    vecs = [vec for items in plan for _, pts, _ in items for vec in pts.values()]
    assert vecs and all(v.mask is not None for v in vecs)
    for vec in vecs[:12]:
        mb = be.pt_coeffs(vec, pscale)
        me = o.encode_coeffs(np.asarray(vec), pscale)
        wh = {b: int(o.const_coeffs(wv, pscale / 2.0 ** s)[0]) for b, wv in vec.wb.items()}
        tol = sum(0.5 + abs(h) / 2.0 + 2.0 ** (s - 1) for h in wh.values()) + 0.5
        assert np.abs(mb - me).max() <= tol
        dec = o.decode(mb.astype(np.float64), pscale)
        for b, h in wh.items():
            blk = slice(b * vec.B, (b + 1) * vec.B)
            bnd = 2.0 ** (s - 1) / pscale + abs(h) * p.n / (2 * pscale)
            assert np.abs(dec[blk] - np.asarray(vec)[blk]).max() <= bnd * len(wh)
    # a derived (rolled) vector is a plain vector again: exact encoding
    r = np.roll(vecs[0], 3)
    assert getattr(r, "mask", None) is None
    assert (be.pt_coeffs(r, pscale) == o.encode_coeffs(np.asarray(r), pscale)).all()


def test_basis_conv(small):
    """Convolutions with basis-mask plaintexts, per rotation and with lazy
    ModDown, decrypt within 1e-5 of FP64 on an image-sharded input (two
    shards) and give other ciphertexts than exact encoding; the
    baby-step/giant-step form refuses them."""
    p, o = small
    rng = np.random.default_rng(32)
    x = rng.uniform(-1, 1, (4, 8, 8))
    w = rng.normal(0, 0.1, (4, 4, 3, 3))
    lay = hl.natural_layout(p.N, 4, 8, 8)
    assert len(lay.shards) == 2
    cts = enc_image(o, x, lay, 6, 2.0 ** 40, 33)
    ref = hl.ref_conv2d(x, w, 1)
    beb = hl.CkksBackend(o, basis=20)
    a, al = hl.conv2d(beb, cts, lay, w, pad=1)
    la, _ = hl.conv2d(beb, cts, lay, w, pad=1, lazy=True)
    e, _ = hl.conv2d(hl.CkksBackend(o), cts, lay, w, pad=1)
    for outs in (a, la):
        assert outs[0].level == 5 and outs[0].scale == 2.0 ** 40
        assert np.abs(dec_image(o, outs, al) - ref).max() < 1e-5
    assert not (a[0].data == e[0].data).all()
    assert not (a[0].data == la[0].data).all()
    with pytest.raises(ValueError):
        hl.conv2d(beb, cts, lay, w, pad=1, bsgs=True)
