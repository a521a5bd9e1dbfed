"""Plaintext and bias addition and the conv -> bias -> GELU -> conv -> pool
block of the GPU library vs the CPU oracle (MI355X, through the C ABI):
bit-exact on a small ring for every evaluation mode and several layouts."""
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
    ctx.keygen(13)
    return ctx, prm, ckks.Oracle(prm, 13)


def encrypt_both(ctx, prm, o, x, level, seed):
    C_, H, W = x.shape
    img = ctx.image_encrypt(x, level, seed)
    lay = hl.natural_layout(prm.N, C_, H, W)
    cts = [o.encrypt(o.encode(v, level, 2.0 ** 40), seed=seed, index=u) for u, v in enumerate(hl.pack(x, lay))]
    for u in range(len(cts)):
        assert (img.shard_export(u) == cts[u].data).all()
    return img, cts, lay


def test_add_pt_bit_exact(deep):
    from paper_2306_09189_amd import hecnn
    ctx, prm, o = deep
    rng = np.random.default_rng(0)
    z1, z2 = rng.uniform(-1, 1, prm.N), rng.uniform(-1, 1, prm.N)
    ct = o.encrypt(o.encode(z1, 5, 2.0 ** 40), seed=1)
    g = ctx.add_pt(ctx.ct_import(ct.data, 5, ct.scale), ctx.encode(z2, 5, 2.0 ** 40))
    assert (g.export() == o.add_pt(ct, o.encode(z2, 5, 2.0 ** 40)).data).all()
    with pytest.raises(hecnn.HecError):
        ctx.add_pt(ctx.ct_import(ct.data, 5, ct.scale), ctx.encode(z2, 5, 2.0 ** 39))
    with pytest.raises(hecnn.HecError):
        ctx.add_pt(ctx.ct_import(ct.data, 5, ct.scale), ctx.encode(z2, 4, 2.0 ** 40))


@pytest.mark.parametrize("shape", [(4, 16, 16), (3, 8, 8), (1, 64, 64)])
def test_add_bias_bit_exact(deep, shape):
    """Image shards, a duplicated layout and channel shards."""
    ctx, prm, o = deep
    x = np.random.default_rng(1).uniform(-1, 1, shape)
    img, cts, lay = encrypt_both(ctx, prm, o, x, 6, 21)
    bias = np.linspace(-0.5, 0.7, shape[0])
    out = ctx.add_bias(img, bias)
    ref = hl.add_bias(hl.CkksBackend(o), cts, lay, bias)
    for u in range(len(ref)):
        assert (out.shard_export(u) == ref[u].data).all()
    assert np.abs(out.decrypt() - (x + bias[:, None, None])).max() < 1e-6


@pytest.mark.parametrize("shape,Co,stride", [((4, 16, 16), 4, 1), ((4, 16, 16), 8, 2), ((3, 8, 8), 5, 1)])
def test_conv_bias_bit_exact(deep, shape, Co, stride):
    """he_conv2d_sharded with its bias argument (the shift of a folded batch
    norm, Section 4.3): the oracle's convolution followed by its per-channel
    bias addition, bit for bit; a bias of the wrong length is refused by the
    binding, weights whose input-channel count differs from the image's too."""
    ctx, prm, o = deep
    rng = np.random.default_rng(sum(shape) + Co)
    x = rng.uniform(-1, 1, shape)
    w = rng.normal(0, 0.2, (Co, shape[0], 3, 3))
    bias = rng.normal(0, 0.5, Co)
    img, cts, lay = encrypt_both(ctx, prm, o, x, 6, 22)
    plan = ctx.conv2d_plan(img, w, stride=stride)
    ctx.gen_rotation_keys(plan.steps())
    out = ctx.conv2d(img, w, stride=stride, bias=bias)
    be = hl.CkksBackend(o)
    oc, ol = hl.conv2d(be, cts, lay, w, pad=1, stride=stride)
    oc = hl.add_bias(be, oc, ol, bias)
    assert out.info()[4] == len(oc)
    for u in range(len(oc)):
        assert out.shard_info(u) == (oc[u].level, oc[u].scale)
        assert (out.shard_export(u) == oc[u].data).all(), u
    ref = hl.ref_conv2d(x, w, 1, stride) + bias[:, None, None]
    assert np.abs(out.decrypt() - ref).max() < 1e-5
    with pytest.raises(ValueError):
        ctx.conv2d(img, w, stride=stride, bias=bias[:-1])
    with pytest.raises(ValueError):
        ctx.conv2d(img, w[:, :-1], stride=stride)
    with pytest.raises(ValueError):
        ctx.conv2d_plan(img, w[:, :-1])


def block_case(ctx, prm, o, shape, Co, mode, seed, bn2=True):
    rng = np.random.default_rng(seed)
    C_, H, W = shape
    x = rng.uniform(-1, 1, shape)
    w1, w2 = rng.normal(0, 0.3, (Co, C_, 3, 3)), rng.normal(0, 0.3, (Co, Co, 3, 3))
    b1 = (rng.uniform(0.5, 1.5, Co), rng.normal(0, 0.5, Co))
    b2 = (rng.uniform(0.5, 1.5, Co), rng.normal(0, 0.5, Co)) if bn2 else None
    bound = 10.0
    coef = C.chebinterpolate(lambda y: gelu(bound * y), 59)
    img, cts, lay = encrypt_both(ctx, prm, o, x, 12, seed)
    blk = ctx.block(img, w1, b1, w2, b2, bound, coef, mode=mode)
    ctx.gen_rotation_keys(blk.steps())
    log("block", shape, Co, "mode", mode)
    out = blk.run(img)
    ref, rlay = hl.basic_block(hl.CkksBackend(o), cts, lay, w1, b1, w2, b2, bound, coef,
                               lazy=(mode == 2), bsgs=(mode == 3))
    Cn, Hn, Wn, mp, t = out.info()
    assert t == len(ref) and (Cn, Hn, Wn) == (Co, H // 2, W // 2)
    for u in range(t):
        assert out.shard_info(u) == (ref[u].level, ref[u].scale)
        assert (out.shard_export(u) == ref[u].data).all(), u
    fp = hl.ref_basic_block(x, w1, b1, w2, b2, bound, coef)
    assert np.abs(out.decrypt() - fp).max() < 1e-4


@pytest.mark.parametrize("mode", [0, 2, 3])
def test_block_bit_exact(deep, mode):
    ctx, prm, o = deep
    block_case(ctx, prm, o, (4, 16, 16), 4, mode, 30 + mode)


def test_block_widening_no_bn2(deep):
    """4 -> 8 channels (more output shards than input shards), no second batch norm."""
    ctx, prm, o = deep
    block_case(ctx, prm, o, (4, 16, 16), 8, 3, 40, bn2=False)


def test_block_duplicated_layout(deep):
    ctx, prm, o = deep
    block_case(ctx, prm, o, (2, 8, 8), 2, 2, 41)


def test_block_errors(deep):
    from paper_2306_09189_amd import hecnn
    ctx, prm, o = deep
    x = np.zeros((4, 16, 16))
    img = ctx.image_encrypt(x, 6, 1)
    w = np.zeros((4, 4, 3, 3))
    bn = (np.ones(4), np.zeros(4))
    coef = C.chebinterpolate(lambda y: gelu(10 * y), 59)
    with pytest.raises(hecnn.HecError):      # degree 59 after a conv needs more than 6 levels
        ctx.block(img, w, bn, w, bn, 10.0, coef)
    img = ctx.image_encrypt(x, 12, 1)
    with pytest.raises(hecnn.HecError):
        ctx.block(img, w, bn, w, bn, 0.0, coef)
    with pytest.raises(hecnn.HecError):
        ctx.block(img, np.zeros((4, 4, 2, 2)), bn, np.zeros((4, 4, 2, 2)), bn, 10.0, coef)
