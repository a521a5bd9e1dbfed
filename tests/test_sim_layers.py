"""The conv / pool schedule (the paper's Section 4) run on cleartext FP64 slot
vectors must equal direct FP64 convolution and pooling (CPU only).

This pins the layout algebra -- rotation offsets, shift masks, partial
convolutions, image shards, duplication, the permutation after
consolidation, strided convolution as convolution + downsampling -- without
any encryption.  Special cases from the paper: a 1x1 kernel is the channel
mixing of Eq. (2); an identity kernel returns the input; a 2x2 channel pools
to its mean.
"""
import numpy as np
import pytest

from oracle import he_layers as hl

QS = [float(2 ** 40 + i) for i in range(40)]


def run_conv(N, x, w, pad, stride):
    C, H, W = x.shape
    lay = hl.natural_layout(N, C, H, W)
    be = hl.SlotSim(N, QS)
    cts = [(v, 10, 1.0) for v in hl.pack(x, lay)]
    outs, ol = hl.conv2d(be, cts, lay, w, pad=pad, stride=stride)
    return hl.unpack([o[0] for o in outs], ol), ol, outs


CASES = [
    # N, C, H, W, Co, k, pad, stride
    (64, 4, 4, 4, 4, 3, 1, 1),        # single shard, d = 1
    (256, 4, 4, 4, 4, 3, 1, 1),       # d = 4 duplication
    (256, 3, 4, 4, 5, 3, 1, 1),       # channel padding to 4, output 5 -> 8 blocks d=1
    (64, 8, 4, 4, 8, 3, 1, 1),        # image shards: 2 in, 2 out
    (64, 16, 4, 4, 4, 3, 1, 1),       # 4 shards in -> 1 shard out
    (64, 4, 4, 4, 16, 3, 1, 1),       # 1 shard in -> 4 shards out
    (256, 4, 8, 8, 4, 3, 1, 2),       # stride 2, one shard -> dup x4
    (64, 8, 4, 4, 8, 3, 1, 2),        # stride 2 from 2 shards -> consolidate + dup x2
    (64, 16, 4, 4, 16, 3, 1, 2),      # stride 2, 4 shards -> 1
    (256, 4, 6, 6, 4, 3, 1, 1),       # non power of two side (padded to 8)
    (256, 4, 8, 8, 4, 3, 0, 1),       # valid (no) padding
    (256, 4, 8, 8, 4, 5, 2, 1),       # 5x5 kernel
    (256, 4, 8, 8, 4, 1, 0, 1),       # 1x1 kernel
]


@pytest.mark.parametrize("case", CASES)
def test_conv_matches_fp64(case):
    N, C, H, W, Co, k, pad, stride = case
    rng = np.random.default_rng(hash(case) % 2 ** 32)
    x = rng.uniform(-1, 1, (C, H, W))
    w = rng.normal(0, 0.3, (Co, C, k, k))
    got, ol, outs = run_conv(N, x, w, pad, stride)
    ref = hl.ref_conv2d(x, w, pad, stride)
    assert got.shape == ref.shape
    assert np.abs(got - ref).max() < 1e-12
    # every copy of a duplicated channel holds the same values
    for u, lam in enumerate(ol.shards):
        for b, f in enumerate(lam):
            if f >= 0:
                blk = outs[u][0][b * ol.B:(b + 1) * ol.B].reshape(ol.mp, ol.mp)[: ol.H, : ol.W]
                assert np.abs(blk - ref[f]).max() < 1e-12


def test_one_by_one_is_channel_mixing():
    """Eq. (2): (M*K)^g = sum_r K^{r+g,g} M^{r+g}."""
    N, c = 64, 4
    rng = np.random.default_rng(0)
    x = rng.uniform(-1, 1, (c, 4, 4))
    K = rng.normal(size=(c, c))          # paper indexing K[f][g]
    w = K.T[:, :, None, None]            # PyTorch [g][f]
    got, _, _ = run_conv(N, x, w, 0, 1)
    ref = np.stack([sum(K[(r + g) % c, g] * x[(r + g) % c] for r in range(c)) for g in range(c)])
    assert np.abs(got - ref).max() < 1e-12


def test_identity_kernel():
    N = 256
    x = np.random.default_rng(1).uniform(-1, 1, (4, 8, 8))
    w = np.zeros((4, 4, 3, 3))
    for f in range(4):
        w[f, f, 1, 1] = 1.0
    got, _, _ = run_conv(N, x, w, 1, 1)
    assert np.abs(got - x).max() < 1e-15


def run_pool(N, x, fused=None, level=10):
    C, H, W = x.shape
    lay = hl.natural_layout(N, C, H, W)
    be = hl.SlotSim(N, QS)
    cts = [(v, level, 1.0) for v in hl.pack(x, lay)]
    outs, ol = hl.avgpool2x2(be, cts, lay, fused=fused)
    return hl.unpack([o[0] for o in outs], ol), ol, outs


@pytest.mark.parametrize("N,C,H", [(64, 4, 4), (256, 4, 8), (64, 8, 4), (64, 16, 4), (64, 32, 4), (1024, 1, 32),
                                   (256, 2, 8), (1024, 4, 16)])
@pytest.mark.parametrize("fused", [False, True])
def test_pool_matches_fp64(N, C, H, fused):
    x = np.random.default_rng(N + C + H).uniform(-1, 1, (C, H, H))
    got, ol, _ = run_pool(N, x, fused=fused)
    assert np.abs(got - hl.ref_avgpool2x2(x)).max() < 1e-12


def test_pool_of_2x2_is_mean_and_permutes():
    x = np.random.default_rng(2).uniform(-1, 1, (16, 2, 2))
    got, ol, _ = run_pool(16, x)    # 4 shards of 4 channels -> 1 shard, permuted
    assert np.abs(got[:, 0, 0] - x.mean(axis=(1, 2))).max() < 1e-15
    lam = ol.shards[0]
    assert sorted(lam) == list(range(16)) and lam != list(range(16))


def test_pool_then_conv_on_permuted_layout():
    """A convolution after a consolidating pool must follow the block map."""
    N = 64
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, (16, 4, 4))
    w = rng.normal(0, 0.3, (8, 16, 3, 3))
    lay = hl.natural_layout(N, 16, 4, 4)
    be = hl.SlotSim(N, QS)
    cts = [(v, 10, 1.0) for v in hl.pack(x, lay)]
    p, pl = hl.avgpool2x2(be, cts, lay)
    c, cl = hl.conv2d(be, p, pl, w, pad=1)
    ref = hl.ref_conv2d(hl.ref_avgpool2x2(x), w, 1)
    assert np.abs(hl.unpack([o[0] for o in c], cl) - ref).max() < 1e-12


def test_conv_then_pool_after_duplication():
    N = 1024
    rng = np.random.default_rng(4)
    x = rng.uniform(-1, 1, (4, 8, 8))   # d = 4
    w = rng.normal(0, 0.3, (4, 4, 3, 3))
    lay = hl.natural_layout(N, 4, 8, 8)
    be = hl.SlotSim(N, QS)
    cts = [(v, 10, 1.0) for v in hl.pack(x, lay)]
    p, pl = hl.avgpool2x2(be, cts, lay)          # dup x4 again -> d = 16
    c, cl = hl.conv2d(be, p, pl, w, pad=1)
    ref = hl.ref_conv2d(hl.ref_avgpool2x2(x), w, 1)
    assert np.abs(hl.unpack([o[0] for o in c], cl) - ref).max() < 1e-12


def test_rotation_counts_match_paper_shapes():
    """Offsets for the 32x32x32 layer of one full shard: 32 channel offsets x 9
    taps, less the zero rotation (287 distinct nonzero amounts)."""
    lay = hl.natural_layout(1 << 15, 32, 32, 32)
    w = np.ones((32, 32, 3, 3))
    ol, plan = hl.conv_plan(lay, w, 1)
    amounts = set(a for a, _ in plan[0])
    assert len(amounts) == 288 and 0 in amounts
    # 112x112x64 padded to 128, 2 channels per shard, 32 shards: 2 x 9 offsets per shard
    lay = hl.natural_layout(1 << 15, 64, 112, 112)
    assert len(lay.shards) == 32 and lay.mp == 128


# ---- channel shards (Section 4.1 "With Channel Shards", Section 4.2 channel-shard pooling) ----

CH_CASES = [
    # N, C, H, Co, k, pad, stride
    (128, 2, 16, 3, 3, 1, 1),    # mp 16: 2 shards per channel
    (64, 2, 16, 2, 3, 1, 1),     # 4 shards per channel
    (32, 1, 16, 2, 3, 1, 1),     # 8 shards per channel
    (64, 3, 14, 2, 3, 1, 1),     # side 14 padded to 16, last rows empty
    (64, 2, 16, 2, 5, 2, 1),     # 5x5 kernel: shifts of two rows across shards
    (128, 2, 16, 2, 3, 0, 1),    # no padding
    (128, 3, 16, 4, 3, 1, 2),    # strided: 2 shards/channel -> image shards
    (64, 2, 16, 2, 3, 1, 2),     # strided: 4 shards/channel -> one ciphertext per channel
]


@pytest.mark.parametrize("case", CH_CASES)
def test_channel_shard_conv(case):
    N, C, H, Co, k, pad, stride = case
    rng = np.random.default_rng(sum(case))
    x = rng.uniform(-1, 1, (C, H, H))
    w = rng.normal(0, 0.3, (Co, C, k, k))
    lay = hl.natural_layout(N, C, H, H)
    assert lay.kind == "channel"
    got, ol, outs = run_conv(N, x, w, pad, stride)
    ref = hl.ref_conv2d(x, w, pad, stride)
    assert got.shape == ref.shape
    assert np.abs(got - ref).max() < 1e-12


@pytest.mark.parametrize("N,C,H", [(128, 1, 16), (128, 2, 16), (128, 3, 16), (64, 2, 16), (32, 2, 16),
                                   (64, 1, 12), (128, 2, 14)])
@pytest.mark.parametrize("fused", [False, True])
def test_channel_shard_pool(N, C, H, fused):
    x = np.random.default_rng(N + C + H).uniform(-1, 1, (C, H, H))
    got, ol, outs = run_pool(N, x, fused=fused)
    assert np.abs(got - hl.ref_avgpool2x2(x)).max() < 1e-12
    if C == 1 and (16 * 16) // N == 2:
        assert ol.kind == "image" and ol.shards == [[0, 0]]   # one channel in two shards: duplicated


def test_channel_shard_stem_then_image_conv():
    """A channel-sharded stem followed by an image-sharded layer (the paper's
    256-px ResNet-50 input needs both kinds)."""
    N = 128
    rng = np.random.default_rng(5)
    x = rng.uniform(-1, 1, (3, 14, 14))
    w1 = rng.normal(0, 0.3, (4, 3, 3, 3))
    w2 = rng.normal(0, 0.3, (4, 4, 3, 3))
    lay = hl.natural_layout(N, 3, 14, 14)
    be = hl.SlotSim(N, QS)
    cts = [(v, 10, 1.0) for v in hl.pack(x, lay)]
    a, al = hl.conv2d(be, cts, lay, w1, pad=1, stride=2)
    assert al.kind == "image"
    b, bl = hl.conv2d(be, a, al, w2, pad=1)
    ref = hl.ref_conv2d(hl.ref_conv2d(x, w1, 1, 2), w2, 1)
    assert np.abs(hl.unpack([o[0] for o in b], bl) - ref).max() < 1e-12


@pytest.mark.parametrize("shape,pool", [((4, 8, 8), False), ((4, 8, 8), True), ((8, 16, 16), True),
                                        ((2, 4, 4), False), ((1, 32, 32), True), ((1, 32, 32), False)])
def test_linear_slot_sim(shape, pool):
    """Linear and pool-linear on cleartext slots equal W @ x (duplicated,
    multi-shard and channel-shard layouts)."""
    N = 256
    rng = np.random.default_rng(sum(shape) + pool)
    x = rng.uniform(-1, 1, shape)
    C, H, W = shape
    O = 5
    Wt = rng.normal(0, 0.1, (O, C) if pool else (O, C * H * W))
    lay = hl.natural_layout(N, C, H, W)
    sim = hl.SlotSim(N, [2.0 ** 40] * 10)
    cts = [(v, 6, 2.0 ** 40) for v in hl.pack(x, lay)]
    out = hl.linear(sim, cts, lay, Wt, pool)
    assert out[1] == 4
    assert np.allclose(out[0][:O], hl.ref_linear(x, Wt, pool), atol=1e-12)
    assert np.allclose(out[0][O:], 0)
