"""GPU library vs the CPU oracle, through the C ABI (MI355X).

Bit-exact: prime chain, encoder integers, keys through encryption, hoisted
and single rotations, rescale, plaintext products, additions, and the full
conv / pool / strided-conv pipelines on several layouts (duplication, image
shards, consolidation with permutation).  Decryptions within 1e-5 of FP64.
Ring sizes span several NTT tiles and the two-pass split.
"""
import sys

import numpy as np
import pytest

from checks import check_ct_decrypt_vs_oracle, check_decrypt_vs_oracle, prm_log_scale, run_pipeline
from oracle import ckks
from oracle import he_layers as hl

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make(logn, L, q0, qb, k, pb, dnum, log_scale, seed):
    from paper_2306_09189_amd import hecnn
    log("ctx logn=%d L=%d k=%d dnum=%d" % (logn, L, k, dnum))
    ctx = hecnn.Context(logn, L, q0, qb, k, pb, dnum, log_scale, device=0)
    prm = ckks.Params(logn, [q0] + [qb] * L, [pb] * k, dnum)
    ctx.keygen(seed)
    return ctx, prm, ckks.Oracle(prm, seed)


@pytest.fixture(scope="module")
def small():
    return make(10, 6, 60, 40, 3, 60, 3, 40, 7)


def test_primes(small):
    ctx, prm, o = small
    assert ctx.primes() == prm.mod


@pytest.mark.parametrize("logn", [10, 13, 16])
def test_encoder_integers(logn):
    from paper_2306_09189_amd import hecnn
    ctx = hecnn.Context(logn, 2, 60, 50, 1, 60, 1, 50, device=0)
    o = ckks.Oracle(ckks.Params(logn, [60, 50, 50], [60], 1), 1)
    rng = np.random.default_rng(logn)
    N = 1 << (logn - 1)
    for scale in (2.0 ** 40, 2.0 ** 50, float(ctx.primes()[2])):
        z = rng.uniform(-1, 1, N)
        assert (ctx.encode_coeffs(z, scale) == o.encode_coeffs(z, scale)).all()
        z = (rng.uniform(0, 1, N) < 0.2) * rng.normal(0, 0.1)
        assert (ctx.encode_coeffs(z, scale) == o.encode_coeffs(z, scale)).all()


def test_import_export_roundtrip(small):
    ctx, prm, o = small
    rng = np.random.default_rng(2)
    lvl = 4
    coeff = np.stack([np.stack([rng.integers(0, q, prm.n, dtype=np.uint64) for q in prm.q[: lvl + 1]])
                      for _ in range(2)])
    ct = ctx.ct_import(coeff, lvl, 2.0 ** 40)
    assert (ct.export() == coeff).all()
    pt = ctx.pt_import(coeff[0], lvl, 3.0)
    assert (pt.export() == coeff[0]).all()


def test_encrypt_decrypt_bit_exact(small):
    ctx, prm, o = small
    z = np.random.default_rng(3).uniform(-1, 1, prm.N)
    for lvl, idx in ((6, 0), (3, 5), (0, 2)):
        pt = ctx.encode(z, lvl, 2.0 ** 40)
        opt = o.encode(z, lvl, 2.0 ** 40)
        assert (pt.export() == opt.limbs).all()
        ct = ctx.encrypt(pt, seed=99, index=idx)
        oct_ = o.encrypt(opt, seed=99, index=idx)
        assert (ct.export() == oct_.data).all()
        assert np.abs(ctx.decrypt(ct) - z).max() < 1e-7


def test_rotations_bit_exact(small):
    ctx, prm, o = small
    z = np.random.default_rng(4).uniform(-1, 1, prm.N)
    steps = [1, 2, 3, 17, prm.N - 1, -5, 0, 100, 511]
    ctx.gen_rotation_keys(steps)
    for lvl in (6, 4, 2, 0):
        opt = o.encode(z, lvl, 2.0 ** 40)
        oct_ = o.encrypt(opt, seed=5, index=lvl)
        ct = ctx.ct_import(oct_.data, lvl, 2.0 ** 40)
        rots = ctx.rotate_hoisted(ct, steps)
        orots = o.rotate_hoisted(oct_, steps)
        for s, r, orr in zip(steps, rots, orots):
            assert (r.export() == orr.data).all(), (lvl, s)
        single = ctx.rotate(ct, 17)
        assert (single.export() == orots[3].data).all()
        assert np.abs(ctx.decrypt(rots[0]) - np.roll(z, -1)).max() < 1e-6


def test_missing_key_is_reported(small):
    from paper_2306_09189_amd import hecnn
    ctx, prm, o = small
    ct = ctx.encrypt(ctx.encode(np.zeros(4), 2, 2.0 ** 40), seed=1)
    with pytest.raises(hecnn.HecError) as e:
        ctx.rotate(ct, 9)
    assert e.value.status == hecnn.HEC_ENOKEY


def test_rescale_mul_add_bit_exact(small):
    from paper_2306_09189_amd import hecnn
    ctx, prm, o = small
    rng = np.random.default_rng(6)
    z, w = rng.uniform(-1, 1, prm.N), rng.uniform(-1, 1, prm.N)
    lvl = 5
    oct_ = o.encrypt(o.encode(z, lvl, 2.0 ** 40), seed=8)
    opt = o.encode(w, lvl, float(prm.q[lvl]))
    ct = ctx.ct_import(oct_.data, lvl, 2.0 ** 40)
    pt = ctx.pt_import(opt.limbs, lvl, float(prm.q[lvl]))
    prod = ctx.mul_pt(ct, pt)
    oprod = o.mul_pt(oct_, opt)
    assert (prod.export() == oprod.data).all()
    s = ctx.add(prod, prod)
    assert (s.export() == o.add(oprod, oprod).data).all()
    ctx.rescale(prod)
    ores = o.rescale(oprod)
    assert (prod.export() == ores.data).all()
    assert prod.level == lvl - 1 and prod.scale == ores.scale
    assert np.abs(ctx.decrypt(prod) - z * w).max() < 1e-6
    with pytest.raises(hecnn.HecError) as e:
        ctx.add(prod, ct)
    assert e.value.status == hecnn.HEC_ELEVEL


@pytest.mark.parametrize("shape,ops", [
    ((4, 8, 8), [("conv", (4, 3), 1), ("pool",)]),                  # d = 2 copies, pool -> dup x4
    ((4, 16, 16), [("conv", (4, 3), 1), ("pool",)]),                # 2 image shards -> consolidate + dup x2
    ((8, 16, 16), [("pool",), ("conv", (8, 3), 1)]),                # 4 shards -> 1 permuted, then conv
    ((16, 16, 16), [("conv", (8, 3), 1), ("pool",)]),               # 8 shards -> 4 -> 1 shard
    ((4, 16, 16), [("conv", (8, 3), 2)]),                           # strided conv: 4 shards -> 1
    ((3, 12, 12), [("conv", (5, 3), 1)]),                           # padding of side and channels
    # channel shards (N = 512 slots): a 32x32 channel spans 2 shards, 64x64 spans 8
    ((2, 32, 32), [("conv", (3, 3), 1), ("pool",)]),                # 6 shards -> groups of 4 + short group
    ((1, 32, 32), [("conv", (1, 3), 1), ("pool",)]),                # one channel in two shards: dup x2
    ((3, 28, 28), [("conv", (4, 3), 2), ("conv", (4, 3), 1)]),      # strided stem, then image shards
    ((1, 64, 64), [("pool",), ("conv", (2, 3), 1)]),                # 8 shards/channel -> 2 shards/channel
    ((4, 16, 16), [("conv", (32, 3), 1)]),                          # 16 outputs: two groups of 8 per launch
])
def test_layers_bit_exact(small, shape, ops):
    ctx, prm, o = small
    rng = np.random.default_rng(sum(shape))
    x = rng.uniform(-1, 1, shape)
    cin = shape[0]
    real_ops = []
    for op in ops:
        if op[0] == "conv":
            co, k = op[1]
            real_ops.append(("conv", rng.normal(0, 0.1, (co, cin, k, k)), op[2]))
            cin = co
        else:
            real_ops.append(op)
    log("layers", shape, [op[0] for op in ops])
    run_pipeline(ctx, prm, o, x, real_ops, 6, seed=31)


@pytest.mark.parametrize("shape,ops", [
    ((4, 8, 8), [("conv", (4, 3), 1)]),                             # one shard, duplicated copies
    ((16, 16, 16), [("conv", (8, 3), 1)]),                          # 8 input shards -> 4 outputs
    ((4, 16, 16), [("conv", (16, 3), 1)]),                          # 2 shards -> 8 outputs
    ((4, 16, 16), [("conv", (8, 3), 2)]),                           # strided conv, 4 shards -> 1
    ((2, 32, 32), [("conv", (3, 3), 1)]),                           # channel shards
    ((8, 16, 16), [("pool",), ("conv", (8, 3), 1)]),                # 4 shards pooled (permuted blocks), then conv
    ((4, 16, 16), [("conv", (4, 3), 1), ("pool",)]),                # 2 shards pooled -> consolidate + dup x2
    ((16, 16, 16), [("conv", (8, 3), 1), ("pool",)]),               # 8 shards -> 4 -> 1
    ((1, 64, 64), [("pool",), ("conv", (2, 3), 1)]),                # channel shards: pooled per shard
    ((4, 8, 8), [("pool",), ("pool",)]),                            # the second pool fused (one level)
])
def test_layers_key_stationary_bit_exact(small, shape, ops):
    """Plan and pooling mode 4 (rotations of all input shards amount by
    amount, each key read once for all shards) give the ciphertexts of mode
    0: compared with the oracle's per-rotation form bit for bit."""
    ctx, prm, o = small
    rng = np.random.default_rng(sum(shape) + 400)
    x = rng.uniform(-1, 1, shape)
    cin = shape[0]
    real_ops = []
    for op in ops:
        if op[0] == "conv":
            co, k = op[1]
            real_ops.append(("conv", rng.normal(0, 0.1, (co, cin, k, k)), op[2]))
            cin = co
        else:
            real_ops.append(op)
    log("key-stationary layers", shape, [op[0] for op in ops])
    run_pipeline(ctx, prm, o, x, real_ops, 6, seed=53, mode=4)


@pytest.mark.parametrize("shape,ops", [
    ((4, 8, 8), [("conv", (4, 3), 1)]),                             # one shard, duplicated copies
    ((4, 16, 16), [("conv", (16, 3), 1), ("pool",)]),               # 2 shards -> 8 outputs (two groups of 4)
    ((16, 16, 16), [("conv", (8, 3), 1)]),                          # 8 input shards -> 4 outputs
    ((4, 16, 16), [("conv", (8, 3), 2)]),                           # strided conv
    ((2, 32, 32), [("conv", (3, 3), 1), ("pool",)]),                # channel shards
    ((3, 28, 28), [("conv", (4, 3), 2), ("conv", (4, 3), 1)]),      # strided stem in channel shards
    ((8, 16, 16), [("pool",), ("conv", (8, 3), 1)]),                # 4 shards pooled -> 1 permuted
    ((1, 64, 64), [("pool",), ("conv", (2, 3), 1)]),                # 8 channel shards pooled
    ((4, 8, 8), [("pool",), ("pool",)]),                            # the second pool fused (one level)
])
def test_layers_lazy_moddown_bit_exact(small, shape, ops):
    ctx, prm, o = small
    rng = np.random.default_rng(sum(shape) + 100)
    x = rng.uniform(-1, 1, shape)
    cin = shape[0]
    real_ops = []
    for op in ops:
        if op[0] == "conv":
            co, k = op[1]
            real_ops.append(("conv", rng.normal(0, 0.1, (co, cin, k, k)), op[2]))
            cin = co
        else:
            real_ops.append(op)
    log("lazy layers", shape, [op[0] for op in ops])
    level = 3 if ops == [("pool",), ("pool",)] else 6
    run_pipeline(ctx, prm, o, x, real_ops, level, seed=37, mode=2)


@pytest.mark.parametrize("shape,ops", [
    ((4, 8, 8), [("conv", (4, 3), 1)]),                             # one shard, duplicated copies
    ((4, 16, 16), [("conv", (16, 3), 1), ("pool",)]),               # 2 shards -> 8 outputs: 72 (giant, output) sums
    ((16, 16, 16), [("conv", (8, 3), 1)]),                          # 8 input shards summed before the giant steps
    ((4, 16, 16), [("conv", (8, 3), 2)]),                           # strided conv
    ((2, 32, 32), [("conv", (3, 3), 1), ("pool",)]),                # channel shards: baby 0 only
    ((3, 28, 28), [("conv", (4, 3), 2), ("conv", (4, 3), 1)]),      # strided stem in channel shards
    ((3, 12, 12), [("conv", (5, 5), 1)]),                           # 5x5 kernel, padded channels
    ((8, 16, 16), [("pool",), ("conv", (8, 3), 1)]),                # 4 shards pooled by baby/giant steps
    ((1, 64, 64), [("pool",), ("conv", (2, 3), 1)]),                # channel shards pooled
    ((4, 8, 8), [("pool",), ("pool",)]),                            # the second pool fused (one level)
])
def test_layers_bsgs_bit_exact(small, shape, ops):
    ctx, prm, o = small
    rng = np.random.default_rng(sum(shape) + 200)
    x = rng.uniform(-1, 1, shape)
    cin = shape[0]
    real_ops = []
    for op in ops:
        if op[0] == "conv":
            co, k = op[1]
            real_ops.append(("conv", rng.normal(0, 0.1, (co, cin, k, k)), op[2]))
            cin = co
        else:
            real_ops.append(op)
    log("bsgs layers", shape, [op[0] for op in ops])
    pad = 2 if shape == (3, 12, 12) else 1
    level = 3 if ops == [("pool",), ("pool",)] else 6
    run_pipeline(ctx, prm, o, x, real_ops, level, seed=43, mode=3, pad=pad)


def test_lazy_zero_rotation_only(small):
    """A 1x1 convolution of one channel per shard needs only the zero
    rotation: the lazy path must then equal the batched path bit for bit."""
    ctx, prm, o = small
    rng = np.random.default_rng(12)
    x = rng.uniform(-1, 1, (1, 16, 16))
    w = rng.normal(0, 0.3, (1, 1, 1, 1))
    got = run_pipeline(ctx, prm, o, x, [("conv", w, 1)], 5, seed=41, mode=2, pad=0)
    img = ctx.image_encrypt(x, 5, 41)
    plan = ctx.conv2d_plan(img, w, pad=0)
    assert plan.steps() == []
    a = plan.run(img)
    plan.set_mode(2)
    b = plan.run(img)
    assert (a.shard_export(0) == b.shard_export(0)).all()
    assert np.abs(got - b.decrypt()).max() == 0


def test_plan_mode_rejected(small):
    from paper_2306_09189_amd import hecnn
    ctx, prm, o = small
    img = ctx.image_encrypt(np.zeros((1, 8, 8)), 3, 1)
    plan = ctx.conv2d_plan(img, np.ones((1, 1, 3, 3)))
    for bad in (5, -1):
        with pytest.raises(hecnn.HecError) as e:
            plan.set_mode(bad)
        assert e.value.status == hecnn.HEC_EINVAL
    for bad in (1, 5):
        with pytest.raises(hecnn.HecError) as e:
            ctx.avgpool(img, mode=bad)
        assert e.value.status == hecnn.HEC_EINVAL


def test_plain_equals_batched(small):
    ctx, prm, o = small
    rng = np.random.default_rng(9)
    x = rng.uniform(-1, 1, (8, 16, 16))
    w = rng.normal(0, 0.1, (8, 8, 3, 3))
    img = ctx.image_encrypt(x, 5, 3)
    plan = ctx.conv2d_plan(img, w)
    ctx.gen_rotation_keys(plan.steps())
    a = plan.run(img)
    plan.set_mode(1)
    b = plan.run(img)
    for u in range(a.info()[4]):
        assert (a.shard_export(u) == b.shard_export(u)).all()


def test_ring_2e13_conv_pool():
    """2N = 2^13, q 3 x 40-bit, one 60-bit special prime, scale 2^40: one
    32x32x4 image, 3x3 conv 4->4 (stride 1, pad 1), then 2x2 average pooling
    fused into one level; bit-exact with the oracle, 1e-5 against FP64."""
    ctx, prm, o = make(13, 2, 40, 40, 1, 60, 3, 40, 2001)
    rng = np.random.default_rng(1001)
    x = rng.uniform(-1, 1, (4, 32, 32))
    w = rng.normal(0, 0.1, (4, 4, 3, 3))
    run_pipeline(ctx, prm, o, x, [("conv", w, 1), ("pool",)], 2, seed=3001)
    run_pipeline(ctx, prm, o, x, [("conv", w, 1), ("pool",)], 2, seed=3002, mode=2)


@pytest.mark.parametrize("shape,pool,O", [((4, 8, 8), False, 3), ((4, 8, 8), True, 5), ((8, 16, 16), True, 10),
                                          ((1, 32, 32), True, 4),
                                          ((8, 16, 16), True, 20)])   # outputs rotated in two key-switch batches
def test_linear_bit_exact(small, shape, pool, O):
    """Linear and pool-linear layers (rotate-and-add dot products) bit-exact
    with the oracle; decrypted within 1e-5 of W @ x."""
    ctx, prm, o = small
    rng = np.random.default_rng(sum(shape) + O)
    x = rng.uniform(-1, 1, shape)
    C, H, W = shape
    Wt = rng.normal(0, 0.1, (O, C) if pool else (O, C * H * W))
    img = ctx.image_encrypt(x, 5, 47)
    ctx.gen_rotation_keys(ctx.linear_steps(img))
    out = ctx.linear(img, Wt, pool)
    lay = hl.natural_layout(prm.N, C, H, W)
    cts = [o.encrypt(o.encode(v, 5, 2.0 ** prm_log_scale(ctx)), seed=47, index=u)
           for u, v in enumerate(hl.pack(x, lay))]
    ref = hl.linear(hl.CkksBackend(o), cts, lay, Wt, pool)
    assert out.info() == (ref.level, ref.scale)
    assert (out.export() == ref.data).all()
    got = ctx.decrypt(out)
    assert np.abs(got[:O] - hl.ref_linear(x, Wt, pool)).max() < 1e-5


@pytest.mark.parametrize("shape,ops,pad,mode", [
    ((2, 8, 16), [("conv", (3, 3), 1), ("pool",)], 1, 0),           # non-square image
    ((2, 16, 8), [("conv", (2, 3), 1), ("pool",)], 1, 3),           # tall image, baby/giant steps
    ((4, 8, 8), [("conv", (4, 1), 1)], 0, 0),                       # 1x1 kernel (Eq. (2) channel mixing)
    ((4, 8, 8), [("conv", (4, 1), 1)], 0, 3),
    ((3, 8, 8), [("conv", (2, 3), 1)], 0, 2),                       # no padding
    ((1, 2, 2), [("pool",)], 1, 0),                                 # smallest image: pools to one pixel
    ((1, 2, 2), [("pool",)], 1, 3),
    ((5, 6, 6), [("conv", (3, 5), 1), ("pool",)], 2, 2),            # 5x5 kernel, pad 2, odd channel count
])
def test_layers_edge_shapes_bit_exact(small, shape, ops, pad, mode):
    """Degenerate and ragged shapes in every evaluation mode: bit for bit with the oracle."""
    ctx, prm, o = small
    rng = np.random.default_rng(sum(shape) + 7 * mode + pad)
    x = rng.uniform(-1, 1, shape)
    cin = shape[0]
    real_ops = []
    for op in ops:
        if op[0] == "conv":
            co, k = op[1]
            real_ops.append(("conv", rng.normal(0, 0.1, (co, cin, k, k)), op[2]))
            cin = co
        else:
            real_ops.append(op)
    log("edge", shape, [op[0] for op in ops], "pad", pad, "mode", mode)
    run_pipeline(ctx, prm, o, x, real_ops, 6, seed=41, mode=mode, pad=pad)


@pytest.mark.parametrize("shape,ops,mode", [
    ((4, 16, 16), [("conv", (4, 3), 1), ("pool",)], 0),             # 2 shards of 2 blocks -> 2 outputs
    ((4, 16, 16), [("conv", (4, 3), 1)], 1),                        # per rotation, unbatched
    ((4, 16, 16), [("conv", (2, 3), 1)], 2),                        # lazy, one output shard
    ((4, 16, 16), [("conv", (4, 3), 1), ("pool",)], 2),             # lazy, two outputs
    ((4, 16, 16), [("conv", (16, 3), 1)], 2),                       # lazy, 8 outputs (wide kernel)
    ((16, 16, 16), [("conv", (8, 3), 1)], 0),                       # 8 inputs -> 4 outputs, batched
    ((16, 16, 16), [("conv", (8, 3), 1)], 2),
    ((4, 16, 16), [("conv", (8, 3), 2)], 2),                        # strided
    ((2, 32, 32), [("pool",), ("conv", (4, 3), 1)], 0),             # channel shards pooled, then basis conv
    ((4, 16, 16), [("conv", (32, 3), 1)], 0),                       # 16 outputs: two groups of 8 per launch
    ((4, 16, 16), [("conv", (48, 3), 1)], 2),                       # 24 outputs: two lazy passes over the terms
])
def test_basis_plan_bit_exact(small, shape, ops, mode):
    """Weight plaintexts in basis-mask form (tap masks per block encoded at
    2^20, weights rounded at q_l / 2^20) bit for bit with the oracle building
    the same integer plaintexts, in the batched, plain and lazy modes.  With
    40-bit primes the form itself is coarse: per product the weight is off by
    up to 2^19 / q_l ~ 5e-7 and the mask by the decoded rounding of its
    encoding, ~ sqrt(n/2) * 0.3 * 2^-20 ~ 6e-6 RMS, so the decrypted
    convolution is held to 5e-5 instead of 1e-5 (the 50-bit primes of the
    2^16 parameters at 2^28 meet 1e-5)."""
    ctx, prm, o = small
    rng = np.random.default_rng(sum(shape) + 300 + mode)
    x = rng.uniform(-1, 1, shape)
    cin = shape[0]
    real_ops = []
    for op in ops:
        if op[0] == "conv":
            co, k = op[1]
            real_ops.append(("conv", rng.normal(0, 0.1, (co, cin, k, k)), op[2]))
            cin = co
        else:
            real_ops.append(op)
    log("basis layers", shape, [op[0] for op in ops], mode)
    run_pipeline(ctx, prm, o, x, real_ops, 6, seed=41, mode=mode, basis=20, tol=5e-5)


def test_basis_plan_errors(small):
    """Basis-mask plans refuse mode 3, more than 2 blocks per shard, channel
    shards and the Q-only flag."""
    from paper_2306_09189_amd import hecnn
    ctx, prm, o = small
    rng = np.random.default_rng(78)
    w = rng.normal(0, 0.1, (4, 4, 3, 3))
    img = ctx.image_encrypt(rng.uniform(-1, 1, (4, 16, 16)), 6, 78)
    plan = ctx.conv2d_plan(img, w, basis=20)
    with pytest.raises(hecnn.HecError):
        plan.set_mode(3)
    with pytest.raises(hecnn.HecError):
        ctx.conv2d_plan(img, w, basis=20, q_only=True)
    with pytest.raises(hecnn.HecError):
        ctx.conv2d_plan(img, w, basis=0)
    small_img = ctx.image_encrypt(rng.uniform(-1, 1, (4, 8, 8)), 6, 79)    # 8 blocks of 64 slots (at most 2)
    with pytest.raises(hecnn.HecError):
        ctx.conv2d_plan(small_img, w, basis=20)
    ch_img = ctx.image_encrypt(rng.uniform(-1, 1, (1, 32, 32)), 6, 80)     # one channel in two shards
    with pytest.raises(hecnn.HecError):
        ctx.conv2d_plan(ch_img, rng.normal(0, 0.1, (1, 1, 3, 3)), basis=20)


def test_q_only_plan(small):
    """A plan whose weight plaintexts are kept over Q only gives the same
    ciphertexts as a full plan in modes 0, 1 and 4 (the products follow
    complete rotations) and refuses modes 2 and 3 (products over Q*P)."""
    from paper_2306_09189_amd import hecnn
    ctx, prm, o = small
    rng = np.random.default_rng(77)
    x = rng.uniform(-1, 1, (4, 16, 16))
    w = rng.normal(0, 0.1, (4, 4, 3, 3))
    img = ctx.image_encrypt(x, 6, 77)
    full = ctx.conv2d_plan(img, w)
    qo = ctx.conv2d_plan(img, w, q_only=True)
    ctx.gen_rotation_keys(full.steps())
    assert qo.steps() == full.steps()
    a = full.run(img)
    for mode in (0, 1, 4):
        qo.set_mode(mode)
        b = qo.run(img)
        for u in range(a.info()[-1]):
            assert (a.shard_export(u) == b.shard_export(u)).all()
    for mode in (2, 3):
        with pytest.raises(hecnn.HecError):
            qo.set_mode(mode)


@pytest.mark.parametrize("shape,co,mode,dsm", [
    ((4, 16, 16), 8, 4, 2),    # image shards: key-stationary conv, lazy downsampling
    ((4, 16, 16), 8, 0, 2),    # batched conv, lazy downsampling
    ((4, 16, 16), 8, 2, 0),    # lazy conv, downsampling by complete rotations
    ((3, 28, 28), 4, 4, 2),    # channel shards (a stem): key-stationary conv, lazy downsampling
    ((8, 16, 16), 8, 0, 4),    # batched conv, key-stationary downsampling
])
def test_strided_downsample_mode_bit_exact(small, shape, co, mode, dsm):
    """A stride-2 plan whose downsampling step takes its own form: the oracle's
    stride-1 convolution in the plan's form followed by its downsampling in
    the chosen form (Section 4.1: strided convolution = convolution, then the
    pooling's downsampling), every shard bit for bit."""
    from paper_2306_09189_amd import hecnn
    ctx, prm, o = small
    rng = np.random.default_rng(400 + 10 * mode + dsm + shape[0])
    x = rng.uniform(-1, 1, shape)
    w = rng.normal(0, 0.1, (co, shape[0], 3, 3))
    level, seed = 6, 4100 + mode
    img = ctx.image_encrypt(x, level, seed)
    plan = ctx.conv2d_plan(img, w, stride=2)
    plan.set_mode(mode)
    plan.set_downsample_mode(dsm)
    ctx.gen_rotation_keys(plan.steps())
    out = plan.run(img)
    lay = hl.natural_layout(prm.N, *shape)
    be = hl.CkksBackend(o)
    cts = [o.encrypt(o.encode(v, level, 2.0 ** 40), seed=seed, index=u) for u, v in enumerate(hl.pack(x, lay))]
    oc, ol = hl.conv2d(be, cts, lay, w, pad=1, stride=1, lazy=(mode == 2))
    dc, dl = hl.downsample_and_merge(be, oc, ol, select=True, lazy=(dsm == 2))
    assert out.info()[4] == len(dc)
    for u in range(len(dc)):
        assert out.shard_info(u) == (dc[u].level, dc[u].scale)
        assert (out.shard_export(u) == dc[u].data).all(), u
    assert np.abs(out.decrypt() - hl.ref_conv2d(x, w, 1, 2)).max() < 1e-5
    check_decrypt_vs_oracle(out, o, dc)
    with pytest.raises(hecnn.HecError):
        plan.set_downsample_mode(3)
    with pytest.raises(hecnn.HecError):
        ctx.conv2d_plan(img, w).set_downsample_mode(2)   # stride 1: no downsampling


def test_release_cached_keeps_results(small):
    """Giving the pools' cached blocks back to the device (hec_ctx_release_cached)
    changes nothing that is computed afterwards."""
    ctx, prm, o = small
    rng = np.random.default_rng(808)
    x = rng.uniform(-1, 1, (4, 16, 16))
    w = rng.normal(0, 0.1, (4, 4, 3, 3))
    img = ctx.image_encrypt(x, 5, 808)
    plan = ctx.conv2d_plan(img, w)
    ctx.gen_rotation_keys(plan.steps())
    a = plan.run(img)
    first = [a.shard_export(u) for u in range(a.info()[4])]
    del a
    ctx.release_cached()
    b = plan.run(img)
    assert all((b.shard_export(u) == f).all() for u, f in enumerate(first))
