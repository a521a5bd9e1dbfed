"""Checks shared by the GPU tests."""
import sys

import numpy as np

from oracle import he_layers as hl


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()

# a GPU decryption lies within 2^-20 of the oracle's decryption of the same
# ciphertext (both decode the same integers; only the decoders' rounding differs)
DECRYPT_TOL = 2.0 ** -20


def check_decrypt_vs_oracle(img, o, cts):
    """Every shard of a GPU image decrypted on the GPU vs the oracle's
    decryption of the oracle ciphertext of that shard (the two are asserted
    bit-identical by the caller); returns the largest difference."""
    worst = 0.0
    for u, ct in enumerate(cts):
        got = img.shard_decrypt(u)
        ref = o.decrypt(ct)
        d = float(np.abs(got - ref).max())
        assert d <= DECRYPT_TOL, (u, d)
        worst = max(worst, d)
    return worst


def check_ct_decrypt_vs_oracle(ctx, ct, o, oct_):
    d = float(np.abs(ctx.decrypt(ct) - o.decrypt(oct_)).max())
    assert d <= DECRYPT_TOL, d
    return d


def run_pipeline(ctx, prm, o, x, ops, level, seed, mode=0, pad=1, basis=None, tol=1e-5):
    """Encrypt x on both sides, apply ops ('conv', w, stride) / ('pool',),
    compare every shard bit for bit after every op; return final decryption.
    mode 2 runs the convolutions with lazy ModDown on both sides, mode 3 by
    baby and giant steps; modes 1 and 4 compute mode 0's ciphertexts; basis =
    s builds their weight plaintexts in basis-mask form on both sides."""
    C, H, W = x.shape
    img = ctx.image_encrypt(x, level, seed)
    lay = hl.natural_layout(prm.N, C, H, W)
    be = hl.CkksBackend(o, basis=basis)
    cts = [o.encrypt(o.encode(v, level, 2.0 ** ctx.prm.log_scale), seed=seed, index=u)
           for u, v in enumerate(hl.pack(x, lay))]
    for u in range(len(cts)):
        assert (img.shard_export(u) == cts[u].data).all(), "encrypt shard %d" % u
    ref = x
    for op in ops:
        if op[0] == "conv":
            w, stride = op[1], op[2]
            plan = ctx.conv2d_plan(img, w, stride=stride, pad=pad, basis=basis)
            plan.set_mode(mode)
            ctx.gen_rotation_keys(plan.steps())
            img = plan.run(img)
            cts, lay = hl.conv2d(be, cts, lay, w, pad=pad, stride=stride, lazy=(mode == 2), bsgs=(mode == 3))
            ref = hl.ref_conv2d(ref, w, pad, stride)
        else:
            ctx.gen_rotation_keys(ctx.avgpool_steps(img))
            img = ctx.avgpool(img, mode=0 if mode == 1 else mode)
            cts, lay = hl.avgpool2x2(be, cts, lay, lazy=(mode == 2), bsgs=(mode == 3))
            ref = hl.ref_avgpool2x2(ref)
        Cn, Hn, Wn, mp, t = img.info()
        assert t == len(cts) and (Hn, Wn, mp) == (lay.H, lay.W, lay.mp)
        for u in range(t):
            if lay.kind == "channel":
                assert img.channel_shard(u) == tuple(lay.shards[u])
            else:
                assert list(img.block_map(u)) == list(lay.shards[u])
            assert img.shard_info(u) == (cts[u].level, cts[u].scale)
            assert (img.shard_export(u) == cts[u].data).all(), (op[0], u)
        log("  op %s ok: %d shards, level %d" % (op[0], t, cts[0].level))
    got = img.decrypt()
    assert np.abs(got - ref).max() < tol
    check_decrypt_vs_oracle(img, o, cts)
    return got


def prm_log_scale(ctx):
    return ctx.prm.log_scale
