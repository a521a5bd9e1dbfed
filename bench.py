"""Benchmark: key-switched rotations/s and HE conv-layer ms at 2N = 2^16.

Workload (one step): the 32x32x32 image at level 20 of ring 2N = 2^16
(q_0 60-bit + 24 x 50-bit primes, 8 x 60-bit special primes, dnum = 3,
scale 2^50) is encoded and encrypted, convolved 3x3 32->32 (stride 1,
pad 1), convolved 3x3 32->64 with stride 2 (two output shards, downsampling,
consolidation into one ciphertext, duplication x2), and decrypted.  Inputs
and weights are synthetic and seeded: x ~ U[-1, 1], w ~ N(0, 0.05^2).
The weight plaintexts of both layers are encoded once before timing (they
are model parameters, resident in HBM like the rotation keys).

One JSON line on stdout; everything else on stderr.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

LOGN, L, Q0, QB, K, PB, DNUM, LOG_SCALE = 16, 24, 60, 50, 8, 60, 3, 50
LEVEL = 20


def eprint(*a):
    print(*a, file=sys.stderr, flush=True)


# Dominant kernel of the timed step (largest share of GPU time in a rocprofv3
# kernel trace of this command), per plan mode.
#  * lazy ModDown (mode 2): the fused key-switch + weight-product kernel
#    k_ks_mac.  It streams the rotation keys and plaintexts once; its work unit
#    is one limb (2^16 words = 512 KiB) moved to or from HBM, counting every key,
#    plaintext and accumulator limb once and the hoisted digits and the input
#    ciphertext once per launch.  Bound: HBM, 8 TB/s.
#  * batched / plain (modes 0, 1): the row pass of the 2^16 forward NTT.  One
#    unit = one limb, 8 butterfly stages x 2^15 butterflies (one modular
#    multiplication each), 2 x 512 KiB moved.  Bound: the VALU.  256 CUs x 64
#    lanes x 2.4 GHz = 39.3 T lane-instructions/s (the fp64 FMA rate, 78.6
#    TFLOP/s / 2; 64-bit integer multiply-add issues at the same rate on gfx950);
#    a 64-bit Shoup modular multiplication needs 10 integer multiply
#    instructions -> 3.93 T modmul/s.
LIMB_BYTES = 8 << LOGN
KERNELS = {
    "k_ks_mac": {"bound": "hbm", "unit": "GB/s", "peak": 8000.0, "per_unit": LIMB_BYTES / 1e9,
                 "bytes_per_unit": LIMB_BYTES,
                 "traffic_file": os.path.join(ROOT, "profiles", "ks_mac_2e16_traffic.txt")},
    "k_ntt16_fwd_rows": {"bound": "alu", "unit": "Tmodmul/s", "peak": 256 * 64 * 2.4e9 / 10 / 1e12,
                         "per_unit": 8 * (1 << 15) / 1e12, "bytes_per_unit": 2 * LIMB_BYTES,
                         "traffic_file": os.path.join(ROOT, "profiles", "ntt16_fwd_rows_2e16_traffic.txt")},
}
DOMINANT = {0: "k_ntt16_fwd_rows", 1: "k_ntt16_fwd_rows", 2: "k_ks_mac", 3: "k_ks_mac"}


def read_traffic(path):
    """key: value lines of a committed PMC summary (None if absent)."""
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            rec[k.strip()] = v.strip()
    return rec


# source regions whose text decides a kernel's code: the modular helpers and
# the kernel itself with its launcher (a change elsewhere in the file leaves a
# recorded PMC measurement valid)
SOURCE_REGIONS = {
    "k_ks_mac": ("typedef u64 u64x2 __attribute__((ext_vector_type(2)));", "__global__ void k_moddown_combine("),
    "k_ntt16_fwd_rows": ("// NTT: merged Cooley-Tukey forward transform", "void hec_ntt_fwd("),
}


def kernel_source_sha(kernel):
    import hashlib
    src = open(os.path.join(ROOT, "paper_2306_09189_amd", "csrc", "hec_kernels.hip")).read()
    h0 = src.index("DEV u64 add_mod(")
    h1 = src.index("// NTT: merged Cooley-Tukey forward transform")
    a, b = SOURCE_REGIONS[kernel]
    i = src.index(a)
    j = src.index(b, i)
    return hashlib.sha256((src[h0:h1] + src[i:j]).encode()).hexdigest()[:16]


def dominant_roofline(kernel, launches, units, kms):
    if not launches or kms <= 0:
        return None
    spec = KERNELS[kernel]
    avg_units = units / launches
    avg_s = kms / launches * 1e-3
    achieved = avg_units * spec["per_unit"] / avg_s
    traffic = None
    rec = read_traffic(spec["traffic_file"])
    if rec and rec.get("source_sha") == kernel_source_sha(kernel):
        traffic = (float(rec["fetch_bytes_per_unit"]) + float(rec["write_bytes_per_unit"])) * avg_units
    return {"bound": spec["bound"], "kernel": kernel, "achieved": achieved, "peak": spec["peak"],
            "unit": spec["unit"], "frac": achieved / spec["peak"], "traffic": traffic,
            "avg_launch_us": avg_s * 1e6, "launches": launches, "avg_units_per_launch": avg_units,
            "algorithmic_bytes_per_launch": avg_units * spec["bytes_per_unit"]}


def rotations_per_step():
    # conv1: 32 channel offsets x 9 taps - the zero rotation; conv2 the same;
    # downsampling of 2 shards: 15 horizontal + 15 vertical each; consolidate 1; duplicate 1
    return 287 + 287 + 2 * 30 + 1 + 1


def cpu_baseline(n_rot, seconds, mode):
    """The CPU oracle (plain C, __int128 arithmetic, OpenMP over limbs) on a
    bounded sample of the same work as the timed step, repeated until `seconds`
    of CPU work; keys and weight plaintexts prepared outside the timed part.
    Modes 0/1: batches of n_rot hoisted key-switched rotations of one level-20
    ciphertext, each multiplied by a weight plaintext and summed.  Mode 2 (lazy
    ModDown): the key-switch products of n_rot rotations multiplied by the
    weights over Q*P, summed, and one ModDown."""
    from oracle import ckks
    prm = ckks.Params(LOGN, [Q0] + [QB] * L, [PB] * K, DNUM)
    o = ckks.Oracle(prm, 2002)
    steps = list(range(1, n_rot + 1))
    for s in steps:
        o.swk(prm.galois(s))
    rng = np.random.default_rng(0)
    ct = o.encrypt(o.encode(rng.uniform(-1, 1, prm.N), LEVEL, 2.0 ** LOG_SCALE), seed=1)
    qlev = float(prm.q[LEVEL])
    ms = [o.encode_coeffs(rng.normal(0, 0.05, prm.N), qlev) for _ in steps]
    qi, qpi = list(range(LEVEL + 1)), o.qp_index(LEVEL)
    if mode == 2:
        pts = [o.limbs_qp(m, LEVEL) for m in ms]

        def work():
            acc = None
            for e, pt in zip(o.keyswitch_raw(ct, steps), pts):
                prod = np.stack([o.mul_limbs(qpi, pt, e[p]) for p in range(2)])
                acc = prod if acc is None else np.stack([o.add_limbs(qpi, acc[p], prod[p]) for p in range(2)])
            return [o.moddown(LEVEL, acc[p]) for p in range(2)]
        what = "lazy-ModDown key-switch products x weights summed over Q*P, one ModDown"
    else:
        pts = [o.limbs_of(m, LEVEL) for m in ms]

        def work():
            acc = None
            for r, pt in zip(o.rotate_hoisted(ct, steps), pts):
                prod = np.stack([o.mul_limbs(qi, pt, r.data[p]) for p in range(2)])
                acc = prod if acc is None else np.stack([o.add_limbs(qi, acc[p], prod[p]) for p in range(2)])
            return acc
        what = "hoisted key-switched rotations x weights summed"
    t = time.perf_counter()
    reps = 0
    while True:
        work()
        reps += 1
        dt = time.perf_counter() - t
        if dt >= seconds:
            break
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": reps * n_rot / dt, "unit": "key-switched rotations/s", "cores": cores, "kind": "oracle",
            "sample": "%d x %d rotations of one level-20 ciphertext (%s), 2N=2^16, dnum=3, OpenMP over limbs "
                      "(%.1f s)" % (reps, n_rot, what, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-rotations", type=int, default=12)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--plain-reps", type=int, default=2)
    ap.add_argument("--mode", type=int, default=2, choices=(0, 1, 2, 3),
                    help="plan mode of the timed step: 0 batched, 1 plain, 2 lazy ModDown, "
                         "3 baby-step/giant-step with double hoisting")
    ap.add_argument("--pmc-run", action="store_true", help="short workload for rocprofv3 --pmc passes")
    ap.add_argument("--profile-run", choices=("gelu", "block"),
                    help="for kernel traces: five degree-59 GELU evaluations on one level-20 ciphertext, or five "
                         "runs of the 16x32x32 block, then exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        eprint("bench.py measures one GPU: the whole path runs on a single MI355X "
               "(sharding across GPUs is described, not implemented); use --gpus 1")
        sys.exit(2)

    import torch
    from paper_2306_09189_amd import hecnn

    torch.cuda.init()
    stream = torch.cuda.current_stream()
    ctx = hecnn.Context(LOGN, L, Q0, QB, K, PB, DNUM, LOG_SCALE, device=0, stream=stream.cuda_stream)
    rng = np.random.default_rng(1002)
    x = rng.uniform(-1, 1, (32, 32, 32))
    w1 = rng.normal(0, 0.05, (32, 32, 3, 3))
    w2 = rng.normal(0, 0.05, (64, 32, 3, 3))
    if args.profile_run:
        from numpy.polynomial import chebyshev as Cheb

        def gelu_f(v):
            return 0.5 * v * (1.0 + np.tanh(np.sqrt(2.0 / np.pi) * (v + 0.044715 * v ** 3)))
        coef = Cheb.chebinterpolate(lambda y: gelu_f(15.0 * y), 59)
        ctx.keygen(2002)
        if args.profile_run == "gelu":
            ct = ctx.encrypt(ctx.encode(rng.uniform(-1, 1, ctx.N), LEVEL, 2.0 ** LOG_SCALE), 6)
            for _ in range(5):
                r = ctx.cheb_eval(ct, coef, -1.0, 1.0)
                del r
        else:
            xb = rng.uniform(-1, 1, (16, 32, 32))
            wb1, wb2 = rng.normal(0, 1 / 12.0, (16, 16, 3, 3)), rng.normal(0, 1 / 12.0, (16, 16, 3, 3))
            bn = (rng.uniform(0.5, 1.5, 16), rng.normal(0, 0.5, 16))
            imb = ctx.image_encrypt(xb, LEVEL, 7)
            blk = ctx.block(imb, wb1, bn, wb2, bn, 15.0, coef, mode=args.mode if args.mode >= 2 else 2)
            ctx.gen_rotation_keys(blk.steps())
            for _ in range(5):
                ob = blk.run(imb)
                del ob
        ctx.sync()
        eprint("profile run done")
        return
    if args.pmc_run:
        # short run for hardware-counter passes: one conv layer, then a plain
        # device copy of exactly 256 MiB to calibrate the byte counters
        ctx.keygen(2002)
        img = ctx.image_encrypt(x, LEVEL, 3002)
        p1 = ctx.conv2d_plan(img, w1, stride=1, pad=1)
        p1.set_mode(args.mode)
        ctx.gen_rotation_keys(p1.steps())
        dom = DOMINANT[args.mode]
        ctx.prof_start(dom)
        o1 = p1.run(img)
        ctx.sync()
        launches, units, kms = ctx.prof_stop()
        eprint("pmc run: %s launches %d algorithmic units %d (%d bytes each)"
               % (dom, launches, units, KERNELS[dom]["bytes_per_unit"]))
        src = torch.ones(1 << 25, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        eprint("pmc run done", o1.info())
        return
    t0 = time.perf_counter()
    ctx.keygen(2002)
    img = ctx.image_encrypt(x, LEVEL, 3002)
    p1 = ctx.conv2d_plan(img, w1, stride=1, pad=1)
    ctx.gen_rotation_keys(p1.steps())
    o1 = p1.run(img)
    p2 = ctx.conv2d_plan(o1, w2, stride=2, pad=1)
    ctx.gen_rotation_keys(p2.steps())
    ctx.sync()
    setup_s = time.perf_counter() - t0
    eprint("setup %.2f s, rotation keys %.1f GiB" % (setup_s, ctx.key_bytes() / 2 ** 30))
    del o1

    from oracle import he_layers as hl  # FP64 reference for the accuracy check only
    ref = hl.ref_conv2d(hl.ref_conv2d(x, w1, 1, 1), w2, 1, 2)

    def step(check=False):
        im = ctx.image_encrypt(x, LEVEL, 3002)
        a = p1.run(im)
        b = p2.run(a)
        y = b.decrypt()
        if check:
            return float(np.abs(y - ref).max())
        return None

    p1.set_mode(args.mode)
    p2.set_mode(args.mode)
    for _ in range(args.warmup):
        step()
    err = step(check=True)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # the dominant kernel is timed launch by launch with HIP events on the
    # library's stream during the timed steps
    dom = DOMINANT[args.mode]
    ctx.prof_start(dom)
    first_launch = ctx.prof_launches(dom)
    ks0 = ctx.keyswitch_count()
    t = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    launches, units, kms = ctx.prof_stop()
    ms_step = wall * 1e3 / args.steps
    # key-switch inner products actually computed in the timed steps (636 per
    # step in modes 0-2; fewer in mode 3, which trades rotations for giant steps)
    ks_step = (ctx.keyswitch_count() - ks0) / args.steps
    value = ks_step * args.steps / wall
    roofline = dominant_roofline(dom, launches, units, kms)
    if roofline:
        # dispatch range of the timed region in a kernel trace of this same command
        roofline["trace_dispatch_range"] = [first_launch, first_launch + launches]

    # conv-layer latency (conv 3x3 32->32) in each plan mode: batched (hoisted
    # ModUp, 16 rotations per key-switch launch), plain (one launch chain per
    # rotation) and lazy ModDown (key switch fused with the weight products)
    def conv_ms(mode, reps):
        p1.set_mode(mode)
        im = ctx.image_encrypt(x, LEVEL, 3002)
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            s = time.perf_counter()
            o = p1.run(im)
            ctx.sync()
            ts.append((time.perf_counter() - s) * 1e3)
            del o
        p1.set_mode(args.mode)
        return float(np.median(ts))

    conv_b = conv_ms(0, 5)
    conv_p = conv_ms(1, max(1, args.plain_reps))
    conv_l = conv_ms(2, 5)
    conv_g = conv_ms(3, 5)

    # the whole step in the other fast mode (lazy ModDown <-> baby-step/giant-step)
    other = 3 if args.mode != 3 else 2
    p1.set_mode(other)
    p2.set_mode(other)
    step()
    err_other = step(check=True)
    torch.cuda.synchronize()
    k0 = ctx.keyswitch_count()
    s = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms_other = (time.perf_counter() - s) * 1e3 / args.steps
    ks_other = (ctx.keyswitch_count() - k0) / args.steps
    p1.set_mode(args.mode)
    p2.set_mode(args.mode)

    # isolated rotations at level 20
    ctx.gen_rotation_keys(list(range(1, 33)))
    ct = ctx.encrypt(ctx.encode(rng.uniform(-1, 1, ctx.N), LEVEL, 2.0 ** LOG_SCALE), 5)
    ctx.sync()
    s = time.perf_counter()
    for _ in range(3):
        rs = ctx.rotate_hoisted(ct, list(range(1, 33)))
        del rs
    ctx.sync()
    rot_hoisted = 96 / (time.perf_counter() - s)
    s = time.perf_counter()
    for i in range(32):
        r = ctx.rotate(ct, 1 + i)
        del r
    ctx.sync()
    rot_single = 32 / (time.perf_counter() - s)

    # GELU as the degree-59 Chebyshev interpolant over [-15, 15] (its map onto
    # [-1, 1] folded into the input) on one ciphertext at level 20, and the
    # conv -> bias -> GELU -> conv -> pool block on a 16x32x32 CIFAR stage
    from numpy.polynomial import chebyshev as Cheb

    def gelu(v):
        return 0.5 * v * (1.0 + np.tanh(np.sqrt(2.0 / np.pi) * (v + 0.044715 * v ** 3)))
    bound = 15.0
    coef = Cheb.chebinterpolate(lambda y: gelu(bound * y), 59)
    zg = rng.uniform(-1, 1, ctx.N)
    ctg = ctx.encrypt(ctx.encode(zg, LEVEL, 2.0 ** LOG_SCALE), 6)
    ts = []
    for _ in range(5):
        ctx.sync()
        s = time.perf_counter()
        g = ctx.cheb_eval(ctg, coef, -1.0, 1.0)
        ctx.sync()
        ts.append((time.perf_counter() - s) * 1e3)
    gelu_ms = float(np.median(ts))
    gelu_err = float(np.abs(ctx.decrypt(g) - gelu(bound * zg)).max())
    gelu_levels = LEVEL - g.level
    del g, ctg
    xb = rng.uniform(-1, 1, (16, 32, 32))
    wb1, wb2 = rng.normal(0, 1 / 12.0, (16, 16, 3, 3)), rng.normal(0, 1 / 12.0, (16, 16, 3, 3))
    bn1 = (rng.uniform(0.5, 1.5, 16), rng.normal(0, 0.5, 16))
    bn2 = (rng.uniform(0.5, 1.5, 16), rng.normal(0, 0.5, 16))
    imb = ctx.image_encrypt(xb, LEVEL, 7)
    bmode = args.mode if args.mode >= 2 else 2
    blk = ctx.block(imb, wb1, bn1, wb2, bn2, bound, coef, mode=bmode)
    ctx.gen_rotation_keys(blk.steps())
    ts = []
    for _ in range(4):
        ctx.sync()
        k0 = ctx.keyswitch_count()
        s = time.perf_counter()
        ob = blk.run(imb)
        ctx.sync()
        ts.append((time.perf_counter() - s) * 1e3)
        ks_block = ctx.keyswitch_count() - k0
    block_ms = float(np.median(ts[1:]))
    block_err = float(np.abs(ob.decrypt() - hl.ref_basic_block(xb, wb1, bn1, wb2, bn2, bound, coef)).max())
    del ob, blk, imb
    # the classifier head of a CIFAR ResNet: global average pooling of a
    # 64x8x8 stage folded into a 64 -> 10 linear layer (rotate-and-add)
    xl = rng.uniform(-1, 1, (64, 8, 8))
    wl = rng.normal(0, 0.1, (10, 64))
    iml = ctx.image_encrypt(xl, LEVEL, 8)
    ctx.gen_rotation_keys(ctx.linear_steps(iml))
    ts = []
    for _ in range(4):
        ctx.sync()
        s = time.perf_counter()
        ol = ctx.linear(iml, wl, True)
        ctx.sync()
        ts.append((time.perf_counter() - s) * 1e3)
    linear_ms = float(np.median(ts[1:]))
    linear_err = float(np.abs(ctx.decrypt(ol)[:10] - hl.ref_linear(xl, wl, True)).max())
    del ol, iml
    # a 112x112x64 stage of an ImageNet ResNet (32 shards of two padded
    # 128x128 channels): conv 3x3 64->64 with basis-mask weight plaintexts
    # (masks at 2^27), then 2x2 pooling with lazy ModDown; second calls timed
    xi = np.clip(rng.normal(0, 1, (64, 112, 112)), -4, 4)
    wi = rng.normal(0, 0.05, (64, 64, 3, 3))
    imi = ctx.image_encrypt(xi, LEVEL, 9)
    pi = ctx.conv2d_plan(imi, wi, basis=27)
    ctx.gen_rotation_keys(pi.steps())
    ctx.gen_rotation_keys(ctx.avgpool_steps(imi))
    inet = {}
    for name, fn in (("conv", lambda: pi.run(imi)), ("pool", lambda: ctx.avgpool(yi, 2))):
        r = fn()
        ctx.sync()
        del r
        s = time.perf_counter()
        r = fn()
        ctx.sync()
        inet[name] = (time.perf_counter() - s) * 1e3
        if name == "conv":
            yi = r
        else:
            zi = r
    inet_err = float(np.abs(zi.decrypt() - hl.ref_avgpool2x2(hl.ref_conv2d(xi, wi, 1))).max())
    del pi, yi, zi, imi

    out = {
        "metric": "key-switched rotations/sec + HE conv-layer ms at 2N=2^16; batched vs plain",
        "value": value,
        "unit": "key-switched rotations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "2N=2^16, 32x32x32 image at level 20: conv3x3 32->32 s1 + conv3x3 32->64 s2 "
                               "(2 shards -> downsample -> 1 ct), encrypt+decrypt included",
                   "ring_dim": 1 << LOGN, "level": LEVEL, "dnum": DNUM, "special_primes": K,
                   "rotations_per_step": rotations_per_step(), "keyswitches_per_step": ks_step},
        "conv_layer_ms_batched": conv_b,
        "conv_layer_ms_plain": conv_p,
        "conv_layer_ms_lazy_moddown": conv_l,
        "conv_layer_ms_bsgs": conv_g,
        "plan_mode": {0: "batched", 1: "plain", 2: "lazy_moddown", 3: "bsgs_double_hoisting"}[args.mode],
        "other_mode": {"plan_mode": {2: "lazy_moddown", 3: "bsgs_double_hoisting"}[other], "ms_per_step": ms_other,
                       "keyswitches_per_step": ks_other, "max_abs_err_vs_fp64": err_other},
        "rot_per_s_hoisted_level20": rot_hoisted,
        "rot_per_s_single_level20": rot_single,
        "gelu_deg59_ms_per_ct_level20": gelu_ms,
        "gelu_levels": gelu_levels,
        "gelu_max_abs_err_vs_gelu": gelu_err,
        "block_16x32x32_ms": block_ms,
        "block_plan_mode": bmode,
        "block_keyswitches": ks_block,
        "block_max_abs_err_vs_fp64": block_err,
        "pool_linear_64x8x8_to_10_ms": linear_ms,
        "pool_linear_max_abs_err_vs_fp64": linear_err,
        "imagenet_112x112x64_conv_ms_basis_mask": inet["conv"],
        "imagenet_112x112x64_pool_ms_lazy": inet["pool"],
        "imagenet_112x112x64_max_abs_err_vs_fp64": inet_err,
        "max_abs_err_vs_fp64": err,
        "gpu_event_ms_per_step": ev0.elapsed_time(ev1) / args.steps,
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_rotations, args.cpu_seconds, args.mode)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
