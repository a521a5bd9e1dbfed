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
#  * batched (mode 0): the key-switch inner product of the hoisted rotation
#    sets, k_ks_inner.  Unit: one limb moved -- per rotation its 2 beta key
#    limbs read and its 2 products written per limb, the shared hoisted digits
#    and the folded c0 read once per launch.  Bound: HBM, 8 TB/s.
#  * plain / key-stationary (modes 1, 4): the row pass of the 2^16 forward NTT
#    (k_ntt16_fwd_rows; its ModDown form finishes each rotation).  Unit: one
#    limb moved -- per transformed limb the limb read and, in the ModDown form,
#    the key-switch product (and where not folded into it sigma_g(c0)) read and
#    the rotated limb written; the twiddle and twist tables are constants and
#    not counted.  At 2^18 butterflies of ~17 VALU instructions per 1-2 MiB
#    moved it issues 2.4-4.3 instructions per byte, below the chip's ridge of
#    39.3 T lane-instructions/s / 8 TB/s = 4.9: its roof is HBM, 8 TB/s.
LIMB_BYTES = 8 << LOGN
KERNELS = {
    "k_ks_mac": {"bound": "hbm", "unit": "GB/s", "peak": 8000.0, "per_unit": LIMB_BYTES / 1e9,
                 "bytes_per_unit": LIMB_BYTES,
                 "traffic_file": os.path.join(ROOT, "profiles", "ks_mac_2e16_traffic.txt"),
                 "valu_file": os.path.join(ROOT, "profiles", "ks_mac_2e16_valu.txt")},
    "k_ntt16_fwd_rows": {"bound": "hbm", "unit": "GB/s", "peak": 8000.0, "per_unit": LIMB_BYTES / 1e9,
                         "bytes_per_unit": LIMB_BYTES,
                         "traffic_file": os.path.join(ROOT, "profiles", "ntt16_fwd_rows_2e16_traffic.txt")},
    "k_ks_inner": {"bound": "hbm", "unit": "GB/s", "peak": 8000.0, "per_unit": LIMB_BYTES / 1e9,
                   "bytes_per_unit": LIMB_BYTES,
                   "traffic_file": os.path.join(ROOT, "profiles", "ks_inner_2e16_traffic.txt"),
                   "valu_file": os.path.join(ROOT, "profiles", "ks_inner_2e16_valu.txt"),
                   # its access mix per (rotation, limb): 2 beta = 6 key streams read, 2 product
                   # streams written, one 64-bit word of each per lane
                   "probe_mix": (6, 2)},
}
DOMINANT = {0: "k_ks_inner", 1: "k_ntt16_fwd_rows", 2: "k_ks_mac", 3: "k_ks_mac", 4: "k_ntt16_fwd_rows"}


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
    "k_ks_mac": ("typedef u64 u64x2 __attribute__((ext_vector_type(2)));",
                 "// Sums of plaintext products over Q: each lane one coefficient of one limb, the"),
    "k_ntt16_fwd_rows": ("// NTT: merged Cooley-Tukey forward transform", "void hec_ntt_fwd("),
    "k_ks_inner": ("// key-switch inner product with the automorphism folded into the read:",
                   "// Key-stationary form of the same products"),
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
    out = {"bound": spec["bound"], "kernel": kernel, "achieved": achieved, "peak": spec["peak"],
           "unit": spec["unit"], "frac": achieved / spec["peak"], "traffic": traffic,
           "avg_launch_us": avg_s * 1e6, "launches": launches, "avg_units_per_launch": avg_units,
           "algorithmic_bytes_per_launch": avg_units * spec["bytes_per_unit"]}
    # VALU issue fraction: the PMC pass's quad-cycles per unit (while the
    # kernel's source is the one measured) x the units of the timed launches /
    # the issue slots of their duration (1024 SIMDs, 2.4 GHz, a wave64
    # instruction per SIMD every 4 cycles)
    rec = read_traffic(spec["valu_file"]) if "valu_file" in spec else None
    if rec and rec.get("source_sha") == kernel_source_sha(kernel):
        qc = float(rec["valu_quad_cycles_per_unit"]) * avg_units
        out["valu"] = {"quad_cycles_per_launch": qc, "issue_frac": qc / (1024 * avg_s * 2.4e9 / 4)}
    return out


def access_mix_probe(ctx, roof):
    """The dominant kernel's access mix without its arithmetic: a kernel that
    reads and writes the same number of 64-bit streams, one word of each per
    lane, over the bytes of the kernel's average launch.  Its bandwidth is what
    this access shape can draw from HBM; `kernel_frac_of_probe` = the kernel's
    achieved bandwidth / the probe's."""
    if not roof or "probe_mix" not in KERNELS[roof["kernel"]]:
        return None
    nr, nw = KERNELS[roof["kernel"]]["probe_mix"]
    words = max(1, round(roof["algorithmic_bytes_per_launch"] / 8 / (nr + nw) / (1 << LOGN))) << LOGN
    us = guarded(lambda: ctx.probe_stream(nr, nw, words, 20))
    if not isinstance(us, float):
        return None
    gbps = (nr + nw) * words * 8 / (us * 1e-6) / 1e9
    return {"streams_read": nr, "streams_written": nw, "bytes_per_launch": (nr + nw) * words * 8,
            "avg_launch_us": us, "achieved": gbps, "unit": "GB/s", "frac_of_peak": gbps / roof["peak"],
            "kernel_frac_of_probe": roof["achieved"] / gbps}


def rotations_per_step():
    # conv1: 32 channel offsets x 9 taps - the zero rotation; conv2 the same;
    # downsampling of 2 shards: 15 horizontal + 15 vertical each; consolidate 1; duplicate 1
    return 287 + 287 + 2 * 30 + 1 + 1


def cpu_baseline(n_rot, seconds, mode):
    """The CPU oracle (plain C, __int128 arithmetic, OpenMP over limbs) on a
    bounded sample of the same work as the timed step, repeated until `seconds`
    of CPU work; keys and weight plaintexts prepared outside the timed part.
    Modes 0/1/4: batches of n_rot hoisted key-switched rotations of one
    level-20 ciphertext, each multiplied by a weight plaintext and summed.
    Mode 2 (lazy ModDown): the key-switch products of n_rot rotations
    multiplied by the weights over Q*P, summed, and one ModDown."""
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
    return {"value": reps * n_rot / dt, "what": what, "reps": reps, "seconds": dt}


def host_cpu():
    """nproc and the CPU model of this host (lscpu)."""
    import subprocess
    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    try:
        nproc = int(subprocess.run(["nproc"], capture_output=True, text=True, timeout=20).stdout.strip())
    except Exception:
        nproc = os.cpu_count()
    return nproc, model


def cpu_baseline_runs(n_rot, seconds, mode):
    """The oracle timed single-threaded and with OpenMP on the host's threads,
    each in its own process (OMP_NUM_THREADS is read at OpenMP start-up)."""
    import subprocess
    nproc, model = host_cpu()
    threads = int(os.environ.get("OMP_NUM_THREADS", nproc or 1))
    res = {}
    for label, nt in (("single_thread", 1), ("openmp", threads)):
        env = dict(os.environ, OMP_NUM_THREADS=str(nt))
        code = ("import json, sys; sys.path.insert(0, %r); import bench; "
                "print(json.dumps(bench.cpu_baseline(%d, %f, %d)))" % (ROOT, n_rot, seconds, mode))
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=900)
        if r.returncode != 0:
            raise RuntimeError("cpu baseline failed: %s" % r.stderr[-2000:])
        res[label] = dict(json.loads(r.stdout.strip().splitlines()[-1]), threads=nt)
    o = res["openmp"]
    return {"value": o["value"], "unit": "key-switched rotations/s", "cores": o["threads"], "kind": "oracle",
            "sample": "%d x %d rotations of one level-20 ciphertext (%s), 2N=2^16, dnum=3 (%.1f s); "
                      "OpenMP over limbs" % (o["reps"], n_rot, o["what"], o["seconds"]),
            "single_thread_value": res["single_thread"]["value"],
            "single_thread_sample": "%d x %d rotations (%.1f s)" % (res["single_thread"]["reps"], n_rot,
                                                                   res["single_thread"]["seconds"]),
            "host_nproc": nproc, "host_cpu_model": model}


def guarded(fn):
    """A secondary measurement: its failure is reported in its own field
    (with the error) instead of ending the run before the line is printed."""
    try:
        return fn()
    except Exception as e:  # noqa: BLE001 -- any failure of the section is recorded, not raised
        eprint("section failed: %r" % (e,))
        return {"error": repr(e)}


def timed(ctx, fn, reps, warm=1):
    """Median wall ms of fn() over reps calls (after warm untimed ones), the
    device drained before and after each."""
    for _ in range(warm):
        r = fn()
        ctx.sync()
        del r
    ts = []
    for _ in range(reps):
        ctx.sync()
        t = time.perf_counter()
        r = fn()
        ctx.sync()
        ts.append((time.perf_counter() - t) * 1e3)
        del r
    return float(np.median(ts))


def rotation_roofline(rate, level):
    """Roofline fractions of complete hoisted key-switched rotations at `level`
    (2N = 2^16, dnum = 3, k = 8): algorithmic bytes per rotation 4 (l+1) + 2 beta
    (l+1+k) limbs (ciphertext in and out, the key), modular multiplications of
    an extra hoisted rotation (key-switch inner product, ModDown: INTT of the
    P limbs, P -> Q conversion, NTT) at 10 VALU multiply instructions each."""
    nq, k, alpha = level + 1, K, 9
    beta = (nq + alpha - 1) // alpha
    limbs = 4 * nq + 2 * beta * (nq + k)
    nbytes = limbs * LIMB_BYTES
    n, logn = 1 << LOGN, LOGN
    modmul = (2 * beta * (nq + k)            # inner product per coefficient
              + 2 * k * nq                   # P -> Q conversion per coefficient
              + 2 * nq + 2 * k) * n          # scaling by P^-1, ... per coefficient (combine, INTT n^-1)
    modmul += (2 * k + 2 * nq) * (n // 2) * logn   # the INTT of the P limbs and the NTT of the Q limbs
    peak_valu = 256 * 64 * 2.4e9 / 10
    return {"rotations_per_s": rate, "level": level, "bytes_per_rotation": nbytes,
            "hbm_GBps": rate * nbytes / 1e9, "hbm_peak_GBps": 8000.0, "hbm_frac": rate * nbytes / 8e12,
            "modmul_per_rotation": modmul, "valu_Tmodmul_s": rate * modmul / 1e12,
            "valu_peak_Tmodmul_s": peak_valu / 1e12, "valu_frac": rate * modmul / peak_valu}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--reps", type=int, default=20, help="repetitions of every sub-measurement (median)")
    ap.add_argument("--cpu-rotations", type=int, default=8)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--skip", default="", help="comma list of extra sections to skip: "
                    "layers,other,rot,gelu,block,linear,imagenet,uneven,serving")
    ap.add_argument("--mode", type=int, default=0, choices=(0, 1, 2, 3, 4),
                    help="plan mode of the timed step: 0 batched (complete key-switched rotations), 1 plain, "
                         "2 lazy ModDown, 3 baby-step/giant-step with double hoisting, 4 key-stationary")
    ap.add_argument("--tune", default="", help="launch parameters to set first, e.g. ntt_row_vals=16,ks_amounts=8 "
                    "(every value gives the same ciphertexts)")
    ap.add_argument("--pmc-run", action="store_true", help="short workload for rocprofv3 --pmc passes")
    ap.add_argument("--profile-run", choices=("gelu", "block", "imagenet", "rotations"),
                    help="for kernel traces: five degree-59 GELU evaluations, five runs of the 16x32x32 block, "
                         "the 112x112x64 stage in mode 4, or 5 x 32 hoisted rotations at level 20, then exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        eprint("bench.py measures one GPU: the whole path runs on a single MI355X "
               "(sharding across GPUs is described, not implemented); use --gpus 1")
        sys.exit(2)
    skip = set(x for x in args.skip.split(",") if x)

    import torch
    from paper_2306_09189_amd import hecnn

    for kv in (x for x in args.tune.split(",") if x):
        name, val = kv.split("=")
        hecnn.tune_set(name.strip(), int(val))
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    ctx = hecnn.Context(LOGN, L, Q0, QB, K, PB, DNUM, LOG_SCALE, device=0, stream=stream.cuda_stream)
    rng = np.random.default_rng(1002)
    x = rng.uniform(-1, 1, (32, 32, 32))
    w1 = rng.normal(0, 0.05, (32, 32, 3, 3))
    w2 = rng.normal(0, 0.05, (64, 32, 3, 3))
    from numpy.polynomial import chebyshev as Cheb

    def gelu(v):
        return 0.5 * v * (1.0 + np.tanh(np.sqrt(2.0 / np.pi) * (v + 0.044715 * v ** 3)))
    bound = 15.0
    coef = Cheb.chebinterpolate(lambda y: gelu(bound * y), 59)
    if args.profile_run:
        ctx.keygen(2002)
        if args.profile_run == "gelu":
            ct = ctx.encrypt(ctx.encode(rng.uniform(-1, 1, ctx.N), LEVEL, 2.0 ** LOG_SCALE), 6)
            for _ in range(5):
                r = ctx.cheb_eval(ct, coef, -1.0, 1.0)
                del r
        elif args.profile_run == "block":
            xb = rng.uniform(-1, 1, (16, 32, 32))
            wb1, wb2 = rng.normal(0, 1 / 12.0, (16, 16, 3, 3)), rng.normal(0, 1 / 12.0, (16, 16, 3, 3))
            bn = (rng.uniform(0.5, 1.5, 16), rng.normal(0, 0.5, 16))
            imb = ctx.image_encrypt(xb, LEVEL, 7)
            blk = ctx.block(imb, wb1, bn, wb2, bn, 15.0, coef, mode=args.mode if args.mode >= 2 else 2)
            ctx.gen_rotation_keys(blk.steps())
            for _ in range(5):
                ob = blk.run(imb)
                del ob
        elif args.profile_run == "imagenet":
            xi = np.clip(rng.normal(0, 1, (64, 112, 112)), -4, 4)
            wi = rng.normal(0, 0.05, (64, 64, 3, 3))
            imi = ctx.image_encrypt(xi, LEVEL, 9)
            pi = ctx.conv2d_plan(imi, wi, basis=27)
            pi.set_mode(4)
            ctx.gen_rotation_keys(pi.steps())
            yi = pi.run(imi)
            ctx.gen_rotation_keys(ctx.avgpool_steps(yi))
            for _ in range(3):
                yi = pi.run(imi)
                zi = ctx.avgpool(yi, 4)
                del zi
        else:
            ctx.gen_rotation_keys(list(range(1, 33)))
            ct = ctx.encrypt(ctx.encode(rng.uniform(-1, 1, ctx.N), LEVEL, 2.0 ** LOG_SCALE), 5)
            for _ in range(5):
                rs = ctx.rotate_hoisted(ct, list(range(1, 33)))
                del rs
        ctx.sync()
        # a plain device copy of exactly 256 MiB last: it calibrates the byte counters of a --pmc pass
        src = torch.ones(1 << 25, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
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

    from oracle import he_layers as hl  # FP64 references for the accuracy checks only
    ref = hl.ref_conv2d(hl.ref_conv2d(x, w1, 1, 1), w2, 1, 2)

    def step(check=False):
        im = ctx.image_encrypt(x, LEVEL, 3002)
        a = p1.run(im)
        b = p2.run(a)
        y = b.decrypt()
        if check:
            return float(np.abs(y - ref).max())
        return None

    def run_steps(mode, nsteps, profile_kernel=None):
        p1.set_mode(mode)
        p2.set_mode(mode)
        for _ in range(args.warmup):
            step()
        err = step(check=True)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        if profile_kernel:
            ctx.prof_start(profile_kernel)
            first = ctx.prof_launches(profile_kernel)
        ks0 = ctx.keyswitch_count()
        t = time.perf_counter()
        ev0.record(stream)
        for _ in range(nsteps):
            step()
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        prof = None
        if profile_kernel:
            launches, units, kms = ctx.prof_stop()
            prof = dominant_roofline(profile_kernel, launches, units, kms)
            if prof:
                prof["trace_dispatch_range"] = [first, first + launches]
        return {"wall": wall, "ms_per_step": wall * 1e3 / nsteps, "gpu_event_ms_per_step":
                ev0.elapsed_time(ev1) / nsteps, "keyswitches_per_step": (ctx.keyswitch_count() - ks0) / nsteps,
                "max_abs_err_vs_fp64": err, "roofline": prof}

    # ---- the timed step (the headline): complete key-switched rotations ----
    main_run = run_steps(args.mode, args.steps, DOMINANT[args.mode])
    ks_step = main_run["keyswitches_per_step"]
    value = ks_step * args.steps / main_run["wall"]
    out = {
        "metric": "key-switched rotations/sec + HE conv-layer ms at 2N=2^16; batched vs plain",
        "value": value,
        "unit": ("key-switched rotations/s (complete: automorphism, key switch, ModDown each)"
                 if args.mode in (0, 1, 4) else "key-switch inner products/s (ModDown once per output sum)"),
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "2N=2^16, 32x32x32 image at level 20: conv3x3 32->32 s1 + conv3x3 32->64 s2 "
                               "(2 shards -> downsample -> 1 ct), encrypt+decrypt included",
                   "ring_dim": 1 << LOGN, "level": LEVEL, "dnum": DNUM, "special_primes": K,
                   "rotations_per_step": rotations_per_step(), "keyswitches_per_step": ks_step},
        "plan_mode": MODE_NAMES[args.mode],
        "max_abs_err_vs_fp64": main_run["max_abs_err_vs_fp64"],
        "gpu_event_ms_per_step": main_run["gpu_event_ms_per_step"],
        "roofline": main_run["roofline"],
        "launch_params": hecnn.tune_describe(),
    }
    eprint("step mode %d: %.2f ms, %.0f rotations/s" % (args.mode, main_run["ms_per_step"], value))
    probe = access_mix_probe(ctx, main_run["roofline"])
    if probe:
        out["roofline"]["access_mix_probe"] = probe

    # ---- the same step in the other modes ----
    if "other" not in skip:
        others = {}
        for mode in (2, 3, 4, 0):
            if mode == args.mode:
                continue
            r = run_steps(mode, args.steps, DOMINANT[mode] if mode == 2 else None)
            others[MODE_NAMES[mode]] = {"ms_per_step": r["ms_per_step"],
                                        "keyswitches_per_step": r["keyswitches_per_step"],
                                        "keyswitches_per_s": r["keyswitches_per_step"] * 1e3 / r["ms_per_step"],
                                        "max_abs_err_vs_fp64": r["max_abs_err_vs_fp64"]}
            if r["roofline"]:
                others[MODE_NAMES[mode]]["roofline"] = r["roofline"]
        out["other_modes"] = others
        p1.set_mode(args.mode)
        p2.set_mode(args.mode)

    # ---- conv-layer ms (conv 3x3 32->32) in every plan mode ----
    if "layers" not in skip:
        im = ctx.image_encrypt(x, LEVEL, 3002)
        layer = {}
        for mode in (1, 0, 4, 2, 3):
            p1.set_mode(mode)
            layer[MODE_NAMES[mode]] = timed(ctx, lambda: p1.run(im), args.reps)
        p1.set_mode(args.mode)
        out["conv_layer_ms"] = layer
        out["conv_layer_ms_plain"] = layer["plain"]
        out["conv_layer_ms_batched"] = layer["batched"]
        del im

    # ---- isolated complete rotations at level 20: hoisted sets and single ----
    if "rot" not in skip:
        ctx.gen_rotation_keys(list(range(1, 33)))
        ct = ctx.encrypt(ctx.encode(rng.uniform(-1, 1, ctx.N), LEVEL, 2.0 ** LOG_SCALE), 5)
        hms = timed(ctx, lambda: ctx.rotate_hoisted(ct, list(range(1, 33))), args.reps)
        sms = timed(ctx, lambda: ctx.rotate(ct, 7), args.reps)
        out["rotation_roofline_hoisted_level20"] = rotation_roofline(32e3 / hms, LEVEL)
        out["rot_per_s_hoisted_level20"] = 32e3 / hms
        out["rot_per_s_single_level20"] = 1e3 / sms
        del ct

    # ---- GELU, the basic block and the pool-linear head ----
    if "gelu" not in skip:
        zg = rng.uniform(-1, 1, ctx.N)
        ctg = ctx.encrypt(ctx.encode(zg, LEVEL, 2.0 ** LOG_SCALE), 6)
        out["gelu_deg59_ms_per_ct_level20"] = timed(ctx, lambda: ctx.cheb_eval(ctg, coef, -1.0, 1.0), args.reps)
        g = ctx.cheb_eval(ctg, coef, -1.0, 1.0)
        out["gelu_levels"] = LEVEL - g.level
        out["gelu_max_abs_err_vs_gelu"] = float(np.abs(ctx.decrypt(g) - gelu(bound * zg)).max())
        del g, ctg
    if "block" not in skip:
        xb = rng.uniform(-1, 1, (16, 32, 32))
        wb1, wb2 = rng.normal(0, 1 / 12.0, (16, 16, 3, 3)), rng.normal(0, 1 / 12.0, (16, 16, 3, 3))
        bn1 = (rng.uniform(0.5, 1.5, 16), rng.normal(0, 0.5, 16))
        bn2 = (rng.uniform(0.5, 1.5, 16), rng.normal(0, 0.5, 16))
        imb = ctx.image_encrypt(xb, LEVEL, 7)
        blk = ctx.block(imb, wb1, bn1, wb2, bn2, bound, coef, mode=2)
        ctx.gen_rotation_keys(blk.steps())
        out["block_16x32x32_ms"] = timed(ctx, lambda: blk.run(imb), args.reps)
        ob = blk.run(imb)
        out["block_max_abs_err_vs_fp64"] = float(np.abs(ob.decrypt() - hl.ref_basic_block(
            xb, wb1, bn1, wb2, bn2, bound, coef)).max())
        del ob, blk, imb
    if "linear" not in skip:
        xl = rng.uniform(-1, 1, (64, 8, 8))
        wl = rng.normal(0, 0.1, (10, 64))
        iml = ctx.image_encrypt(xl, LEVEL, 8)
        ctx.gen_rotation_keys(ctx.linear_steps(iml))
        out["pool_linear_64x8x8_to_10_ms"] = timed(ctx, lambda: ctx.linear(iml, wl, True), args.reps)
        ol = ctx.linear(iml, wl, True)
        out["pool_linear_max_abs_err_vs_fp64"] = float(np.abs(ctx.decrypt(ol)[:10] - hl.ref_linear(xl, wl, True)).max())
        del ol, iml

    # ---- the 112x112x64 ImageNet stage (32 shards): plain vs batched vs key-stationary ----
    if "imagenet" not in skip:
        out["imagenet_112x112x64"] = guarded(lambda: imagenet_stage(ctx, hecnn, hl, rng, args.reps))

    # ---- the uneven batch: 13 instances, 48 ciphertexts at levels 2..24, eager vs one captured graph ----
    ctx.release_cached()  # the cached blocks of the sections before go back to the device
    if "uneven" not in skip:
        out["uneven_batch_48ct"] = guarded(lambda: uneven_batch(ctx, hl, args.reps))

    # ---- serving: Poisson arrivals of the two request shapes ----
    ctx.release_cached()
    if "serving" not in skip:
        out["serving"] = guarded(lambda: serving(ctx, hecnn, hl))

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_runs(args.cpu_rotations, args.cpu_seconds, args.mode)
    print(json.dumps(out), flush=True)


MODE_NAMES = {0: "batched", 1: "plain", 2: "lazy_moddown", 3: "bsgs_double_hoisting", 4: "key_stationary"}


def imagenet_stage(ctx, hecnn, hl, rng, reps):
    """conv 3x3 64->64 (basis-mask weight plaintexts, masks at 2^27) + 2x2
    average pooling of a 64x112x112 activation in 32 shards of two padded
    128x128 channels, level 20, in each evaluation form; the key-stationary
    form's launch parameters chosen by the autotuner first."""
    xi = np.clip(rng.normal(0, 1, (64, 112, 112)), -4, 4)
    wi = rng.normal(0, 0.05, (64, 64, 3, 3))
    imi = ctx.image_encrypt(xi, LEVEL, 9)
    pi = ctx.conv2d_plan(imi, wi, basis=27)
    ctx.gen_rotation_keys(pi.steps())
    y0 = pi.run(imi)
    ctx.gen_rotation_keys(ctx.avgpool_steps(y0))
    del y0
    fp = hl.ref_avgpool2x2(hl.ref_conv2d(xi, wi, 1))
    pi.set_mode(4)
    t = time.perf_counter()
    report = ctx.autotune_conv(pi, imi, reps=2)
    tune_s = time.perf_counter() - t
    res = {"shards": 32, "level": LEVEL, "autotune": {"report": report, "seconds": tune_s,
                                                      "chosen": hecnn.tune_describe()}}
    forms = (("plain", 1, 0), ("batched", 0, 0), ("key_stationary", 4, 4), ("lazy_moddown", 2, 2))
    for name, cmode, pmode in forms:
        pi.set_mode(cmode)
        n = reps
        conv_ms = timed(ctx, lambda: pi.run(imi), n)
        yi = pi.run(imi)
        pool_ms = timed(ctx, lambda: ctx.avgpool(yi, pmode), n)
        zi = ctx.avgpool(yi, pmode)
        err = float(np.abs(zi.decrypt() - fp).max())
        res[name] = {"conv_ms": conv_ms, "pool_ms": pool_ms, "total_ms": conv_ms + pool_ms, "reps": n,
                     "max_abs_err_vs_fp64": err}
        del yi, zi
        eprint("imagenet %s: conv %.1f ms pool %.1f ms err %.2g" % (name, conv_ms, pool_ms, err))
    del pi, imi
    return res


def uneven_batch(ctx, hl, reps):
    """One 64x112x112 instance (32 shards, basis-mask, key-stationary), four
    16x56x56 (2 shards) and eight 32x32x32 (1 shard; lazy ModDown), 48
    ciphertexts, each at its own level drawn uniformly from 2..24, each
    through a 3x3 convolution and rescale: eager launches vs replays of one
    captured HIP graph (the first launch records it)."""
    rng = np.random.default_rng(4004)
    shapes = [(64, 112, 112)] + [(16, 56, 56)] * 4 + [(32, 32, 32)] * 8
    levels = rng.integers(2, 25, size=len(shapes))
    batch = ctx.batch()
    inst = []
    for i, (shape, level) in enumerate(zip(shapes, levels)):
        C = shape[0]
        xx = np.clip(rng.normal(0, 1, shape), -4, 4) if C == 64 else rng.uniform(-1, 1, shape)
        ww = rng.normal(0, 0.05, (C, C, 3, 3))
        im = ctx.image_encrypt(xx, int(level), 6000 + i)
        if C == 64:
            pl = ctx.conv2d_plan(im, ww, basis=27)
            pl.set_mode(4)
        else:
            pl = ctx.conv2d_plan(im, ww)
            pl.set_mode(2)
        ctx.gen_rotation_keys(pl.steps())
        batch.add(pl, im)
        inst.append((xx, ww))
    eager_ms = timed(ctx, lambda: batch.launch(graph=False), reps)
    t = time.perf_counter()
    batch.launch(graph=True)
    ctx.sync()
    capture_ms = (time.perf_counter() - t) * 1e3
    graph_ms = timed(ctx, lambda: batch.launch(graph=True), reps)
    err = 0.0
    for i, (xx, ww) in enumerate(inst):
        err = max(err, float(np.abs(batch.output(i).decrypt() - hl.ref_conv2d(xx, ww, 1)).max()))
    eprint("uneven batch: eager %.1f ms graph %.1f ms (capture %.0f ms) err %.2g" % (eager_ms, graph_ms,
                                                                                   capture_ms, err))
    return {"instances": len(shapes), "ciphertexts": 48, "levels": [int(v) for v in levels],
            "eager_ms": eager_ms, "graph_ms": graph_ms, "first_graph_launch_ms": capture_ms,
            "max_abs_err_vs_fp64": err, "reps": reps}


def serving(ctx, hecnn, hl, n_requests=24, lanes=2, max_batch=4):
    """Encrypted-inference requests under Poisson arrivals: 70 % a 3x32x32
    image (channels padded to 4, duplicated) through conv 3x3 3->32 and 2x2
    average pooling, 30 % a 3x224x224 image (each channel in two shards)
    through the stem conv 3x3 stride 2, 3->64; level 20, keys and plans
    resident; the convolutions key-stationary (mode 4), the pooling and the
    stem's downsampling with lazy ModDown (mode 2).  Saturation throughput
    from a burst, then arrivals at 0.5x and 0.8x of it; p50 / p99 latency
    (submit -> result on the device) and requests/s."""
    rng = np.random.default_rng(5005)
    wa = rng.normal(0, 0.05, (32, 3, 3, 3))
    wb = rng.normal(0, 0.05, (64, 3, 3, 3))
    like_a = ctx.image_encrypt(rng.uniform(-1, 1, (3, 32, 32)), LEVEL, 7001)
    like_b = ctx.image_encrypt(rng.uniform(-1, 1, (3, 224, 224)), LEVEL, 7002)
    pa = ctx.conv2d_plan(like_a, wa)
    pa.set_mode(4)
    ctx.gen_rotation_keys(pa.steps())
    ctx.gen_rotation_keys(ctx.avgpool_steps(pa.run(like_a)))
    pb = ctx.conv2d_plan(like_b, wb, stride=2, q_only=True)
    pb.set_mode(4)
    pb.set_downsample_mode(2)
    ctx.gen_rotation_keys(pb.steps())
    ctx.sync()
    srv = hecnn.Server(ctx, lanes=lanes, max_batch=max_batch, mem_budget=64 << 30)
    res = {"lanes": lanes, "max_batch": max_batch, "mix": "70% 3x32x32 conv 3->32 + pool, 30% 3x224x224 stem "
           "conv s2 3->64", "forms": "convolutions key-stationary (mode 4), pooling and the stem's downsampling "
           "lazy (mode 2)", "level": LEVEL}
    try:
        ma = srv.add_model(pa, like_a, pool_mode=2)
        mb = srv.add_model(pb, like_b)
        res["footprint_bytes"] = {"block": srv.footprint(ma), "stem": srv.footprint(mb)}
        reqs = []
        for i in range(n_requests):
            m = ma if rng.uniform() < 0.7 else mb
            shape = (3, 32, 32) if m == ma else (3, 224, 224)
            xx = rng.uniform(-1, 1, shape)
            reqs.append((m, xx, ctx.image_encrypt(xx, LEVEL, 8000 + i)))
        ctx.sync()
        # saturation: everything at once
        t = time.perf_counter()
        ids = [srv.submit(m, im) for (m, xx, im) in reqs]
        for rid in ids:
            o, _ = srv.poll(rid)
            o.free()
        sat = len(reqs) / (time.perf_counter() - t)
        res["saturation_req_per_s"] = sat
    finally:
        srv.stop()  # its lanes' memory back before the servers of the timed loads start
    for load in (0.5, 0.8):
        srv_l = hecnn.Server(ctx, lanes=lanes, max_batch=max_batch, mem_budget=64 << 30)
        try:
            srv_l.add_model(pa, like_a, pool_mode=2)
            srv_l.add_model(pb, like_b)
            lam = load * sat
            gaps = rng.exponential(1.0 / lam, size=len(reqs))
            t = time.perf_counter()
            due = t
            ids = []
            for (m, xx, im), gap in zip(reqs, gaps):
                due += gap
                d = due - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                ids.append(srv_l.submit(m, im))
            errs, checked = [], {ma: 0, mb: 0}
            for (m, xx, im), rid in zip(reqs, ids):
                o, ms = srv_l.poll(rid)
                if checked[m] < 2:  # accuracy of the first two results of each kind
                    checked[m] += 1
                    w = wa if m == ma else wb
                    ref = (hl.ref_avgpool2x2(hl.ref_conv2d(xx, w, 1)) if m == ma else hl.ref_conv2d(xx, w, 1, 2))
                    errs.append(float(np.abs(o.decrypt() - ref).max()))
                o.free()
            st = srv_l.stats()
            res["load_%.1f" % load] = {"arrival_req_per_s": lam, "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
                                       "mean_ms": st["mean_ms"], "req_per_s": st["req_per_s"],
                                       "batches": st["batches"], "max_concurrent": st["max_concurrent"],
                                       "peak_admitted_bytes": st["peak_mem"],
                                       "max_abs_err_vs_fp64": max(errs) if errs else None}
            eprint("serving load %.1f: p50 %.0f ms p99 %.0f ms %.2f req/s" % (load, st["p50_ms"], st["p99_ms"],
                                                                            st["req_per_s"]))
        finally:
            srv_l.stop()
    return res


if __name__ == "__main__":
    main()
