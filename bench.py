#!/usr/bin/env python3
"""Throughput of the homomorphic d x d matrix product at N = 2^16 on one MI355X.

One step = one batch of `--batch` independent 128 x 128 products (Eq. 4 of
the paper: sigma/tau double-hoisted BSGS, hoisted column/row shifts, n
products, rescale) on ciphertexts already resident in HBM.  Three paths are
timed on the same inputs:
  plain    one product after another, relinearising every product (the
           paper's order of Algorithm DMatrixMult);
  batched  the products stacked so every launch serves all of them (same
           residues as plain, checked here);
  headline batched, with lazy relinearisation (the n tensors summed and
           relinearised once) and the A side's ModDown and Rescale as one
           rounding by P q_l (--two-roundings keeps two; --paper-relin keeps
           the paper's order altogether).
The headline value is the last; the others and the speedups sit beside it.
The headline steps run without per-kernel instrumentation; the same number
of steps is then run again with HIP events around every launch, and the
kernel table and the roofline of the kernel with the largest device time
come from that profiled pass (its step time is printed too).  Also printed:
key-switched rotations/s, per-step latency percentiles, a serving run, the
PCA run and the CPU oracle timed on a bounded sample on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "HE d×d matmuls/s & key-switched rotations/s at N=2^16, batched vs plain; p99"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
CSRC = os.path.join(ROOT, "paper_2305_17341_amd", "csrc")
# source regions a kernel's recorded traffic depends on: (file, first line, last line), matched literally
_MULTSUM_REGIONS = [("kernels.hip", "__device__ __forceinline__ u32 automorph_src(", "}"),
                    ("kernels.hip", "#define MS_MAXB 8", "#undef MS_CASE"),
                    ("he_internal.h", "// Per-modulus constants", "// Host-side objects")]
_NTT_REGIONS = [("kernels.hip", "__device__ __forceinline__ int grid_limb(", "return m.n;\n}"),
                ("kernels.hip", "struct ShoupArith {", "// Galois automorphism in the evaluation domain:"),
                ("he_internal.h", "// Per-modulus constants", "// Host-side objects")]
KERNEL_REGIONS = {"multsum": _MULTSUM_REGIONS, "multsum_rot": _MULTSUM_REGIONS, "multsum_rot_int": _MULTSUM_REGIONS,
                  "ntt_fwd_cols": _NTT_REGIONS, "ntt_fwd_rows": _NTT_REGIONS, "ntt_fwd_rows_sub": _NTT_REGIONS,
                  "ntt_fwd_cols_modup": _NTT_REGIONS}
# the fused ModDown column pass also depends on the conversion's constants and quotient
KERNEL_REGIONS["ntt_fwd_cols_fbc"] = _NTT_REGIONS + [("kernels.hip", "struct FbcArgs {", "bool launch_moddown_fused(")]


def autotune_knobs():
    from paper_2305_17341_amd import autotune
    return tuple(autotune.CANDIDATES)


def kernel_digest(kernel):
    """SHA-256 over the source regions of `kernel` (None if one is missing)"""
    import hashlib
    regions = KERNEL_REGIONS.get(kernel)
    if regions is None:
        return None
    h = hashlib.sha256()
    for fname, first, last in regions:
        with open(os.path.join(CSRC, fname)) as fh:
            text = fh.read()
        if first is not None:
            a = text.find(first)
            if a < 0:
                return None
            b = text.find(last, a + len(first))
            if b < 0:
                return None
            text = text[a:b + len(last)]
        h.update(text.encode())
    return h.hexdigest()


def measured_traffic(kernel, n1, knobs):
    """HBM bytes per launch of `kernel` (FETCH_SIZE + WRITE_SIZE counters,
    scaled by a plain copy's reading) recorded with a digest of the kernel's
    source regions, the baby-step count and the launch knobs the launches
    had; None when absent or any of them differs."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        rec = json.load(fh)
    k = rec.get("kernels", {}).get(kernel)
    if k is None or k.get("source_sha256") != kernel_digest(kernel) or k.get("n1") != n1:
        return None
    if any(knobs.get(name) != v for name, v in k.get("knobs", {}).items()):
        return None
    return k["bytes_per_launch"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def pct(xs, p):
    return float(np.percentile(np.asarray(xs), p)) if xs else None


# one wave64 VALU instruction per SIMD every 4 clocks at full rate: 256 CUs x
# 4 SIMDs x 64 lanes at 2.4 GHz = 39.3 T lane-operations/s
LANE_OPS_PEAK = 256 * 4 * 16 * 2.4e9
# full-rate VALU instructions per lazy FP64 product (mul, fma, mul, rndne, fma, add)
F64_LAZY_INSTR = 6


def valu_ceilings(log=print):
    """measured rates (products/s) of the four product kinds the kernels use
    (he_modmul_peak: eight register-resident chains per thread, no memory),
    best of three, beside the unit-count figure for the lazy FP64 product"""
    from paper_2305_17341_amd import he
    out = {}
    for kind in he.MODMUL_KINDS:
        he.modmul_peak(kind, iters=256, blocks=2048)
        best = max(he.modmul_peak(kind, iters=2048, blocks=8192)[0] for _ in range(3))
        out[kind] = {"measured": best}
    out["f64_lazy"]["from_unit_counts"] = LANE_OPS_PEAK / F64_LAZY_INSTR
    log("[bench] product ceilings (G/s): " + ", ".join(f"{k} {v['measured'] / 1e9:.0f}" for k, v in out.items()))
    return out


def cpu_model():
    """the host's CPU model name and the threads this process may use"""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return model, os.cpu_count() or 1, usable


def _median_time(f, reps):
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        f()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def cpu_baseline(chain, counts, n_rescale, d, log=print):
    """The CPU oracle (plain C, 128-bit % products, OpenMP over limbs) timed on
    this host, every figure a direct measurement:
      * the small (N=2^13, 16x16) and mid (N=2^14, 64x64, (A B) C chained)
        products in full, on all usable threads and on one;
      * one key-switched rotation at N=2^16, level 30 (all threads, one);
      * the operations of the headline product at N=2^16, level 29, each timed
        on its own (median of three): Decompose, the key inner product of one
        rotation, ModDown, Rescale, Tensor.
    `value` (products/s of the headline product) is the sum of the last ones
    weighted by the product's operation counts (from the GPU library's
    counters: Decompose, key inner products, ModDown per product; d tensors,
    `n_rescale` rescales); it is an extrapolation from measured operations,
    labelled as such."""
    from oracle import oracle as O
    from paper_2305_17341_amd import he, inputs as I
    model, nproc, usable = cpu_model()
    threads = int(os.environ.get("OMP_NUM_THREADS", usable))
    out = {"unit": "matmuls/s", "cores": threads, "kind": "oracle", "cpu_model": model, "nproc": nproc,
           "usable_cpus": usable, "measured": {}}
    meas = out["measured"]

    def both(tag, f, reps_all=1):
        O.set_threads(threads)
        t_all = _median_time(f, reps_all)
        O.set_threads(1)
        t_one = _median_time(f, 1)
        O.set_threads(threads)
        meas[tag] = {"s_all_threads": round(t_all, 4), "s_one_thread": round(t_one, 4)}
        log(f"[bench] oracle {tag}: {t_all:.3f} s on {threads} threads, {t_one:.3f} s on one")

    # small and mid products in full
    for ch, n, chained, tag in ((I.SMALL, 16, False, "small_16x16_n13"), (I.MID, 64, True, "mid_64x64_n14_chained")):
        o = O.Oracle(ch.log_n, ch.q_bits, ch.p_bits, seed=5)
        n1 = 1 << ((n.bit_length() - 1 + 1) // 2)   # 2^ceil(log2(n) / 2), the library's default
        steps = sorted(set(he.lintrans_rot_steps("Z", n, n1)) | set(he.lintrans_rot_steps("T", n, n1)) |
                       set(range(1, n1)) | {n1, -n} | {n * j for j in range(1, n1)} | {n * n1})
        o.keygen(rot_steps=steps)
        A, B, Cm = I.uniform_matrix(1, n), I.uniform_matrix(2, n), I.uniform_matrix(3, n)
        ca, cb = o.encrypt(A.ravel(), nonce=1), o.encrypt(B.ravel(), nonce=2)
        if chained:
            def run():
                ab = o.matmul(ca, cb, n, n1, n1)
                o.matmul(ab, o.encrypt(Cm.ravel(), level=ab.level, nonce=3), n, n1, n1)
        else:
            def run():
                o.matmul(ca, cb, n, n1, n1)
        both(tag, run)
        del o
    # rotation and the product's operations at N = 2^16
    o = O.Oracle(chain.log_n, chain.q_bits, chain.p_bits, seed=5)
    o.keygen(rot_steps=[1], relin=True)
    z = np.random.default_rng(0).uniform(-1, 1, o.slots)
    ct = o.encrypt(z, nonce=1)
    both(f"rotation_n16_level{ct.level}", lambda: o.rotate(ct, 1), reps_all=3)
    c29 = o.drop(ct, ct.level - 1)
    lvl = c29.level
    O.set_threads(threads)
    digits = o.decompose(c29.data()[1], lvl)
    h = o.hoisted_rotate_digits(c29, digits, 1)
    ops = {
        "decompose": _median_time(lambda: o.decompose(c29.data()[1], lvl), 3),
        "multsum": _median_time(lambda: o.hoisted_rotate_digits(c29, digits, 1), 3),
        "moddown": _median_time(lambda: o.moddown(h), 3),
        "rescale": _median_time(lambda: o.rescale(c29), 3),
        "tensor": _median_time(lambda: o.tensor(c29, c29), 3),
    }
    meas[f"ops_n16_level{lvl}_s"] = {k: round(v, 4) for k, v in ops.items()}
    n_tensor = d
    t_mm = (counts["decompose"] * ops["decompose"] + counts["multsum"] * ops["multsum"] +
            counts["moddown"] * ops["moddown"] + n_rescale * ops["rescale"] + n_tensor * ops["tensor"])
    out["value"] = 1.0 / t_mm
    out["rotations_per_s"] = 1.0 / meas[f"rotation_n16_level{ct.level}"]["s_all_threads"]
    out["sample"] = (f"oracle on this host ({model}, {threads} threads): the {d}x{d} product at N=2^{chain.log_n} "
                     f"extrapolated from its operations each timed at level {lvl} (median of 3): "
                     f"{counts['decompose']:.0f} Decompose x {ops['decompose']:.3f} s, {counts['multsum']:.0f} key "
                     f"inner products x {ops['multsum']:.3f} s, {counts['moddown']:.0f} ModDown x "
                     f"{ops['moddown']:.3f} s, {n_rescale} Rescale x {ops['rescale']:.3f} s, {n_tensor} Tensor x "
                     f"{ops['tensor']:.3f} s = {t_mm:.1f} s; the small and mid products and one rotation at "
                     f"N=2^16 measured in full (see measured)")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--knobs", default="",
                    help="launch knobs set before the run, e.g. mr_members=4,ms_members=4 (with --no-autotune)")
    ap.add_argument("--no-graph", action="store_true",
                    help="headline steps launched one kernel at a time instead of replaying a recorded HIP graph")
    ap.add_argument("--two-roundings", action="store_true",
                    help="headline keeps the A side's ModDown and Rescale as two roundings")
    ap.add_argument("--paper-relin", action="store_true",
                    help="headline path relinearises every product (default: lazy, once per product)")
    ap.add_argument("--d", type=int, default=128)
    ap.add_argument("--rotations", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-jobs", type=int, default=400,
                    help="jobs per serving trace: the capacity run and each offered load (0: skip serving)")
    ap.add_argument("--serve-loads", default="0.2,0.6,1.0,1.2",
                    help="offered loads of the serving sweep, as fractions of the measured batched capacity")
    ap.add_argument("--pca-components", type=int, default=8, help="components of the PCA run (0: skip it)")
    ap.add_argument("--n1", type=int, default=64,
                    help="baby steps of Z and T and the block size of the column/row shifts (0: the library's "
                         "default, 16 for d = 128); 64 measured fastest for d = 128 (130 keys, 47.8 GiB resident)")
    ap.add_argument("--serve-cov-samples", type=int, default=60000,
                    help="rows of the serving mix's covariance job (256 features)")
    ap.add_argument("--big-covariance", type=int, default=0, metavar="S",
                    help="also run the serving workload's large covariance job alone on S x 256 samples (60000 in "
                         "the workload; about a minute; 0: skip)")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the PPPCA accuracy runs (R2(X), R2(V) on synthetic stand-ins)")
    ap.add_argument("--table3-reps", type=int, default=3,
                    help="repetitions per row of the Z/T decomposition table at N=2^15 (0: skip it)")
    ap.add_argument("--calib-copies", type=int, default=0,
                    help="device copies of one top-level ciphertext at the end (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}): the library runs on one device",
              file=sys.stderr)
        sys.exit(2)

    from paper_2305_17341_amd import he, inputs as I
    chain = I.LARGE
    d, B = args.d, args.batch
    log(f"[bench] context N=2^{chain.log_n}, {len(chain.q_bits)} Q primes, {len(chain.p_bits)} P primes")
    ctx = he.chain_context(chain, seed=1)
    # the product's geometry: baby steps of Z and T, blocks of the shifts
    geo = {"n1_z": args.n1, "n1_t": args.n1} if args.n1 > 0 else {}
    steps = ctx.matmul_rot_steps(d, dict(geo) if geo else None)
    t0 = time.perf_counter()
    ctx.keygen(steps)
    log(f"[bench] keygen: {len(steps)} rotation keys + relin in {time.perf_counter() - t0:.1f} s")
    As = [I.uniform_matrix(100 + i, d) for i in range(B)]
    Bs = [I.uniform_matrix(200 + i, d) for i in range(B)]
    cA = [ctx.encrypt_matrix(a, nonce=1 + i) for i, a in enumerate(As)]
    cB = [ctx.encrypt_matrix(b, nonce=1001 + i) for i, b in enumerate(Bs)]
    ctx.sync()

    BATCHED, LAZY, FUSED, GRAPH = 1, 2, 4, 8
    relin = "paper" if args.paper_relin else "lazy"
    head = {"flags": BATCHED | (0 if args.paper_relin else LAZY | (0 if args.two_roundings else FUSED)) |
            (0 if args.no_graph else GRAPH), **geo}

    class Names(dict):
        def __missing__(self, f):
            parts = ["batched" if f & BATCHED else "plain"]
            parts += [w for bit, w in ((LAZY, "lazy-relin"), (FUSED, "fused-rescale"), (GRAPH, "hip-graph"))
                      if f & bit]
            return "+".join(parts)
    names = Names()

    def timed(opts, profile, warmup=True):
        """warm-up then `--steps` timed steps of B products; returns (seconds, per-step ms, outputs of warm-up)"""
        outs = None
        for w in range(args.warmup if warmup else 0):
            t0 = time.perf_counter()
            outs = ctx.matmul_batch(cA, cB, [d] * B, opts=opts)
            ctx.sync()
            log(f"[bench] warmup {w} ({names[opts['flags'] if opts else 0]}): {time.perf_counter() - t0:.2f} s")
        if profile:
            ctx.profile_enable(True)
        lat = []
        ctx.sync()
        t_start = time.perf_counter()
        for _ in range(args.steps):
            o = ctx.matmul_batch(cA, cB, [d] * B, opts=opts)
            lat.append(ctx.last_op_ms())
            del o
        ctx.sync()
        t_total = time.perf_counter() - t_start
        log(f"[bench] {args.steps} timed steps ({names[opts['flags'] if opts else 0]}): {t_total:.2f} s")
        return t_total, lat, outs

    tuned = None
    for kv in filter(None, args.knobs.split(",")):
        name, v = kv.split("=")
        he.knob_set(name.strip(), int(v))
    tuned = {"knobs": {k: he.knob_get(k) for k in autotune_knobs()}, "step_ms": None}
    if not args.no_autotune:
        from paper_2305_17341_amd import autotune
        # launched one kernel at a time: a recording would keep the shapes it
        # was made with (the headline records after the knobs are set)
        tune_opts = {"flags": head["flags"] & ~GRAPH, **geo}
        warm = ctx.matmul_batch(cA, cB, [d] * B, opts=tune_opts)   # plaintext caches
        ctx.sync()
        del warm
        best, tt = autotune.autotune(ctx, cA, cB, d, opts=tune_opts, log=log)
        tuned = {"knobs": best, "step_ms": tt}

    plain_outs = None
    if not args.no_plain:
        t_plain, lat_plain, plain_outs = timed({"flags": 0, **geo}, False)
        t_bp, lat_bp, bp_outs = timed({"flags": BATCHED, **geo}, False)
        # batching gives the one-at-a-time residues
        same = all(np.array_equal(p.export(), q.export()) for p, q in zip(plain_outs, bp_outs))
        del bp_outs
    # headline: the library as deployed (no per-kernel events; with the
    # recorded graph, the warm-up records it and the timed steps replay it)
    t_total, lat, outs = timed(head, False)
    # the same steps again, launched one kernel at a time with HIP events
    # around every launch: the kernel table, the roofline's per-launch
    # durations and the operation counts come from these
    eager = {"flags": head["flags"] & ~GRAPH, **geo}
    c0 = ctx.op_counts()
    t_prof, _, _ = timed(eager, True, warmup=False)
    c1 = ctx.op_counts()
    fams = ["ntt_fwd_cols", "ntt_fwd_cols_modup", "ntt_fwd_cols_fbc", "ntt_fwd_cols_lift", "ntt_fwd_rows",
            "ntt_fwd_rows_sub",
            "ntt_inv_rows", "ntt_inv_cols", "multsum", "multsum_rot", "multsum_rot_int", "modup", "fbc_prep",
            "fbc_to_q",
            "moddown_final", "rescale_lift", "rescale_final", "elementwise", "tensor", "plift"]
    # device-to-device copies (stacking, gathers before a transform): step
    # time, not algorithmic work, so kept out of the roofline sums
    copy_fams = ["copy_ct", "copy_limbs", "copy_gather", "copy_decompose", "copy_stack", "copy_unstack"]
    prof = {f: ctx.profile_read(f) for f in fams + copy_fams}
    ops = {f: ctx.profile_read_ops(f) for f in fams}
    ctx.profile_enable(False)
    n_mm = args.steps * B
    per_mm = {k: (c1[k] - c0[k]) / n_mm for k in c0}
    # accuracy of a warm-up output against FP64; the headline path batched == alone
    err = float(np.max(np.abs(ctx.decrypt(outs[0], d * d) - (As[0] @ Bs[0]).ravel())))
    alone = ctx.matmul(cA[0], cB[0], d, opts={"flags": head["flags"] & ~(BATCHED | GRAPH), **geo})
    head_same = bool(np.array_equal(alone.export(), outs[0].export()))
    del outs, plain_outs, alone

    # key-switched rotations at the top level: one at a time (plain), and
    # hoisted over a batch (one Decompose, one multi-rotation launch)
    ct = cA[0]
    ctx.sync()
    t0 = time.perf_counter()
    for _ in range(args.rotations):
        r = ctx.rotate(ct, 1)
        del r
    ctx.sync()
    rot_s = args.rotations / (time.perf_counter() - t0) if args.rotations > 0 else None
    rot_steps = list(range(1, args.n1)) if args.n1 > 1 else list(range(1, 16))
    rb = ctx.rotate_many(cA, rot_steps)   # warm-up
    ctx.sync()
    del rb
    t0 = time.perf_counter()
    for _ in range(2):
        rb = ctx.rotate_many(cA, rot_steps)
        del rb
    ctx.sync()
    rot_batched_s = 2 * len(cA) * len(rot_steps) / (time.perf_counter() - t0)
    for _ in range(args.calib_copies):
        r = ctx.rotate(ct, 0)   # step 0: a plain device copy of 2 x 31 limbs
        del r
    ctx.sync()

    value = args.steps * B / t_total
    step_s = t_total / args.steps
    fam_ms = {f: prof[f][0] / args.steps for f in fams + copy_fams}
    dom = max(fams, key=lambda f: prof[f][0])
    ms, launches, nbytes = prof[dom]
    mmf, mmi, unit_bytes = ops[dom]
    avg_ms = ms / max(launches, 1)
    bytes_per_launch = nbytes / max(launches, 1)
    unit_per_launch = unit_bytes / max(launches, 1)
    achieved_io = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    achieved = unit_per_launch / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic(dom, args.n1, {k: he.knob_get(k) for k in autotune_knobs()})
    # VALU side: measured ceilings of the products (lazy FP64 for moduli below
    # 2^46, Shoup for the others) against each family's algorithmic products
    peaks = valu_ceilings(log)
    pf, pi = peaks["f64_lazy"]["measured"], peaks["shoup"]["measured"]

    def valu_floor_s(f):
        a, b, _ = ops[f]
        return a / pf + b / pi
    valu_frac = valu_floor_s(dom) / (ms * 1e-3) if ms > 0 else None
    hbm_frac = achieved / HBM_PEAK_GBS
    step_unit_bytes = sum(ops[f][2] for f in fams) / args.steps
    step_mm = sum(ops[f][0] + ops[f][1] for f in fams) / args.steps
    step_valu_s = sum(valu_floor_s(f) for f in fams) / args.steps
    roofline = {"kernel": dom, "bound": "hbm" if hbm_frac >= (valu_frac or 0) else "alu",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(hbm_frac, 4),
                "traffic": None if traffic is None else round(traffic),
                "avg_launch_ms": round(avg_ms, 5), "launches": launches,
                "algorithmic_bytes_per_launch": round(unit_per_launch),
                "bytes_rule": "key switch unit: each switching key read once per launch (2 beta (l+1+alpha) limbs), "
                              "each member's ciphertext read and written once per rotation (4 (l+1) limbs)",
                "kernel_io_bytes_per_launch": round(bytes_per_launch),
                "kernel_io_achieved": round(achieved_io, 1), "kernel_io_frac": round(achieved_io / HBM_PEAK_GBS, 4),
                "valu": {"modmuls_per_launch": round((mmf + mmi) / max(launches, 1)),
                         "modmuls_f64_share": round(mmf / max(mmf + mmi, 1), 4),
                         "achieved_modmuls_per_s": round((mmf + mmi) / max(launches, 1) / (avg_ms * 1e-3), 1),
                         "frac": None if valu_frac is None else round(valu_frac, 4),
                         "rule": "time the kernel's algorithmic modular products need at the measured ceilings "
                                 "(lazy FP64 products / f64_lazy rate + integer products / shoup rate) over the "
                                 "measured launch time"},
                "valu_ceilings_modmuls_per_s": peaks,
                "step": {"ms": round(step_s * 1e3, 3),
                         "algorithmic_bytes": round(step_unit_bytes),
                         "hbm_frac": round(step_unit_bytes / step_s / (HBM_PEAK_GBS * 1e9), 4),
                         "modmuls": round(step_mm),
                         "valu_frac": round(step_valu_s / step_s, 4)}}
    # sigma, tau, the d column shifts (merged into their ModDowns when the A
    # side rounds once), the final product
    n_rescale = 2 + 1 + (0 if head["flags"] & FUSED else d)
    result = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "matmuls/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * t_total / args.steps, 3),
        "profiled_ms_per_step": round(1e3 * t_prof / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"he_matmul d={d} at N=2^16 (q0 60b + 30x40b, P 3x60b, levels 30->27), "
                               f"uniform[-1,1] FP64 inputs", "d": d, "log_n": chain.log_n, "batch": B,
                   "path": names[head["flags"]], "relinearisation": relin,
                   "variants": None if args.paper_relin else (
                       "lazy relinearisation (the d tensors summed, relinearised once)" +
                       ("" if args.two_roundings else " and one rounding for the A side's ModDown and Rescale") +
                       ": variants of the paper's order (relinearisation per product, two roundings), each with "
                       "its own oracle plan; batched_paper_relin is the paper's order"),
                   "n1": args.n1 if args.n1 > 0 else None, "rotation_keys": len(steps)},
        "batched_residues_equal_alone": head_same,
        "autotune": tuned,
        "plain": None if args.no_plain else {
            "value": round(args.steps * B / t_plain, 4), "unit": "matmuls/s",
            "what": "one product after another, one launch sequence each, relinearisation per product "
                    "(the paper's order)",
            "latency_ms": {"p50": pct(lat_plain, 50), "p99": pct(lat_plain, 99)}},
        "batched_paper_relin": None if args.no_plain else {
            "value": round(args.steps * B / t_bp, 4), "unit": "matmuls/s",
            "latency_ms": {"p50": pct(lat_bp, 50), "p99": pct(lat_bp, 99)},
            "speedup_vs_plain": round(t_plain / t_bp, 3), "residues_identical_to_plain": same},
        "speedup_vs_plain": None if args.no_plain else round(t_plain / t_total, 3),
        "rotations_per_s": round(rot_s, 2) if rot_s else None,
        "rotations_per_s_batched": {"value": round(rot_batched_s, 2),
                                    "what": f"{len(cA)} ciphertexts x {len(rot_steps)} steps per call, hoisted: one "
                                            "Decompose of the batch, one multi-rotation launch, one ModDown per "
                                            "step (he_rotate_many)",
                                    "speedup_vs_plain": round(rot_batched_s / rot_s, 3) if rot_s else None},
        "latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99)},
        "max_abs_err": err,
        "op_counts_per_matmul": per_mm,
        "kernel_ms_per_step": {f: round(v, 3) for f, v in fam_ms.items()},
        "kernel_algorithmic_gbs": {f: round(prof[f][2] / (prof[f][0] * 1e-3) / 1e9, 1)
                                   for f in fams if prof[f][0] > 0},
        # per family: HBM fraction of its algorithmic bytes, and the fraction of
        # its time its algorithmic modular products need at the measured ceilings
        "kernel_fracs": {f: {"hbm": round(ops[f][2] / (prof[f][0] * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
                             "valu": round(valu_floor_s(f) / (prof[f][0] * 1e-3), 4)}
                         for f in fams if prof[f][0] > 0},
        "roofline": roofline,
    }
    # the headline's keys, recorded graph and pool go back to the device
    # before the serving run sizes its budget from the free memory
    ctx.close()
    if args.serve_jobs > 0:
        from paper_2305_17341_amd import serve
        log("[bench] serving run ...")
        result["serving"] = serve.serve_bench(["--jobs", str(args.serve_jobs), "--loads", args.serve_loads,
                                               "--cov-samples", str(args.serve_cov_samples)])
    # each part below builds and closes its own contexts; collect what the
    # previous part left so that its device memory is back before the next
    import gc

    def free_gib():
        from paper_2305_17341_amd import he as H
        return f"{H.device_memory()[0] / 2**30:.0f} GiB free"

    gc.collect()
    if args.pca_components > 0:
        from paper_2305_17341_amd import pca
        log(f"[bench] PCA run ({free_gib()}) ...")
        result["pca"] = pca.pca_bench(l_e=args.pca_components, log=log)
        log("[bench] PCA run, Goldschmidt's inverse square root and packed vector refreshes ...")
        result["pca_goldschmidt_packed"] = pca.pca_bench(l_e=args.pca_components, log=log, goldschmidt=True,
                                                         pack=True)
    gc.collect()
    if args.big_covariance > 0:
        from paper_2305_17341_amd import pca
        log(f"[bench] covariance of {args.big_covariance} x 256 samples ...")
        result["big_covariance"] = pca.covariance_bench(s=args.big_covariance, log=log)
    gc.collect()
    if not args.no_accuracy:
        from paper_2305_17341_amd import pca
        log(f"[bench] PPPCA accuracy runs ({free_gib()}) ...")
        result["pca_accuracy"] = pca.accuracy_bench(log=log)
    gc.collect()
    if args.table3_reps > 0:
        from paper_2305_17341_amd import table3
        log(f"[bench] Z/T decomposition table ({free_gib()}) ...")
        result["table3"] = table3.run(reps=args.table3_reps, log=log)
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle sample ...")
        result["cpu_baseline"] = cpu_baseline(chain, per_mm, n_rescale, d, log=log)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
