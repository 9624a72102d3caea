#!/usr/bin/env python
"""Benchmark: Schwarz-factorised two-flavour determinant-ratio estimates per second on MI355X.

One step = one pass of the whole hot path over one batch: the Schur-complement
estimator of Eq. (8) on the 48x24^3 lattice with 6^4 Schwarz blocks, all 12 noise
vectors of the step as one multi-RHS batch: D_wb hop, four persistent block sweeps,
D_bw hops, projector, one global mixed-precision solve (FP32 BiCGStab inside FP64
defect correction), the FP64 reductions for x_ij and the log-domain combination.
Inputs (synthetic links, complex Gaussian noise) are resident in HBM before timing.

Also measured: the plain FP64 single-RHS GPU path on the same noise vectors, the
agreement of both with the FP64 oracle, the dominant kernel's HBM roofline from HIP
events over the timed region, and the C oracle timed on a bounded CPU sample.
Prints ONE JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
# FP32 vector peak without packed instructions (which the library does not use): 256 CUs x 4 SIMDs x
# 16 lanes x 2 flops (FMA) x 2.4 GHz
FP32_VALU_TFLOPS = 78.6
METRIC = "Dslash GB/s (% HBM peak); det-ratio estimates/s, mixed vs FP64 at 1e-8"
DESCRIPTIONS = {
    "48x24^3": "Schur det-ratio estimate, 48x24^3, 6^4 blocks (512), Wilson-clover c_sw=1, kappa 0.1200->0.1205, "
       "N_hit=12 as one multi-RHS batch, FP32 block/inner solves + FP64 defect correction",
    "64x32^3": "Schur det-ratio estimate, 64x32^3, 8^4 blocks (512), Wilson-clover c_sw=1, kappa 0.1200->0.1205 in "
       "N=4 mass-interpolation steps, 24 RHS as one multi-RHS batch, FP32 block/inner solves + FP64 defect "
       "correction",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=("48x24", "64x32"), default="48x24",
                    help="48x24: 48x24^3, 6^4 blocks, 12 RHS (default); 64x32: 64x32^3, 8^4 blocks, 4 steps, 24 RHS")
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--inner", choices=("fp32", "fp16"), default=None,
                    help="storage of the global inner solver (default: fp32 at 48x24, fp16 at 64x32)")
    ap.add_argument("--fp64-samples", type=int, default=2, help="noise vectors for the FP64 single-RHS path")
    ap.add_argument("--cpu-threads-1", action="store_true",
                    help="also time one oracle estimate on a single thread (about 16x the all-core time)")
    ap.add_argument("--profile-steps", type=int, default=3, help="steps of the profiled pass (kernel timings)")
    ap.add_argument("--stream-gib", type=float, default=4.0, help="GiB of the streaming reference copy (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default schedule options")
    ap.add_argument("--nested", action="store_true",
                    help="time the nested-DD factor instead (64x32^3: 8^4 blocks split into 4^4 blocks)")
    ap.add_argument("--grad", action="store_true",
                    help="time the gradient of log W_gl in kappa2 and the links instead (32x16^3, 4^4 blocks)")
    ap.add_argument("--blockdet", action="store_true",
                    help="time the exact block determinants of both colours instead (48x24^3, 6^4 blocks)")
    ap.add_argument("--one-flavour", action="store_true",
                    help="time the one-flavour estimator (Eq. 11) instead (48x24^3)")
    ap.add_argument("--solver", choices=("bicgstab", "sap-gcr"), default="bicgstab",
                    help="global solver: even-odd BiCGStab or GCR preconditioned by Schwarz sweeps")
    ap.add_argument("--block-kernel", choices=("auto", "global"), default="auto",
                    help="Schwarz block inner solver: LDS-resident where it fits (auto) or the global-memory kernel")
    ap.add_argument("--dslash-reps", type=int, default=20, help="launches per standalone Dslash measurement")
    ap.add_argument("--copy-calibration", type=float, default=0.0, metavar="GIB",
                    help="only run a device-to-device copy of this many GiB (calibrates HBM counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (the estimates of Eq. (8) "
              "are independent, so several GPUs would each run their own noise vectors).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration > 0:
        # three launches of the library's streaming copy (ddwc_stream_copy) of a known size
        import paper_1211_1214_amd as dd
        n = int(args.copy_calibration * (1 << 30)) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(3):
            dd.binding.stream_copy(a, b)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 3,
                          "kernel": "k_stream_copy"}), flush=True)
        return

    import paper_1211_1214_amd as dd
    from paper_1211_1214_amd import inputs

    if args.nested:
        return nested_bench(args, dd, inputs, np, torch)
    if args.grad:
        return grad_bench(args, dd, inputs, np, torch)
    if args.blockdet:
        return blockdet_bench(args, dd, inputs, np, torch)
    if args.one_flavour:
        return one_flavour_bench(args, dd, inputs, np, torch)
    wname = "48x24^3" if args.workload == "48x24" else "64x32^3"
    cfg = inputs.WORKLOADS[wname]
    lat, blk, nhit, nint = cfg["lat"], cfg["blk"], cfg["n_hit"], cfg["n_interp"]
    k1, k2 = cfg["kappa1"], cfg["kappa2"]
    dev = torch.device("cuda:0")
    t = time.time()
    U = inputs.make_links(lat, cfg["eps"], cfg["seed"])
    eta = inputs.make_noise_batch(lat, cfg["seed"], nint, nhit)
    log(f"inputs generated in {time.time() - t:.1f}s")
    Ud = torch.from_numpy(U).to(dev)
    etad = torch.from_numpy(eta).to(dev)
    ctx = dd.Context(Ud, lat, blk, -1, cfg["csw"])
    torch.cuda.synchronize()

    inner = args.inner or ("fp32" if wname == "48x24^3" else "fp16")
    prec = dd.MIXED16 if inner == "fp16" else dd.MIXED32
    if args.solver == "sap-gcr":
        ctx.set_option(dd.binding.OPT_SOLVER, 1)
    if args.block_kernel == "global":
        ctx.set_option(dd.binding.OPT_BLOCK_KERNEL, 1)
    tuned = ctx.autotune(k2, nhit, prec) if not args.no_autotune else None
    log(f"autotune: {tuned}")

    def step():
        return ctx.det_ratio_estimate(k1, k2, etad, op=dd.OP_SCHUR, tol=args.tol, prec=prec)

    for w in range(args.warmup):
        r = step()
        log(f"warmup {w}: log W_gl {r['log_w_gl']:.10f}, {r['stats']}")
    # the timed region: what ships (the autotuned schedule, graph replay allowed, no per-launch events)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        r = step()
        log(f"step {k}: log W_gl {r['log_w_gl']:.10f}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    value = nint * nhit * args.steps / elapsed
    x_mixed = r["x"]
    log(f"timed {args.steps} steps in {elapsed:.3f}s: {value:.2f} estimates/s")

    # profiled pass: the same step with HIP events around every launch on its stream (graphs off
    # while profiling) for the kernel classes and the roofline of the dominant kernel
    psteps = max(1, min(args.profile_steps, args.steps))
    ctx.profile_enable(True)
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    for k in range(psteps):
        step()
    torch.cuda.synchronize()
    prof_elapsed = time.perf_counter() - tp0
    prof = {name: ctx.profile_read(kc) for name, kc in
            (("dslash64", dd.binding.K_DSLASH64), ("dslash32", dd.binding.K_DSLASH32), ("eohop", dd.binding.K_EOHOP),
             ("block", dd.binding.K_BLOCK), ("blas", dd.binding.K_BLAS), ("other", dd.binding.K_OTHER))}
    ctx.profile_enable(False)
    log(f"profiled {psteps} steps in {prof_elapsed:.3f}s; profile {prof}")

    # FP64 single-RHS path on the first noise vectors (all interpolation steps)
    fp64_t = 0.0
    x64 = []
    for j in range(args.fp64_samples):
        torch.cuda.synchronize()
        ta = time.perf_counter()
        r64 = ctx.det_ratio_estimate(k1, k2, etad[:, j:j + 1].contiguous(), op=dd.OP_SCHUR, tol=args.tol,
                                     prec=dd.FP64)
        torch.cuda.synchronize()
        fp64_t += time.perf_counter() - ta
        x64.append(r64["x"][:, 0])
    fp64_rate = nint * args.fp64_samples / fp64_t if args.fp64_samples else None

    dslash = dslash_rates(ctx, dd, inputs, lat, dev, args.dslash_reps) if args.dslash_reps > 0 else None
    stream_gbs = stream_peak(dd, torch, gib=args.stream_gib) if args.stream_gib > 0 else None

    # parity against the stored oracle values (written by tests/golden/make_golden_{48x24,64x32}.py)
    parity = {}
    gpath = os.path.join(ROOT, "tests", "golden", f"oracle_{args.workload}.json")
    golden = json.load(open(gpath)) if os.path.exists(gpath) else None
    if golden:
        worst = 0.0
        for key, xo in golden["x_schur"].items():
            i, j = (0, int(key)) if "," not in key else map(int, key.split(","))
            e = abs(x_mixed[i, j] - xo) / max(abs(xo), 1.0)
            worst = max(worst, e)
            if j < len(x64):
                parity[f"x{i}{j}_fp64_rel"] = abs(x64[j][i] - xo) / max(abs(xo), 1.0)
        parity["x_mixed_rel_max"] = worst
        parity["x_compared"] = len(golden["x_schur"])
        if "log_w_gl" in golden:
            lw = golden["log_w_gl"]
            parity["log_w_gl_oracle"] = lw
            parity["log_w_gl_rel"] = abs(r["log_w_gl"] - lw) / max(abs(lw), 1.0)
            parity["step_var_rel"] = abs(r["step_var"][0] - golden["step_var"]) / golden["step_var"]
    d = max((abs(x_mixed[i, j] - x64[j][i]) / max(abs(x64[j][i]), 1.0) for j in range(len(x64))
             for i in range(nint)), default=None)
    parity["x_mixed_vs_fp64_rel_max"] = d

    # Roofline of the Dslash the metric names: the even-odd hop-and-inverse kernel of the global
    # solver (one kernel; HIP-event durations of its launches in the profiled pass).
    roofline, _ = class_roofline(prof)
    dom = roofline["kernel"]
    ds_ms, ds_b = prof["dslash32"]["ms"] + prof["eohop"]["ms"], prof["dslash32"]["bytes"] + prof["eohop"]["bytes"]
    dslash_gbs = ds_b / (ds_ms * 1e-3) / 1e9 if ds_ms > 0 else None
    block = block_summary(prof["block"])
    if roofline["bound"] == "hbm":
        roofline["traffic"] = measured_traffic(args.workload, dom, ctx.get_option(dd.binding.OPT_OP_THREADS))
        roofline["peak_measured"] = None if stream_gbs is None else round(stream_gbs, 1)
        roofline["frac_of_measured"] = None if not stream_gbs else round(roofline["achieved"] / stream_gbs, 4)
    roofline["timing"] = f"HIP events around each launch on its stream, profiled pass of {psteps} steps"

    cpu = None
    if wname == "48x24^3" and not args.no_cpu_baseline and golden:
        cpu = cpu_baseline(U, eta[0, 0], cfg, golden, args.cpu_threads_1)

    total_ms = sum(p["ms"] for p in prof.values())
    line = {
        "metric": METRIC, "value": round(value, 3), "unit": "estimates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * elapsed / args.steps, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 inner / f64 outer" if inner == "fp32" else "f16 storage, f32 arithmetic inner / f64 outer",
        "data": "synthetic",
        "config": {"workload": DESCRIPTIONS[wname] + ("" if inner == "fp32" else
                                                 "; global inner solver in FP16 storage (per-site scales, FP16 links)"),
                   "lattice": list(lat), "blocks": list(blk), "n_interp": nint, "n_hit": nhit, "tol": args.tol,
                   "inner": inner, "solver": args.solver, "block_kernel": args.block_kernel},
        "roofline": roofline,
        "schedule": tuned,
        "cpu_baseline": cpu,
        "dslash": dslash,
        "block_solver": block,
        "dslash32_in_solver_gbs": None if dslash_gbs is None else round(dslash_gbs, 1),
        "dslash32_in_solver_frac": None if dslash_gbs is None else round(dslash_gbs / HBM_PEAK_GBS, 4),
        "fp64_single_rhs_estimates_per_s": None if fp64_rate is None else round(fp64_rate, 3),
        "speedup_vs_fp64_single_rhs": None if not fp64_rate else round(value / fp64_rate, 2),
        "parity": parity,
        "log_w_gl": r["log_w_gl"],
        "profiled_ms_per_step": round(1e3 * prof_elapsed / psteps, 3),
        "kernel_time_share": {k: round(p["ms"] / total_ms, 3) for k, p in prof.items()} if total_ms else None,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


def stream_peak(dd, torch, gib=4.0, reps=5):
    """The library's streaming reference copy (ddwc_stream_copy) of a `gib` GiB buffer: read plus
    written bytes over the shortest of `reps` durations from torch events on the launch stream."""
    n = int(gib * (1 << 30)) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    dd.binding.stream_copy(a, b)
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dd.binding.stream_copy(a, b)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) * 1e-3)
    gbs = 2 * 4 * n / min(times) / 1e9
    log(f"stream copy: {gbs:.0f} GB/s (read + write, {gib} GiB)")
    del a, b
    return gbs


def block_summary(pb):
    """The persistent block solver class: launches, duration, and its ALU roofline (FP32 vector
    rate without packed instructions); its working set is on chip and in the caches, so an HBM
    fraction does not apply."""
    if not pb["launches"]:
        return None
    flops = pb["bytes"]  # the block class accumulates flops in the byte slot (see the library's model)
    tf = flops / (pb["ms"] * 1e-3) / 1e12 if pb["ms"] > 0 else 0.0
    return {"launches": pb["launches"], "avg_launch_us": round(1e3 * pb["ms"] / pb["launches"], 2),
            "bound": "alu", "achieved": round(tf, 2), "peak": FP32_VALU_TFLOPS, "unit": "TFLOP/s",
            "frac": round(tf / FP32_VALU_TFLOPS, 4)}


def kernel_sources_digest():
    """Digest of the library's kernel sources and build flags: a stored counter measurement is
    used only while it matches the code that is running."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1211_1214_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h")):
            h.update(f.encode())
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(fh.read())
    with open(os.path.join(ROOT, "paper_1211_1214_amd", "build.py"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


# kernel whose counters stand for each profiler class
# kernel of a profiling class in the counter records; {nt}: the operator workgroup size in use
CLASS_KERNEL = {"eohop": "void ddwc::k_eo_hopinv<float, true, true, {nt}>", "block": "ddwc::k_blk_lds"}


def nested_bench(args, dd, inputs, np, torch):
    """Nested DD on the 64x32^3 workload: the Schur factor of the 8^4 blocks of each colour over
    4^4 inner blocks (ddwc_det_ratio_nested), the first interpolation step with 24 RHS per
    colour, FP16 storage in the inner solves.  One timed step = both colours."""
    cfg = inputs.WORKLOADS["64x32^3"]
    lat, blk, nhit = cfg["lat"], cfg["blk"], cfg["n_hit"]
    inner = (4, 4, 4, 4)
    m1, m2 = 1 / (2 * cfg["kappa1"]) - 4, 1 / (2 * cfg["kappa2"]) - 4
    k_step = 1 / (2 * (m1 + (m2 - m1) / cfg["n_interp"] + 4))
    prec = dd.MIXED16 if (args.inner or "fp16") == "fp16" else dd.MIXED32
    dev = torch.device("cuda:0")
    t = time.time()
    Ud = torch.from_numpy(inputs.make_links(lat, cfg["eps"], cfg["seed"])).to(dev)
    O = dd.Context(Ud, lat, blk, -1, cfg["csw"])
    I = dd.Context(Ud, lat, inner, -1, cfg["csw"])
    del Ud
    etas = [torch.from_numpy(inputs.make_noise_batch(lat, 40 + c, 1, nhit)).to(dev) for c in (0, 1)]
    log(f"nested: contexts and noise in {time.time() - t:.1f}s")

    def step():
        return [O.det_ratio_nested(I, c, cfg["kappa1"], k_step, etas[c], tol=args.tol, prec=prec) for c in (0, 1)]

    for w in range(args.warmup):
        r = step()
        log(f"nested warmup {w}: log W_c {r[0]['log_w']:.10f} {r[1]['log_w']:.10f}")
    for c in (O, I):
        c.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        r = step()
        log(f"nested step {k}: log W_c {r[0]['log_w']:.10f} {r[1]['log_w']:.10f}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = class_profile(dd, [O, I])
    for c in (O, I):
        c.profile_enable(False)
    value = 2 * nhit * args.steps / elapsed
    roofline, share = class_roofline(prof)
    parity = {}
    gpath = os.path.join(ROOT, "tests", "golden", "oracle_nested_64x32.json")
    if os.path.exists(gpath):
        for key, xo in json.load(open(gpath))["x_nested"].items():
            c, i, j = map(int, key.split(","))
            parity[f"x{c}_{i}{j}_rel"] = abs(r[c]["x"][i, j] - xo) / max(abs(xo), 1.0)
    line = {
        "metric": "nested-DD Schur-factor estimates/s", "value": round(value, 3), "unit": "estimates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f16 storage, f32 arithmetic inner / f64 outer" if prec == dd.MIXED16 else "f32 inner / f64 outer",
        "data": "synthetic",
        "config": {"workload": "nested DD factor, 64x32^3, 8^4 outer blocks split into 4^4 inner blocks, "
                               "Wilson-clover c_sw=1, step kappa 0.1200 -> m_1 of 4 interpolation steps, 24 RHS "
                               "per outer colour, both colours per step",
                   "lattice": list(lat), "outer_blocks": list(blk), "inner_blocks": list(inner), "n_hit": nhit,
                   "tol": args.tol},
        "roofline": roofline,
        "cpu_baseline": None,
        "parity": parity,
        "log_w": [r[0]["log_w"], r[1]["log_w"]],
        "kernel_time_share": share,
    }
    print(json.dumps(line), flush=True)
    O.close()
    I.close()


CLASSES = ("dslash64", "dslash32", "eohop", "block", "blas", "other")


def class_profile(dd, ctxs):
    """Launches, milliseconds and algorithmic bytes per kernel class, summed over contexts."""
    ids = {"dslash64": dd.binding.K_DSLASH64, "dslash32": dd.binding.K_DSLASH32, "eohop": dd.binding.K_EOHOP,
           "block": dd.binding.K_BLOCK, "blas": dd.binding.K_BLAS, "other": dd.binding.K_OTHER}
    prof = {}
    for name in CLASSES:
        reads = [c.profile_read(ids[name]) for c in ctxs]
        prof[name] = {k: sum(r[k] for r in reads) for k in reads[0]}
    return prof


def class_roofline(prof):
    """HBM roofline of the Dslash: the even-odd hop kernel, else the operator class with the most
    time; when no operator class ran (FP64-only or block-only paths), the ALU roofline of the
    persistent block solver, whose class accumulates the model's flops (its working set is on chip
    and in the caches).  Also the time share of every class."""
    ops = [k for k in ("eohop", "dslash32", "dslash64") if prof[k]["launches"]]
    total_ms = sum(p["ms"] for p in prof.values())
    share = {k: round(p["ms"] / total_ms, 3) for k, p in prof.items()} if total_ms else None
    if not ops:
        b = block_summary(prof["block"]) or {"launches": 0, "avg_launch_us": 0.0, "achieved": 0.0, "frac": 0.0}
        return ({"bound": "alu", "achieved": b["achieved"], "peak": FP32_VALU_TFLOPS, "unit": "TFLOP/s",
                 "frac": b["frac"], "traffic": None, "kernel": "block", "launches": b["launches"],
                 "avg_launch_us": b["avg_launch_us"]}, share)
    dom = "eohop" if "eohop" in ops else max(ops, key=lambda k: prof[k]["ms"])
    pd = prof[dom]
    per_ms = pd["ms"] / max(pd["launches"], 1)
    per_b = pd["bytes"] / max(pd["launches"], 1)
    achieved = per_b / (per_ms * 1e-3) / 1e9 if pd["ms"] > 0 else 0.0
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dom, "launches": pd["launches"],
            "avg_launch_us": round(per_ms * 1e3, 2), "bytes_per_launch": per_b}
    return roof, share


def grad_bench(args, dd, inputs, np, torch):
    """Differentiation on the 32x16^3 workload (4^4 blocks, N_hit = 8): d log W_gl / d kappa2 and
    d log W_gl / dU through ddwc_det_ratio_grad (adjoint solves, force kernels), Schur form, FP32
    inner solves.  One timed step = one gradient over all N_hit noise vectors."""
    cfg = inputs.WORKLOADS["32x16^3"]
    lat, blk, nhit, nint = cfg["lat"], cfg["blk"], cfg["n_hit"], cfg["n_interp"]
    k1, k2 = cfg["kappa1"], cfg["kappa2"]
    dev = torch.device("cuda:0")
    ctx = dd.Context(torch.from_numpy(inputs.make_links(lat, cfg["eps"], cfg["seed"])).to(dev), lat, blk, -1,
                     cfg["csw"])
    eta = torch.from_numpy(inputs.make_noise_batch(lat, cfg["seed"], nint, nhit)).to(dev)
    tuned = ctx.autotune(k2, nhit, dd.MIXED32) if not args.no_autotune else None
    r = ctx.det_ratio_estimate(k1, k2, eta, op=dd.OP_SCHUR, tol=args.tol, prec=dd.MIXED32)
    # dL/dx_ij of L = log W_gl = sum_i [logsumexp_j(-x_ij) - ln N_hit]
    a = -r["x"] - (-r["x"]).max(axis=1, keepdims=True)
    gx = -np.exp(a) / np.exp(a).sum(axis=1, keepdims=True)

    def step():
        return ctx.det_ratio_grad(k1, k2, eta, gx, op=dd.OP_SCHUR, tol=args.tol, prec=dd.MIXED32)

    for _ in range(args.warmup):
        g = step()
    ctx.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        g = step()
        log(f"grad step {k}: dlogW/dkappa2 {g['dkappa2']:.10e}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = class_profile(dd, [ctx])
    ctx.profile_enable(False)
    roofline, share = class_roofline(prof)
    line = {
        "metric": "gradient estimates/s (d log W_gl / d kappa2 and d / dU, per noise vector)",
        "value": round(nint * nhit * args.steps / elapsed, 3), "unit": "estimates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32 inner / f64 outer",
        "data": "synthetic",
        "config": {"workload": "gradient of log W_gl, 32x16^3, 4^4 blocks, Wilson-clover c_sw=1, kappa "
                               "0.1200->0.1205, N_hit=8 as one multi-RHS batch, Schur form",
                   "lattice": list(lat), "blocks": list(blk), "n_hit": nhit, "tol": args.tol},
        "roofline": roofline, "schedule": tuned, "cpu_baseline": None,
        "dkappa2": g["dkappa2"], "dU_norm": float(g["dU"].abs().pow(2).sum().sqrt()),
        "kernel_time_share": share,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


def blockdet_bench(args, dd, inputs, np, torch):
    """Exact block determinants on the 48x24^3 workload: ln|det D_k(m)| of all 512 blocks of 6^4
    (even-odd reduced matrices of dimension 7776 assembled by the library's kernels, batched
    complex LU by rocSOLVER).  One timed step = both colours at one mass."""
    cfg = inputs.WORKLOADS["48x24^3"]
    lat, blk = cfg["lat"], cfg["blk"]
    dev = torch.device("cuda:0")
    ctx = dd.Context(torch.from_numpy(inputs.make_links(lat, cfg["eps"], cfg["seed"])).to(dev), lat, blk, -1,
                     cfg["csw"])
    nblk = int(np.prod([l // b for l, b in zip(lat, blk)]))
    n = 12 * int(np.prod(blk)) // 2
    for _ in range(args.warmup):
        ctx.block_logdet(cfg["kappa2"], 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        la = [ctx.block_logdet(cfg["kappa2"], c)[0] for c in (0, 1)]
        log(f"blockdet step {k}: sum ln|det| {sum(x.sum() for x in la):.10e}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    flops = nblk * 8.0 / 3.0 * n ** 3  # complex LU of the even-odd reduced block matrices
    achieved = flops * args.steps / elapsed / 1e12
    line = {
        "metric": "block determinants/s", "value": round(nblk * args.steps / elapsed, 3), "unit": "blocks/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "ln|det D_k| of all 512 Schwarz blocks (6^4, both colours) at 48x24^3, "
                               "even-odd reduced dimension 7776, batched complex LU",
                   "lattice": list(lat), "blocks": list(blk), "matrix_dim": n},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 2), "peak": 78.6, "unit": "TFLOP/s",
                     "frac": round(achieved / 78.6, 4), "traffic": None, "kernel": "complex LU (rocSOLVER getrf)",
                     "note": "8/3 n^3 real flops per block over the wall time of the whole call, assembly included"},
        "cpu_baseline": None,
        "sum_logabs": float(sum(x.sum() for x in la)),
    }
    print(json.dumps(line), flush=True)
    ctx.close()


def one_flavour_bench(args, dd, inputs, np, torch):
    """The one-flavour estimator (Eq. 11) on the 48x24^3 workload, 12 RHS, FP32 inner solves."""
    cfg = inputs.WORKLOADS["48x24^3"]
    lat, blk, nhit, nint = cfg["lat"], cfg["blk"], cfg["n_hit"], cfg["n_interp"]
    k1, k2 = cfg["kappa1"], cfg["kappa2"]
    dev = torch.device("cuda:0")
    ctx = dd.Context(torch.from_numpy(inputs.make_links(lat, cfg["eps"], cfg["seed"])).to(dev), lat, blk, -1,
                     cfg["csw"])
    etad = torch.from_numpy(inputs.make_noise_batch(lat, cfg["seed"], nint, nhit)).to(dev)
    tuned = ctx.autotune(k2, nhit, dd.MIXED32) if not args.no_autotune else None

    def step():
        return ctx.det_ratio_estimate(k1, k2, etad, op=dd.OP_SCHUR, tol=args.tol, prec=dd.MIXED32, n_f=1,
                                      allow=(dd.binding.EUNDEF,))

    for _ in range(args.warmup):
        r = step()
    ctx.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        r = step()
        log(f"one-flavour step {k}: log W {r['log_w_gl']:.10f}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = class_profile(dd, [ctx])
    ctx.profile_enable(False)
    roofline, share = class_roofline(prof)
    line = {
        "metric": "one-flavour det-ratio estimates/s", "value": round(nint * nhit * args.steps / elapsed, 3),
        "unit": "estimates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * elapsed / args.steps, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 inner / f64 outer", "data": "synthetic",
        "config": {"workload": "one-flavour Schur estimate (Eq. 11), 48x24^3, 6^4 blocks, N_hit=12 as one "
                               "multi-RHS batch", "lattice": list(lat), "blocks": list(blk), "n_hit": nhit,
                   "tol": args.tol},
        "roofline": roofline, "schedule": tuned, "cpu_baseline": None, "log_w": r["log_w_gl"],
        "status": r["status"], "kernel_time_share": share,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


def measured_traffic(workload, kclass, op_threads=256):
    """HBM bytes per dispatch (FETCH_SIZE and WRITE_SIZE, calibrated) of the kernel of `kclass`,
    from profiles/traffic_<workload>.json if it was measured on the current sources, else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    name = CLASS_KERNEL.get(kclass)
    name = name.format(nt=op_threads) if name else None
    if not name or not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("sources") != kernel_sources_digest():
        return None
    for k, v in rec["kernels"].items():
        if k.startswith(name):
            return v["read_bytes"] + v["write_bytes"]
    return None


def dslash_rates(ctx, dd, inputs, lat, dev, reps):
    """Standalone full-lattice Dslash D(m) psi through ddwc_dslash_apply: FP64 with one RHS and
    FP32 with 12 RHS.  The kernel's own HIP-event time (layout conversion excluded) and the
    algorithmic bytes of the library's byte model give GB/s."""
    import torch
    out = {}
    for name, nrhs, prec, kc in (("fp64_1rhs", 1, dd.FP64, dd.binding.K_DSLASH64),
                                 ("fp32_12rhs", 12, dd.MIXED32, dd.binding.K_DSLASH32)):
        psi = torch.from_numpy(inputs.make_spinor(lat, 5, nrhs=nrhs)).to(dev)
        ctx.dslash_apply(0.1205, psi, prec=prec)
        torch.cuda.synchronize()
        ctx.profile_enable(True)
        for _ in range(reps):
            ctx.dslash_apply(0.1205, psi, prec=prec)
        torch.cuda.synchronize()
        p = ctx.profile_read(kc)
        ctx.profile_enable(False)
        us = 1e3 * p["ms"] / max(p["launches"], 1)
        gbs = p["bytes"] / (p["ms"] * 1e-3) / 1e9 if p["ms"] > 0 else 0.0
        out[name] = {"launches": p["launches"], "avg_launch_us": round(us, 2),
                     "bytes_per_launch": p["bytes"] / max(p["launches"], 1),
                     "gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
        log(f"standalone Dslash {name}: {us:.1f} us/launch, {gbs:.0f} GB/s")
        del psi
    return out


def cpu_baseline(U, eta0, cfg, golden, one_thread):
    """The C oracle timed on the host: one complete Schur estimate (all five solves to 1e-13, the
    exponent checked against the stored oracle value) on every core, and the oracle's Dslash in
    GB/s under the library's byte model (1536 bytes per site in FP64) on every core and on one
    thread; optionally the complete estimate on one thread too."""
    import numpy as np
    from oracle import cref, dirac
    t = time.time()
    R = cref.CRef(U, cfg["lat"], cfg["blk"], cfg["csw"], -1)
    setup = time.time() - t
    cores = cref.CRef.threads()
    m1, m2 = dirac.mass(cfg["kappa1"]), dirac.mass(cfg["kappa2"])
    V = int(np.prod(cfg["lat"]))

    def dslash_gbs(reps):
        psi = eta0
        R.dslash(m2, psi)
        ts = []
        for _ in range(reps):
            ta = time.perf_counter()
            R.dslash(m2, psi)
            ts.append(time.perf_counter() - ta)
        ts.sort()
        return 1536.0 * V / ts[len(ts) // 2] / 1e9

    g_all = dslash_gbs(5)
    t = time.time()
    x, iters, secs = R.exponent_recorded("schur", "diff", m1, m2, eta0, 1e-13)
    wall = time.time() - t
    xo = golden["x_schur"]["0"]
    out = {"value": round(1.0 / wall, 5), "unit": "estimates/s", "cores": cores, "kind": "oracle",
           "sample": f"one complete Schur estimate x_00 of the same 48x24^3 workload (difference form, its "
                     f"{len(iters)} BiCGStab solves to 1e-13: {iters} iterations) in {wall:.1f}s on {cores} "
                     f"threads, x_00 = {x!r} (stored oracle value {xo!r})",
           "x00_rel": abs(x - xo) / max(abs(xo), 1.0),
           "dslash_gbs": round(g_all, 2), "setup_s": round(setup, 1)}
    cref.CRef.set_threads(1)
    out["dslash_gbs_1thread"] = round(dslash_gbs(2), 2)
    if one_thread:
        t = time.time()
        R.exponent("schur", "diff", m1, m2, eta0, 1e-13)
        out["value_1thread"] = round(1.0 / (time.time() - t), 6)
    cref.CRef.set_threads(cores)
    R.close()
    log(f"cpu baseline: {out}")
    return out


if __name__ == "__main__":
    main()
