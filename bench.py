#!/usr/bin/env python
"""Benchmark of the FFT-HSS GMRES hot path on one MI355X.

Workload: the 3D 256^3 periodic midpoint workload (alpha 0.02, dt = 13.3x the
explicit exchange limit, h = (0, 0, 1), smooth 8-mode field plus 1% broadband;
llg_workloads id 4).  One benchmark step is one midpoint time step: a Picard
loop whose every iterate is one saddle solve to true relative residual 1e-10.

Timed: K steps (default 5, the workload's whole run from its initial state;
W optional untimed steps before them) bracketed by device synchronization,
first with FP32-preconditioned FGMRES(30)-IR (the headline value, solves/s),
then the same steps from the same initial state with plain FP64 FFT-HSS
GMRES(30).  Before it, two untimed passes over the same headline steps: a
warm-up (kernels, first touch of the workspace) and one that brackets every
kernel with HIP events (llg_profile_enable) for the per-kind table; during the
headline timed region the library brackets only the dominant kind, whose
roofline is reported.  Also reported: the paper's protocol (median of 3 solves after one
warm-up on the first Picard system), standalone fft_hss_apply / llg_matvec
bandwidth, a labelled variant of the precision form (left-preconditioned
inner GMRES on the fused float32 M^{-1} A), the preconditioner comparison of
the paper (split FFT-HSS, symmetric part, none) on its largest grids, and the
FP64 CPU oracle timed on a bounded sample.

Prints one JSON line on stdout; progress goes to stderr.
"""

import argparse
import json
import os
import platform
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "GMRES solves/s to 1e-10 at 3D 256^3 (FP32-prec vs FP64); fft_hss_apply GB/s vs peak"


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5,
                    help="timed midpoint steps (5: the whole run of the 256^3 midpoint workload)")
    ap.add_argument("--warmup", type=int, default=0,
                    help="untimed steps before the timed ones (the timed steps then start later in the run); "
                         "kernels and buffers are warmed by an untimed pass in any case")
    ap.add_argument("--n", type=int, default=256, help="grid points per axis (256 = the workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison run")
    ap.add_argument("--inner-rtol", type=float, default=1e-3,
                    help="relative tolerance of each inner cycle of the precision form (1e-3 is the fastest of 1e-6..3e-2 at 256^3)")
    ap.add_argument("--no-comparison", action="store_true", help="skip the preconditioner comparison")
    ap.add_argument("--no-paper-protocol", action="store_true", help="skip the paper-protocol solves")
    ap.add_argument("--no-variant", action="store_true",
                    help="skip the left-preconditioned FP32-IR variant run")
    ap.add_argument("--op-reps", type=int, default=20)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy 5 times (counter calibration) and exit")
    ap.add_argument("--orth", default="dcgs2", choices=["dcgs2", "cgs2"],
                    help="Arnoldi orthogonalization: CGS2 with delayed re-orthogonalization, or 3-pass CGS2")
    return ap.parse_args()


def run_steps(P, ctx, prm, m0_dev, spec, prec, warmup, steps, inner_rtol, profile, orth):
    import torch
    m = m0_dev.clone()
    n = ctx.nx
    vh = torch.zeros((3, ctx.nz, ctx.ny, ctx.nx), dtype=torch.float64, device=ctx.device)
    lam = torch.zeros((1, ctx.nz, ctx.ny, ctx.nx), dtype=torch.float64, device=ctx.device)
    kw = dict(picard_tol=spec["picard_tol"], picard_max=spec["picard_max"], restart=spec["restart"],
              rtol=spec["rtol"], prec=prec, inner_rtol=inner_rtol, max_outer=20, orth=orth)
    for i in range(warmup):
        st = P.llg_step_midpoint(ctx, prm, m, vh, lam, **kw)
        log(f"{prec} warm-up step {i}: picard {st['picard_iters']} lin {st['lin_iters_total']}")
    torch.cuda.synchronize()
    if profile:
        # profile: "all" or a list of kernel kinds to bracket with HIP events
        P.llg_profile_select(ctx, None if profile == "all" else profile)
        P.llg_profile_enable(ctx, True)
    stats = []
    t0 = time.perf_counter()
    for i in range(steps):
        st = P.llg_step_midpoint(ctx, prm, m, vh, lam, **kw)
        stats.append(st)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = None
    if profile:
        P.llg_profile_enable(ctx, False)
        prof = P.llg_profile_read(ctx)
        P.llg_profile_select(ctx, None)
    for i, st in enumerate(stats):
        log(f"{prec} step {i}: picard {st['picard_iters']} lin {st['lin_iters_total']} "
            f"len_err {st['max_len_err']:.2e} defect-correction "
            f"{st['dissipation_defect'] - st['inexact_correction']:.2e}")
    del n
    return t1 - t0, stats, prof, m


def paper_protocol(P, ctx, prm, m0_dev, spec, prec, inner_rtol, orth):
    """Median of 3 solves after one warm-up, first Picard system of step 1
    (frozen midpoint m^0, right-hand side C_hat Delta_N m^0 + (1+alpha^2) h)."""
    import torch
    p2 = P.Params(alpha=prm.alpha, cexc=prm.cexc, dt=prm.dt, theta=0.5, shift=prm.shift, h_uniform=prm.h_uniform)
    b = P.llg_rhs(ctx, p2, m0_dev)
    times, iters = [], []
    for i in range(4):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, st = P.gmres_solve(ctx, p2, m0_dev, b, restart=spec["restart"], rtol=spec["rtol"], prec=prec,
                              inner_rtol=inner_rtol, orth=orth)
        torch.cuda.synchronize()
        if i > 0:
            times.append(time.perf_counter() - t0)
            iters.append(st["iters"])
    return dict(median_s=statistics.median(times), iters=iters, rel_res_true=st["rel_res_true"],
                outer_steps=st["outer_steps"])


def op_bandwidth(P, ctx, prm, m0_dev, reps):
    """Standalone fft_hss_apply and llg_matvec timings (torch events on the
    current stream, which is the stream the library launches on)."""
    import torch
    ng = ctx.ng
    out = {}
    p = torch.randn((4,) + tuple(m0_dev.shape[1:]), dtype=torch.float64, device=ctx.device)
    z = torch.empty_like(p)
    m32 = m0_dev.float()
    p32, z32 = p.float(), torch.empty_like(p, dtype=torch.float32)
    for name, fn, bpn in [
        ("fft_hss_apply_f64", lambda: P.fft_hss_apply(ctx, prm, m0_dev, p, z), 88.0),
        ("llg_matvec_f64", lambda: P.llg_matvec(ctx, prm, m0_dev, p, z), 88.0),
        ("fft_hss_apply_f32", lambda: P.fft_hss_apply_f32(ctx, prm, m32, p32, z32), 44.0),
        ("llg_matvec_f32", lambda: P.llg_matvec_f32(ctx, prm, m32, p32, z32), 44.0),
    ]:
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        gbs = bpn * ng / (ms * 1e-3) / 1e9
        out[name] = dict(ms=round(ms, 4), compulsory_GBs=round(gbs, 1), frac_of_peak=round(gbs / HBM_PEAK_GBS, 4),
                         applies_per_s=round(1e3 / ms, 1))
        log(f"{name}: {ms:.3f} ms, {gbs:.0f} GB/s (compulsory {bpn:.0f} B/node)")
    return out


def measured_traffic(kernel_kind, bytes_per_launch):
    """HBM bytes per launch of ``kernel_kind`` from the committed hardware-counter
    summary (profiles/traffic_3d256_midpoint.md), scaled to this run's
    algorithmic bytes per launch; None when the summary has no entry for the
    kernel or the kernel source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_3d256_midpoint.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        parts = line.split()
        if len(parts) == 5 and parts[0] == "bench-traffic:" and parts[1] == kernel_kind:
            src = os.path.join(ROOT, "paper_2607_15290_amd", "csrc", parts[3])
            if not os.path.exists(src):
                return None
            if hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] != parts[4]:
                return None
            return float(parts[2]) * bytes_per_launch
    return None


def precond_comparison(P, torch, W):
    """Sec. 4.3 on the GPU: one Euler system (k = 1e-2, alpha = 0.2, lambda =
    0.5, smooth manufactured right-hand side, GMRES(50), rtol 1e-8) on the
    largest grids of the paper's comparison, 256^2 and 48^3, solved with the
    split FFT-HSS preconditioner, the symmetric part alone and no
    preconditioner; median of 3 solves after one warm-up.  The paper's CPU
    timings of the same systems are quoted beside the GPU's."""
    out = {}
    alpha, k = 0.2, 1e-2
    paper = {"2d_256": (0.236, 15.45), "3d_48": (0.684, 3.20)}
    for key, dim, n in (("2d_256", 2, 256), ("3d_48", 3, 48)):
        nz = 1 if dim == 2 else n
        m, _ = W.manufactured(n, dim, 0.0, alpha)
        _, F = W.manufactured(n, dim, k, alpha)
        ctx = P.Context(n, n, nz, 2 * np.pi / n, 0)
        md = torch.from_numpy(np.ascontiguousarray(m)).to("cuda:0")
        hf = torch.from_numpy(np.ascontiguousarray(F / (1 + alpha ** 2))).to("cuda:0")
        prm_b = P.Params(alpha=alpha, cexc=1.0, dt=k, theta=1.0, shift=0.5, h_field=hf)
        b = P.llg_rhs(ctx, prm_b, md)
        prm = P.Params(alpha=alpha, cexc=1.0, dt=k, theta=1.0, shift=0.5)
        res = {}
        for pc in ("fft_hss", "symmetric", "none"):
            _, st = P.gmres_solve(ctx, prm, md, b, restart=50, rtol=1e-8, orth="cgs2", precond=pc)
            times = []
            for _ in range(3):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, st = P.gmres_solve(ctx, prm, md, b, restart=50, rtol=1e-8, orth="cgs2", precond=pc)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
            res[pc] = dict(iters=st["iters"], median_ms=round(1e3 * statistics.median(times), 3),
                           rel_res_true=st["rel_res_true"])
        res["speedup_split_vs_none"] = round(res["none"]["median_ms"] / res["fft_hss"]["median_ms"], 2)
        res["paper_cpu_split_s"], res["paper_speedup_split_vs_none"] = paper[key]
        out[key] = res
        ctx.close()
    return out


def cpu_baseline(spec, m0_np, gpu_iters_per_solve):
    """FP64 oracle on the host, bounded sample: one application of the
    preconditioned operator M^{-1} A (one matvec and one FFT-HSS apply, the
    operator work of one GMRES iteration) on the first Picard system of step 1
    at full size, scaled to solves/s with the GPU FP64 run's mean iterations
    per solve.  The Arnoldi vector updates are not included (they are a small
    part of the oracle's time next to its FFTs)."""
    from oracle import operators
    from oracle.grid import Grid
    n = spec["n"]
    g = Grid(n, n, spec["nz"], h=spec["h"])
    op = operators.Params(alpha=spec["alpha"], cexc=1.0, dt=spec["dt"], theta=0.5, shift=spec["shift"],
                          h_uniform=spec["h_uniform"])
    v = np.random.default_rng(1).standard_normal((4,) + m0_np.shape[1:])
    t0 = time.perf_counter()
    operators.hss_apply(g, op, m0_np, operators.matvec(g, op, m0_np, v))
    t_iter = time.perf_counter() - t0
    sps = 1.0 / (t_iter * gpu_iters_per_solve)
    return dict(value=sps, unit="solves/s", cores=1, kind="oracle",
                sample=(f"FP64 NumPy oracle (single-threaded numpy.fft) on {platform.processor() or 'the host CPU'}: "
                        f"one M^-1 A application at {n}^3 took {t_iter:.1f} s; scaled by the GPU FP64 run's "
                        f"{gpu_iters_per_solve:.1f} GMRES iterations per solve"),
                seconds_per_iteration=t_iter)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the library has no multi-GPU path.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import llg_workloads as W
    import paper_2607_15290_amd as P

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_calibration:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")  # 1 GiB
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 8, "copy_bytes_written": b.numel() * 8, "copies": 5}))
        return
    log("generating workload 4 (3D midpoint)")
    spec = W.make(4, n=args.n)
    n = spec["n"]
    m0 = spec["m0"]
    ctx = P.Context(n, n, n, spec["h"], 0)
    m0_dev = torch.from_numpy(m0).to("cuda:0")
    prm = P.Params(alpha=spec["alpha"], cexc=1.0, dt=spec["dt"], theta=0.5, shift=spec["shift"],
                   h_uniform=spec["h_uniform"])

    log("operator bandwidth")
    ops = op_bandwidth(P, ctx, prm, m0_dev, args.op_reps)

    # Untimed pass with every kernel bracketed by HIP events: per-kind totals
    # and the dominant kind.  The timed pass repeats the same steps from the
    # same state (the library is deterministic, so the work is identical) and
    # brackets only the dominant kind, which keeps event overhead out of the
    # headline while its roofline is still measured in the timed region.
    log("FP32-IR midpoint steps, untimed warm-up pass (first touch of the workspace)")
    run_steps(P, ctx, prm, m0_dev, spec, "fp32_ir", args.warmup, args.steps, args.inner_rtol, None, args.orth)
    log("FP32-IR midpoint steps, untimed pass with all kernels profiled")
    _, _, prof_all, _ = run_steps(P, ctx, prm, m0_dev, spec, "fp32_ir", args.warmup, args.steps,
                                  args.inner_rtol, "all", args.orth)
    dom_kind = max(prof_all.items(), key=lambda kv: kv[1]["total_ms"])[0]
    log(f"FP32-IR midpoint steps, timed (events around {dom_kind} only)")
    t32, st32, prof, _ = run_steps(P, ctx, prm, m0_dev, spec, "fp32_ir", args.warmup, args.steps,
                                   args.inner_rtol, [dom_kind], args.orth)
    solves32 = sum(s["picard_iters"] for s in st32)
    lin32 = sum(s["lin_iters_total"] for s in st32)
    res = {}
    if not args.no_fp64:
        log("FP64 midpoint steps (one untimed step first to load its kernels)")
        run_steps(P, ctx, prm, m0_dev, spec, "fp64", 0, 1, args.inner_rtol, False, args.orth)
        t64, st64, _, _ = run_steps(P, ctx, prm, m0_dev, spec, "fp64", args.warmup, args.steps, args.inner_rtol,
                                    False, args.orth)
        solves64 = sum(s["picard_iters"] for s in st64)
        lin64 = sum(s["lin_iters_total"] for s in st64)
        res["fp64"] = dict(solves_per_s=solves64 / t64, steps_per_s=args.steps / t64, ms_per_step=1e3 * t64 / args.steps,
                           solves=solves64,
                           gmres_iters=lin64, iters_per_solve=lin64 / solves64)
    if not args.no_variant:
        log("FP32-IR variant with left-preconditioned inner GMRES (one fused float32 pipeline per iteration)")
        run_steps(P, ctx, prm, m0_dev, spec, "fp32_ir_left", 0, 1, args.inner_rtol, False, args.orth)
        tl, stl, _, _ = run_steps(P, ctx, prm, m0_dev, spec, "fp32_ir_left", args.warmup, args.steps,
                                  args.inner_rtol, False, args.orth)
        solvesl = sum(s["picard_iters"] for s in stl)
        linl = sum(s["lin_iters_total"] for s in stl)
        res["fp32_ir_left"] = dict(solves_per_s=solvesl / tl, steps_per_s=args.steps / tl,
                                   ms_per_step=1e3 * tl / args.steps, solves=solvesl, gmres_iters=linl,
                                   iters_per_solve=linl / solvesl,
                                   max_len_err=max(s["max_len_err"] for s in stl))
    comparison = None
    if not args.no_comparison:
        log("preconditioner comparison (256^2 and 48^3)")
        comparison = precond_comparison(P, torch, W)
    pp32 = pp64 = None
    if not args.no_paper_protocol:
        log("paper protocol (median of 3 after 1 warm-up)")
        pp32 = paper_protocol(P, ctx, prm, m0_dev, spec, "fp32_ir", args.inner_rtol, args.orth)
        pp64 = (paper_protocol(P, ctx, prm, m0_dev, spec, "fp64", args.inner_rtol, args.orth)
                if not args.no_fp64 else None)

    # dominant kernel of the headline timed region
    dom_name, dom = max(prof.items(), key=lambda kv: kv[1]["total_ms"])
    achieved = dom["bytes"] / (dom["total_ms"] * 1e-3) / 1e9
    avg_us = 1e3 * dom["total_ms"] / dom["launches"]
    bpl = dom["bytes"] / dom["launches"]
    traffic = measured_traffic(dom_name, bpl)
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4),
                    traffic=round(traffic) if traffic is not None else None, traffic_unit="HBM bytes per launch",
                    kernel=dom_name, avg_launch_us=round(avg_us, 2), launches=dom["launches"],
                    bytes_per_launch=round(bpl))
    kernels = {k: dict(launches=v["launches"], total_ms=round(v["total_ms"], 3),
                       GBs=round(v["bytes"] / (v["total_ms"] * 1e-3) / 1e9, 1) if v["total_ms"] > 0 else None)
               for k, v in sorted(prof_all.items(), key=lambda kv: -kv[1]["total_ms"])}

    value = solves32 / t32
    line = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * t32 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-preconditioned/f64",
        "data": "synthetic",
        "config": {"workload": f"3d_{n}_midpoint", "grid": [n, n, n], "scheme": "midpoint", "alpha": spec["alpha"],
                   "dt": spec["dt"], "shift": spec["shift"], "h_uniform": list(spec["h_uniform"]),
                   "m0": "8 lowest modes + 1% broadband", "solver": "FGMRES(30)-IR, fp32 FFT-HSS + fp32 matvec",
                   "rtol": spec["rtol"], "picard_tol": spec["picard_tol"], "inner_rtol": args.inner_rtol,
                   "orthogonalization": "CGS2, re-orthogonalization delayed one iteration" if args.orth == "dcgs2"
                   else "CGS2, three passes",
                   "parallelism": "1 GPU"},
        "fp32_ir": dict(solves_per_s=value, steps_per_s=args.steps / t32, picard_per_step=solves32 / args.steps,
                        solves=solves32, gmres_iters=lin32, iters_per_solve=lin32 / solves32,
                        max_len_err=max(s["max_len_err"] for s in st32)),
        "fp64": res.get("fp64"),
        "fp32_ir_left_variant": res.get("fp32_ir_left"),
        "fp32_ir_over_fp64": (value / res["fp64"]["solves_per_s"]) if "fp64" in res else None,
        "paper_protocol": {"fp32_ir": pp32, "fp64": pp64},
        "precond_comparison": comparison,
        "ops": ops,
        "roofline": roofline,
        "kernels": kernels,
    }
    if not args.no_cpu_baseline:
        ips = res["fp64"]["iters_per_solve"] if "fp64" in res else lin32 / solves32
        log("CPU oracle baseline (bounded sample)")
        line["cpu_baseline"] = cpu_baseline(spec, m0, ips)
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
