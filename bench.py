#!/usr/bin/env python
"""Benchmark of the FFT-HSS GMRES hot path on one MI355X.

Default workload (4): the 3D 256^3 periodic midpoint workload (alpha 0.02,
dt = 13.3x the explicit exchange limit, h = (0, 0, 1), smooth 8-mode field
plus 1% broadband).  One benchmark step is one midpoint time step: a Picard
loop whose every iterate is one saddle solve to true relative residual 1e-10.
Timed: K steps (W untimed steps before them) bracketed by device
synchronization, first with FP32-preconditioned FGMRES(30)-IR (the headline
value, solves/s), then the same steps from the same initial state with plain
FP64 FFT-HSS GMRES(30), the left-preconditioned FP32-IR variant, and the
FP32-IR run with the velocity-based Picard test (the length-error trade).
Before the headline timed pass, two untimed passes over the same steps: a
warm-up and one that brackets every kernel with HIP events for the per-kind
table; the timed pass brackets only the dominant kind, whose roofline is
reported.  Also: the paper's protocol (median of 3 solves after one warm-up
on the first Picard system), standalone fft_hss_apply / llg_matvec
bandwidth (compulsory and pass-model bytes), the preconditioner comparison
of the paper on its largest grids, and the FP64 CPU oracle timed on the
host's cores.

--workload 1, 2, 3, 5 measure the other workloads the same way (one JSON
line each, its own metric): 1 = 2D 32^2 projected Euler (FP64), 2 = 2D 512^2
midpoint (FP64, 10 steps), 3 = 3D 128^3 projected Euler (FP32-IR beside
FP64, 20 steps), 5 = 2D 256^2 differentiation (20 midpoint steps forward,
checkpoints every 5, adjoint backward).

Prints one JSON line on stdout; progress goes to stderr.
"""

import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
INFINITY_CACHE_BYTES = 256 << 20
METRIC = "GMRES solves/s to 1e-10 at 3D 256^3 (FP32-prec vs FP64); fft_hss_apply GB/s vs peak"

# Pass-model planes per node of one operator application (one read of every
# plane a pass reads, one write of every plane it writes; a row of three half
# spectra counts as three planes): 3D apply = x-fwd 3+3, three axis passes
# 6 each, x-inv 3 + 1 (multiplier plane of p) + 3 (m) + 4 (z) = 35; matvec
# reads all 4 planes of x in its epilogue = 38; 2D has one axis pass.
PASS_PLANES = {("apply", 3): 35, ("matvec", 3): 38, ("apply", 2): 23, ("matvec", 2): 26}


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", type=int, default=4, choices=[1, 2, 3, 4, 5],
                    help="workload id (4: the 256^3 midpoint headline)")
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: the workload's whole run; 5 for workload 4)")
    ap.add_argument("--warmup", type=int, default=0,
                    help="untimed steps before the timed ones (the timed steps then start later in the run); "
                         "kernels and buffers are warmed by an untimed pass in any case")
    ap.add_argument("--n", type=int, default=None, help="grid points per axis (default: the workload's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-protocol", action="store_true",
                    help="CPU baseline with the paper's protocol (median of 3 after one warm-up) even where one "
                         "solve takes long")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison run")
    ap.add_argument("--inner-rtol", type=float, default=1e-3,
                    help="relative tolerance of each inner cycle of the precision form (1e-3 is the fastest of "
                         "1e-6..3e-2 at 256^3)")
    ap.add_argument("--no-comparison", action="store_true", help="skip the preconditioner comparison")
    ap.add_argument("--no-paper-protocol", action="store_true", help="skip the paper-protocol solves")
    ap.add_argument("--no-variant", action="store_true",
                    help="skip the left-preconditioned FP32-IR variant and the velocity-Picard run")
    ap.add_argument("--op-reps", type=int, default=20)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy 5 times (counter calibration) and exit")
    ap.add_argument("--orth", default="dcgs2", choices=["dcgs2", "cgs2"],
                    help="Arnoldi orthogonalization: CGS2 with delayed re-orthogonalization, or 3-pass CGS2")
    return ap.parse_args()


def host_cores():
    """Cores this process may run on (the GPU machine grants one GPU's share)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_model():
    """CPU model name from /proc/cpuinfo (no subprocess)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def set_oracle_threads(n):
    """The oracle's FFTs use n worker threads (scipy.fft workers); its other
    arithmetic is NumPy element-wise code (single-threaded)."""
    from oracle import fourier
    fourier.WORKERS = n


# ---------------------------------------------------------------------------
# timing helpers
# ---------------------------------------------------------------------------
def profiled_timing(P, ctx, runner, log_label):
    """Three passes of a StepsRunner from the same initial state (each after
    its untimed prepare(): m0 and the W warm-up steps): an untimed warm-up
    pass, an untimed pass with every kernel of the K steps bracketed by HIP
    events (per-kind table), and the timed pass of the K steps with events
    around the dominant kind only.  Returns (seconds of the timed pass, its
    result, per-kind table, dominant-kind record of the timed pass)."""
    import torch
    log(f"{log_label}: untimed warm-up pass")
    runner.prepare()
    runner.run()
    log(f"{log_label}: untimed pass with every kernel profiled")
    runner.prepare()
    torch.cuda.synchronize()
    P.llg_profile_select(ctx, None)
    P.llg_profile_enable(ctx, True)
    runner.run()
    P.llg_profile_enable(ctx, False)
    prof_all = P.llg_profile_read(ctx)
    dom_kind = dominant_kind(prof_all)
    log(f"{log_label}: timed pass (events around {dom_kind} only)")
    runner.prepare()
    P.llg_profile_select(ctx, [dom_kind])
    torch.cuda.synchronize()
    P.llg_profile_enable(ctx, True)
    t0 = time.perf_counter()
    out = runner.run()
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    P.llg_profile_enable(ctx, False)
    prof = P.llg_profile_read(ctx)
    P.llg_profile_select(ctx, None)
    return t, out, prof_all, prof


def dominant_kind(prof):
    """The kernel kind with the largest total time among those that stream
    the grid (the value reductions, a few kilobytes each, are excluded: on
    small grids their launch latency would otherwise rank first)."""
    cands = {k: v for k, v in prof.items() if k != "reduce"} or prof
    return max(cands.items(), key=lambda kv: kv[1]["total_ms"])[0]


_COPY_GBS = None


def copy_ceiling():
    """A reference streaming rate for context: torch's device copy of 1 GiB
    (read + write bytes over the median of 10 timed copies after one
    warm-up), measured once per run.  It is not the fastest copy this GPU
    can run (a hand-written copy with non-temporal hints reaches more)."""
    global _COPY_GBS
    if _COPY_GBS is None:
        import torch
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        b.copy_(a)
        ts = []
        for _ in range(10):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            b.copy_(a)
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e-3)
        ts.sort()
        _COPY_GBS = 2 * a.numel() * 8 / ts[len(ts) // 2] / 1e9
        del a, b
    return _COPY_GBS


def roofline_of(prof, footprint_bytes, grid, traffic_kernel=None):
    dom_name = dominant_kind(prof)
    dom = prof[dom_name]
    achieved = dom["bytes"] / (dom["total_ms"] * 1e-3) / 1e9
    bpl = dom["bytes"] / dom["launches"]
    traffic = (measured_traffic(dom_name, bpl, grid)
               if traffic_kernel is None or traffic_kernel == dom_name else None)
    r = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
             frac=round(achieved / HBM_PEAK_GBS, 4),
             traffic=round(traffic) if traffic is not None else None, traffic_unit="HBM bytes per launch",
             kernel=dom_name, avg_launch_us=round(1e3 * dom["total_ms"] / dom["launches"], 2),
             launches=dom["launches"], bytes_per_launch=round(bpl))
    # context, not the peak: the same kernel against torch's device copy
    cgbs = copy_ceiling()
    r["torch_copy_GBs"] = round(cgbs, 1)
    r["frac_of_torch_copy"] = round(achieved / cgbs, 4)
    if footprint_bytes < INFINITY_CACHE_BYTES:
        r["note"] = (f"working set {footprint_bytes / 2**20:.3g} MiB fits the 256 MiB Infinity Cache: the rate "
                     f"is cache/latency bound, not an HBM figure; quote applies/s and solves/s")
    return r


def kernel_table(prof_all):
    return {k: dict(launches=v["launches"], total_ms=round(v["total_ms"], 3),
                    GBs=round(v["bytes"] / (v["total_ms"] * 1e-3) / 1e9, 1) if v["total_ms"] > 0 else None)
            for k, v in sorted(prof_all.items(), key=lambda kv: -kv[1]["total_ms"])}


def measured_traffic(kernel_kind, bytes_per_launch, grid):
    """HBM bytes per launch of ``kernel_kind`` from the committed hardware-counter
    summary (profiles/traffic_3d256_midpoint.md), scaled to this run's
    algorithmic bytes per launch; None when the summary has no entry for the
    kernel on this grid (a ratio measured on one grid says nothing about
    another, least of all one whose working set stays in the Infinity Cache)
    or the kernel source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_3d256_midpoint.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        parts = line.split()
        if (len(parts) == 6 and parts[0] == "bench-traffic:" and parts[1] == kernel_kind
                and parts[5] == "x".join(str(int(v)) for v in grid)):
            src = os.path.join(ROOT, "paper_2607_15290_amd", "csrc", parts[3])
            if not os.path.exists(src):
                return None
            if hashlib.sha256(open(src, "rb").read()).hexdigest()[:16] != parts[4]:
                return None
            return float(parts[2]) * bytes_per_launch
    return None


def op_bandwidth(P, ctx, prm, m0_dev, reps):
    """Standalone fft_hss_apply and llg_matvec timings (torch events on the
    current stream, which is the stream the library launches on): applies/s,
    and GB/s on compulsory bytes (one read of p / x and m, one write of the
    output: 11 scalars per node) and on the pass model (PASS_PLANES)."""
    import torch
    ng = ctx.ng
    dim = 2 if ctx.nz == 1 else 3
    out = {}
    p = torch.randn((4,) + tuple(m0_dev.shape[1:]), dtype=torch.float64, device=ctx.device)
    z = torch.empty_like(p)
    m32 = m0_dev.float()
    p32, z32 = p.float(), torch.empty_like(p, dtype=torch.float32)
    for name, fn, op, eb in [
        ("fft_hss_apply_f64", lambda: P.fft_hss_apply(ctx, prm, m0_dev, p, z), "apply", 8),
        ("llg_matvec_f64", lambda: P.llg_matvec(ctx, prm, m0_dev, p, z), "matvec", 8),
        ("fft_hss_apply_f32", lambda: P.fft_hss_apply_f32(ctx, prm, m32, p32, z32), "apply", 4),
        ("llg_matvec_f32", lambda: P.llg_matvec_f32(ctx, prm, m32, p32, z32), "matvec", 4),
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
        comp = 11.0 * eb * ng / (ms * 1e-3) / 1e9
        pm = PASS_PLANES[(op, dim)] * eb * ng / (ms * 1e-3) / 1e9
        out[name] = dict(ms=round(ms, 4), applies_per_s=round(1e3 / ms, 1),
                         compulsory_GBs=round(comp, 1), compulsory_frac=round(comp / HBM_PEAK_GBS, 4),
                         pass_model_bytes_per_node=PASS_PLANES[(op, dim)] * eb,
                         pass_model_GBs=round(pm, 1), pass_model_frac=round(pm / HBM_PEAK_GBS, 4),
                         meets_60pct_target=bool(pm / HBM_PEAK_GBS >= 0.6))
        log(f"{name}: {ms:.3f} ms, pass model {pm:.0f} GB/s ({pm / HBM_PEAK_GBS:.2f} of peak), "
            f"compulsory {comp:.0f} GB/s")
    return out


class StepsRunner:
    """The workload's scheme from m0.  prepare() restarts from m0 and runs the
    W untimed warm-up steps; run() then runs the K steps that are timed and
    returns their statistics."""

    def __init__(self, P, ctx, prm, m0_dev, spec, prec, warmup, steps, inner_rtol, orth, picard_norm="midpoint"):
        self.P, self.ctx, self.prm, self.m0, self.spec = P, ctx, prm, m0_dev, spec
        self.prec, self.warmup, self.steps = prec, warmup, steps
        self.inner_rtol, self.orth, self.picard_norm = inner_rtol, orth, picard_norm

    def _step(self):
        P, spec = self.P, self.spec
        if spec["scheme"] == "midpoint":
            return P.llg_step_midpoint(self.ctx, self.prm, self.m, self.vh, self.lam, picard_tol=spec["picard_tol"],
                                       picard_max=spec["picard_max"], restart=spec["restart"], rtol=spec["rtol"],
                                       prec=self.prec, inner_rtol=self.inner_rtol, max_outer=20, orth=self.orth,
                                       picard_norm=self.picard_norm)
        if spec["wid"] == 1:
            self.m.copy_(self.m0)  # the workload is one step: every timed step repeats it
        return P.llg_step_euler(self.ctx, self.prm, self.m, restart=spec["restart"], rtol=spec["rtol"],
                                prec=self.prec, inner_rtol=self.inner_rtol, max_outer=20, orth=self.orth)

    def prepare(self):
        import torch
        self.m = self.m0.clone()
        self.vh = torch.zeros_like(self.m)
        self.lam = torch.zeros((1,) + tuple(self.m.shape[1:]), dtype=torch.float64, device=self.ctx.device)
        for _ in range(self.warmup):
            self._step()

    def run(self):
        return [self._step() for _ in range(self.steps)]


class CallRunner:
    """A whole timed unit with no warm-up part (the differentiation
    workload's trajectory), in the StepsRunner interface."""

    def __init__(self, fn):
        self.fn = fn

    def prepare(self):
        pass

    def run(self):
        return self.fn()


def timed_steps(runner):
    """prepare() untimed, then (seconds, statistics) of run() bracketed by
    device synchronizations."""
    import torch
    runner.prepare()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = runner.run()
    torch.cuda.synchronize()
    return time.perf_counter() - t0, out


def summarize(stats, t, steps):
    solves = sum(s["picard_iters"] for s in stats)
    lin = sum(s["lin_iters_total"] for s in stats)
    return dict(solves_per_s=solves / t, steps_per_s=steps / t, ms_per_step=1e3 * t / steps,
                solves=solves, picard_per_step=solves / steps, gmres_iters=lin, iters_per_solve=lin / solves,
                max_len_err=max(s["max_len_err"] for s in stats))


def log_steps(label, stats):
    for i, st in enumerate(stats):
        log(f"{label} step {i}: picard {st['picard_iters']} lin {st['lin_iters_total']} "
            f"len_err {st['max_len_err']:.2e} defect-correction "
            f"{st['dissipation_defect'] - st['inexact_correction']:.2e}")


def paper_protocol(P, ctx, prm, m0_dev, spec, prec, inner_rtol, orth):
    """Median of 3 solves after one warm-up, first system of step 1 (Picard:
    frozen midpoint m^0; right-hand side C_hat Delta_N m^0 + (1+alpha^2) h)."""
    import torch
    b = P.llg_rhs(ctx, prm, m0_dev)
    times, iters = [], []
    for i in range(4):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, st = P.gmres_solve(ctx, prm, m0_dev, b, restart=spec["restart"], rtol=spec["rtol"], prec=prec,
                              inner_rtol=inner_rtol, orth=orth)
        torch.cuda.synchronize()
        if i > 0:
            times.append(time.perf_counter() - t0)
            iters.append(st["iters"])
    return dict(median_s=statistics.median(times), iters=iters, rel_res_true=st["rel_res_true"],
                outer_steps=st["outer_steps"])


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


# ---------------------------------------------------------------------------
# CPU oracle baselines (the oracle as it is, on the host's cores)
# ---------------------------------------------------------------------------
def timed_protocol(fn, protocol, long_s=8.0):
    """The paper's protocol, median of 3 after one warm-up.  When the first
    call alone takes longer than long_s seconds (and the full protocol was
    not asked for), that one cold call is the measurement, which keeps the
    sample to tens of seconds.  Returns (seconds, timed calls, warm-up used,
    result)."""
    t0 = time.perf_counter()
    out = fn()
    tw = time.perf_counter() - t0
    if not protocol and tw > long_s:
        return tw, 1, False, out
    times = []
    for _ in range(3):
        t0 = time.perf_counter()
        out = fn()
        times.append(time.perf_counter() - t0)
    return statistics.median(times), 3, True, out


def cpu_solve_baseline(spec, n_sample, protocol, scale_to_nodes=None):
    """Oracle FP64 left-preconditioned GMRES(30) on the first system of the
    workload's first step (midpoint: the first Picard system), at n_sample
    points per axis; solves/s measured there, projected to the workload's
    grid by the node ratio when the sample is smaller."""
    import llg_workloads as W
    from oracle import steppers
    from oracle.grid import Grid
    from oracle.operators import Params as OP
    cores = host_cores()
    set_oracle_threads(cores)
    sp = W.make(spec["wid"], n=n_sample)
    if n_sample != spec["n"]:
        # the same stiffness relative to the sample grid (13.3 x its explicit limit, or 10 h^2)
        if spec["dt_rule"] == "10h2":
            sp["dt"] = 10.0 / n_sample ** 2
        else:
            sp["dt"] = W.dt_explicit_multiple(W.EXPLICIT_RATIO, sp["alpha"], n_sample, sp["dim"])
    g = Grid(sp["nx"], sp["ny"], sp["nz"], h=sp["h"])
    op = OP(alpha=sp["alpha"], cexc=1.0, dt=sp["dt"], theta=sp["theta"], shift=sp["shift"],
            h_uniform=sp["h_uniform"], h_field=sp["h_field"])
    m0 = sp["m0"]
    b = steppers.rhs(g, op, m0)
    med, reps, warm, (x, info) = timed_protocol(lambda: steppers.solve_saddle(g, op, m0, b, rtol=sp["rtol"],
                                                                              restart=sp["restart"]), protocol)
    rate = 1.0 / med
    nodes = g.ng
    target_nodes = scale_to_nodes or nodes
    value = rate * nodes / target_nodes
    what = "median of 3 after one warm-up" if warm else "one cold solve, the protocol's repeats skipped to bound the sample"
    sample = (f"FP64 NumPy/SciPy oracle on {cores} host cores ({cpu_model()}; scipy.fft workers={cores}, NumPy "
              f"element-wise single-threaded): left-preconditioned GMRES(30) to 1e-10 on the first "
              f"{'Picard ' if sp['scheme'] == 'midpoint' else ''}system of the workload's recipe at "
              f"{sp['n']}^{sp['dim']} ({info['iters']} iterations, {med:.2f} s, {what})")
    if target_nodes != nodes:
        sample += (f"; projected to the {spec['n']}^{spec['dim']} workload by the node ratio "
                   f"{target_nodes / nodes:.0f} (iteration counts are mesh-independent at bounded stiffness; "
                   f"the FFT's log factor is ignored, which favors the CPU)")
    return dict(value=value, unit="solves/s", cores=cores, kind="oracle", sample=sample,
                sample_grid=[sp["nx"], sp["ny"], sp["nz"]], sample_solves_per_s=rate, sample_iters=info["iters"],
                sample_seconds=med, timed_solves=reps, cpu_model=cpu_model())


def cpu_adjoint_baseline(spec, protocol):
    """Oracle cost of one differentiation trajectory of workload 5: one
    midpoint step and one adjoint step at 256^2, timed (median of 3 after a
    warm-up), scaled to the trajectory: 20 forward steps, 20 recomputed steps
    and 20 adjoint steps."""
    from oracle import adjoint, steppers
    from oracle.grid import Grid
    from oracle.operators import Params as OP
    cores = host_cores()
    set_oracle_threads(cores)
    g = Grid(spec["nx"], spec["ny"], spec["nz"], h=spec["h"])
    op = OP(alpha=spec["alpha"], cexc=1.0, dt=spec["dt"], theta=0.5, shift=spec["shift"],
            h_uniform=spec["h_uniform"], h_field=spec["h_field"])
    m0 = spec["m0"]
    t_fwd, r1, _, (m1, v, r, info) = timed_protocol(
        lambda: steppers.midpoint_step(g, op, m0, rtol=spec["rtol"], picard_tol=spec["picard_tol"]), protocol)
    gbar = np.zeros_like(m1)
    gbar[2] = 2 * m1[2]
    t_adj, r2, _, _ = timed_protocol(lambda: adjoint.step_adjoint(g, op, m0, v, r, gbar, rtol=1e-12), protocol)
    steps = spec["steps"]
    t_traj = 2 * steps * t_fwd + steps * t_adj
    return dict(value=1.0 / t_traj, unit="trajectories/s (forward + backward)", cores=cores, kind="oracle",
                sample=(f"FP64 NumPy/SciPy oracle on {cores} host cores ({cpu_model()}): one midpoint step "
                        f"({info['picard_iters']} Picard solves, {t_fwd:.2f} s) and one adjoint step "
                        f"({t_adj:.2f} s) at {spec['n']}^2, median of {r1} (after a warm-up when 3), scaled to "
                        f"{steps} forward + {steps} recomputed + {steps} adjoint steps"),
                cpu_model=cpu_model())


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------
def base_line(args, metric, value, unit, ms_per_step, steps, dtype, config):
    return {"metric": metric, "value": round(value, 4), "unit": unit, "n_gpus": 1, "steps": steps,
            "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}


def load_workload(W, wid, n):
    spec = W.make(wid, n=n)
    spec["wid"] = wid
    spec["dt_rule"] = W.WORKLOADS[wid]["dt"]
    return spec


def params_of(P, spec, torch):
    hf = torch.from_numpy(spec["h_field"]).to("cuda:0") if spec.get("h_field") is not None else None
    return P.Params(alpha=spec["alpha"], cexc=1.0, dt=spec["dt"], theta=spec["theta"], shift=spec["shift"],
                    h_uniform=spec["h_uniform"], h_field=hf)


def footprint(spec, prec):
    """Bytes a typical Arnoldi pass touches: four float64 saddle vectors (the
    output, the magnetization and two basis directions); below the 256 MiB
    Infinity Cache the measured rates are cache/latency figures."""
    ng = spec["nx"] * spec["ny"] * spec["nz"]
    return ng * 4 * 8 * 4


def grid_of(spec):
    return (spec["nx"], spec["ny"], spec["nz"])


def run_headline(args, P, W, torch):
    steps = args.steps or 5
    log("generating workload 4 (3D midpoint)")
    spec = load_workload(W, 4, args.n)
    n = spec["n"]
    ctx = P.Context(n, n, n, spec["h"], 0)
    m0_dev = torch.from_numpy(spec["m0"]).to("cuda:0")
    prm = params_of(P, spec, torch)

    log("operator bandwidth")
    ops = op_bandwidth(P, ctx, prm, m0_dev, args.op_reps)

    run32 = StepsRunner(P, ctx, prm, m0_dev, spec, "fp32_ir", args.warmup, steps, args.inner_rtol, args.orth)
    t32, st32, prof_all, prof = profiled_timing(P, ctx, run32, "FP32-IR midpoint steps")
    log_steps("fp32_ir", st32)
    fp32 = summarize(st32, t32, steps)
    res = {}
    if not args.no_fp64:
        log("FP64 midpoint steps (one untimed step first to load its kernels)")
        timed_steps(StepsRunner(P, ctx, prm, m0_dev, spec, "fp64", 0, 1, args.inner_rtol, args.orth))
        t64, st64 = timed_steps(StepsRunner(P, ctx, prm, m0_dev, spec, "fp64", args.warmup, steps, args.inner_rtol,
                                            args.orth))
        res["fp64"] = summarize(st64, t64, steps)
    if not args.no_variant:
        log("FP32-IR variant with left-preconditioned inner GMRES (one fused float32 pipeline per iteration)")
        timed_steps(StepsRunner(P, ctx, prm, m0_dev, spec, "fp32_ir_left", 0, 1, args.inner_rtol, args.orth))
        tl, stl = timed_steps(StepsRunner(P, ctx, prm, m0_dev, spec, "fp32_ir_left", args.warmup, steps,
                                          args.inner_rtol, args.orth))
        res["fp32_ir_left"] = summarize(stl, tl, steps)
        log("FP32-IR with the velocity-based Picard test (length-error trade)")
        tv, stv = timed_steps(StepsRunner(P, ctx, prm, m0_dev, spec, "fp32_ir", args.warmup, steps, args.inner_rtol,
                                          args.orth, picard_norm="velocity"))
        res["fp32_ir_velocity_picard"] = summarize(stv, tv, steps)
        log_steps("fp32_ir velocity-Picard", stv)
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

    value = fp32["solves_per_s"]
    line = base_line(args, METRIC, value, "solves/s", fp32["ms_per_step"], steps, "f32-preconditioned/f64", {
        "workload": f"3d_{n}_midpoint", "grid": [n, n, n], "scheme": "midpoint", "alpha": spec["alpha"],
        "dt": spec["dt"], "shift": spec["shift"], "h_uniform": list(spec["h_uniform"]),
        "m0": "8 lowest modes + 1% broadband", "solver": "FGMRES(30)-IR, fp32 FFT-HSS + fp32 matvec",
        "rtol": spec["rtol"], "picard_tol": spec["picard_tol"], "inner_rtol": args.inner_rtol,
        "orthogonalization": "CGS2, re-orthogonalization delayed one iteration" if args.orth == "dcgs2"
        else "CGS2, three passes", "parallelism": "1 GPU"})
    line.update({
        "fp32_ir": fp32,
        "fp64": res.get("fp64"),
        "fp32_ir_left_variant": res.get("fp32_ir_left"),
        "picard_length_trade": ({
            "midpoint_change_test": dict(steps_per_s=fp32["steps_per_s"], max_len_err=fp32["max_len_err"],
                                         picard_per_step=fp32["picard_per_step"]),
            "velocity_change_test": dict(steps_per_s=res["fp32_ir_velocity_picard"]["steps_per_s"],
                                         max_len_err=res["fp32_ir_velocity_picard"]["max_len_err"],
                                         picard_per_step=res["fp32_ir_velocity_picard"]["picard_per_step"])}
            if "fp32_ir_velocity_picard" in res else None),
        "fp32_ir_over_fp64": (value / res["fp64"]["solves_per_s"]) if "fp64" in res else None,
        "paper_protocol": {"fp32_ir": pp32, "fp64": pp64},
        "precond_comparison": comparison,
        "ops": ops,
        "roofline": roofline_of(prof, footprint(spec, "fp32_ir"), grid_of(spec)),
        "kernels": kernel_table(prof_all),
    })
    if not args.no_cpu_baseline:
        log("CPU oracle baseline (first Picard system of the workload recipe at 128^3)")
        line["cpu_baseline"] = cpu_solve_baseline(spec, min(128, n), args.cpu_protocol,
                                                  scale_to_nodes=spec["nx"] * spec["ny"] * spec["nz"])
    ctx.close()
    return line


def run_solver_workload(args, P, W, torch, wid):
    """Workloads 1-3: time K steps of the workload (each precision it names),
    the standalone operators, the dominant kernel's roofline and the oracle
    baseline on the full-size first system."""
    spec = load_workload(W, wid, args.n)
    steps = args.steps or (spec["steps"] if wid != 1 else 5)
    n, nz = spec["n"], spec["nz"]
    log(f"workload {wid}: {spec['name']} at {n}^{spec['dim']}")
    ctx = P.Context(n, n, nz, spec["h"], 0)
    m0_dev = torch.from_numpy(spec["m0"]).to("cuda:0")
    prm = params_of(P, spec, torch)
    ops = op_bandwidth(P, ctx, prm, m0_dev, args.op_reps)
    precs = list(spec["prec"])
    head = precs[0]
    runh = StepsRunner(P, ctx, prm, m0_dev, spec, head, args.warmup, steps, args.inner_rtol, args.orth)
    th, sth, prof_all, prof = profiled_timing(P, ctx, runh, f"{head} steps")
    log_steps(head, sth)
    summ = {head: summarize(sth, th, steps)}
    for prec in precs[1:]:
        log(f"{prec} steps")
        runp = StepsRunner(P, ctx, prm, m0_dev, spec, prec, args.warmup, steps, args.inner_rtol, args.orth)
        timed_steps(runp)
        tp, stp = timed_steps(runp)
        summ[prec] = summarize(stp, tp, steps)
    pp = {}
    if not args.no_paper_protocol:
        log("paper protocol (median of 3 after 1 warm-up)")
        for prec in precs:
            pp[prec] = paper_protocol(P, ctx, prm, m0_dev, spec, prec, args.inner_rtol, args.orth)
    value = summ[head]["solves_per_s"]
    metric = (f"GMRES solves/s to 1e-10, {spec['dim']}D {n}^{spec['dim']} "
              f"{'projected Euler' if spec['scheme'] == 'euler' else 'midpoint'} "
              f"({'FP32-prec FGMRES-IR vs FP64' if 'fp32_ir' in precs else 'FP64'})")
    line = base_line(args, metric, value, "solves/s", summ[head]["ms_per_step"], steps,
                     "f32-preconditioned/f64" if head == "fp32_ir" else "f64", {
                         "workload": spec["name"], "grid": [n, n, nz], "scheme": spec["scheme"],
                         "alpha": spec["alpha"], "dt": spec["dt"], "shift": spec["shift"],
                         "h_uniform": list(spec["h_uniform"]), "m0": spec["m0_kind"] if "m0_kind" in spec else
                         W.WORKLOADS[wid]["m0"], "rtol": spec["rtol"], "inner_rtol": args.inner_rtol,
                         "steps_per_run": spec["steps"], "parallelism": "1 GPU"})
    line.update({p: s for p, s in summ.items()})
    if "fp64" in summ and head != "fp64":
        line["fp32_ir_over_fp64"] = summ[head]["solves_per_s"] / summ["fp64"]["solves_per_s"]
    line.update({"paper_protocol": pp, "ops": ops,
                 "roofline": roofline_of(prof, footprint(spec, head), grid_of(spec)),
                 "kernels": kernel_table(prof_all)})
    if not args.no_cpu_baseline:
        log("CPU oracle baseline (first system at full size)")
        line["cpu_baseline"] = cpu_solve_baseline(spec, n, args.cpu_protocol)
    ctx.close()
    return line


def adjoint_step_comparison(P, ctx, spec, prm, m0, hf0, torch):
    """The adjoint of the workload's first step, solved with GMRES
    right-preconditioned by M^{-T} in one pipeline per iteration (orth dcgs2,
    the default) and left-preconditioned on M^{-T} J^T in two (orth cgs2):
    iterations and median time of 3 after one warm-up each."""
    m = m0.clone()
    vh = torch.zeros_like(m)
    lam = torch.zeros((1,) + tuple(m.shape[1:]), dtype=torch.float64, device=ctx.device)
    prm_f = P.Params(alpha=prm.alpha, cexc=1.0, dt=prm.dt, theta=0.5, shift=prm.shift,
                     h_uniform=spec["h_uniform"], h_field=hf0)
    P.llg_step_midpoint(ctx, prm_f, m, vh, lam, picard_tol=spec["picard_tol"], rtol=spec["rtol"])
    gbar0 = torch.zeros_like(m)
    gbar0[2] = 2 * m[2]
    out = {}
    for label, orth in (("right_one_pipeline", "dcgs2"), ("left_two_pipelines", "cgs2")):
        times = []
        for i in range(4):
            gb = gbar0.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st = P.llg_step_midpoint_adjoint(ctx, prm_f, m0, vh, lam, gb, None, None, rtol=1e-10, orth=orth)
            torch.cuda.synchronize()
            if i:
                times.append(time.perf_counter() - t0)
        out[label] = dict(iters=st["iters"], median_ms=round(1e3 * statistics.median(times), 3),
                          rel_res_true=st["rel_res_true"])
    out["speedup_right_vs_left"] = round(out["left_two_pipelines"]["median_ms"] /
                                         out["right_one_pipeline"]["median_ms"], 3)
    return out


def run_adjoint_workload(args, P, W, torch):
    """Workload 5: forward (20 midpoint steps, checkpoints every 5) and
    backward (recompute each segment, one transposed saddle solve per step)
    of the differentiable trajectory; value = trajectories/s (forward +
    backward)."""
    spec = load_workload(W, 5, args.n)
    n = spec["n"]
    nsteps = args.steps or spec["steps"]
    log(f"workload 5: {n}^2 differentiation, {nsteps} steps")
    ctx = P.Context(n, n, 1, spec["h"], 0)
    m0 = torch.from_numpy(spec["m0"]).to("cuda:0")
    hf0 = torch.from_numpy(spec["h_field"]).to("cuda:0")
    hu0 = torch.tensor(spec["h_uniform"], dtype=torch.float64)
    prm = P.Params(alpha=spec["alpha"], cexc=1.0, dt=spec["dt"], theta=0.5, shift=spec["shift"])
    ops = op_bandwidth(P, ctx, P.Params(alpha=spec["alpha"], dt=spec["dt"], theta=0.5, shift=spec["shift"]), m0,
                       args.op_reps)
    times = {}

    def run():
        m = m0.clone().requires_grad_(True)
        hu = hu0.clone().requires_grad_(True)
        hf = hf0.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mN = P.midpoint_trajectory(ctx, prm, m, hu, hf, nsteps=nsteps, ckpt_every=spec["ckpt_every"],
                                   picard_tol=spec["picard_tol"], rtol=spec["rtol"], adjoint_rtol=1e-10)
        loss = (mN[2] ** 2).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        times["fwd"], times["bwd"] = t1 - t0, t2 - t1
        return float(loss.item()), float(m.grad.norm().item()), float(hf.grad.norm().item()), list(hu.grad.tolist())

    t, out, prof_all, prof = profiled_timing(P, ctx, CallRunner(run), "trajectory forward + backward")
    loss, gm, ghf, ghu = out
    log("one adjoint step: right-preconditioned one-pipeline solve vs the left two-pipeline form")
    adj = adjoint_step_comparison(P, ctx, spec, prm, m0, hf0, torch)
    line = base_line(args, f"differentiable trajectories/s (forward + backward), 2D {n}^2 midpoint, {nsteps} "
                           f"steps, checkpoints every {spec['ckpt_every']}", 1.0 / t,
                     "trajectories/s", 1e3 * t / nsteps, nsteps, "f64", {
                         "workload": spec["name"], "grid": [n, n, 1], "scheme": "midpoint", "alpha": spec["alpha"],
                         "dt": spec["dt"], "shift": spec["shift"], "h_uniform": list(spec["h_uniform"]),
                         "h_field": "N(0, 0.1^2)", "loss": "sum m_z^2 at the last step", "rtol": spec["rtol"],
                         "adjoint_rtol": 1e-10, "ckpt_every": spec["ckpt_every"], "parallelism": "1 GPU"})
    line.update({"forward_s": times["fwd"], "backward_s": times["bwd"], "loss": loss, "adjoint_step": adj,
                 "grad_norms": {"m0": gm, "h_field": ghf, "h_uniform": ghu}, "ops": ops,
                 "roofline": roofline_of(prof, footprint(spec, "fp64"), grid_of(spec)),
                 "kernels": kernel_table(prof_all)})
    if not args.no_cpu_baseline:
        log("CPU oracle baseline (one forward and one adjoint step at full size)")
        line["cpu_baseline"] = cpu_adjoint_baseline(spec, args.cpu_protocol)
    ctx.close()
    return line


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
    if args.workload == 4:
        line = run_headline(args, P, W, torch)
    elif args.workload == 5:
        line = run_adjoint_workload(args, P, W, torch)
    else:
        line = run_solver_workload(args, P, W, torch, args.workload)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
