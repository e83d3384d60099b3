"""Parity at the workloads' full sizes, in the launch configuration the
benchmark uses: one step against the oracle where the oracle finishes in
seconds, otherwise the oracle's own operator applied to the GPU solution
(true residual recomputed on the host), plus the midpoint invariants."""

import numpy as np
import pytest
import torch

import llg_workloads as W
import paper_2607_15290_amd as P
from oracle import operators, steppers
from oracle.grid import Grid
from oracle.operators import Params as OP
from tests.gpu_util import announce, assert_elem, dev, host

pytestmark = pytest.mark.gpu


def _setup(wid):
    spec = W.make(wid)
    n, nz = spec["n"], spec["nz"]
    g = Grid(n, n, nz, h=spec["h"])
    kw = dict(alpha=spec["alpha"], cexc=1.0, dt=spec["dt"], theta=spec["theta"], shift=spec["shift"],
              h_uniform=spec["h_uniform"])
    ctx = P.Context(n, n, nz, spec["h"], 0)
    return spec, g, kw, ctx


def test_workload2_midpoint_512():
    announce("workload 2: 512^2 midpoint, 10 steps")
    spec, g, kw, ctx = _setup(2)
    op = OP(**kw)
    m_ref, v_ref, l_ref, info = steppers.midpoint_step(g, op, spec["m0"], rtol=1e-10, picard_tol=1e-10)
    m = dev(spec["m0"])
    vh = torch.zeros_like(m)
    lam = torch.zeros((1,) + tuple(m.shape[1:]), dtype=torch.float64, device="cuda:0")
    prm = P.Params(**kw)
    e_prev = None
    for step in range(spec["steps"]):
        st = P.llg_step_midpoint(ctx, prm, m, vh, lam, picard_tol=spec["picard_tol"], rtol=spec["rtol"])
        if step == 0:
            assert abs(st["picard_iters"] - info["picard_iters"]) <= 1
            # both sides converge Picard and GMRES to 1e-10
            assert np.max(np.abs(host(m) - m_ref)) <= 1e-10
            assert_elem(host(vh), v_ref, 1e-8, "v")
            len_ref = steppers.midpoint_diagnostics(g, op, spec["m0"], m_ref, v_ref, l_ref)["max_len_err"]
            assert st["max_len_err"] <= 2 * len_ref + 1e-12
        assert st["converged"] == 1
        # The Picard test stops on the change of the frozen midpoint, (k/2)||dv||
        # <= 1e-10 ||m_hat||; the length defect 2 k m^{n+1/2}.v then carries a
        # k^2 |dv| |v| term of about 1e-9 at this stiffness.
        assert st["max_len_err"] <= 5e-9
        scale = abs(st["energy_before"])
        assert abs(st["dissipation_defect"] - st["inexact_correction"]) <= 1e-13 * scale
        if e_prev is not None:
            assert abs(st["energy_before"] - e_prev) <= 1e-12 * scale
        e_prev = st["energy_after"]
    ctx.close()


def test_workload3_euler_128_fp32ir_vs_fp64():
    announce("workload 3: 128^3 Euler broadband, FP32-IR vs FP64, oracle residual")
    spec, g, kw, ctx = _setup(3)
    op = OP(**kw)
    prm = P.Params(**kw)
    m0 = spec["m0"]
    b = steppers.rhs(g, op, m0)
    x64, s64 = P.gmres_solve(ctx, prm, dev(m0), dev(b), rtol=1e-10)
    x32, s32 = P.gmres_solve(ctx, prm, dev(m0), dev(b), rtol=1e-10, prec="fp32_ir", inner_rtol=1e-5)
    for x, s in ((x64, s64), (x32, s32)):
        assert s["converged"] == 1
        xr = host(x)
        r = b - operators.matvec(g, op, m0, xr)
        assert np.linalg.norm(r) <= 1.05e-10 * np.linalg.norm(b)
    assert_elem(host(x32), host(x64), 1e-8, "x fp32-ir vs fp64")
    # two Euler steps in each precision agree
    ms = []
    for prec in ("fp64", "fp32_ir"):
        m = dev(m0)
        for _ in range(2):
            st = P.llg_step_euler(ctx, prm, m, rtol=1e-10, prec=prec, inner_rtol=1e-5)
            assert st["converged"] == 1 and st["max_len_err"] <= 1e-14
        ms.append(host(m))
    assert np.max(np.abs(ms[0] - ms[1])) <= 1e-9
    ctx.close()


def test_workload4_midpoint_256_first_solve_and_step():
    announce("workload 4: 256^3 midpoint, first Picard solve against the oracle operator")
    spec, g, kw, ctx = _setup(4)
    op = OP(**kw)
    prm = P.Params(**kw)
    m0 = spec["m0"]
    md = dev(m0)
    b = P.llg_rhs(ctx, prm, md)
    bh = host(b)
    # right-hand side against the oracle (one FFT Laplacian)
    assert_elem(bh, steppers.rhs(g, op, m0), 1e-12, "rhs")
    # the benchmark's inner tolerance (1e-3) and a tight one, each accepted on
    # the oracle's own residual
    for prec, inner in (("fp64", 1e-3), ("fp32_ir", 1e-3), ("fp32_ir", 1e-5), ("fp32_ir_left", 1e-3)):
        x, s = P.gmres_solve(ctx, prm, md, b, rtol=1e-10, prec=prec, inner_rtol=inner)
        assert s["converged"] == 1
        r = bh - operators.matvec(g, op, m0, host(x))
        print(f"  {prec} inner {inner}: iters {s['iters']} oracle residual "
              f"{np.linalg.norm(r) / np.linalg.norm(bh):.2e}", flush=True)
        assert np.linalg.norm(r) <= 1.05e-10 * np.linalg.norm(bh), prec
        del x
    vh = torch.zeros_like(md)
    lam = torch.zeros((1,) + tuple(md.shape[1:]), dtype=torch.float64, device="cuda:0")
    st = P.llg_step_midpoint(ctx, prm, md, vh, lam, picard_tol=1e-10, rtol=1e-10, prec="fp32_ir", inner_rtol=1e-3)
    assert st["converged"] == 1 and st["max_len_err"] <= 1e-9
    assert abs(st["dissipation_defect"] - st["inexact_correction"]) <= 1e-13 * abs(st["energy_before"])
    ctx.close()
