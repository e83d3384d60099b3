"""GPU parity of gmres_solve and the steppers against the FP64 oracle."""

import numpy as np
import pytest
import torch

import llg_workloads as W
import paper_2607_15290_amd as P
from oracle import dense, operators, steppers
from oracle.grid import Grid
from tests.gpu_util import announce, assert_elem, both_params, dev, host, unit_field

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape,theta", [((8, 8, 1), 1.0), ((4, 8, 1), 0.5), ((4, 4, 4), 1.0)])
def test_gmres_matches_dense_solve(shape, theta):
    nx, ny, nz = shape
    announce(f"gmres dense {shape}")
    h = 1.0 / nx
    g = Grid(nx, ny, nz, h=h)
    prm, op = both_params(alpha=0.1, dt=5e-3, theta=theta, shift=0.5)
    m = unit_field((nz, ny, nx), 1)
    b = np.random.default_rng(2).standard_normal((4, nz, ny, nx))
    xs = dense.solve(g, op, m, b)
    ctx = P.Context(nx, ny, nz, h, 0)
    x, st = P.gmres_solve(ctx, prm, dev(m), dev(b), rtol=1e-14)
    assert st["converged"] == 1 and st["rel_res_true"] <= 1e-14
    assert_elem(host(x), xs, 1e-12, "x")
    assert st["restarts"] == st["cycles"] - 1 and st["ms"] > 0
    # the transposed system A^T x = b, preconditioned by M^T
    xt, stt = P.gmres_solve(ctx, prm, dev(m), dev(b), rtol=1e-14, transpose=True)
    assert stt["converged"] == 1 and stt["rel_res_true"] <= 1e-14
    assert_elem(host(xt), np.linalg.solve(dense.saddle_matrix(g, op, m).T, b.ravel()).reshape(b.shape), 1e-12,
                "x (transposed)")
    ctx.close()


@pytest.mark.parametrize("shape", [(32, 32, 1), (64, 16, 1), (16, 16, 16)])
def test_gmres_matches_oracle_gmres(shape):
    nx, ny, nz = shape
    announce(f"gmres oracle {shape}")
    h = 1.0 / nx
    g = Grid(nx, ny, nz, h=h)
    prm, op = both_params(alpha=0.1, dt=10 * h * h, theta=1.0, shift=0.5, h_uniform=(0.0, 0.0, 0.5))
    m = unit_field((nz, ny, nx), 4, smooth=20.0)
    b = steppers.rhs(g, op, m)
    xr, ir = steppers.solve_saddle(g, op, m, b, rtol=1e-10)
    ctx = P.Context(nx, ny, nz, h, 0)
    x, st = P.gmres_solve(ctx, prm, dev(m), dev(b), rtol=1e-10)
    assert st["converged"] == 1
    assert abs(st["iters"] - ir["iters"]) <= 1
    # both solutions within the tolerance-scaled distance of each other
    assert_elem(host(x), xr, 1e-8, "x")
    # transposed system against the oracle's transposed GMRES (left, M^T)
    xtr, itr = steppers.solve_saddle(g, op, m, b, rtol=1e-10, transpose=True)
    xt, stt = P.gmres_solve(ctx, prm, dev(m), dev(b), rtol=1e-10, transpose=True)
    assert stt["converged"] == 1 and abs(stt["iters"] - itr["iters"]) <= 1
    assert_elem(host(xt), xtr, 1e-8, "x (transposed)")
    ctx.close()


def _workload_system(nx, ny, nz, seed):
    """First Picard system of a midpoint step of the 3D workloads' kind
    (alpha 0.02, dt 13.3 times the explicit limit, h = (0, 0, 1), smooth field
    with a 1% rough part) on an nx x ny x nz grid."""
    h = 1.0 / nx
    g = Grid(nx, ny, nz, h=h)
    dt = W.dt_explicit_multiple(13.3, 0.02, max(nx, ny, nz), 3)
    prm, op = both_params(alpha=0.02, cexc=1.0, dt=dt, theta=0.5, shift=0.5, h_uniform=(0.0, 0.0, 1.0))
    m = unit_field((nz, ny, nx), seed, smooth=30.0)
    m = m + 0.01 * unit_field((nz, ny, nx), seed + 1)
    m = m / np.sqrt((m * m).sum(0))
    return g, prm, op, m, steppers.rhs(g, op, m)


@pytest.mark.parametrize("shape", [(256, 256, 8), (256, 8, 256)])
def test_gmres_all_precisions_match_oracle_on_256_lines(shape):
    """GMRES(30) to 1e-10 on grids whose lines are 256 points long (the
    kernels of the 256^3 workload: x passes of half-length 128, 256-point
    axis passes, the fused Arnoldi products of the matvec / M^{-1} A passes)
    against the oracle's solvers: float64 left-preconditioned GMRES, the
    flexible precision form (FP32 inner operator) and its left variant, each
    with the same restart, tolerances and inner stopping rule.  Iteration
    counts within one of the oracle's, solutions element-wise to the
    tolerance-scaled distance 1e-8."""
    from oracle import gmres as og
    nx, ny, nz = shape
    announce(f"gmres vs oracle on 256-point lines {shape}")
    g, prm, op, m, b = _workload_system(nx, ny, nz, 31)
    A = lambda v: operators.matvec(g, op, m, v)
    M = lambda v: operators.hss_apply(g, op, m, v)
    ctx = P.Context(nx, ny, nz, 1.0 / nx, 0)
    md, bd = dev(m), dev(b)
    xr, ir = steppers.solve_saddle(g, op, m, b, rtol=1e-10)
    x, st = P.gmres_solve(ctx, prm, md, bd, rtol=1e-10)
    print(f"  fp64 iters gpu {st['iters']} oracle {ir['iters']}", flush=True)
    assert st["converged"] == 1 and abs(st["iters"] - ir["iters"]) <= 1
    assert_elem(host(x), xr, 1e-8, "fp64 x")
    for prec, inner in (("fp32_ir", "flexible"), ("fp32_ir_left", "left")):
        xo, io = og.fgmres_ir(A, M, b, restart=30, rtol=1e-10, inner_rtol=1e-3, max_outer=20, inner=inner)
        x, st = P.gmres_solve(ctx, prm, md, bd, rtol=1e-10, prec=prec, inner_rtol=1e-3)
        print(f"  {prec} iters gpu {st['iters']} / {st['outer_steps']} oracle {io['iters']} / {io['outer_steps']}",
              flush=True)
        assert st["converged"] == 1 and io["converged"]
        assert abs(st["iters"] - io["iters"]) <= 1 and st["outer_steps"] == io["outer_steps"], (prec, st, io)
        assert_elem(host(x), xo, 1e-8, f"{prec} x")
    ctx.close()


def test_uniform_state_at_large_grid():
    """m and h constant: v = alpha h_T - m0 x h_T, lam = (1+alpha^2) m0.h0 at
    any grid size (here 256^3, the headline grid)."""
    n = 256
    announce("uniform state 256^3")
    prm = P.Params(alpha=0.02, dt=2.74e-7, theta=0.5, shift=0.5, h_uniform=(0.3, -0.2, 1.0))
    m0 = np.array([0.48, -0.6, 0.64])
    m0 /= np.linalg.norm(m0)
    ctx = P.Context(n, n, n, 1.0 / n, 0)
    m = torch.empty((3, n, n, n), dtype=torch.float64, device="cuda:0")
    for c in range(3):
        m[c].fill_(m0[c])
    h0 = np.array(prm.h_uniform)
    b = torch.zeros((4, n, n, n), dtype=torch.float64, device="cuda:0")
    for c in range(3):
        b[c].fill_((1 + prm.alpha ** 2) * h0[c])
    x, st = P.gmres_solve(ctx, prm, m, b, rtol=1e-12)
    hT = h0 - (m0 @ h0) * m0
    v = prm.alpha * hT - np.cross(m0, hT)
    lam = (1 + prm.alpha ** 2) * (m0 @ h0)
    for c in range(3):
        assert torch.max(torch.abs(x[c] - v[c])).item() <= 1e-12
    assert torch.max(torch.abs(x[3] - lam)).item() <= 1e-12
    del m, b, x
    ctx.close()


def test_euler_step_matches_oracle_first_workload():
    import llg_workloads as W
    spec = W.make(1)
    announce("euler 32^2 workload 1")
    n = spec["n"]
    g = Grid(n, n, 1, h=spec["h"])
    kw = dict(alpha=spec["alpha"], cexc=1.0, dt=spec["dt"], theta=1.0, shift=0.5, h_uniform=spec["h_uniform"])
    prm, op = both_params(**kw)
    m0 = spec["m0"]
    m_ref, v_ref, lam_ref, info = steppers.euler_step(g, op, m0, rtol=1e-10, restart=30)
    ctx = P.Context(n, n, 1, spec["h"], 0)
    md = dev(m0)
    v = torch.empty((3, 1, n, n), dtype=torch.float64, device="cuda:0")
    lam = torch.empty((1, 1, n, n), dtype=torch.float64, device="cuda:0")
    st = P.llg_step_euler(ctx, prm, md, v, lam, rtol=1e-10)
    assert st["converged"] == 1
    assert abs(st["lin_iters_total"] - info["iters"]) <= 1
    assert_elem(host(v), v_ref, 1e-8, "v")
    assert np.max(np.abs(host(md) - m_ref)) <= 1e-10
    assert st["max_len_err"] <= 1e-14
    ctx.close()


def test_midpoint_steps_invariants_and_oracle():
    n = 32
    announce("midpoint 32^2")
    h = 1.0 / n
    g = Grid(n, n, 1, h=h)
    # the differentiation workload's time step (10 h^2 of its 256^2 grid)
    kw = dict(alpha=0.1, cexc=1.0, dt=10 / 256 ** 2, theta=0.5, shift=0.5, h_uniform=(0.0, 0.0, 0.5))
    prm, op = both_params(**kw)
    m0 = unit_field((1, n, n), 9, smooth=4.0)
    ctx = P.Context(n, n, 1, h, 0)
    md = dev(m0)
    vh = torch.zeros((3, 1, n, n), dtype=torch.float64, device="cuda:0")
    lam = torch.zeros((1, 1, n, n), dtype=torch.float64, device="cuda:0")
    m_ref, v_ref, l_ref = m0, None, None
    for step in range(3):
        # Picard change of the frozen midpoint to 1e-13: the length defect 2 k chi
        # then stays below 1e-12
        st = P.llg_step_midpoint(ctx, prm, md, vh, lam, picard_tol=1e-13, picard_max=60, rtol=1e-13)
        m_ref, v_ref, l_ref, info = steppers.midpoint_step(g, op, m_ref, v_ref, l_ref, rtol=1e-13, picard_tol=1e-13,
                                                           picard_max=60)
        assert st["converged"] == 1
        assert st["max_len_err"] <= 1e-12
        scale = abs(st["energy_before"]) + abs(st["energy_after"])
        assert abs(st["dissipation_defect"] - st["inexact_correction"]) <= 1e-13 * scale
        assert st["energy_after"] <= st["energy_before"]
        assert np.max(np.abs(host(md) - m_ref)) <= 1e-10
    ctx.close()


def test_fp32_ir_matches_fp64():
    n = 64
    announce("fp32-ir 64^2 and 32^3")
    for shape in [(1, n, n), (32, 32, 32)]:
        nz, ny, nx = shape
        h = 1.0 / nx
        g = Grid(nx, ny, nz, h=h)
        # 13.3 times the explicit exchange limit, as in the 3D workloads
        dt = W.dt_explicit_multiple(13.3, 0.05, nx, 2 if nz == 1 else 3)
        prm, op = both_params(alpha=0.05, dt=dt, theta=0.5, shift=0.5, h_uniform=(0.0, 0.0, 1.0))
        m = unit_field(shape, 3, smooth=30.0)
        b = steppers.rhs(g, op, m)
        ctx = P.Context(nx, ny, nz, h, 0)
        x64, s64 = P.gmres_solve(ctx, prm, dev(m), dev(b), rtol=1e-10)
        # flexible inner GMRES (the precision form) and the left-preconditioned
        # inner variant, each with both Arnoldi variants
        for prec in ("fp32_ir", "fp32_ir_left"):
            for orth in ("dcgs2", "cgs2"):
                x32, s32 = P.gmres_solve(ctx, prm, dev(m), dev(b), rtol=1e-10, prec=prec, inner_rtol=1e-5,
                                         orth=orth)
                assert s32["converged"] == 1 and s32["rel_res_true"] <= 1e-10, (prec, orth)
                assert s32["outer_steps"] >= 2
                assert_elem(host(x32), host(x64), 1e-8, f"{prec} {orth} x")
                # inner iterations comparable to the float64 solve's
                assert s32["iters"] <= 2 * s64["iters"] + 10, (prec, orth, s32["iters"], s64["iters"])
        ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32_ir", "fp32_ir_left"])
@pytest.mark.parametrize("restart", [1, 2, 5, 31])
def test_restart_boundaries_match_dense_solve(prec, restart):
    """Delayed-CGS2 cycles that run to the restart length (the last basis
    direction and, in the precision form, the matvec's fused inner products
    over all restart + 1 directions), from restart 1 to the largest the
    delayed variant allows: a random right-hand side and a large shift make
    the preconditioned system slow enough that every cycle is cut at the
    restart length."""
    nx, ny, nz = 8, 8, 1
    announce(f"restart boundaries {prec} restart={restart}")
    h = 1.0 / nx
    g = Grid(nx, ny, nz, h=h)
    prm, op = both_params(alpha=0.1, dt=5e-3, theta=1.0, shift=8.0)
    m = unit_field((nz, ny, nx), 5)
    b = np.random.default_rng(7).standard_normal((4, nz, ny, nx))
    xs = dense.solve(g, op, m, b)
    ctx = P.Context(nx, ny, nz, h, 0)
    x, st = P.gmres_solve(ctx, prm, dev(m), dev(b), restart=restart, rtol=1e-12, prec=prec, inner_rtol=1e-12,
                          max_outer=2000, maxiter=20000)
    assert st["converged"] == 1 and st["rel_res_true"] <= 1e-12, st
    # at least one cycle was cut at the restart length
    assert st["iters"] > restart, st
    assert_elem(host(x), xs, 1e-9, "x")
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32_ir", "fp32_ir_left"])
def test_uniform_state_more_xinv_blocks_than_partial_rows(prec):
    """GMRES at the largest line count, 512 x 384 x 384 (147,456 rows): the
    float64 x-inverse pass (two rows per block) has more blocks than the
    reduction's partial rows, so its Arnoldi inner products fall back to the
    separate pass; the float32 passes (four rows per block) keep them fused.
    The uniform-state closed form fixes the answer."""
    nx, ny, nz = 512, 384, 384
    announce(f"uniform state 512x384x384 {prec}")
    prm = P.Params(alpha=0.02, dt=2.74e-7, theta=0.5, shift=0.5, h_uniform=(0.3, -0.2, 1.0))
    m0 = np.array([0.48, -0.6, 0.64])
    m0 /= np.linalg.norm(m0)
    ctx = P.Context(nx, ny, nz, 1.0 / nx, 0)
    m = torch.empty((3, nz, ny, nx), dtype=torch.float64, device="cuda:0")
    for c in range(3):
        m[c].fill_(m0[c])
    h0 = np.array(prm.h_uniform)
    b = torch.zeros((4, nz, ny, nx), dtype=torch.float64, device="cuda:0")
    for c in range(3):
        b[c].fill_((1 + prm.alpha ** 2) * h0[c])
    x, st = P.gmres_solve(ctx, prm, m, b, rtol=1e-12, restart=4, prec=prec, inner_rtol=1e-6)
    assert st["converged"] == 1
    hT = h0 - (m0 @ h0) * m0
    v = prm.alpha * hT - np.cross(m0, hT)
    lam = (1 + prm.alpha ** 2) * (m0 @ h0)
    for c in range(3):
        assert torch.max(torch.abs(x[c] - v[c])).item() <= 1e-12
    assert torch.max(torch.abs(x[3] - lam)).item() <= 1e-12
    del m, b, x
    ctx.close()
