"""GPU parity of the delayed-CGS2 update carried by the next operator's first
x pass (k_xfwd_upd, llg_solver_opts::fuse_update = 1 forces it on any grid).

Each of the four operators that take it -- the float64 fused M^{-1} A pass,
the precision form's float32 apply, the left variant's float32 M^{-1} A and
the right-preconditioned adjoint's one pipeline -- is run with the fused
update on small grids chosen for their x-pass blocks: a block covering more
lines than the grid has (a ragged, partly dead block), mixed-radix lines, and
a stiff system whose cycles run to 30 columns (steps past the eighth switch
to the separate update pass within the cycle); 256-point x lines (the
instantiations of the 256^3 runs); and one 3D grid above 2^20 nodes, where
no operator is launched ahead of the host's decision on the cycle.
Solutions are compared element-wise with the oracle's solvers, iteration
counts with the oracle's and with the unfused path's."""

import numpy as np
import pytest

import llg_workloads as W
import paper_2607_15290_amd as P
from oracle import adjoint, gmres as og, operators, steppers
from oracle.grid import Grid
from oracle.operators import Params as OP
from tests.gpu_util import announce, assert_elem, both_params, dev, host, unit_field

pytestmark = pytest.mark.gpu

# (nx, ny, nz, dt as a multiple of the explicit exchange limit)
CASES = [
    (32, 32, 1, 13.3),   # float32 x pass: one 64-line block, half of it dead
    (24, 10, 6, 13.3),   # half-length 12 (radices 4, 3), 60 lines
    (40, 6, 4, 13.3),    # half-length 20 (radices 4, 5), 24 lines
    (64, 64, 1, 400.0),  # stiff: full cycles, fused and separate updates mixed
    # 256-point x lines, the instantiations of the 256^3 runs (half-length
    # 128: 8 lines per float32 block, 4 per float64 block)
    (256, 6, 6, 13.3),   # 36 lines (radix 3 along y and z): the last float32 block half dead
    (256, 10, 1, 400.0),  # stiff, 10 lines: full cycles; the last block of either precision partly dead
    (512, 10, 1, 13.3),  # 512-point x lines (the 512^3 capacity run's instantiations): 4 lines per
                         # float32 block, the last one half dead
    # above 2^20 nodes, where the next operator is not launched ahead of the
    # host's decision: the cycle waits for each step (1.3M nodes; the
    # oracle's three solves take up to a minute)
    pytest.param(256, 80, 64, 13.3, marks=pytest.mark.timeout(600)),
]


def _system(nx, ny, nz, mult, seed=5):
    h = 1.0 / nx
    g = Grid(nx, ny, nz, h=h)
    dt = W.dt_explicit_multiple(mult, 0.02, max(nx, ny, nz), 2 if nz == 1 else 3)
    prm, op = both_params(alpha=0.02, cexc=1.0, dt=dt, theta=0.5, shift=0.5, h_uniform=(0.0, 0.0, 1.0))
    m = unit_field((nz, ny, nx), seed, smooth=12.0)
    m = m + 0.01 * unit_field((nz, ny, nx), seed + 1)
    m = m / np.sqrt((m * m).sum(0))
    return g, prm, op, m, steppers.rhs(g, op, m)


@pytest.mark.parametrize("nx,ny,nz,mult", CASES)
def test_fused_update_solves_match_oracle(nx, ny, nz, mult):
    announce(f"fused update solves {nx}x{ny}x{nz} dt x{mult}")
    g, prm, op, m, b = _system(nx, ny, nz, mult)
    A = lambda v: operators.matvec(g, op, m, v)
    M = lambda v: operators.hss_apply(g, op, m, v)
    ctx = P.Context(nx, ny, nz, 1.0 / nx, 0)
    md, bd = dev(m), dev(b)
    xr, ir = steppers.solve_saddle(g, op, m, b, rtol=1e-10)
    x, st = P.gmres_solve(ctx, prm, md, bd, rtol=1e-10, fuse_update="always")
    _, sn = P.gmres_solve(ctx, prm, md, bd, rtol=1e-10, fuse_update="never")
    print(f"  fp64 iters fused {st['iters']} unfused {sn['iters']} oracle {ir['iters']}", flush=True)
    assert st["converged"] == 1 and abs(st["iters"] - ir["iters"]) <= 1 and abs(st["iters"] - sn["iters"]) <= 1
    assert_elem(host(x), xr, 1e-8, "fp64 x")
    if mult > 100:
        assert st["iters"] > 30, "the stiff case must run full cycles"
    for prec, inner in (("fp32_ir", "flexible"), ("fp32_ir_left", "left")):
        xo, io = og.fgmres_ir(A, M, b, restart=30, rtol=1e-10, inner_rtol=1e-3, max_outer=20, inner=inner)
        x, st = P.gmres_solve(ctx, prm, md, bd, rtol=1e-10, prec=prec, inner_rtol=1e-3, fuse_update="always")
        _, sn = P.gmres_solve(ctx, prm, md, bd, rtol=1e-10, prec=prec, inner_rtol=1e-3, fuse_update="never")
        print(f"  {prec} iters fused {st['iters']} unfused {sn['iters']} oracle {io['iters']}", flush=True)
        assert st["converged"] == 1 and io["converged"]
        assert abs(st["iters"] - io["iters"]) <= 1 and abs(st["iters"] - sn["iters"]) <= 1, (prec, st, io)
        assert_elem(host(x), xo, 1e-8, f"{prec} x")
    ctx.close()


def _adjoint_case(g, op, prm, ctx, m_n):
    """One adjoint step solved with the fused update forced on and off,
    against the oracle's right-preconditioned adjoint."""
    m1, v, r, _ = steppers.midpoint_step(g, op, m_n, rtol=1e-14, picard_tol=1e-13, picard_max=100)
    gbar = np.zeros_like(m1)
    gbar[2] = 2 * m1[2]
    gb_ref, hf_ref, _, _, info = adjoint.step_adjoint(g, op, m_n, v, r, gbar, rtol=1e-12, side="right")
    iters = {}
    for fuse in ("always", "never"):
        gb = dev(gbar)
        hbf = dev(np.zeros_like(gbar))
        _, st = P.llg_step_midpoint_adjoint(ctx, prm, dev(m_n), dev(v), dev(r), gb, hbf, [0.0, 0.0, 0.0],
                                           rtol=1e-12, fuse_update=fuse)
        assert st["converged"] == 1
        iters[fuse] = st["iters"]
        assert_elem(host(gb), gb_ref, 1e-9, f"gbar ({fuse})")
        assert_elem(host(hbf), hf_ref, 1e-9, f"hbar_field ({fuse})")
    print(f"  adjoint iters fused {iters['always']} unfused {iters['never']} oracle {info['iters']}", flush=True)
    assert abs(iters["always"] - info["iters"]) <= 1 and abs(iters["always"] - iters["never"]) <= 1


@pytest.mark.parametrize("n", [32, 48])
def test_fused_update_adjoint_matches_oracle(n):
    """The right-preconditioned adjoint solve (prologue M2^{-T}) with the
    fused update, against the oracle's right-preconditioned adjoint."""
    announce(f"fused update adjoint {n}^2")
    spec = W.make(5, n=n)
    kw = dict(alpha=spec["alpha"], cexc=1.0, dt=spec["dt"], theta=0.5, shift=spec["shift"])
    g = Grid(n, n, 1, h=spec["h"])
    op = OP(h_uniform=spec["h_uniform"], **kw)
    ctx = P.Context(n, n, 1, spec["h"], 0)
    _adjoint_case(g, op, P.Params(h_uniform=spec["h_uniform"], **kw), ctx, spec["m0"])
    ctx.close()


@pytest.mark.parametrize("nx", [256, 512])
def test_fused_update_adjoint_long_lines(nx):
    """The adjoint's float64 fused pass on 256- and 512-point x lines (4 and
    2 lines per block): 10 lines, so at 256 the last block is half dead."""
    announce(f"fused update adjoint {nx}x10")
    g, prm, op, m, _ = _system(nx, 10, 1, 13.3)
    ctx = P.Context(nx, 10, 1, 1.0 / nx, 0)
    _adjoint_case(g, op, prm, ctx, m)
    ctx.close()
