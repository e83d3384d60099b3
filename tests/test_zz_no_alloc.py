"""gmres_solve_noalloc (the library's static workspace) against gmres_solve
(a caller workspace) through the C ABI: two solves in a row, the second on a
smaller grid, in every precision; both paths run the same kernels in the
same order, so the solutions and statistics agree bitwise.  A grid whose
workspace exceeds the static array is rejected with LLG_ENOMEM."""

import numpy as np
import pytest
import torch

import paper_2607_15290_amd as P
from paper_2607_15290_amd.llg import LLGError
from tests.gpu_util import announce, dev, unit_field

pytestmark = pytest.mark.gpu


def _system(nx, ny, nz, seed):
    m = unit_field((nz, ny, nx), seed, smooth=10.0)
    b = np.random.default_rng(seed + 1).standard_normal((4, nz, ny, nx))
    return m, b


@pytest.mark.parametrize("prec", ["fp64", "fp32_ir", "fp32_ir_left"])
def test_noalloc_matches_workspace_solve(prec):
    for (nx, ny, nz) in [(256, 256, 1), (64, 32, 16)]:  # second call: smaller input
        announce(f"noalloc vs workspace {prec} {(nx, ny, nz)}")
        h = 1.0 / nx
        prm = P.Params(alpha=0.1, cexc=1.0, dt=10 * h * h, theta=0.5, shift=0.5, h_uniform=(0.0, 0.0, 0.5))
        m, _ = _system(nx, ny, nz, 3)
        ctx = P.Context(nx, ny, nz, h, 0)
        md = dev(m)
        bd = P.llg_rhs(ctx, prm, md)  # a time step's right-hand side
        kw = dict(rtol=1e-10, prec=prec, inner_rtol=1e-3)
        x_ref, st_ref = P.gmres_solve(ctx, prm, md, bd, **kw)
        x_na, st_na = P.gmres_solve_noalloc(ctx, prm, md, bd, **kw)
        torch.cuda.synchronize()
        assert st_ref["converged"] == 1 and st_na["converged"] == 1
        assert torch.equal(x_na, x_ref)
        for key in ("iters", "cycles", "outer_steps", "rel_res_true", "rel_res_prec"):
            assert st_na[key] == st_ref[key], key
        ctx.close()


def test_noalloc_rejects_grids_beyond_the_static_workspace():
    announce("noalloc rejects 512^2 at restart 30")
    n = 512
    ctx = P.Context(n, n, 1, 1.0 / n, 0)
    nbytes = ctx.lib.llg_workspace_bytes(ctx.handle, 30, 0)
    assert nbytes > 128 << 20
    m, b = _system(n, n, 1, 5)
    prm = P.Params(alpha=0.1, dt=1e-6, theta=0.5)
    with pytest.raises(LLGError) as ei:
        P.gmres_solve_noalloc(ctx, prm, dev(m), dev(b))
    assert ei.value.name == "LLG_ENOMEM"
    # a restart length whose workspace fits is accepted on the same grid
    x, st = P.gmres_solve_noalloc(ctx, prm, dev(m), dev(b), restart=4, rtol=1e-8)
    assert st["converged"] == 1
    ctx.close()
