"""Differentiable midpoint time stepping (torch.autograd.Function).

Forward: ``nsteps`` projection-free midpoint steps (Sec. 3.3) through the C
ABI, keeping only checkpoints (m, v^{n-1/2}, multiplier) every ``ckpt_every``
steps.  Backward: for each segment, newest first, recompute the segment's
steps from its checkpoint (bitwise identical to the forward, since every
kernel and reduction of the library is deterministic), then back-propagate
through each step with llg_step_midpoint_adjoint: one transposed saddle
solve J^T mu = (k gbar, 0) preconditioned by the transposed split FFT-HSS
operator on the step's midpoint.

Differentiable inputs: the initial magnetization m0 (3 planes), the uniform
applied field (3 float64 scalars) and the spatial applied field (3 planes).
"""

import torch

from . import llg as L


class LLGMidpoint(torch.autograd.Function):
    @staticmethod
    def forward(fctx, m0, h_uniform, h_field, ctx, params, nsteps, ckpt_every, solver):
        hu = tuple(float(v) for v in h_uniform.detach().cpu().tolist())
        prm = L.Params(alpha=params.alpha, cexc=params.cexc, dt=params.dt, theta=0.5, shift=params.shift,
                       h_uniform=hu, h_field=h_field.detach().contiguous() if h_field is not None else None,
                       demag=params.demag, aniso_k=params.aniso_k, aniso_axis=params.aniso_axis)
        m = m0.detach().clone().contiguous()
        vh = torch.zeros_like(m)
        lam = torch.zeros((1,) + tuple(m.shape[1:]), dtype=m.dtype, device=m.device)
        step_kw = {k: v for k, v in solver.items() if k != "adjoint_rtol"}
        ckpts = []
        for n in range(nsteps):
            if n % ckpt_every == 0:
                ckpts.append((n, m.clone(), vh.clone(), lam.clone()))
            L.llg_step_midpoint(ctx, prm, m, vh, lam, **step_kw)
        fctx.save_for_backward(*[t for c in ckpts for t in c[1:]])
        fctx.meta = (ctx, prm, nsteps, ckpt_every, solver, [c[0] for c in ckpts], h_field is not None,
                     h_uniform.device)
        return m

    @staticmethod
    def backward(fctx, g_out):
        ctx, prm, nsteps, ckpt_every, solver, starts, has_field, hu_device = fctx.meta
        saved = fctx.saved_tensors
        gbar = g_out.detach().clone().contiguous()
        hbar_field = torch.zeros_like(gbar) if has_field else None
        hbar_u = [0.0, 0.0, 0.0]
        adj_kw = dict(restart=solver.get("restart", 30), rtol=solver.get("adjoint_rtol", 1e-12))
        step_kw = {k: v for k, v in solver.items() if k != "adjoint_rtol"}
        for s in reversed(range(len(starts))):
            n0 = starts[s]
            n1 = min(n0 + ckpt_every, nsteps)
            m, vh, lam = (t.clone() for t in saved[3 * s:3 * s + 3])
            states = []
            for _ in range(n0, n1):
                m_n = m.clone()
                L.llg_step_midpoint(ctx, prm, m, vh, lam, **step_kw)
                states.append((m_n, vh.clone(), lam.clone()))
            for (m_n, v, r) in reversed(states):
                hbar_u, _ = L.llg_step_midpoint_adjoint(ctx, prm, m_n, v, r, gbar, hbar_field, hbar_u, **adj_kw)
        g_hu = torch.tensor(hbar_u, dtype=torch.float64, device=hu_device)
        return gbar, g_hu, hbar_field, None, None, None, None, None


def midpoint_trajectory(ctx, params, m0, h_uniform, h_field=None, nsteps=1, ckpt_every=5, picard_tol=1e-10,
                        picard_max=50, restart=30, rtol=1e-10, adjoint_rtol=1e-12):
    """m_N after ``nsteps`` midpoint steps from m0, differentiable in m0,
    h_uniform (tensor of 3 float64) and h_field (3 planes or None)."""
    solver = dict(picard_tol=picard_tol, picard_max=picard_max, restart=restart, rtol=rtol,
                  adjoint_rtol=adjoint_rtol)
    return LLGMidpoint.apply(m0, h_uniform, h_field, ctx, params, int(nsteps), int(ckpt_every), solver)
