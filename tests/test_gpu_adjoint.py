"""GPU parity of the differentiation form: the adjoint of one midpoint step
against the oracle adjoint (the one-pipeline right-preconditioned solve and
the two-pipeline left one, with the oracle's iteration counts at 256^2), and the checkpointed autograd trajectory (the
differentiation workload: 20 midpoint steps, checkpoints every 5, loss
sum m_z^2) against the oracle's adjoint chain and central finite differences
(step 1e-6) on the 16^2 copy, and against finite differences at 256^2."""

import numpy as np
import pytest
import torch

import llg_workloads as W
import paper_2607_15290_amd as P
from oracle import adjoint, steppers
from oracle.grid import Grid
from oracle.operators import Params as OP
from tests.gpu_util import announce, assert_elem, dev, host

pytestmark = pytest.mark.gpu

TIGHT = dict(picard_tol=1e-12, picard_max=100, rtol=1e-13, adjoint_rtol=1e-13)


def _spec(n):
    spec = W.make(5, n=n)
    kw = dict(alpha=spec["alpha"], cexc=1.0, dt=spec["dt"], theta=0.5, shift=spec["shift"])
    return spec, kw


def test_adjoint_step_matches_oracle():
    n = 16
    announce("adjoint step 16^2")
    spec, kw = _spec(n)
    g = Grid(n, n, 1, h=spec["h"])
    hf = spec["h_field"]
    op = OP(h_uniform=spec["h_uniform"], h_field=hf, **kw)
    m_n = spec["m0"]
    m1, v, r, info = steppers.midpoint_step(g, op, m_n, rtol=1e-14, picard_tol=1e-13, picard_max=100)
    gbar = np.zeros_like(m1)
    gbar[2] = 2 * m1[2]
    gb_ref, hf_ref, hu_ref, mu, _ = adjoint.step_adjoint(g, op, m_n, v, r, gbar, rtol=1e-14)
    ctx = P.Context(n, n, 1, spec["h"], 0)
    prm = P.Params(h_uniform=spec["h_uniform"], h_field=dev(hf), **kw)
    gb = dev(gbar)
    hbf = torch.zeros_like(gb)
    hu, st = P.llg_step_midpoint_adjoint(ctx, prm, dev(m_n), dev(v), dev(r), gb, hbf, [0.0, 0.0, 0.0], rtol=1e-14)
    assert st["converged"] == 1
    assert_elem(host(gb), gb_ref, 1e-10, "gbar")
    assert_elem(host(hbf), hf_ref, 1e-10, "hbar_field")
    np.testing.assert_allclose(hu, hu_ref, rtol=1e-10, atol=1e-14 * np.abs(hu_ref).max())
    ctx.close()


def _gpu_loss(ctx, kw, m0, hu, hf, nsteps):
    prm = P.Params(**kw)
    m = P.midpoint_trajectory(ctx, prm, m0, hu, hf, nsteps=nsteps, ckpt_every=5, **TIGHT)
    return float((m[2] ** 2).sum().item())


def test_autograd_trajectory_small_copy():
    n, nsteps = 16, 20
    announce("autograd 16^2 x 20 steps")
    spec, kw = _spec(n)
    g = Grid(n, n, 1, h=spec["h"])
    ctx = P.Context(n, n, 1, spec["h"], 0)
    m0 = dev(spec["m0"]).requires_grad_(True)
    hu = torch.tensor(spec["h_uniform"], dtype=torch.float64, requires_grad=True)
    hf = dev(spec["h_field"]).requires_grad_(True)
    prm = P.Params(**kw)
    mN = P.midpoint_trajectory(ctx, prm, m0, hu, hf, nsteps=nsteps, ckpt_every=5, **TIGHT)
    loss = (mN[2] ** 2).sum()
    loss.backward()
    # oracle chain on the same inputs
    op = OP(h_uniform=spec["h_uniform"], h_field=spec["h_field"], **kw)
    m, v, r = spec["m0"], None, None
    traj = []
    for _ in range(nsteps):
        m_new, v, r, info = steppers.midpoint_step(g, op, m, v, r, rtol=1e-14, picard_tol=1e-13, picard_max=100)
        traj.append((m, v, r))
        m = m_new
    assert_elem(host(mN), m, 1e-10, "m_N")
    gb = np.zeros_like(m)
    gb[2] = 2 * m[2]
    ghf = np.zeros_like(m)
    ghu = np.zeros(3)
    for (m_n, vv, rr) in reversed(traj):
        gb, a, b, _, _ = adjoint.step_adjoint(g, op, m_n, vv, rr, gb, rtol=1e-14)
        ghf += a
        ghu += b
    assert_elem(host(m0.grad), gb, 1e-8, "dL/dm0")
    assert_elem(host(hf.grad), ghf, 1e-8, "dL/dh_field")
    np.testing.assert_allclose(hu.grad.numpy(), ghu, rtol=1e-8)
    # central differences (step 1e-6) through the GPU forward
    eps = 1e-6
    base = dict(m0=m0.detach(), hu=hu.detach(), hf=hf.detach())
    for c in range(3):
        e = torch.zeros(3, dtype=torch.float64)
        e[c] = eps
        fp = _gpu_loss(ctx, kw, base["m0"], base["hu"] + e, base["hf"], nsteps)
        fm = _gpu_loss(ctx, kw, base["m0"], base["hu"] - e, base["hf"], nsteps)
        assert hu.grad[c].item() == pytest.approx((fp - fm) / (2 * eps), rel=1e-5, abs=1e-8)
    rng = np.random.default_rng(0)
    for _ in range(2):
        d = dev(rng.standard_normal(hf.shape))
        fp = _gpu_loss(ctx, kw, base["m0"], base["hu"], base["hf"] + eps * d, nsteps)
        fm = _gpu_loss(ctx, kw, base["m0"], base["hu"], base["hf"] - eps * d, nsteps)
        assert float((hf.grad * d).sum()) == pytest.approx((fp - fm) / (2 * eps), rel=1e-5, abs=1e-8)
    ctx.close()


def test_autograd_full_size_finite_differences():
    n, nsteps = 256, 20
    announce("autograd 256^2 x 20 steps (FD on the uniform field)")
    spec, kw = _spec(n)
    ctx = P.Context(n, n, 1, spec["h"], 0)
    m0 = dev(spec["m0"])
    hu = torch.tensor(spec["h_uniform"], dtype=torch.float64, requires_grad=True)
    hf = dev(spec["h_field"]).requires_grad_(True)
    prm = P.Params(**kw)
    mN = P.midpoint_trajectory(ctx, prm, m0, hu, hf, nsteps=nsteps, ckpt_every=5, **TIGHT)
    (mN[2] ** 2).sum().backward()
    eps = 1e-6
    for c in (0, 2):
        e = torch.zeros(3, dtype=torch.float64)
        e[c] = eps
        fp = _gpu_loss(ctx, kw, m0, hu.detach() + e, hf.detach(), nsteps)
        fm = _gpu_loss(ctx, kw, m0, hu.detach() - e, hf.detach(), nsteps)
        assert hu.grad[c].item() == pytest.approx((fp - fm) / (2 * eps), rel=1e-5, abs=1e-6)
    ctx.close()


@pytest.mark.parametrize("orth", ["dcgs2", "cgs2"])
def test_adjoint_step_full_size_against_oracle(orth):
    """One adjoint step of the differentiation workload at 256^2 (its full
    size) after its first forward step: dcgs2 takes the right-preconditioned
    one-pipeline solve, cgs2 the left-preconditioned two-pipeline one; each
    against the oracle's GMRES with the same preconditioning side: iteration
    counts within one, gbar_n and hbar element-wise to the tolerance-scaled
    distance."""
    n = 256
    announce(f"adjoint step 256^2 {orth}")
    spec, kw = _spec(n)
    g = Grid(n, n, 1, h=spec["h"])
    hf = spec["h_field"]
    op = OP(h_uniform=spec["h_uniform"], h_field=hf, **kw)
    m_n = spec["m0"]
    m1, v, r, info = steppers.midpoint_step(g, op, m_n, rtol=1e-12, picard_tol=1e-12, picard_max=100)
    gbar = np.zeros_like(m1)
    gbar[2] = 2 * m1[2]
    side = "right" if orth == "dcgs2" else "left"
    gb_ref, hf_ref, hu_ref, mu, ainfo = adjoint.step_adjoint(g, op, m_n, v, r, gbar, rtol=1e-10, side=side)
    ctx = P.Context(n, n, 1, spec["h"], 0)
    prm = P.Params(h_uniform=spec["h_uniform"], h_field=dev(hf), **kw)
    gb = dev(gbar)
    hbf = torch.zeros_like(gb)
    hu, st = P.llg_step_midpoint_adjoint(ctx, prm, dev(m_n), dev(v), dev(r), gb, hbf, [0.0, 0.0, 0.0], rtol=1e-10,
                                         orth=orth)
    print(f"  adjoint iters gpu {st['iters']} oracle ({side}) {ainfo['iters']}, {st['ms']:.1f} ms", flush=True)
    assert st["converged"] == 1 and abs(st["iters"] - ainfo["iters"]) <= 1
    assert_elem(host(gb), gb_ref, 1e-8, "gbar")
    assert_elem(host(hbf), hf_ref, 1e-8, "hbar_field")
    np.testing.assert_allclose(hu, hu_ref, rtol=1e-8)
    ctx.close()
