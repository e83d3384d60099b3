"""Pins of the midpoint adjoint: the dense Jacobian against central finite
differences of the residual of eq. "C-N" (Sec. 3.3) written out directly, the
matrix-free J^T against the dense transpose, and the whole adjoint against
central finite differences of the oracle's forward midpoint stepper."""

import numpy as np
import pytest

from oracle import adjoint, dense, fourier, nodal, steppers
from oracle.grid import Grid
from oracle.operators import Params


def _state(g, seed, amp=1.0):
    rng = np.random.default_rng(seed)
    m = rng.standard_normal((3,) + g.shape)
    mh = np.fft.fftn(m, axes=(-3, -2, -1)) * np.exp(-g.s / g.s.max() * 6)
    m = np.fft.ifftn(mh, axes=(-3, -2, -1)).real
    return m / np.sqrt(nodal.dot(m, m))


def _residual(g, prm, m_n, h, u):
    k = prm.dt
    v, r = u[:3], u[3]
    mh = m_n + 0.5 * k * v
    out = np.empty_like(u)
    out[:3] = (prm.alpha * v + nodal.cross(mh, v) + prm.c_hat * fourier.neg_laplacian(g, mh)
               + mh * r - (1 + prm.alpha ** 2) * h)
    out[3] = -nodal.dot(mh, v)
    return out


def test_dense_jacobian_is_derivative_of_residual():
    g = Grid(4, 4, 1, h=0.25)
    prm = Params(alpha=0.1, dt=0.05, theta=0.5, shift=0.5)
    rng = np.random.default_rng(0)
    m_n = _state(g, 1)
    h = rng.standard_normal((3,) + g.shape)
    u = rng.standard_normal((4,) + g.shape)
    J = dense.midpoint_jacobian(g, prm, m_n, u[:3], u[3])
    eps = 1e-6
    for trial in range(4):
        du = rng.standard_normal(u.shape)
        fd = (_residual(g, prm, m_n, h, u + eps * du) - _residual(g, prm, m_n, h, u - eps * du)) / (2 * eps)
        np.testing.assert_allclose(J @ du.ravel(), fd.ravel(), atol=1e-8 * np.abs(fd).max())
        np.testing.assert_allclose(adjoint.jacobian_apply(g, prm, m_n, u[:3], u[3], du).ravel(),
                                   J @ du.ravel(), atol=1e-12 * np.abs(J).max())
        np.testing.assert_allclose(adjoint.jacobian_transpose_apply(g, prm, m_n, u[:3], u[3], du).ravel(),
                                   J.T @ du.ravel(), atol=1e-12 * np.abs(J).max())


def _forward(g, prm, m0, hu, hf, nsteps):
    p = Params(alpha=prm.alpha, cexc=prm.cexc, dt=prm.dt, shift=prm.shift, h_uniform=tuple(hu), h_field=hf)
    m, v, lam = m0, None, None
    traj = []
    for _ in range(nsteps):
        m_new, v, lam, info = steppers.midpoint_step(g, p, m, v, lam, rtol=1e-14, picard_tol=1e-14, picard_max=100)
        assert info["converged"]
        traj.append((m, v, lam))
        m = m_new
    return m, traj


def _loss(m):
    return float((m[2] ** 2).sum())


@pytest.mark.parametrize("dense_solve", [False, True])
def test_adjoint_matches_central_differences(dense_solve):
    g = Grid(6, 6, 1, h=1.0 / 6)
    prm = Params(alpha=0.1, dt=0.01, theta=0.5, shift=0.5)
    rng = np.random.default_rng(3)
    m0 = _state(g, 4)
    hu = np.array([0.0, 0.0, 0.5])
    hf = 0.1 * rng.standard_normal((3,) + g.shape)
    nsteps = 3
    mN, traj = _forward(g, prm, m0, hu, hf, nsteps)
    gbar = np.zeros_like(mN)
    gbar[2] = 2 * mN[2]
    p = Params(alpha=prm.alpha, dt=prm.dt, shift=prm.shift, h_uniform=tuple(hu), h_field=hf)
    hbar_f = np.zeros_like(hf)
    hbar_u = np.zeros(3)
    for (m_n, v, lam) in reversed(traj):
        gbar, hf_b, hu_b, mu, info = adjoint.step_adjoint(g, p, m_n, v, lam, gbar, rtol=1e-14, dense=dense_solve)
        hbar_f += hf_b
        hbar_u += hu_b
    eps = 1e-6
    for c in range(3):
        e = np.zeros(3)
        e[c] = eps
        fd = (_loss(_forward(g, prm, m0, hu + e, hf, nsteps)[0]) - _loss(_forward(g, prm, m0, hu - e, hf, nsteps)[0])) / (2 * eps)
        assert hbar_u[c] == pytest.approx(fd, rel=1e-5, abs=1e-9)
    for trial in range(2):
        d = rng.standard_normal(hf.shape)
        fd = (_loss(_forward(g, prm, m0, hu, hf + eps * d, nsteps)[0]) - _loss(_forward(g, prm, m0, hu, hf - eps * d, nsteps)[0])) / (2 * eps)
        assert float((hbar_f * d).sum()) == pytest.approx(fd, rel=1e-5, abs=1e-9)
        dm = rng.standard_normal(m0.shape)
        fd = (_loss(_forward(g, prm, m0 + eps * dm, hu, hf, nsteps)[0]) - _loss(_forward(g, prm, m0 - eps * dm, hu, hf, nsteps)[0])) / (2 * eps)
        assert float((gbar * dm).sum()) == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_right_preconditioned_transposed_jacobian_identity():
    """Without a lower-order field, J^T M^{-T} = [I + (N - lambda I) M1^{-1}] M2^{-T}
    with M1 = calH + lambda I, M2 = calS(m_half) + lambda I and N = J^T - calH
    node-wise: checked on the dense assembled matrices, and N against the
    dense difference."""
    g = Grid(4, 4, 1, h=0.25)
    prm = Params(alpha=0.1, dt=0.05, theta=0.5, shift=0.5)
    rng = np.random.default_rng(4)
    m_n = _state(g, 2)
    v = 0.3 * rng.standard_normal((3,) + g.shape)
    r = rng.standard_normal(g.shape)
    J = dense.midpoint_jacobian(g, prm, m_n, v, r)
    m_half = m_n + 0.5 * prm.dt * v
    M1, M2 = dense.hss_factors(g, prm, m_half)
    calH = M1 - prm.shift * np.eye(M1.shape[0])
    Nd = J.T - calH
    n = g.ng
    # N is node-wise: no coupling between different nodes (up to the rounding
    # of the dense Laplacian's symmetry)
    for i in range(n):
        for j in range(n):
            if i != j:
                assert np.all(np.abs(Nd[np.ix_(np.arange(4) * n + i, np.arange(4) * n + j)]) <= 1e-13)
    x = rng.standard_normal((4,) + g.shape)
    np.testing.assert_allclose(adjoint.nodal_part(prm, m_n, v, r, x).ravel(), Nd @ x.ravel(), atol=1e-13)
    lhs = J.T @ np.linalg.inv((M1 @ M2).T)
    rhs = (np.eye(4 * n) + (Nd - prm.shift * np.eye(4 * n)) @ np.linalg.inv(M1)) @ np.linalg.inv(M2.T)
    np.testing.assert_allclose(lhs, rhs, atol=1e-12 * np.abs(lhs).max())


def test_right_preconditioned_adjoint_matches_dense():
    """The adjoint solved with right preconditioning equals the dense one."""
    g = Grid(8, 8, 1, h=1.0 / 8)
    prm = Params(alpha=0.1, dt=1e-3, theta=0.5, shift=0.5, h_uniform=(0.0, 0.0, 0.5))
    m_n = _state(g, 3)
    m1, v, r, _ = steppers.midpoint_step(g, prm, m_n, rtol=1e-14, picard_tol=1e-13, picard_max=100)
    gbar = np.random.default_rng(5).standard_normal(m1.shape)
    want = adjoint.step_adjoint(g, prm, m_n, v, r, gbar, dense=True)
    got = adjoint.step_adjoint(g, prm, m_n, v, r, gbar, rtol=1e-13, side="right")
    assert got[4]["converged"]
    for a, b in zip(got[:4], want[:4]):
        np.testing.assert_allclose(a, b, atol=1e-9 * np.abs(b).max())
