"""Pins of the matrix-free saddle operator and the split FFT-HSS
preconditioner against the dense assembled matrices (Sec. 2.4, 3.1, 3.2) and
the algebraic identities of Sec. 3.4 (Theorem "Full saddle two-step
contraction": M - (lambda I - calH)(lambda I - calS) = 2 lambda A and
M^{-1} A = (I - T)/(2 lambda))."""

import numpy as np
import pytest

from oracle import dense, nodal, operators
from oracle.grid import Grid
from oracle.operators import Params

CASES = [((1, 4, 4), dict(alpha=0.2, dt=1e-2, theta=1.0, shift=0.5)),
         ((1, 6, 4), dict(alpha=0.05, dt=3e-3, theta=0.5, shift=0.25)),
         ((4, 4, 4), dict(alpha=0.1, dt=2e-2, theta=1.0, shift=1.5)),
         ((1, 5, 5), dict(alpha=0.3, dt=5e-2, theta=0.5, shift=0.7))]


def _setup(shape, kw, seed=0, unit=True):
    g = Grid(shape[2], shape[1], shape[0], lengths=(1.0, 1.0, 1.0))
    prm = Params(cexc=1.0, **kw)
    rng = np.random.default_rng(seed)
    m = rng.standard_normal((3,) + g.shape)
    if unit:
        m /= np.sqrt(nodal.dot(m, m))
    x = rng.standard_normal((4,) + g.shape)
    return g, prm, m, x


@pytest.mark.parametrize("shape,kw", CASES)
def test_matvec_matches_dense(shape, kw):
    g, prm, m, x = _setup(shape, kw)
    A = dense.saddle_matrix(g, prm, m)
    np.testing.assert_allclose(operators.matvec(g, prm, m, x).ravel(), A @ x.ravel(), atol=1e-12 * np.abs(A).max())
    np.testing.assert_allclose(operators.matvec_transpose(g, prm, m, x).ravel(), A.T @ x.ravel(),
                               atol=1e-12 * np.abs(A).max())


@pytest.mark.parametrize("shape,kw", CASES)
def test_hermitian_skew_parts_and_constraint(shape, kw):
    g, prm, m, _ = _setup(shape, kw, unit=False)
    calH, calS = dense.saddle_parts(g, prm, m)
    A = calH + calS
    np.testing.assert_allclose(calH, 0.5 * (A + A.T), atol=1e-14)
    np.testing.assert_allclose(calS, 0.5 * (A - A.T), atol=1e-14)
    n = g.ng
    B = -A[3 * n:, :3 * n]          # constraint row is -B
    np.testing.assert_allclose(B @ B.T, np.diag(nodal.dot(m, m).ravel()), atol=1e-14)
    assert np.min(np.linalg.eigvalsh(calH[:3 * n, :3 * n])) >= prm.alpha * (1 - 1e-12)


@pytest.mark.parametrize("shape,kw", CASES)
def test_hss_apply_equals_dense_factor_inverses(shape, kw):
    """The preconditioner equals the product of the exact HSS factor inverses
    to 1e-12 (relative), plain and transposed."""
    g, prm, m, x = _setup(shape, kw, seed=1)
    M1, M2 = dense.hss_factors(g, prm, m)
    ref = np.linalg.solve(M2, np.linalg.solve(M1, x.ravel()))
    got = operators.hss_apply(g, prm, m, x).ravel()
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
    M = M1 @ M2
    reft = np.linalg.solve(M.T, x.ravel())
    gott = operators.hss_apply(g, prm, m, x, transpose=True).ravel()
    assert np.linalg.norm(gott - reft) <= 1e-12 * np.linalg.norm(reft)


@pytest.mark.parametrize("shape,kw", CASES)
def test_hss_identities(shape, kw):
    g, prm, m, _ = _setup(shape, kw, seed=2)
    calH, calS = dense.saddle_parts(g, prm, m)
    lam = prm.shift
    eye = np.eye(calH.shape[0])
    A = calH + calS
    M = (calH + lam * eye) @ (calS + lam * eye)
    np.testing.assert_allclose(M - (lam * eye - calH) @ (lam * eye - calS), 2 * lam * A, atol=1e-11 * np.abs(M).max())
    T = (np.linalg.solve(lam * eye + calS, lam * eye - calH)
         @ np.linalg.solve(lam * eye + calH, lam * eye - calS))
    np.testing.assert_allclose(np.linalg.solve(M, A), (eye - T) / (2 * lam), atol=1e-11)


@pytest.mark.parametrize("shape,kw", CASES)
def test_fused_preconditioned_operator_identity(shape, kw):
    """M^{-1} A x = M2^{-1} [x + M1^{-1} ((calS - lambda I) x)] since
    A = M1 + (calS - lambda I)."""
    g, prm, m, x = _setup(shape, kw, seed=3)
    lam = prm.shift
    u = nodal.s_apply(m, x) - lam * x
    fused = operators.m2_solve(m, prm, x + operators.m1_solve(g, prm, u))
    plain = operators.precond_op(g, prm, m, x)
    assert np.linalg.norm(fused - plain) <= 1e-13 * np.linalg.norm(plain)


@pytest.mark.parametrize("shape,kw", CASES)
def test_residual_under_a_nodal_block_change(shape, kw):
    """A(m) depends on m only through its nodal blocks (Sec. 2.4, eq. "saddle
    point system"), so for fixed b and x the residual at a new m follows from
    the old one by a nodal correction: b - A(m + dm) x = (b - A(m) x)
    - (dm x v + dm r, -dm . v).  The GPU midpoint loop carries its residual
    from one Picard system to the next this way; here both sides come from
    the dense matrix."""
    g, prm, m, x = _setup(shape, kw, seed=3, unit=False)
    dm = 1e-2 * np.random.default_rng(4).standard_normal(m.shape)
    b = np.random.default_rng(5).standard_normal(x.shape)
    A0 = dense.saddle_matrix(g, prm, m)
    A1 = dense.saddle_matrix(g, prm, m + dm)
    r0 = b.ravel() - A0 @ x.ravel()
    r1 = b.ravel() - A1 @ x.ravel()
    v, lam = x[:3], x[3]
    corr = np.empty_like(x)
    corr[:3] = nodal.cross(dm, v) + dm * lam
    corr[3] = -nodal.dot(dm, v)
    assert np.max(np.abs(r1 - (r0 - corr.ravel()))) <= 1e-13 * np.max(np.abs(r1))
