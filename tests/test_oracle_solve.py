"""Pins of the oracle GMRES: the dense direct solve (Proposition 1 makes the
solution unique), the uniform-state closed form derived from the tangent
equation, the even-step residual bound of the Theorem "Full saddle two-step
contraction", and the paper's printed iteration counts: the preconditioner
comparison on the smooth one-step system (Sec. 4.3, exact), the shift sweep
(Sec. 4.4, exact minimum and band) and the random right-hand-side mesh study
(Sec. 4.5, soft)."""

import json
import os

import numpy as np

import llg_workloads
import pytest

from oracle import dense, fourier, gmres, manufactured, nodal, operators, steppers, theory
from oracle.grid import Grid
from oracle.operators import Params

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_printed_values.json")))


@pytest.mark.parametrize("shape,theta", [((1, 4, 4), 1.0), ((1, 8, 6), 0.5), ((4, 4, 4), 1.0)])
def test_gmres_matches_dense_solve(shape, theta):
    g = Grid(shape[2], shape[1], shape[0], h=1.0 / shape[2])
    prm = Params(alpha=0.1, dt=5e-3, theta=theta, shift=0.5)
    rng = np.random.default_rng(11)
    m = rng.standard_normal((3,) + g.shape)
    m /= np.sqrt(nodal.dot(m, m))
    b = rng.standard_normal((4,) + g.shape)
    xs = dense.solve(g, prm, m, b)
    x, info = steppers.solve_saddle(g, prm, m, b, rtol=1e-14, restart=30)
    assert info["converged"]
    assert np.linalg.norm(x - xs) <= 1e-12 * np.linalg.norm(xs)


@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_uniform_state_closed_form(theta):
    """m = m0, h = h0 constant: v = alpha h_T - m0 x h_T, r = (1+alpha^2) m0.h0."""
    g = Grid(8, 8, 4, h=1.0 / 8)
    prm = Params(alpha=0.07, dt=1e-3, theta=theta, shift=0.5, h_uniform=(0.3, -0.2, 0.9))
    m0 = np.array([0.48, -0.6, 0.64])
    m0 = m0 / np.linalg.norm(m0)
    m = np.broadcast_to(m0.reshape(3, 1, 1, 1), (3,) + g.shape).copy()
    b = steppers.rhs(g, prm, m)
    x, info = steppers.solve_saddle(g, prm, m, b, rtol=1e-14)
    h0 = np.array(prm.h_uniform)
    hT = h0 - (m0 @ h0) * m0
    v_ref = prm.alpha * hT - np.cross(m0, hT)
    r_ref = (1 + prm.alpha ** 2) * (m0 @ h0)
    np.testing.assert_allclose(x[:3].reshape(3, -1), np.repeat(v_ref[:, None], g.ng, 1), atol=1e-13)
    np.testing.assert_allclose(x[3], r_ref, atol=1e-13)


def test_even_step_gmres_bound():
    """||r_{2j}|| / ||r_0|| <= kappa vartheta_2^j for unrestarted GMRES
    (unit magnetization, so kappa = 1)."""
    g = Grid(8, 8, 1, lengths=(1.0, 2 * np.pi, 2 * np.pi))
    prm = Params(alpha=0.2, dt=10.24 / 64, theta=1.0, shift=0.5)
    rng = np.random.default_rng(5)
    m = rng.standard_normal((3,) + g.shape)
    m /= np.sqrt(nodal.dot(m, m))
    b = np.zeros((4,) + g.shape)
    b[:3] = rng.standard_normal((3,) + g.shape)
    A = dense.saddle_matrix(g, prm, m)
    M1, M2 = dense.hss_factors(g, prm, m)
    P = np.linalg.solve(M2, np.linalg.solve(M1, A))
    r0 = np.linalg.solve(M2, np.linalg.solve(M1, b.ravel()))
    beta = theory.beta_n(prm.alpha, 1.0, prm.dt, prm.c_hat, g.max_symbol())
    qh = theory.q_bar(0.5, prm.alpha, beta)
    th2 = theory.vartheta2(qh, theory.gamma_m(0.5, 1.0))
    # exact GMRES residuals: min over the Krylov space, via least squares
    K = [r0 / np.linalg.norm(r0)]
    for j in range(1, 2 * 8 + 1):
        w = P @ K[-1]
        for q in K:
            w -= (q @ w) * q
        for q in K:
            w -= (q @ w) * q
        K.append(w / np.linalg.norm(w))
    Q = np.array(K).T
    for jj in range(1, 9):
        Qk = Q[:, :2 * jj]
        PQ = P @ Qk
        y, *_ = np.linalg.lstsq(PQ, r0, rcond=None)
        res = np.linalg.norm(r0 - PQ @ y) / np.linalg.norm(r0)
        assert res <= th2 ** jj * (1 + 1e-10)


def _smooth_system(n):
    g = Grid(n, n, 1, lengths=(1.0, 2 * np.pi, 2 * np.pi))
    prm = Params(alpha=0.2, dt=1e-2, theta=1.0, shift=0.5)
    m, _ = manufactured.grid_fields(g, 0.0, prm.alpha)
    _, F = manufactured.grid_fields(g, prm.dt, prm.alpha)
    return g, prm, m, steppers.rhs(g, prm, m, forcing=F)


@pytest.mark.parametrize("n", [32, 256])
def test_smooth_rhs_iteration_counts_match_paper(n):
    """Sec. 4.3: the smooth one-step Euler system, GMRES(50), rtol 1e-8.  The
    printed counts (split 11, symmetric part 18, unpreconditioned 22 at N = 32
    and 175 at N = 256) are reproduced exactly by this GMRES."""
    gold = GOLD["smooth_rhs_iterations"]
    g, prm, m, b = _smooth_system(n)
    A = lambda x: operators.matvec(g, prm, m, x)
    counts = {}
    for name, M in [("split", lambda x: operators.hss_apply(g, prm, m, x)),
                    ("symmetric", lambda x: operators.symmetric_apply(g, prm, x)),
                    ("none", lambda x: x)]:
        x, info = gmres.gmres(A, M, b, restart=50, rtol=1e-8, maxiter=3000)
        assert info["converged"]
        counts[name] = info["iters"]
    assert counts["split"] == gold["split_2d"]
    assert counts["symmetric"] == gold["symmetric_2d"]
    assert counts["none"] == gold["unpreconditioned_2d"][str(n)]


def test_smooth_rhs_iteration_counts_3d_match_paper():
    """Sec. 4.3 in 3D on (0, 2 pi)^3 with the 3D manufactured family
    (oracle.manufactured): split 13, symmetric part 26 and, at N = 16,
    unpreconditioned 24 iterations, as printed."""
    gold = GOLD["smooth_rhs_iterations"]
    for n in (16, 24):
        g = Grid(n, n, n, lengths=(2 * np.pi,) * 3)
        prm = Params(alpha=0.2, dt=1e-2, theta=1.0, shift=0.5)
        m, _ = manufactured.grid_fields(g, 0.0, prm.alpha)
        _, F = manufactured.grid_fields(g, prm.dt, prm.alpha)
        b = steppers.rhs(g, prm, m, forcing=F)
        A = lambda x: operators.matvec(g, prm, m, x)
        counts = {}
        for name, M in [("split", lambda x: operators.hss_apply(g, prm, m, x)),
                        ("symmetric", lambda x: operators.symmetric_apply(g, prm, x)),
                        ("none", lambda x: x)]:
            x, info = gmres.gmres(A, M, b, restart=50, rtol=1e-8, maxiter=3000)
            assert info["converged"]
            counts[name] = info["iters"]
        assert counts["split"] == gold["split_3d"]
        assert counts["symmetric"] == gold["symmetric_3d"]
        if n == 16:
            assert counts["none"] == gold["unpreconditioned_3d"]["16"]


def test_manufactured_3d_derivatives():
    """The analytic d_t m and Delta m of the 3D manufactured family against a
    central difference in t and the spectral Laplacian (exact for these modes)."""
    g = Grid(12, 12, 12, lengths=(2 * np.pi,) * 3)
    zz, yy, xx = g.coords()
    t, e = 0.3, 1e-6
    m = manufactured.m_exact_3d(xx, yy, zz, t)
    np.testing.assert_allclose(nodal.dot(m, m), 1.0, atol=1e-15)
    fd = (manufactured.m_exact_3d(xx, yy, zz, t + e) - manufactured.m_exact_3d(xx, yy, zz, t - e)) / (2 * e)
    np.testing.assert_allclose(manufactured.dt_m_exact_3d(xx, yy, zz, t), fd, atol=1e-8)
    np.testing.assert_allclose(manufactured.lap_m_exact_3d(xx, yy, zz, t), -fourier.neg_laplacian(g, m),
                               atol=1e-13)


def _split_count(g, prm, m, b):
    x, info = gmres.gmres(lambda x: operators.matvec(g, prm, m, x),
                          lambda x: operators.hss_apply(g, prm, m, x), b, restart=50, rtol=1e-8, maxiter=5000)
    assert info["converged"]
    return info["iters"]


def test_lambda_sweep_matches_paper():
    """Sec. 4.4: the shift sweep 2^-3..2^4 on the smooth system.  The minimum
    (10 iterations at lambda = 0.25), the 10..12 band on [0.25, 1] and the
    N = 256 count at lambda = 16 (42) are reproduced exactly; the N = 64 count
    at lambda = 16 is a soft pin (27 here, 32 printed)."""
    gold = GOLD["lambda_sweep"]
    counts = {}
    for n, lams in [(64, [2.0 ** e for e in range(-3, 5)]), (256, [0.25, 16.0])]:
        g = Grid(n, n, 1, lengths=(1.0, 2 * np.pi, 2 * np.pi))
        for lam in lams:
            prm = Params(alpha=0.2, dt=1e-2, theta=1.0, shift=lam)
            m, _ = manufactured.grid_fields(g, 0.0, prm.alpha)
            _, F = manufactured.grid_fields(g, prm.dt, prm.alpha)
            counts[(n, lam)] = _split_count(g, prm, m, steppers.rhs(g, prm, m, forcing=F))
    sweep64 = {lam: c for (n, lam), c in counts.items() if n == 64}
    assert min(sweep64.values()) == gold["min_iters"]
    assert min(sweep64, key=sweep64.get) == gold["argmin"]
    for lam in gold["band_lambdas"]:
        assert gold["band"][0] <= sweep64[lam] <= gold["band"][1]
    # counts grow once lambda leaves the band
    tail = [sweep64[2.0 ** e] for e in range(0, 5)]
    assert tail == sorted(tail)
    assert counts[(256, 0.25)] == gold["min_iters"]
    assert counts[(256, 16.0)] == gold["lambda16"]["256"]
    assert abs(sweep64[16.0] - gold["lambda16"]["64"]) <= 6


def test_random_rhs_mesh_dependence():
    """Sec. 4.5: Gaussian velocity right-hand sides.  The seeds are the
    paper's but its generator is unstated, so the counts are soft pins
    (within 6 %): bounded stiffness k N^2 = 10.24 keeps the count flat near
    55, fixed k = 1e-2 makes it grow with N (checked up to N = 64 here; the
    N = 256 value 608 is checked on the GPU)."""
    gold = GOLD["random_rhs"]
    tol = gold["soft_rel"]
    med = {}
    for regime, n in [("fixed", 32), ("fixed", 64), ("bounded", 64), ("bounded", 128)]:
        g = Grid(n, n, 1, lengths=(1.0, 2 * np.pi, 2 * np.pi))
        k = 1e-2 if regime == "fixed" else 10.24 / n ** 2
        prm = Params(alpha=0.2, dt=k, theta=1.0, shift=0.5)
        m, _ = manufactured.grid_fields(g, 0.0, prm.alpha)
        c = sorted(_split_count(g, prm, m, llg_workloads.gaussian_rhs(n, s)) for s in gold["seeds"])
        med[(regime, n)] = c[1]
    lo, hi = gold["bounded_range"]
    for n in (64, 128):
        assert lo * (1 - tol) <= med[("bounded", n)] <= hi * (1 + tol)
    assert abs(med[("fixed", 32)] - gold["fixed_k"]["32"]) <= tol * gold["fixed_k"]["32"]
    assert med[("fixed", 64)] >= 1.8 * med[("fixed", 32)]


def test_fgmres_ir_matches_gmres():
    g = Grid(16, 16, 1, h=1.0 / 16)
    prm = Params(alpha=0.05, dt=10 / 256, theta=0.5, shift=0.5)
    rng = np.random.default_rng(9)
    m = rng.standard_normal((3,) + g.shape)
    m /= np.sqrt(nodal.dot(m, m))
    b = steppers.rhs(g, prm, m)
    A = lambda x: operators.matvec(g, prm, m, x)
    M = lambda x: operators.hss_apply(g, prm, m, x)
    x1, i1 = gmres.gmres(A, M, b, rtol=1e-12)
    x2, i2 = gmres.fgmres_ir(A, M, b, rtol=1e-12, inner_rtol=1e-4)
    assert i1["converged"] and i2["converged"] and i2["outer_steps"] >= 2
    assert np.linalg.norm(x2 - x1) <= 1e-10 * np.linalg.norm(x1)
