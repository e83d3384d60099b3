"""Pins of the closed-form bounds against the numbers printed in Sec. 4.3 and
Sec. 4.4."""

import json
import os

import numpy as np
import pytest

from oracle import theory
from oracle.grid import Grid

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_printed_values.json")))
C_HAT = 1.0 + 0.2 ** 2


def test_bounded_stiffness_numbers():
    gold = GOLD["bounded_stiffness"]
    for n in (32, 64, 128, 256):
        g = Grid(n, n, 1, lengths=(1.0, 2 * np.pi, 2 * np.pi))
        k = gold["k_times_N2"] / n ** 2
        beta = theory.beta_n(0.2, 1.0, k, C_HAT, g.max_symbol())
        assert beta == pytest.approx(gold["h_max"], abs=5e-5)
        qh = theory.q_bar(0.5, 0.2, beta)
        assert qh == pytest.approx(gold["q_H"], abs=5e-5)
        th = theory.vartheta2(qh, theory.gamma_m(0.5, 1.0))
        assert th == pytest.approx(gold["vartheta2"], abs=5e-5)
        assert theory.explicit_limit_ratio(k, C_HAT, g.max_symbol(), 0.2) == pytest.approx(gold["explicit_limit_ratio"], abs=5e-3)
        assert k * C_HAT * g.max_symbol() == pytest.approx(gold["k_Chat_max_symbol"], abs=5e-5)
        assert beta / 0.2 == pytest.approx(gold["condition_number"], abs=0.05)


def test_fixed_k_vartheta2_and_lambda_bd():
    gold = GOLD["fixed_k_vartheta2"]
    g = Grid(gold["N"], gold["N"], 1, lengths=(1.0, 2 * np.pi, 2 * np.pi))
    beta = theory.beta_n(0.2, 1.0, gold["dt"], C_HAT, g.max_symbol())
    th = theory.vartheta2(theory.q_bar(0.5, 0.2, beta), theory.gamma_m(0.5, 1.0))
    assert th == pytest.approx(gold["vartheta2"], abs=5e-5)
    lb = GOLD["lambda_bd"]
    for n, ref in zip(lb["N"], lb["lambda_bd"]):
        g = Grid(n, n, 1, lengths=(1.0, 2 * np.pi, 2 * np.pi))
        beta = theory.beta_n(0.2, 1.0, 1e-2, C_HAT, g.max_symbol())
        assert theory.lambda_bd(0.2, beta) == pytest.approx(ref, abs=5e-3)


def test_kappa_is_the_condition_number_of_the_nodal_factor():
    """kappa_lambda of the full-saddle contraction theorem: the singular values of
    lambda I + calS lie between sqrt(lambda^2 + m_-^2) and sqrt(lambda^2 +
    m_+^2) (nodal norms in [m_-, m_+]), so kappa_lambda is its 2-norm
    condition number.  Checked against the SVD of the dense assembled
    factor for magnetizations of non-unit length."""
    from oracle import dense, nodal
    from oracle.operators import Params
    g = Grid(4, 4, 1, h=0.25)
    rng = np.random.default_rng(3)
    m = rng.standard_normal((3,) + g.shape)
    m /= np.sqrt(nodal.dot(m, m))
    m *= rng.uniform(0.4, 1.9, size=g.shape)[None]
    norms = np.sqrt(nodal.dot(m, m))
    for lam in (0.25, 0.5, 2.0):
        prm = Params(alpha=0.2, dt=1e-2, shift=lam)
        _, M2 = dense.hss_factors(g, prm, m)
        sv = np.linalg.svd(M2, compute_uv=False)
        assert sv.min() == pytest.approx(np.sqrt(lam ** 2 + norms.min() ** 2), rel=1e-12)
        assert sv.max() == pytest.approx(np.sqrt(lam ** 2 + norms.max() ** 2), rel=1e-12)
        assert theory.kappa(lam, norms.min(), norms.max()) == pytest.approx(sv.max() / sv.min(), rel=1e-12)
    # unit magnetization: kappa = 1 and gamma_m = 2 lambda / (lambda^2 + 1) (the theorem's special case)
    assert theory.kappa(0.5, 1.0, 1.0) == 1.0
    assert theory.gamma_m(0.5, 1.0) == pytest.approx(2 * 0.5 / (0.5 ** 2 + 1))


@pytest.mark.parametrize("kap,th,eps", [(1.0, 0.9574, 1e-8), (1.7, 0.9993, 1e-10), (3.2, 0.5, 1e-3),
                                        (1.0, 0.8, 0.5)])
def test_iteration_bound_is_the_first_even_count_meeting_the_bound(kap, th, eps):
    """2 ceil(log(kappa/eps) / log(1/vartheta)) of the uniform iteration bound
    is the smallest 2j with kappa vartheta^j <= eps: brute force over j."""
    j = 0
    while kap * th ** j > eps:
        j += 1
    assert theory.iteration_bound(kap, th, eps) == 2 * j


def test_iteration_bound_holds_for_exact_gmres():
    """Unrestarted left-preconditioned GMRES on a dense saddle system with
    non-unit nodal lengths reaches ||r_2j|| / ||r_0|| <= eps within
    iteration_bound(kappa_lambda, vartheta_2, eps) iterations."""
    from oracle import dense, nodal
    from oracle.operators import Params
    g = Grid(8, 8, 1, lengths=(1.0, 2 * np.pi, 2 * np.pi))
    prm = Params(alpha=0.2, dt=10.24 / 64, theta=1.0, shift=0.5)
    rng = np.random.default_rng(7)
    m = rng.standard_normal((3,) + g.shape)
    m /= np.sqrt(nodal.dot(m, m))
    m *= rng.uniform(0.8, 1.25, size=g.shape)[None]
    norms = np.sqrt(nodal.dot(m, m))
    b = rng.standard_normal(4 * g.ng)
    A = dense.saddle_matrix(g, prm, m)
    M1, M2 = dense.hss_factors(g, prm, m)
    P = np.linalg.solve(M2, np.linalg.solve(M1, A))
    r0 = np.linalg.solve(M2, np.linalg.solve(M1, b))
    beta = theory.beta_n(prm.alpha, 1.0, prm.dt, prm.c_hat, g.max_symbol())
    qh = theory.q_bar(prm.shift, prm.alpha, beta)
    th2 = theory.vartheta2(qh, theory.gamma_m(prm.shift, norms.min(), norms.max()))
    kap = theory.kappa(prm.shift, norms.min(), norms.max())
    eps = 1e-6
    bound = theory.iteration_bound(kap, th2, eps)
    # exact GMRES residual after j steps: least squares over the Krylov space
    K = [r0 / np.linalg.norm(r0)]
    need = None
    for j in range(1, bound + 1):
        w = P @ K[-1]
        for _ in range(2):
            for q in K:
                w -= (q @ w) * q
        K.append(w / np.linalg.norm(w))
        PQ = P @ np.array(K[:j]).T
        y, *_ = np.linalg.lstsq(PQ, r0, rcond=None)
        if np.linalg.norm(r0 - PQ @ y) <= eps * np.linalg.norm(r0):
            need = j
            break
    assert need is not None and need <= bound
