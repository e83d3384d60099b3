"""Pins of the nodal algebra against the printed matrices of eqs. (S),
(Lambda) and "inverse S" and the identities printed beside them (Sec. 3.2)."""

import numpy as np
import pytest

from oracle import nodal


@pytest.mark.parametrize("seed", range(5))
def test_inverse_s_printed_matrix_is_inverse(seed):
    rng = np.random.default_rng(seed)
    mi = rng.standard_normal(3) * rng.uniform(0.2, 3.0)
    lam = rng.uniform(0.05, 5.0)
    St = nodal.s_tilde(mi)
    inv = nodal.inverse_s_matrix(mi, lam)
    np.testing.assert_allclose(inv @ (St + lam * np.eye(4)), np.eye(4), atol=1e-14 * (1 + np.abs(mi).max() / lam))
    np.testing.assert_allclose(inv, np.linalg.inv(St + lam * np.eye(4)), atol=1e-14 * max(1.0, 1 / lam))


@pytest.mark.parametrize("seed", range(5))
def test_s_tilde_identities(seed):
    rng = np.random.default_rng(10 + seed)
    mi = rng.standard_normal(3)
    lam = rng.uniform(0.1, 2.0)
    St = nodal.s_tilde(mi)
    n2 = float(mi @ mi)
    np.testing.assert_allclose(St.T, -St)
    np.testing.assert_allclose(St @ St, -n2 * np.eye(4), atol=1e-14 * n2)
    Q = lam * np.eye(4) + St
    np.testing.assert_allclose(Q.T @ Q, (lam * lam + n2) * np.eye(4), atol=1e-13 * (lam * lam + n2))
    np.testing.assert_allclose(np.linalg.inv(Q), (lam * np.eye(4) - St) / (lam * lam + n2), atol=1e-14)


def test_lambda_is_cross_product():
    rng = np.random.default_rng(2)
    mi, v = rng.standard_normal(3), rng.standard_normal(3)
    np.testing.assert_allclose(nodal.lambda_matrix(mi) @ v, np.cross(mi, v), atol=1e-15)
    m = rng.standard_normal((3, 2, 3, 4))
    w = rng.standard_normal((3, 2, 3, 4))
    ref = np.moveaxis(np.cross(np.moveaxis(m, 0, -1), np.moveaxis(w, 0, -1)), -1, 0)
    np.testing.assert_allclose(nodal.cross(m, w), ref, atol=1e-14)


def test_vectorized_nodal_solves_match_per_node_inverse():
    rng = np.random.default_rng(4)
    m = rng.standard_normal((3, 1, 3, 5))
    w = rng.standard_normal((4, 1, 3, 5))
    lam = 0.37
    z = nodal.s_shift_solve(m, w, lam)
    zt = nodal.s_shift_solve_transpose(m, w, lam)
    for j in range(3):
        for i in range(5):
            mi = m[:, 0, j, i]
            M = nodal.s_tilde(mi) + lam * np.eye(4)
            np.testing.assert_allclose(z[:, 0, j, i], np.linalg.solve(M, w[:, 0, j, i]), atol=1e-13)
            np.testing.assert_allclose(zt[:, 0, j, i], np.linalg.solve(M.T, w[:, 0, j, i]), atol=1e-13)
    x = rng.standard_normal((4, 1, 3, 5))
    sx = nodal.s_apply(m, x)
    for j in range(3):
        for i in range(5):
            np.testing.assert_allclose(sx[:, 0, j, i], nodal.s_tilde(m[:, 0, j, i]) @ x[:, 0, j, i], atol=1e-14)
