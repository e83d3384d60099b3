"""Pins of the time steppers: the paper's printed temporal errors and orders
(Sec. 4.2), exact nodal length of the converged midpoint step, the exact
dissipation identity and its inexact-solve correction (Proposition "Nodal
constraint and discrete energy law", Remark "Effect of an inexact midpoint
solve"), and the uniform-state reductions."""

import json
import os

import numpy as np
import pytest

from oracle import manufactured, nodal, steppers
from oracle.grid import Grid
from oracle.operators import Params

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_printed_values.json")))


@pytest.mark.parametrize("scheme,key,order", [("euler", "euler_error", 1), ("midpoint", "midpoint_error", 2)])
def test_temporal_errors_match_paper(scheme, key, order):
    gold = GOLD["temporal_convergence"]
    g = Grid(64, 64, 1, lengths=(1.0, 2 * np.pi, 2 * np.pi))
    errs = []
    for k in (1e-2, 5e-3, 2.5e-3, 1.25e-3):
        e, info = manufactured.run(g, 0.2, k, 0.1, scheme, restart=50)
        errs.append(e)
        if scheme == "midpoint":
            assert info["max_len_err"] < 1e-11
    # printed to four significant digits
    assert errs[0] == pytest.approx(gold[key][0], rel=1e-3)
    assert errs[-1] == pytest.approx(gold[key][1], rel=1e-3)
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(orders - order) < 2e-3), orders


def _random_unit(g, seed):
    rng = np.random.default_rng(seed)
    m = rng.standard_normal((3,) + g.shape)
    # smooth it a little so the Picard iteration converges at moderate k
    mh = np.fft.fftn(m, axes=(-3, -2, -1)) * np.exp(-0.5 * g.s / g.s.max() * 40)
    m = np.fft.ifftn(mh, axes=(-3, -2, -1)).real
    return m / np.sqrt(nodal.dot(m, m))


def test_midpoint_length_and_energy_law():
    g = Grid(16, 16, 1, h=1.0 / 16)
    prm = Params(alpha=0.1, dt=5e-4, shift=0.5, h_uniform=(0.0, 0.0, 0.5))
    m = _random_unit(g, 1)
    v = lam = None
    for _ in range(3):
        m_new, v, lam, info = steppers.midpoint_step(g, prm, m, v, lam, rtol=1e-14, picard_tol=1e-12)
        assert info["converged"]
        d = steppers.midpoint_diagnostics(g, prm, m, m_new, v, lam)
        assert d["max_len_err"] < 1e-12
        assert d["energy_after"] < d["energy_before"]
        # exact law: g(m^{n+1}) - g(m^n) = -alpha k/(1+alpha^2) ||v||_N^2
        assert abs(d["dissipation_defect"]) < 1e-10 * abs(d["energy_after"] - d["energy_before"])
        m = m_new


@pytest.mark.parametrize("rtol", [1e-3, 1e-6, 1e-12])
def test_inexact_correction_identity(rtol):
    """defect == k/(1+alpha^2)[rho(v) - chi(r)] for any (v, r), however
    loosely the saddle system was solved."""
    g = Grid(16, 8, 1, h=1.0 / 16)
    prm = Params(alpha=0.2, dt=5e-3, shift=0.5, h_uniform=(0.1, 0.0, 0.7))
    m = _random_unit(g, 2)
    m_new, v, lam, info = steppers.midpoint_step(g, prm, m, rtol=rtol, picard_tol=1e-12, picard_max=3)
    d = steppers.midpoint_diagnostics(g, prm, m, m_new, v, lam)
    scale = abs(d["energy_before"]) + prm.alpha * prm.dt * d["v_norm2"]
    assert abs(d["dissipation_defect"] - d["inexact_correction"]) <= 1e-14 * scale
    # length defect = 2 k chi: |m^{n+1}|^2 - |m^n|^2 = 2k m_half . v
    lhs = nodal.dot(m_new, m_new) - nodal.dot(m, m)
    rhs = 2 * prm.dt * nodal.dot(0.5 * (m + m_new), v)
    np.testing.assert_allclose(lhs, rhs, atol=1e-15)


def test_uniform_state_midpoint_reduction():
    """Constant m0 and h0: the midpoint step reduces to 4 scalar equations
    alpha v + m_half x v + m_half r = (1+alpha^2) h0, m_half . v = 0 with
    m_half = m0 + (k/2) v; solved here by Newton's method."""
    g = Grid(4, 4, 4, h=0.25)
    prm = Params(alpha=0.3, dt=0.05, shift=0.5, h_uniform=(0.5, 0.2, -0.1))
    m0 = np.array([0.0, 0.6, 0.8])
    m = np.broadcast_to(m0.reshape(3, 1, 1, 1), (3,) + g.shape).copy()
    m_new, v, lam, info = steppers.midpoint_step(g, prm, m, rtol=1e-15, picard_tol=1e-15, picard_max=80)
    h0 = np.array(prm.h_uniform)
    a, k = prm.alpha, prm.dt

    def F(u):
        vv, rr = u[:3], u[3]
        mh = m0 + 0.5 * k * vv
        return np.concatenate([a * vv + np.cross(mh, vv) + mh * rr - (1 + a * a) * h0, [mh @ vv]])

    u = np.zeros(4)
    for _ in range(50):
        Jm = np.zeros((4, 4))
        for i in range(4):
            e = np.zeros(4)
            e[i] = 1e-7
            Jm[:, i] = (F(u + e) - F(u - e)) / 2e-7
        u = u - np.linalg.solve(Jm, F(u))
    assert np.abs(F(u)).max() < 1e-15
    np.testing.assert_allclose(v.reshape(3, -1), np.repeat(u[:3, None], g.ng, 1), atol=1e-12)
    np.testing.assert_allclose(lam, u[3], atol=1e-12)


def test_euler_uniform_state_step():
    g = Grid(8, 4, 1, h=0.125)
    prm = Params(alpha=0.1, dt=0.02, shift=0.5, h_uniform=(0.0, 1.0, 0.0))
    m0 = np.array([1.0, 0.0, 0.0])
    m = np.broadcast_to(m0.reshape(3, 1, 1, 1), (3,) + g.shape).copy()
    m_new, v, lam, info = steppers.euler_step(g, prm, m, rtol=1e-14)
    h0 = np.array(prm.h_uniform)
    hT = h0 - (m0 @ h0) * m0
    vr = prm.alpha * hT - np.cross(m0, hT)
    mr = (m0 + prm.dt * vr) / np.linalg.norm(m0 + prm.dt * vr)
    np.testing.assert_allclose(m_new.reshape(3, -1), np.repeat(mr[:, None], g.ng, 1), atol=1e-13)
