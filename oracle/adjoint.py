"""Adjoint of the converged midpoint step.

Test infrastructure: part of the float64 CPU oracle (see the package docstring).

Write u = (v, r) and m_half = m^n + (k/2) v.  The converged step solves the
residual of eq. "C-N" (Sec. 3.3) with the lower-order field h:

    R_v = alpha v + m_half x v + C_hat (-Delta_N) m_half + m_half r
          - (1+alpha^2) (L_low m_half + h)
    R_r = -m_half . v

(L_low: the linear, symmetric part of the lower-order field, oracle.fields)
and sets m^{n+1} = m^n + k v.  Differentiating (m_half x v = m^n x v), with
K_low = (k/2)(1 + alpha^2) L_low:

    J = dR/du = [[alpha I + [m^n]_x + (k/2) C_hat (-Delta_N) + (k/2) r I - K_low, m_half],
                 [-(m_half + (k/2) v)^T,                                           0     ]].

For a loss L(m^{n+1}) with gbar = dL/dm^{n+1}, let mu = J^{-T} (k gbar, 0).  Then
dL/dh = (1 + alpha^2) mu_v and

    dL/dm^n = gbar - [v x mu_v + C_hat (-Delta_N) mu_v + r mu_v - v mu_r
                      - (1 + alpha^2) L_low mu_v].

The transposed solve is preconditioned with the transposed split FFT-HSS
operator built on m_half, M^{-T} = (calH + lambda I)^{-1} (calS(m_half) +
lambda I)^{-T}: on the left (GMRES on M^{-T} J^T), or on the right (GMRES on
J^T M^{-T}, mu = M^{-T} y).  Without a lower-order field J^T = calH + N with
N nodal (J^T's velocity block differs from H = alpha I + (k/2) C_hat (-Delta_N)
only by node-wise terms), so

    J^T M^{-T} = [I + (N - lambda I) (calH + lambda I)^{-1}] (calS + lambda I)^{-T},

one nodal solve, one Fourier solve and one nodal combination: nodal_part
gives N.
"""

from dataclasses import replace

import numpy as np

from . import dense as dense_mod
from . import fields, fourier, nodal, operators
from .gmres import gmres, gmres_right


def jacobian_transpose_apply(g, prm, m_n, v, r, mu):
    """J^T mu for the midpoint residual (theta = 1/2)."""
    k = prm.dt
    m_half = m_n + 0.5 * k * v
    m_next = m_n + k * v
    mv, mr = mu[:3], mu[3]
    out = np.empty_like(mu)
    out[:3] = (fourier.h_apply(g, mv, prm.alpha, 0.5 * k * prm.c_hat)
               - nodal.cross(m_n, mv) + 0.5 * k * r * mv - m_next * mr
               - 0.5 * k * (1.0 + prm.alpha ** 2) * fields.low_linear(g, prm, mv))
    out[3] = nodal.dot(m_half, mv)
    return out


def jacobian_apply(g, prm, m_n, v, r, du):
    """J du (used to check the transpose)."""
    k = prm.dt
    m_half = m_n + 0.5 * k * v
    dv, dr = du[:3], du[3]
    out = np.empty_like(du)
    out[:3] = (fourier.h_apply(g, dv, prm.alpha, 0.5 * k * prm.c_hat)
               + nodal.cross(m_n, dv) + 0.5 * k * r * dv + m_half * dr
               - 0.5 * k * (1.0 + prm.alpha ** 2) * fields.low_linear(g, prm, dv))
    out[3] = -nodal.dot(m_half + 0.5 * k * v, dv)
    return out


def nodal_part(prm, m_n, v, r, mu):
    """N mu = J^T mu - calH mu (no lower-order field): node-wise
    (-m^n x mu_v + (k/2) r mu_v - m^{n+1} mu_r, m_half . mu_v)."""
    k = prm.dt
    m_half = m_n + 0.5 * k * v
    m_next = m_n + k * v
    mv, mr = mu[:3], mu[3]
    out = np.empty_like(mu)
    out[:3] = -nodal.cross(m_n, mv) + 0.5 * k * r * mv - m_next * mr
    out[3] = nodal.dot(m_half, mv)
    return out


def step_adjoint(g, prm, m_n, v, r, gbar, rtol=1e-12, restart=30, dense=False, side="left"):
    """Back-propagate gbar = dL/dm^{n+1} through one converged midpoint step.
    side: "left" (GMRES on M^{-T} J^T) or "right" (GMRES on J^T M^{-T}).

    Returns (gbar_n, hbar_field, hbar_uniform, mu, info)."""
    prm2 = replace(prm, theta=0.5)
    k = prm.dt
    rhs = np.zeros((4,) + g.shape)
    rhs[:3] = k * gbar
    if dense:
        J = dense_mod.midpoint_jacobian(g, prm2, m_n, v, r)
        mu = np.linalg.solve(J.T, rhs.ravel()).reshape(rhs.shape)
        info = dict(iters=0, converged=True)
    else:
        m_half = m_n + 0.5 * k * v
        solver = gmres if side == "left" else gmres_right
        mu, info = solver(lambda x: jacobian_transpose_apply(g, prm2, m_n, v, r, x),
                          lambda x: operators.hss_apply(g, prm2, m_half, x, transpose=True),
                          rhs, restart=restart, rtol=rtol)
    muv, mur = mu[:3], mu[3]
    hbar_field = (1.0 + prm.alpha ** 2) * muv
    hbar_uniform = hbar_field.reshape(3, -1).sum(axis=1)
    gbar_n = gbar - (nodal.cross(v, muv) + prm.c_hat * fourier.neg_laplacian(g, muv)
                     + r * muv - v * mur - (1.0 + prm.alpha ** 2) * fields.low_linear(g, prm, muv))
    return gbar_n, hbar_field, hbar_uniform, mu, info
