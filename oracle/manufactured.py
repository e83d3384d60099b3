"""Manufactured solution of the temporal-convergence test (Sec. 4.2).

Test infrastructure: part of the float64 CPU oracle (see the package docstring).

On (0, 2 pi)^2, m_e(x, t) = (sin(t+x) cos(t+y), cos(t+x) cos(t+y), sin(t+y)),
a unit periodic field.  The forcing is obtained by substituting m_e, d_t m_e
and Delta m_e into the tangent-plane equation
    alpha d_t m + m x d_t m = (1+alpha^2) [h_eff - (m . h_eff) m],
h_eff = cexc Delta m + h_low; it enters the scheme as F = (1+alpha^2) h_low:
    F = alpha d_t m_e + m_e x d_t m_e - (1+alpha^2) cexc [Delta m_e - (m_e . Delta m_e) m_e].
(Any component along m_e is absorbed by the multiplier.)  Derivatives are
written out analytically here.

Reading: the forcing that reproduces the printed errors of Sec. 4.2 to every
printed digit is the unprojected one, F = alpha d_t m_e + m_e x d_t m_e -
(1+alpha^2) cexc Delta m_e (``project=False``, the default); the projected
variant keeps the orders but changes the error constants.

Three dimensions (reading; the paper names no 3D field for its 3D
preconditioner comparison, Sec. 4.3): on (0, 2 pi)^3 the same family with
a = t + x + z, b = t + y + z, i.e. m_e = (sin a cos b, cos a cos b, sin b),
whose t = 0 value is the initial field of the 3D energy test (Sec. 4.6).
With it the comparison counts printed for N = 16..48 are reproduced exactly.
With u_a, u_b the partial derivatives in a and b:
    d_t m = m_a + m_b,  Delta m = 2 m_aa + 2 m_bb + 2 m_ab,
    m_a = (cos a cos b, -sin a cos b, 0),  m_b = (-sin a sin b, -cos a sin b, cos b),
    m_aa = -(m_1, m_2, 0),  m_bb = -m,  m_ab = (-cos a sin b, sin a sin b, 0).
"""

import numpy as np

from . import nodal


def m_exact(x, y, t):
    a, b = t + x, t + y
    return np.stack([np.sin(a) * np.cos(b), np.cos(a) * np.cos(b), np.sin(b)])


def dt_m_exact(x, y, t):
    a, b = t + x, t + y
    return np.stack([np.cos(a) * np.cos(b) - np.sin(a) * np.sin(b),
                     -np.sin(a) * np.cos(b) - np.cos(a) * np.sin(b),
                     np.cos(b)])


def lap_m_exact(x, y, t):
    m = m_exact(x, y, t)
    return np.stack([-2.0 * m[0], -2.0 * m[1], -m[2]])


def forcing(x, y, t, alpha, cexc=1.0, project=False):
    m = m_exact(x, y, t)
    mt = dt_m_exact(x, y, t)
    lap = lap_m_exact(x, y, t)
    if project:
        lap = lap - nodal.dot(m, lap) * m
    return alpha * mt + nodal.cross(m, mt) - (1.0 + alpha ** 2) * cexc * lap


def _ab3(x, y, z, t):
    return t + x + z, t + y + z


def m_exact_3d(x, y, z, t):
    a, b = _ab3(x, y, z, t)
    return np.stack([np.sin(a) * np.cos(b), np.cos(a) * np.cos(b), np.sin(b)])


def dt_m_exact_3d(x, y, z, t):
    a, b = _ab3(x, y, z, t)
    ma = np.stack([np.cos(a) * np.cos(b), -np.sin(a) * np.cos(b), np.zeros_like(a)])
    mb = np.stack([-np.sin(a) * np.sin(b), -np.cos(a) * np.sin(b), np.cos(b)])
    return ma + mb


def lap_m_exact_3d(x, y, z, t):
    a, b = _ab3(x, y, z, t)
    m = m_exact_3d(x, y, z, t)
    maa = np.stack([-m[0], -m[1], np.zeros_like(a)])
    mab = np.stack([-np.cos(a) * np.sin(b), np.sin(a) * np.sin(b), np.zeros_like(a)])
    return 2.0 * maa - 2.0 * m + 2.0 * mab


def forcing_3d(x, y, z, t, alpha, cexc=1.0, project=False):
    m = m_exact_3d(x, y, z, t)
    mt = dt_m_exact_3d(x, y, z, t)
    lap = lap_m_exact_3d(x, y, z, t)
    if project:
        lap = lap - nodal.dot(m, lap) * m
    return alpha * mt + nodal.cross(m, mt) - (1.0 + alpha ** 2) * cexc * lap


def grid_fields(g, t, alpha, cexc=1.0, project=False):
    """(m_e, F) sampled on the grid, shaped (3, nz, ny, nx): the 2D field when
    nz = 1, the 3D family otherwise."""
    zz, yy, xx = g.coords()
    if g.dim == 2:
        return (m_exact(xx, yy, t), forcing(xx, yy, t, alpha, cexc, project))
    return (m_exact_3d(xx, yy, zz, t), forcing_3d(xx, yy, zz, t, alpha, cexc, project))


def run(g, alpha, dt, t_end, scheme, shift=0.5, restart=50, rtol=1e-10, picard_tol=1e-10,
        project=False, cexc=1.0):
    """Integrate the manufactured problem to t_end; return (error, info).

    error = mean over the three components of the nodal max-norm error at
    t_end (Sec. 4.2).  Euler samples the forcing at t_{n+1}, midpoint at
    t_{n+1/2}."""
    from .operators import Params
    from . import steppers
    prm = Params(alpha=alpha, cexc=cexc, dt=dt, shift=shift)
    nsteps = int(round(t_end / dt))
    m, _ = grid_fields(g, 0.0, alpha, cexc, project)
    v = lam = None
    max_lin = 0.0
    max_len = 0.0
    for n in range(nsteps):
        if scheme == "euler":
            _, F = grid_fields(g, (n + 1) * dt, alpha, cexc, project)
            m, v, lam, info = steppers.euler_step(g, prm, m, forcing=F, restart=restart, rtol=rtol)
            max_lin = max(max_lin, info["rel_res_true"])
        else:
            _, F = grid_fields(g, (n + 0.5) * dt, alpha, cexc, project)
            m, v, lam, info = steppers.midpoint_step(g, prm, m, v, lam, forcing=F, restart=restart,
                                                     rtol=rtol, picard_tol=picard_tol)
            max_len = max(max_len, float(np.max(np.abs(np.sqrt(nodal.dot(m, m)) - 1.0))))
    me, _ = grid_fields(g, nsteps * dt, alpha, cexc, project)
    err = float(np.mean(np.max(np.abs(m - me).reshape(3, -1), axis=1)))
    return err, dict(max_len_err=max_len, max_lin_res=max_lin)

