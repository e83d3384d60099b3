"""Time steppers, right-hand side, energy and midpoint diagnostics.

Test infrastructure: part of the float64 CPU oracle (see the package docstring).

* Projected implicit Euler (Sec. 2.4, eq. "total system 2"; Sec. 3.2, last
  paragraph): solve A(m^n) (v, r) = (f, 0) with theta = 1 and
  f = C_hat Delta_N m^n + (1 + alpha^2) h_low, then m_hat = m^n + k v and
  m^{n+1} = m_hat / |m_hat| node by node.
* Projection-free midpoint scheme (Sec. 3.3, eqs. "C-N" and "hatm"): Picard
  iteration on the frozen midpoint m_hat^p = m^n + (k/2) v^{p-1} (p = 0 uses
  the previous step's velocity, zero on the first step), each iterate one
  saddle solve with theta = 1/2 on the frozen midpoint; after convergence
  m^{n+1} = m^n + k v.
* Discrete energy g_N(m) = (u, v)_N-weighted sum of cexc/2 m.(-Delta_N m)
  plus the lower-order densities (demagnetizing, anisotropy, Zeeman; see
  oracle.fields), a quadratic-affine energy, and the dissipation identity
  with its inexact-solve correction (Proposition "Nodal constraint and
  discrete energy law", Remark "Effect of an inexact midpoint solve").

The lower-order field h_low(m) = L_low m + h_ext (oracle.fields) is explicit
in the Euler step (evaluated at m^n) and frozen at the Picard midpoint m_hat^p
in the midpoint step, so the right-hand side is rebuilt at every Picard
iteration.  A caller may add an explicit forcing F = (1 + alpha^2) h(t)
(manufactured solutions).
"""

from dataclasses import replace

import numpy as np

from . import fields, fourier, nodal, operators
from .gmres import gmres


def rhs(g, prm, m, forcing=None, m_low=None):
    """b = (f, 0) with f = C_hat Delta_N m + (1 + alpha^2) h_low(m_low)
    (+ forcing); m_low defaults to m."""
    b = np.zeros((4,) + g.shape)
    b[:3] = (-prm.c_hat * fourier.neg_laplacian(g, m)
             + (1.0 + prm.alpha ** 2) * fields.h_low(g, prm, m if m_low is None else m_low))
    if forcing is not None:
        b[:3] += forcing
    return b


def solve_saddle(g, prm, m, b, x0=None, restart=30, rtol=1e-10, maxiter=2000, transpose=False):
    """GMRES on A(m) x = b, left-preconditioned by the split FFT-HSS M; with
    transpose, GMRES on A(m)^T x = b left-preconditioned by M^T."""
    if transpose:
        return gmres(lambda x: operators.matvec_transpose(g, prm, m, x),
                     lambda x: operators.hss_apply(g, prm, m, x, transpose=True),
                     b, x0=x0, restart=restart, rtol=rtol, maxiter=maxiter)
    return gmres(lambda x: operators.matvec(g, prm, m, x),
                 lambda x: operators.hss_apply(g, prm, m, x),
                 b, x0=x0, restart=restart, rtol=rtol, maxiter=maxiter)


def euler_step(g, prm, m, forcing=None, restart=30, rtol=1e-10):
    """One projected implicit Euler step (theta = 1).

    Returns (m_new, v, r, info)."""
    prm1 = replace(prm, theta=1.0)
    b = rhs(g, prm1, m, forcing)
    x, info = solve_saddle(g, prm1, m, b, restart=restart, rtol=rtol)
    v = x[:3]
    m_hat = m + prm.dt * v
    m_new = m_hat / np.sqrt(nodal.dot(m_hat, m_hat))
    return m_new, v, x[3], info


def midpoint_step(g, prm, m, v_prev=None, lam_prev=None, forcing=None, restart=30,
                  rtol=1e-10, picard_tol=1e-10, picard_max=50, picard_norm="midpoint"):
    """One projection-free midpoint step (theta = 1/2) with Picard iteration.

    v_prev / lam_prev: velocity and multiplier of the previous step (the p = 0
    frozen midpoint and the GMRES initial guess); None on the first step.
    Convergence (v^{-1} = v_prev):
      picard_norm "midpoint": ||m_hat^{p+1} - m_hat^p||_2 <= picard_tol ||m_hat^{p+1}||_2,
          i.e. (k/2) ||v^p - v^{p-1}|| <= picard_tol ||m^n + (k/2) v^p||, the
          change of the fixed-point iterate of Proposition "Local convergence
          of the midpoint Picard iteration";
      picard_norm "velocity": ||v^p - v^{p-1}||_2 <= picard_tol ||v^p||_2.
    Returns (m_new, v, r, info)."""
    prm2 = replace(prm, theta=0.5)
    k = prm.dt
    b = rhs(g, prm2, m, forcing)
    v_old = np.zeros((3,) + g.shape) if v_prev is None else np.array(v_prev, dtype=np.float64)
    x0 = None
    if v_prev is not None:
        x0 = np.zeros((4,) + g.shape)
        x0[:3] = v_prev
        if lam_prev is not None:
            x0[3] = lam_prev
    info = dict(picard_iters=0, lin_iters=[], converged=False, picard_rel_change=np.inf)
    x = None
    for _ in range(picard_max):
        m_hat = m + 0.5 * k * v_old
        if fields.has_low(prm):
            b = rhs(g, prm2, m, forcing, m_low=m_hat)
        x, linfo = solve_saddle(g, prm2, m_hat, b, x0=x0, restart=restart, rtol=rtol)
        info["picard_iters"] += 1
        info["lin_iters"].append(linfo["iters"])
        v = x[:3]
        if picard_norm == "midpoint":
            change = 0.5 * k * np.linalg.norm(v - v_old)
            ref = np.linalg.norm(m + 0.5 * k * v)
        else:
            change = np.linalg.norm(v - v_old)
            ref = np.linalg.norm(v)
        info["picard_rel_change"] = change / ref if ref > 0 else change
        v_old = v
        x0 = x
        if change <= picard_tol * ref:
            info["converged"] = True
            break
    v = x[:3]
    m_new = m + k * v
    return m_new, v, x[3], info


def energy(g, prm, m):
    """g_N(m) = sum_i w [cexc/2 m_i.(-Delta_N m)_i + lower-order densities],
    w = |Omega|/N_g; the lower-order densities are -1/2 demag m.h_dem[m] +
    K (1 - (e.m)^2) - m.h_ext (oracle.fields)."""
    lap = fourier.neg_laplacian(g, m)
    dens = 0.5 * prm.cexc * nodal.dot(m, lap) + fields.low_energy_density(g, prm, m)
    return g.weight * float(dens.sum())


def midpoint_diagnostics(g, prm, m_old, m_new, v, r):
    """Energy change, dissipation defect and the inexact-solve correction.

    defect     = g_N(m^{n+1}) - g_N(m^n) + alpha k/(1+alpha^2) ||v||_N^2
    correction = k/(1+alpha^2) [rho(v) - chi(r)], where rho and chi are the
    primal and constraint residual functionals of eq. "C-N" at the exact
    midpoint (m^n + m^{n+1})/2, weighted by w = |Omega|/N_g.
    The Remark on inexact solves states defect == correction identically.
    """
    k, a = prm.dt, prm.alpha
    w = g.weight
    mh = 0.5 * (m_old + m_new)
    res_v = (a * v + nodal.cross(mh, v) + prm.c_hat * fourier.neg_laplacian(g, mh)
             + mh * r - (1.0 + a * a) * fields.h_low(g, prm, mh))
    res_c = nodal.dot(v, mh)
    rho_v = w * float(nodal.dot(res_v, v).sum())
    chi_r = w * float((res_c * r).sum())
    e0 = energy(g, prm, m_old)
    e1 = energy(g, prm, m_new)
    vnorm2 = w * float(nodal.dot(v, v).sum())
    defect = e1 - e0 + a * k / (1.0 + a * a) * vnorm2
    correction = k / (1.0 + a * a) * (rho_v - chi_r)
    len_err = float(np.max(np.abs(np.sqrt(nodal.dot(m_new, m_new)) - 1.0)))
    return dict(energy_before=e0, energy_after=e1, dissipation_defect=defect,
                inexact_correction=correction, max_len_err=len_err, v_norm2=vnorm2,
                rho_v=rho_v, chi_r=chi_r)
