"""Matrix-free saddle operator and the split FFT-HSS preconditioner.

Test infrastructure: part of the float64 CPU oracle (see the package docstring).

* Saddle matrix (Sec. 2.4, eq. "saddle point system", with the (2,1) block
  -B as in the remark that follows it, and Sec. 3.1, eq. (HS)):
      A = [[H + S, B^T], [-B, 0]],  H = alpha I + theta k C_hat (-Delta_N),
      S v = m x v,  B^T r = m r,  -B v = -m . v,
  C_hat = (1 + alpha^2) * cexc, cexc the normalized exchange coefficient.
* Hermitian / skew-Hermitian parts (Sec. 3.1): calH = diag(H, 0),
  calS = [[S, B^T], [-B, 0]].
* Preconditioner (Sec. 3.2): M = (calH + lambda I)(calS + lambda I), applied as
  Algorithm 1 (the FFT solve with calH + lambda I) followed by the nodal solve
  with calS + lambda I (eq. "inverse S").  Its transpose is
  M^{-T} = (calH + lambda I)^{-1} (calS + lambda I)^{-T}.
"""

from dataclasses import dataclass, field

import numpy as np

from . import fourier, nodal


@dataclass
class Params:
    """Physical and solver parameters of one saddle system.

    alpha: damping; cexc: normalized exchange coefficient (1 in the paper's
    runs); dt: time step k; theta: 1 (Euler) or 1/2 (midpoint); shift: the HSS
    shift lambda; h_uniform: uniform applied field; h_field: optional spatial
    applied field of shape (3, nz, ny, nx); demag: coefficient of the
    periodic demagnetizing field (0 off, 1 for the normalized field of the
    magnetostatic problem); aniso_k, aniso_axis: uniaxial anisotropy
    coefficient K and easy axis e (field 2 K e (e.m)).
    """
    alpha: float = 0.2
    cexc: float = 1.0
    dt: float = 1e-2
    theta: float = 1.0
    shift: float = 0.5
    h_uniform: tuple = (0.0, 0.0, 0.0)
    h_field: np.ndarray = field(default=None, repr=False)
    demag: float = 0.0
    aniso_k: float = 0.0
    aniso_axis: tuple = (0.0, 0.0, 1.0)

    @property
    def c_hat(self):
        return (1.0 + self.alpha ** 2) * self.cexc

    @property
    def h_coef(self):
        """Coefficient of -Delta_N in H: theta k C_hat."""
        return self.theta * self.dt * self.c_hat

    def h_ext(self, shape):
        """Applied field on the grid (3, nz, ny, nx)."""
        hu = np.asarray(self.h_uniform, dtype=np.float64).reshape(3, 1, 1, 1)
        out = np.broadcast_to(hu, (3,) + tuple(shape)).copy()
        if self.h_field is not None:
            out += self.h_field
        return out


def matvec(g, prm, m, x):
    """A x for x = (v, r) of shape (4, nz, ny, nx)."""
    v, r = x[:3], x[3]
    y = np.empty_like(x)
    y[:3] = fourier.h_apply(g, v, prm.alpha, prm.h_coef) + nodal.cross(m, v) + m * r
    y[3] = -nodal.dot(m, v)
    return y


def matvec_transpose(g, prm, m, x):
    """A^T x = (H v - m x v - m r, m . v)."""
    v, r = x[:3], x[3]
    y = np.empty_like(x)
    y[:3] = fourier.h_apply(g, v, prm.alpha, prm.h_coef) - nodal.cross(m, v) - m * r
    y[3] = nodal.dot(m, v)
    return y


def m1_solve(g, prm, p):
    """(calH + lambda I)^{-1} p: Algorithm 1."""
    lam = prm.shift
    w = np.empty_like(p)
    w[:3] = fourier.h_solve(g, p[:3], prm.alpha + lam, prm.h_coef)
    w[3] = p[3] / lam
    return w


def m2_solve(m, prm, w):
    """(calS + lambda I)^{-1} w, nodal (eq. "inverse S")."""
    return nodal.s_shift_solve(m, w, prm.shift)


def hss_apply(g, prm, m, p, transpose=False):
    """z = M^{-1} p = (calS + lambda I)^{-1} (calH + lambda I)^{-1} p, or
    M^{-T} p = (calH + lambda I)^{-1} (calS + lambda I)^{-T} p."""
    if transpose:
        return m1_solve(g, prm, nodal.s_shift_solve_transpose(m, p, prm.shift))
    return m2_solve(m, prm, m1_solve(g, prm, p))


def symmetric_apply(g, prm, p):
    """(lambda I + calH)^{-1} p: the symmetric-part comparison preconditioner
    (Sec. 4.1)."""
    return m1_solve(g, prm, p)


def precond_op(g, prm, m, x):
    """M^{-1} A x, computed the plain way (one matvec, then one apply)."""
    return hss_apply(g, prm, m, matvec(g, prm, m, x))
