"""Lower-order field h_low = h_dem + h_ani + h_ext and its energy.

Test infrastructure: part of the float64 CPU oracle.

* Free energy and effective field (Sec. 2.1, the energy g(m) and eq. "heff"):
  with the normalized coefficients, the anisotropy energy density is
  K (1 - (e.m)^2) and its field 2 K e (e.m); the Zeeman density is -m.h_ext.
* Periodic demagnetizing field (Sec. 2.2, eq. "hdem", periodic cell with the
  zero-mean potential): h_dem = -grad phi with Delta phi = div m.  In Fourier
  variables phi^ = -i (xi~ . m^) / |xi|^2 and h_dem^ = -xi~ (xi~ . m^) / |xi|^2,
  zero at xi = 0.  Its energy density is -1/2 m.h_dem.
* Reading (the paper does not discretize grad and div separately): the first
  derivatives grad and div are spectral with wave vector xi~, equal to xi
  except that the Nyquist component of an even-length axis is set to zero (the
  usual choice for an odd derivative of real data, so h_dem stays real), while
  the Poisson operator is the same -Delta_N as the exchange term (|xi|^2 with
  the Nyquist wave number kept).

The whole lower-order field is affine in m: h_low(m) = L_low m + h_ext, and
L_low = demag * D + 2 K e e^T is symmetric and constant in space, so the
energy is quadratic-affine, the class covered by the discrete energy law of
Sec. 3.3 (Proposition "Nodal constraint and discrete energy law").
"""

import numpy as np

from . import fourier, nodal
from .grid import wavenumbers


def derivative_wavevector(g):
    """(xi~_x, xi~_y, xi~_z), each broadcastable to (nz, ny, nx): physical wave
    numbers with the Nyquist entry of an even-length axis set to zero."""
    def axis(n, length):
        k = wavenumbers(n).astype(np.float64)
        if n % 2 == 0:
            k[n // 2] = 0.0
        return 2.0 * np.pi * k / float(length)

    xx = axis(g.nx, g.lengths[2])[None, None, :]
    xy = axis(g.ny, g.lengths[1])[None, :, None]
    xz = (axis(g.nz, g.lengths[0]) if g.nz > 1 else np.zeros(1))[:, None, None]
    return xx, xy, xz


def demag_field(g, m):
    """Periodic demagnetizing field of m (3, nz, ny, nx), unit coefficient."""
    mh = fourier.fftn(m)
    xi = derivative_wavevector(g)
    s = g.s
    safe = np.where(s > 0, s, 1.0)
    proj = (xi[0] * mh[0] + xi[1] * mh[1] + xi[2] * mh[2]) / safe
    proj = np.where(s > 0, proj, 0.0)
    out = np.empty(m.shape)
    for c in range(3):
        out[c] = -fourier.ifftn(xi[c] * proj).real
    return out


def anisotropy_field(prm, m):
    """2 K e (e.m), uniaxial easy axis e."""
    e = np.asarray(prm.aniso_axis, dtype=np.float64).reshape(3, 1, 1, 1)
    return 2.0 * prm.aniso_k * e * nodal.dot(e, m)


def low_linear(g, prm, u):
    """L_low u = demag * h_dem[u] + 2 K e (e.u): the linear part of h_low."""
    out = anisotropy_field(prm, u)
    if prm.demag != 0.0:
        out = out + prm.demag * demag_field(g, u)
    return out


def h_low(g, prm, m):
    """h_low(m) = L_low m + h_ext (uniform plus optional spatial field)."""
    return low_linear(g, prm, m) + prm.h_ext(g.shape)


def has_low(prm):
    """True when the lower-order field depends on m."""
    return prm.demag != 0.0 or prm.aniso_k != 0.0


def low_energy_density(g, prm, m):
    """Node values of -1/2 demag m.h_dem[m] + K (1 - (e.m)^2) - m.h_ext."""
    e = np.asarray(prm.aniso_axis, dtype=np.float64).reshape(3, 1, 1, 1)
    dens = prm.aniso_k * (1.0 - nodal.dot(e, m) ** 2) - nodal.dot(m, prm.h_ext(g.shape))
    if prm.demag != 0.0:
        dens = dens - 0.5 * prm.demag * nodal.dot(m, demag_field(g, m))
    return dens
