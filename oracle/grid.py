"""Periodic grid and the Fourier symbol of -Delta_N (Sec. 2.3, "Periodic
spectral discretization").

Test infrastructure: part of the float64 CPU oracle (see the package docstring).

The cell is prod_l (0, L_l) with N_l nodes per axis and spacing h, so
L_l = N_l * h.  A Fourier mode with integer wave number k_l has physical wave
number xi_l = 2*pi*k_l / L_l, and -Delta_N acts on it by |xi|^2.  The wave
numbers of an N-point axis are k in {0, .., N/2-1, -N/2, .., -1} (FFT order);
the Nyquist mode enters |xi|^2 with |k| = N/2, which is what makes
max |xi|^2 = N^2/2 on (0, 2*pi)^2 (Sec. 4.4, bounded-stiffness paragraph).
"""

import numpy as np


def wavenumbers(n):
    """Integer wave numbers of an n-point periodic axis in FFT order."""
    k = np.arange(n, dtype=np.int64)
    return np.where(k <= (n - 1) // 2, k, k - n)


def xi_axis(n, length):
    """Physical wave numbers xi = 2 pi k / L of one axis (float64)."""
    return 2.0 * np.pi * wavenumbers(n).astype(np.float64) / float(length)


def symbol(shape, lengths):
    """|xi|^2 on a grid of shape (nz, ny, nx) with cell lengths (Lz, Ly, Lx)."""
    nz, ny, nx = shape
    xz = xi_axis(nz, lengths[0]) if nz > 1 else np.zeros(1)
    xy = xi_axis(ny, lengths[1])
    xx = xi_axis(nx, lengths[2])
    return xz[:, None, None] ** 2 + xy[None, :, None] ** 2 + xx[None, None, :] ** 2


class Grid:
    """Uniform periodic grid: (nx, ny, nz) nodes, spacing h, L_l = n_l h.

    nz = 1 means a two-dimensional problem.
    """

    def __init__(self, nx, ny, nz=1, h=None, lengths=None):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        if lengths is not None:
            self.lengths = tuple(float(v) for v in lengths)  # (Lz, Ly, Lx)
        else:
            hh = 1.0 / self.nx if h is None else float(h)
            self.lengths = (self.nz * hh, self.ny * hh, self.nx * hh)
        self.shape = (self.nz, self.ny, self.nx)
        self.ng = self.nx * self.ny * self.nz
        self.dim = 2 if self.nz == 1 else 3
        self.volume = float(np.prod(self.lengths[3 - self.dim:]))
        # quadrature weight of the discrete inner product (u, v)_N
        self.weight = self.volume / self.ng
        self.s = symbol(self.shape, self.lengths)

    @property
    def h(self):
        return min(self.lengths[2] / self.nx, self.lengths[1] / self.ny,
                   *( [self.lengths[0] / self.nz] if self.dim == 3 else []))

    def coords(self):
        """Node coordinates (z, y, x) arrays of shape (nz, ny, nx)."""
        z = np.arange(self.nz) * (self.lengths[0] / self.nz)
        y = np.arange(self.ny) * (self.lengths[1] / self.ny)
        x = np.arange(self.nx) * (self.lengths[2] / self.nx)
        return np.meshgrid(z, y, x, indexing="ij")

    def max_symbol(self):
        return float(self.s.max())
