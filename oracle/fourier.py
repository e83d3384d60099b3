"""FFT tier of the spectral operators (Sec. 2.3 and Algorithm 1).

Test infrastructure: part of the float64 CPU oracle (see the package docstring).

-Delta_N u = iFFT(|xi|^2 FFT(u)) over the spatial axes, and the shifted
exchange block (a + b(-Delta_N)) and its inverse are the same Fourier-diagonal
multiplications.  scipy.fft, the FFT library of the paper's own runs
(Sec. 4.1), serves as the library DFT; the dense tier checks it against an
O(N_g^2) DFT.  WORKERS sets its thread count (1 unless a caller that times
the oracle on several host cores raises it).
"""

import scipy.fft

_AXES = (-3, -2, -1)

WORKERS = 1


def fftn(u):
    """DFT over the three spatial axes (complex result)."""
    return scipy.fft.fftn(u, axes=_AXES, workers=WORKERS)


def ifftn(u):
    """Inverse DFT over the three spatial axes (normalized by 1/N_g)."""
    return scipy.fft.ifftn(u, axes=_AXES, workers=WORKERS)


def fourier_multiply(u, mult):
    """Apply the real, even Fourier multiplier ``mult`` (shape (nz,ny,nx)) to
    each grid function in ``u`` (shape (..., nz, ny, nx))."""
    return ifftn(fftn(u) * mult).real


def neg_laplacian(g, u):
    """-Delta_N u (symbol |xi|^2)."""
    return fourier_multiply(u, g.s)


def h_apply(g, u, a, b):
    """(a I + b (-Delta_N)) u, the velocity block H of Sec. 3.1 when
    a = alpha and b = theta k C_hat."""
    return fourier_multiply(u, a + b * g.s)


def h_solve(g, u, a, b):
    """(a I + b (-Delta_N))^{-1} u: steps 1-3 of Algorithm 1 with
    a = alpha + lambda and b = theta k C_hat."""
    return fourier_multiply(u, 1.0 / (a + b * g.s))
