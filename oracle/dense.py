"""Dense tier: naive DFT matrices and the assembled saddle system.

Test infrastructure: part of the float64 CPU oracle (see the package docstring).

Used only on grids of at most a few hundred nodes, to check the FFT tier and
to provide the direct solve x = A^{-1} b that Proposition 1 (well-posedness)
guarantees is unique.  The DFT is written out as exp(-2 pi i j k / n), with no
FFT library involved.
"""

import numpy as np

from . import nodal
from .grid import wavenumbers


def dft_matrix(n):
    """F[k, j] = exp(-2 pi i k j / n): the naive n-point DFT."""
    j = np.arange(n)
    return np.exp(-2j * np.pi * np.outer(j, j) / n)


def grid_dft(g):
    """DFT over the node index x + nx (y + ny z): kron(Fz, Fy, Fx)."""
    return np.kron(dft_matrix(g.nz), np.kron(dft_matrix(g.ny), dft_matrix(g.nx)))


def neg_laplacian_matrix(g):
    """D = F^{-1} diag(|xi|^2) F, real symmetric (N_g x N_g)."""
    F = grid_dft(g)
    # |xi|^2 listed in the same (kz, ky, kx) C order as the rows of F
    kz = 2 * np.pi * wavenumbers(g.nz) / g.lengths[0] if g.nz > 1 else np.zeros(1)
    ky = 2 * np.pi * wavenumbers(g.ny) / g.lengths[1]
    kx = 2 * np.pi * wavenumbers(g.nx) / g.lengths[2]
    s = (kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2).ravel()
    D = (np.conj(F).T @ (s[:, None] * F)) / g.ng
    return D.real


def low_linear_matrix(g, prm):
    """Dense L_low (3 N_g x 3 N_g, component-major): demag * D_dem + 2 K e e^T,
    with D_dem = -F^{-1} diag(xi~_c xi~_d / |xi|^2) F (zero at xi = 0), xi~ the
    derivative wave vector whose Nyquist entries are zero."""
    n = g.ng
    F = grid_dft(g)

    def axis(nn, length, nyq_zero):
        k = wavenumbers(nn).astype(np.float64)
        if nyq_zero and nn % 2 == 0:
            k[nn // 2] = 0.0
        return 2 * np.pi * k / length if nn > 1 else np.zeros(1)

    def grid3(nyq_zero):
        kz = axis(g.nz, g.lengths[0], nyq_zero)
        ky = axis(g.ny, g.lengths[1], nyq_zero)
        kx = axis(g.nx, g.lengths[2], nyq_zero)
        shp = (len(kz), len(ky), len(kx))
        return [np.broadcast_to(kx[None, None, :], shp).ravel(),
                np.broadcast_to(ky[None, :, None], shp).ravel(),
                np.broadcast_to(kz[:, None, None], shp).ravel()]

    xi = grid3(False)
    xt = grid3(True)
    s = xi[0] ** 2 + xi[1] ** 2 + xi[2] ** 2
    inv = np.where(s > 0, 1.0 / np.where(s > 0, s, 1.0), 0.0)
    e = np.asarray(prm.aniso_axis, dtype=np.float64)
    L = np.zeros((3 * n, 3 * n))
    for c in range(3):
        for d in range(3):
            blk = 2.0 * prm.aniso_k * e[c] * e[d] * np.eye(n)
            if prm.demag != 0.0:
                sym = xt[c] * xt[d] * inv
                blk = blk - prm.demag * ((np.conj(F).T @ (sym[:, None] * F)) / n).real
            L[c * n:(c + 1) * n, d * n:(d + 1) * n] = blk
    return L


def derivative_matrix(n, length):
    """First-derivative matrix of the trigonometric interpolant on an even
    n-point periodic axis of length L, sampled at the nodes: the textbook
    closed form D[i, j] = (pi / L) (-1)^(i-j) cot(pi (i-j) / n), D[i, i] = 0
    (Trefethen, Spectral Methods in MATLAB, ch. 3), written out with no DFT.
    Differentiating the interpolant of the Nyquist mode cos(pi x / h) gives
    -(pi/h) sin(pi x / h), zero at every node, so D maps that mode to 0."""
    if n % 2:
        raise ValueError("derivative_matrix: even n only")
    i = np.arange(n)
    d = i[:, None] - i[None, :]
    with np.errstate(divide="ignore", invalid="ignore"):
        D = (np.pi / length) * np.where(d % 2 == 0, 1.0, -1.0) / np.tan(np.pi * d / n)
    D[d == 0] = 0.0
    return D


def demag_matrix_interpolant(g):
    """Dense periodic demagnetizing operator built from the interpolant
    derivatives: h = G L^+ Div m, with G / Div the gradient / divergence of
    the trigonometric interpolant (derivative_matrix along each axis), L =
    -Delta_N from the naive DFT and L^+ its pseudo-inverse (zero-mean
    potential).  Returns the 3 N_g x 3 N_g matrix in component-major order."""
    n = g.ng
    eye = lambda k: np.eye(k)
    axes = []
    if g.nx > 1:
        axes.append(np.kron(eye(g.nz), np.kron(eye(g.ny), derivative_matrix(g.nx, g.lengths[2]))))
    if g.ny > 1:
        axes.append(np.kron(eye(g.nz), np.kron(derivative_matrix(g.ny, g.lengths[1]), eye(g.nx))))
    if g.nz > 1:
        axes.append(np.kron(derivative_matrix(g.nz, g.lengths[0]), np.kron(eye(g.ny), eye(g.nx))))
    while len(axes) < 3:
        axes.append(np.zeros((n, n)))
    Lp = np.linalg.pinv(neg_laplacian_matrix(g), rcond=1e-12, hermitian=True)
    div = np.hstack(axes)
    grad = np.vstack(axes)
    return grad @ Lp @ div


def block_indices(g):
    n = g.ng
    return [np.arange(c * n, (c + 1) * n) for c in range(4)]


def saddle_parts(g, prm, m):
    """Dense (calH, calS) of Sec. 3.1, eq. (HS), in the block order
    (v1, v2, v3, r), each block N_g wide."""
    n = g.ng
    D = neg_laplacian_matrix(g)
    Hb = prm.alpha * np.eye(n) + prm.h_coef * D
    calH = np.zeros((4 * n, 4 * n))
    for c in range(3):
        calH[c * n:(c + 1) * n, c * n:(c + 1) * n] = Hb
    calS = np.zeros((4 * n, 4 * n))
    mf = m.reshape(3, n)
    for i in range(n):
        blk = nodal.s_tilde(mf[:, i])
        rows = np.arange(4) * n + i
        calS[np.ix_(rows, rows)] = blk
    return calH, calS


def saddle_matrix(g, prm, m):
    calH, calS = saddle_parts(g, prm, m)
    return calH + calS


def hss_factors(g, prm, m):
    """Dense M1 = calH + lambda I and M2 = calS + lambda I."""
    calH, calS = saddle_parts(g, prm, m)
    eye = np.eye(calH.shape[0])
    return calH + prm.shift * eye, calS + prm.shift * eye


def solve(g, prm, m, b):
    """Direct solve of A x = b (b, x of shape (4, nz, ny, nx))."""
    A = saddle_matrix(g, prm, m)
    return np.linalg.solve(A, b.ravel()).reshape(b.shape)


def midpoint_jacobian(g, prm, m_n, v, r):
    """Dense Jacobian J of the midpoint residual with respect to (v, r),
    assembled block by block from the dense -Delta_N and the nodal blocks
    (theta = 1/2; see oracle.adjoint for the formula)."""
    n = g.ng
    k = prm.dt
    D = neg_laplacian_matrix(g)
    mn = m_n.reshape(3, n)
    vv = v.reshape(3, n)
    rr = np.asarray(r).reshape(n)
    mh = mn + 0.5 * k * vv
    mc = mh + 0.5 * k * vv
    J = np.zeros((4 * n, 4 * n))
    Hb = prm.alpha * np.eye(n) + 0.5 * k * prm.c_hat * D
    for c in range(3):
        J[c * n:(c + 1) * n, c * n:(c + 1) * n] = Hb + 0.5 * k * np.diag(rr)
    J[:3 * n, :3 * n] -= 0.5 * k * (1.0 + prm.alpha ** 2) * low_linear_matrix(g, prm)
    for i in range(n):
        L = nodal.lambda_matrix(mn[:, i])
        rows = np.arange(3) * n + i
        J[np.ix_(rows, rows)] += L
        J[rows, 3 * n + i] = mh[:, i]
        J[3 * n + i, rows] = -mc[:, i]
    return J
