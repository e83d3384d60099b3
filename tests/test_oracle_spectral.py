"""Pins of the oracle's spectral tier against definitions that do not use it:
the trigonometric eigenfunctions of -Delta_N (Sec. 2.3), the naive DFT, and
the Nyquist convention fixed by max|xi|^2 = N^2/2 on (0, 2 pi)^2 (Sec. 4.4)."""

import numpy as np
import pytest

from oracle import dense, fourier
from oracle.grid import Grid, wavenumbers


def test_wavenumbers_fft_order():
    assert list(wavenumbers(4)) == [0, 1, -2, -1]
    assert list(wavenumbers(5)) == [0, 1, 2, -2, -1]
    assert list(wavenumbers(8)) == [0, 1, 2, 3, -4, -3, -2, -1]


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8])
def test_naive_dft_matches_numpy_fft(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    np.testing.assert_allclose(dense.dft_matrix(n) @ x, np.fft.fft(x), rtol=0, atol=1e-13)


@pytest.mark.parametrize("shape,lengths", [((1, 8, 8), (1.0, 1.0, 1.0)),
                                           ((1, 6, 4), (1.0, 2 * np.pi, 1.5)),
                                           ((4, 4, 8), (0.5, 1.0, 2.0)),
                                           ((1, 5, 7), (1.0, 1.0, 1.0))])
def test_neg_laplacian_on_trig_modes(shape, lengths):
    """-Delta_N cos(xi.x) = |xi|^2 cos(xi.x) for every resolved mode,
    including the Nyquist mode cos(pi x / h)."""
    g = Grid(shape[2], shape[1], shape[0], lengths=lengths)
    z, y, x = g.coords()
    for kz in range(-(g.nz // 2), g.nz // 2 + 1):
        for ky in range(-(g.ny // 2), g.ny // 2 + 1):
            for kx in range(0, g.nx // 2 + 1):
                xi = (2 * np.pi * kz / lengths[0], 2 * np.pi * ky / lengths[1], 2 * np.pi * kx / lengths[2])
                if g.nz == 1:
                    xi = (0.0, xi[1], xi[2])
                phase = xi[0] * z + xi[1] * y + xi[2] * x
                s = xi[0] ** 2 + xi[1] ** 2 + xi[2] ** 2
                for f in (np.cos(phase), np.sin(phase)):
                    got = fourier.neg_laplacian(g, f)
                    # sin of a Nyquist mode vanishes on the nodes: both sides are 0
                    np.testing.assert_allclose(got, s * f, rtol=0, atol=1e-11 * max(1.0, s))


def test_nyquist_max_symbol_two_pi_square():
    """max |xi|^2 = N^2/2 on (0, 2 pi)^2 (Sec. 4.4)."""
    for n in (32, 64, 256):
        g = Grid(n, n, 1, lengths=(1.0, 2 * np.pi, 2 * np.pi))
        assert g.max_symbol() == pytest.approx(n * n / 2, rel=1e-14)


@pytest.mark.parametrize("shape", [(1, 4, 4), (1, 6, 4), (4, 4, 4), (1, 5, 5), (2, 3, 4)])
def test_dense_laplacian_matches_fft_tier(shape):
    g = Grid(shape[2], shape[1], shape[0], lengths=(1.0, 1.3, 0.7))
    D = dense.neg_laplacian_matrix(g)
    assert np.abs(D - D.T).max() < 1e-12 * np.abs(D).max()
    np.testing.assert_allclose(D @ np.ones(g.ng), 0.0, atol=1e-10)
    rng = np.random.default_rng(7)
    u = rng.standard_normal(g.shape)
    np.testing.assert_allclose(D @ u.ravel(), fourier.neg_laplacian(g, u).ravel(), rtol=0,
                               atol=1e-12 * np.abs(D).max() * np.abs(u).max() * g.ng)
    ev = np.sort(np.linalg.eigvalsh(D))
    np.testing.assert_allclose(ev, np.sort(g.s.ravel()), rtol=0, atol=1e-10 * ev.max())


def test_h_solve_inverts_h_apply():
    g = Grid(8, 8, 4, h=0.125)
    rng = np.random.default_rng(3)
    u = rng.standard_normal((3,) + g.shape)
    w = fourier.h_solve(g, fourier.h_apply(g, u, 0.7, 0.3), 0.7, 0.3)
    np.testing.assert_allclose(w, u, rtol=0, atol=1e-12)
