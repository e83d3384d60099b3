"""Pins of the lower-order field (oracle.fields) and of the midpoint stepper
with it: the demagnetizing field of a single Fourier mode in closed form, its
Nyquist reading against the textbook interpolant-derivative matrices, the
dense DFT-matrix tier, the analytic energy of the paper's 3D initial field,
the printed results of the 3D energy test (Sec. 4.6), the exact energy law
with demagnetization and anisotropy, and the adjoint of a step with them."""

import json
import os

import numpy as np
import pytest

from oracle import adjoint, dense, fields, fourier, nodal, steppers
from oracle.grid import Grid
from oracle.operators import Params

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_printed_values.json")))
E3 = GOLD["energy_test_3d"]


def _coords(g):
    z, y, x = np.meshgrid(*[np.arange(n) * (L / n) for n, L in zip(g.shape, g.lengths)], indexing="ij")
    return x, y, z


@pytest.mark.parametrize("kvec,amp", [((1, 2, 0), (0.3, -1.0, 0.7)), ((2, -1, 1), (1.0, 0.5, -0.25)),
                                      ((0, 0, 3), (0.2, 0.1, 1.0))])
def test_demag_of_one_mode(kvec, amp):
    """m = A cos(xi.x) with xi = 2 pi k / L: the periodic magnetostatic problem
    Delta phi = div m, h = -grad phi gives h = -xi (xi.A) cos(xi.x) / |xi|^2."""
    g = Grid(8, 6, 8, lengths=(2.0, 1.5, 3.0))
    x, y, z = _coords(g)
    xi = 2 * np.pi * np.array(kvec) / np.array([g.lengths[2], g.lengths[1], g.lengths[0]])
    ph = xi[0] * x + xi[1] * y + xi[2] * z
    A = np.array(amp)
    m = A[:, None, None, None] * np.cos(ph)[None]
    h = fields.demag_field(g, m)
    want = -(xi * (xi @ A) / (xi @ xi))[:, None, None, None] * np.cos(ph)[None]
    np.testing.assert_allclose(h, want, atol=1e-13)
    # uniform magnetization: zero field (zero-mean potential)
    np.testing.assert_allclose(fields.demag_field(g, np.ones((3,) + g.shape)), 0.0, atol=1e-15)


def test_demag_matches_dense_tier_and_is_negative_semidefinite():
    g = Grid(4, 4, 4, lengths=(1.0, 1.3, 0.8))
    prm = Params(demag=1.0, aniso_k=0.3, aniso_axis=(1 / 3, 2 / 3, 2 / 3))
    rng = np.random.default_rng(5)
    u = rng.standard_normal((3,) + g.shape)
    L = dense.low_linear_matrix(g, prm)
    np.testing.assert_allclose(fields.low_linear(g, prm, u).ravel(), L @ u.ravel(), atol=1e-13)
    np.testing.assert_allclose(L, L.T, atol=1e-14)
    D = dense.low_linear_matrix(g, Params(demag=1.0, aniso_k=0.0))
    ev = np.linalg.eigvalsh(D)
    # -D is an orthogonal projection (onto gradient fields without Nyquist content)
    assert ev.max() < 1e-13 and ev.min() > -1 - 1e-13


def test_derivative_matrix_closed_form():
    """The interpolant-derivative matrix (written from its cot formula, no DFT)
    differentiates every resolved mode exactly and is skew."""
    n, length = 10, 1.7
    x = np.arange(n) * length / n
    D = dense.derivative_matrix(n, length)
    for k in range(1, n // 2):
        xi = 2 * np.pi * k / length
        np.testing.assert_allclose(D @ np.sin(xi * x), xi * np.cos(xi * x), atol=1e-12)
        np.testing.assert_allclose(D @ np.cos(xi * x), -xi * np.sin(xi * x), atol=1e-12)
    np.testing.assert_allclose(D, -D.T, atol=1e-14)
    np.testing.assert_allclose(D @ np.ones(n), 0.0, atol=1e-13)


@pytest.mark.parametrize("shape,lengths", [((1, 4, 6), (1.0, 0.8, 1.2)), ((4, 4, 4), (1.0, 1.3, 0.8)),
                                           ((2, 6, 4), (0.5, 1.1, 0.9)), ((6, 4, 8), (2.0, 1.0, 1.5))])
def test_demag_nyquist_reading_matches_interpolant_derivatives(shape, lengths):
    """Pin of the Nyquist reading of the demagnetizing field: grad and div are
    the derivatives of the trigonometric interpolant sampled at the nodes
    (the textbook cot matrices of dense.derivative_matrix, no DFT), the
    Poisson solve the pseudo-inverse of the naive-DFT -Delta_N.  On random
    fields, whose spectra fill every Nyquist plane, oracle.fields.demag_field
    equals h = G L^+ Div m; keeping the Nyquist entries of xi~ would not."""
    nz, ny, nx = shape
    g = Grid(nx, ny, nz, lengths=lengths)
    m = np.random.default_rng(11).standard_normal((3,) + g.shape)
    want = (dense.demag_matrix_interpolant(g) @ m.ravel()).reshape(m.shape)
    np.testing.assert_allclose(fields.demag_field(g, m), want, atol=1e-13)


def test_demag_of_the_nyquist_mode_is_zero():
    """m = (cos(pi x / h), 0, 0): the interpolant's divergence -(pi/h) sin(pi x/h)
    vanishes at every node, so the discrete potential and field are zero (the
    reading that kept the Nyquist entry would give h = -m instead)."""
    for g in (Grid(8, 6, 1, lengths=(1.0, 0.75, 1.0)), Grid(6, 4, 8, lengths=(1.0, 0.5, 0.75))):
        x, _, _ = _coords(g)
        hx = g.lengths[2] / g.nx
        m = np.zeros((3,) + g.shape)
        m[0] = np.cos(np.pi * x / hx)
        np.testing.assert_allclose(fields.demag_field(g, m), 0.0, atol=1e-13)
        D = dense.demag_matrix_interpolant(g)
        np.testing.assert_allclose(D @ m.ravel(), 0.0, atol=1e-12)


def _energy_case(n):
    g = Grid(n, n, n, lengths=(2 * np.pi,) * 3)
    prm = Params(alpha=E3["alpha"], cexc=1.0, dt=E3["k"], shift=E3["lambda"], h_uniform=tuple(E3["h_ext"]),
                 demag=1.0, aniso_k=E3["aniso_k"], aniso_axis=(0.0, 0.0, 1.0))
    x, y, z = _coords(g)
    m = np.array([np.sin(x + z) * np.cos(y + z), np.cos(x + z) * np.cos(y + z), np.sin(y + z)])
    return g, prm, m


def test_initial_energy_terms_closed_form():
    """With a = x+z, b = y+z: |grad m|^2 = 2 cos^2 b + 2 (mean 3, exchange 3/2);
    K (1 - m_z^2) has mean K/2 = 0.1; the modes (1,1,2), (1,-1,0), (0,1,1)
    carry demag energy 1/48 + 1/16 + 1/8 = 5/24; the Zeeman mean is 0.  The
    total 1.8083333... is the paper's printed initial energy."""
    g, prm, m = _energy_case(16)
    vol = (2 * np.pi) ** 3
    w = g.weight / vol
    exch = w * 0.5 * float(nodal.dot(m, fourier.neg_laplacian(g, m)).sum())
    dem = -w * 0.5 * float(nodal.dot(m, fields.demag_field(g, m)).sum())
    ani = w * prm.aniso_k * float((1 - m[2] ** 2).sum())
    zee = -w * float(nodal.dot(m, prm.h_ext(g.shape)).sum())
    assert exch == pytest.approx(1.5, abs=1e-14)
    assert dem == pytest.approx(5 / 24, abs=1e-14)
    assert ani == pytest.approx(0.1, abs=1e-14)
    assert zee == pytest.approx(0.0, abs=1e-15)
    assert steppers.energy(g, prm, m) / vol == pytest.approx(E3["energy_initial"], abs=1e-10)


def _run_energy_test(n):
    g, prm, m = _energy_case(n)
    vol = (2 * np.pi) ** 3
    tol = E3["tol"]
    nsteps = int(round(E3["T"] / E3["k"]))
    v = lam = None
    energies, lens, pics, its, gaps = [steppers.energy(g, prm, m) / vol], [], [], [], []
    for _ in range(nsteps):
        m1, v, lam, info = steppers.midpoint_step(g, prm, m, v, lam, restart=50, rtol=tol, picard_tol=tol)
        assert info["converged"]
        d = steppers.midpoint_diagnostics(g, prm, m, m1, v, lam)
        energies.append(d["energy_after"] / vol)
        lens.append(d["max_len_err"])
        pics.append(info["picard_iters"])
        its += info["lin_iters"]
        gaps.append(abs(d["dissipation_defect"] - d["inexact_correction"]) / vol)
        m = m1
    return energies, lens, pics, its, gaps


@pytest.mark.parametrize("n", [16, 24, 32])
def test_energy_test_matches_paper(n):
    energies, lens, pics, its, gaps = _run_energy_test(n)
    half_ulp = 0.5 * 10.0 ** -E3["printed_decimals"]
    assert abs(energies[-1] - E3["energy_final"][str(n)]) <= half_ulp
    assert all(b < a for a, b in zip(energies, energies[1:]))
    # printed to three significant digits: 1.68e-10 (N = 24) .. 1.87e-10
    lo, hi = E3["len_err_range"]
    assert lo - 0.005e-10 <= max(lens) <= hi + 0.005e-10
    assert pics == [E3["picard_per_step"]] * len(pics)
    # GMRES iterations per solve: printed 7.84..8.88 over N = 16, 24, 32
    lo, hi = E3["gmres_per_solve_range"]
    assert lo - 0.25 <= np.mean(its) <= hi
    assert max(gaps) < 2 * E3["defect_correction_gap"]


def test_energy_law_exact_with_lower_order_field():
    """Converged midpoint steps with demag + anisotropy + Zeeman satisfy
    g(m^{n+1}) - g(m^n) = -alpha k/(1+alpha^2) ||v||_N^2 and |m^{n+1}| = 1."""
    g = Grid(8, 8, 8, lengths=(2.0, 2.0, 2.0))
    prm = Params(alpha=0.1, dt=2e-3, shift=0.5, h_uniform=(0.2, -0.1, 0.3), demag=1.0, aniso_k=0.5,
                 aniso_axis=(0.6, 0.0, 0.8))
    rng = np.random.default_rng(11)
    m = rng.standard_normal((3,) + g.shape)
    m = np.fft.ifftn(np.fft.fftn(m, axes=(-3, -2, -1)) * np.exp(-g.s / g.s.max() * 12), axes=(-3, -2, -1)).real
    m /= np.sqrt(nodal.dot(m, m))
    v = lam = None
    for _ in range(2):
        m1, v, lam, info = steppers.midpoint_step(g, prm, m, v, lam, rtol=1e-14, picard_tol=1e-14, picard_max=100)
        assert info["converged"]
        d = steppers.midpoint_diagnostics(g, prm, m, m1, v, lam)
        drop = d["energy_before"] - d["energy_after"]
        assert drop > 0
        assert abs(d["dissipation_defect"]) < 1e-9 * drop
        assert d["max_len_err"] < 1e-12
        m = m1


def _residual(g, prm, m_n, u):
    """Residual of eq. "C-N" written out, lower-order field at the midpoint."""
    k = prm.dt
    v, r = u[:3], u[3]
    mh = m_n + 0.5 * k * v
    out = np.empty_like(u)
    out[:3] = (prm.alpha * v + nodal.cross(mh, v) + prm.c_hat * fourier.neg_laplacian(g, mh)
               + mh * r - (1 + prm.alpha ** 2) * fields.h_low(g, prm, mh))
    out[3] = -nodal.dot(mh, v)
    return out


def test_jacobian_with_lower_order_field():
    g = Grid(4, 4, 4, lengths=(1.0, 1.0, 1.0))
    prm = Params(alpha=0.1, dt=0.05, theta=0.5, shift=0.5, demag=1.0, aniso_k=0.4, aniso_axis=(0.0, 0.6, 0.8),
                 h_uniform=(0.1, 0.0, 0.2))
    rng = np.random.default_rng(2)
    m_n = rng.standard_normal((3,) + g.shape)
    m_n /= np.sqrt(nodal.dot(m_n, m_n))
    u = rng.standard_normal((4,) + g.shape)
    J = dense.midpoint_jacobian(g, prm, m_n, u[:3], u[3])
    eps = 1e-6
    for _ in range(3):
        du = rng.standard_normal(u.shape)
        fd = (_residual(g, prm, m_n, u + eps * du) - _residual(g, prm, m_n, u - eps * du)) / (2 * eps)
        np.testing.assert_allclose(J @ du.ravel(), fd.ravel(), atol=1e-8 * np.abs(fd).max())
        np.testing.assert_allclose(adjoint.jacobian_transpose_apply(g, prm, m_n, u[:3], u[3], du).ravel(),
                                   J.T @ du.ravel(), atol=1e-12 * np.abs(J).max())


def test_adjoint_with_lower_order_field_matches_central_differences():
    g = Grid(6, 6, 1, h=1.0 / 6)
    base = dict(alpha=0.1, dt=0.01, shift=0.5, demag=1.0, aniso_k=0.3, aniso_axis=(1 / 3, 2 / 3, 2 / 3))
    rng = np.random.default_rng(8)
    m0 = rng.standard_normal((3,) + g.shape)
    m0 = np.fft.ifftn(np.fft.fftn(m0, axes=(-3, -2, -1)) * np.exp(-g.s / g.s.max() * 6), axes=(-3, -2, -1)).real
    m0 /= np.sqrt(nodal.dot(m0, m0))
    hu = np.array([0.0, 0.1, 0.4])
    hf = 0.1 * rng.standard_normal((3,) + g.shape)

    def forward(m, hu_, hf_):
        p = Params(h_uniform=tuple(hu_), h_field=hf_, **base)
        v = lam = None
        traj = []
        for _ in range(3):
            m1, v, lam, info = steppers.midpoint_step(g, p, m, v, lam, rtol=1e-14, picard_tol=1e-13,
                                                      picard_max=100)
            assert info["converged"]
            traj.append((m, v, lam))
            m = m1
        return m, traj

    loss = lambda m: float((m[2] ** 2).sum())
    mN, traj = forward(m0, hu, hf)
    p = Params(h_uniform=tuple(hu), h_field=hf, **base)
    gbar = np.zeros_like(mN)
    gbar[2] = 2 * mN[2]
    hbar_u = np.zeros(3)
    hbar_f = np.zeros_like(hf)
    for (m_n, v, lam) in reversed(traj):
        gbar, hf_b, hu_b, _, _ = adjoint.step_adjoint(g, p, m_n, v, lam, gbar, rtol=1e-14)
        hbar_u += hu_b
        hbar_f += hf_b
    eps = 1e-6
    for c in range(3):
        e = np.zeros(3)
        e[c] = eps
        fd = (loss(forward(m0, hu + e, hf)[0]) - loss(forward(m0, hu - e, hf)[0])) / (2 * eps)
        assert hbar_u[c] == pytest.approx(fd, rel=1e-5, abs=1e-9)
    d = rng.standard_normal(hf.shape)
    fd = (loss(forward(m0, hu, hf + eps * d)[0]) - loss(forward(m0, hu, hf - eps * d)[0])) / (2 * eps)
    assert float((hbar_f * d).sum()) == pytest.approx(fd, rel=1e-5, abs=1e-9)
    dm = rng.standard_normal(m0.shape)
    fd = (loss(forward(m0 + eps * dm, hu, hf)[0]) - loss(forward(m0 - eps * dm, hu, hf)[0])) / (2 * eps)
    assert float((gbar * dm).sum()) == pytest.approx(fd, rel=1e-5, abs=1e-9)
