"""Seeded synthetic inputs for the periodic LLG saddle-point workloads.

This module is shared by the tests, the benchmark and the oracle's callers.
It holds no arithmetic of the solver: it only draws initial magnetizations,
applied fields and parameters.  Every workload lives on the unit cell [0,1]^d
with h = 1/N and normalized exchange coefficient 1; inputs are generated once
on the host with numpy.random.default_rng(20260724 + workload id).

Mode sets
* "K lowest modes": the zero wave vector plus the K-1 lowest nonzero
  half-space integer wave vectors k = (kx, ky[, kz]) ordered by |k|^2, then
  lexicographically (half-space: first nonzero component positive).  Each
  component is m_c = a_c0 + sum_j a_cj cos(2 pi k_j.x) + b_cj sin(2 pi k_j.x)
  with coefficients iid N(0,1), drawn in (c, j, cos/sin) order.
* "broadband": every nonzero wave vector of the grid (|k|_inf <= N/2), amplitude
  1/|k| and a uniform random phase; the field is the real part of the inverse
  DFT of that spectrum (phases drawn in (c, kz, ky, kx) FFT order).
Fields are normalized node by node; if min |m| < 1e-3 rms |m| before
normalization the seed is advanced by one (and the used seed is reported).
The test is relative to the field's RMS nodal norm because the raw broadband
field has an arbitrary overall scale.

The five workloads (the paper's own runs use (0, 2 pi)^d; these are synthetic
stand-ins of the same structure):
  1  2D 32^2,  projected Euler, 1 step,  alpha 0.1,  dt = 10 h^2, h = (0,0,0.5), 4 modes, FP64
  2  2D 512^2, midpoint, 10 steps, alpha 0.05, dt = 13.3 x explicit limit, h = (0,0,1), 8 modes, FP64
  3  3D 128^3, projected Euler, 20 steps, alpha 0.2, dt = 13.3 x limit, h = (0,0,1), broadband,
     FP32-preconditioned FGMRES-IR beside plain FP64
  4  3D 256^3, midpoint, 5 steps, alpha 0.02, dt = 13.3 x limit, h = (0,0,1),
     8 modes + 1% broadband, FP32-preconditioned FGMRES-IR beside plain FP64
  5  2D 256^2 (and a 16^2 copy with the same dt), midpoint, 20 steps, alpha 0.1,
     dt = 10 h^2 (256^2), h_uniform (0,0,0.5) + h_field ~ N(0, 0.1^2), 4 modes;
     differentiation workload (loss sum m_z^2 at the last step)
"""

import itertools
import math

import numpy as np

BASE_SEED = 20260724
EXPLICIT_RATIO = 13.3


def lowest_modes(dim, count):
    """The ``count`` lowest half-space integer wave vectors, zero first."""
    rad = int(math.ceil(math.sqrt(count))) + 2
    cands = []
    for k in itertools.product(range(-rad, rad + 1), repeat=dim):
        nz = [c for c in k if c != 0]
        if k != (0,) * dim and nz[0] < 0:
            continue
        cands.append((sum(c * c for c in k), k))
    cands.sort()
    return [k for _, k in cands[:count]]


def _coords(n, dim):
    x = np.arange(n) / n
    if dim == 2:
        yy, xx = np.meshgrid(x, x, indexing="ij")
        return (xx, yy)
    zz, yy, xx = np.meshgrid(x, x, x, indexing="ij")
    return (xx, yy, zz)


def _shape(n, dim):
    return (1, n, n) if dim == 2 else (n, n, n)


def modes_field(n, dim, count, rng):
    xs = _coords(n, dim)
    ks = lowest_modes(dim, count)
    out = np.empty((3,) + _shape(n, dim))
    for c in range(3):
        f = np.full(xs[0].shape, rng.standard_normal())
        for k in ks[1:]:
            a, b = rng.standard_normal(2)
            ph = 2 * np.pi * sum(kk * xx for kk, xx in zip(k, xs))
            f = f + a * np.cos(ph) + b * np.sin(ph)
        out[c] = f.reshape(out.shape[1:])
    return out


def broadband_field(n, dim, rng):
    shape = _shape(n, dim)
    k1 = np.fft.fftfreq(n, 1.0 / n)
    kz = k1 if dim == 3 else np.zeros(1)
    kabs = np.sqrt(kz[:, None, None] ** 2 + k1[None, :, None] ** 2 + k1[None, None, :] ** 2)
    amp = np.where(kabs > 0, 1.0 / np.where(kabs > 0, kabs, 1.0), 0.0)
    phase = rng.uniform(0.0, 2 * np.pi, size=(3,) + shape)
    spec = amp[None] * np.exp(1j * phase)
    return np.fft.ifftn(spec, axes=(-3, -2, -1)).real


def _normalize(f):
    return f / np.sqrt(f[0] ** 2 + f[1] ** 2 + f[2] ** 2)


def _min_norm(f):
    """min_i |f_i| relative to the RMS nodal norm."""
    nrm = np.sqrt(f[0] ** 2 + f[1] ** 2 + f[2] ** 2)
    return float(nrm.min() / np.sqrt(np.mean(nrm * nrm)))


def initial_m(n, dim, kind, seed):
    """Draw m0 ('modes4', 'modes8', 'broadband', 'modes8+bb1') and return
    (m0, rng, seed_used); the rng continues after the m0 draws."""
    while True:
        rng = np.random.default_rng(seed)
        if kind == "modes4":
            f = modes_field(n, dim, 4, rng)
        elif kind == "modes8":
            f = modes_field(n, dim, 8, rng)
        elif kind == "broadband":
            f = broadband_field(n, dim, rng)
        elif kind == "modes8+bb1":
            sm = modes_field(n, dim, 8, rng)
            if _min_norm(sm) < 1e-3:
                seed += 1
                continue
            u = broadband_field(n, dim, rng)
            f = _normalize(sm) + 0.01 * u / np.sqrt(np.mean(u * u))
        else:
            raise ValueError(kind)
        if _min_norm(f) >= 1e-3:
            return _normalize(f), rng, seed
        seed += 1


def max_symbol_unit_cell(n, dim):
    """max |xi|^2 on [0,1]^d with n nodes per axis: d (pi n)^2."""
    return dim * (math.pi * n) ** 2


def dt_explicit_multiple(ratio, alpha, n, dim, cexc=1.0):
    """k with k C_hat max|xi|^2 = ratio * 2 alpha (C_hat = (1+alpha^2) cexc)."""
    return ratio * 2.0 * alpha / ((1.0 + alpha * alpha) * cexc * max_symbol_unit_cell(n, dim))


WORKLOADS = {
    1: dict(name="2d_32_euler", n=32, dim=2, scheme="euler", steps=1, alpha=0.1, dt="10h2",
            h_uniform=(0.0, 0.0, 0.5), m0="modes4", prec=("fp64",)),
    2: dict(name="2d_512_midpoint", n=512, dim=2, scheme="midpoint", steps=10, alpha=0.05,
            dt="explicit", h_uniform=(0.0, 0.0, 1.0), m0="modes8", prec=("fp64",)),
    3: dict(name="3d_128_euler_broadband", n=128, dim=3, scheme="euler", steps=20, alpha=0.2,
            dt="explicit", h_uniform=(0.0, 0.0, 1.0), m0="broadband", prec=("fp32_ir", "fp64")),
    4: dict(name="3d_256_midpoint", n=256, dim=3, scheme="midpoint", steps=5, alpha=0.02,
            dt="explicit", h_uniform=(0.0, 0.0, 1.0), m0="modes8+bb1", prec=("fp32_ir", "fp64")),
    5: dict(name="2d_256_midpoint_adjoint", n=256, dim=2, scheme="midpoint", steps=20, alpha=0.1,
            dt="10h2", h_uniform=(0.0, 0.0, 0.5), m0="modes4", prec=("fp64",), ckpt_every=5,
            h_field_std=0.1),
}

COMMON = dict(cexc=1.0, shift=0.5, restart=30, rtol=1e-10, picard_tol=1e-10, picard_max=50)


def make(wid, n=None, seed=None):
    """Materialize workload ``wid`` (optionally at another grid size n, with
    the same time step as the full-size workload).  Returns a dict with m0
    (3, nz, ny, nx) float64, h_field or None, and all parameters."""
    spec = dict(WORKLOADS[wid])
    spec.update(COMMON)
    n_full = spec["n"]
    n = n_full if n is None else int(n)
    if spec["dt"] == "10h2":
        dt = 10.0 / n_full ** 2
    else:
        dt = dt_explicit_multiple(EXPLICIT_RATIO, spec["alpha"], n_full, spec["dim"])
    seed0 = BASE_SEED + wid if seed is None else seed
    m0, rng, used = initial_m(n, spec["dim"], spec["m0"], seed0)
    h_field = None
    if spec.get("h_field_std"):
        h_field = spec["h_field_std"] * rng.standard_normal((3,) + m0.shape[1:])
    nz = 1 if spec["dim"] == 2 else n
    spec.update(n=n, nx=n, ny=n, nz=nz, h=1.0 / n, dt=dt, m0=m0, h_field=h_field,
                seed_used=used, theta=1.0 if spec["scheme"] == "euler" else 0.5)
    return spec


def gaussian_rhs(n, seed, dim=2):
    """Random-right-hand-side study input: a Gaussian velocity right-hand side
    (numpy.random.default_rng(seed).standard_normal over the 3 planes, SoA),
    scaled to unit 2-norm, with a zero multiplier plane.  Shape (4, [nz,] ny, nx)
    with nz = 1 in 2D."""
    shape = _shape(n, dim)
    f = np.random.default_rng(seed).standard_normal((3,) + shape)
    b = np.zeros((4,) + shape)
    b[:3] = f / np.linalg.norm(f)
    return b


def manufactured(n, dim, t, alpha, cexc=1.0):
    """Problem data of the manufactured-solution runs (temporal convergence
    and preconditioner comparison) on (0, 2 pi)^dim with n nodes per axis:
    the unit field m_e(x, t) and its source term F (entering as the applied
    field F / (1 + alpha^2)), sampled at the nodes, shapes (3, nz, ny, nx).

    2D: a = t + x, b = t + y; 3D: a = t + x + z, b = t + y + z;
    m_e = (sin a cos b, cos a cos b, sin b),
    F = alpha d_t m_e + m_e x d_t m_e - (1 + alpha^2) cexc Delta m_e."""
    ax = 2.0 * np.pi * np.arange(n) / n
    if dim == 2:
        yy, xx = np.meshgrid(ax, ax, indexing="ij")
        a, b = (t + xx)[None], (t + yy)[None]
    else:
        zz, yy, xx = np.meshgrid(ax, ax, ax, indexing="ij")
        a, b = t + xx + zz, t + yy + zz
    sa, ca, sb, cb = np.sin(a), np.cos(a), np.sin(b), np.cos(b)
    zero = np.zeros_like(a)
    m = np.stack([sa * cb, ca * cb, sb])
    m_a = np.stack([ca * cb, -sa * cb, zero])
    m_b = np.stack([-sa * sb, -ca * sb, cb])
    m_aa = np.stack([-sa * cb, -ca * cb, zero])
    m_ab = np.stack([-ca * sb, sa * sb, zero])
    m_bb = -m
    if dim == 2:
        dt_m, lap = m_a + m_b, m_aa + m_bb
    else:
        dt_m, lap = m_a + m_b, 2.0 * (m_aa + m_bb + m_ab)
    cr = np.stack([m[1] * dt_m[2] - m[2] * dt_m[1], m[2] * dt_m[0] - m[0] * dt_m[2],
                   m[0] * dt_m[1] - m[1] * dt_m[0]])
    F = alpha * dt_m + cr - (1.0 + alpha ** 2) * cexc * lap
    return m, F
