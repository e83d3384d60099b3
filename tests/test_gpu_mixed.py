"""GPU parity on grids whose sizes are not powers of two (radix-3 and radix-5
line FFTs: N = 3 * 2^a, 5 * 2^a) and on cells with different spacings per
axis (Sec. 2.3: the periodic cell prod_l (0, L_l), wave numbers 2 pi k / L_l).
Every such line length is exercised as the x half-length and as a y and a z
length, against the FP64 oracle's FFT tier and, on tiny grids, the dense
assembled matrices."""

import math

import numpy as np
import pytest

import paper_2607_15290_amd as P
from oracle import dense, fields, operators, steppers
from oracle.grid import Grid
from tests.gpu_util import announce, assert_elem, both_params, dev, host, unit_field

pytestmark = pytest.mark.gpu


def fp32_bound(shape):
    """Element-wise float32 pipeline bound relative to max |ref|: one float32
    unit roundoff per butterfly level of each forward and inverse line DFT
    (a mixed radix-3/5 length counts as its next power of two), plus 16 for
    input rounding and the nodal arithmetic."""
    levels = sum(2 * math.ceil(math.log2(n)) for n in shape if n > 1)
    return (levels + 16) * 2.0 ** -24

KW = dict(alpha=0.1, cexc=1.0, dt=2e-3, theta=1.0, shift=0.5)
MIXED = [6, 10, 12, 20, 24, 40, 48, 80, 96, 160, 192, 320, 384]


def _case(nx, ny, nz, seed, lengths=None, kw=KW, unit=True):
    if lengths is None:
        lengths = (nx / 64.0, ny / 64.0, nz / 64.0)
    lx, ly, lz = lengths
    g = Grid(nx, ny, nz, lengths=(lz, ly, lx))
    m = unit_field((nz, ny, nx), seed) if unit else np.random.default_rng(seed).standard_normal((3, nz, ny, nx))
    p = np.random.default_rng(seed + 1).standard_normal((4, nz, ny, nx))
    prm, op = both_params(**kw)
    ctx = P.Context(nx, ny, nz, lengths=lengths)
    return g, m, p, prm, op, ctx


@pytest.mark.parametrize("shape", [(6, 4, 1), (10, 6, 1), (12, 10, 1), (6, 6, 6), (20, 4, 6), (4, 12, 10)])
def test_mixed_sizes_match_dense(shape):
    nx, ny, nz = shape
    announce(f"dense parity, mixed sizes {shape}")
    g, m, p, prm, op, ctx = _case(nx, ny, nz, 3, lengths=(1.0, 0.8, 1.3), kw=dict(KW, dt=0.05), unit=False)
    M1, M2 = dense.hss_factors(g, op, m)
    A = dense.saddle_matrix(g, op, m)
    md, pd = dev(m), dev(p)
    z = host(P.fft_hss_apply(ctx, prm, md, pd)).ravel()
    assert_elem(z, np.linalg.solve(M2, np.linalg.solve(M1, p.ravel())), 1e-12, "apply")
    y = host(P.llg_matvec(ctx, prm, md, pd)).ravel()
    assert_elem(y, A @ p.ravel(), 1e-12, "matvec")
    ctx.close()


# each mixed length as the x half-length (nx = 2n), as ny and as nz
SHAPES = ([(2 * n, 8, 1) for n in MIXED if 2 * n <= 512 and n <= 256 and n not in (320, 384)]
          + [(8, n, 1) for n in MIXED] + [(4, 4, n) for n in MIXED]
          + [(24, 24, 24), (48, 48, 48), (40, 20, 12), (96, 48, 24), (20, 192, 10)])


@pytest.mark.parametrize("shape", SHAPES)
def test_mixed_sizes_match_fft_oracle(shape):
    nx, ny, nz = shape
    announce(f"fft-tier parity, mixed sizes {shape}")
    g, m, p, prm, op, ctx = _case(nx, ny, nz, 7)
    md, pd = dev(m), dev(p)
    for tr in (False, True):
        z = host(P.fft_hss_apply(ctx, prm, md, pd, transpose=tr))
        assert_elem(z, operators.hss_apply(g, op, m, p, transpose=tr), 1e-12, "apply")
        y = host(P.llg_matvec(ctx, prm, md, pd, transpose=tr))
        ref = operators.matvec_transpose(g, op, m, p) if tr else operators.matvec(g, op, m, p)
        assert_elem(y, ref, 1e-12, "matvec")
    ctx.close()


# cells with spacing about 1/20 keep k C_hat |xi|^2 moderate (plain GMRES needs
# a few hundred iterations at most); far stiffer cells need more refinement
# steps than the default limit, on every grid size
@pytest.mark.parametrize("shape,lengths", [((24, 24, 24), (1.0, 1.2, 0.9)), ((96, 40, 1), (4.0, 4.8, 1.0)),
                                           ((20, 12, 48), (1.0, 0.6, 2.4))])
def test_mixed_sizes_float32_and_solve(shape, lengths):
    nx, ny, nz = shape
    announce(f"float32 operators and FP32-IR solve, mixed sizes {shape}")
    g, m, p, prm, op, ctx = _case(nx, ny, nz, 11, lengths=lengths)
    m32, p32 = dev(m).float(), dev(p).float()
    mh, ph = host(m32), host(p32)  # the float32 inputs, exactly, in float64
    tol = fp32_bound(shape)
    z = host(P.fft_hss_apply_f32(ctx, prm, m32, p32))
    assert_elem(z, operators.hss_apply(g, op, mh, ph), tol, "f32 apply")
    y = host(P.llg_matvec_f32(ctx, prm, m32, p32))
    assert_elem(y, operators.matvec(g, op, mh, ph), tol, "f32 matvec")
    # the solves use a smooth magnetization (float32 refinement needs the
    # preconditioned system to be well conditioned in float32)
    ms = unit_field((nz, ny, nx), 12, smooth=8.0)
    b = steppers.rhs(g, op, ms)
    xref, _ = steppers.solve_saddle(g, op, ms, b, rtol=1e-12)
    x64, s64 = P.gmres_solve(ctx, prm, dev(ms), dev(b), rtol=1e-12)
    assert s64["converged"] == 1
    assert_elem(host(x64), xref, 1e-9, "fp64 x")
    x32, s32 = P.gmres_solve(ctx, prm, dev(ms), dev(b), rtol=1e-10, prec="fp32_ir")
    assert s32["converged"] == 1
    assert_elem(host(x32), xref, 1e-7, "fp32-ir x")
    ctx.close()


@pytest.mark.parametrize("shape,lengths", [((24, 24, 24), (2.0, 2.0, 2.0)), ((40, 24, 1), (1.0, 0.6, 1.0)),
                                           ((12, 20, 48), (0.5, 0.8, 1.9))])
def test_mixed_sizes_lower_order_field(shape, lengths):
    nx, ny, nz = shape
    announce(f"lower-order rhs/energy, mixed sizes {shape}")
    low = dict(demag=1.0, aniso_k=0.3, aniso_axis=(0.0, 0.6, 0.8), h_uniform=(0.1, 0.0, 0.2))
    g, m, p, prm, op, ctx = _case(nx, ny, nz, 5, lengths=lengths, kw=dict(KW, **low))
    b = host(P.llg_rhs(ctx, prm, dev(m)))
    assert_elem(b, steppers.rhs(g, op, m), 1e-13, "rhs")
    e = P.llg_energy(ctx, prm, dev(m))
    eref = steppers.energy(g, op, m)
    assert abs(e - eref) <= 1e-13 * abs(eref)
    ctx.close()
