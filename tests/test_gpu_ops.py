"""GPU parity of the operators behind the C ABI: the saddle matvec, the split
FFT-HSS apply (plain and transposed) in float64 and float32, against the FP64
oracle -- the dense assembled matrices on tiny grids and the FFT tier on
grids that span several tiles with ragged column tiles, up to full workload
sizes."""

import numpy as np
import pytest
import torch

import paper_2607_15290_amd as P
from oracle import dense, operators
from oracle.grid import Grid
from tests.gpu_util import announce, both_params, dev, host, rel, unit_field

pytestmark = pytest.mark.gpu

KW = dict(alpha=0.1, cexc=1.0, dt=2e-3, theta=1.0, shift=0.5)


def _case(nx, ny, nz, seed, kw=KW, unit=True):
    h = 1.0 / nx
    g = Grid(nx, ny, nz, h=h)
    m = unit_field((nz, ny, nx), seed) if unit else np.random.default_rng(seed).standard_normal((3, nz, ny, nx))
    p = np.random.default_rng(seed + 1).standard_normal((4, nz, ny, nx))
    prm, op = both_params(**kw)
    ctx = P.Context(nx, ny, nz, h, 0)
    return g, m, p, prm, op, ctx


@pytest.mark.parametrize("shape", [(4, 4, 1), (8, 4, 1), (4, 8, 1), (8, 8, 1), (4, 4, 4), (8, 4, 4)])
@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_apply_and_matvec_match_dense(shape, theta):
    nx, ny, nz = shape
    announce(f"dense parity {shape} theta={theta}")
    kw = dict(KW, theta=theta, dt=0.05)
    g, m, p, prm, op, ctx = _case(nx, ny, nz, 3, kw, unit=False)
    M1, M2 = dense.hss_factors(g, op, m)
    A = dense.saddle_matrix(g, op, m)
    md, pd = dev(m), dev(p)
    z = host(P.fft_hss_apply(ctx, prm, md, pd)).ravel()
    zref = np.linalg.solve(M2, np.linalg.solve(M1, p.ravel()))
    assert rel(z, zref) <= 1e-12
    zt = host(P.fft_hss_apply(ctx, prm, md, pd, transpose=True)).ravel()
    assert rel(zt, np.linalg.solve((M1 @ M2).T, p.ravel())) <= 1e-12
    y = host(P.llg_matvec(ctx, prm, md, pd)).ravel()
    assert rel(y, A @ p.ravel()) <= 1e-12
    yt = host(P.llg_matvec(ctx, prm, md, pd, transpose=True)).ravel()
    assert rel(yt, A.T @ p.ravel()) <= 1e-12
    ctx.close()


SHAPES = [(16, 16, 1), (32, 64, 1), (128, 32, 1), (512, 8, 1), (16, 32, 8), (64, 16, 32), (32, 32, 32),
          (8, 128, 16), (256, 8, 4)]


@pytest.mark.parametrize("shape", SHAPES)
def test_operators_match_fft_oracle(shape):
    nx, ny, nz = shape
    announce(f"fft-tier parity {shape}")
    g, m, p, prm, op, ctx = _case(nx, ny, nz, 7)
    md, pd = dev(m), dev(p)
    for tr in (False, True):
        z = host(P.fft_hss_apply(ctx, prm, md, pd, transpose=tr))
        assert rel(z, operators.hss_apply(g, op, m, p, transpose=tr)) <= 1e-12
        y = host(P.llg_matvec(ctx, prm, md, pd, transpose=tr))
        ref = operators.matvec_transpose(g, op, m, p) if tr else operators.matvec(g, op, m, p)
        assert rel(y, ref) <= 1e-12
    # in-place apply (z aliases p)
    q = pd.clone()
    P.fft_hss_apply(ctx, prm, md, q, z=q)
    assert rel(host(q), operators.hss_apply(g, op, m, p)) <= 1e-12
    ctx.close()


@pytest.mark.parametrize("shape", [(16, 16, 1), (64, 32, 1), (32, 16, 16), (64, 64, 64)])
def test_float32_operators(shape):
    """float32 pipelines against the float64 oracle; bound: a few FFT passes
    of float32 rounding, 2e-6 relative."""
    nx, ny, nz = shape
    announce(f"fp32 parity {shape}")
    g, m, p, prm, op, ctx = _case(nx, ny, nz, 11)
    mf, pf = dev(m, torch.float32), dev(p, torch.float32)
    for tr in (False, True):
        z = host(P.fft_hss_apply_f32(ctx, prm, mf, pf, transpose=tr))
        assert rel(z, operators.hss_apply(g, op, m, p, transpose=tr)) <= 2e-6
        y = host(P.llg_matvec_f32(ctx, prm, mf, pf, transpose=tr))
        ref = operators.matvec_transpose(g, op, m, p) if tr else operators.matvec(g, op, m, p)
        assert rel(y, ref) <= 2e-6
    ctx.close()


def test_run_to_run_bitwise():
    g, m, p, prm, op, ctx = _case(64, 32, 16, 5)
    md, pd = dev(m), dev(p)
    a = host(P.fft_hss_apply(ctx, prm, md, pd))
    b = host(P.fft_hss_apply(ctx, prm, md, pd))
    assert np.array_equal(a, b)
    ctx.close()
