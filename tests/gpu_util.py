"""Helpers of the GPU parity tests: device transfer and seeded fields."""

import numpy as np
import torch

import paper_2607_15290_amd as P


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda:0", dtype=dtype)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def unit_field(shape, seed, smooth=None):
    rng = np.random.default_rng(seed)
    m = rng.standard_normal((3,) + shape)
    if smooth:
        k = [np.fft.fftfreq(n, 1.0 / n) for n in shape]
        kk = k[0][:, None, None] ** 2 + k[1][None, :, None] ** 2 + k[2][None, None, :] ** 2
        m = np.fft.ifftn(np.fft.fftn(m, axes=(1, 2, 3)) * np.exp(-kk / smooth), axes=(1, 2, 3)).real
    return m / np.sqrt((m * m).sum(0))


def elem_err(a, ref):
    """Element-wise parity measure: max_i |a_i - ref_i| / max_i |ref_i|.  One
    element off by more than the bound fails, however many are right."""
    a = np.asarray(a, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    assert a.shape == ref.shape, (a.shape, ref.shape)
    scale = float(np.max(np.abs(ref)))
    return float(np.max(np.abs(a - ref))) / (scale if scale > 0 else 1.0)


def assert_elem(a, ref, tol, what=""):
    """Assert elem_err(a, ref) <= tol and print the measured value."""
    e = elem_err(a, ref)
    print(f"  {what} elem_err {e:.3e} (bound {tol:.1e})", flush=True)
    assert e <= tol, (what, e, tol)


def both_params(**kw):
    from oracle.operators import Params as OP
    return P.Params(**kw), OP(**kw)


def announce(msg):
    print(msg, flush=True)
