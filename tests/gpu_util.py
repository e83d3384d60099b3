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


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def both_params(**kw):
    from oracle.operators import Params as OP
    return P.Params(**kw), OP(**kw)


def announce(msg):
    print(msg, flush=True)
