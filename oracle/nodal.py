"""Nodal algebra of the skew/constraint block (Sec. 3.1, eqs. (Bi), (S),
(Lambda); Sec. 3.2, eq. "inverse S").

Test infrastructure: part of the float64 CPU oracle (see the package docstring).

At node i the skew/constraint block acting on (v_i, r_i) is

    S~_i = [[Lambda_i, B_i^T], [-B_i, 0]],  B_i = m_i^T,  Lambda_i = [m_i]_x,

so Lambda_i v = m_i x v.  (S~_i + lambda I)^{-1} is the printed 4x4 matrix of
eq. "inverse S" written with p = m / lambda.
"""

import numpy as np


def cross(a, b):
    """Pointwise a x b for fields of shape (3, ...)."""
    return np.stack([a[1] * b[2] - a[2] * b[1],
                     a[2] * b[0] - a[0] * b[2],
                     a[0] * b[1] - a[1] * b[0]])


def dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def lambda_matrix(mi):
    """Lambda_i of eq. (Lambda) for one node (3-vector)."""
    m1, m2, m3 = mi
    return np.array([[0.0, -m3, m2], [m3, 0.0, -m1], [-m2, m1, 0.0]])


def s_tilde(mi):
    """The 4x4 nodal block S~_i of eq. (S)."""
    out = np.zeros((4, 4))
    out[:3, :3] = lambda_matrix(mi)
    out[:3, 3] = mi
    out[3, :3] = -np.asarray(mi)
    return out


def inverse_s_matrix(mi, lam):
    """(S~_i + lambda I)^{-1} exactly as printed in eq. "inverse S"."""
    p1, p2, p3 = np.asarray(mi, dtype=np.float64) / lam
    mat = np.array([[1.0, p3, -p2, -p1],
                    [-p3, 1.0, p1, -p2],
                    [p2, -p1, 1.0, -p3],
                    [p1, p2, p3, 1.0]])
    return mat / (lam * (p1 * p1 + p2 * p2 + p3 * p3 + 1.0))


def s_apply(m, x):
    """(S x) for the whole grid: (m x v + m r, -m . v)."""
    v, r = x[:3], x[3]
    out = np.empty_like(x)
    out[:3] = cross(m, v) + m * r
    out[3] = -dot(m, v)
    return out


def s_shift_solve(m, w, lam):
    """(S + lambda I)^{-1} w node by node, using the matrix of eq.
    "inverse S" (p = m / lambda), applied to all nodes at once."""
    p = m / lam
    p1, p2, p3 = p
    w1, w2, w3, w4 = w
    scale = 1.0 / (lam * (p1 * p1 + p2 * p2 + p3 * p3 + 1.0))
    out = np.empty_like(w)
    out[0] = (w1 + p3 * w2 - p2 * w3 - p1 * w4) * scale
    out[1] = (-p3 * w1 + w2 + p1 * w3 - p2 * w4) * scale
    out[2] = (p2 * w1 - p1 * w2 + w3 - p3 * w4) * scale
    out[3] = (p1 * w1 + p2 * w2 + p3 * w3 + w4) * scale
    return out


def s_shift_solve_transpose(m, w, lam):
    """(S + lambda I)^{-T} w: the transpose of the printed matrix."""
    p = m / lam
    p1, p2, p3 = p
    w1, w2, w3, w4 = w
    scale = 1.0 / (lam * (p1 * p1 + p2 * p2 + p3 * p3 + 1.0))
    out = np.empty_like(w)
    out[0] = (w1 - p3 * w2 + p2 * w3 + p1 * w4) * scale
    out[1] = (p3 * w1 + w2 - p1 * w3 + p2 * w4) * scale
    out[2] = (-p2 * w1 + p1 * w2 + w3 + p3 * w4) * scale
    out[3] = (-p1 * w1 - p2 * w2 - p3 * w3 + w4) * scale
    return out
