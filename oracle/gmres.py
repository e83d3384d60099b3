"""Restarted GMRES and flexible GMRES with iterative refinement.

Test infrastructure: part of the float64 CPU oracle (see the package docstring).

The paper preconditions GMRES on the left with the split FFT-HSS operator
(Sec. 3.2) and accepts a solve by the relative residual of the full saddle
system (Sec. 4.1).  This is the textbook restarted GMRES (Saad, Iterative
Methods for Sparse Linear Systems, Alg. 6.9 with left preconditioning) using
modified Gram-Schmidt Arnoldi and Givens rotations.

Stopping rule (the paper names only "relative linear tolerance"; this reading
is shared with the library): with target = rtol ||b||_2 and the true residual
rho = ||b - A x||_2 at the start of a cycle, the cycle stops once the
preconditioned residual estimate |g_{j+1}| falls to (target / rho) times its
starting value beta = ||M^{-1} r||_2, or at the restart length.  The solve is
accepted only when the recomputed true residual satisfies rho <= target;
otherwise a new cycle starts from the updated iterate.

The precision form (FGMRES-IR) is GMRES-based iterative refinement (Carson and
Higham 2017) with flexible GMRES (Saad 1993) as the inner solver; in the
oracle every operation is float64.
"""

import numpy as np


def _givens(a, b):
    if b == 0.0:
        return 1.0, 0.0
    r = np.hypot(a, b)
    return a / r, b / r


def gmres(apply_a, apply_m, b, x0=None, restart=30, rtol=1e-10, maxiter=2000):
    """Left-preconditioned restarted GMRES on M^{-1} A x = M^{-1} b.

    apply_a, apply_m: callables on arrays shaped like b.
    Returns (x, info) with info = dict(iters, restarts, converged,
    rel_res_true, rel_res_prec, cycles).
    """
    shape = b.shape
    bv = b.ravel()
    bnorm = np.linalg.norm(bv)
    x = np.zeros_like(bv) if x0 is None else np.array(x0, dtype=np.float64).ravel().copy()
    info = dict(iters=0, restarts=0, converged=False, rel_res_true=0.0, rel_res_prec=0.0, cycles=[])
    if bnorm == 0.0:
        info.update(converged=True)
        return np.zeros(shape), info
    target = rtol * bnorm
    r = bv - apply_a(x.reshape(shape)).ravel() if x0 is not None else bv.copy()
    rho = np.linalg.norm(r)
    while True:
        info["rel_res_true"] = rho / bnorm
        if rho <= target:
            info["converged"] = True
            break
        if info["iters"] >= maxiter:
            break
        if info["cycles"]:
            info["restarts"] += 1
        z = apply_m(r.reshape(shape)).ravel()
        beta = np.linalg.norm(z)
        eta = target / rho
        m = restart
        V = np.zeros((m + 1, bv.size))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        gvec = np.zeros(m + 1)
        gvec[0] = beta
        V[0] = z / beta
        j_done = 0
        for j in range(m):
            w = apply_m(apply_a(V[j].reshape(shape))).ravel()
            for i in range(j + 1):  # modified Gram-Schmidt
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):  # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            cs[j], sn[j] = _givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            gvec[j + 1] = -sn[j] * gvec[j]
            gvec[j] = cs[j] * gvec[j]
            info["iters"] += 1
            j_done = j + 1
            if abs(gvec[j + 1]) <= eta * beta or info["iters"] >= maxiter:
                break
        y = np.zeros(j_done)
        for i in range(j_done - 1, -1, -1):  # back substitution
            y[i] = (gvec[i] - np.dot(H[i, i + 1:j_done], y[i + 1:])) / H[i, i]
        x = x + V[:j_done].T @ y
        info["rel_res_prec"] = abs(gvec[j_done]) / np.linalg.norm(apply_m(b).ravel())
        info["cycles"].append(j_done)
        r = bv - apply_a(x.reshape(shape)).ravel()
        rho = np.linalg.norm(r)
    return x.reshape(shape), info


def gmres_right(apply_a, apply_m, b, x0=None, restart=30, rtol=1e-10, maxiter=2000):
    """Right-preconditioned restarted GMRES (Saad, Alg. 9.5): A M^{-1} u = r
    from u = 0 in each cycle, x += M^{-1} V y at the cycle's end.  The cycle's
    residual estimate |g_{j+1}| is the true residual of the iterate (in exact
    arithmetic), so a cycle stops when it reaches rtol ||b||; the solve is
    accepted on the recomputed true residual, as in ``gmres``.
    Returns (x, info) like ``gmres``."""
    shape = b.shape
    bv = b.ravel()
    bnorm = np.linalg.norm(bv)
    x = np.zeros_like(bv) if x0 is None else np.array(x0, dtype=np.float64).ravel().copy()
    info = dict(iters=0, restarts=0, converged=False, rel_res_true=0.0, rel_res_prec=0.0, cycles=[])
    if bnorm == 0.0:
        info.update(converged=True)
        return np.zeros(shape), info
    target = rtol * bnorm
    r = bv - apply_a(x.reshape(shape)).ravel() if x0 is not None else bv.copy()
    rho = np.linalg.norm(r)
    while True:
        info["rel_res_true"] = rho / bnorm
        if rho <= target:
            info["converged"] = True
            break
        if info["iters"] >= maxiter:
            break
        if info["cycles"]:
            info["restarts"] += 1
        m = restart
        V = np.zeros((m + 1, bv.size))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        gvec = np.zeros(m + 1)
        gvec[0] = rho
        V[0] = r / rho
        j_done = 0
        for j in range(m):
            w = apply_a(apply_m(V[j].reshape(shape))).ravel()
            for i in range(j + 1):  # modified Gram-Schmidt
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            cs[j], sn[j] = _givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            gvec[j + 1] = -sn[j] * gvec[j]
            gvec[j] = cs[j] * gvec[j]
            info["iters"] += 1
            j_done = j + 1
            if abs(gvec[j + 1]) <= target or info["iters"] >= maxiter:
                break
        y = np.zeros(j_done)
        for i in range(j_done - 1, -1, -1):
            y[i] = (gvec[i] - np.dot(H[i, i + 1:j_done], y[i + 1:])) / H[i, i]
        x = x + apply_m((V[:j_done].T @ y).reshape(shape)).ravel()
        info["rel_res_prec"] = abs(gvec[j_done]) / bnorm
        info["cycles"].append(j_done)
        r = bv - apply_a(x.reshape(shape)).ravel()
        rho = np.linalg.norm(r)
    return x.reshape(shape), info


def fgmres_cycle(apply_a, apply_m, r, restart, inner_rtol):
    """One right-preconditioned flexible GMRES cycle on A d = r from d = 0.

    Stops when the residual estimate |g_{j+1}| <= inner_rtol ||r|| or after
    ``restart`` steps.  Returns (d, steps)."""
    shape = r.shape
    rv = r.ravel()
    beta = np.linalg.norm(rv)
    if beta == 0.0:
        return np.zeros(shape), 0
    m = restart
    V = np.zeros((m + 1, rv.size))
    Z = np.zeros((m, rv.size))
    H = np.zeros((m + 1, m))
    cs = np.zeros(m)
    sn = np.zeros(m)
    gvec = np.zeros(m + 1)
    gvec[0] = beta
    V[0] = rv / beta
    j_done = 0
    for j in range(m):
        Z[j] = apply_m(V[j].reshape(shape)).ravel()
        w = apply_a(Z[j].reshape(shape)).ravel()
        for i in range(j + 1):
            H[i, j] = np.dot(w, V[i])
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] > 0.0:
            V[j + 1] = w / H[j + 1, j]
        for i in range(j):
            t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
            H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
            H[i, j] = t
        cs[j], sn[j] = _givens(H[j, j], H[j + 1, j])
        H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
        H[j + 1, j] = 0.0
        gvec[j + 1] = -sn[j] * gvec[j]
        gvec[j] = cs[j] * gvec[j]
        j_done = j + 1
        if abs(gvec[j + 1]) <= inner_rtol * beta:
            break
    y = np.zeros(j_done)
    for i in range(j_done - 1, -1, -1):
        y[i] = (gvec[i] - np.dot(H[i, i + 1:j_done], y[i + 1:])) / H[i, i]
    return (Z[:j_done].T @ y).reshape(shape), j_done


def left_cycle(apply_a, apply_m, r, restart, inner_rtol):
    """One left-preconditioned GMRES cycle on M^{-1} A d = M^{-1} r from d = 0:
    stops when the preconditioned residual estimate |g_{j+1}| <= inner_rtol
    ||M^{-1} r|| or after ``restart`` steps.  Returns (d, steps)."""
    shape = r.shape
    z = apply_m(r).ravel()
    beta = np.linalg.norm(z)
    if beta == 0.0:
        return np.zeros(shape), 0
    m = restart
    V = np.zeros((m + 1, z.size))
    H = np.zeros((m + 1, m))
    cs = np.zeros(m)
    sn = np.zeros(m)
    gvec = np.zeros(m + 1)
    gvec[0] = beta
    V[0] = z / beta
    j_done = 0
    for j in range(m):
        w = apply_m(apply_a(V[j].reshape(shape))).ravel()
        for i in range(j + 1):
            H[i, j] = np.dot(w, V[i])
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        if H[j + 1, j] > 0.0:
            V[j + 1] = w / H[j + 1, j]
        for i in range(j):
            t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
            H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
            H[i, j] = t
        cs[j], sn[j] = _givens(H[j, j], H[j + 1, j])
        H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
        H[j + 1, j] = 0.0
        gvec[j + 1] = -sn[j] * gvec[j]
        gvec[j] = cs[j] * gvec[j]
        j_done = j + 1
        if abs(gvec[j + 1]) <= inner_rtol * beta:
            break
    y = np.zeros(j_done)
    for i in range(j_done - 1, -1, -1):
        y[i] = (gvec[i] - np.dot(H[i, i + 1:j_done], y[i + 1:])) / H[i, i]
    return (V[:j_done].T @ y).reshape(shape), j_done


def fgmres_ir(apply_a, apply_m, b, x0=None, restart=30, rtol=1e-10, inner_rtol=1e-6,
              max_outer=20, inner="flexible"):
    """Iterative refinement: r = b - A x; A d = r by one inner Krylov cycle;
    x += d; until ||r|| <= rtol ||b||.

    inner = "flexible": a right-preconditioned flexible GMRES cycle (the
    precision form); inner = "left": a left-preconditioned GMRES cycle (the
    variant whose operator is M^{-1} A).  Reading of the inner tolerance
    shared with the library: a cycle never asks for more than the outer
    target needs, so it stops at the relative reduction
    max(inner_rtol, rtol ||b|| / ||r||)."""
    bnorm = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    info = dict(iters=0, outer_steps=0, converged=False, rel_res_true=0.0)
    if bnorm == 0.0:
        info["converged"] = True
        return np.zeros_like(b), info
    cycle = fgmres_cycle if inner == "flexible" else left_cycle
    r = b - apply_a(x)
    rho = np.linalg.norm(r)
    while rho > rtol * bnorm and info["outer_steps"] < max_outer:
        eta = max(inner_rtol, rtol * bnorm / rho)
        d, steps = cycle(apply_a, apply_m, r, restart, eta)
        x = x + d
        info["iters"] += steps
        info["outer_steps"] += 1
        r = b - apply_a(x)
        rho = np.linalg.norm(r)
    info["rel_res_true"] = rho / bnorm
    info["converged"] = bool(rho <= rtol * bnorm)
    return x, info
