"""Python binding of the C ABI (include/llg.h) on torch tensors.

Argument marshalling only: every step of the numerical path runs in the HIP
library.  Tensors must be contiguous torch tensors on the context's GPU,
float64 (float32 for the *_f32 functions), with 3 planes (m, v) or 4 planes
(saddle unknowns (v1, v2, v3, lam)) of nx*ny*nz nodes each; the shape is free
as long as the element count matches (e.g. (4, nz, ny, nx)).
"""

import ctypes
from dataclasses import dataclass, field
from typing import Optional

import torch

from . import _lib as L

FP64 = 0
FP32_IR = 1
FP32_IR_LEFT = 2
_PREC = {"fp64": FP64, "fp32_ir": FP32_IR, "fp32_ir_left": FP32_IR_LEFT, FP64: FP64, FP32_IR: FP32_IR,
         FP32_IR_LEFT: FP32_IR_LEFT}


class LLGError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        self.name = L.STATUS.get(status, str(status))
        msg = L.load().llg_last_error().decode()
        super().__init__(f"{where}: {self.name}: {msg}")


def _check(status, where):
    if status != 0:
        raise LLGError(status, where)


@dataclass
class Params:
    """Physical parameters (llg_params): alpha, cexc, dt (k), theta, shift
    (the HSS lambda), uniform applied field, optional spatial field tensor
    (3 planes, float64, on the GPU), demagnetizing-field coefficient (0 or
    1), uniaxial anisotropy coefficient K and unit easy axis."""
    alpha: float = 0.2
    cexc: float = 1.0
    dt: float = 1e-2
    theta: float = 1.0
    shift: float = 0.5
    h_uniform: tuple = (0.0, 0.0, 0.0)
    h_field: Optional[torch.Tensor] = field(default=None, repr=False)
    demag: float = 0.0
    aniso_k: float = 0.0
    aniso_axis: tuple = (0.0, 0.0, 1.0)

    def c_struct(self, ctx=None):
        """The llg_params struct.  With a context, the spatial field (read by the
        kernels through a raw pointer) is checked against that context's grid."""
        if self.h_field is not None and ctx is not None:
            ctx.check(self.h_field, 3, name="h_field")
        p = L.LLGParams()
        p.alpha, p.cexc, p.dt, p.theta, p.shift = (float(self.alpha), float(self.cexc), float(self.dt),
                                                   float(self.theta), float(self.shift))
        for i in range(3):
            p.h_uniform[i] = float(self.h_uniform[i])
        p.h_field = self.h_field.data_ptr() if self.h_field is not None else None
        p.demag, p.aniso_k = float(self.demag), float(self.aniso_k)
        for i in range(3):
            p.aniso_axis[i] = float(self.aniso_axis[i])
        return p


ORTH = {"dcgs2": 0, "cgs2": 1, 0: 0, 1: 1}
PRECOND = {"fft_hss": 0, "symmetric": 1, "none": 2, 0: 0, 1: 1, 2: 2}
PICARD_NORM = {"midpoint": 0, "velocity": 1, 0: 0, 1: 1}
FUSE_UPDATE = {"auto": 0, "always": 1, "never": -1, 0: 0, 1: 1, -1: -1}


def _opts(restart, maxiter, rtol, prec, inner_rtol, max_outer, use_x0, orth="dcgs2", precond="fft_hss",
          picard_norm="midpoint", transpose=False, fuse_update="auto"):
    o = L.LLGSolverOpts()
    o.transpose = int(bool(transpose))
    o.fuse_update = FUSE_UPDATE[fuse_update]
    o.orth = ORTH[orth]
    o.precond = PRECOND[precond]
    o.picard_norm = PICARD_NORM[picard_norm]
    o.restart, o.maxiter, o.max_outer, o.use_x0 = int(restart), int(maxiter), int(max_outer), int(use_x0)
    o.rtol, o.inner_rtol = float(rtol), float(inner_rtol)
    o.prec = _PREC[prec]
    return o


def _stats_dict(s):
    return {name: getattr(s, name) for name, _ in s._fields_}


def aligned_ptr(t, name="tensor"):
    """Device address of a tensor, which the C ABI requires 16-byte aligned."""
    ptr = t.data_ptr()
    if ptr % 16:
        raise ValueError(f"{name} must start at a 16-byte aligned address")
    return ptr


class Context:
    """An llg_ctx: grid nx x ny x nz (nz = 1 for 2-D) on one GPU, with either
    one spacing h (cell lengths n h) or explicit cell lengths
    lengths = (lx, ly, lz) (llg_ctx_create_cell)."""

    def __init__(self, nx, ny, nz=1, h=None, device=0, lengths=None):
        self.lib = L.load()
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.device = torch.device("cuda", int(device))
        self.ng = self.nx * self.ny * self.nz
        if lengths is None:
            self.h = float(1.0 / nx if h is None else h)
            self.lengths = (self.nx * self.h, self.ny * self.h, self.nz * self.h)
        else:
            self.lengths = tuple(float(v) for v in lengths)
            self.h = None
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            if lengths is None:
                s = self.lib.llg_ctx_create(ctypes.byref(handle), self.nx, self.ny, self.nz, self.h, int(device))
            else:
                s = self.lib.llg_ctx_create_cell(ctypes.byref(handle), self.nx, self.ny, self.nz, *self.lengths,
                                                 int(device))
            _check(s, "llg_ctx_create")
        self.handle = handle
        self._work = {}

    def close(self):
        if getattr(self, "handle", None):
            self.lib.llg_ctx_destroy(self.handle)
            self.handle = None
            self._work = {}

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace(self, restart=30, prec="fp64"):
        """The Krylov workspace for (restart, prec), one at a time: switching
        frees the previous one and hands torch's cached blocks back to the
        device first, so that two workspaces of a large grid (hundreds of GB
        each) never need to coexist in the cache."""
        key = (int(restart), _PREC[prec])
        if key not in self._work:
            nbytes = self.lib.llg_workspace_bytes(self.handle, key[0], key[1])
            if nbytes == 0:
                raise ValueError("bad workspace request")
            if self._work:
                self._work.clear()
                torch.cuda.empty_cache()
            self._work[key] = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return self._work[key]

    def stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def check(self, t, planes, dtype=torch.float64, name="tensor"):
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.device != self.device or t.dtype != dtype or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {dtype} tensor on {self.device}")
        if t.numel() != planes * self.ng:
            raise ValueError(f"{name} must hold {planes} planes of {self.ng} nodes")
        return aligned_ptr(t, name)

    def new(self, planes, dtype=torch.float64):
        return torch.empty((planes, self.nz, self.ny, self.nx), dtype=dtype, device=self.device)


def llg_matvec(ctx, params, m, x, y=None, transpose=False):
    """y = A x (or A^T x).  See llg_matvec in include/llg.h."""
    y = ctx.new(4) if y is None else y
    p = params.c_struct(ctx)
    _check(ctx.lib.llg_matvec(ctx.handle, ctypes.byref(p), ctx.check(m, 3, name="m"), ctx.check(x, 4, name="x"),
                              ctx.check(y, 4, name="y"), int(bool(transpose)), ctx.stream()), "llg_matvec")
    return y


def fft_hss_apply(ctx, params, m, p, z=None, transpose=False):
    """z = M^{-1} p (or M^{-T} p).  See fft_hss_apply in include/llg.h."""
    z = ctx.new(4) if z is None else z
    pr = params.c_struct(ctx)
    _check(ctx.lib.fft_hss_apply(ctx.handle, ctypes.byref(pr), ctx.check(m, 3, name="m"), ctx.check(p, 4, name="p"),
                                 ctx.check(z, 4, name="z"), int(bool(transpose)), ctx.stream()), "fft_hss_apply")
    return z


def llg_matvec_f32(ctx, params, m, x, y=None, transpose=False):
    y = ctx.new(4, torch.float32) if y is None else y
    p = params.c_struct(ctx)
    f = torch.float32
    _check(ctx.lib.llg_matvec_f32(ctx.handle, ctypes.byref(p), ctx.check(m, 3, f, "m"), ctx.check(x, 4, f, "x"),
                                  ctx.check(y, 4, f, "y"), int(bool(transpose)), ctx.stream()), "llg_matvec_f32")
    return y


def fft_hss_apply_f32(ctx, params, m, p, z=None, transpose=False):
    z = ctx.new(4, torch.float32) if z is None else z
    pr = params.c_struct(ctx)
    f = torch.float32
    _check(ctx.lib.fft_hss_apply_f32(ctx.handle, ctypes.byref(pr), ctx.check(m, 3, f, "m"), ctx.check(p, 4, f, "p"),
                                     ctx.check(z, 4, f, "z"), int(bool(transpose)), ctx.stream()),
           "fft_hss_apply_f32")
    return z


def _basis_args(ctx, basis):
    """(pointer, count, stride, dots tensor) of optional Arnoldi basis vectors:
    a contiguous float64 tensor of nb vectors of 4 planes each."""
    if basis is None:
        return None, 0, 0, None
    if basis.dtype != torch.float64 or not basis.is_contiguous() or basis.device != ctx.device:
        raise ValueError(f"basis must be a contiguous float64 tensor on {ctx.device}")
    if basis.numel() % (4 * ctx.ng):
        raise ValueError("basis must hold whole vectors of 4 planes")
    nb = basis.numel() // (4 * ctx.ng)
    dots = torch.empty(max(nb, 1), dtype=torch.float64, device=ctx.device)
    return aligned_ptr(basis, "basis"), nb, 4 * ctx.ng, dots


def llg_precond_op(ctx, params, m, x, y=None, basis=None):
    """y = M^{-1} A x in one pipeline; with basis (nb vectors of 4 planes) also
    the Arnoldi products basis_q . y.  Returns y, or (y, dots) with a basis.
    See llg_precond_op in include/llg.h."""
    y = ctx.new(4) if y is None else y
    pr = params.c_struct(ctx)
    bp, nb, ld, dots = _basis_args(ctx, basis)
    _check(ctx.lib.llg_precond_op(ctx.handle, ctypes.byref(pr), ctx.check(m, 3, name="m"), ctx.check(x, 4, name="x"),
                                  ctx.check(y, 4, name="y"), bp, nb, ld,
                                  aligned_ptr(dots, "dots") if dots is not None else None, ctx.stream()),
           "llg_precond_op")
    return y if basis is None else (y, dots)


def llg_precond_op_f32(ctx, params, m, x, side=0, z=None, y=None, basis=None):
    """float32 preconditioned operators between float64 vectors: side 0,
    y = M^{-1} A x (one float32 pipeline); side 1, z = M^{-1} x (float32) and
    y = A z.  m is float32.  Returns (y, dots) (dots None without a basis).
    See llg_precond_op_f32 in include/llg.h."""
    y = ctx.new(4) if y is None else y
    if side == 1 and z is None:
        z = ctx.new(4, torch.float32)
    pr = params.c_struct(ctx)
    bp, nb, ld, dots = _basis_args(ctx, basis)
    f = torch.float32
    _check(ctx.lib.llg_precond_op_f32(ctx.handle, ctypes.byref(pr), ctx.check(m, 3, f, "m"),
                                      ctx.check(x, 4, name="x"), ctx.check(y, 4, name="y"),
                                      ctx.check(z, 4, f, "z") if z is not None else None, int(side), bp, nb, ld,
                                      aligned_ptr(dots, "dots") if dots is not None else None, ctx.stream()),
           "llg_precond_op_f32")
    return y, dots


def gmres_solve(ctx, params, m, b, x=None, use_x0=False, restart=30, rtol=1e-10, maxiter=3000, prec="fp64",
                inner_rtol=1e-5, max_outer=20, check=True, orth="dcgs2", precond="fft_hss", transpose=False,
                fuse_update="auto"):
    """Solve A(m) x = b (or A(m)^T x = b with transpose); returns (x, stats).
    fuse_update: "auto", "always" or "never" (llg_solver_opts::fuse_update).
    See gmres_solve in include/llg.h."""
    if x is None:
        x = ctx.new(4)
        use_x0 = False
    o = _opts(restart, maxiter, rtol, prec, inner_rtol, max_outer, use_x0, orth, precond, transpose=transpose,
              fuse_update=fuse_update)
    st = L.LLGSolverStats()
    work = ctx.workspace(restart, prec)
    pr = params.c_struct(ctx)
    s = ctx.lib.gmres_solve(ctx.handle, ctypes.byref(pr), ctx.check(m, 3, name="m"), ctx.check(b, 4, name="b"),
                            ctx.check(x, 4, name="x"), ctypes.byref(o), ctypes.byref(st), work.data_ptr(),
                            work.numel(), ctx.stream())
    stats = _stats_dict(st)
    stats["status"] = L.STATUS.get(s, s)
    if check:
        _check(s, "gmres_solve")
    return x, stats


def gmres_solve_noalloc(ctx, params, m, b, x=None, use_x0=False, restart=30, rtol=1e-10, maxiter=3000,
                        prec="fp64", inner_rtol=1e-5, max_outer=20, check=True, orth="dcgs2", precond="fft_hss",
                        fuse_update="auto"):
    """gmres_solve on the library's static workspace (no caller workspace,
    no device allocation in the call); returns (x, stats).  See
    gmres_solve_noalloc in include/llg.h."""
    if x is None:
        x = ctx.new(4)
        use_x0 = False
    o = _opts(restart, maxiter, rtol, prec, inner_rtol, max_outer, use_x0, orth, precond, fuse_update=fuse_update)
    st = L.LLGSolverStats()
    pr = params.c_struct(ctx)
    s = ctx.lib.gmres_solve_noalloc(ctx.handle, ctypes.byref(pr), ctx.check(m, 3, name="m"),
                                    ctx.check(b, 4, name="b"), ctx.check(x, 4, name="x"), ctypes.byref(o),
                                    ctypes.byref(st), ctx.stream())
    stats = _stats_dict(st)
    stats["status"] = L.STATUS.get(s, s)
    if check:
        _check(s, "gmres_solve_noalloc")
    return x, stats


def llg_step_euler(ctx, params, m, v_out=None, lam_out=None, restart=30, rtol=1e-10, maxiter=3000, prec="fp64",
                   inner_rtol=1e-5, max_outer=20, check=True, orth="dcgs2", fuse_update="auto"):
    """One projected Euler step; m is updated in place.  Returns stats."""
    o = _opts(restart, maxiter, rtol, prec, inner_rtol, max_outer, 0, orth, fuse_update=fuse_update)
    st = L.LLGStepStats()
    work = ctx.workspace(restart, prec)
    pr = params.c_struct(ctx)
    s = ctx.lib.llg_step_euler(ctx.handle, ctypes.byref(pr), ctx.check(m, 3, name="m"),
                               ctx.check(v_out, 3, name="v_out") if v_out is not None else None,
                               ctx.check(lam_out, 1, name="lam_out") if lam_out is not None else None,
                               ctypes.byref(o), ctypes.byref(st), work.data_ptr(), work.numel(), ctx.stream())
    stats = _stats_dict(st)
    stats["status"] = L.STATUS.get(s, s)
    if check:
        _check(s, "llg_step_euler")
    return stats


def llg_step_midpoint(ctx, params, m, v_half=None, lam=None, picard_tol=1e-10, picard_max=50, restart=30,
                      rtol=1e-10, maxiter=3000, prec="fp64", inner_rtol=1e-5, max_outer=20, check=True,
                      orth="dcgs2", picard_norm="midpoint", fuse_update="auto"):
    """One midpoint step; m, v_half, lam updated in place.  picard_norm:
    "midpoint" (change of the frozen midpoint, default) or "velocity".
    Returns stats."""
    o = _opts(restart, maxiter, rtol, prec, inner_rtol, max_outer, 1, orth, picard_norm=picard_norm,
              fuse_update=fuse_update)
    st = L.LLGStepStats()
    work = ctx.workspace(restart, prec)
    pr = params.c_struct(ctx)
    s = ctx.lib.llg_step_midpoint(ctx.handle, ctypes.byref(pr), ctx.check(m, 3, name="m"),
                                  ctx.check(v_half, 3, name="v_half") if v_half is not None else None,
                                  ctx.check(lam, 1, name="lam") if lam is not None else None,
                                  float(picard_tol), int(picard_max), ctypes.byref(o), ctypes.byref(st),
                                  work.data_ptr(), work.numel(), ctx.stream())
    stats = _stats_dict(st)
    stats["status"] = L.STATUS.get(s, s)
    if check:
        _check(s, "llg_step_midpoint")
    return stats


def llg_step_midpoint_adjoint(ctx, params, m_n, v, lam, gbar, hbar_field=None, hbar_uniform=None, restart=30,
                              rtol=1e-12, maxiter=3000, check=True, orth="dcgs2", fuse_update="auto"):
    """Back-propagate gbar (in/out) through one converged midpoint step.
    hbar_field (tensor, +=) and hbar_uniform (list of 3 floats, +=) are
    accumulated.  Returns (hbar_uniform, stats)."""
    o = _opts(restart, maxiter, rtol, "fp64", 1e-5, 1, 0, orth, fuse_update=fuse_update)
    st = L.LLGSolverStats()
    work = ctx.workspace(restart, "fp64")
    hu = (ctypes.c_double * 3)(*(hbar_uniform if hbar_uniform is not None else (0.0, 0.0, 0.0)))
    pr = params.c_struct(ctx)
    s = ctx.lib.llg_step_midpoint_adjoint(ctx.handle, ctypes.byref(pr), ctx.check(m_n, 3, name="m_n"),
                                          ctx.check(v, 3, name="v"), ctx.check(lam, 1, name="lam"),
                                          ctx.check(gbar, 3, name="gbar"),
                                          ctx.check(hbar_field, 3, name="hbar_field") if hbar_field is not None else None,
                                          ctypes.cast(hu, L.c_double_p), ctypes.byref(o), ctypes.byref(st),
                                          work.data_ptr(), work.numel(), ctx.stream())
    stats = _stats_dict(st)
    stats["status"] = L.STATUS.get(s, s)
    if check:
        _check(s, "llg_step_midpoint_adjoint")
    return [hu[0], hu[1], hu[2]], stats


def llg_rhs(ctx, params, m, b=None):
    """b = (C_hat Delta_N m + (1+alpha^2) h_low(m), 0).  See llg_rhs in include/llg.h."""
    b = ctx.new(4) if b is None else b
    pr = params.c_struct(ctx)
    _check(ctx.lib.llg_rhs(ctx.handle, ctypes.byref(pr), ctx.check(m, 3, name="m"), ctx.check(b, 4, name="b"),
                           ctx.stream()), "llg_rhs")
    return b


def llg_energy(ctx, params, m):
    e = ctypes.c_double()
    pr = params.c_struct(ctx)
    _check(ctx.lib.llg_energy(ctx.handle, ctypes.byref(pr), ctx.check(m, 3, name="m"), ctypes.byref(e), ctx.stream()),
           "llg_energy")
    return e.value


def llg_profile_enable(ctx, enable=True):
    """Start (clear) or stop per-kernel HIP-event timing in the library."""
    _check(ctx.lib.llg_profile_enable(ctx.handle, int(bool(enable))), "llg_profile_enable")


def llg_profile_select(ctx, kinds=None):
    """Record only the named kernel kinds (list of names; None: all)."""
    arg = None if not kinds else ",".join(kinds).encode()
    _check(ctx.lib.llg_profile_select(ctx.handle, arg), "llg_profile_select")


def llg_profile_read(ctx):
    """Per-kernel totals recorded since llg_profile_enable:
    {name: dict(launches, total_ms, bytes)}."""
    buf = (L.LLGKernelProfile * 64)()
    n = ctx.lib.llg_profile_read(ctx.handle, buf, 64)
    if n < 0:
        raise LLGError(6, "llg_profile_read")
    return {buf[i].name.decode(): dict(launches=buf[i].launches, total_ms=buf[i].total_ms, bytes=buf[i].bytes)
            for i in range(min(n, 64))}
