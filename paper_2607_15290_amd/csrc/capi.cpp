// C ABI of the library (include/llg.h): context, argument checks, the
// operator entry points, the GMRES drivers and the time steppers.
//
// Host code only; every step of the numerical path runs in the HIP kernels of
// the other translation units.  The host keeps the small Hessenberg least-
// squares problem (Givens rotations, back substitution) of GMRES, which needs
// j + 2 scalars per Arnoldi step read back from the device.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <functional>
#include <initializer_list>
#include <string>
#include <vector>

#include "krylov.h"

struct llg_ctx {
  llg::Ctx c;
};

namespace llg {

Profiler* profiler_new();
void profiler_delete(Profiler* p);
void profiler_enable(Profiler* p, bool on);
bool profiler_select(Profiler* p, const char* kinds);
int profiler_read(Profiler* p, llg_kernel_profile* out, int max_entries);

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

SymArgs sym_for(const Ctx& c, double a, double b, bool invert) {
  SymArgs s{};
  s.a = a;
  s.b = b;
  s.cx = 2.0 * M_PI / c.Lx;
  s.cy = 2.0 * M_PI / c.Ly;
  s.cz = c.dim == 3 ? 2.0 * M_PI / c.Lz : 0.0;
  s.inv_ng = 1.0 / double(c.ng);
  s.invert = invert ? 1 : 0;
  return s;
}

namespace {

bool is_fin(double v) { return std::isfinite(v); }

llg_status fail(llg_status s, const std::string& msg) {
  set_error(msg);
  return s;
}

// Every device pointer of the ABI must be 16-byte aligned (the kernels issue
// 16-byte vector loads and stores on the Krylov vectors and plane pairs).
bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

llg_status check_aligned(std::initializer_list<const void*> ptrs) {
  for (const void* q : ptrs)
    if (q && !aligned16(q)) return fail(LLG_EARG, "device pointers must be 16-byte aligned");
  return LLG_OK;
}

llg_status check_params(const llg_params* p) {
  if (!p) return fail(LLG_EARG, "params is null");
  if (p->h_field && !aligned16(p->h_field)) return fail(LLG_EARG, "h_field must be 16-byte aligned");
  if (!is_fin(p->alpha) || p->alpha <= 0) return fail(LLG_EARG, "alpha must be finite and > 0");
  if (!is_fin(p->shift) || p->shift <= 0) return fail(LLG_EARG, "shift (HSS lambda) must be finite and > 0");
  if (!is_fin(p->dt) || p->dt < 0) return fail(LLG_EARG, "dt must be finite and >= 0");
  if (!is_fin(p->theta) || p->theta <= 0 || p->theta > 1) return fail(LLG_EARG, "theta must be in (0, 1]");
  if (!is_fin(p->cexc) || p->cexc < 0) return fail(LLG_EARG, "cexc must be finite and >= 0");
  for (int i = 0; i < 3; ++i)
    if (!is_fin(p->h_uniform[i])) return fail(LLG_EARG, "h_uniform must be finite");
  if (!is_fin(p->demag) || !is_fin(p->aniso_k)) return fail(LLG_EARG, "demag and aniso_k must be finite");
  if (p->aniso_k != 0.0) {
    const double* e = p->aniso_axis;
    if (!is_fin(e[0]) || !is_fin(e[1]) || !is_fin(e[2]) ||
        std::fabs(e[0] * e[0] + e[1] * e[1] + e[2] * e[2] - 1.0) > 1e-12)
      return fail(LLG_EARG, "aniso_axis must be a unit vector");
  }
  return LLG_OK;
}

llg_status check_opts(const llg_solver_opts* o) {
  if (!o) return fail(LLG_EARG, "solver options are null");
  if (o->restart < 1 || o->restart > kMaxDots - 2) return fail(LLG_EARG, "restart must be in [1, 62]");
  if (o->maxiter < 1) return fail(LLG_EARG, "maxiter must be >= 1");
  if (!is_fin(o->rtol) || o->rtol <= 0 || o->rtol >= 1) return fail(LLG_EARG, "rtol must be in (0, 1)");
  if (o->prec != LLG_FP64 && o->prec != LLG_FP32_IR && o->prec != LLG_FP32_IR_LEFT)
    return fail(LLG_EARG, "unknown precision");
  if (o->orth != 0 && o->orth != 1) return fail(LLG_EARG, "orth must be 0 (delayed CGS2) or 1 (CGS2)");
  if (o->precond < 0 || o->precond > 2) return fail(LLG_EARG, "precond must be 0, 1 or 2");
  if (o->precond != 0 && o->prec != LLG_FP64) return fail(LLG_EARG, "comparison preconditioners run in float64");
  if (o->orth == 0 && o->restart > 31) return fail(LLG_EARG, "delayed CGS2 supports restart <= 31");
  if (o->picard_norm != 0 && o->picard_norm != 1) return fail(LLG_EARG, "picard_norm must be 0 or 1");
  if (o->transpose != 0 && o->transpose != 1) return fail(LLG_EARG, "transpose must be 0 or 1");
  if (o->fuse_update < -1 || o->fuse_update > 1) return fail(LLG_EARG, "fuse_update must be -1, 0 or 1");
  if (o->prec != LLG_FP64) {
    if (o->max_outer < 1) return fail(LLG_EARG, "max_outer must be >= 1");
    if (!is_fin(o->inner_rtol) || o->inner_rtol <= 0 || o->inner_rtol >= 1)
      return fail(LLG_EARG, "inner_rtol must be in (0, 1)");
  }
  return LLG_OK;
}

NodalArgs nodal_for(const llg_params* p) {
  NodalArgs na{};
  na.lam = p->shift;
  na.hs = 1.0 + p->alpha * p->alpha;
  na.chat = (1.0 + p->alpha * p->alpha) * p->cexc;
  na.hu0 = p->h_uniform[0];
  na.hu1 = p->h_uniform[1];
  na.hu2 = p->h_uniform[2];
  na.half_k = 0.5 * p->dt;
  na.hfield = p->h_field;
  return na;
}

double hcoef(const llg_params* p) { return p->theta * p->dt * (1.0 + p->alpha * p->alpha) * p->cexc; }

// True when the lower-order field depends on m (demagnetization or anisotropy).
bool has_low(const llg_params* p) { return p->demag != 0.0 || p->aniso_k != 0.0; }

// Multiplier s_id I + s_ex |xi|^2 I + scale (demag xi~ xi~^T / |xi|^2 - 2 K e e^T).
// (0, cexc, 1) gives -(h_exc + h_dem + h_ani), (0, 0, 1) the lower-order part alone.
FieldArgs field_for(const Ctx& c, const llg_params* p, double s_id, double s_ex, double scale) {
  FieldArgs f{};
  f.s_id = s_id;
  f.s_ex = s_ex;
  f.s_dm = scale * p->demag;
  f.s_an = -scale * 2.0 * p->aniso_k;
  f.e0 = p->aniso_axis[0];
  f.e1 = p->aniso_axis[1];
  f.e2 = p->aniso_axis[2];
  f.cx = 2.0 * M_PI / c.Lx;
  f.cy = 2.0 * M_PI / c.Ly;
  f.cz = c.dim == 3 ? 2.0 * M_PI / c.Lz : 0.0;
  f.inv_ng = 1.0 / double(c.ng);
  return f;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

llg_status ensure_device(const Ctx& c) {
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return fail(LLG_EHIP, "hipGetDevice failed");
  if (cur != c.device && hipSetDevice(c.device) != hipSuccess) return fail(LLG_EHIP, "hipSetDevice failed");
  return LLG_OK;
}

#define CHK(expr)                                                                          \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(LLG_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define CHK_STATUS(expr)             \
  do {                               \
    llg_status s_ = (expr);          \
    if (s_ != LLG_OK) return s_;     \
  } while (0)

// ---- pipelines (float64) ---------------------------------------------------
hipError_t pipe_d(const Ctx& c, int pro, int epi, const SymArgs& sym, const NodalArgs& na, const double* in,
                  const double* m, double* out, hipStream_t st, const double* aux_v = nullptr,
                  const double* aux_r = nullptr, const BasisDots* bd = nullptr) {
  PipeIO<double, double, double> io{in, m, out, c.ng, aux_v, aux_r};
  return run_pipeline<double, double, double>(c, pro, epi, sym, na, io, st, bd, c.dots);
}

// A x (theta, k from p)
hipError_t op_matvec(const Ctx& c, const llg_params* p, const double* m, const double* x, double* y, bool tr,
                     hipStream_t st) {
  return pipe_d(c, PRO_COPY3, tr ? EPI_MATVEC_T : EPI_MATVEC, sym_for(c, p->alpha, hcoef(p), false), nodal_for(p),
                x, m, y, st);
}
// M^{-1} p or M^{-T} p
hipError_t op_apply(const Ctx& c, const llg_params* p, const double* m, const double* x, double* z, bool tr,
                    hipStream_t st) {
  return pipe_d(c, tr ? PRO_M2T : PRO_COPY3, tr ? EPI_APPLY_T : EPI_APPLY,
                sym_for(c, p->alpha + p->shift, hcoef(p), true), nodal_for(p), x, m, z, st);
}
// M^{-1} A x in one pipeline (with bd: also the Arnoldi inner products of z in c.dots)
hipError_t op_fused(const Ctx& c, const llg_params* p, const double* m, const double* x, double* z, hipStream_t st,
                    const BasisDots* bd = nullptr, bool spec_ready = false) {
  return pipe_d(c, spec_ready ? PRO_NONE : PRO_SMINUS, EPI_FUSED, sym_for(c, p->alpha + p->shift, hcoef(p), true),
                nodal_for(p), x, m, z, st, nullptr, nullptr, bd);
}
// (-Delta_N) u for 3 planes
hipError_t op_lap(const Ctx& c, const double* u, double* out, hipStream_t st) {
  NodalArgs na{};
  return pipe_d(c, PRO_COPY3, EPI_STORE3, sym_for(c, 0.0, 1.0, false), na, u, nullptr, out, st);
}
// b = (C_hat Delta_N m + (1+alpha^2) h_ext, 0); with lap, also (-Delta_N) m (as op_lap)
hipError_t op_rhs(const Ctx& c, const llg_params* p, const double* m, double* b, hipStream_t st,
                  double* lap = nullptr) {
  PipeIO<double, double, double> io{m, nullptr, b, c.ng, nullptr, nullptr};
  io.out_f = lap;
  return run_pipeline<double, double, double>(c, PRO_COPY3, EPI_RHS, sym_for(c, 0.0, 1.0, false), nodal_for(p), io,
                                              st);
}
// One lower-order field pipeline (3x3 multiplier fa, prologue PRO_COPY3).
hipError_t op_field(const Ctx& c, const FieldArgs& fa, int epi, const NodalArgs& na, const double* in, double* out,
                    hipStream_t st, const double* m = nullptr, const double* aux_v = nullptr,
                    const double* aux_r = nullptr) {
  PipeIO<double, double, double> io{in, m, out, c.ng, aux_v, aux_r};
  return run_field(c, fa, epi, na, io, st);
}
// -(h_exc + h_dem + h_ani)(u) for 3 planes: cexc (-Delta_N) u - L_low u
hipError_t op_negfield(const Ctx& c, const llg_params* p, const double* u, double* out, hipStream_t st) {
  return op_field(c, field_for(c, p, 0.0, p->cexc, 1.0), EPI_STORE3, NodalArgs{}, u, out, st);
}
// Explicit right-hand side b = (C_hat Delta_N m + (1+alpha^2) h_low(m), 0)
hipError_t op_rhs_low(const Ctx& c, const llg_params* p, const double* m, double* b, hipStream_t st) {
  if (!has_low(p)) return op_rhs(c, p, m, b, st);
  NodalArgs na = nodal_for(p);
  na.chat = na.hs;  // b_v = -(1+alpha^2) F + (1+alpha^2) h_ext with F = -(h_exc + h_dem + h_ani)
  return op_field(c, field_for(c, p, 0.0, p->cexc, 1.0), EPI_RHS, na, m, b, st);
}

// Number of x-inverse blocks of a float64 pipeline (one residual partial
// each); the launch shape is XCfg<double, nh> (pipeline_kernels.h).
int xinv_blocks(const Ctx& c) {
  const int nh = c.geom.nh;
  const int key = x_plan_key(8, nh);
  const int tpl = nh / plan_p(key);
  const int lx = 64 / tpl;
  return int(((long long)c.ny * c.nz + lx - 1) / lx);
}

// r = b - A x in residual form (fused into the operator's last pass); the
// squared norm of r lands in c.scal[0].
using ResidOp = std::function<hipError_t(const double* x, const double* b, double* r)>;

ResidOp resid_op(const Ctx& c, int epi, const SymArgs& sym, const NodalArgs& na, const double* m, hipStream_t st,
                 const double* aux_v = nullptr, const double* aux_r = nullptr) {
  return [&c, epi, sym, na, m, st, aux_v, aux_r](const double* x, const double* b, double* r) -> hipError_t {
    PipeIO<double, double, double> io{x, m, r, c.ng, aux_v, aux_r};
    io.rhs = b;
    io.red = c.partial;
    hipError_t e = run_pipeline<double, double, double>(c, PRO_COPY3, epi, sym, na, io, st);
    if (e != hipSuccess) return e;
    return reduce_flat(c, xinv_blocks(c), c.scal, st);
  };
}

// Read n doubles of device memory (after the stream's queued work).
llg_status fetch(const Ctx& c, const double* dev, int n, hipStream_t st, double* host_out) {
  CHK(hipMemcpyAsync(c.host, dev, sizeof(double) * n, hipMemcpyDeviceToHost, st));
  CHK(hipStreamSynchronize(st));
  std::memcpy(host_out, c.host, sizeof(double) * n);
  return LLG_OK;
}

// ---- workspace -----------------------------------------------------------
size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

struct Work {
  double* V = nullptr;   // (R + 2) x n4: basis (R + 1 columns) and the Arnoldi operator output
  double* r = nullptr;   // n4
  double* t = nullptr;   // n4 temporary
  float* Z = nullptr;    // R x n4 (precision form)
  float* m32 = nullptr;  // 3 ng   (precision form)
  float* W32 = nullptr;  // n4     (precision form: the float32 operator output of an Arnoldi step)
  double* b = nullptr;   // n4  stepper right-hand side
  double* x = nullptr;   // n4  stepper unknown
  double* m0 = nullptr;  // 3 ng
  double* mh = nullptr;  // 3 ng
  double* vold = nullptr;// 3 ng
  double* l0 = nullptr;  // 3 ng
  double* l1 = nullptr;  // 3 ng
  size_t bytes = 0;
};

Work carve(const Ctx& c, int R, int prec, void* base) {
  const size_t n4 = 4 * size_t(c.ng), n3 = 3 * size_t(c.ng);
  Work w;
  char* p = static_cast<char*>(base);
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* q = p ? p + off : nullptr;
    off += align256(bytes);
    return q;
  };
  w.V = reinterpret_cast<double*>(take(sizeof(double) * n4 * (R + 2)));
  w.r = reinterpret_cast<double*>(take(sizeof(double) * n4));
  w.t = reinterpret_cast<double*>(take(sizeof(double) * n4));
  if (prec == LLG_FP32_IR) w.Z = reinterpret_cast<float*>(take(sizeof(float) * n4 * R));
  if (prec != LLG_FP64) w.m32 = reinterpret_cast<float*>(take(sizeof(float) * n3));
  if (prec != LLG_FP64) w.W32 = reinterpret_cast<float*>(take(sizeof(float) * n4));
  w.b = reinterpret_cast<double*>(take(sizeof(double) * n4));
  w.x = reinterpret_cast<double*>(take(sizeof(double) * n4));
  w.m0 = reinterpret_cast<double*>(take(sizeof(double) * n3));
  w.mh = reinterpret_cast<double*>(take(sizeof(double) * n3));
  w.vold = reinterpret_cast<double*>(take(sizeof(double) * n3));
  w.l0 = reinterpret_cast<double*>(take(sizeof(double) * n3));
  w.l1 = reinterpret_cast<double*>(take(sizeof(double) * n3));
  w.bytes = off;
  return w;
}

// ---- GMRES ---------------------------------------------------------------
using Op = std::function<hipError_t(const double* in, double* out)>;

struct Hess {
  int R;
  std::vector<double> H, cs, sn, g;
  explicit Hess(int r) : R(r), H(size_t(r + 1) * r, 0.0), cs(r, 0.0), sn(r, 0.0), g(r + 1, 0.0) {}
  double& h(int i, int j) { return H[size_t(i) * R + j]; }
  // Insert column j (values col[0..j+1]), rotate, return |g[j+1]|.
  double add_column(int j, const double* col) {
    for (int i = 0; i <= j + 1; ++i) h(i, j) = col[i];
    for (int i = 0; i < j; ++i) {
      const double t = cs[i] * h(i, j) + sn[i] * h(i + 1, j);
      h(i + 1, j) = -sn[i] * h(i, j) + cs[i] * h(i + 1, j);
      h(i, j) = t;
    }
    const double a = h(j, j), b = h(j + 1, j);
    if (b == 0.0) {
      cs[j] = 1.0;
      sn[j] = 0.0;
    } else {
      const double rr = std::hypot(a, b);
      cs[j] = a / rr;
      sn[j] = b / rr;
    }
    h(j, j) = cs[j] * a + sn[j] * b;
    h(j + 1, j) = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    return std::fabs(g[j + 1]);
  }
  void solve(int k, Coefs& y) {
    y.n = k;
    for (int i = k - 1; i >= 0; --i) {
      double s = g[i];
      for (int l = i + 1; l < k; ++l) s -= h(i, l) * y.c[l];
      y.c[i] = s / h(i, i);
    }
  }
};

// One Arnoldi step on V_{j+1} (already holding the new direction): CGS2 against
// V_0..V_j, normalization, column of H.  Returns status; fills col[0..j+1].
llg_status arnoldi_step(const Ctx& c, double* V, long long n4, int j, double* col, hipStream_t st) {
  double* w = V + size_t(j + 1) * n4;
  const int nv = j + 1;
  CHK(cgs_dots(c, V, n4, nv, w, n4, c.dots, st));
  CHK(cgs_update_dots(c, V, n4, nv, c.dots, w, n4, c.dots2, st));
  CHK(cgs_update_norm(c, V, n4, nv, c.dots2, w, w, n4, c.scal, st));
  double hv[3 * kMaxDots];
  CHK(hipMemcpyAsync(c.host, c.dots, sizeof(double) * 3 * kMaxDots, hipMemcpyDeviceToHost, st));
  CHK(hipStreamSynchronize(st));
  std::memcpy(hv, c.host, sizeof(hv));
  for (int i = 0; i < nv; ++i) col[i] = hv[i] + hv[kMaxDots + i];
  const double nrm2 = hv[2 * kMaxDots];
  if (!is_fin(nrm2)) return fail(LLG_ENAN, "non-finite Arnoldi norm");
  col[j + 1] = std::sqrt(nrm2);
  if (nrm2 > 0.0) CHK(scale_invnorm(c, w, w, c.scal, n4, st));
  return LLG_OK;
}

// One Krylov cycle with CGS2 whose re-orthogonalization is delayed by one
// iteration: two streaming passes over the basis and one host round trip per
// iteration.
//
// The device holds the raw directions U = [u_0 .. u_j] (u_0 = the start
// vector, not normalized, at u0; u_i, i >= 1, at U1 + (i - 1) n4); the
// orthonormal basis is Q = U T^{-1}, T upper triangular with column j =
// [a; beta_j].  Entering iteration j the host knows a = Q_j^T u_j and beta_j
// = ||u_j - Q_j a|| (from the previous update pass), which finalizes column
// j-1 of the Hessenberg matrix (h_{j-1} + a, subdiagonal beta_j) before any
// further work, so a converged cycle launches nothing extra.  Then
//   w = Op(u_j)                                  (u_j not yet re-orthogonalized)
//   pass 1: p = U_{j+1}^T w, i.e. b = Q_j^T w = T_j^{-T} p_{<j}, d = u_j.w = p_j
//   pass 2: u_{j+1} = (w - Q_j b - e_j q_j)/beta_j = (w - U_{j+1} gamma)/beta_j,
//           gamma = T_{j+1}^{-1} [b; e_j], e_j = (d - a.b)/beta_j (the first
//           projection of Op q_j, up to the factor 1/beta_j: Q_{j+1}^T Op q_j =
//           ([b; e_j] - g)/beta_j with g = H a, the part of Op(Q_j a) given by
//           the Arnoldi relation); pass 2 also forms U_{j+1}^T u_{j+1} (so a' =
//           T_{j+1}^{-T} of it) and ||u_{j+1}||^2.
// The returned coefficients multiply U (left form) or Ztilde (flexible form:
// Op also stores Ztilde_j = M^{-1} u_j, and Z = Ztilde T^{-1} like Q).
struct CycleResult {
  int k = 0;
  double beta0 = 0, gres = 0;
  Coefs y{};
};

// With op_dots the operator also leaves pass 1's p = U_{j+1}^T w in c.dots
// (it receives the basis layout); otherwise it ignores that argument.
// The fused M^{-1} A pass (float64 GMRES and the left precision variant) and
// the precision form's matvec take delayed-CGS2 pass 1 inside their last x
// pass (the precision form: measured 2.5% more solves/s at 256^3 than the
// separate pass); 0 selects the separate pass.
#ifndef LLG_FUSE_DOTS
#define LLG_FUSE_DOTS 1
#endif
// The operator output W is float64, or float32 for the precision form's
// float32 operators (exact: their values are float32).  The last argument
// (spec_ready) tells the operator that its first x pass already ran, fused
// with the previous step's pass 2 (FirstUpd), so it starts at the next pass.
template <typename TW>
using ArnoldiOpT = std::function<hipError_t(int, const double*, TW*, const BasisDots*, bool)>;
using ArnoldiOp = ArnoldiOpT<double>;

// Pass 2 of step j carried by the first x pass of the operator of step j + 1
// (k_xfwd_upd): ok(j) says whether an instantiation covers step j; run forms
// u_{j+1}, leaves the operator's x spectra in the spectral buffer and
// reduces [U_{j+1}^T u_{j+1}, |u_{j+1}|^2] into out.  Used when a step j + 1
// may follow (it saves the operator's read of u_{j+1} and one launch); when
// the cycle then stops at step j, the spectra are discarded.
#ifndef LLG_FUSE_UPDATE
#define LLG_FUSE_UPDATE 1
#endif
template <typename TW>
struct FirstUpd {
  std::function<bool(int)> ok;
  std::function<hipError_t(const UpdFirst&, const TW*, double*)> run;
};

template <typename TW>
llg_status cycle_dcgs2(const Ctx& c, const ArnoldiOpT<TW>& op, bool op_dots, const double* u0, double* U1, TW* W,
                       long long n4, double c0, int R, double eta, int maxiter, int& iters, CycleResult& out,
                       hipStream_t st, const FirstUpd<TW>* fu = nullptr) {
  if (R >= kDcgsMaxCols) return fail(LLG_EARG, "delayed CGS2 needs restart <= 31");
  Hess hs(R);
  std::vector<double> Hraw(size_t(R + 1) * R, 0.0), T(size_t(R + 1) * (R + 1), 0.0),
      TI(size_t(R + 1) * (R + 1), 0.0);
  std::vector<double> hprev, a, b(R + 1), col(R + 2), g(R + 2), vals(2 * kMaxDots);
  auto HR = [&](int i, int jj) -> double& { return Hraw[size_t(i) * R + jj]; };
  auto TT = [&](int i, int jj) -> double& { return T[size_t(i) * (R + 1) + jj]; };
  auto MI = [&](int i, int jj) -> double& { return TI[size_t(i) * (R + 1) + jj]; };
  if (!is_fin(c0)) return fail(LLG_ENAN, "non-finite Krylov start vector");
  double beta = c0 > 0 ? std::sqrt(c0) : 0.0;
  out.beta0 = beta;
  hs.g[0] = beta;
  int k = 0;
  if (beta == 0.0) {
    out.k = 0;
    return LLG_OK;
  }
  // Small grids whose updates never take the fused pass leave the operator's
  // pass-1 block partials unreduced, in the upper half of the partial buffer
  // (the update pass's own partials use the lower half), for the update pass
  // to reduce: one launch fewer per step.
  const bool speculate = c.ng <= kSpeculateMaxNodes;
  const bool defer = speculate && op_dots && !(LLG_FUSE_UPDATE && fu && fu->ok(0));
  double* const defer_part = c.partial + size_t(kRedBlocksMax) * kMaxDots / 2;
  int defer_nb = 0;
  // Operator of step jj on u_jj into W, its pass-1 products into pslot.
  hipError_t op_err = hipSuccess;
  auto launch_op = [&](int jj, double* pslot, bool spec_ready) {
    const double* ujj = jj == 0 ? u0 : U1 + size_t(jj - 1) * n4;
    hipError_t e;
    if (op_dots) {
      BasisDots bq{u0, U1, n4, jj + 1, nullptr};
      bq.out = pslot;
      if (defer) {
        bq.defer = defer_part;
        bq.defer_nb = &defer_nb;
      }
      e = op(jj, ujj, W, &bq, spec_ready);
    } else {
      e = op(jj, ujj, W, nullptr, spec_ready);
      if (e == hipSuccess) e = dcgs_dots(c, u0, U1, n4, jj, W, n4, pslot, st);
    }
    if (e != hipSuccess && op_err == hipSuccess) op_err = e;
  };
  bool ahead = false;  // step j's operator was launched during step j - 1
  bool ready = false;  // step j's first x pass ran with pass 2 of step j - 1
  for (int j = 0;; ++j) {
    if (j > 0) {
      for (int i = 0; i < j; ++i) col[i] = hprev[i] + a[i];
      col[j] = beta;
      for (int i = 0; i <= j; ++i) HR(i, j - 1) = col[i];
      out.gres = hs.add_column(j - 1, col.data());
      iters++;
      k = j;
      if (out.gres <= eta * out.beta0 || iters >= maxiter || j == R || beta == 0.0) break;
    }
    // column j of T = [a; beta] and of T^{-1} = [-T_j^{-1} a / beta; 1 / beta]
    DcgsCoef cf{};
    for (int i = 0; i < j; ++i) TT(i, j) = a[i];
    TT(j, j) = beta;
    for (int i = 0; i < j; ++i) {
      double sgm = 0;
      for (int l = i; l < j; ++l) sgm += MI(i, l) * a[l];
      MI(i, j) = -sgm / beta;
    }
    MI(j, j) = 1.0 / beta;
    for (int i = 0; i < j; ++i) cf.a[i] = a[i];
    for (int i = 0; i <= j; ++i) cf.minv[i] = MI(i, j);
    cf.inv_beta = 1.0 / beta;
    cf.j = j;
    // pass-1 products of step j go to slot j % 2 (c.dots or c.dots_b), so the
    // operator of step j + 1, launched ahead, cannot overwrite them
    double* pslot = (j & 1) ? c.dots_b : c.dots;
    if (!ahead) launch_op(j, pslot, ready);
    const bool more = j + 1 < R && iters + 1 < maxiter;  // a step j + 1 may follow
    const bool fuse = LLG_FUSE_UPDATE && fu && more && fu->ok(j);
    if (fuse) {
      UpdFirst ua;
      ua.u0 = u0;
      ua.U1 = U1;
      ua.ld = n4;
      ua.j = j;
      ua.inv_beta = cf.inv_beta;
      ua.unew = U1 + size_t(j) * n4;
      ua.partial = c.partial;
      CHK(dcgs_coef(c, cf, pslot, &ua.gamma, st));
      CHK(fu->run(ua, W, c.dots2));
    } else {
      DeferredDots dd;
      if (defer && defer_nb > 0) {
        dd.part = defer_part;
        dd.nb = defer_nb;
        dd.out = pslot;
        dd.mirror = c.hmirror_dev + (pslot - c.dots);
      }
      CHK(dcgs_update(c, u0, U1, n4, cf, pslot, W, U1 + size_t(j) * n4, n4, c.dots2, st, &dd));
    }
    // one round trip: pass-1 dots p and the pass-2 dots of u_{j+1}, which their
    // reductions (on small grids the update pass itself) also wrote into the
    // mapped host mirror.  On small grids the
    // next step's operator (on u_{j+1}, which no host decision changes) is
    // queued first, and the host waits only for this step's passes; when the
    // cycle then ends, that work is discarded.
    ahead = speculate && more;
    ready = fuse;
    if (ahead) {
      CHK(hipEventRecord(c.ev, st));
      launch_op(j + 1, ((j + 1) & 1) ? c.dots_b : c.dots, ready);
      CHK(hipEventSynchronize(c.ev));
    } else {
      CHK(hipStreamSynchronize(st));
    }
    if (op_err != hipSuccess) {
      CHK(op_err);
    }
    std::memcpy(vals.data(), c.hmirror + (pslot - c.dots), sizeof(double) * kMaxDots);
    std::memcpy(vals.data() + kMaxDots, c.hmirror + kMaxDots, sizeof(double) * kMaxDots);
    const double* p = vals.data();
    const double* s = vals.data() + kMaxDots;
    const double d = p[j];
    const double cn = s[j + 1];
    // b = T_j^{-T} p_{<j};  a' = T_{j+1}^{-T} s_{<=j}
    for (int i = 0; i < j; ++i) {
      double sgm = 0;
      for (int l = 0; l <= i; ++l) sgm += MI(l, i) * p[l];
      b[i] = sgm;
    }
    std::vector<double> an(j + 1);
    for (int i = 0; i <= j; ++i) {
      double sgm = 0;
      for (int l = 0; l <= i; ++l) sgm += MI(l, i) * s[l];
      an[i] = sgm;
    }
    double ab = 0, aa = 0;
    for (int i = 0; i < j; ++i) ab += a[i] * b[i];
    for (int i = 0; i <= j; ++i) aa += an[i] * an[i];
    if (!is_fin(d) || !is_fin(cn) || !is_fin(aa)) return fail(LLG_ENAN, "non-finite Arnoldi inner products");
    // first projection of Op q_j: h_j = ([b; e_j] - g) / beta, g = H_{0:j+1,0:j} a
    for (int r = 0; r <= j; ++r) {
      double sgm = 0;
      for (int i = std::max(0, r - 1); i < j; ++i) sgm += HR(r, i) * a[i];
      g[r] = sgm;
    }
    hprev.assign(j + 1, 0.0);
    for (int i = 0; i < j; ++i) hprev[i] = (b[i] - g[i]) / beta;
    hprev[j] = ((d - ab) / beta - g[j]) / beta;
    a.swap(an);
    const double beta2 = cn - aa;
    beta = beta2 > 0 ? std::sqrt(beta2) : 0.0;
  }
  out.k = k;
  hs.solve(k, out.y);
  // Q = U T^{-1} (and Z = Ztilde T^{-1}): coefficients on U solve T yt = y
  for (int i = k - 1; i >= 0; --i) {
    double sgm = out.y.c[i];
    for (int l = i + 1; l < k; ++l) sgm -= TT(i, l) * out.y.c[l];
    out.y.c[i] = sgm / TT(i, i);
  }
  return LLG_OK;
}

struct SolveResult {
  int iters = 0, cycles = 0, outer = 0, converged = 0;
  double rel_true = 0, rel_prec = 0;
  double bnorm = -1;  // ||b||_2 as computed (or taken from the hints)
  bool r_valid = false;  // the workspace's r holds b - A x for the returned x
};

// What a caller that solves repeatedly (the midpoint Picard loop) already
// knows about the inputs of the next solve.
struct SolveHints {
  double bnorm = -1;       // ||b||_2 of an unchanged b (< 0: unknown)
  bool m_checked = false;  // m is finite with no zero node
  bool m32_ready = false;  // the workspace's float32 m holds float(m)
  double rnorm = -1;       // >= 0: the workspace's r holds b - A x0 for the
                           // initial guess x0, with this 2-norm
};

// Left-preconditioned restarted GMRES (FP64) with true-residual acceptance.
// A: true operator, M: preconditioner, MA: M^{-1} A.
// MAd (optional): MA that also leaves the delayed-CGS2 pass-1 inner products
// of its output in c.dots (run_pipeline's BasisDots), and starts after its
// first x pass when spec_ready; fu (optional, with MAd): that first pass
// fused with the previous step's pass 2.
using OpDots = std::function<hipError_t(const double* in, double* out, const BasisDots* bd, bool spec_ready)>;
llg_status gmres_left(const Ctx& c, const ResidOp& RA, const Op& M, const Op& MA, const double* b, double* x,
                      const llg_solver_opts& o, Work& w, SolveResult& res, hipStream_t st,
                      const OpDots* MAd = nullptr, const SolveHints& hints = {},
                      const FirstUpd<double>* fu = nullptr) {
  const long long n4 = 4 * c.ng;
  const int R = o.restart;
  double bnorm = hints.bnorm;
  if (bnorm < 0) {
    double nb[2];
    CHK(dot_and_norm(c, b, nullptr, n4, c.scal, st));
    CHK_STATUS(fetch(c, c.scal, 2, st, nb));
    bnorm = std::sqrt(nb[1]);
  }
  res.bnorm = bnorm;
  if (!is_fin(bnorm)) return fail(LLG_ENAN, "right-hand side is not finite");
  if (bnorm == 0.0) {
    CHK(hipMemsetAsync(x, 0, sizeof(double) * n4, st));
    CHK(hipStreamSynchronize(st));
    res.converged = 1;
    return LLG_OK;
  }
  const double target = o.rtol * bnorm;
  double rn[2];
  double rho;
  if (o.use_x0 && hints.rnorm >= 0) {
    rho = hints.rnorm;
  } else if (o.use_x0) {
    CHK(RA(x, b, w.r));
    CHK_STATUS(fetch(c, c.scal, 1, st, rn));
    rho = std::sqrt(rn[0]);
  } else {
    CHK(hipMemsetAsync(x, 0, sizeof(double) * n4, st));
    CHK(hipMemcpyAsync(w.r, b, sizeof(double) * n4, hipMemcpyDeviceToDevice, st));
    rho = bnorm;
  }
  res.r_valid = true;  // every later x update recomputes r
  double beta0 = -1.0;
  Hess hs(R);
  std::vector<double> col(R + 2);
  while (true) {
    if (!is_fin(rho)) return fail(LLG_ENAN, "non-finite residual");
    res.rel_true = rho / bnorm;
    if (rho <= target) {
      res.converged = 1;
      break;
    }
    if (res.iters >= o.maxiter) break;
    res.cycles++;
    if (o.orth == 0) {
      // basis directions u_0 .. u_R in columns 0 .. R of V, Op output in column R + 1
      double* U0 = w.V;
      double* W = w.V + size_t(R + 1) * n4;
      CHK(M(w.r, U0));
      double un[2];
      CHK(dot_and_norm(c, U0, nullptr, n4, c.scal, st));
      CHK_STATUS(fetch(c, c.scal, 2, st, un));
      CycleResult cr;
      auto op = [&](int, const double* u, double* wout, const BasisDots* bq, bool ready) {
        return MAd ? (*MAd)(u, wout, bq, ready) : MA(u, wout);
      };
      CHK_STATUS(cycle_dcgs2<double>(c, op, MAd != nullptr && LLG_FUSE_DOTS != 0, U0, U0 + n4, W, n4, un[1], R,
                                     target / rho, o.maxiter, res.iters, cr, st, MAd ? fu : nullptr));
      if (!is_fin(cr.beta0)) return fail(LLG_ENAN, "non-finite preconditioned residual");
      if (beta0 < 0) beta0 = cr.beta0;
      res.rel_prec = beta0 > 0 ? cr.gres / beta0 : 0.0;
      if (cr.k == 0) break;
      CHK(lincomb(c, n4, cr.y, U0, n4, x, st));
      CHK(RA(x, b, w.r));
      CHK_STATUS(fetch(c, c.scal, 1, st, rn));
      rho = std::sqrt(rn[0]);
      continue;
    }
    CHK(M(w.r, w.V));
    double bb[2];
    CHK(dot_and_norm(c, w.V, nullptr, n4, c.scal, st));
    CHK_STATUS(fetch(c, c.scal, 2, st, bb));
    const double beta = std::sqrt(bb[1]);
    if (!is_fin(beta)) return fail(LLG_ENAN, "non-finite preconditioned residual");
    if (beta == 0.0) break;
    if (beta0 < 0) beta0 = beta;
    CHK(scale_invnorm(c, w.V, w.V, c.scal + 1, n4, st));
    const double eta = target / rho;
    std::fill(hs.g.begin(), hs.g.end(), 0.0);
    hs.g[0] = beta;
    int k = 0;
    for (int j = 0; j < R; ++j) {
      CHK(MA(w.V + size_t(j) * n4, w.V + size_t(j + 1) * n4));
      CHK_STATUS(arnoldi_step(c, w.V, n4, j, col.data(), st));
      const double gres = hs.add_column(j, col.data());
      res.iters++;
      k = j + 1;
      res.rel_prec = gres / beta0;
      if (gres <= eta * beta || res.iters >= o.maxiter || col[j + 1] == 0.0) break;
    }
    Coefs y{};
    hs.solve(k, y);
    CHK(lincomb(c, n4, y, w.V, n4, x, st));
    CHK(RA(x, b, w.r));
    CHK_STATUS(fetch(c, c.scal, 1, st, rn));
    rho = std::sqrt(rn[0]);
  }
  if (!res.converged) return fail(LLG_ENOCONV, "GMRES reached maxiter before the tolerance");
  return LLG_OK;
}

// Right-preconditioned restarted GMRES (FP64, delayed CGS2): GMRES on
// A M^{-1} u = r from u = 0 in each cycle, x += M^{-1} (U y) at its end.  The
// cycle's residual estimate is the true residual of the iterate, so a cycle
// stops at the target itself; the solve is accepted on the recomputed true
// residual.  AMd: the operator A M^{-1} in one pipeline, which also leaves the
// delayed-CGS2 pass-1 products in c.dots when given the basis.
llg_status gmres_right(const Ctx& c, const ResidOp& RA, const Op& M, const OpDots& AMd, const double* b, double* x,
                       const llg_solver_opts& o, Work& w, SolveResult& res, hipStream_t st,
                       const FirstUpd<double>* fu = nullptr) {
  const long long n4 = 4 * c.ng;
  const int R = o.restart;
  double nb[2];
  CHK(dot_and_norm(c, b, nullptr, n4, c.scal, st));
  CHK_STATUS(fetch(c, c.scal, 2, st, nb));
  const double bnorm = std::sqrt(nb[1]);
  res.bnorm = bnorm;
  if (!is_fin(bnorm)) return fail(LLG_ENAN, "right-hand side is not finite");
  if (bnorm == 0.0) {
    CHK(hipMemsetAsync(x, 0, sizeof(double) * n4, st));
    CHK(hipStreamSynchronize(st));
    res.converged = 1;
    return LLG_OK;
  }
  const double target = o.rtol * bnorm;
  double rn[2];
  double rho;
  if (o.use_x0) {
    CHK(RA(x, b, w.r));
    CHK_STATUS(fetch(c, c.scal, 1, st, rn));
    rho = std::sqrt(rn[0]);
  } else {
    CHK(hipMemsetAsync(x, 0, sizeof(double) * n4, st));
    CHK(hipMemcpyAsync(w.r, b, sizeof(double) * n4, hipMemcpyDeviceToDevice, st));
    rho = bnorm;
  }
  res.r_valid = true;
  // u_0 = r (raw), u_1 .. u_R in columns 0 .. R - 1 of V, operator output in
  // column R + 1 (also the preconditioned update at the cycle's end)
  double* W = w.V + size_t(R + 1) * n4;
  while (true) {
    if (!is_fin(rho)) return fail(LLG_ENAN, "non-finite residual");
    res.rel_true = rho / bnorm;
    if (rho <= target) {
      res.converged = 1;
      break;
    }
    if (res.iters >= o.maxiter) break;
    res.cycles++;
    CycleResult cr;
    auto op = [&](int, const double* u, double* wout, const BasisDots* bq, bool ready) {
      return AMd(u, wout, bq, ready);
    };
    CHK_STATUS(cycle_dcgs2<double>(c, op, LLG_FUSE_DOTS != 0, w.r, w.V, W, n4, rho * rho, R, target / rho, o.maxiter,
                                   res.iters, cr, st, fu));
    res.rel_prec = cr.gres / bnorm;
    if (cr.k == 0) break;
    // t = U y = y_0 u_0 + sum_{i >= 1} y_i u_i, then x += M^{-1} t
    CHK(axpby(c, n4, cr.y.c[0], w.r, 0.0, w.r, w.t, st));
    if (cr.k > 1) {
      Coefs rest{};
      rest.n = cr.k - 1;
      for (int i = 1; i < cr.k; ++i) rest.c[i - 1] = cr.y.c[i];
      CHK(lincomb(c, n4, rest, w.V, n4, w.t, st));
    }
    CHK(M(w.t, W));
    CHK(axpby(c, n4, 1.0, x, 1.0, W, x, st));
    CHK(RA(x, b, w.r));
    CHK_STATUS(fetch(c, c.scal, 1, st, rn));
    rho = std::sqrt(rn[0]);
  }
  if (!res.converged) return fail(LLG_ENOCONV, "GMRES reached maxiter before the tolerance");
  return LLG_OK;
}

// Precision form: FP64 iterative refinement around right-preconditioned
// flexible GMRES whose preconditioner and matvec run in float32 (LLG_FP32_IR),
// or around left-preconditioned GMRES on the fused float32 M^{-1} A
// (LLG_FP32_IR_LEFT, one float32 pipeline per inner iteration).
llg_status gmres_ir(const Ctx& c, const llg_params* p, const double* m, const double* b, double* x,
                    const llg_solver_opts& o, Work& w, SolveResult& res, hipStream_t st, const SolveHints& hints) {
  const long long n4 = 4 * c.ng;
  const int R = o.restart;
  if (!hints.m32_ready) CHK(to_f32(c, 3 * c.ng, m, w.m32, st));
  const SymArgs sym_ap = sym_for(c, p->alpha + p->shift, hcoef(p), true);
  const SymArgs sym_mv = sym_for(c, p->alpha, hcoef(p), false);
  const NodalArgs na = nodal_for(p);
  double bnorm = hints.bnorm;
  if (bnorm < 0) {
    double nb[2];
    CHK(dot_and_norm(c, b, nullptr, n4, c.scal, st));
    CHK_STATUS(fetch(c, c.scal, 2, st, nb));
    bnorm = std::sqrt(nb[1]);
  }
  res.bnorm = bnorm;
  if (!is_fin(bnorm)) return fail(LLG_ENAN, "right-hand side is not finite");
  if (bnorm == 0.0) {
    CHK(hipMemsetAsync(x, 0, sizeof(double) * n4, st));
    CHK(hipStreamSynchronize(st));
    res.converged = 1;
    return LLG_OK;
  }
  const double target = o.rtol * bnorm;
  const ResidOp RA = resid_op(c, EPI_MATVEC, sym_for(c, p->alpha, hcoef(p), false), na, m, st);
  double rn[2];
  double rho;
  if (o.use_x0 && hints.rnorm >= 0) {
    rho = hints.rnorm;
  } else if (o.use_x0) {
    CHK(RA(x, b, w.r));
    CHK_STATUS(fetch(c, c.scal, 1, st, rn));
    rho = std::sqrt(rn[0]);
  } else {
    CHK(hipMemsetAsync(x, 0, sizeof(double) * n4, st));
    CHK(hipMemcpyAsync(w.r, b, sizeof(double) * n4, hipMemcpyDeviceToDevice, st));
    rho = bnorm;
  }
  res.r_valid = true;  // every later x update recomputes r
  Hess hs(R);
  std::vector<double> col(R + 2);
  while (true) {
    if (!is_fin(rho)) return fail(LLG_ENAN, "non-finite residual");
    res.rel_true = rho / bnorm;
    if (rho <= target) {
      res.converged = 1;
      break;
    }
    if (res.outer >= o.max_outer || res.iters >= o.maxiter) break;
    res.outer++;
    res.cycles++;
    const double eta = std::max(o.inner_rtol, target / rho);
    if (o.prec == LLG_FP32_IR_LEFT) {
      // inner GMRES on M^{-1} A d = M^{-1} r, both operators in float32 on
      // float64 Krylov vectors; stop when the preconditioned residual has
      // fallen by eta; x += Q y in float64
      // basis in columns 0 .. R of V (delayed CGS2: raw directions; classic
      // CGS2: orthonormal vectors), Op output in column R + 1
      double* Q = w.V;
      double* W = w.V + size_t(R + 1) * n4;
      PipeIO<float, double, double> io_m{w.r, w.m32, Q, c.ng, nullptr, nullptr};
      CHK((run_pipeline<float, double, double>(c, PRO_COPY3, EPI_APPLY, sym_ap, na, io_m, st)));
      double un[2];
      CHK(dot_and_norm(c, Q, nullptr, n4, c.scal, st));
      CHK_STATUS(fetch(c, c.scal, 2, st, un));
      auto opl = [&](int, const double* u, double* wout, const BasisDots* bq) -> hipError_t {
        PipeIO<float, double, double> io{u, w.m32, wout, c.ng, nullptr, nullptr};
        return run_pipeline<float, double, double>(c, PRO_SMINUS, EPI_FUSED, sym_ap, na, io, st, bq, c.dots);
      };
      CycleResult cr;
      if (o.orth == 0) {
        // delayed CGS2: the fused float32 operator's output goes to W32 in float32
        ArnoldiOpT<float> opl32 = [&](int, const double* u, float* wout, const BasisDots* bq,
                                      bool ready) -> hipError_t {
          PipeIO<float, double, float> io{u, w.m32, wout, c.ng, nullptr, nullptr};
          return run_pipeline<float, double, float>(c, ready ? PRO_NONE : PRO_SMINUS, EPI_FUSED, sym_ap, na, io,
                                                    st, bq, c.dots);
        };
        const FirstUpd<float> fu{
            [&](int j) { return xfwd_upd_supported(c, PRO_SMINUS, true, j, o.fuse_update); },
            [&](const UpdFirst& ua, const float* wv, double* out) {
              return run_xfwd_upd(c, PRO_SMINUS, na, ua, wv, w.m32, out, st);
            }};
        CHK_STATUS(cycle_dcgs2<float>(c, opl32, LLG_FUSE_DOTS != 0, Q, Q + n4, w.W32, n4, un[1], R, eta,
                                      o.maxiter, res.iters, cr, st, &fu));
      } else {
        const double beta = std::sqrt(un[1]);
        if (!is_fin(beta)) return fail(LLG_ENAN, "non-finite preconditioned residual");
        if (beta == 0.0) break;
        CHK(scale_invnorm(c, Q, Q, c.scal + 1, n4, st));
        std::fill(hs.g.begin(), hs.g.end(), 0.0);
        hs.g[0] = beta;
        cr.beta0 = beta;
        for (int j = 0; j < R; ++j) {
          CHK(opl(j, Q + size_t(j) * n4, Q + size_t(j + 1) * n4, nullptr));
          CHK_STATUS(arnoldi_step(c, Q, n4, j, col.data(), st));
          cr.gres = hs.add_column(j, col.data());
          res.iters++;
          cr.k = j + 1;
          if (cr.gres <= eta * beta || res.iters >= o.maxiter || col[j + 1] == 0.0) break;
        }
        hs.solve(cr.k, cr.y);
      }
      res.rel_prec = cr.beta0 > 0 ? cr.gres / cr.beta0 : 0.0;
      if (cr.k == 0) break;
      CHK(lincomb(c, n4, cr.y, Q, n4, x, st));
      CHK(RA(x, b, w.r));
      CHK_STATUS(fetch(c, c.scal, 1, st, rn));
      rho = std::sqrt(rn[0]);
      continue;
    }
    if (o.orth == 0) {
      // u_0 = r (the residual buffer is consumed as the cycle's start vector),
      // u_1 .. u_R in columns 0 .. R - 1 of V, Op output in column R + 1
      // operator output in float32 (W32): the float32 matvec's values exactly
      ArnoldiOpT<float> op = [&](int j, const double* u, float* wout, const BasisDots* bq,
                                 bool ready) -> hipError_t {
        return run_apply_matvec(c, sym_ap, sym_mv, na, u, w.m32, w.Z + size_t(j) * n4, wout, st, bq, c.dots,
                                ready);
      };
      const FirstUpd<float> fu{
          [&](int j) { return xfwd_upd_supported(c, PRO_COPY3, true, j, o.fuse_update); },
          [&](const UpdFirst& ua, const float* wv, double* out) {
            return run_xfwd_upd(c, PRO_COPY3, na, ua, wv, w.m32, out, st);
          }};
      CycleResult cr;
      CHK_STATUS(cycle_dcgs2<float>(c, op, LLG_FUSE_DOTS != 0, w.r, w.V, w.W32, n4, rho * rho, R, eta, o.maxiter,
                                    res.iters, cr, st, &fu));
      res.rel_prec = cr.gres / bnorm;
      if (cr.k == 0) break;
      CHK(lincomb(c, n4, cr.y, w.Z, n4, x, st));
      CHK(RA(x, b, w.r));
      CHK_STATUS(fetch(c, c.scal, 1, st, rn));
      rho = std::sqrt(rn[0]);
      continue;
    }
    CHK(axpby(c, n4, 1.0 / rho, w.r, 0.0, w.r, w.V, st));
    std::fill(hs.g.begin(), hs.g.end(), 0.0);
    hs.g[0] = rho;
    int k = 0;
    for (int j = 0; j < R; ++j) {
      CHK(run_apply_matvec(c, sym_ap, sym_mv, na, w.V + size_t(j) * n4, w.m32, w.Z + size_t(j) * n4,
                           w.V + size_t(j + 1) * n4, st));
      CHK_STATUS(arnoldi_step(c, w.V, n4, j, col.data(), st));
      const double gres = hs.add_column(j, col.data());
      res.iters++;
      k = j + 1;
      res.rel_prec = gres / bnorm;
      if (gres <= eta * rho || res.iters >= o.maxiter || col[j + 1] == 0.0) break;
    }
    Coefs y{};
    hs.solve(k, y);
    CHK(lincomb(c, n4, y, w.Z, n4, x, st));
    CHK(RA(x, b, w.r));
    CHK_STATUS(fetch(c, c.scal, 1, st, rn));
    rho = std::sqrt(rn[0]);
  }
  if (!res.converged) return fail(LLG_ENOCONV, "refinement reached its limit before the tolerance");
  return LLG_OK;
}

llg_status check_m(const Ctx& c, const double* m, hipStream_t st) {
  double o[2];
  CHK(m_check(c, m, c.scal, st));
  CHK_STATUS(fetch(c, c.scal, 2, st, o));
  if (o[1] != 0.0) return fail(LLG_ENAN, "magnetization contains non-finite values");
  if (!(o[0] > 1e-300)) return fail(LLG_EZERO_M, "some nodal magnetization is zero (Proposition 1 needs m_i != 0)");
  return LLG_OK;
}

llg_status solve(const Ctx& c, const llg_params* p, const double* m, const double* b, double* x,
                 const llg_solver_opts& o, Work& w, SolveResult& res, hipStream_t st, const SolveHints& hints = {}) {
  if (!hints.m_checked) CHK_STATUS(check_m(c, m, st));
  if (o.transpose) {
    // A^T x = b with GMRES left-preconditioned by M^T: operator M^{-T} A^T (a
    // transposed matvec, then the transposed preconditioner; the symmetric
    // comparison preconditioner is its own transpose)
    const ResidOp RAT = resid_op(c, EPI_MATVEC_T, sym_for(c, p->alpha, hcoef(p), false), nodal_for(p), m, st);
    const long long n4 = 4 * c.ng;
    Op MT = [&](const double* in, double* out) -> hipError_t {
      if (o.precond == 0) return op_apply(c, p, m, in, out, true, st);
      if (o.precond == 1)
        return pipe_d(c, PRO_COPY3, EPI_APPLY_SYM, sym_for(c, p->alpha + p->shift, hcoef(p), true), nodal_for(p),
                      in, m, out, st);
      return hipMemcpyAsync(out, in, sizeof(double) * n4, hipMemcpyDeviceToDevice, st);
    };
    Op MTAT = [&](const double* in, double* out) -> hipError_t {
      hipError_t e = op_matvec(c, p, m, in, w.t, true, st);
      if (e != hipSuccess) return e;
      return MT(w.t, out);
    };
    return gmres_left(c, RAT, MT, MTAT, b, x, o, w, res, st, nullptr, hints);
  }
  if (o.prec != LLG_FP64) return gmres_ir(c, p, m, b, x, o, w, res, st, hints);
  const ResidOp RA = resid_op(c, EPI_MATVEC, sym_for(c, p->alpha, hcoef(p), false), nodal_for(p), m, st);
  if (o.precond == 1) {  // symmetric part (lambda I + calH)^{-1}
    const SymArgs sa = sym_for(c, p->alpha + p->shift, hcoef(p), true);
    Op M = [&](const double* in, double* out) {
      return pipe_d(c, PRO_COPY3, EPI_APPLY_SYM, sa, nodal_for(p), in, m, out, st);
    };
    Op MA = [&](const double* in, double* out) {
      return pipe_d(c, PRO_SMINUS, EPI_FUSED_SYM, sa, nodal_for(p), in, m, out, st);
    };
    return gmres_left(c, RA, M, MA, b, x, o, w, res, st, nullptr, hints);
  }
  if (o.precond == 2) {  // no preconditioner
    const long long n4 = 4 * c.ng;
    Op M = [&](const double* in, double* out) {
      return hipMemcpyAsync(out, in, sizeof(double) * n4, hipMemcpyDeviceToDevice, st);
    };
    Op MA = [&](const double* in, double* out) { return op_matvec(c, p, m, in, out, false, st); };
    return gmres_left(c, RA, M, MA, b, x, o, w, res, st, nullptr, hints);
  }
  Op M = [&](const double* in, double* out) { return op_apply(c, p, m, in, out, false, st); };
  Op MA = [&](const double* in, double* out) { return op_fused(c, p, m, in, out, st); };
  OpDots MAd = [&](const double* in, double* out, const BasisDots* bd, bool ready) {
    return op_fused(c, p, m, in, out, st, bd, ready);
  };
  const FirstUpd<double> fu{[&](int j) { return xfwd_upd_supported(c, PRO_SMINUS, false, j, o.fuse_update); },
                            [&](const UpdFirst& ua, const double* wv, double* out) {
                              return run_xfwd_upd(c, PRO_SMINUS, nodal_for(p), ua, wv, m, out, st);
                            }};
  return gmres_left(c, RA, M, MA, b, x, o, w, res, st, &MAd, hints, &fu);
}

void fill_stats(const SolveResult& r, llg_solver_stats* s) {
  if (!s) return;
  s->iters = r.iters;
  s->cycles = r.cycles;
  s->outer_steps = r.outer;
  s->converged = r.converged;
  s->rel_res_true = r.rel_true;
  s->rel_res_prec = r.rel_prec;
  s->restarts = r.cycles > 0 ? r.cycles - 1 : 0;
  s->ms = 0.0;
}

using Clock = std::chrono::steady_clock;
double ms_since(Clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
}

// g_N(m): with the lower-order field the nodal density is 1/2 m.F - m.h_ext + K,
// F = -(h_exc + h_dem + h_ani)(m); without it 1/2 cexc m.(-Delta_N m) - m.h_ext.
// One pipeline (the field pipeline with a lower-order field) whose last pass
// reduces the density: no field is stored.
llg_status energy_of(const Ctx& c, const llg_params* p, const double* m, double* e, hipStream_t st) {
  const bool low = has_low(p);
  NodalArgs na = nodal_for(p);
  na.chat = low ? 1.0 : p->cexc;
  PipeIO<double, double, double> io{m, m, nullptr, c.ng, nullptr, nullptr};
  io.red = c.partial;
  if (low) CHK(run_field(c, field_for(c, p, 0.0, p->cexc, 1.0), EPI_ENERGY, na, io, st));
  else CHK((run_pipeline<double, double, double>(c, PRO_COPY3, EPI_ENERGY, sym_for(c, 0.0, 1.0, false), na, io,
                                                 st)));
  CHK(reduce_flat(c, xinv_blocks(c), c.scal, st));
  double s;
  CHK_STATUS(fetch(c, c.scal, 1, st, &s));
  const double vol = c.Lx * c.Ly * (c.dim == 3 ? c.Lz : 1.0);
  *e = s * vol / double(c.ng) + (low ? p->aniso_k * vol : 0.0);
  return LLG_OK;
}

}  // namespace
}  // namespace llg

using namespace llg;

// ---------------------------------------------------------------------------
extern "C" {

const char* llg_last_error(void) { return g_err.c_str(); }

llg_status llg_ctx_create_cell(llg_ctx** out, int nx, int ny, int nz, double lx, double ly, double lz,
                               int device) {
  if (!out) return fail(LLG_EARG, "out is null");
  *out = nullptr;
  if (nx % 2 != 0 || !nh_supported(nx / 2) || !axis_supported(ny) || !(nz == 1 || axis_supported(nz)))
    return fail(LLG_EARG,
                "unsupported grid: nx must be 2 n with n in {2..256} of the form 2^a, 3*2^a or 5*2^a; ny and "
                "nz (or nz = 1) even, in [4, 512], of the form 2^a, 3*2^a or 5*2^a");
  if (!is_fin(lx) || lx <= 0 || !is_fin(ly) || ly <= 0 || !is_fin(lz) || lz <= 0)
    return fail(LLG_EARG, "cell lengths must be finite and > 0");
  if (device < 0) return fail(LLG_EARG, "device must be >= 0");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device >= ndev) return fail(LLG_EHIP, "no such HIP device");
  if (hipSetDevice(device) != hipSuccess) return fail(LLG_EHIP, "hipSetDevice failed");
  scratch_setup(device);
  llg_ctx* ctx = new llg_ctx();
  Ctx& c = ctx->c;
  c.nx = nx;
  c.ny = ny;
  c.nz = nz;
  c.dim = nz == 1 ? 2 : 3;
  c.device = device;
  c.Lx = lx;
  c.Ly = ly;
  c.Lz = lz;
  c.ng = (long long)nx * ny * nz;
  c.geom.nx = nx;
  c.geom.ny = ny;
  c.geom.nz = nz;
  c.geom.nh = nx / 2;
  c.geom.cs = 3 * (nx / 2 + 1);
  c.geom.rs = (c.geom.cs + 15) / 16 * 16;
  c.geom.ng = c.ng;
  c.spec_bytes = sizeof(cx<double>) * size_t(c.geom.rs) * ny * nz;
  auto cleanup = [&](llg_status s, const std::string& m) {
    llg_ctx_destroy(ctx);
    return fail(s, m);
  };
  c.prof = profiler_new();
  if (hipMalloc(&c.spec, c.spec_bytes) != hipSuccess) return cleanup(LLG_ENOMEM, "spectral scratch allocation failed");
  if (hipMalloc(&c.partial, sizeof(double) * kRedBlocksMax * kMaxDots) != hipSuccess)
    return cleanup(LLG_ENOMEM, "reduction buffer allocation failed");
  if (hipMalloc(&c.dots, sizeof(double) * kDotsSlots * kMaxDots) != hipSuccess)
    return cleanup(LLG_ENOMEM, "reduction buffer allocation failed");
  c.dots2 = c.dots + kMaxDots;
  c.scal = c.dots + 2 * kMaxDots;
  c.dots_b = c.dots + 4 * kMaxDots;
  if (hipEventCreateWithFlags(&c.ev, hipEventDisableTiming) != hipSuccess)
    return cleanup(LLG_EHIP, "event creation failed");
  if (hipMalloc(&c.tri, sizeof(double) * (kDcgsMaxCols * kDcgsMaxCols + kDcgsMaxCols)) != hipSuccess)
    return cleanup(LLG_ENOMEM, "reduction buffer allocation failed");
  if (hipHostMalloc(reinterpret_cast<void**>(&c.hmirror), sizeof(double) * kDotsSlots * kMaxDots,
                    hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess)
    return cleanup(LLG_ENOMEM, "pinned host buffer allocation failed");
  if (hipHostGetDevicePointer(reinterpret_cast<void**>(&c.hmirror_dev), c.hmirror, 0) != hipSuccess)
    return cleanup(LLG_EHIP, "device address of the pinned host buffer");
  if (hipHostMalloc(reinterpret_cast<void**>(&c.host), sizeof(double) * 4 * kMaxDots, hipHostMallocDefault) !=
      hipSuccess)
    return cleanup(LLG_ENOMEM, "pinned host buffer allocation failed");
  const int ns[3] = {nx, ny, nz};
  for (int a = 0; a < 3; ++a) {
    const int n = ns[a];
    if (n < 2) continue;
    std::vector<cx<double>> td(n);
    std::vector<cx<float>> tf(n);
    for (int m = 0; m < n; ++m) {
      const long double ang = -2.0L * 3.14159265358979323846264338327950288L * (long double)m / (long double)n;
      td[m] = {(double)cosl(ang), (double)sinl(ang)};
      tf[m] = {(float)cosl(ang), (float)sinl(ang)};
    }
    if (hipMalloc(&c.tw_d[a], sizeof(cx<double>) * n) != hipSuccess ||
        hipMalloc(&c.tw_f[a], sizeof(cx<float>) * n) != hipSuccess)
      return cleanup(LLG_ENOMEM, "twiddle allocation failed");
    if (hipMemcpy(c.tw_d[a], td.data(), sizeof(cx<double>) * n, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c.tw_f[a], tf.data(), sizeof(cx<float>) * n, hipMemcpyHostToDevice) != hipSuccess)
      return cleanup(LLG_EHIP, "twiddle upload failed");
  }
  *out = ctx;
  return LLG_OK;
}

llg_status llg_ctx_create(llg_ctx** out, int nx, int ny, int nz, double h, int device) {
  if (!is_fin(h) || h <= 0) {
    if (out) *out = nullptr;
    return fail(LLG_EARG, "h must be finite and > 0");
  }
  return llg_ctx_create_cell(out, nx, ny, nz, nx * h, ny * h, nz * h, device);
}

llg_status llg_ctx_destroy(llg_ctx* ctx) {
  if (!ctx) return LLG_OK;
  Ctx& c = ctx->c;
  int cur = -1;
  (void)hipGetDevice(&cur);
  if (cur != c.device) (void)hipSetDevice(c.device);
  (void)hipDeviceSynchronize();
  for (int a = 0; a < 3; ++a) {
    if (c.tw_d[a]) (void)hipFree(c.tw_d[a]);
    if (c.tw_f[a]) (void)hipFree(c.tw_f[a]);
  }
  if (c.spec) (void)hipFree(c.spec);
  if (c.partial) (void)hipFree(c.partial);
  if (c.dots) (void)hipFree(c.dots);
  if (c.tri) (void)hipFree(c.tri);
  if (c.host) (void)hipHostFree(c.host);
  if (c.hmirror) (void)hipHostFree(c.hmirror);
  if (c.ev) (void)hipEventDestroy(c.ev);
  if (c.prof) profiler_delete(c.prof);
  delete ctx;
  return LLG_OK;
}

size_t llg_workspace_bytes(const llg_ctx* ctx, int restart, int prec) {
  if (!ctx || restart < 1 || restart > kMaxDots - 2 ||
      (prec != LLG_FP64 && prec != LLG_FP32_IR && prec != LLG_FP32_IR_LEFT))
    return 0;
  return carve(ctx->c, restart, prec, nullptr).bytes;
}

llg_status llg_profile_enable(llg_ctx* ctx, int enable) {
  if (!ctx || !ctx->c.prof) return fail(LLG_EARG, "null context");
  profiler_enable(ctx->c.prof, enable != 0);
  return LLG_OK;
}

llg_status llg_profile_select(llg_ctx* ctx, const char* kinds) {
  if (!ctx || !ctx->c.prof) return fail(LLG_EARG, "null context");
  if (!profiler_select(ctx->c.prof, kinds)) return fail(LLG_EARG, "unknown kernel kind in the selection");
  return LLG_OK;
}

int llg_profile_read(llg_ctx* ctx, llg_kernel_profile* out, int max_entries) {
  if (!ctx || !ctx->c.prof || max_entries < 0) {
    set_error("llg_profile_read: bad argument");
    return -1;
  }
  if (ensure_device(ctx->c) != LLG_OK) return -1;
  const int n = profiler_read(ctx->c.prof, out, max_entries);
  if (n < 0) set_error("llg_profile_read: event query failed");
  return n;
}

llg_status llg_matvec(llg_ctx* ctx, const llg_params* prm, const double* m, const double* x, double* y,
                      int transpose, void* stream) {
  if (!ctx || !m || !x || !y) return fail(LLG_EARG, "null argument");
  if (x == y) return fail(LLG_EARG, "llg_matvec: y must not alias x");
  CHK_STATUS(check_aligned({m, x, y}));
  CHK_STATUS(check_params(prm));
  CHK_STATUS(ensure_device(ctx->c));
  CHK(op_matvec(ctx->c, prm, m, x, y, transpose != 0, as_stream(stream)));
  return LLG_OK;
}

llg_status fft_hss_apply(llg_ctx* ctx, const llg_params* prm, const double* m, const double* p, double* z,
                         int transpose, void* stream) {
  if (!ctx || !m || !p || !z) return fail(LLG_EARG, "null argument");
  CHK_STATUS(check_aligned({m, p, z}));
  CHK_STATUS(check_params(prm));
  CHK_STATUS(ensure_device(ctx->c));
  CHK(op_apply(ctx->c, prm, m, p, z, transpose != 0, as_stream(stream)));
  return LLG_OK;
}

llg_status llg_matvec_f32(llg_ctx* ctx, const llg_params* prm, const float* m, const float* x, float* y,
                          int transpose, void* stream) {
  if (!ctx || !m || !x || !y) return fail(LLG_EARG, "null argument");
  if (x == y) return fail(LLG_EARG, "llg_matvec_f32: y must not alias x");
  CHK_STATUS(check_aligned({m, x, y}));
  CHK_STATUS(check_params(prm));
  CHK_STATUS(ensure_device(ctx->c));
  const Ctx& c = ctx->c;
  PipeIO<float, float, float> io{x, m, y, c.ng, nullptr, nullptr};
  CHK((run_pipeline<float, float, float>(c, PRO_COPY3, transpose ? EPI_MATVEC_T : EPI_MATVEC,
                                         sym_for(c, prm->alpha, hcoef(prm), false), nodal_for(prm), io,
                                         as_stream(stream))));
  return LLG_OK;
}

llg_status fft_hss_apply_f32(llg_ctx* ctx, const llg_params* prm, const float* m, const float* p, float* z,
                             int transpose, void* stream) {
  if (!ctx || !m || !p || !z) return fail(LLG_EARG, "null argument");
  CHK_STATUS(check_aligned({m, p, z}));
  CHK_STATUS(check_params(prm));
  CHK_STATUS(ensure_device(ctx->c));
  const Ctx& c = ctx->c;
  PipeIO<float, float, float> io{p, m, z, c.ng, nullptr, nullptr};
  CHK((run_pipeline<float, float, float>(c, transpose ? PRO_M2T : PRO_COPY3, transpose ? EPI_APPLY_T : EPI_APPLY,
                                         sym_for(c, prm->alpha + prm->shift, hcoef(prm), true), nodal_for(prm), io,
                                         as_stream(stream))));
  return LLG_OK;
}

}  // extern "C"

namespace {
// Arnoldi-product arguments of llg_precond_op(_f32): none, or nbasis in
// [1, kBasisDotsMax] vectors at an even stride ld >= 4 N_g, and a device
// output of nbasis doubles.
llg_status basis_dots(const Ctx& c, const double* basis, int nbasis, long long ld, double* dots, BasisDots& bd) {
  bd = BasisDots{};
  if (nbasis == 0) {
    if (basis || dots) return fail(LLG_EARG, "basis and dots must be NULL when nbasis = 0");
    return LLG_OK;
  }
  if (nbasis < 0 || nbasis > kBasisDotsMax) return fail(LLG_EARG, "nbasis must be in [0, 32]");
  if (!basis || !dots) return fail(LLG_EARG, "basis and dots are required when nbasis > 0");
  if (ld < 4 * c.ng || ld % 2 != 0) return fail(LLG_EARG, "ld must be even and at least 4 N_g");
  CHK_STATUS(check_aligned({basis, dots}));
  bd.u0 = basis;
  bd.U1 = basis + ld;
  bd.ld = ld;
  bd.nv = nbasis;
  return LLG_OK;
}
}  // namespace

extern "C" {

llg_status llg_precond_op(llg_ctx* ctx, const llg_params* prm, const double* m, const double* x, double* y,
                          const double* basis, int nbasis, long long ld, double* dots, void* stream) {
  if (!ctx || !m || !x || !y) return fail(LLG_EARG, "null argument");
  if (x == y) return fail(LLG_EARG, "llg_precond_op: y must not alias x");
  CHK_STATUS(check_aligned({m, x, y}));
  CHK_STATUS(check_params(prm));
  const Ctx& c = ctx->c;
  BasisDots bd;
  CHK_STATUS(basis_dots(c, basis, nbasis, ld, dots, bd));
  CHK_STATUS(ensure_device(c));
  hipStream_t st = as_stream(stream);
  PipeIO<double, double, double> io{x, m, y, c.ng, nullptr, nullptr};
  CHK((run_pipeline<double, double, double>(c, PRO_SMINUS, EPI_FUSED, sym_for(c, prm->alpha + prm->shift, hcoef(prm),
                                                                              true),
                                            nodal_for(prm), io, st, bd.nv > 0 ? &bd : nullptr, dots)));
  return LLG_OK;
}

llg_status llg_precond_op_f32(llg_ctx* ctx, const llg_params* prm, const float* m, const double* x, double* y,
                              float* z, int side, const double* basis, int nbasis, long long ld, double* dots,
                              void* stream) {
  if (!ctx || !m || !x || !y) return fail(LLG_EARG, "null argument");
  if (side != 0 && side != 1) return fail(LLG_EARG, "side must be 0 (left, fused) or 1 (flexible)");
  if (side == 1 && !z) return fail(LLG_EARG, "side 1 needs the float32 output z");
  if (x == y || (side == 1 && (static_cast<const void*>(z) == static_cast<const void*>(x) ||
                               static_cast<const void*>(z) == static_cast<const void*>(y))))
    return fail(LLG_EARG, "llg_precond_op_f32: x, y and z must not alias");
  CHK_STATUS(check_aligned({m, x, y, z}));
  CHK_STATUS(check_params(prm));
  const Ctx& c = ctx->c;
  BasisDots bd;
  CHK_STATUS(basis_dots(c, basis, nbasis, ld, dots, bd));
  CHK_STATUS(ensure_device(c));
  hipStream_t st = as_stream(stream);
  const SymArgs sym_ap = sym_for(c, prm->alpha + prm->shift, hcoef(prm), true);
  const NodalArgs na = nodal_for(prm);
  if (side == 0) {
    PipeIO<float, double, double> io{x, m, y, c.ng, nullptr, nullptr};
    CHK((run_pipeline<float, double, double>(c, PRO_SMINUS, EPI_FUSED, sym_ap, na, io, st,
                                             bd.nv > 0 ? &bd : nullptr, dots)));
  } else {
    CHK(run_apply_matvec(c, sym_ap, sym_for(c, prm->alpha, hcoef(prm), false), na, x, m, z, y, st,
                         bd.nv > 0 ? &bd : nullptr, dots));
  }
  return LLG_OK;
}

llg_status gmres_solve(llg_ctx* ctx, const llg_params* prm, const double* m, const double* b, double* x,
                       const llg_solver_opts* opts, llg_solver_stats* stats, void* work, size_t work_bytes,
                       void* stream) {
  return gmres_solve_work(ctx, prm, m, b, x, opts, stats, work, work_bytes, stream);
}

}  // extern "C"

int llg::ctx_device(const llg_ctx* ctx) { return ctx ? ctx->c.device : -1; }

llg_status llg::gmres_solve_work(llg_ctx* ctx, const llg_params* prm, const double* m, const double* b, double* x,
                                 const llg_solver_opts* opts, llg_solver_stats* stats, void* work,
                                 size_t work_bytes, void* stream) {
  const auto t0 = Clock::now();
  if (!ctx || !m || !b || !x || !work) return fail(LLG_EARG, "null argument");
  CHK_STATUS(check_aligned({m, b, x, work}));
  CHK_STATUS(check_params(prm));
  CHK_STATUS(check_opts(opts));
  if (x == b) return fail(LLG_EARG, "gmres_solve: x must not alias b");
  if (opts->transpose && opts->prec != LLG_FP64) return fail(LLG_EARG, "transposed solves run in float64");
  const Ctx& c = ctx->c;
  Work w = carve(c, opts->restart, opts->prec, work);
  if (work_bytes < w.bytes) return fail(LLG_ENOMEM, "workspace smaller than llg_workspace_bytes()");
  CHK_STATUS(ensure_device(c));
  SolveResult r;
  const llg_status s = solve(c, prm, m, b, x, *opts, w, r, as_stream(stream));
  fill_stats(r, stats);
  if (stats) stats->ms = ms_since(t0);
  return s;
}

extern "C" {

llg_status llg_rhs(llg_ctx* ctx, const llg_params* prm, const double* m, double* b, void* stream) {
  if (!ctx || !m || !b) return fail(LLG_EARG, "null argument");
  CHK_STATUS(check_aligned({m, b}));
  CHK_STATUS(check_params(prm));
  CHK_STATUS(ensure_device(ctx->c));
  CHK(op_rhs_low(ctx->c, prm, m, b, as_stream(stream)));
  return LLG_OK;
}

llg_status llg_energy(llg_ctx* ctx, const llg_params* prm, const double* m, double* energy, void* stream) {
  if (!ctx || !m || !energy) return fail(LLG_EARG, "null argument");
  CHK_STATUS(check_params(prm));
  CHK_STATUS(ensure_device(ctx->c));
  CHK_STATUS(check_aligned({m}));
  return energy_of(ctx->c, prm, m, energy, as_stream(stream));
}

llg_status llg_step_euler(llg_ctx* ctx, const llg_params* prm, double* m, double* v_out, double* lam_out,
                          const llg_solver_opts* opts, llg_step_stats* stats, void* work, size_t work_bytes,
                          void* stream) {
  if (!ctx || !m || !work) return fail(LLG_EARG, "null argument");
  CHK_STATUS(check_aligned({m, v_out, lam_out, work}));
  CHK_STATUS(check_params(prm));
  CHK_STATUS(check_opts(opts));
  const Ctx& c = ctx->c;
  Work w = carve(c, opts->restart, opts->prec, work);
  if (work_bytes < w.bytes) return fail(LLG_ENOMEM, "workspace smaller than llg_workspace_bytes()");
  CHK_STATUS(ensure_device(c));
  hipStream_t st = as_stream(stream);
  llg_params p1 = *prm;
  p1.theta = 1.0;
  llg_solver_opts o = *opts;
  o.use_x0 = 0;
  o.transpose = 0;
  const long long ng = c.ng;
  if (stats) std::memset(stats, 0, sizeof(*stats));
  double e0 = 0;
  if (stats) CHK_STATUS(energy_of(c, &p1, m, &e0, st));
  CHK(op_rhs_low(c, &p1, m, w.b, st));
  SolveResult r;
  const llg_status s = solve(c, &p1, m, w.b, w.x, o, w, r, st);
  if (stats) {
    stats->picard_iters = 1;
    stats->lin_iters_total = r.iters;
    stats->converged = r.converged;
  }
  if (s != LLG_OK) return s;
  double len;
  CHK(euler_update(c, m, w.x, p1.dt, c.scal, st));
  CHK_STATUS(fetch(c, c.scal, 1, st, &len));
  if (v_out) CHK(hipMemcpyAsync(v_out, w.x, sizeof(double) * 3 * ng, hipMemcpyDeviceToDevice, st));
  if (lam_out) CHK(hipMemcpyAsync(lam_out, w.x + 3 * ng, sizeof(double) * ng, hipMemcpyDeviceToDevice, st));
  if (stats) {
    double e1 = 0, vv[2];
    CHK_STATUS(energy_of(c, &p1, m, &e1, st));
    CHK(dot_and_norm(c, w.x, nullptr, 3 * ng, c.scal, st));
    CHK_STATUS(fetch(c, c.scal, 2, st, vv));
    const double wq = c.Lx * c.Ly * (c.dim == 3 ? c.Lz : 1.0) / double(ng);
    stats->max_len_err = len;
    stats->energy_before = e0;
    stats->energy_after = e1;
    stats->v_norm2 = wq * vv[1];
    const double a = p1.alpha;
    stats->dissipation_defect = e1 - e0 + a * p1.dt / (1 + a * a) * stats->v_norm2;
  }
  CHK(hipStreamSynchronize(st));
  return LLG_OK;
}

llg_status llg_step_midpoint(llg_ctx* ctx, const llg_params* prm, double* m, double* v_half, double* lam,
                             double picard_tol, int picard_max, const llg_solver_opts* opts,
                             llg_step_stats* stats, void* work, size_t work_bytes, void* stream) {
  if (!ctx || !m || !work) return fail(LLG_EARG, "null argument");
  CHK_STATUS(check_aligned({m, v_half, lam, work}));
  CHK_STATUS(check_params(prm));
  CHK_STATUS(check_opts(opts));
  if (!is_fin(picard_tol) || picard_tol <= 0 || picard_max < 1)
    return fail(LLG_EARG, "picard_tol must be > 0 and picard_max >= 1");
  const Ctx& c = ctx->c;
  Work w = carve(c, opts->restart, opts->prec, work);
  if (work_bytes < w.bytes) return fail(LLG_ENOMEM, "workspace smaller than llg_workspace_bytes()");
  CHK_STATUS(ensure_device(c));
  hipStream_t st = as_stream(stream);
  const long long ng = c.ng;
  llg_params p2 = *prm;
  p2.theta = 0.5;
  llg_solver_opts o = *opts;
  o.use_x0 = 1;
  o.transpose = 0;
  const double k = prm->dt;
  if (stats) std::memset(stats, 0, sizeof(*stats));
  CHK(hipMemcpyAsync(w.m0, m, sizeof(double) * 3 * ng, hipMemcpyDeviceToDevice, st));
  // Step-constant part of the right-hand side, C_hat Delta_N m^n + (1+alpha^2) h_ext.
  // With a lower-order field it is kept in l0 and (1+alpha^2) L_low m_hat^p is
  // added at every Picard iteration (the field frozen at the midpoint, eq. "C-N").
  const bool low = has_low(prm);
  // without a lower-order field the diagnostics' (-Delta_N) m^n comes with the RHS
  const bool lap0 = !low && stats;
  CHK(op_rhs(c, &p2, w.m0, w.b, st, lap0 ? w.l0 : nullptr));
  if (low) CHK(hipMemcpyAsync(w.l0, w.b, sizeof(double) * 3 * ng, hipMemcpyDeviceToDevice, st));
  const FieldArgs fa_low = field_for(c, prm, 0.0, 0.0, 1.0);
  const NodalArgs na2 = nodal_for(&p2);
  if (v_half) {
    CHK(hipMemcpyAsync(w.vold, v_half, sizeof(double) * 3 * ng, hipMemcpyDeviceToDevice, st));
    CHK(hipMemcpyAsync(w.x, v_half, sizeof(double) * 3 * ng, hipMemcpyDeviceToDevice, st));
  } else {
    CHK(hipMemsetAsync(w.vold, 0, sizeof(double) * 3 * ng, st));
    CHK(hipMemsetAsync(w.x, 0, sizeof(double) * 3 * ng, st));
  }
  if (lam) CHK(hipMemcpyAsync(w.x + 3 * ng, lam, sizeof(double) * ng, hipMemcpyDeviceToDevice, st));
  else CHK(hipMemsetAsync(w.x + 3 * ng, 0, sizeof(double) * ng, st));
  CHK(nodal_axpy3(c, w.m0, 0.5 * k, w.vold, w.mh, st));
  int iters = 0, pic = 0;
  bool pconv = false, lconv = true;
  double change = 0;
  llg_status lin = LLG_OK;
  // Later solves of the loop reuse what the previous iteration established:
  // ||b|| (b is fixed within the step unless the lower-order field is
  // refrozen), the zero-node test and the float32 copy of m_hat (both from
  // the Picard update that formed m_hat).
  SolveHints hints;
  float* mh32 = opts->prec != LLG_FP64 ? w.m32 : nullptr;
  for (int p = 0; p < picard_max; ++p) {
    if (low) {
      CHK(op_field(c, fa_low, EPI_ADDF, na2, w.mh, w.b, st, nullptr, w.l0));
      hints.bnorm = -1;
      hints.rnorm = -1;
    }
    SolveResult r;
    lin = solve(c, &p2, w.mh, w.b, w.x, o, w, r, st, hints);
    iters += r.iters;
    pic++;
    if (lin != LLG_OK && lin != LLG_ENOCONV) return lin;
    if (lin == LLG_ENOCONV) lconv = false;
    if (!low) hints.bnorm = r.bnorm;
    // ||v^p - v^{p-1}||^2, ||v^p||^2, ||m_hat^{p+1}||^2, zero nodes of m_hat^{p+1};
    // vold <- v^p, mh <- m_hat^{p+1} (and its float32 copy).  Without a
    // lower-order field b is fixed, and only the nodal blocks of A change with
    // m_hat, so the residual of the solution for the next system is the
    // previous residual minus a nodal correction (updated in the same pass).
    const bool upd_r = !low && r.r_valid;
    double dn[5];
    CHK(picard_update(c, w.m0, w.x, w.vold, w.mh, 0.5 * k, c.scal, st, mh32, upd_r ? w.r : nullptr));
    CHK_STATUS(fetch(c, c.scal, 5, st, dn));
    hints.m_checked = true;
    hints.m32_ready = mh32 != nullptr;
    hints.rnorm = upd_r ? std::sqrt(dn[4]) : -1;
    const double dd = std::sqrt(dn[0]);
    const double num = opts->picard_norm == 0 ? 0.5 * k * dd : dd;
    const double ref = std::sqrt(opts->picard_norm == 0 ? dn[2] : dn[1]);
    change = ref > 0 ? num / ref : num;
    if (!is_fin(change)) return fail(LLG_ENAN, "non-finite Picard update");
    if (num <= picard_tol * ref) {
      pconv = true;
      break;
    }
    if (dn[3] > 0) return fail(LLG_EZERO_M, "some nodal midpoint magnetization is zero (Proposition 1 needs m_i != 0)");
  }
  CHK(nodal_axpy3(c, w.m0, k, w.x, m, st));
  if (v_half) CHK(hipMemcpyAsync(v_half, w.x, sizeof(double) * 3 * ng, hipMemcpyDeviceToDevice, st));
  if (lam) CHK(hipMemcpyAsync(lam, w.x + 3 * ng, sizeof(double) * ng, hipMemcpyDeviceToDevice, st));
  if (stats) {
    stats->picard_iters = pic;
    stats->lin_iters_total = iters;
    stats->converged = (pconv && lconv) ? 1 : 0;
    stats->picard_rel_change = change;
    // l0 = F(m^n), l1 = F(v) with F = C_hat/(1+alpha^2) (-Delta_N) (no lower-order
    // field) or -(h_exc + h_dem + h_ani) (with it); the diagnostic kernel uses
    // linearity for m^{n+1} = m^n + k v and the exact midpoint m^n + (k/2) v.
    NodalArgs nd = nodal_for(prm);
    double ecoef = prm->cexc;
    if (low) {
      CHK(op_negfield(c, prm, w.m0, w.l0, st));
      CHK(op_negfield(c, prm, w.x, w.l1, st));
      nd.chat = nd.hs;
      ecoef = 1.0;
    } else {
      if (!lap0) CHK(op_lap(c, w.m0, w.l0, st));
      CHK(op_lap(c, w.x, w.l1, st));
    }
    double d[5], len;
    CHK(midpoint_diag(c, nd, prm->alpha, ecoef, k, w.m0, w.x, w.x + 3 * ng, w.l0, w.l1, c.scal, st));
    CHK_STATUS(fetch(c, c.scal, 5, st, d));
    CHK(len_err(c, m, c.scal, st));
    CHK_STATUS(fetch(c, c.scal, 1, st, &len));
    const double vol = c.Lx * c.Ly * (c.dim == 3 ? c.Lz : 1.0);
    const double wq = vol / double(ng);
    const double econst = low ? prm->aniso_k * vol : 0.0;
    const double a = prm->alpha;
    stats->energy_before = wq * d[0] + econst;
    stats->energy_after = wq * d[1] + econst;
    stats->v_norm2 = wq * d[2];
    stats->dissipation_defect = stats->energy_after - stats->energy_before + a * k / (1 + a * a) * stats->v_norm2;
    stats->inexact_correction = k / (1 + a * a) * (wq * d[3] - wq * d[4]);
    stats->max_len_err = len;
  }
  CHK(hipStreamSynchronize(st));
  if (!lconv) return fail(LLG_ENOCONV, "a Picard linear solve did not converge");
  if (!pconv) return fail(LLG_EPICARD, "Picard iteration reached picard_max");
  return LLG_OK;
}

llg_status llg_step_midpoint_adjoint(llg_ctx* ctx, const llg_params* prm, const double* m_n, const double* v,
                                     const double* lam, double* gbar, double* hbar_field, double* hbar_uniform,
                                     const llg_solver_opts* opts, llg_solver_stats* stats, void* work,
                                     size_t work_bytes, void* stream) {
  const auto t0 = Clock::now();
  if (!ctx || !m_n || !v || !lam || !gbar || !work) return fail(LLG_EARG, "null argument");
  CHK_STATUS(check_aligned({m_n, v, lam, gbar, hbar_field, work}));
  CHK_STATUS(check_params(prm));
  CHK_STATUS(check_opts(opts));
  if (opts->prec != LLG_FP64) return fail(LLG_EARG, "the adjoint solve runs in float64 only");
  const Ctx& c = ctx->c;
  Work w = carve(c, opts->restart, opts->prec, work);
  if (work_bytes < w.bytes) return fail(LLG_ENOMEM, "workspace smaller than llg_workspace_bytes()");
  CHK_STATUS(ensure_device(c));
  hipStream_t st = as_stream(stream);
  const long long ng = c.ng, n4 = 4 * ng;
  llg_params p2 = *prm;
  p2.theta = 0.5;
  const double k = prm->dt;
  // midpoint m_half = m^n + (k/2) v builds the transposed preconditioner
  CHK(nodal_axpy3(c, m_n, 0.5 * k, v, w.mh, st));
  CHK_STATUS(check_m(c, w.mh, st));
  // rhs = (k gbar, 0)
  CHK(axpby(c, 3 * ng, k, gbar, 0.0, gbar, w.b, st));
  CHK(hipMemsetAsync(w.b + 3 * ng, 0, sizeof(double) * ng, st));
  const SymArgs sym_h = sym_for(c, p2.alpha, hcoef(&p2), false);
  const NodalArgs na = nodal_for(&p2);
  // With a lower-order field the velocity block of J^T gains -(k/2)(1+alpha^2) L_low,
  // so its Fourier part is the 3x3 multiplier alpha + (k/2)(1+alpha^2)[cexc |xi|^2 - L_low^].
  const bool low = has_low(prm);
  const FieldArgs fa_jt = field_for(c, prm, p2.alpha, hcoef(&p2), 0.5 * k * na.hs);
  Op JT = [&](const double* in, double* out) {
    if (low) return op_field(c, fa_jt, EPI_JT, na, in, out, st, m_n, v, lam);
    return pipe_d(c, PRO_COPY3, EPI_JT, sym_h, na, in, m_n, out, st, v, lam);
  };
  Op MT = [&](const double* in, double* out) { return op_apply(c, &p2, w.mh, in, out, true, st); };
  Op MTJT = [&](const double* in, double* out) {
    hipError_t e = JT(in, w.t);
    if (e != hipSuccess) return e;
    return MT(w.t, out);
  };
  llg_solver_opts o = *opts;
  o.use_x0 = 0;
  o.transpose = 0;
  ResidOp RJT = resid_op(c, EPI_JT, sym_h, na, m_n, st, v, lam);
  if (low) {
    RJT = [&c, fa_jt, na, m_n, st, v, lam](const double* x, const double* b, double* r) -> hipError_t {
      PipeIO<double, double, double> io{x, m_n, r, c.ng, v, lam};
      io.rhs = b;
      io.red = c.partial;
      hipError_t e = run_field(c, fa_jt, EPI_JT, na, io, st);
      if (e != hipSuccess) return e;
      return reduce_flat(c, xinv_blocks(c), c.scal, st);
    };
  }
  SolveResult r;
  llg_status s;
  if (!low && o.orth == 0) {
    // one pipeline per iteration: J^T M^{-T} = [I + (N - lambda I)(calH + lambda I)^{-1}]
    // (calS + lambda I)^{-T} with N node-wise, right preconditioning
    const SymArgs sym_ap = sym_for(c, p2.alpha + p2.shift, hcoef(&p2), true);
    OpDots JTMT = [&](const double* in, double* out, const BasisDots* bd, bool ready) -> hipError_t {
      PipeIO<double, double, double> io{in, w.mh, out, c.ng, v, lam};
      return run_pipeline<double, double, double>(c, ready ? PRO_NONE : PRO_M2T, EPI_JT_RIGHT, sym_ap, na, io, st,
                                                  bd, c.dots);
    };
    const FirstUpd<double> fu{[&](int j) { return xfwd_upd_supported(c, PRO_M2T, false, j, o.fuse_update); },
                              [&](const UpdFirst& ua, const double* wv, double* out) {
                                return run_xfwd_upd(c, PRO_M2T, na, ua, wv, w.mh, out, st);
                              }};
    s = gmres_right(c, RJT, MT, JTMT, w.b, w.x, o, w, r, st, &fu);
  } else {
    s = gmres_left(c, RJT, MT, MTJT, w.b, w.x, o, w, r, st);
  }
  fill_stats(r, stats);
  if (stats) stats->ms = ms_since(t0);
  if (s != LLG_OK) return s;
  // gbar update and field gradients: gbar -= v x mu_v + chat F mu_v + r mu_v - v mu_r,
  // F = (-Delta_N) (chat = C_hat) or -(h_exc + h_dem + h_ani) (chat = 1 + alpha^2)
  NodalArgs nf = na;
  if (low) {
    CHK(op_negfield(c, prm, w.x, w.l0, st));
    nf.chat = nf.hs;
  } else {
    CHK(op_lap(c, w.x, w.l0, st));
  }
  CHK(adjoint_finish(c, nf, v, lam, w.x, w.l0, gbar, hbar_field, c.scal, st));
  double hs3[3];
  CHK_STATUS(fetch(c, c.scal, 3, st, hs3));
  if (hbar_uniform)
    for (int i = 0; i < 3; ++i) hbar_uniform[i] += hs3[i];
  (void)n4;
  return LLG_OK;
}

}  // extern "C"
