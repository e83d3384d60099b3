// Launchers of the streaming vector kernels (krylov.hip) and the nodal
// kernels of the steppers (nodal.hip).
#pragma once
#include "llg_internal.h"

namespace llg {

struct Coefs {
  double c[64];
  int n;
};

// Delayed CGS2 keeps the basis as the raw directions U = [u_0 .. u_j]
// (column 0 at u0, column i >= 1 at U1 + (i - 1) ld); Q = U T^{-1} with T
// upper triangular, column j of T = [a; beta_j], a = Q_j^T u_j.
struct DcgsCoef {
  double a[kDcgsMaxCols];     // a = Q_j^T u_j (entries 0..j-1)
  double minv[kDcgsMaxCols];  // column j of T^{-1}: [-T_j^{-1} a / beta_j; 1 / beta_j]
  double inv_beta;            // 1 / beta_j
  int j;
};

// Pass 1: out = [U_i.w (i <= j)].  j < kDcgsMaxCols.  w is float64, or the
// float32 output of a float32 operator (its values convert exactly).
hipError_t dcgs_dots(const Ctx& c, const double* u0, const double* U1, long long ld, int j, const double* w,
                     long long n, double* out, hipStream_t st);
hipError_t dcgs_dots(const Ctx& c, const double* u0, const double* U1, long long ld, int j, const float* w,
                     long long n, double* out, hipStream_t st);
// Pass-1 products left unreduced by the operator's last pass (small grids,
// BasisDots::defer): nb block partials per value at part, value-major.  The
// update pass reduces them (the same fixed order in every block), uses them,
// and stores the reduced values at out (device) and mirror (host-mapped).
struct DeferredDots {
  const double* part = nullptr;
  int nb = 0;
  double* out = nullptr;
  double* mirror = nullptr;
};

// Pass 2 (p = pass-1 output on the device): with gamma = T_{j+1}^{-1} [b; e_j],
// b = T_j^{-T} p_{<j}, e_j = (p_j - a.b) / beta_j (computed on the device),
//   unew = (w - U gamma) / beta_j,   out = [U_i.unew (i <= j), unew.unew].
// unew must not alias w or a basis column 0..j.
// With dp (dp->nb > 0) p is not read: the pass-1 products come from dp.
hipError_t dcgs_update(const Ctx& c, const double* u0, const double* U1, long long ld, const DcgsCoef& cf,
                       const double* p, const double* w, double* unew, long long n, double* out, hipStream_t st,
                       const DeferredDots* dp = nullptr);
hipError_t dcgs_update(const Ctx& c, const double* u0, const double* U1, long long ld, const DcgsCoef& cf,
                       const double* p, const float* w, double* unew, long long n, double* out, hipStream_t st,
                       const DeferredDots* dp = nullptr);

// The coefficient step of pass 2 alone (k_dcgs_coef): gamma (device, j + 1
// values) for a pass 2 run elsewhere (k_xfwd_upd).
hipError_t dcgs_coef(const Ctx& c, const DcgsCoef& cf, const double* p, const double** gamma, hipStream_t st);

// out[i] = sum (or max) of the nb value-major partials of value i, i < nv
hipError_t reduce_partials(const Ctx& c, int nb, int nv, double* out, bool is_max, hipStream_t st);
// Blocks of a reducing streaming kernel over n elements: about four elements
// per thread, at most kNodalBlocksMax; depends only on n (deterministic order).
constexpr int kNodalBlocksMax = 16384;
inline int nodal_blocks(long long n) {
  long long g = (n + 4 * kRedThreads - 1) / (4 * kRedThreads);
  if (g > kNodalBlocksMax) g = kNodalBlocksMax;
  return int(g < 1 ? 1 : g);
}
// out[i] = sum of the nb value-major partials of value i, i < nv (1024-thread reducer)
hipError_t reduce_partials_n(const Ctx& c, int nb, int nv, double* out, hipStream_t st);
// Blocks of a delayed-CGS2 pass over n2 16-byte elements: one element per
// thread of a 512-thread block (2 kRedThreads), at most kRedBlocksMax blocks
// (grid-strided beyond); depends only on n2 (deterministic order).
inline int red_blocks(long long n2) {
  long long g = (n2 + 2 * kRedThreads - 1) / (2 * kRedThreads);
  if (g > kRedBlocksMax) g = kRedBlocksMax;
  return int(g < 1 ? 1 : g);
}
// out[0] = sum of c.partial[0 .. nb) (the x-inverse residual partials)
hipError_t reduce_flat(const Ctx& c, int nb, double* out, hipStream_t st);
// out[i] = V_i . w  (i < nv; V_i = V + i*ld)
hipError_t cgs_dots(const Ctx& c, const double* V, long long ld, int nv, const double* w, long long n, double* out,
                    hipStream_t st);
// w -= sum_i cf[i] V_i ; out[i] = V_i . w
hipError_t cgs_update_dots(const Ctx& c, const double* V, long long ld, int nv, const double* cf, double* w,
                           long long n, double* out, hipStream_t st);
// out_vec = w - sum_i cf[i] V_i ; out_nrm2[0] = ||out_vec||^2
hipError_t cgs_update_norm(const Ctx& c, const double* V, long long ld, int nv, const double* cf, const double* w,
                           double* out_vec, long long n, double* out_nrm2, hipStream_t st);
hipError_t scale_invnorm(const Ctx& c, double* y, const double* x, const double* nrm2, long long n, hipStream_t st);
hipError_t axpby(const Ctx& c, long long n, double a, const double* x, double b, const double* y, double* out, hipStream_t st);
hipError_t lincomb(const Ctx& c, long long n, const Coefs& cf, const double* V, long long ld, double* x, hipStream_t st);
hipError_t lincomb(const Ctx& c, long long n, const Coefs& cf, const float* V, long long ld, double* x, hipStream_t st);
hipError_t to_f32(const Ctx& c, long long n, const double* a, float* b, hipStream_t st);
// out[0] = x.y (x.x if y null), out[1] = x.x
hipError_t dot_and_norm(const Ctx& c, const double* x, const double* y, long long n, double* out, hipStream_t st);

// ---- nodal.hip ----
// out[0] = min_i |m_i|^2, out[1] = 1 if any entry of m is non-finite
hipError_t m_check(const Ctx& c, const double* m, double* out, hipStream_t st);
// m <- (m + k v) / |m + k v| ; out[0] = max_i | |m_i| - 1 | after normalization
hipError_t euler_update(const Ctx& c, double* m, const double* v, double k, double* out, hipStream_t st);
// out = m + a v  (3 planes)
hipError_t nodal_axpy3(const Ctx& c, const double* m, double a, const double* v, double* out, hipStream_t st);
// v = the velocity planes of the saddle unknown x = (v, lam) (4 planes).
// out = {||v - vold||^2, ||v||^2, ||m0 + a v||^2, number of nodes with |m0 + a v|^2 <= 1e-300,
// ||r_new||^2}; then vold <- v, mh <- m0 + a v (3 planes), mh32 <- float(mh) when set, and
// when r is set (4 planes, r = b - A(mh) x on entry) r <- r - (dm x v + dm lam, -dm . v),
// dm = a (v - vold): the residual of x for the system at the new mh.
hipError_t picard_update(const Ctx& c, const double* m0, const double* v, double* vold, double* mh, double a,
                         double* out, hipStream_t st, float* mh32 = nullptr, double* r = nullptr);
// max_i | |m_i| - 1 |
hipError_t len_err(const Ctx& c, const double* m, double* out, hipStream_t st);
// Midpoint diagnostics (see nodal.hip); out[0..6]
hipError_t midpoint_diag(const Ctx& c, const NodalArgs& na, double alpha, double cexc, double k, const double* m0,
                         const double* v, const double* r, const double* lm0, const double* lv, double* out,
                         hipStream_t st);
// Adjoint helpers (nodal.hip)
hipError_t adjoint_finish(const Ctx& c, const NodalArgs& na, const double* v, const double* r, const double* mu,
                          const double* lmu, double* gbar, double* hbar_field, double* out_hsum, hipStream_t st);

}  // namespace llg
