// Spectral pipeline: layout, argument blocks, prologue / epilogue modes.
//
// A pipeline applies one real, even Fourier multiplier to three real grid
// planes ("filtered fields") and combines the result node by node with other
// planes.  Every operator of the hot path is such a pipeline:
//
//   matvec      A x         : filtered v with a + b|xi|^2, a = alpha,
//                             b = theta k C_hat (Sec. 2.4, eq. "saddle point
//                             system"), epilogue adds m x v + m r, -m.v
//   apply       M^{-1} p    : filtered p_v with 1/(alpha + lambda + b|xi|^2)
//                             (Algorithm 1), epilogue = closed-form 4x4
//                             nodal inverse (eq. "inverse S")
//   apply^T     M^{-T} p    : prologue = transposed nodal inverse, then
//                             Algorithm 1
//   fused       M^{-1} A x  : M2^{-1}[x + M1^{-1}((calS - lambda I) x)], an
//                             identity because A = M1 + calS - lambda I
//   adjoint     J^T M^{-T} y: [I + (N - lambda I) M1^{-1}] M2^{-T} y, N = J^T -
//                             calH node-wise (the midpoint Jacobian, no
//                             lower-order field); right preconditioning
//   rhs         C_hat Delta_N m + (1+alpha^2) h (Sec. 2.4, eq. "total system")
//
// Grid planes are SoA, node index i = x + nx (y + ny z).  Between passes the
// three filtered fields live in one complex spectral buffer: each (y, z) row
// holds three half spectra (kx = 0..nx/2) back to back, 3 (nx/2+1) complex
// values, padded to a row stride rs that is a multiple of 16 elements.
#pragma once
#include "fft_core.h"

namespace llg {

// Line lengths with kernel instantiations: half-lengths nx/2 of the x passes
// and lengths of the y / z passes (plans in fft_core.h).
#define LLG_FOR_NH(X) \
  X(2) X(3) X(4) X(5) X(6) X(8) X(10) X(12) X(16) X(20) X(24) X(32) X(40) X(48) X(64) X(80) X(96) X(128) \
  X(160) X(192) X(256)
#define LLG_FOR_AXIS(X) \
  X(4) X(6) X(8) X(10) X(12) X(16) X(20) X(24) X(32) X(40) X(48) X(64) X(80) X(96) X(128) X(160) X(192) \
  X(256) X(320) X(384) X(512)

// FFT plan key of the x passes for elements of elem_bytes bytes and half-length
// nh: the float64 passes at nh = 128, 256 take the finer plan (fewer points
// per thread, half the LDS per block; see kPlanFine).
__host__ __device__ constexpr int x_plan_key(int elem_bytes, int nh) {
  return (elem_bytes == 8 && (nh == 128 || nh == 256)) ? (nh | kPlanFine) : nh;
}

// FFT plan key of the y / z passes: with LLG_AXIS_FINE_F64 the float64
// passes at N = 256 take the finer plan as well.
#ifndef LLG_AXIS_FINE_F64
#define LLG_AXIS_FINE_F64 0
#endif
__host__ __device__ constexpr int axis_plan_key(int elem_bytes, int n) {
  return (LLG_AXIS_FINE_F64 && elem_bytes == 8 && n == 256) ? (n | kPlanFine) : n;
}

inline bool nh_supported(int n) {
#define LLG_EQ(v) || n == v
  return false LLG_FOR_NH(LLG_EQ);
}
inline bool axis_supported(int n) { return false LLG_FOR_AXIS(LLG_EQ); }
#undef LLG_EQ

struct SpecGeom {
  int nx, ny, nz, nh;  // nh = nx / 2
  int cs;              // 3 (nh + 1) valid columns per row
  int rs;              // row stride in complex elements
  long long ng;        // nodes
};

struct SymArgs {
  double a, b;           // multiplier a + b |xi|^2 (or its inverse)
  double cx, cy, cz;     // 2 pi / L per axis
  double inv_ng;         // 1 / N_g
  int invert;            // 1: use 1 / (a + b |xi|^2)
};

struct NodalArgs {
  double lam;            // HSS shift lambda
  double hs;             // 1 + alpha^2 (field scaling)
  double chat;           // C_hat
  double hu0, hu1, hu2;  // uniform applied field
  double half_k;         // k / 2 (adjoint operator)
  const double* hfield;  // optional spatial field (3 planes) or null
};

enum ProMode : int {
  PRO_NONE = -1,   // no x-forward pass: the spectral buffer already holds the
                   // filtered fields' x spectra (left by k_xfwd_upd)
  PRO_COPY3 = 0,   // u = in[0..2]
  PRO_SMINUS = 1,  // u = m x v + m r - lambda v  (first half of the fused op)
  PRO_M2T = 2,     // u = ((lambda I + S~) p)_v / (lambda^2 + |m|^2)
};

enum EpiMode : int {
  EPI_STORE3 = 0,    // out[0..2] = F
  EPI_APPLY = 1,     // out = M2^{-1} (F, p_r / lambda)
  EPI_APPLY_T = 2,   // out = (F, ((lambda I + S~) p)_r / (lambda d))
  EPI_MATVEC = 3,    // out = (F + m x v + m r, -m.v)
  EPI_MATVEC_T = 4,  // out = (F - m x v - m r, m.v)
  EPI_FUSED = 5,     // out = M2^{-1} (x + (F, (-m.v - lambda r) / lambda))
  EPI_RHS = 6,       // out = (-C_hat F + (1+alpha^2) h, 0)
  EPI_JT = 7,        // out = J^T mu of the midpoint residual (adjoint), F = H mu_v
  EPI_APPLY_SYM = 8, // out = (F, p_r / lambda): (lambda I + calH)^{-1} p alone
  EPI_FUSED_SYM = 9, // out = x + (F, (-m.v - lambda r) / lambda): (lambda I + calH)^{-1} A x
  EPI_ADDF = 10,     // out = (aux_v - (1+alpha^2) F, 0): right-hand side with the lower-order field
  EPI_ENERGY = 11,   // no output: per-block partial sums of chat/2 m.F - m.h (discrete energy density)
  EPI_JT_RIGHT = 12, // out = J^T M^{-T} y of the midpoint adjoint, right-preconditioned (one pipeline,
                     // prologue PRO_M2T on m = m_half, F = (calH + lambda I)^{-1} of the prologue)
};

// Symmetric 3x3 Fourier multiplier of the lower-order field pipeline:
//   M(xi) = (s_id + s_ex |xi|^2) I + s_dm xi~ xi~^T / |xi|^2 + s_an e e^T,
// xi~ = xi with the Nyquist entry of each axis set to zero (spectral first
// derivative of real data), the demagnetizing term zero at xi = 0.  With
// s_id = 0, s_ex = cexc, s_dm = demag, s_an = -2K the output is minus the
// linear part of the effective field (exchange, periodic demagnetization of
// Sec. 2.2, uniaxial anisotropy of Sec. 2.1).
struct FieldArgs {
  double s_id, s_ex, s_dm, s_an;
  double e0, e1, e2;   // easy axis
  double cx, cy, cz;   // 2 pi / L per axis
  double inv_ng;
};

// Pointers of one pipeline call.  "in" planes feed the prologue (and are
// re-read by epilogues that need x or p); "m" is the magnetization the
// nodal blocks are built on.
template <typename T, typename TIn, typename TOut>
struct PipeIO {
  const TIn* in;     // 4 planes (x or p), or 3 planes for PRO_COPY3 + EPI_STORE3/RHS
  const T* m;        // 3 planes (may be null for modes that do not use it)
  TOut* out;         // 4 planes (3 for EPI_STORE3)
  long long ng;
  const T* aux_v;    // EPI_JT, EPI_JT_RIGHT: forward velocity v (3 planes)
  const T* aux_r;    // EPI_JT, EPI_JT_RIGHT: forward multiplier (1 plane)
  // Residual form: when rhs is set, the pipeline writes out = rhs - (operator
  // output) and each x-inverse block stores the partial sum of squares of its
  // outputs at red[blockIdx.x].  EPI_ENERGY writes no output and stores the
  // block's partial sum of the energy density at red[blockIdx.x].
  const TOut* rhs = nullptr;
  double* red = nullptr;
  // EPI_RHS: when set, the filtered fields F = (-Delta_N) in (3 planes) are
  // stored here as well.
  T* out_f = nullptr;
};

// Arnoldi inner products taken by an x-inverse pass on its own output (the
// precision form's matvec): with basis directions u_0 at u0 and u_i at
// U1 + (i - 1) ld (1 <= i < nv), each block stores the partial sums of
// u_i . out over its nodes at partial[i * gridDim.x + blockIdx.x].
constexpr int kBasisDotsMax = 32;
struct BasisDots {
  const double* u0 = nullptr;
  const double* U1 = nullptr;
  long long ld = 0;
  int nv = 0;
  double* partial = nullptr;
  double* out = nullptr;  // when set, the reduced products go here instead of the caller's default
  // Deferred reduction (small grids): when defer is set and the pass has at
  // most kDeferMaxBlocks blocks, it leaves its block partials at defer
  // (value-major) instead of reducing them and stores its block count at
  // *defer_nb; otherwise it reduces as usual (products at out) and stores 0.
  // The Arnoldi update pass reduces deferred partials.
  double* defer = nullptr;
  int* defer_nb = nullptr;
};
// Largest block count of a pass whose products are left for deferred reduction.
constexpr int kDeferMaxBlocks = 64;

// Delayed-CGS2 pass 2 of Arnoldi step j carried by the first x pass of the
// operator of step j + 1 (k_xfwd_upd): with basis directions u_0 at u0 and
// u_q at U1 + (q - 1) ld, the pass forms
//   u_new = (w - sum_{q <= j} gamma_q u_q) * inv_beta
// node by node, stores it at unew (the next basis direction), feeds it to
// the operator's prologue, and leaves the block partials of u_q . u_new
// (q <= j) and u_new . u_new at partial[q * gridDim.x + blockIdx.x],
// q = 0 .. j + 1.
struct UpdFirst {
  const double* u0 = nullptr;
  const double* U1 = nullptr;
  long long ld = 0;
  int j = 0;
  const double* gamma = nullptr;  // j + 1 coefficients (device)
  double inv_beta = 0;
  double* unew = nullptr;         // must not alias w or a basis column 0..j
  double* partial = nullptr;
};

}  // namespace llg
