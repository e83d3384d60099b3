// Streaming vector kernels of the Krylov solvers and the steppers.
//
// All reductions are two-stage and deterministic: a fixed grid of kRedBlocks
// blocks accumulates per-thread partial sums in a fixed order, reduces them
// across the block by wavefront shuffles, and writes one partial per block;
// a second kernel sums the kRedBlocks partials of each value in a fixed tree.
// The grid never depends on timing, so every reduced value is bitwise
// reproducible from run to run.
//
// Arnoldi orthogonalization is classical Gram-Schmidt with one
// re-orthogonalization (CGS2), as three streaming passes over the basis:
//   A: h = V^T w;   B: w -= V h, s = V^T w;   C: w -= V s, ||w||^2.
#include <cmath>
#include <utility>

#include "krylov.h"

namespace llg {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Non-temporal 16-byte load / store: the Krylov vectors (hundreds of MB each)
// are streamed once per pass and never reused from cache before eviction.
__device__ __forceinline__ double2 ldnt(const double2* p) {
  double2 v;
  v.x = __builtin_nontemporal_load(&p->x);
  v.y = __builtin_nontemporal_load(&p->y);
  return v;
}
__device__ __forceinline__ void stnt(double2* p, double2 v) {
  __builtin_nontemporal_store(v.x, &p->x);
  __builtin_nontemporal_store(v.y, &p->y);
}

// Reduce acc[0..nv) over the block and store partial[blockIdx.x * kMaxDots + i].
template <int MAXV, bool MAX = false>
__device__ __forceinline__ void block_store(double (&acc)[MAXV], int nv, double* __restrict__ partial) {
  __shared__ double sm[kRedThreads / 64][MAXV];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < MAXV; ++i) {
    if (i < nv) {
      const double s = MAX ? wave_max(acc[i]) : wave_sum(acc[i]);
      if (lane == 0) sm[wv][i] = s;
    }
  }
  __syncthreads();
  if (threadIdx.x < nv) {
    double s = sm[0][threadIdx.x];
#pragma unroll
    for (int w = 1; w < kRedThreads / 64; ++w) s = MAX ? fmax(s, sm[w][threadIdx.x]) : s + sm[w][threadIdx.x];
    partial[blockIdx.x * kMaxDots + threadIdx.x] = s;
  }
}

// out[i] = sum (or max) over blocks of partial[b * kMaxDots + i]; one block per value.
template <bool MAX>
__global__ __launch_bounds__(kRedThreads) void k_reduce(const double* __restrict__ partial, int nb,
                                                       double* __restrict__ out) {
  const int i = blockIdx.x;
  double s = MAX ? -INFINITY : 0.0;
  for (int b = threadIdx.x; b < nb; b += kRedThreads) {
    const double v = partial[b * kMaxDots + i];
    s = MAX ? fmax(s, v) : s + v;
  }
  __shared__ double sm[kRedThreads / 64];
  s = MAX ? wave_max(s) : wave_sum(s);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = sm[0];
    for (int w = 1; w < kRedThreads / 64; ++w) t = MAX ? fmax(t, sm[w]) : t + sm[w];
    out[i] = t;
  }
}

// out[0] = sum of partial[0 .. nb) (stride 1), fixed order
__global__ __launch_bounds__(kRedThreads) void k_reduce_flat(const double* __restrict__ partial, int nb,
                                                            double* __restrict__ out) {
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += kRedThreads) s += partial[b];
  __shared__ double sm[kRedThreads / 64];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = sm[0];
    for (int w = 1; w < kRedThreads / 64; ++w) t += sm[w];
    out[0] = t;
  }
}

// ---- CGS2 passes ----------------------------------------------------------
template <int MAXV>
__global__ __launch_bounds__(kRedThreads) void k_mdot(const double* __restrict__ V, long long ld, int nv,
                                                     const double* __restrict__ w, long long n,
                                                     double* __restrict__ partial) {
  double acc[MAXV];
#pragma unroll
  for (int i = 0; i < MAXV; ++i) acc[i] = 0.0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
    const double we = w[e];
#pragma unroll
    for (int i = 0; i < MAXV; ++i)
      if (i < nv) acc[i] = fma(V[i * ld + e], we, acc[i]);
  }
  block_store<MAXV>(acc, nv, partial);
}

template <int MAXV>
__global__ __launch_bounds__(kRedThreads) void k_update_mdot(const double* __restrict__ V, long long ld, int nv,
                                                            const double* __restrict__ c, double* __restrict__ w,
                                                            long long n, double* __restrict__ partial) {
  double acc[MAXV], cc[MAXV];
#pragma unroll
  for (int i = 0; i < MAXV; ++i) {
    acc[i] = 0.0;
    cc[i] = i < nv ? c[i] : 0.0;
  }
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
    double vv[MAXV];
    double we = w[e];
#pragma unroll
    for (int i = 0; i < MAXV; ++i)
      if (i < nv) {
        vv[i] = V[i * ld + e];
        we = fma(-cc[i], vv[i], we);
      }
    w[e] = we;
#pragma unroll
    for (int i = 0; i < MAXV; ++i)
      if (i < nv) acc[i] = fma(vv[i], we, acc[i]);
  }
  block_store<MAXV>(acc, nv, partial);
}

template <int MAXV>
__global__ __launch_bounds__(kRedThreads) void k_update_norm(const double* __restrict__ V, long long ld, int nv,
                                                            const double* __restrict__ c,
                                                            const double* __restrict__ w, double* __restrict__ out,
                                                            long long n, double* __restrict__ partial) {
  double cc[MAXV];
#pragma unroll
  for (int i = 0; i < MAXV; ++i) cc[i] = i < nv ? c[i] : 0.0;
  double acc[1] = {0.0};
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
    double we = w[e];
#pragma unroll
    for (int i = 0; i < MAXV; ++i)
      if (i < nv) we = fma(-cc[i], V[i * ld + e], we);
    out[e] = we;
    acc[0] = fma(we, we, acc[0]);
  }
  block_store<1>(acc, 1, partial);
}

// ---- CGS2 with delayed re-orthogonalization (two passes per iteration) -------
// Both passes are instantiated for the exact number J of basis vectors, so
// every basis load of a thread is unconditional and the loads of one element
// are all in flight together.
//
// Pass 1: out = [Q_i.u (i < J), Q_i.w (i < J), u.u, u.w]  (HAS_W = false: only
// Q_i.u and u.u).  Streams Q_0..Q_{J-1}, u and w once.
template <int J, bool HAS_W>
__global__ __launch_bounds__(kRedThreads) void k_dcgs_dots(const double2* __restrict__ Q, long long ld2,
                                                          const double2* __restrict__ u,
                                                          const double2* __restrict__ w, long long n2,
                                                          double* __restrict__ partial) {
  constexpr int NA = J > 0 ? J : 1;
  double au[NA], aw[NA];
#pragma unroll
  for (int i = 0; i < NA; ++i) au[i] = aw[i] = 0.0;
  double cuu = 0.0, cuw = 0.0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n2; e += stride) {
    const double2 uu = ldnt(u + e);
    double2 ww{0.0, 0.0};
    if constexpr (HAS_W) ww = ldnt(w + e);
    double2 q[NA];
#pragma unroll
    for (int i = 0; i < J; ++i) q[i] = ldnt(Q + i * ld2 + e);
    cuu = fma(uu.x, uu.x, fma(uu.y, uu.y, cuu));
    if constexpr (HAS_W) cuw = fma(uu.x, ww.x, fma(uu.y, ww.y, cuw));
#pragma unroll
    for (int i = 0; i < J; ++i) {
      au[i] = fma(q[i].x, uu.x, fma(q[i].y, uu.y, au[i]));
      if constexpr (HAS_W) aw[i] = fma(q[i].x, ww.x, fma(q[i].y, ww.y, aw[i]));
    }
  }
  __shared__ double sm[kRedThreads / 64][2 * J + 2];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < J; ++i) {
    const double x = wave_sum(au[i]);
    const double y = HAS_W ? wave_sum(aw[i]) : 0.0;
    if (lane == 0) {
      sm[wv][i] = x;
      sm[wv][J + i] = y;
    }
  }
  {
    const double x = wave_sum(cuu), y = HAS_W ? wave_sum(cuw) : 0.0;
    if (lane == 0) {
      sm[wv][2 * J] = x;
      sm[wv][2 * J + 1] = y;
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * J + 2) {
    double t = sm[0][threadIdx.x];
#pragma unroll
    for (int k = 1; k < kRedThreads / 64; ++k) t += sm[k][threadIdx.x];
    partial[blockIdx.x * kMaxDots + threadIdx.x] = t;
  }
}

// Pass 2: q_J = (u - sum_i a_i Q_i) / beta ;  u <- (w - sum_i e_i Q_i - e_J q_J) / beta.
template <int J>
__global__ __launch_bounds__(256) void k_dcgs_update(const double2* __restrict__ Q, long long ld2, DcgsCoef cf,
                                                    double2* u, const double2* __restrict__ w,
                                                    double2* __restrict__ qj, long long n2) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n2; e += stride) {
    double2 sa = ldnt(u + e), se = ldnt(w + e);
    double2 q[J > 0 ? J : 1];
#pragma unroll
    for (int i = 0; i < J; ++i) q[i] = ldnt(Q + i * ld2 + e);
#pragma unroll
    for (int i = 0; i < J; ++i) {
      sa.x = fma(-cf.a[i], q[i].x, sa.x);
      sa.y = fma(-cf.a[i], q[i].y, sa.y);
      se.x = fma(-cf.e[i], q[i].x, se.x);
      se.y = fma(-cf.e[i], q[i].y, se.y);
    }
    const double2 qn{sa.x * cf.inv_beta, sa.y * cf.inv_beta};
    stnt(qj + e, qn);
    stnt(u + e, double2{(se.x - cf.ej * qn.x) * cf.inv_beta, (se.y - cf.ej * qn.y) * cf.inv_beta});
  }
}

// ---- simple vector kernels -------------------------------------------------
__global__ void k_scale_invnorm(double* __restrict__ y, const double* __restrict__ x,
                                const double* __restrict__ nrm2, long long n) {
  const double s = 1.0 / sqrt(nrm2[0]);
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) y[e] = x[e] * s;
}

__global__ void k_axpby(long long n, double a, const double* __restrict__ x, double b,
                        const double* __restrict__ y, double* __restrict__ out) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride)
    out[e] = a * x[e] + b * y[e];
}

template <typename TV>
__global__ void k_lincomb(long long n, Coefs cf, const TV* __restrict__ V, long long ld,
                          double* __restrict__ x) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
    double s = x[e];
    for (int i = 0; i < cf.n; ++i) s = fma(cf.c[i], double(V[i * ld + e]), s);
    x[e] = s;
  }
}

template <typename TA, typename TB>
__global__ void k_convert(long long n, const TA* __restrict__ a, TB* __restrict__ b) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) b[e] = TB(a[e]);
}

// sum of x.y and of x.x over n elements (two values)
__global__ __launch_bounds__(kRedThreads) void k_dot2(const double* __restrict__ x, const double* __restrict__ y,
                                                     long long n, double* __restrict__ partial) {
  double acc[2] = {0.0, 0.0};
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
    const double a = x[e];
    acc[0] = fma(a, y ? y[e] : a, acc[0]);
    acc[1] = fma(a, a, acc[1]);
  }
  block_store<2>(acc, 2, partial);
}

// sum (a - b)^2 and sum a^2
__global__ __launch_bounds__(kRedThreads) void k_diffnorm(const double* __restrict__ a, const double* __restrict__ b,
                                                         long long n, double* __restrict__ partial) {
  double acc[2] = {0.0, 0.0};
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
    const double av = a[e], d = av - (b ? b[e] : 0.0);
    acc[0] = fma(d, d, acc[0]);
    acc[1] = fma(av, av, acc[1]);
  }
  block_store<2>(acc, 2, partial);
}

// ---- host launchers --------------------------------------------------------
static inline unsigned grid_for(long long n) {
  long long g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  return (unsigned)(g < 1 ? 1 : g);
}

hipError_t reduce_partials_n(const Ctx& c, int nb, int nv, double* out, hipStream_t st) {
  ProfScope ps(c.prof, st, KK_REDUCE, 8.0 * nb * nv);
  hipLaunchKernelGGL((k_reduce<false>), dim3(nv), dim3(kRedThreads), 0, st, c.partial, nb, out);
  return hipGetLastError();
}

hipError_t reduce_flat(const Ctx& c, int nb, double* out, hipStream_t st) {
  ProfScope ps(c.prof, st, KK_REDUCE, 8.0 * nb);
  hipLaunchKernelGGL(k_reduce_flat, dim3(1), dim3(kRedThreads), 0, st, c.partial, nb, out);
  return hipGetLastError();
}

hipError_t reduce_partials(const Ctx& c, int nv, double* out, bool is_max, hipStream_t st) {
  ProfScope ps(c.prof, st, KK_REDUCE, 8.0 * kRedBlocks * nv);
  if (is_max)
    hipLaunchKernelGGL((k_reduce<true>), dim3(nv), dim3(kRedThreads), 0, st, c.partial, kRedBlocks, out);
  else
    hipLaunchKernelGGL((k_reduce<false>), dim3(nv), dim3(kRedThreads), 0, st, c.partial, kRedBlocks, out);
  return hipGetLastError();
}

template <int MAXV>
static void mdot_t(const Ctx& c, const double* V, long long ld, int nv, const double* w, long long n, hipStream_t st) {
  hipLaunchKernelGGL((k_mdot<MAXV>), dim3(kRedBlocks), dim3(kRedThreads), 0, st, V, ld, nv, w, n, c.partial);
}
hipError_t cgs_dots(const Ctx& c, const double* V, long long ld, int nv, const double* w, long long n, double* out,
                    hipStream_t st) {
  {
  ProfScope ps(c.prof, st, KK_CGS_DOTS, 8.0 * n * (nv + 1));
  if (nv <= 8) mdot_t<8>(c, V, ld, nv, w, n, st);
  else if (nv <= 16) mdot_t<16>(c, V, ld, nv, w, n, st);
  else if (nv <= 32) mdot_t<32>(c, V, ld, nv, w, n, st);
  else mdot_t<64>(c, V, ld, nv, w, n, st);
  }
  return reduce_partials(c, nv, out, false, st);
}

template <int MAXV>
static void upd_t(const Ctx& c, const double* V, long long ld, int nv, const double* cf, double* w, long long n,
                  hipStream_t st) {
  hipLaunchKernelGGL((k_update_mdot<MAXV>), dim3(kRedBlocks), dim3(kRedThreads), 0, st, V, ld, nv, cf, w, n, c.partial);
}
hipError_t cgs_update_dots(const Ctx& c, const double* V, long long ld, int nv, const double* cf, double* w,
                           long long n, double* out, hipStream_t st) {
  {
  ProfScope ps(c.prof, st, KK_CGS_UPDATE_DOTS, 8.0 * n * (nv + 2));
  if (nv <= 8) upd_t<8>(c, V, ld, nv, cf, w, n, st);
  else if (nv <= 16) upd_t<16>(c, V, ld, nv, cf, w, n, st);
  else if (nv <= 32) upd_t<32>(c, V, ld, nv, cf, w, n, st);
  else upd_t<64>(c, V, ld, nv, cf, w, n, st);
  }
  return reduce_partials(c, nv, out, false, st);
}

template <int MAXV>
static void updn_t(const Ctx& c, const double* V, long long ld, int nv, const double* cf, const double* w,
                   double* o, long long n, hipStream_t st) {
  hipLaunchKernelGGL((k_update_norm<MAXV>), dim3(kRedBlocks), dim3(kRedThreads), 0, st, V, ld, nv, cf, w, o, n,
                     c.partial);
}
hipError_t cgs_update_norm(const Ctx& c, const double* V, long long ld, int nv, const double* cf, const double* w,
                           double* out_vec, long long n, double* out_nrm2, hipStream_t st) {
  {
  ProfScope ps(c.prof, st, KK_CGS_UPDATE_NORM, 8.0 * n * (nv + 2));
  if (nv <= 8) updn_t<8>(c, V, ld, nv, cf, w, out_vec, n, st);
  else if (nv <= 16) updn_t<16>(c, V, ld, nv, cf, w, out_vec, n, st);
  else if (nv <= 32) updn_t<32>(c, V, ld, nv, cf, w, out_vec, n, st);
  else updn_t<64>(c, V, ld, nv, cf, w, out_vec, n, st);
  }
  return reduce_partials(c, 1, out_nrm2, false, st);
}


template <int J>
static void dd_t(const Ctx& c, const double* Q, long long ld, const double* u, const double* w, long long n,
                 hipStream_t st) {
  auto Q2 = reinterpret_cast<const double2*>(Q);
  auto u2 = reinterpret_cast<const double2*>(u);
  auto w2 = reinterpret_cast<const double2*>(w);
  const int nb = red_blocks(n / 2);
  if (w)
    hipLaunchKernelGGL((k_dcgs_dots<J, true>), dim3(nb), dim3(kRedThreads), 0, st, Q2, ld / 2, u2, w2, n / 2,
                       c.partial);
  else
    hipLaunchKernelGGL((k_dcgs_dots<J, false>), dim3(nb), dim3(kRedThreads), 0, st, Q2, ld / 2, u2, w2,
                       n / 2, c.partial);
}

template <int J>
static void du_t(const Ctx& c, const double* Q, long long ld, const DcgsCoef& cf, double* u, const double* w,
                 double* qj, long long n, hipStream_t st) {
  const long long n2 = n / 2;
  long long g = (n2 + 255) / 256;  // one 16-byte element per thread
  if (g > (1LL << 30)) g = 1LL << 30;
  hipLaunchKernelGGL((k_dcgs_update<J>), dim3((unsigned)g), dim3(256), 0, st, reinterpret_cast<const double2*>(Q),
                     ld / 2, cf, reinterpret_cast<double2*>(u), reinterpret_cast<const double2*>(w),
                     reinterpret_cast<double2*>(qj), n2);
}

// Runtime J -> template instantiation J = 0..31.
template <template <int> class F, int J = 0>
struct JDispatch {
  template <typename... A>
  static void run(int j, A&&... args) {
    if (j == J) F<J>::go(std::forward<A>(args)...);
    else if constexpr (J < 31) JDispatch<F, J + 1>::run(j, std::forward<A>(args)...);
  }
};
template <int J>
struct DotsF {
  template <typename... A>
  static void go(A&&... a) { dd_t<J>(std::forward<A>(a)...); }
};
template <int J>
struct UpdF {
  template <typename... A>
  static void go(A&&... a) { du_t<J>(std::forward<A>(a)...); }
};

hipError_t dcgs_dots(const Ctx& c, const double* Q, long long ld, int j, const double* u, const double* w,
                     long long n, double* out, hipStream_t st) {
  if (j < 0 || j > 31) return hipErrorInvalidValue;
  {
    ProfScope ps(c.prof, st, KK_CGS_DOTS, 8.0 * n * (j + (w ? 2 : 1)));
    JDispatch<DotsF>::run(j, c, Q, ld, u, w, n, st);
  }
  return reduce_partials_n(c, red_blocks(n / 2), 2 * j + 2, out, st);
}

hipError_t dcgs_update(const Ctx& c, const double* Q, long long ld, const DcgsCoef& cf, double* u, const double* w,
                       double* qj, long long n, hipStream_t st) {
  if (cf.j < 0 || cf.j > 31) return hipErrorInvalidValue;
  ProfScope ps(c.prof, st, KK_CGS_UPDATE_DOTS, 8.0 * n * (cf.j + 4));
  JDispatch<UpdF>::run(cf.j, c, Q, ld, cf, u, w, qj, n, st);
  return hipGetLastError();
}

hipError_t scale_invnorm(const Ctx& c, double* y, const double* x, const double* nrm2, long long n, hipStream_t st) {
  ProfScope ps(c.prof, st, KK_SCALE, 16.0 * n);
  hipLaunchKernelGGL(k_scale_invnorm, dim3(grid_for(n)), dim3(256), 0, st, y, x, nrm2, n);
  return hipGetLastError();
}

hipError_t axpby(const Ctx& c, long long n, double a, const double* x, double b, const double* y, double* out,
                 hipStream_t st) {
  ProfScope ps(c.prof, st, KK_AXPBY, 24.0 * n);
  hipLaunchKernelGGL(k_axpby, dim3(grid_for(n)), dim3(256), 0, st, n, a, x, b, y, out);
  return hipGetLastError();
}

hipError_t lincomb(const Ctx& c, long long n, const Coefs& cf, const double* V, long long ld, double* x,
                   hipStream_t st) {
  ProfScope ps(c.prof, st, KK_LINCOMB, double(n) * (8.0 * cf.n + 16.0));
  hipLaunchKernelGGL((k_lincomb<double>), dim3(grid_for(n)), dim3(256), 0, st, n, cf, V, ld, x);
  return hipGetLastError();
}
hipError_t lincomb(const Ctx& c, long long n, const Coefs& cf, const float* V, long long ld, double* x,
                   hipStream_t st) {
  ProfScope ps(c.prof, st, KK_LINCOMB, double(n) * (4.0 * cf.n + 16.0));
  hipLaunchKernelGGL((k_lincomb<float>), dim3(grid_for(n)), dim3(256), 0, st, n, cf, V, ld, x);
  return hipGetLastError();
}

hipError_t to_f32(const Ctx& c, long long n, const double* a, float* b, hipStream_t st) {
  ProfScope ps(c.prof, st, KK_CONVERT, 12.0 * n);
  hipLaunchKernelGGL((k_convert<double, float>), dim3(grid_for(n)), dim3(256), 0, st, n, a, b);
  return hipGetLastError();
}

hipError_t dot_and_norm(const Ctx& c, const double* x, const double* y, long long n, double* out, hipStream_t st) {
  {
  ProfScope ps(c.prof, st, KK_DOT2, 8.0 * n * (y ? 2 : 1));
  hipLaunchKernelGGL(k_dot2, dim3(kRedBlocks), dim3(kRedThreads), 0, st, x, y, n, c.partial);
  }
  return reduce_partials(c, 2, out, false, st);
}

hipError_t diff_norms(const Ctx& c, const double* a, const double* b, long long n, double* out, hipStream_t st) {
  {
  ProfScope ps(c.prof, st, KK_DOT2, 8.0 * n * (b ? 2 : 1));
  hipLaunchKernelGGL(k_diffnorm, dim3(kRedBlocks), dim3(kRedThreads), 0, st, a, b, n, c.partial);
  }
  return reduce_partials(c, 2, out, false, st);
}

}  // namespace llg
