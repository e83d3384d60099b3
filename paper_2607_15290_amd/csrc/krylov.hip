// Streaming vector kernels of the Krylov solvers and the steppers.
//
// All reductions are two-stage and deterministic: a grid whose size depends
// only on the vector length accumulates per-thread partial sums in a fixed
// order, reduces them across the block by wavefront shuffles, and writes one
// partial per block; a second kernel sums the partials of each value in a
// fixed tree.  The grid never depends on timing, so every reduced value is
// bitwise reproducible from run to run.
//
// Arnoldi orthogonalization is classical Gram-Schmidt with one
// re-orthogonalization (CGS2), as three streaming passes over the basis:
//   A: h = V^T w;   B: w -= V h, s = V^T w;   C: w -= V s, ||w||^2.
#include <cmath>
#include <cstdint>
#include <type_traits>
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
// The operator output w of an Arnoldi step, as a pair of float64 values: a
// float64 vector, or the float32 output of the precision form's operators
// (whose float32 values convert to float64 exactly).
__device__ __forceinline__ double2 ldw(const double2* p) { return ldnt(p); }
__device__ __forceinline__ double2 ldw(const float2* p) {
  return double2{double(__builtin_nontemporal_load(&p->x)), double(__builtin_nontemporal_load(&p->y))};
}

// Reduce acc[0..nv) over the block and store partial[i * gridDim.x + blockIdx.x]
// (value-major: the partials of one value are contiguous).
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
    partial[(long long)threadIdx.x * gridDim.x + blockIdx.x] = s;
  }
}

// out[i] = sum (or max) over blocks of partial[i * nb + b]; one block per value.
template <bool MAX>
__global__ __launch_bounds__(kRedThreads) void k_reduce(const double* __restrict__ partial, int nb,
                                                       double* __restrict__ out) {
  const int i = blockIdx.x;
  double s = MAX ? -INFINITY : 0.0;
  for (int b = threadIdx.x; b < nb; b += kRedThreads) {
    const double v = partial[(long long)i * nb + b];
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

// out[i] = sum_b partial[i * nb + b]: value-major partials, one block of 1024
// threads per value, four independent accumulators per thread (fixed order).
__global__ __launch_bounds__(1024) void k_reduce_vmajor(const double* __restrict__ partial, int nb,
                                                       double* __restrict__ out, double* __restrict__ hout) {
  const double* p = partial + (long long)blockIdx.x * nb;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int b = threadIdx.x;
  for (; b + 3 * 1024 < nb; b += 4 * 1024) {
    s0 += p[b];
    s1 += p[b + 1024];
    s2 += p[b + 2048];
    s3 += p[b + 3072];
  }
  for (; b < nb; b += 1024) s0 += p[b];
  double s = (s0 + s1) + (s2 + s3);
  __shared__ double sm[1024 / 64];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = sm[0];
    for (int w = 1; w < 1024 / 64; ++w) t += sm[w];
    out[blockIdx.x] = t;
    if (hout) hout[blockIdx.x] = t;
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
// The basis is kept as the raw Arnoldi directions U = [u_0 .. u_J] (column 0
// at u0, column i >= 1 at U1 + (i - 1) ld); the orthonormal basis is implicit,
// Q = U T^{-1}, with T upper triangular (column j = [Q_j^T u_j; beta_j]).
// Storing U instead of Q saves one vector store per iteration: q_j is never
// written.  Both passes are instantiated for the exact column count J + 1,
// so every basis load of a thread is unconditional and the loads of one
// element are all in flight together; loads and stores are non-temporal.
// Blocks of kDcgsThreads threads, one double2 per thread on a full-size grid
// (measured 2-7% faster than two per thread, and faster than batching several
// elements' loads per thread, whose extra streams in flight lower the DRAM
// efficiency).
constexpr int kDcgsThreads = 512;
// The update pass of vectors of at most this many 16-byte pairs runs as one block.
constexpr long long kDcgsSingleMaxN2 = 4 * kDcgsThreads;
// Unused dynamic LDS of the update pass caps the blocks per CU.  With a
// float64 operator output w it caps the pass at two 512-thread blocks per CU
// (16 waves): fewer concurrent vector streams keep the DRAM pages of the
// j + 3 streams open longer, measured 3% faster than the uncapped pass at
// 256^3 (one block per CU is 40% slower; the read-only pass 1 gains nothing
// from a cap).  With the float32 w of the precision form three blocks per CU
// are fastest (421 us against 433 us with two and 427 us uncapped, 256^3).
#ifndef LLG_DCGS_UPDATE_LDS
#define LLG_DCGS_UPDATE_LDS 65536
#endif
#ifndef LLG_DCGS_UPDATE_LDS_F32W
#define LLG_DCGS_UPDATE_LDS_F32W 40960
#endif

// With mirror (single-block launches only) the block's sums are the final
// values and are also written to the host-mapped mirror.
template <int NV>
__device__ __forceinline__ void dcgs_block_store(const double (&acc)[NV], double* __restrict__ partial,
                                                 double* __restrict__ mirror = nullptr) {
  __shared__ double sm[kDcgsThreads / 64][NV];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const double y = wave_sum(acc[i]);
    if (lane == 0) sm[wv][i] = y;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double t = sm[0][threadIdx.x];
#pragma unroll
    for (int k = 1; k < kDcgsThreads / 64; ++k) t += sm[k][threadIdx.x];
    partial[(long long)threadIdx.x * gridDim.x + blockIdx.x] = t;
    if (mirror) mirror[threadIdx.x] = t;
  }
}

// Pass 1: out = [U_i.w (i <= J)], value-major partials.  W2: double2 or
// float2 (w stored in float32).
template <int J, typename W2>
__global__ __launch_bounds__(kDcgsThreads) void k_dcgs_dots(const double2* __restrict__ u0,
                                                          const double2* __restrict__ U1, long long ld2,
                                                          const W2* __restrict__ w, long long n2,
                                                          double* __restrict__ partial) {
  double acc[J + 1];
#pragma unroll
  for (int i = 0; i <= J; ++i) acc[i] = 0.0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n2; e += stride) {
    const double2 ww = ldw(w + e);
    double2 q[J + 1];
    q[0] = ldnt(u0 + e);
#pragma unroll
    for (int i = 1; i <= J; ++i) q[i] = ldnt(U1 + (i - 1) * ld2 + e);
#pragma unroll
    for (int i = 0; i <= J; ++i) acc[i] = fma(q[i].x, ww.x, fma(q[i].y, ww.y, acc[i]));
  }
  dcgs_block_store<J + 1>(acc, partial);
}

// Projection coefficients of pass 2.  With p = U_{j+1}^T w (pass 1, on the
// device) and Minv = T^{-1} (columns 0..j-1 in minv from the earlier steps,
// column j in cf):
//   b = Q_j^T w = Minv_j^T p_{<j},   e_j = q_j.w = (p_j - a.b) / beta_j,
//   Q_{j+1} [b; e_j] = U_{j+1} gamma,   gamma = Minv_{j+1} [b; e_j].
// The coefficient step inside a block: columns 0..j of Minv (column j from
// cf) and p are staged in LDS with coalesced loads by the whole block, then
// the first wavefront runs the two short triangular products from LDS (from
// global memory each term of those loops would wait out a cache latency).
// gs (LDS) receives gamma; with store, the block keeps column j of Minv for
// the later steps.  Every thread of the block calls it.
__device__ __forceinline__ void dcgs_coef_block(const DcgsCoef& cf, const double* __restrict__ p,
                                                double* __restrict__ minv, bool store, double* gs) {
  __shared__ double ms[kDcgsMaxCols * kDcgsMaxCols];  // column-major, columns 0..j
  __shared__ double ps[kDcgsMaxCols];
  __shared__ double v[64];
  const int l = threadIdx.x, j = cf.j;
  for (int t = l; t < (j + 1) * kDcgsMaxCols; t += blockDim.x)
    ms[t] = t < j * kDcgsMaxCols ? minv[t] : cf.minv[t - j * kDcgsMaxCols];
  if (l <= j) ps[l] = p[l];
  __syncthreads();
  if (l < 64) {
    double b = 0.0;
    if (l < j)
      for (int k = 0; k <= l; ++k) b = fma(ms[l * kDcgsMaxCols + k], ps[k], b);
    const double ab = wave_sum(l < j ? cf.a[l] * b : 0.0);
    const double e = (ps[j] - ab) * cf.inv_beta;
    v[l] = l < j ? b : (l == j ? e : 0.0);
  }
  __syncthreads();
  if (l <= j) {
    double g = 0.0;
    for (int k = l; k <= j; ++k) g = fma(ms[k * kDcgsMaxCols + l], v[k], g);
    gs[l] = g;
    if (store) minv[j * kDcgsMaxCols + l] = cf.minv[l];
  }
  __syncthreads();
}

// Pass 2's coefficients as a kernel of their own (one block of one wavefront).
__global__ __launch_bounds__(64) void k_dcgs_coef(DcgsCoef cf, const double* __restrict__ p,
                                                  double* __restrict__ minv, double* __restrict__ gamma) {
  __shared__ double gs[kDcgsMaxCols];
  dcgs_coef_block(cf, p, minv, true, gs);
  if (threadIdx.x <= cf.j) gamma[threadIdx.x] = gs[threadIdx.x];
}

// Pass 2: unew = (w - U gamma) / beta_j, and, for the next step,
// out = [U_i.unew (i <= J), unew.unew], value-major partials.  With COEF the
// pass forms gamma itself (dcgs_coef_block, from cf and the pass-1 products
// p) instead of reading the coefficient kernel's output: on small grids that
// saves a launch per step, where launches, not bytes, set the time.
template <int J, typename W2, bool COEF>
__global__ __launch_bounds__(kDcgsThreads) void k_dcgs_update(const double2* __restrict__ u0,
                                                            const double2* __restrict__ U1, long long ld2,
                                                            const double* __restrict__ gamma, double inv_beta,
                                                            const W2* __restrict__ w,
                                                            double2* __restrict__ unew, long long n2,
                                                            double* __restrict__ partial, DcgsCoef cf,
                                                            const double* __restrict__ p, double* __restrict__ minv,
                                                            DeferredDots dp, double* __restrict__ mirror) {
  double gm[J + 1];
  if constexpr (COEF) {
    __shared__ double gs[kDcgsMaxCols];
    __shared__ double pr[kDcgsMaxCols];
    const double* pp = p;
    if (dp.nb > 0) {
      // reduce the deferred pass-1 partials: value q by wavefront q mod 8
      const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
      for (int q = wv; q <= cf.j; q += kDcgsThreads / 64) {
        double t = 0.0;
        for (int b = lane; b < dp.nb; b += 64) t += dp.part[(long long)q * dp.nb + b];
        t = wave_sum(t);
        if (lane == 0) pr[q] = t;
      }
      __syncthreads();
      if (blockIdx.x == 0 && threadIdx.x <= cf.j) {
        dp.out[threadIdx.x] = pr[threadIdx.x];
        dp.mirror[threadIdx.x] = pr[threadIdx.x];
      }
      pp = pr;
    }
    dcgs_coef_block(cf, pp, minv, blockIdx.x == 0, gs);
#pragma unroll
    for (int i = 0; i <= J; ++i) gm[i] = gs[i];
  } else {
#pragma unroll
    for (int i = 0; i <= J; ++i) gm[i] = gamma[i];
  }
  double acc[J + 2];
#pragma unroll
  for (int i = 0; i < J + 2; ++i) acc[i] = 0.0;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n2; e += stride) {
    double2 se = ldw(w + e);
    double2 q[J + 1];
    q[0] = ldnt(u0 + e);
#pragma unroll
    for (int i = 1; i <= J; ++i) q[i] = ldnt(U1 + (i - 1) * ld2 + e);
#pragma unroll
    for (int i = 0; i <= J; ++i) {
      se.x = fma(-gm[i], q[i].x, se.x);
      se.y = fma(-gm[i], q[i].y, se.y);
    }
    const double2 un{se.x * inv_beta, se.y * inv_beta};
    stnt(unew + e, un);
#pragma unroll
    for (int i = 0; i <= J; ++i) acc[i] = fma(q[i].x, un.x, fma(q[i].y, un.y, acc[i]));
    acc[J + 1] = fma(un.x, un.x, fma(un.y, un.y, acc[J + 1]));
  }
  dcgs_block_store<J + 2>(acc, partial, mirror);
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

// x += sum_i c_i V_i, instantiated for the exact count K so the K basis loads
// of an element group are issued together.  With VEC each thread takes four
// consecutive elements (one 16-byte load per float32 vector, two per float64
// vector; the host checks the 16-byte alignment), otherwise one element.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <typename TV>
__device__ __forceinline__ void ld4(const TV* p, TV (&v)[4]) {
  if constexpr (sizeof(TV) == 4) {
    const f32x4 a = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p));
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
  } else {
    const f64x2 a = __builtin_nontemporal_load(reinterpret_cast<const f64x2*>(p));
    const f64x2 b = __builtin_nontemporal_load(reinterpret_cast<const f64x2*>(p) + 1);
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
  }
}
template <typename TV, int K, bool VEC>
__global__ void k_lincomb(long long n, Coefs cf, const TV* __restrict__ V, long long ld, double* __restrict__ x) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  const long long t0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long done = 0;
  if constexpr (VEC) {
    const long long n4 = n / 4;
    for (long long g = t0; g < n4; g += stride) {
      const long long e = 4 * g;
      TV vv[K > 0 ? K : 1][4];
#pragma unroll
      for (int i = 0; i < K; ++i) ld4(V + i * ld + e, vv[i]);
      double2* xp = reinterpret_cast<double2*>(x + e);
      double2 s0 = xp[0], s1 = xp[1];
#pragma unroll
      for (int i = 0; i < K; ++i) {
        s0.x = fma(cf.c[i], double(vv[i][0]), s0.x);
        s0.y = fma(cf.c[i], double(vv[i][1]), s0.y);
        s1.x = fma(cf.c[i], double(vv[i][2]), s1.x);
        s1.y = fma(cf.c[i], double(vv[i][3]), s1.y);
      }
      xp[0] = s0;
      xp[1] = s1;
    }
    done = 4 * n4;
  }
  for (long long e = done + t0; e < n; e += stride) {
    TV vv[K > 0 ? K : 1];
#pragma unroll
    for (int i = 0; i < K; ++i) vv[i] = __builtin_nontemporal_load(V + i * ld + e);
    double s = x[e];
#pragma unroll
    for (int i = 0; i < K; ++i) s = fma(cf.c[i], double(vv[i]), s);
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

// ---- host launchers --------------------------------------------------------
static inline unsigned grid_for(long long n) {
  long long g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  return (unsigned)(g < 1 ? 1 : g);
}

hipError_t reduce_partials_n(const Ctx& c, int nb, int nv, double* out, hipStream_t st) {
  ProfScope ps(c.prof, st, KK_REDUCE, 8.0 * nb * nv);
  // results landing in the Arnoldi slots are mirrored into host memory, so
  // the host reads them after a stream synchronize without a copy
  double* hout = (out >= c.dots && out < c.dots + kDotsSlots * kMaxDots) ? c.hmirror_dev + (out - c.dots) : nullptr;
  hipLaunchKernelGGL(k_reduce_vmajor, dim3(nv), dim3(1024), 0, st, c.partial, nb, out, hout);
  return hipGetLastError();
}

hipError_t reduce_flat(const Ctx& c, int nb, double* out, hipStream_t st) {
  ProfScope ps(c.prof, st, KK_REDUCE, 8.0 * nb);
  hipLaunchKernelGGL(k_reduce_flat, dim3(1), dim3(kRedThreads), 0, st, c.partial, nb, out);
  return hipGetLastError();
}

hipError_t reduce_partials(const Ctx& c, int nb, int nv, double* out, bool is_max, hipStream_t st) {
  ProfScope ps(c.prof, st, KK_REDUCE, 8.0 * nb * nv);
  if (is_max)
    hipLaunchKernelGGL((k_reduce<true>), dim3(nv), dim3(kRedThreads), 0, st, c.partial, nb, out);
  else
    hipLaunchKernelGGL((k_reduce<false>), dim3(nv), dim3(kRedThreads), 0, st, c.partial, nb, out);
  return hipGetLastError();
}

template <int MAXV>
static void mdot_t(const Ctx& c, const double* V, long long ld, int nv, const double* w, long long n, hipStream_t st) {
  hipLaunchKernelGGL((k_mdot<MAXV>), dim3(nodal_blocks(n)), dim3(kRedThreads), 0, st, V, ld, nv, w, n, c.partial);
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
  return reduce_partials(c, nodal_blocks(n), nv, out, false, st);
}

template <int MAXV>
static void upd_t(const Ctx& c, const double* V, long long ld, int nv, const double* cf, double* w, long long n,
                  hipStream_t st) {
  hipLaunchKernelGGL((k_update_mdot<MAXV>), dim3(nodal_blocks(n)), dim3(kRedThreads), 0, st, V, ld, nv, cf, w, n,
                     c.partial);
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
  return reduce_partials(c, nodal_blocks(n), nv, out, false, st);
}

template <int MAXV>
static void updn_t(const Ctx& c, const double* V, long long ld, int nv, const double* cf, const double* w,
                   double* o, long long n, hipStream_t st) {
  hipLaunchKernelGGL((k_update_norm<MAXV>), dim3(nodal_blocks(n)), dim3(kRedThreads), 0, st, V, ld, nv, cf, w, o, n,
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
  return reduce_partials(c, nodal_blocks(n), 1, out_nrm2, false, st);
}


// float2 / double2 view of a float32 / float64 operator output
template <typename TW>
using pair_of = typename std::conditional<std::is_same<TW, float>::value, float2, double2>::type;

template <int J, typename TW>
static void dd_t(const Ctx& c, const double* u0, const double* U1, long long ld, const TW* w, long long n,
                 hipStream_t st) {
  hipLaunchKernelGGL((k_dcgs_dots<J, pair_of<TW>>), dim3(red_blocks(n / 2)), dim3(kDcgsThreads), 0, st,
                     reinterpret_cast<const double2*>(u0), reinterpret_cast<const double2*>(U1), ld / 2,
                     reinterpret_cast<const pair_of<TW>*>(w), n / 2, c.partial);
}

template <int J, typename TW>
static void du_t(const Ctx& c, const double* u0, const double* U1, long long ld, const double* gamma,
                 const DcgsCoef& cf, const double* p, const DeferredDots& dp, const TW* w, double* unew, long long n,
                 double* part, double* mirror, hipStream_t st) {
  constexpr unsigned lds = std::is_same<TW, float>::value ? LLG_DCGS_UPDATE_LDS_F32W : LLG_DCGS_UPDATE_LDS;
  const dim3 grid(mirror ? 1 : red_blocks(n / 2)), block(kDcgsThreads);
  const double2* a0 = reinterpret_cast<const double2*>(u0);
  const double2* a1 = reinterpret_cast<const double2*>(U1);
  const pair_of<TW>* wp = reinterpret_cast<const pair_of<TW>*>(w);
  double2* un = reinterpret_cast<double2*>(unew);
  if (gamma)
    hipLaunchKernelGGL((k_dcgs_update<J, pair_of<TW>, false>), grid, block, lds, st, a0, a1, ld / 2, gamma,
                       cf.inv_beta, wp, un, n / 2, part, cf, p, c.tri, dp, mirror);
  else
    hipLaunchKernelGGL((k_dcgs_update<J, pair_of<TW>, true>), grid, block, lds, st, a0, a1, ld / 2, nullptr,
                       cf.inv_beta, wp, un, n / 2, part, cf, p, c.tri, dp, mirror);
}

// Runtime J -> template instantiation J = 0..kDcgsMaxCols - 1.
template <template <int> class F, int J = 0>
struct JDispatch {
  template <typename... A>
  static void run(int j, A&&... args) {
    if (j == J) F<J>::go(std::forward<A>(args)...);
    else if constexpr (J < kDcgsMaxCols - 1) JDispatch<F, J + 1>::run(j, std::forward<A>(args)...);
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

template <typename TW>
static hipError_t dcgs_dots_t(const Ctx& c, const double* u0, const double* U1, long long ld, int j, const TW* w,
                              long long n, double* out, hipStream_t st) {
  if (j < 0 || j >= kDcgsMaxCols) return hipErrorInvalidValue;
  {
    ProfScope ps(c.prof, st, KK_CGS_DOTS, double(n) * (8.0 * (j + 1) + sizeof(TW)));
    JDispatch<DotsF>::run(j, c, u0, U1, ld, w, n, st);
  }
  return reduce_partials_n(c, red_blocks(n / 2), j + 1, out, st);
}
hipError_t dcgs_dots(const Ctx& c, const double* u0, const double* U1, long long ld, int j, const double* w,
                     long long n, double* out, hipStream_t st) {
  return dcgs_dots_t(c, u0, U1, ld, j, w, n, out, st);
}
hipError_t dcgs_dots(const Ctx& c, const double* u0, const double* U1, long long ld, int j, const float* w,
                     long long n, double* out, hipStream_t st) {
  return dcgs_dots_t(c, u0, U1, ld, j, w, n, out, st);
}

hipError_t dcgs_coef(const Ctx& c, const DcgsCoef& cf, const double* p, const double** gamma, hipStream_t st) {
  if (cf.j < 0 || cf.j >= kDcgsMaxCols) return hipErrorInvalidValue;
  double* g = c.tri + kDcgsMaxCols * kDcgsMaxCols;
  {
    ProfScope ps(c.prof, st, KK_REDUCE, 8.0 * (cf.j + 1) * (cf.j + 3));
    hipLaunchKernelGGL(k_dcgs_coef, dim3(1), dim3(64), 0, st, cf, p, c.tri, g);
  }
  *gamma = g;
  return hipGetLastError();
}

template <typename TW>
static hipError_t dcgs_update_t(const Ctx& c, const double* u0, const double* U1, long long ld, const DcgsCoef& cf,
                                const double* p, const TW* w, double* unew, long long n, double* out,
                                hipStream_t st, const DeferredDots* dpp) {
  if (cf.j < 0 || cf.j >= kDcgsMaxCols) return hipErrorInvalidValue;
  const DeferredDots dp = dpp ? *dpp : DeferredDots{};
  if (dp.nb > 0 && (!dp.part || !dp.out || !dp.mirror)) return hipErrorInvalidValue;
  // small grids (and deferred pass-1 products): the update pass forms gamma
  // itself (one launch fewer)
  const double* gamma = nullptr;
  if (c.ng > kSpeculateMaxNodes && dp.nb == 0) {
    hipError_t e = dcgs_coef(c, cf, p, &gamma, st);
    if (e != hipSuccess) return e;
  }
  // Vectors of at most kDcgsSingleMaxN2 pairs: one block (grid-strided)
  // whose sums are the final products, written to out and, for a mirrored
  // slot, to its host mirror: no reduction launch.
  const bool single = n / 2 <= kDcgsSingleMaxN2 && out >= c.dots && out < c.dots + kDotsSlots * kMaxDots;
  {
    // j + 1 directions read, w read, u_new written
    ProfScope ps(c.prof, st, KK_CGS_UPDATE_DOTS, double(n) * (8.0 * (cf.j + 2) + sizeof(TW)));
    JDispatch<UpdF>::run(cf.j, c, u0, U1, ld, gamma, cf, p, dp, w, unew, n, single ? out : c.partial,
                         single ? c.hmirror_dev + (out - c.dots) : nullptr, st);
  }
  if (single) return hipGetLastError();
  return reduce_partials_n(c, red_blocks(n / 2), cf.j + 2, out, st);
}
hipError_t dcgs_update(const Ctx& c, const double* u0, const double* U1, long long ld, const DcgsCoef& cf,
                       const double* p, const double* w, double* unew, long long n, double* out, hipStream_t st,
                       const DeferredDots* dp) {
  return dcgs_update_t(c, u0, U1, ld, cf, p, w, unew, n, out, st, dp);
}
hipError_t dcgs_update(const Ctx& c, const double* u0, const double* U1, long long ld, const DcgsCoef& cf,
                       const double* p, const float* w, double* unew, long long n, double* out, hipStream_t st,
                       const DeferredDots* dp) {
  return dcgs_update_t(c, u0, U1, ld, cf, p, w, unew, n, out, st, dp);
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

template <typename TV, int K>
struct LincombF {
  static void go(const Ctx& c, long long n, const Coefs& cf, const TV* V, long long ld, double* x, hipStream_t st) {
    (void)c;
    const bool vec = (reinterpret_cast<uintptr_t>(V) % 16 == 0) && (reinterpret_cast<uintptr_t>(x) % 16 == 0) &&
                     (ld % 4 == 0);
    long long g = ((vec ? n / 4 : n) + 255) / 256;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    if (vec)
      hipLaunchKernelGGL((k_lincomb<TV, K, true>), dim3((unsigned)g), dim3(256), 0, st, n, cf, V, ld, x);
    else
      hipLaunchKernelGGL((k_lincomb<TV, K, false>), dim3((unsigned)g), dim3(256), 0, st, n, cf, V, ld, x);
  }
};
template <typename TV, int K = 1>
static void lincomb_dispatch(int k, const Ctx& c, long long n, const Coefs& cf, const TV* V, long long ld, double* x,
                             hipStream_t st) {
  if (k == K) LincombF<TV, K>::go(c, n, cf, V, ld, x, st);
  else if constexpr (K < 32) lincomb_dispatch<TV, K + 1>(k, c, n, cf, V, ld, x, st);
}

hipError_t lincomb(const Ctx& c, long long n, const Coefs& cf, const double* V, long long ld, double* x,
                   hipStream_t st) {
  if (cf.n < 1) return hipSuccess;
  if (cf.n > 64) return hipErrorInvalidValue;
  ProfScope ps(c.prof, st, KK_LINCOMB, double(n) * (8.0 * cf.n + 16.0 * ((cf.n + 31) / 32)));
  for (int i0 = 0; i0 < cf.n; i0 += 32) {  // chunks of at most 32 vectors
    Coefs part{};
    part.n = cf.n - i0 < 32 ? cf.n - i0 : 32;
    for (int i = 0; i < part.n; ++i) part.c[i] = cf.c[i0 + i];
    lincomb_dispatch<double>(part.n, c, n, part, V + (long long)i0 * ld, ld, x, st);
  }
  return hipGetLastError();
}
hipError_t lincomb(const Ctx& c, long long n, const Coefs& cf, const float* V, long long ld, double* x,
                   hipStream_t st) {
  if (cf.n < 1) return hipSuccess;
  if (cf.n > 64) return hipErrorInvalidValue;
  ProfScope ps(c.prof, st, KK_LINCOMB, double(n) * (4.0 * cf.n + 16.0 * ((cf.n + 31) / 32)));
  for (int i0 = 0; i0 < cf.n; i0 += 32) {  // chunks of at most 32 vectors
    Coefs part{};
    part.n = cf.n - i0 < 32 ? cf.n - i0 : 32;
    for (int i = 0; i < part.n; ++i) part.c[i] = cf.c[i0 + i];
    lincomb_dispatch<float>(part.n, c, n, part, V + (long long)i0 * ld, ld, x, st);
  }
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
  hipLaunchKernelGGL(k_dot2, dim3(nodal_blocks(n)), dim3(kRedThreads), 0, st, x, y, n, c.partial);
  }
  return reduce_partials(c, nodal_blocks(n), 2, out, false, st);
}

}  // namespace llg
