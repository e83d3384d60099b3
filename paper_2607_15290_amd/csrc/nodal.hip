// Nodal kernels of the time steppers and their diagnostics.
//
//   euler_update   projected Euler update m <- (m + k v)/|m + k v| (Sec. 3.2)
//   nodal_axpy3    frozen midpoint m^n + (k/2) v and the update m^n + k v
//                  (Sec. 3.3, eq. "hatm")
//   picard_update  Picard change norms and the next frozen midpoint
//   midpoint_diag  energies, ||v||^2 and the residual functionals rho(v) and
//                  chi(r) of eq. "C-N" at the exact midpoint (Remark on the
//                  effect of an inexact midpoint solve)
//   adjoint_finish back-propagation through m^n of one midpoint step
#include <cmath>

#include "krylov.h"

namespace llg {

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double wmax(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// op 0: sum, 1: max, 2: min
template <int NV, int OP>
__device__ __forceinline__ void bstore(double (&acc)[NV], double* __restrict__ partial) {
  __shared__ double sm[kRedThreads / 64][NV];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = acc[i];
    if (OP == 0) s = wsum(s);
    else if (OP == 1) s = wmax(s);
    else s = -wmax(-s);
    if (lane == 0) sm[w][i] = s;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = sm[0][threadIdx.x];
    for (int k = 1; k < kRedThreads / 64; ++k) {
      const double o = sm[k][threadIdx.x];
      s = OP == 0 ? s + o : (OP == 1 ? fmax(s, o) : fmin(s, o));
    }
    partial[(long long)threadIdx.x * gridDim.x + blockIdx.x] = s;
  }
}

// Node-pair loop: thread-strided over pairs (i, i + 1), i even (n_x is even,
// so every plane holds whole pairs); every plane access is one 16-byte
// non-temporal load or store.
#define PAIR_LOOP(i, ng)                                                                 \
  for (long long i = 2 * ((long long)blockIdx.x * blockDim.x + threadIdx.x); i < (ng); \
       i += 2 * (long long)gridDim.x * blockDim.x)

struct Pr {
  double v[2];
  __device__ double operator[](int h) const { return v[h]; }
};
__device__ __forceinline__ Pr ldp(const double* __restrict__ p) {
  return Pr{{__builtin_nontemporal_load(p), __builtin_nontemporal_load(p + 1)}};
}
__device__ __forceinline__ void stp(double* __restrict__ p, double a, double b) {
  __builtin_nontemporal_store(a, p);
  __builtin_nontemporal_store(b, p + 1);
}

__global__ __launch_bounds__(kRedThreads) void k_m_check(const double* __restrict__ m, long long ng,
                                                        double* __restrict__ partial) {
  double mn[1] = {INFINITY};
  double bad[1] = {0.0};
  PAIR_LOOP(i, ng) {
    const Pr a = ldp(m + i), b = ldp(m + ng + i), c = ldp(m + 2 * ng + i);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const double n2 = a[h] * a[h] + b[h] * b[h] + c[h] * c[h];
      if (!isfinite(n2)) bad[0] = 1.0;
      mn[0] = fmin(mn[0], n2);
    }
  }
  bstore<1, 2>(mn, partial);
  __syncthreads();
  bstore<1, 1>(bad, partial + gridDim.x);
}

__global__ __launch_bounds__(kRedThreads) void k_euler_update(double* __restrict__ m, const double* __restrict__ v,
                                                             double k, long long ng, double* __restrict__ partial) {
  double mx[1] = {0.0};
  PAIR_LOOP(i, ng) {
    Pr mc[3], vc[3];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      mc[f] = ldp(m + f * ng + i);
      vc[f] = ldp(v + f * ng + i);
    }
    double o[3][2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      double a = mc[0][h] + k * vc[0][h], b = mc[1][h] + k * vc[1][h], c = mc[2][h] + k * vc[2][h];
      const double s = 1.0 / sqrt(a * a + b * b + c * c);
      a *= s;
      b *= s;
      c *= s;
      o[0][h] = a;
      o[1][h] = b;
      o[2][h] = c;
      mx[0] = fmax(mx[0], fabs(sqrt(a * a + b * b + c * c) - 1.0));
    }
#pragma unroll
    for (int f = 0; f < 3; ++f) stp(m + f * ng + i, o[f][0], o[f][1]);
  }
  bstore<1, 1>(mx, partial);
}

// out = m + a v over n values (n even)
__global__ void k_axpy3(const double* __restrict__ m, double a, const double* __restrict__ v,
                        double* __restrict__ out, long long n) {
  PAIR_LOOP(i, n) {
    const Pr x = ldp(m + i), y = ldp(v + i);
    stp(out + i, x[0] + a * y[0], x[1] + a * y[1]);
  }
}

// Picard bookkeeping of the midpoint step, one pass over 3 planes:
// partial sums of ||v - vold||^2, ||v||^2 and ||m0 + a v||^2, then vold <- v
// and mh <- m0 + a v (the next frozen midpoint).
__global__ __launch_bounds__(kRedThreads) void k_picard_update(const double* __restrict__ m0,
                                                              const double* __restrict__ x,
                                                              double* __restrict__ vold, double* __restrict__ mh,
                                                              float* __restrict__ mh32, double* __restrict__ r,
                                                              double a, long long ng, double* __restrict__ partial) {
  double acc[5] = {0, 0, 0, 0, 0};
  PAIR_LOOP(i, ng) {
    Pr xv[3], vo[3], mz[3];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      xv[f] = ldp(x + f * ng + i);
      vo[f] = ldp(vold + f * ng + i);
      mz[f] = ldp(m0 + f * ng + i);
    }
    double mm[2] = {0, 0}, dm[3][2], mi[3][2];
#pragma unroll
    for (int f = 0; f < 3; ++f) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const double vi = xv[f][h], d = vi - vo[f][h];
        mi[f][h] = mz[f][h] + a * vi;
        acc[0] += d * d;
        acc[1] += vi * vi;
        mm[h] += mi[f][h] * mi[f][h];
        dm[f][h] = a * d;
      }
      stp(vold + f * ng + i, xv[f][0], xv[f][1]);
      stp(mh + f * ng + i, mi[f][0], mi[f][1]);
      if (mh32) {
        __builtin_nontemporal_store(float(mi[f][0]), mh32 + f * ng + i);
        __builtin_nontemporal_store(float(mi[f][1]), mh32 + f * ng + i + 1);
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      acc[2] += mm[h];
      acc[3] += mm[h] <= 1e-300 ? 1.0 : 0.0;
    }
    if (r) {
      // r -= (dm x v + dm lam, -dm . v), dm = m_hat^{p+1} - m_hat^p
      const Pr lam = ldp(x + 3 * ng + i);
      Pr rc[4];
#pragma unroll
      for (int f = 0; f < 4; ++f) rc[f] = ldp(r + f * ng + i);
      double ro[4][2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const double v0 = xv[0][h], v1 = xv[1][h], v2 = xv[2][h];
        const double d0 = dm[0][h], d1 = dm[1][h], d2 = dm[2][h];
        const double c0 = d1 * v2 - d2 * v1;
        const double c1 = d2 * v0 - d0 * v2;
        const double c2 = d0 * v1 - d1 * v0;
        ro[0][h] = rc[0][h] - (c0 + d0 * lam[h]);
        ro[1][h] = rc[1][h] - (c1 + d1 * lam[h]);
        ro[2][h] = rc[2][h] - (c2 + d2 * lam[h]);
        ro[3][h] = rc[3][h] + (d0 * v0 + d1 * v1 + d2 * v2);
        acc[4] += ro[0][h] * ro[0][h] + ro[1][h] * ro[1][h] + ro[2][h] * ro[2][h] + ro[3][h] * ro[3][h];
      }
#pragma unroll
      for (int f = 0; f < 4; ++f) stp(r + f * ng + i, ro[f][0], ro[f][1]);
    }
  }
  bstore<5, 0>(acc, partial);
}

__global__ __launch_bounds__(kRedThreads) void k_len_err(const double* __restrict__ m, long long ng,
                                                        double* __restrict__ partial) {
  double mx[1] = {0.0};
  PAIR_LOOP(i, ng) {
    const Pr a = ldp(m + i), b = ldp(m + ng + i), c = ldp(m + 2 * ng + i);
#pragma unroll
    for (int h = 0; h < 2; ++h) mx[0] = fmax(mx[0], fabs(sqrt(a[h] * a[h] + b[h] * b[h] + c[h] * c[h]) - 1.0));
  }
  bstore<1, 1>(mx, partial);
}

// applied field at the node pair (i, i + 1): uniform part plus the optional spatial field
__device__ __forceinline__ void field_pair(const NodalArgs& na, long long ng, long long i, double (&h)[3][2]) {
  const double hu[3] = {na.hu0, na.hu1, na.hu2};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (na.hfield) {
      const Pr f = ldp(na.hfield + c * ng + i);
      h[c][0] = hu[c] + f[0];
      h[c][1] = hu[c] + f[1];
    } else {
      h[c][0] = h[c][1] = hu[c];
    }
  }
}

__global__ __launch_bounds__(kRedThreads) void k_midpoint_diag(NodalArgs na, double alpha, double cexc, double k,
                                                              const double* __restrict__ m0,
                                                              const double* __restrict__ v,
                                                              const double* __restrict__ r,
                                                              const double* __restrict__ lm0,
                                                              const double* __restrict__ lv, long long ng,
                                                              double* __restrict__ partial) {
  double acc[5] = {0, 0, 0, 0, 0};
  PAIR_LOOP(i, ng) {
    double hp[3][2];
    field_pair(na, ng, i, hp);
    Pr am[3], vm[3], l0m[3], lvm[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      am[c] = ldp(m0 + c * ng + i);
      vm[c] = ldp(v + c * ng + i);
      l0m[c] = ldp(lm0 + c * ng + i);
      lvm[c] = ldp(lv + c * ng + i);
    }
    const Pr rp = ldp(r + i);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      double a[3], vv[3], l0[3], l1[3], m1[3], mh[3], lmh[3], h[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        a[c] = am[c][q];
        vv[c] = vm[c][q];
        l0[c] = l0m[c][q];
        h[c] = hp[c][q];
        m1[c] = a[c] + k * vv[c];
        mh[c] = a[c] + 0.5 * k * vv[c];
        l1[c] = l0[c] + k * lvm[c][q];
        lmh[c] = l0[c] + 0.5 * k * lvm[c][q];
      }
      const double rr = rp[q];
      const double cr[3] = {mh[1] * vv[2] - mh[2] * vv[1], mh[2] * vv[0] - mh[0] * vv[2],
                            mh[0] * vv[1] - mh[1] * vv[0]};
      double e0 = 0, e1 = 0, v2 = 0, rho = 0, mv = 0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        e0 += 0.5 * cexc * a[c] * l0[c] - a[c] * h[c];
        e1 += 0.5 * cexc * m1[c] * l1[c] - m1[c] * h[c];
        v2 += vv[c] * vv[c];
        const double rv = alpha * vv[c] + cr[c] + na.chat * lmh[c] + mh[c] * rr - na.hs * h[c];
        rho += rv * vv[c];
        mv += vv[c] * mh[c];
      }
      acc[0] += e0;
      acc[1] += e1;
      acc[2] += v2;
      acc[3] += rho;
      acc[4] += mv * rr;
    }
  }
  bstore<5, 0>(acc, partial);
}

// gbar -= v x mu_v + C_hat L mu_v + r mu_v - v mu_r ; hbar_field += hs mu_v ; sums of hs mu_v
__global__ __launch_bounds__(kRedThreads) void k_adjoint_finish(NodalArgs na, const double* __restrict__ v,
                                                               const double* __restrict__ r,
                                                               const double* __restrict__ mu,
                                                               const double* __restrict__ lmu,
                                                               double* __restrict__ gbar,
                                                               double* __restrict__ hbar, long long ng,
                                                               double* __restrict__ partial) {
  double acc[3] = {0, 0, 0};
  PAIR_LOOP(i, ng) {
    Pr vp[3], mp[3], lp[3], gp[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      vp[c] = ldp(v + c * ng + i);
      mp[c] = ldp(mu + c * ng + i);
      lp[c] = ldp(lmu + c * ng + i);
      gp[c] = ldp(gbar + c * ng + i);
    }
    const Pr mrp = ldp(mu + 3 * ng + i), rp = ldp(r + i);
    double go[3][2], hb[3][2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const double vv[3] = {vp[0][q], vp[1][q], vp[2][q]}, mv[3] = {mp[0][q], mp[1][q], mp[2][q]};
      const double mr = mrp[q], rr = rp[q];
      const double cr[3] = {vv[1] * mv[2] - vv[2] * mv[1], vv[2] * mv[0] - vv[0] * mv[2],
                            vv[0] * mv[1] - vv[1] * mv[0]};
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        go[c][q] = gp[c][q] - (cr[c] + na.chat * lp[c][q] + rr * mv[c] - vv[c] * mr);
        hb[c][q] = na.hs * mv[c];
        acc[c] += hb[c][q];
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      stp(gbar + c * ng + i, go[c][0], go[c][1]);
      if (hbar) {
        const Pr o = ldp(hbar + c * ng + i);
        stp(hbar + c * ng + i, o[0] + hb[c][0], o[1] + hb[c][1]);
      }
    }
  }
  bstore<3, 0>(acc, partial);
}

__global__ __launch_bounds__(kRedThreads) void k_reduce_min_max(const double* __restrict__ partial, int nb,
                                                               double* __restrict__ out) {
  double mn[1] = {INFINITY}, mx[1] = {-INFINITY};
  for (int b = threadIdx.x; b < nb; b += kRedThreads) {
    mn[0] = fmin(mn[0], partial[b]);
    mx[0] = fmax(mx[0], partial[nb + b]);
  }
  __shared__ double sm[2][kRedThreads / 64];
  const double a = -wmax(-mn[0]), b = wmax(mx[0]);
  if ((threadIdx.x & 63) == 0) {
    sm[0][threadIdx.x >> 6] = a;
    sm[1][threadIdx.x >> 6] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double x = sm[0][0], y = sm[1][0];
    for (int w = 1; w < kRedThreads / 64; ++w) {
      x = fmin(x, sm[0][w]);
      y = fmax(y, sm[1][w]);
    }
    out[0] = x;
    out[1] = y;
  }
}

// ---- launchers --------------------------------------------------------------
static inline unsigned grid_n(long long n) {
  long long g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  return (unsigned)(g < 1 ? 1 : g);
}

// Profiler bytes of the nodal kernels: one read of every plane a kernel reads
// and one write of every plane it writes (8 bytes per node and plane).
hipError_t m_check(const Ctx& c, const double* m, double* out, hipStream_t st) {
  hipError_t e_ = hipSuccess;
  {
  ProfScope ps(c.prof, st, KK_NODAL, 24.0 * c.ng);
  const int nb = nodal_blocks(c.ng);
  hipLaunchKernelGGL(k_m_check, dim3(nb), dim3(kRedThreads), 0, st, m, c.ng, c.partial);
  hipLaunchKernelGGL((k_reduce_min_max), dim3(1), dim3(kRedThreads), 0, st, c.partial, nb, out);
  e_ = hipGetLastError();
  }
  return e_;
}

hipError_t euler_update(const Ctx& c, double* m, const double* v, double k, double* out, hipStream_t st) {
  hipError_t e_ = hipSuccess;
  {
  ProfScope ps(c.prof, st, KK_NODAL, 72.0 * c.ng);
  hipLaunchKernelGGL(k_euler_update, dim3(nodal_blocks(c.ng)), dim3(kRedThreads), 0, st, m, v, k, c.ng, c.partial);
  e_ = reduce_partials(c, nodal_blocks(c.ng), 1, out, true, st);
  }
  return e_;
}

hipError_t nodal_axpy3(const Ctx& c, const double* m, double a, const double* v, double* out, hipStream_t st) {
  hipError_t e_ = hipSuccess;
  {
  ProfScope ps(c.prof, st, KK_NODAL, 72.0 * c.ng);
  hipLaunchKernelGGL(k_axpy3, dim3(grid_n(3 * c.ng)), dim3(256), 0, st, m, a, v, out, 3 * c.ng);
  e_ = hipGetLastError();
  }
  return e_;
}

hipError_t len_err(const Ctx& c, const double* m, double* out, hipStream_t st) {
  hipError_t e_ = hipSuccess;
  {
  ProfScope ps(c.prof, st, KK_NODAL, 24.0 * c.ng);
  hipLaunchKernelGGL(k_len_err, dim3(nodal_blocks(c.ng)), dim3(kRedThreads), 0, st, m, c.ng, c.partial);
  e_ = reduce_partials(c, nodal_blocks(c.ng), 1, out, true, st);
  }
  return e_;
}

hipError_t midpoint_diag(const Ctx& c, const NodalArgs& na, double alpha, double cexc, double k, const double* m0,
                         const double* v, const double* r, const double* lm0, const double* lv, double* out,
                         hipStream_t st) {
  hipError_t e_ = hipSuccess;
  {
  ProfScope ps(c.prof, st, KK_NODAL, (104.0 + (na.hfield ? 24.0 : 0.0)) * c.ng);
  hipLaunchKernelGGL(k_midpoint_diag, dim3(nodal_blocks(c.ng)), dim3(kRedThreads), 0, st, na, alpha, cexc, k, m0, v,
                     r, lm0, lv, c.ng, c.partial);
  e_ = reduce_partials(c, nodal_blocks(c.ng), 5, out, false, st);
  }
  return e_;
}

hipError_t picard_update(const Ctx& c, const double* m0, const double* v, double* vold, double* mh, double a,
                         double* out, hipStream_t st, float* mh32, double* r) {
  hipError_t e_ = hipSuccess;
  {
  // m0, v, vold read; vold, mh written; the float32 copy; r (4 planes) and lam read-modify-write
  ProfScope ps(c.prof, st, KK_NODAL, (120.0 + (mh32 ? 12.0 : 0.0) + (r ? 72.0 : 0.0)) * c.ng);
  hipLaunchKernelGGL(k_picard_update, dim3(nodal_blocks(c.ng)), dim3(kRedThreads), 0, st, m0, v, vold, mh, mh32, r, a,
                     c.ng, c.partial);
  e_ = reduce_partials(c, nodal_blocks(c.ng), 5, out, false, st);
  }
  return e_;
}

hipError_t adjoint_finish(const Ctx& c, const NodalArgs& na, const double* v, const double* r, const double* mu,
                          const double* lmu, double* gbar, double* hbar_field, double* out_hsum, hipStream_t st) {
  hipError_t e_ = hipSuccess;
  {
  // v, r, mu (4 planes), L mu read; gbar (and hbar) read and written
  ProfScope ps(c.prof, st, KK_NODAL, (136.0 + (hbar_field ? 48.0 : 0.0)) * c.ng);
  hipLaunchKernelGGL(k_adjoint_finish, dim3(nodal_blocks(c.ng)), dim3(kRedThreads), 0, st, na, v, r, mu, lmu, gbar,
                     hbar_field, c.ng, c.partial);
  e_ = reduce_partials(c, nodal_blocks(c.ng), 3, out_hsum, false, st);
  }
  return e_;
}

}  // namespace llg
