// Kernels of the spectral pipeline (see pipeline.h for the operators).
//
//   k_xfwd : per (y, z) row, compute the three fields to filter (prologue),
//            real-to-complex DFT along x of each (half-length complex DFT of
//            the even/odd packing plus the split step), write the row of three
//            half spectra.
//   k_axis : DFTs along y or z of W spectral columns at a time; the last
//            axis pass of the pipeline runs forward DFT -> Fourier multiplier
//            -> inverse DFT on the data while it is in registers.
//   k_xinv : per row, complex-to-real inverse DFT along x of the three fields,
//            then the nodal epilogue and the output write.
//
// In two dimensions a pipeline is k_xfwd, k_axis(y, fused), k_xinv; in three
// it is k_xfwd, k_axis(y, fwd), k_axis(z, fused), k_axis(y, inv), k_xinv.
#pragma once
#include "pipeline.h"

namespace llg {

// Launch shape of the x passes for element type T and half-length NH.  The
// float64 passes at NH = 128, 256 use the finer plan (8 points per thread):
// half the lines per block, half the LDS, twice the blocks per CU.
template <typename T, int NH>
struct XCfg {
  static constexpr int KEY = x_plan_key(int(sizeof(T)), NH);
  static constexpr int P = plan_p(KEY);
  static constexpr int TPL = NH / P;
  static constexpr int LX = 64 / TPL;           // rows per block
  static constexpr int NT = 192;                // 3 fields x LX rows x TPL
  static constexpr int SL = NH + (NH >> 4) + 1; // LDS line stride (complex)
};

__device__ __forceinline__ int xphys(int pos) { return pos + (pos >> 4); }

// Grid planes (inputs, magnetization, outputs) are streamed with non-temporal
// hints: each is touched once per pipeline and is far larger than the caches.
// The spectral buffer is accessed with ordinary (cacheable) loads and stores:
// it is reused by the next pass, and in float32 (about 200 MB at 256^3) much
// of it stays in the 256 MB Infinity Cache between passes.
#ifndef LLG_PIPE_NT
#define LLG_PIPE_NT 1
#endif
// Node pairs per thread whose plane loads are issued together in the x passes
// (float32: 6, about 4% faster x-forward at 256^3 than 3; float64: 3, the
// larger batch costs occupancy).
#ifndef LLG_XBATCH_F32
#define LLG_XBATCH_F32 6
#endif
#ifndef LLG_XBATCH_F64
#define LLG_XBATCH_F64 3
#endif
// the same for the precision form's junction pass k_xmid (256^3: 191 us with
// 6, 200 with 3, 204 with 4)
#ifndef LLG_XMID_BATCH
#define LLG_XMID_BATCH LLG_XBATCH_F32
#endif
template <typename U>
__device__ __forceinline__ U ld_s(const U* p) {
#if LLG_PIPE_NT
  return __builtin_nontemporal_load(p);
#else
  return *p;
#endif
}
template <typename U>
__device__ __forceinline__ void st_s(U* p, U v) {
#if LLG_PIPE_NT
  __builtin_nontemporal_store(v, p);
#else
  *p = v;
#endif
}

template <typename U>
__device__ __forceinline__ void load2(const U* __restrict__ p, U& a, U& b) {
  a = ld_s(p);
  b = ld_s(p + 1);
}

template <typename U>
__device__ __forceinline__ void store2(U* __restrict__ p, U a, U b) {
  st_s(p, a);
  st_s(p + 1, b);
}

// Pair access at a wave-uniform plane base plus a 32-bit per-lane byte
// offset: the load takes the scalar-base address form, so a pass touching
// many planes keeps one offset register instead of a 64-bit address per plane.
template <typename U>
__device__ __forceinline__ void load2_at(const U* __restrict__ base, unsigned boff, U& a, U& b) {
  load2(reinterpret_cast<const U*>(reinterpret_cast<const char*>(base) + boff), a, b);
}
template <typename U>
__device__ __forceinline__ void store2_at(U* __restrict__ base, unsigned boff, U a, U b) {
  store2(reinterpret_cast<U*>(reinterpret_cast<char*>(base) + boff), a, b);
}

// ---------------------------------------------------------------------------
// Nodal algebra (Sec. 3.1, eqs. (S) and (Lambda); Sec. 3.2, eq. "inverse S")
// ---------------------------------------------------------------------------
template <typename T>
struct V3 {
  T x, y, z;
};
template <typename T>
__device__ __forceinline__ V3<T> cross3(V3<T> a, V3<T> b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <typename T>
__device__ __forceinline__ T dot3(V3<T> a, V3<T> b) {
  return a.x * b.x + a.y * b.y + a.z * b.z;
}

// (S~ + lambda I)^{-1} (w, wr) = (lambda w - m x w - wr m, m.w + lambda wr) / (lambda^2 + |m|^2)
template <typename T>
__device__ __forceinline__ void shift_solve(V3<T> m, V3<T> w, T wr, T lam, V3<T>& zv, T& zr) {
  const T inv_d = T(1) / (lam * lam + dot3(m, m));
  const V3<T> c = cross3(m, w);
  zv.x = (lam * w.x - c.x - wr * m.x) * inv_d;
  zv.y = (lam * w.y - c.y - wr * m.y) * inv_d;
  zv.z = (lam * w.z - c.z - wr * m.z) * inv_d;
  zr = (dot3(m, w) + lam * wr) * inv_d;
}
// (S~ + lambda I)^{-T} (w, wr) = (lambda w + m x w + wr m, -m.w + lambda wr) / (lambda^2 + |m|^2)
template <typename T>
__device__ __forceinline__ void shift_solve_t(V3<T> m, V3<T> w, T wr, T lam, V3<T>& zv, T& zr) {
  const T inv_d = T(1) / (lam * lam + dot3(m, m));
  const V3<T> c = cross3(m, w);
  zv.x = (lam * w.x + c.x + wr * m.x) * inv_d;
  zv.y = (lam * w.y + c.y + wr * m.y) * inv_d;
  zv.z = (lam * w.z + c.z + wr * m.z) * inv_d;
  zr = (lam * wr - dot3(m, w)) * inv_d;
}

// ---------------------------------------------------------------------------
// Prologue: values of the three filtered fields at nodes i and i+1, split into
// a load phase (raw plane values) and a compute phase so that the loads of
// several node pairs can be issued together.
// ---------------------------------------------------------------------------
template <typename T, typename TIn, int PRO>
struct ProRaw {
  static constexpr int NV = PRO == PRO_COPY3 ? 3 : 4;
  static constexpr int NM = PRO == PRO_COPY3 ? 0 : 3;
  TIn v[NV][2];
  T m[NM > 0 ? NM : 1][2];
};

template <typename T, typename TIn, int PRO>
__device__ __forceinline__ void prologue_load(const TIn* __restrict__ in, const T* __restrict__ m, long long ng,
                                              long long i, ProRaw<T, TIn, PRO>& r) {
  using R = ProRaw<T, TIn, PRO>;
#pragma unroll
  for (int f = 0; f < R::NV; ++f) load2(in + f * ng + i, r.v[f][0], r.v[f][1]);
#pragma unroll
  for (int f = 0; f < R::NM; ++f) load2(m + f * ng + i, r.m[f][0], r.m[f][1]);
}

template <typename T, typename TIn, int PRO>
__device__ __forceinline__ void prologue_compute(const ProRaw<T, TIn, PRO>& r, const NodalArgs& na,
                                                 cx<T> (&u)[3]) {
  if constexpr (PRO == PRO_COPY3) {
#pragma unroll
    for (int f = 0; f < 3; ++f) u[f] = {T(r.v[f][0]), T(r.v[f][1])};
  } else {
    const T lam = T(na.lam);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const V3<T> mv{r.m[0][h], r.m[1][h], r.m[2][h]};
      const V3<T> v{T(r.v[0][h]), T(r.v[1][h]), T(r.v[2][h])};
      const T rr = T(r.v[3][h]);
      V3<T> o;
      if constexpr (PRO == PRO_SMINUS) {
        const V3<T> c = cross3(mv, v);
        o = {c.x + mv.x * rr - lam * v.x, c.y + mv.y * rr - lam * v.y, c.z + mv.z * rr - lam * v.z};
      } else {  // PRO_M2T
        T orr;
        shift_solve_t(mv, v, rr, lam, o, orr);
      }
      if (h == 0) {
        u[0].x = o.x;
        u[1].x = o.y;
        u[2].x = o.z;
      } else {
        u[0].y = o.x;
        u[1].y = o.y;
        u[2].y = o.z;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Epilogue on the node pair (i, i+1): load phase (16-byte pair loads of the
// planes the mode needs) and compute phase.  F = filtered fields.
// ---------------------------------------------------------------------------
template <typename T, typename TIn, typename TOut, int EPI>
struct EpiRaw {
  static constexpr bool NODAL = !(EPI == EPI_STORE3 || EPI == EPI_RHS || EPI == EPI_ADDF || EPI == EPI_ENERGY);
  TIn v[4][2];   // x or p planes (nodal modes)
  T m[3][2];     // magnetization (nodal modes)
  T av[3][2];    // forward velocity (EPI_JT)
  T ar[2];       // forward multiplier (EPI_JT)
  double hf[3][2];  // spatial field (EPI_RHS)
  TOut rb[4][2];    // right-hand side (residual form)
};

template <typename T, typename TIn, typename TOut, int EPI>
__device__ __forceinline__ void epilogue_load(const PipeIO<T, TIn, TOut>& io, const NodalArgs& na, long long i,
                                              EpiRaw<T, TIn, TOut, EPI>& r) {
  const long long ng = io.ng;
  if constexpr (EpiRaw<T, TIn, TOut, EPI>::NODAL) {
    // the apply modes need only the multiplier plane of p
    constexpr bool ONLY_R = EPI == EPI_APPLY || EPI == EPI_APPLY_SYM;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      if (!ONLY_R || f == 3) load2(io.in + f * ng + i, r.v[f][0], r.v[f][1]);
      else r.v[f][0] = r.v[f][1] = TIn(0);
    }
    if constexpr (EPI != EPI_APPLY_SYM) {
#pragma unroll
      for (int f = 0; f < 3; ++f) load2(io.m + f * ng + i, r.m[f][0], r.m[f][1]);
    } else {
#pragma unroll
      for (int f = 0; f < 3; ++f) r.m[f][0] = r.m[f][1] = T(0);
    }
    if constexpr (EPI == EPI_JT || EPI == EPI_JT_RIGHT) {
#pragma unroll
      for (int f = 0; f < 3; ++f) load2(io.aux_v + f * ng + i, r.av[f][0], r.av[f][1]);
      load2(io.aux_r + i, r.ar[0], r.ar[1]);
    }
  } else if constexpr (EPI == EPI_ADDF) {
#pragma unroll
    for (int f = 0; f < 3; ++f) load2(io.aux_v + f * ng + i, r.av[f][0], r.av[f][1]);
  } else if constexpr (EPI == EPI_RHS || EPI == EPI_ENERGY) {
    if constexpr (EPI == EPI_ENERGY) {
#pragma unroll
      for (int f = 0; f < 3; ++f) load2(io.m + f * ng + i, r.m[f][0], r.m[f][1]);
    }
    if (na.hfield) {
#pragma unroll
      for (int f = 0; f < 3; ++f) load2(na.hfield + f * ng + i, r.hf[f][0], r.hf[f][1]);
    } else {
#pragma unroll
      for (int f = 0; f < 3; ++f) r.hf[f][0] = r.hf[f][1] = 0.0;
    }
  }
  if (io.rhs) {
    constexpr int NOUT = EPI == EPI_STORE3 ? 3 : 4;
#pragma unroll
    for (int f = 0; f < NOUT; ++f) load2(io.rhs + f * ng + i, r.rb[f][0], r.rb[f][1]);
  }
}

template <typename T, typename TIn, typename TOut, int EPI>
__device__ __forceinline__ void epilogue_compute(const EpiRaw<T, TIn, TOut, EPI>& r, int h, const T (&F)[3],
                                                 const NodalArgs& na, T (&o)[4]) {
  const T lam = T(na.lam);
  if constexpr (EPI == EPI_STORE3) {
    o[0] = F[0];
    o[1] = F[1];
    o[2] = F[2];
    o[3] = T(0);
  } else if constexpr (EPI == EPI_ADDF) {
    const T hs = T(na.hs);
    o[0] = r.av[0][h] - hs * F[0];
    o[1] = r.av[1][h] - hs * F[1];
    o[2] = r.av[2][h] - hs * F[2];
    o[3] = T(0);
  } else if constexpr (EPI == EPI_ENERGY) {
    // energy density chat/2 m.F - m.h, F = (-Delta_N) m (chat = cexc) or minus
    // the linear effective field (chat = 1); h = uniform + spatial field
    const T c = T(na.chat);
    const V3<T> m{r.m[0][h], r.m[1][h], r.m[2][h]};
    const V3<T> hf{T(na.hu0) + T(r.hf[0][h]), T(na.hu1) + T(r.hf[1][h]), T(na.hu2) + T(r.hf[2][h])};
    o[0] = T(0.5) * c * dot3(m, V3<T>{F[0], F[1], F[2]}) - dot3(m, hf);
    o[1] = o[2] = o[3] = T(0);
  } else if constexpr (EPI == EPI_RHS) {
    const T c = T(na.chat), hs = T(na.hs);
    o[0] = -c * F[0] + hs * (T(na.hu0) + T(r.hf[0][h]));
    o[1] = -c * F[1] + hs * (T(na.hu1) + T(r.hf[1][h]));
    o[2] = -c * F[2] + hs * (T(na.hu2) + T(r.hf[2][h]));
    o[3] = T(0);
  } else {
    const V3<T> m{r.m[0][h], r.m[1][h], r.m[2][h]};
    const V3<T> v{T(r.v[0][h]), T(r.v[1][h]), T(r.v[2][h])};
    const T rr = T(r.v[3][h]);
    if constexpr (EPI == EPI_APPLY) {
      V3<T> z;
      T zr;
      shift_solve(m, V3<T>{F[0], F[1], F[2]}, rr / lam, lam, z, zr);
      o[0] = z.x;
      o[1] = z.y;
      o[2] = z.z;
      o[3] = zr;
    } else if constexpr (EPI == EPI_APPLY_T) {
      const T inv_d = T(1) / (lam * lam + dot3(m, m));
      o[0] = F[0];
      o[1] = F[1];
      o[2] = F[2];
      o[3] = (lam * rr - dot3(m, v)) * inv_d / lam;
    } else if constexpr (EPI == EPI_MATVEC || EPI == EPI_MATVEC_T) {
      const V3<T> c = cross3(m, v);
      const T sg = EPI == EPI_MATVEC ? T(1) : T(-1);
      o[0] = F[0] + sg * (c.x + m.x * rr);
      o[1] = F[1] + sg * (c.y + m.y * rr);
      o[2] = F[2] + sg * (c.z + m.z * rr);
      o[3] = -sg * dot3(m, v);
    } else if constexpr (EPI == EPI_JT) {
      // J^T mu = (H mu_v - m^n x mu_v + (k/2) r_f mu_v - m^{n+1} mu_r, m_half . mu_v),
      // m = m^n, (v_f, r_f) the forward solution, m^{n+1} = m^n + k v_f,
      // m_half = m^n + (k/2) v_f; here v = mu_v and rr = mu_r.
      const T hk = T(na.half_k);
      const V3<T> vf{r.av[0][h], r.av[1][h], r.av[2][h]};
      const T rf = r.ar[h];
      const V3<T> c = cross3(m, v);
      const V3<T> m1{m.x + T(2) * hk * vf.x, m.y + T(2) * hk * vf.y, m.z + T(2) * hk * vf.z};
      const V3<T> mh{m.x + hk * vf.x, m.y + hk * vf.y, m.z + hk * vf.z};
      o[0] = F[0] - c.x + hk * rf * v.x - m1.x * rr;
      o[1] = F[1] - c.y + hk * rf * v.y - m1.y * rr;
      o[2] = F[2] - c.z + hk * rf * v.z - m1.z * rr;
      o[3] = dot3(mh, v);
    } else if constexpr (EPI == EPI_JT_RIGHT) {
      // m = m_half, (v, rr) = y; u = (S~ + lambda I)^{-T} y (the prologue's
      // nodal solve, recomputed), w = (F, u_r / lambda) = (calH + lambda I)^{-1} u;
      // out = u + N w - lambda w with N w = (-m^n x w_v + (k/2) r_f w_v -
      // m^{n+1} w_r, m_half . w_v), m^n = m_half - (k/2) v_f, m^{n+1} = m_half +
      // (k/2) v_f; the multiplier row reduces to m_half . w_v.
      const T hk = T(na.half_k);
      const V3<T> vf{r.av[0][h], r.av[1][h], r.av[2][h]};
      const T rf = r.ar[h];
      V3<T> u;
      T ur;
      shift_solve_t(m, v, rr, lam, u, ur);
      const V3<T> wv{F[0], F[1], F[2]};
      const T wr = ur / lam;
      const V3<T> mn{m.x - hk * vf.x, m.y - hk * vf.y, m.z - hk * vf.z};
      const V3<T> m1{m.x + hk * vf.x, m.y + hk * vf.y, m.z + hk * vf.z};
      const V3<T> c = cross3(mn, wv);
      const T s = hk * rf - lam;
      o[0] = u.x - c.x + s * wv.x - m1.x * wr;
      o[1] = u.y - c.y + s * wv.y - m1.y * wr;
      o[2] = u.z - c.z + s * wv.z - m1.z * wr;
      o[3] = dot3(m, wv);
    } else if constexpr (EPI == EPI_APPLY_SYM) {
      o[0] = F[0];
      o[1] = F[1];
      o[2] = F[2];
      o[3] = rr / lam;
    } else if constexpr (EPI == EPI_FUSED_SYM) {
      const T ur = -dot3(m, v) - lam * rr;
      o[0] = v.x + F[0];
      o[1] = v.y + F[1];
      o[2] = v.z + F[2];
      o[3] = rr + ur / lam;
    } else {  // EPI_FUSED
      const T ur = -dot3(m, v) - lam * rr;
      const V3<T> w{v.x + F[0], v.y + F[1], v.z + F[2]};
      const T wr = rr + ur / lam;
      V3<T> z;
      T zr;
      shift_solve(m, w, wr, lam, z, zr);
      o[0] = z.x;
      o[1] = z.y;
      o[2] = z.z;
      o[3] = zr;
    }
  }
}

// ---------------------------------------------------------------------------
// Shared phases of the x passes (every thread of the block calls them; they
// contain block barriers).  lds holds 3 fields x LX lines x SL complex.
// ---------------------------------------------------------------------------
// LDS holds the real node pairs (u[2k], u[2k+1]) of each line at position k:
// half-length complex DFT, split step U[k] = E[k] + w^k O[k] (E/O the DFTs of
// the even/odd samples), store of the rows of three half spectra.
template <typename T, int NH>
__device__ __forceinline__ void x_r2c_store(cx<T>* lds, long long line0, long long nlines,
                                            cx<T>* __restrict__ spec, const SpecGeom& g,
                                            const cx<T>* __restrict__ twx) {
  using C = XCfg<T, NH>;
  const int tid = threadIdx.x;
  const int t = tid % C::TPL, ln = tid / C::TPL;
  cx<T>* line_lds = lds + ln * C::SL;
  auto acc = [line_lds](int pos) -> cx<T>& { return line_lds[xphys(pos)]; };
  cx<T> v[C::P];
#pragma unroll
  for (int q = 0; q < C::P; ++q) v[in_slot<C::KEY>(q)] = acc(t + C::TPL * q);
  line_fft<T, C::KEY, -1>(v, t, acc, twx, 2);
  __syncthreads();
#pragma unroll
  for (int s = 0; s < C::P; ++s) acc(t + C::TPL * out_q<C::KEY>(s)) = v[s];
  __syncthreads();
  constexpr int CS = 3 * (NH + 1);
  for (int e = tid; e < C::LX * CS; e += C::NT) {
    const int l = e / CS, col = e % CS;
    const long long line = line0 + l;
    if (line >= nlines) continue;
    const int f = col / (NH + 1), k = col % (NH + 1);
    const cx<T>* Z = lds + (f * C::LX + l) * C::SL;
    const cx<T> a = Z[xphys(k == NH ? 0 : k)];
    const cx<T> bc = Z[xphys(k == 0 ? 0 : NH - k)];
    const cx<T> b{bc.x, -bc.y};
    const cx<T> E{T(0.5) * (a.x + b.x), T(0.5) * (a.y + b.y)};
    const cx<T> O{T(0.5) * (a.y - b.y), T(-0.5) * (a.x - b.x)};
    const cx<T> w = twx[k];
    spec[line * g.rs + col] = cadd(E, cmul(w, O));
  }
}

// Load the rows of three half spectra of the block's lines, undo the split
// step (Z[k] = (U[k] + conj U[NH-k]) + i w^{-k} (U[k] - conj U[NH-k])) and run
// the inverse half-length DFT; on return LDS position k of each line holds the
// node pair (2k, 2k+1) of each field.
template <typename T, int NH>
__device__ __forceinline__ void x_load_c2r(cx<T>* lds, long long line0, long long nlines,
                                           const cx<T>* __restrict__ spec, const SpecGeom& g,
                                           const cx<T>* __restrict__ twx) {
  using C = XCfg<T, NH>;
  const int tid = threadIdx.x;
  constexpr int CS = 3 * (NH + 1);
  {
    constexpr int NV = C::LX * CS;
    constexpr int ITERS = (NV + C::NT - 1) / C::NT;
#pragma unroll
    for (int it = 0; it < ITERS; ++it) {
      const int e0 = tid + it * C::NT;
      const int e = e0 < NV ? e0 : NV - 1;
      const int l = e / CS, col = e % CS;
      const long long line = line0 + l < nlines ? line0 + l : nlines - 1;
      const cx<T> val = spec[line * g.rs + col];
      if (e0 < NV) {
        const int f = col / (NH + 1), k = col % (NH + 1);
        lds[(f * C::LX + l) * C::SL + xphys(k)] = line0 + l < nlines ? val : cx<T>{T(0), T(0)};
      }
    }
  }
  __syncthreads();
  const int t = tid % C::TPL, ln = tid / C::TPL;
  cx<T>* line_lds = lds + ln * C::SL;
  auto acc = [line_lds](int pos) -> cx<T>& { return line_lds[xphys(pos)]; };
  cx<T> v[C::P];
#pragma unroll
  for (int q = 0; q < C::P; ++q) {
    const int k = t + C::TPL * q;
    const cx<T> a = acc(k);
    const cx<T> bc = acc(NH - k);
    const cx<T> e{a.x + bc.x, a.y - bc.y};
    const cx<T> d{a.x - bc.x, a.y + bc.y};
    const cx<T> o = cmulc(d, twx[k]);
    v[in_slot<C::KEY>(q)] = {e.x - o.y, e.y + o.x};
  }
  line_fft<T, C::KEY, 1>(v, t, acc, twx, 2);
  __syncthreads();
#pragma unroll
  for (int s = 0; s < C::P; ++s) acc(t + C::TPL * out_q<C::KEY>(s)) = v[s];
  __syncthreads();
}

// ---------------------------------------------------------------------------
// k_xfwd
// ---------------------------------------------------------------------------
template <typename T, typename TIn, int NH, int PRO>
__global__ __launch_bounds__(192) void k_xfwd(const TIn* __restrict__ in, const T* __restrict__ m,
                                              cx<T>* __restrict__ spec, SpecGeom g, NodalArgs na,
                                              const cx<T>* __restrict__ twx) {
  using C = XCfg<T, NH>;
  __shared__ cx<T> lds[3 * C::LX * C::SL];
  const int tid = threadIdx.x;
  const long long nlines = (long long)g.ny * g.nz;
  const long long line0 = (long long)blockIdx.x * C::LX;
  constexpr int NX = 2 * NH;

  // Copy-in with the prologue.  Indices are clamped instead of guarded so that
  // the global loads of all iterations are unconditional and can be in flight
  // together; only the LDS writes are predicated.
  constexpr int NPAIR = C::LX * NH;
  constexpr int ITERS = (NPAIR + C::NT - 1) / C::NT;
  constexpr int BATCH = sizeof(T) == 4 ? LLG_XBATCH_F32 : LLG_XBATCH_F64;
#pragma unroll
  for (int it0 = 0; it0 < ITERS; it0 += BATCH) {
    ProRaw<T, TIn, PRO> raw[BATCH];
#pragma unroll
    for (int b = 0; b < BATCH; ++b) {
      if (it0 + b < ITERS) {
        const int e0 = tid + (it0 + b) * C::NT;
        const int e = e0 < NPAIR ? e0 : NPAIR - 1;
        const int l = e / NH, xp = e % NH;
        const long long line = line0 + l < nlines ? line0 + l : nlines - 1;
        prologue_load<T, TIn, PRO>(in, m, g.ng, line * NX + 2 * xp, raw[b]);
      }
    }
#pragma unroll
    for (int b = 0; b < BATCH; ++b) {
      if (it0 + b < ITERS) {
        const int e0 = tid + (it0 + b) * C::NT;
        const int e = e0 < NPAIR ? e0 : NPAIR - 1;
        const int l = e / NH, xp = e % NH;
        cx<T> u[3];
        prologue_compute<T, TIn, PRO>(raw[b], na, u);
        if (e0 < NPAIR) {
          const bool live = line0 + l < nlines;
#pragma unroll
          for (int f = 0; f < 3; ++f) lds[(f * C::LX + l) * C::SL + xphys(xp)] = live ? u[f] : cx<T>{T(0), T(0)};
        }
      }
    }
  }
  __syncthreads();
  x_r2c_store<T, NH>(lds, line0, nlines, spec, g, twx);
}

// ---------------------------------------------------------------------------
// k_xfwd_upd: the x-forward pass of an Arnoldi step's operator that first
// forms its own input, the next basis direction of delayed CGS2 (UpdFirst):
// the separate update pass would write u_new and this pass read it straight
// back.
//   Phase 1, one (plane, node pair) per loop trip as in the update pass: the
//   loads of w and of the j + 1 basis directions are issued together, u_new
//   is stored, its inner products accumulated (the directions stay in
//   registers between the two uses), and u_new is parked in LDS in the
//   precision T of the passes (the prologue converts its input to T first).
//   Phase 2: the prologue PRO on the parked values, into the DFT layout.
// JB >= j bounds the columns held (the guards q <= j are uniform branches).
// W: float (the precision form's float32 operator output, converted exactly)
// or double.
// ---------------------------------------------------------------------------
// Items per trip of k_xfwd_upd with at most 4 directions (2 with up to 8).
// At 256^3 4 is fastest: 2, 3 and 6 made the pass 0.5-0.8% slower.
#ifndef LLG_UPD_NB_SMALL
#define LLG_UPD_NB_SMALL 4
#endif
template <typename T, typename W, int NH, int PRO, int JB>
__global__ __launch_bounds__(192) void k_xfwd_upd(UpdFirst ua, const W* __restrict__ w, const T* __restrict__ m,
                                                  cx<T>* __restrict__ spec, SpecGeom g, NodalArgs na,
                                                  const cx<T>* __restrict__ twx) {
  using C = XCfg<T, NH>;
  constexpr bool NODAL = PRO != PRO_COPY3;  // the prologue needs all four planes and m
  __shared__ cx<T> lds[3 * C::LX * C::SL];
  __shared__ cx<T> lds_r[NODAL ? C::LX * NH : 1];  // plane 3 of u_new (nodal prologues)
  __shared__ double dred[C::NT / 64][JB + 2];
  const int tid = threadIdx.x;
  const long long nlines = (long long)g.ny * g.nz;
  const long long line0 = (long long)blockIdx.x * C::LX;
  constexpr int NX = 2 * NH;
  constexpr int NPAIR = C::LX * NH;
  const int J = ua.j;
  double gm[JB + 1];
#pragma unroll
  for (int q = 0; q <= JB; ++q) gm[q] = q <= J ? ua.gamma[q] : 0.0;
  double acc[JB + 2];  // u_q . u_new (q <= j), then u_new . u_new
#pragma unroll
  for (int q = 0; q < JB + 2; ++q) acc[q] = 0.0;
  const long long np = (long long)(line0 + C::LX <= nlines ? C::LX : nlines - line0) * NH;  // live pairs
  // NB items per trip: all their loads are issued before any store (the
  // stores could alias them as far as the compiler knows), which keeps
  // NB (j + 2) loads of each wave in flight
  constexpr int NB = JB <= 3 ? LLG_UPD_NB_SMALL : 2;
  static_assert(JB <= 7, "more directions than a batch of items keeps in registers");
  constexpr int NITEM = 4 * NPAIR;
#pragma unroll 1
  for (int t0 = tid; t0 < NITEM; t0 += NB * C::NT) {
    long long k[NB];
    int slot[NB];
    bool live[NB];
    double s0[NB], s1[NB], q0[NB][JB + 1], q1[NB][JB + 1];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int tt = t0 + b * C::NT;
      const int t = tt < NITEM ? tt : NITEM - 1;
      const int f = t / NPAIR, e = t - f * NPAIR;
      const int l = e / NH, xp = e - l * NH;
      live[b] = tt < NITEM && e < np;
      k[b] = f * g.ng + (e < np ? line0 + l : line0) * NX + 2 * xp;
      // LDS destination: DFT slot of field f, or (plane 3) the parking row
      slot[b] = tt >= NITEM ? -1 : (f < 3 ? (f * C::LX + l) * C::SL + xphys(xp) : -2 - e);
      W w0, w1;
      load2(w + k[b], w0, w1);
      s0[b] = double(w0);
      s1[b] = double(w1);
#pragma unroll
      for (int q = 0; q <= JB; ++q) {
        if (q <= J) load2((q == 0 ? ua.u0 : ua.U1 + (q - 1) * ua.ld) + k[b], q0[b][q], q1[b][q]);
      }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
#pragma unroll
      for (int q = 0; q <= JB; ++q) {
        if (q <= J) {
          s0[b] = fma(-gm[q], q0[b][q], s0[b]);
          s1[b] = fma(-gm[q], q1[b][q], s1[b]);
        }
      }
      const double a0 = s0[b] * ua.inv_beta, a1 = s1[b] * ua.inv_beta;
      if (live[b]) store2(ua.unew + k[b], a0, a1);
      const double d0 = live[b] ? a0 : 0.0, d1 = live[b] ? a1 : 0.0;
#pragma unroll
      for (int q = 0; q <= JB; ++q) {
        if (q <= J) acc[q] = fma(q0[b][q], d0, fma(q1[b][q], d1, acc[q]));
      }
      acc[JB + 1] = fma(d0, d0, fma(d1, d1, acc[JB + 1]));
      const cx<T> v{T(d0), T(d1)};  // dead lines filter zeros
      if (slot[b] >= 0) lds[slot[b]] = v;
      else if constexpr (NODAL) {
        if (slot[b] <= -2) lds_r[-2 - slot[b]] = v;
      }
    }
  }
  // block partials of the inner products (fixed order: deterministic)
  const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
  for (int q = 0; q < JB + 2; ++q) {
    if (q <= J || q == JB + 1) {
      double s = acc[q];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
      if (lane == 0) dred[wv][q] = s;
    }
  }
  __syncthreads();
  if (tid <= J + 1) {
    const int src = tid <= J ? tid : JB + 1;
    double s = dred[0][src];
#pragma unroll
    for (int k = 1; k < C::NT / 64; ++k) s += dred[k][src];
    ua.partial[(long long)tid * gridDim.x + blockIdx.x] = s;
  }
  if constexpr (NODAL) {
    // prologue in place: each node pair's slots are read and rewritten by
    // the one thread that handles the pair here
    constexpr int ITERS = (NPAIR + C::NT - 1) / C::NT;
#pragma unroll
    for (int it = 0; it < ITERS; ++it) {
      const int e = tid + it * C::NT;
      if (e < NPAIR) {
        const int l = e / NH, xp = e - l * NH;
        const bool live = e < np;
        const long long i = (live ? line0 + l : line0) * NX + 2 * xp;
        ProRaw<T, T, PRO> raw;
#pragma unroll
        for (int f = 0; f < 3; ++f) load2(m + f * g.ng + i, raw.m[f][0], raw.m[f][1]);
#pragma unroll
        for (int f = 0; f < 3; ++f) {
          const cx<T> v = lds[(f * C::LX + l) * C::SL + xphys(xp)];
          raw.v[f][0] = v.x;
          raw.v[f][1] = v.y;
        }
        raw.v[3][0] = lds_r[e].x;
        raw.v[3][1] = lds_r[e].y;
        cx<T> u[3];
        prologue_compute<T, T, PRO>(raw, na, u);
#pragma unroll
        for (int f = 0; f < 3; ++f) lds[(f * C::LX + l) * C::SL + xphys(xp)] = live ? u[f] : cx<T>{T(0), T(0)};
      }
    }
    __syncthreads();
  }
  x_r2c_store<T, NH>(lds, line0, nlines, spec, g, twx);
}

// ---------------------------------------------------------------------------
// k_xinv
// ---------------------------------------------------------------------------
// With DOTS (a matvec or fused M^{-1} A pass writing a float64 Krylov
// vector) the pass also forms the inner products of its output with the
// Arnoldi basis directions (BasisDots), from the output values it still
// holds in registers: the separate inner-product pass and its read of the
// output disappear.
template <typename T, typename TIn, typename TOut, int NH, int EPI, bool DOTS = false>
__global__ __launch_bounds__(192) void k_xinv(PipeIO<T, TIn, TOut> io, const cx<T>* __restrict__ spec,
                                              SpecGeom g, NodalArgs na, const cx<T>* __restrict__ twx,
                                              BasisDots bd) {
  static_assert(!DOTS || EPI == EPI_MATVEC || EPI == EPI_FUSED || EPI == EPI_JT_RIGHT,
                "dots: Krylov output of a matvec or fused pass");
  using C = XCfg<T, NH>;
  __shared__ cx<T> lds[3 * C::LX * C::SL];
  const int tid = threadIdx.x;
  const long long nlines = (long long)g.ny * g.nz;
  const long long line0 = (long long)blockIdx.x * C::LX;
  constexpr int NX = 2 * NH;
  constexpr int CS = 3 * (NH + 1);

  x_load_c2r<T, NH>(lds, line0, nlines, spec, g, twx);

  // Epilogue: clamped (unconditional) loads issued a batch of node pairs at
  // a time, predicated stores.
  double rsum = 0.0;
  constexpr int NPAIR = C::LX * NH;
  constexpr int ITERS = (NPAIR + C::NT - 1) / C::NT;
  constexpr int BATCH = sizeof(T) == 4 ? LLG_XBATCH_F32 : LLG_XBATCH_F64;
  constexpr int KEEP = DOTS ? ITERS : 1;
  T keep0[KEEP][4], keep1[KEEP][4];  // outputs of the thread's node pairs (0 where not live)
#pragma unroll
  for (int it0 = 0; it0 < ITERS; it0 += BATCH) {
  EpiRaw<T, TIn, TOut, EPI> raw[BATCH];
#pragma unroll
  for (int b = 0; b < BATCH; ++b) {
    if (it0 + b < ITERS) {
      const int e0 = tid + (it0 + b) * C::NT;
      const int e = e0 < NPAIR ? e0 : NPAIR - 1;
      const int l = e / NH, xp = e % NH;
      const long long line = line0 + l < nlines ? line0 + l : nlines - 1;
      epilogue_load<T, TIn, TOut, EPI>(io, na, line * NX + 2 * xp, raw[b]);
    }
  }
#pragma unroll
  for (int b = 0; b < BATCH; ++b) {
    if (it0 + b >= ITERS) continue;
    const int e0 = tid + (it0 + b) * C::NT;
    const int e = e0 < NPAIR ? e0 : NPAIR - 1;
    const int l = e / NH, xp = e % NH;
    const bool live = e0 < NPAIR && line0 + l < nlines;
    const long long line = line0 + l < nlines ? line0 + l : nlines - 1;
    const long long i = line * NX + 2 * xp;
    cx<T> fz[3];
#pragma unroll
    for (int f = 0; f < 3; ++f) fz[f] = lds[(f * C::LX + l) * C::SL + xphys(xp)];
    T o0[4], o1[4];
    {
      const T F0[3] = {fz[0].x, fz[1].x, fz[2].x};
      epilogue_compute<T, TIn, TOut, EPI>(raw[b], 0, F0, na, o0);
      const T F1[3] = {fz[0].y, fz[1].y, fz[2].y};
      epilogue_compute<T, TIn, TOut, EPI>(raw[b], 1, F1, na, o1);
    }
    if constexpr (EPI == EPI_RHS) {
      if (io.out_f && live) {
#pragma unroll
        for (int f = 0; f < 3; ++f) store2(io.out_f + f * io.ng + i, fz[f].x, fz[f].y);
      }
    }
    constexpr int NOUT = EPI == EPI_STORE3 ? 3 : (EPI == EPI_ENERGY ? 0 : 4);
    if constexpr (EPI == EPI_ENERGY) {
      if (live) rsum += double(o0[0]) + double(o1[0]);
    }
    if (io.rhs) {
#pragma unroll
      for (int f = 0; f < NOUT; ++f) {
        o0[f] = T(raw[b].rb[f][0]) - o0[f];
        o1[f] = T(raw[b].rb[f][1]) - o1[f];
        if (live) rsum += double(o0[f]) * double(o0[f]) + double(o1[f]) * double(o1[f]);
      }
    }
    if (live) {
#pragma unroll
      for (int f = 0; f < NOUT; ++f) store2(io.out + f * io.ng + i, TOut(o0[f]), TOut(o1[f]));
    }
    if constexpr (DOTS) {
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        keep0[it0 + b][f] = live ? o0[f] : T(0);
        keep1[it0 + b][f] = live ? o1[f] : T(0);
      }
    }
  }
  }
  if constexpr (DOTS) {
    // u_q . out for q < nv: per column, the clamped (unconditional) loads of
    // all the thread's node pairs are in flight together; dead pairs weigh 0.
    __shared__ double dred[C::NT / 64][kBasisDotsMax];
    const int lane = tid & 63, wv = tid >> 6;
    for (int q = 0; q < bd.nv; ++q) {
      const double* col = q == 0 ? bd.u0 : bd.U1 + (q - 1) * bd.ld;
      double t = 0.0;
#pragma unroll
      for (int it = 0; it < ITERS; ++it) {
        const int e0 = tid + it * C::NT;
        const int e = e0 < NPAIR ? e0 : NPAIR - 1;
        const int l = e / NH, xp = e % NH;
        const long long line = line0 + l < nlines ? line0 + l : nlines - 1;
        const long long i = line * NX + 2 * xp;
#pragma unroll
        for (int f = 0; f < 4; ++f) {
          double a0, a1;
          load2(col + f * io.ng + i, a0, a1);
          t = fma(a0, double(keep0[it][f]), fma(a1, double(keep1[it][f]), t));
        }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
      if (lane == 0) dred[wv][q] = t;
    }
    __syncthreads();
    if (tid < bd.nv) {
      double t = dred[0][tid];
#pragma unroll
      for (int k = 1; k < C::NT / 64; ++k) t += dred[k][tid];
      bd.partial[(long long)tid * gridDim.x + blockIdx.x] = t;
    }
  }
  if (io.red) {
    // block partial of the residual norm or of the energy (fixed order: deterministic)
    __shared__ double rs[C::NT / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) rsum += __shfl_xor(rsum, off, 64);
    if ((tid & 63) == 0) rs[tid >> 6] = rsum;
    __syncthreads();
    if (tid == 0) {
      double t = rs[0];
#pragma unroll
      for (int k = 1; k < C::NT / 64; ++k) t += rs[k];
      io.red[blockIdx.x] = t;
    }
  }
}

// ---------------------------------------------------------------------------
// k_xmid: the junction of the precision form's two float32 pipelines.  One
// kernel finishes the preconditioner apply (C2R along x, closed-form nodal
// inverse, z = M^{-1} v written as the flexible basis vector) and starts the
// matvec on z (R2C along x of z's velocity planes), handing z over in LDS:
// the matvec's x-forward pass and its read of z disappear.  Each node pair
// is owned by one thread, which reads the apply's field from an LDS slot and
// writes z back into the same slot.
// ---------------------------------------------------------------------------
template <int NH>
__global__ __launch_bounds__(192) void k_xmid(PipeIO<float, double, float> io, cx<float>* __restrict__ spec,
                                              SpecGeom g, NodalArgs na, const cx<float>* __restrict__ twx) {
  using T = float;
  using C = XCfg<T, NH>;
  __shared__ cx<T> lds[3 * C::LX * C::SL];
  const int tid = threadIdx.x;
  const long long nlines = (long long)g.ny * g.nz;
  const long long line0 = (long long)blockIdx.x * C::LX;
  constexpr int NX = 2 * NH;
  x_load_c2r<T, NH>(lds, line0, nlines, spec, g, twx);

  constexpr int NPAIR = C::LX * NH;
  constexpr int ITERS = (NPAIR + C::NT - 1) / C::NT;
  constexpr int BATCH = LLG_XMID_BATCH;
#pragma unroll
  for (int it0 = 0; it0 < ITERS; it0 += BATCH) {
    EpiRaw<T, double, T, EPI_APPLY> raw[BATCH];
#pragma unroll
    for (int b = 0; b < BATCH; ++b) {
      if (it0 + b < ITERS) {
        const int e0 = tid + (it0 + b) * C::NT;
        const int e = e0 < NPAIR ? e0 : NPAIR - 1;
        const int l = e / NH, xp = e % NH;
        const long long line = line0 + l < nlines ? line0 + l : nlines - 1;
        epilogue_load<T, double, T, EPI_APPLY>(io, na, line * NX + 2 * xp, raw[b]);
      }
    }
#pragma unroll
    for (int b = 0; b < BATCH; ++b) {
      if (it0 + b >= ITERS) continue;
      const int e0 = tid + (it0 + b) * C::NT;
      if (e0 >= NPAIR) continue;  // clamped duplicate: neither stored nor handed over
      const int l = e0 / NH, xp = e0 % NH;
      const bool live = line0 + l < nlines;
      const long long line = live ? line0 + l : nlines - 1;
      const long long i = line * NX + 2 * xp;
      cx<T> fz[3];
#pragma unroll
      for (int f = 0; f < 3; ++f) fz[f] = lds[(f * C::LX + l) * C::SL + xphys(xp)];
      T o0[4], o1[4];
      {
        const T F0[3] = {fz[0].x, fz[1].x, fz[2].x};
        epilogue_compute<T, double, T, EPI_APPLY>(raw[b], 0, F0, na, o0);
        const T F1[3] = {fz[0].y, fz[1].y, fz[2].y};
        epilogue_compute<T, double, T, EPI_APPLY>(raw[b], 1, F1, na, o1);
      }
      if (live) {
#pragma unroll
        for (int f = 0; f < 4; ++f) store2(io.out + f * io.ng + i, o0[f], o1[f]);
      }
#pragma unroll
      for (int f = 0; f < 3; ++f)
        lds[(f * C::LX + l) * C::SL + xphys(xp)] = live ? cx<T>{o0[f], o1[f]} : cx<T>{T(0), T(0)};
    }
  }
  __syncthreads();
  x_r2c_store<T, NH>(lds, line0, nlines, spec, g, twx);
}

// ---------------------------------------------------------------------------
// k_axis: DFTs along y (axis 1) or z (axis 2).  MODE 0 forward, 1 inverse,
// 2 forward -> multiplier -> inverse.
// ---------------------------------------------------------------------------
// Spectral columns per axis block (elements of elem_bytes bytes); mixed-radix
// lengths up to 24 run one thread per line.  At N = 512 the LDS of a block
// (N (W + 1) elements) limits W: float32 takes LLG_AXIS_W512_F32 columns,
// float64 LLG_AXIS_W512_F64 (8 each: 64- and 128-byte row segments).  At
// 512^3, float32 ran 4.37 solves/s with 8 columns, 4.35 with 16 and 3.49
// with 4; float64 3.09 with 8 against 2.93 with 4 (512^2: 822 against 803).
#ifndef LLG_AXIS_W512_F32
#define LLG_AXIS_W512_F32 8
#endif
#ifndef LLG_AXIS_W512_F64
#define LLG_AXIS_W512_F64 8
#endif
// float32 passes along 256-point lines: 16 columns (8 made them 30% slower,
// 32 made the fused pass 35% slower)
#ifndef LLG_AXIS_W256_F32
#define LLG_AXIS_W256_F32 16
#endif
__host__ __device__ constexpr int axis_w(int elem_bytes, int n) {
  return n <= 16 ? 64
                 : (n >= 512 ? (elem_bytes == 4 ? LLG_AXIS_W512_F32 : LLG_AXIS_W512_F64)
                             : (n == 256 && elem_bytes == 4 ? LLG_AXIS_W256_F32
                                                             : ((n & (n - 1)) != 0 && n <= 24 ? 64 : 16)));
}

template <typename T, int N, int MODE>
__global__ __launch_bounds__(axis_w(int(sizeof(T)), N) * (N / plan_p(axis_plan_key(int(sizeof(T)), N)))) void k_axis(
    cx<T>* __restrict__ spec, SpecGeom g, int axis, SymArgs sym, const cx<T>* __restrict__ tw) {
  constexpr int KEY = axis_plan_key(int(sizeof(T)), N);
  constexpr int P = plan_p(KEY), TPL = N / P, W = axis_w(int(sizeof(T)), N);
  __shared__ cx<T> lds[N * (W + 1)];
  const int c = threadIdx.x % W, t = threadIdx.x / W;
  // XCD-aware block numbering.  Blocks are dispatched to the 8 XCDs (each
  // with its own L2) round-robin by linear id; renumbered, every XCD runs one
  // contiguous range of (column group, outer) blocks instead.
  //  * Along y the outer index is the z plane, so each XCD then streams its
  //    own contiguous slab of the spectrum (256^3: y passes 4-5% faster in
  //    float32, up to 14% in float64).
  //  * Row segments shorter than a 128-byte line (float32 at N = 512: 8
  //    columns, 64 bytes) share each line with the next column group, whose
  //    half is then an L2 hit (512^3: all three passes 2-5% faster).
  // Along z with whole-line segments it gains nothing (each block spans every
  // z plane anyway), and those passes keep the plain numbering.  The
  // renumbering is a bijection of the grid.
  int col, outer;
  if (W * sizeof(cx<T>) < 128 || axis == 1) {
    constexpr unsigned kXcd = 8;
    const unsigned nb = gridDim.x * gridDim.y, lin = blockIdx.x + gridDim.x * blockIdx.y;
    const unsigned xcd = lin % kXcd, k = lin / kXcd, per = nb / kXcd, rem = nb % kXcd;
    const unsigned logical = xcd < rem ? xcd * (per + 1) + k : rem * (per + 1) + (xcd - rem) * per + k;
    col = (logical % gridDim.x) * W + c;
    outer = logical / gridDim.x;
  } else {
    col = blockIdx.x * W + c;
    outer = blockIdx.y;
  }
  long long sp, so;
  if (axis == 1) {
    sp = g.rs;
    so = (long long)g.rs * g.ny;
  } else {
    sp = (long long)g.rs * g.ny;
    so = g.rs;
  }
  const bool valid = col < g.cs;
  cx<T>* base = spec + outer * so + (valid ? col : 0);
  cx<T> v[P];
#pragma unroll
  for (int q = 0; q < P; ++q) v[in_slot<KEY>(q)] = base[(t + TPL * q) * sp];
  if (!valid) {
#pragma unroll
    for (int q = 0; q < P; ++q) v[q] = cx<T>{T(0), T(0)};
  }
  cx<T>* col_lds = lds + c;
  auto acc = [col_lds](int pos) -> cx<T>& { return col_lds[pos * (W + 1)]; };

  if constexpr (MODE == 0 || MODE == 1) {
    line_fft<T, KEY, MODE == 0 ? -1 : 1>(v, t, acc, tw, 1);
  } else {
    line_fft<T, KEY, -1>(v, t, acc, tw, 1);
    // Fourier multiplier (a + b |xi|^2)^{+-1} / N_g
    const int kx = col % (g.nh + 1);
    const double xx = sym.cx * kx;
    double base2 = xx * xx;
    if (axis == 2) {
      const int ky = outer < g.ny / 2 ? outer : outer - g.ny;
      const double yy = sym.cy * ky;
      base2 += yy * yy;
    }
    const double caxis = axis == 1 ? sym.cy : sym.cz;
    cx<T> w[P];
#pragma unroll
    for (int s = 0; s < P; ++s) {
      const int q = out_q<KEY>(s);
      const int kp = t + TPL * q;
      const int ks = kp < N / 2 ? kp : kp - N;
      const double aa = caxis * ks;
      const double lam2 = base2 + aa * aa;
      double mult = sym.a + sym.b * lam2;
      mult = sym.invert ? sym.inv_ng / mult : sym.inv_ng * mult;
      w[in_slot<KEY>(q)] = cscale(v[s], T(mult));
    }
    line_fft<T, KEY, 1>(w, t, acc, tw, 1);
#pragma unroll
    for (int s = 0; s < P; ++s) v[s] = w[s];
  }
  if (valid) {
#pragma unroll
    for (int s = 0; s < P; ++s) base[(t + TPL * out_q<KEY>(s)) * sp] = v[s];
  }
}

}  // namespace llg
