// Device building blocks of the batched line FFTs used by every spectral pass.
//
// The exchange block H = a I + b(-Delta_N) of the saddle operator and the
// shifted factor calH + lambda I of the split preconditioner are diagonal in
// Fourier space (Sec. 2.3; Sec. 3.2, Algorithm 1).  Every spectral pass of the
// library is therefore a set of independent 1-D DFTs along one grid axis
// ("lines"), each computed by a small team of threads with a Stockham
// autosort schedule: a line of N complex points is held by TPL = N / P
// threads, P points each, and the radix stages exchange data through LDS.
//
// Conventions
//  * forward DFT X[k] = sum_n x[n] exp(-2 pi i k n / N), inverse with +i, both
//    unnormalized (the 1/N_g factor is folded into the Fourier symbol);
//  * a thread t of a line always holds, at the start of the first stage and at
//    the end of the last stage, the positions t + TPL*q, q = 0..P-1; the slot
//    of position q is fixed at compile time (in_slot / out_q below), so
//    global loads/stores and the fused forward->scale->inverse hand-over need
//    no data movement;
//  * twiddles come from a per-length table tw[m] = exp(-2 pi i m / L) built on
//    the host in extended precision.

#pragma once
#include <hip/hip_runtime.h>

namespace llg {

template <typename T>
struct cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.x * s, a.y * s}; }
// multiply by -i (DIR = -1, forward) or +i (DIR = +1, inverse)
template <typename T, int DIR>
__device__ __forceinline__ cx<T> mul_dir_i(cx<T> a) {
  return DIR < 0 ? cx<T>{a.y, -a.x} : cx<T>{-a.y, a.x};
}

// ---------------------------------------------------------------------------
// Radix plans: P points per thread, TPL = N / P threads per line (always a
// power of two), up to four stages whose radices all divide P.
//   N:   2   4   8  16  32    64    128    256     512      1024
//   R:  [2] [4] [8][16][8,4] [8,8] [16,8] [16,16] [8,8,8] [16,16,4]
// Lengths 3 * 2^k and 5 * 2^k (the grids N = 24, 48 of the paper's 3D
// experiments, among others) keep the odd factor inside P:
//   N:   3   5   6     10    12    20    24    40 (P 20)  48 (P 12)  80 (P 20)
//   R:  [3] [5] [2,3] [2,5] [4,3] [4,5] [8,3] [4,2,5]    [4,4,3]    [4,4,5]
//   N:   96 (P 24)  160 (P 20)  192 (P 24)  320 (P 20)  384 (P 24)
//   R:  [8,4,3]    [4,4,2,5]   [8,8,3]     [4,4,4,5]   [8,4,4,3]
// ---------------------------------------------------------------------------
// A plan key is the line length N, or N | kPlanFine for a plan with fewer
// points per thread (more threads per line, one more LDS exchange): the
// float64 x passes use it at N = 128, 256 to halve their LDS per block.
constexpr int kPlanFine = 1 << 16;
__host__ __device__ constexpr int plan_n(int key) { return key & (kPlanFine - 1); }

struct Plan {
  int p, nst, r0, r1, r2, r3;
};
__host__ __device__ constexpr Plan plan_of(int n) {
  switch (n) {
    case 128 | kPlanFine: return {8, 3, 8, 4, 4, 1};
    case 256 | kPlanFine: return {8, 3, 8, 8, 4, 1};
    case 2: return {2, 1, 2, 1, 1, 1};
    case 3: return {3, 1, 3, 1, 1, 1};
    case 4: return {4, 1, 4, 1, 1, 1};
    case 5: return {5, 1, 5, 1, 1, 1};
    case 6: return {6, 2, 2, 3, 1, 1};
    case 8: return {8, 1, 8, 1, 1, 1};
    case 10: return {10, 2, 2, 5, 1, 1};
    case 12: return {12, 2, 4, 3, 1, 1};
    case 16: return {16, 1, 16, 1, 1, 1};
    case 20: return {20, 2, 4, 5, 1, 1};
    case 24: return {24, 2, 8, 3, 1, 1};
    case 32: return {8, 2, 8, 4, 1, 1};
    case 40: return {20, 3, 4, 2, 5, 1};
    case 48: return {12, 3, 4, 4, 3, 1};
    case 64: return {8, 2, 8, 8, 1, 1};
    case 80: return {20, 3, 4, 4, 5, 1};
    case 96: return {24, 3, 8, 4, 3, 1};
    case 128: return {16, 2, 16, 8, 1, 1};
    case 160: return {20, 4, 4, 4, 2, 5};
    case 192: return {24, 3, 8, 8, 3, 1};
    case 256: return {16, 2, 16, 16, 1, 1};
    case 320: return {20, 4, 4, 4, 4, 5};
    case 384: return {24, 4, 8, 4, 4, 3};
    case 512: return {8, 3, 8, 8, 8, 1};
    case 1024: return {16, 3, 16, 16, 4, 1};
    default: return {0, 0, 1, 1, 1, 1};
  }
}
// true for the plan keys that have a plan
__host__ __device__ constexpr bool plan_ok(int n) { return plan_of(n).p > 0; }
__host__ __device__ constexpr int plan_p(int n) { return plan_of(n).p; }
__host__ __device__ constexpr int plan_stages(int n) { return plan_of(n).nst; }
__host__ __device__ constexpr int plan_radix(int n, int s) {
  return s == 0 ? plan_of(n).r0 : s == 1 ? plan_of(n).r1 : s == 2 ? plan_of(n).r2 : plan_of(n).r3;
}
// product of the radices of the stages before s
__host__ __device__ constexpr int plan_ns(int n, int s) {
  return s == 0 ? 1 : plan_ns(n, s - 1) * plan_radix(n, s - 1);
}
// Slot of input position t + TPL*q.  The first stage (radix R0, B0 = P/R0
// butterflies per thread) reads position t + TPL*(b + r*B0) in slot b*R0 + r;
// when R0 = P this is slot q.  (KEY: plan key, see kPlanFine.)
template <int KEY>
__device__ __forceinline__ constexpr int in_slot(int q) {
  constexpr int B0 = plan_p(KEY) / plan_radix(KEY, 0);
  return (q % B0) * plan_radix(KEY, 0) + q / B0;
}
// position index q held by output slot s of the last stage
template <int KEY>
__device__ __forceinline__ constexpr int out_q(int slot) {
  constexpr int P = plan_p(KEY);
  constexpr int R = plan_radix(KEY, plan_stages(KEY) - 1);
  return (slot / R) + (slot % R) * (P / R);
}

// ---------------------------------------------------------------------------
// In-register DFTs of size 2, 3, 4, 5, 8, 16 (natural order in and out).
// ---------------------------------------------------------------------------
template <typename T, int DIR>
__device__ __forceinline__ void dft2(cx<T>& a, cx<T>& b) {
  cx<T> t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <typename T, int DIR>
__device__ __forceinline__ void dft4(cx<T>& x0, cx<T>& x1, cx<T>& x2, cx<T>& x3) {
  cx<T> s02 = cadd(x0, x2), d02 = csub(x0, x2);
  cx<T> s13 = cadd(x1, x3), d13 = mul_dir_i<T, DIR>(csub(x1, x3));
  x0 = cadd(s02, s13);
  x2 = csub(s02, s13);
  x1 = cadd(d02, d13);
  x3 = csub(d02, d13);
}

template <typename T>
struct Consts {
  static constexpr T r2 = T(0.70710678118654752440084436210484903928483593768847);
  static constexpr T c8 = T(0.92387953251128675612818318939678828682241662586364);  // cos(pi/8)
  static constexpr T s8 = T(0.38268343236508977172845998403039886676134456248563);  // sin(pi/8)
};

// multiply by exp(DIR * 2 pi i * e / 16), e = 0..9 (compile time)
template <typename T, int DIR, int E>
__device__ __forceinline__ cx<T> w16(cx<T> a) {
  constexpr T r2 = Consts<T>::r2, c = Consts<T>::c8, s = Consts<T>::s8;
  constexpr int e = E % 16;
  if constexpr (e == 0) return a;
  else if constexpr (e == 4) return mul_dir_i<T, DIR>(a);
  else if constexpr (e == 8) return {-a.x, -a.y};
  else if constexpr (e == 12) return mul_dir_i<T, -DIR>(a);
  else {
    // angle = DIR * 2 pi e / 16 ; cos/sin from the octant table
    constexpr int ea = e;  // 1..15 except 4, 8, 12
    constexpr T cs[16] = {T(1), c, r2, s, T(0), -s, -r2, -c, T(-1), -c, -r2, -s, T(0), s, r2, c};
    constexpr T sn[16] = {T(0), s, r2, c, T(1), c, r2, s, T(0), -s, -r2, -c, T(-1), -c, -r2, -s};
    constexpr T wr = cs[ea];
    constexpr T wi = DIR < 0 ? -sn[ea] : sn[ea];
    return {a.x * wr - a.y * wi, a.x * wi + a.y * wr};
  }
}

template <typename T, int DIR>
__device__ __forceinline__ void dft8(cx<T>* v) {
  // even / odd split: E = DFT4(v0, v2, v4, v6), O = DFT4(v1, v3, v5, v7)
  dft4<T, DIR>(v[0], v[2], v[4], v[6]);
  dft4<T, DIR>(v[1], v[3], v[5], v[7]);
  cx<T> o1 = w16<T, DIR, 2>(v[3]);
  cx<T> o2 = w16<T, DIR, 4>(v[5]);
  cx<T> o3 = w16<T, DIR, 6>(v[7]);
  cx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6], o0 = v[1];
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, o1);
  v[5] = csub(e1, o1);
  v[2] = cadd(e2, o2);
  v[6] = csub(e2, o2);
  v[3] = cadd(e3, o3);
  v[7] = csub(e3, o3);
}

template <typename T, int DIR>
__device__ __forceinline__ void dft16(cx<T>* v) {
  // n = n1 + 4 n2, k = k2 + 4 k1
  dft4<T, DIR>(v[0], v[4], v[8], v[12]);
  dft4<T, DIR>(v[1], v[5], v[9], v[13]);
  dft4<T, DIR>(v[2], v[6], v[10], v[14]);
  dft4<T, DIR>(v[3], v[7], v[11], v[15]);
  // v[n1 + 4 k2] *= w16^(n1 k2)
  v[5] = w16<T, DIR, 1>(v[5]);
  v[9] = w16<T, DIR, 2>(v[9]);
  v[13] = w16<T, DIR, 3>(v[13]);
  v[6] = w16<T, DIR, 2>(v[6]);
  v[10] = w16<T, DIR, 4>(v[10]);
  v[14] = w16<T, DIR, 6>(v[14]);
  v[7] = w16<T, DIR, 3>(v[7]);
  v[11] = w16<T, DIR, 6>(v[11]);
  v[15] = w16<T, DIR, 9>(v[15]);
  // DFT4 over n1 for each k2; result index k2 + 4 k1 lands at slot 4 k2 + k1
  dft4<T, DIR>(v[0], v[1], v[2], v[3]);
  dft4<T, DIR>(v[4], v[5], v[6], v[7]);
  dft4<T, DIR>(v[8], v[9], v[10], v[11]);
  dft4<T, DIR>(v[12], v[13], v[14], v[15]);
  // transpose the 4x4 index grid back to natural order
  cx<T> t;
  t = v[1]; v[1] = v[4]; v[4] = t;
  t = v[2]; v[2] = v[8]; v[8] = t;
  t = v[3]; v[3] = v[12]; v[12] = t;
  t = v[6]; v[6] = v[9]; v[9] = t;
  t = v[7]; v[7] = v[13]; v[13] = t;
  t = v[11]; v[11] = v[14]; v[14] = t;
}

// DFT of size 3: with w = exp(DIR 2 pi i / 3), X1,2 = x0 - (x1 + x2)/2 +- i DIR (sqrt 3 / 2)(x1 - x2)
template <typename T, int DIR>
__device__ __forceinline__ void dft3(cx<T>* v) {
  constexpr T h3 = T(0.86602540378443864676372317075293618347140262690519);  // sqrt(3)/2
  const cx<T> s = cadd(v[1], v[2]);
  const cx<T> d = cscale(mul_dir_i<T, DIR>(csub(v[1], v[2])), h3);
  const cx<T> a{v[0].x - T(0.5) * s.x, v[0].y - T(0.5) * s.y};
  v[0] = cadd(v[0], s);
  v[1] = cadd(a, d);
  v[2] = csub(a, d);
}

// DFT of size 5 from the sums and differences of the mirrored inputs:
// X1,4 = A1 +- i DIR B1, X2,3 = A2 +- i DIR B2 with
// A1 = x0 + c1 (x1+x4) + c2 (x2+x3), A2 = x0 + c2 (x1+x4) + c1 (x2+x3),
// B1 = s1 (x1-x4) + s2 (x2-x3),     B2 = s2 (x1-x4) - s1 (x2-x3),
// c1,2 = cos(2 pi/5), cos(4 pi/5), s1,2 = sin(2 pi/5), sin(4 pi/5).
template <typename T, int DIR>
__device__ __forceinline__ void dft5(cx<T>* v) {
  constexpr T c1 = T(0.30901699437494742410229341718281905886436174199705);
  constexpr T c2 = T(-0.80901699437494742410229341718281905886436174199705);
  constexpr T s1 = T(0.95105651629515357211643933337938214340569863412575);
  constexpr T s2 = T(0.58778525229247312916870595463907276859765243764315);
  const cx<T> p1 = cadd(v[1], v[4]), m1 = csub(v[1], v[4]);
  const cx<T> p2 = cadd(v[2], v[3]), m2 = csub(v[2], v[3]);
  const cx<T> x0 = v[0];
  const cx<T> a1{x0.x + c1 * p1.x + c2 * p2.x, x0.y + c1 * p1.y + c2 * p2.y};
  const cx<T> a2{x0.x + c2 * p1.x + c1 * p2.x, x0.y + c2 * p1.y + c1 * p2.y};
  const cx<T> b1 = mul_dir_i<T, DIR>(cx<T>{s1 * m1.x + s2 * m2.x, s1 * m1.y + s2 * m2.y});
  const cx<T> b2 = mul_dir_i<T, DIR>(cx<T>{s2 * m1.x - s1 * m2.x, s2 * m1.y - s1 * m2.y});
  v[0] = cadd(x0, cadd(p1, p2));
  v[1] = cadd(a1, b1);
  v[4] = csub(a1, b1);
  v[2] = cadd(a2, b2);
  v[3] = csub(a2, b2);
}

template <typename T, int R, int DIR>
__device__ __forceinline__ void dft(cx<T>* v) {
  if constexpr (R == 1) {
  } else if constexpr (R == 2) dft2<T, DIR>(v[0], v[1]);
  else if constexpr (R == 3) dft3<T, DIR>(v);
  else if constexpr (R == 4) dft4<T, DIR>(v[0], v[1], v[2], v[3]);
  else if constexpr (R == 5) dft5<T, DIR>(v);
  else if constexpr (R == 8) dft8<T, DIR>(v);
  else dft16<T, DIR>(v);
}

// ---------------------------------------------------------------------------
// One Stockham radix-R stage on registers: twiddle then DFT.  Butterfly b of
// thread t is j = t + TPL*b; its inputs are positions j + r N/R; its outputs
// go to (j/Ns)*Ns*R + j%Ns + r*Ns.  tw: table exp(-2 pi i m / N), m < N,
// possibly a strided view (stride tws) of a longer table.
// ---------------------------------------------------------------------------
template <typename T, int KEY, int S, int DIR>
__device__ __forceinline__ void stage_compute(cx<T>* v, int t, const cx<T>* __restrict__ tw, int tws) {
  constexpr int N = plan_n(KEY);
  constexpr int P = plan_p(KEY), TPL = N / P, R = plan_radix(KEY, S), B = P / R, NS = plan_ns(KEY, S);
#pragma unroll
  for (int b = 0; b < B; ++b) {
    if constexpr (NS > 1) {
      // twiddles w^r, r = 1..R-1, from one table load: w^2 = w w, then
      // w^r = w^(r-2) w^2 (at most ~R/2 roundings per power)
      const int j = t + TPL * b;
      const int k = j % NS;
      const cx<T> w1 = tw[(k * (N / (NS * R))) * tws];
      const cx<T> w2 = cmul(w1, w1);
      cx<T> wr[R];
      wr[1] = w1;
#pragma unroll
      for (int r = 2; r < R; ++r) wr[r] = r == 2 ? w2 : cmul(wr[r - 2], w2);
#pragma unroll
      for (int r = 1; r < R; ++r) v[b * R + r] = DIR < 0 ? cmul(v[b * R + r], wr[r]) : cmulc(v[b * R + r], wr[r]);
    }
    dft<T, R, DIR>(v + b * R);
  }
}

// Output position of slot (b*R + r) of stage S for thread t.
template <int KEY, int S>
__device__ __forceinline__ int stage_out_pos(int t, int slot) {
  constexpr int N = plan_n(KEY);
  constexpr int P = plan_p(KEY), TPL = N / P, R = plan_radix(KEY, S), NS = plan_ns(KEY, S);
  const int b = slot / R, r = slot % R;
  const int j = t + TPL * b;
  return (j / NS) * NS * R + (j % NS) + r * NS;
}
// Input position of slot (b*R + r) of stage S for thread t.
template <int KEY, int S>
__device__ __forceinline__ int stage_in_pos(int t, int slot) {
  constexpr int N = plan_n(KEY);
  constexpr int P = plan_p(KEY), TPL = N / P, R = plan_radix(KEY, S);
  const int b = slot / R, r = slot % R;
  return t + TPL * b + r * (N / R);
}

// Exchange through LDS between stage S-1 and stage S, then compute stage S.
template <typename T, int KEY, int S, int DIR, class Lds>
__device__ __forceinline__ void next_stage(cx<T>* v, int t, Lds lds, const cx<T>* __restrict__ tw, int tws) {
  constexpr int P = plan_p(KEY);
  __syncthreads();
#pragma unroll
  for (int s = 0; s < P; ++s) lds(stage_out_pos<KEY, S - 1>(t, s)) = v[s];
  __syncthreads();
#pragma unroll
  for (int s = 0; s < P; ++s) v[s] = lds(stage_in_pos<KEY, S>(t, s));
  stage_compute<T, KEY, S, DIR>(v, t, tw, tws);
}

// Full line FFT on registers, exchanging through LDS between stages.
// Lds is an accessor with operator()(pos) -> cx<T>& for this thread's line.
// Starts with the input pattern (slot in_slot(q) <-> position t + TPL q) and
// ends with the output pattern (slot s <-> position t + TPL out_q(s)).
// Contains block barriers when there is more than one stage: every thread of
// the block must call it the same number of times.
template <typename T, int KEY, int DIR, class Lds>
__device__ __forceinline__ void line_fft(cx<T>* v, int t, Lds lds, const cx<T>* __restrict__ tw, int tws) {
  constexpr int NST = plan_stages(KEY);
  static_assert(plan_ok(KEY), "no FFT plan for this length");
  stage_compute<T, KEY, 0, DIR>(v, t, tw, tws);
  if constexpr (NST > 1) next_stage<T, KEY, 1, DIR>(v, t, lds, tw, tws);
  if constexpr (NST > 2) next_stage<T, KEY, 2, DIR>(v, t, lds, tw, tws);
  if constexpr (NST > 3) next_stage<T, KEY, 3, DIR>(v, t, lds, tw, tws);
}

}  // namespace llg
