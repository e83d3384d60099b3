// Delayed-CGS2 pass 2 fused into the x-forward pass of the next Arnoldi
// operator: host dispatch of k_xfwd_upd (pipeline_kernels.h) over the
// half-lengths and basis-column bounds it is instantiated for.
//
// The separate update pass streams w and the j + 1 basis directions, writes
// u_new, and the next operator's x-forward pass reads u_new straight back;
// here one pass does both, so the read of u_new (three or four float64
// planes, 24-32 bytes per node) and one launch per Arnoldi step disappear.
// Where the fused pass is slower it is not used:
//  * steps with j > 7: with more than 8 directions a thread holds one item's
//    loads at a time at two or three waves per SIMD, where the update pass
//    keeps 24 waves per CU in flight (measured slower at 128^3);
//  * grids whose x pass has fewer than 4096 blocks (one per LX lines): too
//    few to keep the update's loads in flight and to fill the last round of
//    blocks (512^2: 55 us against 22 + 12 us for the two passes; 128^3, 2048
//    blocks: slower as well), and grids needing more blocks than the partial
//    buffer has rows.
// At 256^3 (8192 float32 / 16384 float64 blocks) the fused pass takes 473 us
// where the two passes took 424 + 115 us.
#include "krylov.h"
#include "pipeline_kernels.h"

namespace llg {

#define LLG_FOR_NH_UPD(X) LLG_FOR_NH(X)
constexpr int kUpdMaxJ = 7;
constexpr unsigned kUpdMinBlocks = 4096;  // 16 per CU

namespace {

template <typename T, typename W, int NH, int PRO, int JB>
void upd_launch(const Ctx& c, const NodalArgs& na, const UpdFirst& ua, const W* w, const T* m, unsigned grid,
                hipStream_t st) {
  const cx<T>* tw;
  if constexpr (std::is_same<T, double>::value) tw = c.tw_d[0]; else tw = c.tw_f[0];
  hipLaunchKernelGGL((k_xfwd_upd<T, W, NH, PRO, JB>), dim3(grid), dim3(XCfg<T, NH>::NT), 0, st, ua, w, m,
                     reinterpret_cast<cx<T>*>(c.spec), c.geom, na, tw);
}

template <typename T, int NH>
unsigned upd_grid(const Ctx& c) {
  const long long lines = (long long)c.ny * c.nz;
  return (unsigned)((lines + XCfg<T, NH>::LX - 1) / XCfg<T, NH>::LX);
}

template <typename T, typename W, int NH, int PRO>
hipError_t upd_nh(const Ctx& c, const NodalArgs& na, const UpdFirst& ua, const W* w, const T* m, double* out,
                  hipStream_t st) {
  const unsigned grid = upd_grid<T, NH>(c);
  const long long lines = (long long)c.ny * c.nz;
  {
    // w, the j + 1 directions and the prologue's m read, u_new and the x
    // spectra written
    constexpr int nm = PRO == PRO_COPY3 ? 0 : 3;
    const double node_b = 4.0 * sizeof(W) + 32.0 * (ua.j + 2) + nm * sizeof(T);
    ProfScope ps(c.prof, st, KK_XFWD_UPD, double(c.ng) * node_b + double(c.geom.cs) * lines * 2 * sizeof(T));
    if (ua.j <= 1) upd_launch<T, W, NH, PRO, 1>(c, na, ua, w, m, grid, st);
    else if (ua.j <= 3) upd_launch<T, W, NH, PRO, 3>(c, na, ua, w, m, grid, st);
    else upd_launch<T, W, NH, PRO, 7>(c, na, ua, w, m, grid, st);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return reduce_partials_n(c, int(grid), ua.j + 2, out, st);
}

template <typename T, typename W, int NH>
hipError_t upd_pro(const Ctx& c, int pro, const NodalArgs& na, const UpdFirst& ua, const W* w, const T* m,
                   double* out, hipStream_t st) {
  if constexpr (std::is_same<T, float>::value) {
    switch (pro) {
      case PRO_COPY3: return upd_nh<T, W, NH, PRO_COPY3>(c, na, ua, w, m, out, st);
      case PRO_SMINUS: return upd_nh<T, W, NH, PRO_SMINUS>(c, na, ua, w, m, out, st);
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (pro) {
      case PRO_SMINUS: return upd_nh<T, W, NH, PRO_SMINUS>(c, na, ua, w, m, out, st);
      case PRO_M2T: return upd_nh<T, W, NH, PRO_M2T>(c, na, ua, w, m, out, st);
      default: return hipErrorInvalidValue;
    }
  }
}

template <typename T>
bool grid_fits(const Ctx& c, bool small_ok) {
  switch (c.geom.nh) {
#define LLG_CASE(n) \
  case n: return (small_ok || upd_grid<T, n>(c) >= kUpdMinBlocks) && upd_grid<T, n>(c) <= (unsigned)kRedBlocksMax;
    LLG_FOR_NH_UPD(LLG_CASE)
#undef LLG_CASE
    default: return false;
  }
}

template <typename T, typename W>
hipError_t run_t(const Ctx& c, int pro, const NodalArgs& na, const UpdFirst& ua, const W* w, const T* m,
                 double* out, hipStream_t st) {
  if (!xfwd_upd_supported(c, pro, std::is_same<T, float>::value, ua.j, 1)) return hipErrorInvalidValue;
  switch (c.geom.nh) {
#define LLG_CASE(n) \
  case n: return upd_pro<T, W, n>(c, pro, na, ua, w, m, out, st);
    LLG_FOR_NH_UPD(LLG_CASE)
#undef LLG_CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

bool xfwd_upd_supported(const Ctx& c, int pro, bool f32, int j, int policy) {
  if (policy < 0 || j < 0 || j > kUpdMaxJ) return false;
  if (f32 ? (pro != PRO_COPY3 && pro != PRO_SMINUS) : (pro != PRO_SMINUS && pro != PRO_M2T)) return false;
  return f32 ? grid_fits<float>(c, policy > 0) : grid_fits<double>(c, policy > 0);
}

hipError_t run_xfwd_upd(const Ctx& c, int pro, const NodalArgs& na, const UpdFirst& ua, const float* w,
                        const float* m32, double* out, hipStream_t st) {
  return run_t<float, float>(c, pro, na, ua, w, m32, out, st);
}
hipError_t run_xfwd_upd(const Ctx& c, int pro, const NodalArgs& na, const UpdFirst& ua, const double* w,
                        const double* m, double* out, hipStream_t st) {
  return run_t<double, double>(c, pro, na, ua, w, m, out, st);
}

}  // namespace llg
