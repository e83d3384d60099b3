// Axis passes of the spectral pipeline (DFTs along y or z, see
// pipeline_kernels.h).  Dispatches the runtime axis length to a kernel
// instantiation.
#include "llg_internal.h"
#include "pipeline_kernels.h"

namespace llg {

template <typename T, int N>
static hipError_t axis_n(const Ctx& c, int axis, int mode, const SymArgs& sym, cx<T>* spec, hipStream_t st) {
  constexpr int W = axis_w(int(sizeof(T)), N), TPL = N / plan_p(axis_plan_key(int(sizeof(T)), N));
  const unsigned gx = (unsigned)((c.geom.cs + W - 1) / W);
  const unsigned gy = (unsigned)(axis == 1 ? c.nz : c.ny);
  const cx<T>* tw;
  if constexpr (std::is_same<T, double>::value) tw = c.tw_d[axis];
  else tw = c.tw_f[axis];
  const double bytes = 2.0 * c.geom.cs * double(c.ny) * c.nz * 2 * sizeof(T);
  ProfScope ps(c.prof, st, mode == 0 ? KK_AXIS_FWD : (mode == 1 ? KK_AXIS_INV : KK_AXIS_FUSED), bytes);
  switch (mode) {
    case 0: hipLaunchKernelGGL((k_axis<T, N, 0>), dim3(gx, gy), dim3(W * TPL), 0, st, spec, c.geom, axis, sym, tw); break;
    case 1: hipLaunchKernelGGL((k_axis<T, N, 1>), dim3(gx, gy), dim3(W * TPL), 0, st, spec, c.geom, axis, sym, tw); break;
    default: hipLaunchKernelGGL((k_axis<T, N, 2>), dim3(gx, gy), dim3(W * TPL), 0, st, spec, c.geom, axis, sym, tw); break;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_axis(const Ctx& c, int axis, int mode, const SymArgs& sym, cx<T>* spec, hipStream_t st) {
  const int n = axis == 1 ? c.ny : c.nz;
  switch (n) {
#define LLG_CASE(v) \
  case v: return axis_n<T, v>(c, axis, mode, sym, spec, st);
    LLG_FOR_AXIS(LLG_CASE)
#undef LLG_CASE
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_axis<double>(const Ctx&, int, int, const SymArgs&, cx<double>*, hipStream_t);
template hipError_t launch_axis<float>(const Ctx&, int, int, const SymArgs&, cx<float>*, hipStream_t);

}  // namespace llg
