// Host dispatch of one spectral pipeline: x-forward, axis passes, x-inverse.
// Included by the per-precision translation units, which instantiate
// run_pipeline for the type combinations they need.
#pragma once
#include "llg_internal.h"
#include "krylov.h"
#include "pipeline_kernels.h"

namespace llg {

// Which (prologue, epilogue) modes exist for a type combination.  The mixed
// combinations serve only the precision form: float32 apply reading float64
// Krylov vectors (and the fused M^{-1} A of the left variant, whose float32
// output goes to the Arnoldi pass), float32 matvec writing float64 Krylov
// vectors, and float32 apply / fused M^{-1} A between float64 Krylov vectors.
template <typename T, typename TIn, typename TOut>
constexpr bool has_pro(int pro) {
  if (pro == PRO_NONE) return true;
  if constexpr (std::is_same<T, TIn>::value && std::is_same<T, TOut>::value) return true;
  else if constexpr (std::is_same<TIn, double>::value) return pro == PRO_COPY3 || pro == PRO_SMINUS;
  else return pro == PRO_COPY3;
}
template <typename T, typename TIn, typename TOut>
constexpr bool has_epi(int epi) {
  if constexpr (std::is_same<T, TIn>::value && std::is_same<T, TOut>::value)
    return (epi != EPI_ENERGY && epi != EPI_JT_RIGHT) || std::is_same<T, double>::value;
  else if constexpr (std::is_same<TIn, double>::value) return epi == EPI_APPLY || epi == EPI_FUSED;
  else return epi == EPI_MATVEC;
}

template <typename T, typename TIn, typename TOut, int NH, int PRO>
void launch_xfwd(const Ctx& c, const NodalArgs& na, const PipeIO<T, TIn, TOut>& io, hipStream_t st) {
  if constexpr (has_pro<T, TIn, TOut>(PRO)) {
    using C = XCfg<T, NH>;
    const long long lines = (long long)c.ny * c.nz;
    const unsigned grid = (unsigned)((lines + C::LX - 1) / C::LX);
    const cx<T>* tw;
    if constexpr (std::is_same<T, double>::value) tw = c.tw_d[0]; else tw = c.tw_f[0];
    const double in_b = PRO == PRO_COPY3 ? 3.0 * sizeof(TIn) : 4.0 * sizeof(TIn) + 3.0 * sizeof(T);
    ProfScope ps(c.prof, st, KK_XFWD, double(c.ng) * in_b + double(c.geom.cs) * lines * 2 * sizeof(T));
    hipLaunchKernelGGL((k_xfwd<T, TIn, NH, PRO>), dim3(grid), dim3(C::NT), 0, st, io.in, io.m,
                       reinterpret_cast<cx<T>*>(c.spec), c.geom, na, tw);
  }
}

// Per-node bytes of an x-inverse epilogue's plane reads and writes.
template <typename T, typename TIn, typename TOut, int EPI>
double xinv_node_bytes(const NodalArgs& na, const PipeIO<T, TIn, TOut>& io) {
  double node_b = 0;
  if (EPI == EPI_STORE3) node_b = 3.0 * sizeof(TOut);
  else if (EPI == EPI_RHS) node_b = 4.0 * sizeof(TOut) + (na.hfield ? 24.0 : 0.0) + (io.out_f ? 3.0 * sizeof(T) : 0.0);
  else if (EPI == EPI_APPLY) node_b = 1.0 * sizeof(TIn) + 3.0 * sizeof(T) + 4.0 * sizeof(TOut);
  else if (EPI == EPI_APPLY_SYM) node_b = 1.0 * sizeof(TIn) + 4.0 * sizeof(TOut);
  else if (EPI == EPI_JT || EPI == EPI_JT_RIGHT) node_b = 4.0 * sizeof(TIn) + 7.0 * sizeof(T) + 4.0 * sizeof(TOut);
  else if (EPI == EPI_ADDF) node_b = 3.0 * sizeof(T) + 4.0 * sizeof(TOut);
  else if (EPI == EPI_ENERGY) node_b = 3.0 * sizeof(T) + (na.hfield ? 24.0 : 0.0);
  else node_b = 4.0 * sizeof(TIn) + 3.0 * sizeof(T) + 4.0 * sizeof(TOut);
  if (io.rhs) node_b += 4.0 * sizeof(TOut);
  return node_b;
}

template <typename T, typename TIn, typename TOut, int NH, int EPI>
void launch_xinv(const Ctx& c, const NodalArgs& na, const PipeIO<T, TIn, TOut>& io, hipStream_t st) {
  if constexpr (has_epi<T, TIn, TOut>(EPI)) {
    using C = XCfg<T, NH>;
    const long long lines = (long long)c.ny * c.nz;
    const unsigned grid = (unsigned)((lines + C::LX - 1) / C::LX);
    const cx<T>* tw;
    if constexpr (std::is_same<T, double>::value) tw = c.tw_d[0]; else tw = c.tw_f[0];
    const double node_b = xinv_node_bytes<T, TIn, TOut, EPI>(na, io);
    ProfScope ps(c.prof, st, KK_XINV, double(c.ng) * node_b + double(c.geom.cs) * lines * 2 * sizeof(T));
    hipLaunchKernelGGL((k_xinv<T, TIn, TOut, NH, EPI>), dim3(grid), dim3(C::NT), 0, st, io,
                       reinterpret_cast<const cx<T>*>(c.spec), c.geom, na, tw, BasisDots{});
  }
}

// x-inverse pass that also forms the Arnoldi inner products of its float64
// output (dots_out[q] = u_q . out, q < bd.nv, on the device).
template <typename T, typename TIn, typename TOut, int NH, int EPI>
hipError_t launch_xinv_dots(const Ctx& c, const NodalArgs& na, const PipeIO<T, TIn, TOut>& io, const BasisDots& bd,
                            double* dots_out, hipStream_t st) {
  using C = XCfg<T, NH>;
  if (bd.nv < 1 || bd.nv > kBasisDotsMax || io.rhs) return hipErrorInvalidValue;
  const long long lines = (long long)c.ny * c.nz;
  const unsigned grid = (unsigned)((lines + C::LX - 1) / C::LX);
  if (bd.defer_nb) *bd.defer_nb = 0;
  if (grid > (unsigned)kRedBlocksMax) {
    // more blocks than partial rows (the largest grids in float64): plain
    // pass, then the separate inner-product pass over the output
    launch_xinv<T, TIn, TOut, NH, EPI>(c, na, io, st);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return dcgs_dots(c, bd.u0, bd.U1, bd.ld, bd.nv - 1, io.out, 4 * c.ng, dots_out, st);
  }
  const cx<T>* tw;
  if constexpr (std::is_same<T, double>::value) tw = c.tw_d[0]; else tw = c.tw_f[0];
  // defer only over few blocks: every block of the update pass sums all of
  // them (at 64 blocks one launch fewer per step gained 4%; at 256 the sums
  // cost more than the launch)
  const bool defer = bd.defer && grid <= unsigned(kDeferMaxBlocks);
  BasisDots kd = bd;
  kd.partial = defer ? bd.defer : c.partial;
  {
    const double node_b = xinv_node_bytes<T, TIn, TOut, EPI>(na, io) + 4.0 * 8 * bd.nv;
    ProfScope ps(c.prof, st, KK_XINV_DOTS, double(c.ng) * node_b + double(c.geom.cs) * lines * 2 * sizeof(T));
    hipLaunchKernelGGL((k_xinv<T, TIn, TOut, NH, EPI, true>), dim3(grid), dim3(C::NT), 0, st, io,
                       reinterpret_cast<const cx<T>*>(c.spec), c.geom, na, tw, kd);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (defer) {
    *bd.defer_nb = int(grid);
    return hipSuccess;
  }
  return reduce_partials_n(c, int(grid), bd.nv, dots_out, st);
}

template <typename T, typename TIn, typename TOut, int NH>
hipError_t run_nh(const Ctx& c, int pro, int epi, const SymArgs& sym, const NodalArgs& na,
                  const PipeIO<T, TIn, TOut>& io, hipStream_t st, const BasisDots* bd, double* dots_out) {
  // a mode without an instantiation for this type combination is an error,
  // never a silently skipped pass
  if (!has_pro<T, TIn, TOut>(pro) || !has_epi<T, TIn, TOut>(epi)) return hipErrorInvalidValue;
  switch (pro) {
    case PRO_COPY3: launch_xfwd<T, TIn, TOut, NH, PRO_COPY3>(c, na, io, st); break;
    case PRO_SMINUS: launch_xfwd<T, TIn, TOut, NH, PRO_SMINUS>(c, na, io, st); break;
    case PRO_M2T: launch_xfwd<T, TIn, TOut, NH, PRO_M2T>(c, na, io, st); break;
    case PRO_NONE: break;  // x spectra already in place (k_xfwd_upd)
    default: return hipErrorInvalidValue;
  }
  cx<T>* spec = reinterpret_cast<cx<T>*>(c.spec);
  hipError_t e;
  if (c.dim == 2) {
    if ((e = launch_axis<T>(c, 1, 2, sym, spec, st)) != hipSuccess) return e;
  } else {
    if ((e = launch_axis<T>(c, 1, 0, sym, spec, st)) != hipSuccess) return e;
    if ((e = launch_axis<T>(c, 2, 2, sym, spec, st)) != hipSuccess) return e;
    if ((e = launch_axis<T>(c, 1, 1, sym, spec, st)) != hipSuccess) return e;
  }
  if (bd && bd->nv > 0) {
    if (bd->out) dots_out = bd->out;
    // the Arnoldi inner products ride on the fused preconditioned passes only
    if constexpr (has_epi<T, TIn, TOut>(EPI_FUSED)) {
      if (epi == EPI_FUSED) return launch_xinv_dots<T, TIn, TOut, NH, EPI_FUSED>(c, na, io, *bd, dots_out, st);
      if constexpr (has_epi<T, TIn, TOut>(EPI_JT_RIGHT)) {
        if (epi == EPI_JT_RIGHT)
          return launch_xinv_dots<T, TIn, TOut, NH, EPI_JT_RIGHT>(c, na, io, *bd, dots_out, st);
      }
      return hipErrorInvalidValue;
    } else {
      return hipErrorInvalidValue;
    }
  }
  switch (epi) {
    case EPI_STORE3: launch_xinv<T, TIn, TOut, NH, EPI_STORE3>(c, na, io, st); break;
    case EPI_APPLY: launch_xinv<T, TIn, TOut, NH, EPI_APPLY>(c, na, io, st); break;
    case EPI_APPLY_T: launch_xinv<T, TIn, TOut, NH, EPI_APPLY_T>(c, na, io, st); break;
    case EPI_MATVEC: launch_xinv<T, TIn, TOut, NH, EPI_MATVEC>(c, na, io, st); break;
    case EPI_MATVEC_T: launch_xinv<T, TIn, TOut, NH, EPI_MATVEC_T>(c, na, io, st); break;
    case EPI_FUSED: launch_xinv<T, TIn, TOut, NH, EPI_FUSED>(c, na, io, st); break;
    case EPI_RHS: launch_xinv<T, TIn, TOut, NH, EPI_RHS>(c, na, io, st); break;
    case EPI_JT: launch_xinv<T, TIn, TOut, NH, EPI_JT>(c, na, io, st); break;
    case EPI_APPLY_SYM: launch_xinv<T, TIn, TOut, NH, EPI_APPLY_SYM>(c, na, io, st); break;
    case EPI_FUSED_SYM: launch_xinv<T, TIn, TOut, NH, EPI_FUSED_SYM>(c, na, io, st); break;
    case EPI_ENERGY: launch_xinv<T, TIn, TOut, NH, EPI_ENERGY>(c, na, io, st); break;
    case EPI_JT_RIGHT: launch_xinv<T, TIn, TOut, NH, EPI_JT_RIGHT>(c, na, io, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Axis passes of one pipeline on the spectral buffer: y forward, z fused,
// y inverse (3D) or y fused (2D).
template <typename T>
hipError_t run_axes(const Ctx& c, const SymArgs& sym, hipStream_t st) {
  cx<T>* spec = reinterpret_cast<cx<T>*>(c.spec);
  hipError_t e;
  if (c.dim == 2) return launch_axis<T>(c, 1, 2, sym, spec, st);
  if ((e = launch_axis<T>(c, 1, 0, sym, spec, st)) != hipSuccess) return e;
  if ((e = launch_axis<T>(c, 2, 2, sym, spec, st)) != hipSuccess) return e;
  return launch_axis<T>(c, 1, 1, sym, spec, st);
}

// One inner iteration's operator of the precision form: z = M^{-1} v in
// float32 (z kept as the flexible basis vector) and w = A z in float32 with a
// float64 result; the junction of the two pipelines is the fused k_xmid pass.
// The matvec's output w is float64 (a Krylov vector) or float32 (the Arnoldi
// operator output of the precision form, whose float32 values convert to
// float64 exactly when the Arnoldi pass reads them).  spec_ready: the apply's
// x-forward pass already ran (k_xfwd_upd with PRO_COPY3).
template <int NH, typename TW>
hipError_t run_apply_matvec_nh(const Ctx& c, const SymArgs& sym_ap, const SymArgs& sym_mv, const NodalArgs& na,
                               const double* v, const float* m32, float* z, TW* w, const BasisDots* bd,
                               double* dots_out, bool spec_ready, hipStream_t st) {
  using C = XCfg<float, NH>;
  PipeIO<float, double, float> io_ap{v, m32, z, c.ng, nullptr, nullptr};
  PipeIO<float, float, TW> io_mv{z, m32, w, c.ng, nullptr, nullptr};
  if (!spec_ready) launch_xfwd<float, double, float, NH, PRO_COPY3>(c, na, io_ap, st);
  hipError_t e;
  if ((e = run_axes<float>(c, sym_ap, st)) != hipSuccess) return e;
  {
    const long long lines = (long long)c.ny * c.nz;
    const unsigned grid = (unsigned)((lines + C::LX - 1) / C::LX);
    const double bytes = 2.0 * double(c.geom.cs) * lines * sizeof(cx<float>) + double(c.ng) * (8.0 + 12.0 + 16.0);
    ProfScope ps(c.prof, st, KK_XMID, bytes);
    hipLaunchKernelGGL((k_xmid<NH>), dim3(grid), dim3(C::NT), 0, st, io_ap, reinterpret_cast<cx<float>*>(c.spec),
                       c.geom, na, c.tw_f[0]);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if ((e = run_axes<float>(c, sym_mv, st)) != hipSuccess) return e;
  if (!bd || bd->nv == 0) {
    launch_xinv<float, float, TW, NH, EPI_MATVEC>(c, na, io_mv, st);
    return hipGetLastError();
  }
  if (bd->out) dots_out = bd->out;
  // matvec with the Arnoldi inner products of w (out[q] = u_q . w, q < nv)
  return launch_xinv_dots<float, float, TW, NH, EPI_MATVEC>(c, na, io_mv, *bd, dots_out, st);
}

template <typename T, typename TIn, typename TOut>
hipError_t run_pipeline(const Ctx& c, int pro, int epi, const SymArgs& sym, const NodalArgs& na,
                        const PipeIO<T, TIn, TOut>& io, hipStream_t st, const BasisDots* bd, double* dots_out) {
  switch (c.geom.nh) {
#define LLG_CASE(n) \
  case n: return run_nh<T, TIn, TOut, n>(c, pro, epi, sym, na, io, st, bd, dots_out);
    LLG_FOR_NH(LLG_CASE)
#undef LLG_CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace llg
