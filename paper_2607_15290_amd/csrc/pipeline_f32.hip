// float32 spectral pipelines: all-float32 operators and the mixed operators
// of the precision form (float32 apply of a float64 Krylov vector, float32
// matvec producing a float64 Krylov vector, float32 apply and fused M^{-1} A
// between float64 Krylov vectors).
#include "pipeline_run.h"

namespace llg {
template hipError_t run_pipeline<float, float, float>(const Ctx&, int, int, const SymArgs&, const NodalArgs&,
                                                      const PipeIO<float, float, float>&, hipStream_t,
                                                         const BasisDots*, double*);
template hipError_t run_pipeline<float, double, float>(const Ctx&, int, int, const SymArgs&, const NodalArgs&,
                                                       const PipeIO<float, double, float>&, hipStream_t,
                                                         const BasisDots*, double*);
template hipError_t run_pipeline<float, float, double>(const Ctx&, int, int, const SymArgs&, const NodalArgs&,
                                                       const PipeIO<float, float, double>&, hipStream_t,
                                                         const BasisDots*, double*);
template hipError_t run_pipeline<float, double, double>(const Ctx&, int, int, const SymArgs&, const NodalArgs&,
                                                        const PipeIO<float, double, double>&, hipStream_t,
                                                         const BasisDots*, double*);

template <typename TW>
static hipError_t apply_matvec_t(const Ctx& c, const SymArgs& sym_ap, const SymArgs& sym_mv, const NodalArgs& na,
                                 const double* v, const float* m32, float* z, TW* w, hipStream_t st,
                                 const BasisDots* bd, double* dots_out, bool spec_ready) {
  switch (c.geom.nh) {
#define LLG_CASE(n) \
  case n: return run_apply_matvec_nh<n, TW>(c, sym_ap, sym_mv, na, v, m32, z, w, bd, dots_out, spec_ready, st);
    LLG_FOR_NH(LLG_CASE)
#undef LLG_CASE
    default: return hipErrorInvalidValue;
  }
}
hipError_t run_apply_matvec(const Ctx& c, const SymArgs& sym_ap, const SymArgs& sym_mv, const NodalArgs& na,
                            const double* v, const float* m32, float* z, double* w, hipStream_t st,
                            const BasisDots* bd, double* dots_out, bool spec_ready) {
  return apply_matvec_t(c, sym_ap, sym_mv, na, v, m32, z, w, st, bd, dots_out, spec_ready);
}
hipError_t run_apply_matvec(const Ctx& c, const SymArgs& sym_ap, const SymArgs& sym_mv, const NodalArgs& na,
                            const double* v, const float* m32, float* z, float* w, hipStream_t st,
                            const BasisDots* bd, double* dots_out, bool spec_ready) {
  return apply_matvec_t(c, sym_ap, sym_mv, na, v, m32, z, w, st, bd, dots_out, spec_ready);
}
}  // namespace llg
