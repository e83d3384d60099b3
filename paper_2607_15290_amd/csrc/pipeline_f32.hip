// float32 spectral pipelines: all-float32 operators and the mixed operators
// of the precision form (float32 apply of a float64 Krylov vector, float32
// matvec producing a float64 Krylov vector, float32 apply and fused M^{-1} A
// between float64 Krylov vectors).
#include "pipeline_run.h"

namespace llg {
template hipError_t run_pipeline<float, float, float>(const Ctx&, int, int, const SymArgs&, const NodalArgs&,
                                                      const PipeIO<float, float, float>&, hipStream_t);
template hipError_t run_pipeline<float, double, float>(const Ctx&, int, int, const SymArgs&, const NodalArgs&,
                                                       const PipeIO<float, double, float>&, hipStream_t);
template hipError_t run_pipeline<float, float, double>(const Ctx&, int, int, const SymArgs&, const NodalArgs&,
                                                       const PipeIO<float, float, double>&, hipStream_t);
template hipError_t run_pipeline<float, double, double>(const Ctx&, int, int, const SymArgs&, const NodalArgs&,
                                                        const PipeIO<float, double, double>&, hipStream_t);
}  // namespace llg
