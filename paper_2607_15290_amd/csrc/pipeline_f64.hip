// float64 spectral pipelines.
#include "pipeline_run.h"

namespace llg {
template hipError_t run_pipeline<double, double, double>(const Ctx&, int, int, const SymArgs&, const NodalArgs&,
                                                         const PipeIO<double, double, double>&, hipStream_t,
                                                         const BasisDots*, double*);
}  // namespace llg
