// Host-side internals shared by the translation units of the library.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/llg.h"
#include "pipeline.h"

namespace llg {

// Per-thread last error message (llg_last_error).
void set_error(const std::string& msg);

#define LLG_HIP_CHECK(expr)                                                            \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) {                                                            \
      ::llg::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));             \
      return LLG_EHIP;                                                                 \
    }                                                                                  \
  } while (0)

// Number of blocks used by every streaming reduction (fixed per context so the
// reduction order, and hence every reduced value, is bitwise reproducible).
constexpr int kRedBlocksMax = 65536;  // partial buffer rows (large dot passes)
constexpr int kRedThreads = 256;
constexpr int kMaxDots = 64;
constexpr int kDcgsMaxCols = 32;  // delayed-CGS2 basis columns (restart <= 31)
constexpr int kDotsSlots = 5;     // kMaxDots-sized slots of Ctx::dots (see Ctx)
// Small grids, where an Arnoldi step's time is set by launches and round
// trips rather than bytes: grids of at most this many nodes launch the next
// step's operator before the host round trip of the current step (its work is
// short next to the round trip, and it is discarded when the cycle ends), and
// their update pass forms its own coefficients (one launch fewer per step).
constexpr long long kSpeculateMaxNodes = 1 << 20;

// Kernel kinds known to the event profiler.
enum KernelKind : int {
  KK_XFWD = 0, KK_AXIS_FWD, KK_AXIS_FUSED, KK_AXIS_INV, KK_XINV, KK_CGS_DOTS, KK_CGS_UPDATE_DOTS,
  KK_CGS_UPDATE_NORM, KK_REDUCE, KK_SCALE, KK_AXPBY, KK_LINCOMB, KK_CONVERT, KK_DOT2, KK_NODAL, KK_FIELD3,
  KK_XMID, KK_XINV_DOTS, KK_XFWD_UPD, KK_COUNT
};
const char* kernel_kind_name(int k);

struct Profiler;
// Bracket one launch with events when the context's profiler is on.
struct ProfScope {
  Profiler* p;
  hipStream_t st;
  int kind;
  double bytes;
  hipEvent_t a;
  ProfScope(Profiler* prof, hipStream_t s, int k, double b);
  ~ProfScope();
};

struct Ctx {
  Profiler* prof = nullptr;
  int nx = 0, ny = 0, nz = 0, dim = 0, device = 0;
  double Lx = 0, Ly = 0, Lz = 0;  // cell lengths (spacing L / n per axis)
  long long ng = 0;
  SpecGeom geom{};
  cx<double>* tw_d[3] = {nullptr, nullptr, nullptr};  // exp(-2 pi i m / n_axis)
  cx<float>* tw_f[3] = {nullptr, nullptr, nullptr};
  void* spec = nullptr;  // spectral scratch (complex double capacity)
  size_t spec_bytes = 0;
  double* partial = nullptr;  // kRedBlocksMax x kMaxDots reduction partials
  // Reduced values (device), kDotsSlots x kMaxDots doubles: dots (slot 0),
  // dots2 (CGS2 re-orthogonalization), scal (two slots of small scalars),
  // dots_b (the second Arnoldi pass-1 slot, for the step launched ahead).
  double* dots = nullptr;
  double* dots2 = nullptr;
  double* scal = nullptr;
  double* dots_b = nullptr;
  double* host = nullptr;     // pinned host mirror (4 * kMaxDots doubles)
  double* hmirror = nullptr;      // pinned, device-mapped host copy of the reduced values (same layout)
  double* hmirror_dev = nullptr;  // its device address
  hipEvent_t ev = nullptr;    // marks the end of an Arnoldi step's second pass
  double* tri = nullptr;      // delayed-CGS2 T^{-1} (kDcgsMaxCols^2, column-major) + kDcgsMaxCols coefficients
};

SymArgs sym_for(const Ctx& c, double a, double b, bool invert);

// gmres_solve on a given workspace (capi.cpp); the C entry points
// gmres_solve and gmres_solve_noalloc both run it.
llg_status gmres_solve_work(llg_ctx* ctx, const llg_params* prm, const double* m, const double* b, double* x,
                            const llg_solver_opts* opts, llg_solver_stats* stats, void* work, size_t work_bytes,
                            void* stream);
// Device of a context (-1 for null).
int ctx_device(const llg_ctx* ctx);

// Static workspace of gmres_solve_noalloc (noalloc.hip): its size, and the
// once-per-device lookup of its device address, run by llg_ctx_create with
// the context's device current.
constexpr size_t kScratchBytes = size_t(128) << 20;
void scratch_setup(int device);

// Launch one spectral pipeline (pipeline.h).  Defined per type combination
// in the pipeline_*.hip translation units.
// With bd (bd->nv > 0; fused M^{-1} A passes with a float64 output only) the
// last pass also leaves the Arnoldi inner products u_q . out in dots_out.
template <typename T, typename TIn, typename TOut>
hipError_t run_pipeline(const Ctx& c, int pro, int epi, const SymArgs& sym, const NodalArgs& na,
                        const PipeIO<T, TIn, TOut>& io, hipStream_t st, const BasisDots* bd = nullptr,
                        double* dots_out = nullptr);

// Precision-form inner operator (pipeline_f32.hip): z = M^{-1} v (float32,
// stored) and w = A z (float32, float64 result), the two pipelines joined by
// one fused x pass.  With bd (bd->nv > 0) the last pass also forms the
// Arnoldi inner products dots_out[q] = u_q . w, q < bd->nv (device).
// spec_ready: the x spectra of v are already in the spectral buffer
// (run_xfwd_upd with PRO_COPY3), so the apply's x-forward pass is skipped.
hipError_t run_apply_matvec(const Ctx& c, const SymArgs& sym_ap, const SymArgs& sym_mv, const NodalArgs& na,
                            const double* v, const float* m32, float* z, double* w, hipStream_t st,
                            const BasisDots* bd = nullptr, double* dots_out = nullptr, bool spec_ready = false);
// The same with a float32 w (the flexible cycle's operator output: the
// float32 matvec's values, read exactly by the Arnoldi pass).
hipError_t run_apply_matvec(const Ctx& c, const SymArgs& sym_ap, const SymArgs& sym_mv, const NodalArgs& na,
                            const double* v, const float* m32, float* z, float* w, hipStream_t st,
                            const BasisDots* bd = nullptr, double* dots_out = nullptr, bool spec_ready = false);

// Delayed-CGS2 pass 2 of step ua.j fused into the x-forward pass of the next
// operator (xfwd_upd.hip): k_xfwd_upd forms, stores and feeds u_new to the
// prologue `pro` (PRO_COPY3: the precision form's float32 apply; PRO_SMINUS:
// a fused M^{-1} A; PRO_M2T: the right-preconditioned adjoint), leaves the
// operator's x spectra in the spectral buffer for a pipeline started with
// PRO_NONE, and reduces [u_q . u_new (q <= j), u_new . u_new] into out.
// T = float: float32 passes with a float32 w and float32 m; T = double:
// float64 passes and w.  xfwd_upd_supported says whether to take it for this
// grid, prologue and ua.j under the policy of llg_solver_opts::fuse_update
// (-1 never, 0 large grids, 1 wherever an instantiation covers the grid).
bool xfwd_upd_supported(const Ctx& c, int pro, bool f32, int j, int policy);
hipError_t run_xfwd_upd(const Ctx& c, int pro, const NodalArgs& na, const UpdFirst& ua, const float* w,
                        const float* m32, double* out, hipStream_t st);
hipError_t run_xfwd_upd(const Ctx& c, int pro, const NodalArgs& na, const UpdFirst& ua, const double* w,
                        const double* m, double* out, hipStream_t st);

// Lower-order field pipeline (field.hip, float64): forward DFTs of three
// planes, the 3x3 multiplier of FieldArgs, inverse DFTs, then the x-inverse
// epilogue `epi` (EPI_STORE3, EPI_RHS, EPI_ADDF or EPI_JT; prologue PRO_COPY3).
hipError_t run_field(const Ctx& c, const FieldArgs& fa, int epi, const NodalArgs& na,
                     const PipeIO<double, double, double>& io, hipStream_t st);

// Axis passes (axis.hip).
template <typename T>
hipError_t launch_axis(const Ctx& c, int axis, int mode, const SymArgs& sym, cx<T>* spec, hipStream_t st);

}  // namespace llg
