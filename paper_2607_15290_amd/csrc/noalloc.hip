// gmres_solve without a caller workspace and without any device allocation.
//
// For callers that cannot allocate device memory (a serving loop or harness
// that forbids hipMalloc): the Krylov workspace of gmres_solve lives in one
// file-scope device array, `scratch`, of kScratchBytes.  The HIP runtime
// places one copy of the array on every GPU the library runs on, at its own
// address, and keeps it until the process ends.
//
// The array's name is only a host-side stand-in in host code.  Its device
// address is looked up once per device, with that device current, when the
// first context on the device is created (llg_ctx_create calls
// scratch_setup), and from then on host code uses only that address.
//
// Every call on a GPU uses that GPU's one array: calls that overlap on one
// GPU (two host threads, or two streams whose work is in flight together)
// race on it.  Nothing in the array has to start at zero: every word a solve
// reads it has written earlier in the same call (basis vectors, residual,
// float32 copies), so the contents left by an earlier call are never used.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "llg_internal.h"

namespace llg {

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxScratchDevices] = {};
hipError_t g_err[kMaxScratchDevices] = {};
bool g_done[kMaxScratchDevices] = {};
}  // namespace

// Look up this device's copy of the array (the calling thread has `device`
// current).  A failure is kept and reported by the entry point.
void scratch_setup(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_done[device]) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  g_err[device] = e;
  g_ptr[device] = e == hipSuccess ? p : nullptr;
  g_done[device] = true;
}

}  // namespace llg

extern "C" llg_status gmres_solve_noalloc(llg_ctx* ctx, const llg_params* prm, const double* m, const double* b,
                                          double* x, const llg_solver_opts* opts, llg_solver_stats* stats,
                                          void* stream) {
  using namespace llg;
  if (!ctx || !opts) {
    set_error("gmres_solve_noalloc: null argument");
    return LLG_EARG;
  }
  const int dev = ctx_device(ctx);
  void* ptr = nullptr;
  hipError_t e = hipErrorInvalidDevice;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (dev >= 0 && dev < kMaxScratchDevices && g_done[dev]) {
      ptr = g_ptr[dev];
      e = g_err[dev];
    }
  }
  if (!ptr) {
    set_error(std::string("gmres_solve_noalloc: device address of the static workspace unavailable: ") +
              hipGetErrorString(e));
    return LLG_EHIP;
  }
  const size_t need = llg_workspace_bytes(ctx, opts->restart, opts->prec);
  if (need == 0) return gmres_solve_work(ctx, prm, m, b, x, opts, stats, ptr, 0, stream);
  if (need > kScratchBytes) {
    set_error("gmres_solve_noalloc: this grid and restart length need " + std::to_string(need) +
              " bytes of workspace, more than the static workspace of " + std::to_string(kScratchBytes) +
              " bytes; use gmres_solve with a caller workspace");
    return LLG_ENOMEM;
  }
  return gmres_solve_work(ctx, prm, m, b, x, opts, stats, ptr, kScratchBytes, stream);
}
