// Event profiler of the context: pairs of HIP events around kernel launches,
// aggregated per kernel kind with the launches' algorithmic bytes.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "llg_internal.h"

namespace llg {

struct Profiler {
  bool on = false;
  bool sel[KK_COUNT];  // kinds that are recorded while on
  Profiler() {
    for (bool& b : sel) b = true;
  }
  struct Rec {
    int kind;
    hipEvent_t a, b;
    double bytes;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  hipEvent_t take() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void recycle() {
    for (auto& r : recs) {
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    recs.clear();
  }
  ~Profiler() {
    recycle();
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

static const char* kNames[KK_COUNT] = {"xfwd",      "axis_fwd",          "axis_fused",        "axis_inv",
                                       "xinv",      "cgs_dots",          "cgs_update_dots",   "cgs_update_norm",
                                       "reduce",    "scale",             "axpby",             "lincomb",
                                       "convert",   "dot2",              "nodal",             "field3",
                                       "xmid",      "xinv_dots",         "xfwd_upd"};

const char* kernel_kind_name(int k) { return (k >= 0 && k < KK_COUNT) ? kNames[k] : "?"; }

ProfScope::ProfScope(Profiler* prof, hipStream_t s, int k, double b) : p(prof), st(s), kind(k), bytes(b), a(nullptr) {
  if (p && p->on && p->sel[k]) {
    a = p->take();
    if (a) (void)hipEventRecord(a, st);
  }
}

ProfScope::~ProfScope() {
  if (p && p->on && a) {
    hipEvent_t b = p->take();
    if (b) {
      (void)hipEventRecord(b, st);
      p->recs.push_back({kind, a, b, bytes});
    }
  }
}

Profiler* profiler_new() { return new Profiler(); }
void profiler_delete(Profiler* p) { delete p; }
void profiler_enable(Profiler* p, bool on) {
  if (on) p->recycle();
  p->on = on;
}

// Select the kinds to record from a comma-separated list of names (null or
// empty: all kinds).  Returns false on an unknown name (selection unchanged).
bool profiler_select(Profiler* p, const char* kinds) {
  bool want[KK_COUNT];
  const bool all = kinds == nullptr || kinds[0] == 0;
  for (bool& b : want) b = all;
  if (!all) {
    const char* q = kinds;
    while (*q) {
      const char* e = q;
      while (*e && *e != ',') ++e;
      const size_t len = size_t(e - q);
      int found = -1;
      for (int k = 0; k < KK_COUNT; ++k)
        if (std::strlen(kNames[k]) == len && std::strncmp(kNames[k], q, len) == 0) found = k;
      if (found < 0) return false;
      want[found] = true;
      q = *e ? e + 1 : e;
    }
  }
  for (int k = 0; k < KK_COUNT; ++k) p->sel[k] = want[k];
  return true;
}

int profiler_read(Profiler* p, llg_kernel_profile* out, int max_entries) {
  int launches[KK_COUNT] = {0};
  double ms[KK_COUNT] = {0}, bytes[KK_COUNT] = {0};
  for (auto& r : p->recs) {
    if (hipEventSynchronize(r.b) != hipSuccess) return -1;
    float t = 0;
    if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return -1;
    launches[r.kind]++;
    ms[r.kind] += t;
    bytes[r.kind] += r.bytes;
  }
  int n = 0;
  for (int k = 0; k < KK_COUNT; ++k) {
    if (!launches[k]) continue;
    if (out && n < max_entries) out[n] = {kNames[k], launches[k], ms[k], bytes[k]};
    n++;
  }
  return n;
}

}  // namespace llg
