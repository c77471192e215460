// Measurement hook: when enabled, every launch of an instrumented kernel is bracketed by HIP
// events on the stream it is launched on, and the algorithmic bytes that launch must move
// (each field read or written once) are accumulated per kernel family.  Process-wide; used
// by the benchmark to time the dominant kernel inside the solver's own launch sequence.
#include <hip/hip_runtime.h>

#include <vector>

#include "probe.hpp"

namespace jfnk {

namespace {
struct Fam {
  std::vector<hipEvent_t> starts, stops;
  double ms = 0.0;
  long long launches = 0;
  double bytes = 0.0;
};
bool g_enabled = false;
Fam g_fam[KF_COUNT];
std::vector<hipEvent_t> g_pool;

hipEvent_t take() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void drain(Fam& f) {
  for (size_t i = 0; i < f.starts.size(); ++i) {
    float ms = 0.0f;
    if (hipEventSynchronize(f.stops[i]) == hipSuccess &&
        hipEventElapsedTime(&ms, f.starts[i], f.stops[i]) == hipSuccess)
      f.ms += ms;
    g_pool.push_back(f.starts[i]);
    g_pool.push_back(f.stops[i]);
  }
  f.starts.clear();
  f.stops.clear();
}
}  // namespace

const char* const kFamNames[KF_COUNT] = {
    "residual_value", "residual_fd_jv", "residual_exact_jv", "vjp_stage_a", "vjp_stage_b",
    "vjp_fold", "gs_dots", "gs_update", "lincomb",
    "mg_presmooth", "mg_prolong_smooth1", "mg_smooth2", "mg_coarse", "cg_apply_dot",
    "cg_update", "cg_pupdate", "dot", "pbp_in", "pbp_out", "scaled_norm", "mg_restrict_resid",
    "mg_down", "mg_up", "fd_shift"};

bool probe_events(int fam, double bytes, hipEvent_t* start, hipEvent_t* stop) {
  *start = nullptr;
  *stop = nullptr;
  if (!g_enabled || fam < 0 || fam >= KF_COUNT) return false;
  Fam& f = g_fam[fam];
  if (f.starts.size() >= 4096) drain(f);
  hipEvent_t a = take(), b = take();
  if (!a || !b) {
    if (a) g_pool.push_back(a);
    if (b) g_pool.push_back(b);
    return false;
  }
  f.starts.push_back(a);
  f.stops.push_back(b);
  f.bytes += bytes;
  f.launches += 1;
  *start = a;
  *stop = b;
  return true;
}

void probe_enable(bool on) {
  for (auto& f : g_fam) {
    drain(f);
    f = Fam();
  }
  g_enabled = on;
}

bool probe_read(int fam, double* ms, long long* launches, double* bytes) {
  if (fam < 0 || fam >= KF_COUNT) return false;
  drain(g_fam[fam]);
  *ms = g_fam[fam].ms;
  *launches = g_fam[fam].launches;
  *bytes = g_fam[fam].bytes;
  return true;
}

}  // namespace jfnk
