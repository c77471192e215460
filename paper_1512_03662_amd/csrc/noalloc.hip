// jfnk_cfl_dt_noalloc: the CFL time step without a context and without any allocation, for
// callers that cannot allocate device memory (code under HIP graph capture, tight serving
// loops).  The max-reduction's block partials live in the file-scope device array below;
// its device address is looked up once per device and passed to the kernels.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/jfnk.h"
#include "kernels.hpp"

namespace jfnk {
std::string grid_of_problem(const jfnk_problem* p, Grid* G);
void set_context_free_error(const std::string& msg);
}  // namespace jfnk

using namespace jfnk;

// one partial per reduction block (at most kRedBlocks of them; 8 KiB on every device)
constexpr int kScratchDoubles = kRedBlocks;
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on device dev (current), looked up on the first call there
hipError_t scratch_on(int dev, double** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

int fail(int code, const std::string& msg) {
  set_context_free_error(msg);
  return code;
}

}  // namespace

extern "C" int jfnk_cfl_dt_noalloc(const jfnk_problem* prob, const double* X, double cfl, double* dt_out,
                                   void* hip_stream) {
  if (!X || !dt_out) return fail(JFNK_E_INVALID, "null array");
  if (!(cfl > 0.0 && cfl < HUGE_VAL)) return fail(JFNK_E_INVALID, "cfl must be positive and finite");
  Grid G;
  const std::string why = grid_of_problem(prob, &G);
  if (!why.empty()) return fail(JFNK_E_INVALID, why);
  const int nb = cfl_partials(G);
  if (nb > kScratchDoubles)
    return fail(JFNK_E_INVALID, "the reduction needs more partials than the static scratch holds");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(JFNK_E_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(JFNK_E_DEVICE, "device ordinal beyond the scratch table");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if (s) {
    hipDevice_t sd = -1;
    e = hipStreamGetDevice(s, &sd);
    if (e != hipSuccess) return fail(JFNK_E_DEVICE, std::string("hipStreamGetDevice: ") + hipGetErrorString(e));
    if (sd != dev) return fail(JFNK_E_INVALID, "the stream's device must be the current device");
  }
  double* part = nullptr;
  e = scratch_on(dev, &part);
  if (e != hipSuccess) return fail(JFNK_E_DEVICE, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
  double hmin = G.dx[0];
  for (int d = 1; d < G.nd; ++d) hmin = (G.dx[d] < hmin) ? G.dx[d] : hmin;
  launch_cfl_dt_dev(G, X, cfl * hmin, part, dt_out, s);
  e = hipGetLastError();
  if (e != hipSuccess) return fail(JFNK_E_DEVICE, std::string("launch: ") + hipGetErrorString(e));
  return JFNK_OK;
}
