// Per-kernel timing hook (see probe.hip).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

namespace jfnk {

enum KFam {
  KF_RESID_VALUE = 0,
  KF_RESID_FD,
  KF_RESID_TANGENT,
  KF_VJP_A,
  KF_VJP_B,
  KF_VJP_FOLD,
  KF_GS_DOTS,
  KF_GS_UPDATE,
  KF_LINCOMB,
  KF_MG_PRE,
  KF_MG_PROLONG,
  KF_MG_SMOOTH2,
  KF_MG_COARSE,
  KF_CG_APPLY,
  KF_CG_UPDATE,
  KF_CG_PUPDATE,
  KF_DOT,
  KF_PBP_IN,
  KF_PBP_OUT,
  KF_SCALED,
  KF_MG_RESTRICT,
  KF_MG_DOWN,
  KF_MG_UP,
  KF_FD_SHIFT,
  KF_COUNT
};

extern const char* const kFamNames[KF_COUNT];

// When probing is enabled, hands out a start/stop event pair registered for family fam
// (with the launch's algorithmic bytes) and returns true.
bool probe_events(int fam, double bytes, hipEvent_t* start, hipEvent_t* stop);

// Launch a kernel; while probing, the start/stop events are attached to the dispatch itself
// (they time the kernel's execution, not the surrounding queue).
template <class F, class... Args>
inline void launch_k(int fam, double bytes, F kernel, dim3 grid, dim3 block, unsigned shm,
                     hipStream_t s, Args... args) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  probe_events(fam, bytes, &e0, &e1);
  hipExtLaunchKernelGGL(kernel, grid, block, shm, s, e0, e1, 0, args...);
}

void probe_enable(bool on);
bool probe_read(int fam, double* ms, long long* launches, double* bytes);

}  // namespace jfnk
