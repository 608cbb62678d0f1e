// Shared host-side definitions of the cqc library: status handling, HIP error
// mapping, kernel launch tracing.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cstdint>
#include <string>

#include "../../include/cqc.h"

namespace cqc {

// Thread-local detail string of the last failing call.
void set_error(const std::string &msg);
const char *error_detail();

struct Status {
  int code = CQC_OK;
  static Status ok() { return Status{}; }
  static Status fail(int c, const std::string &msg) {
    set_error(msg);
    Status s;
    s.code = c;
    return s;
  }
  bool good() const { return code == CQC_OK; }
};

#define CQC_HIP_TRY(expr)                                                    \
  do {                                                                       \
    hipError_t e_ = (expr);                                                  \
    if (e_ != hipSuccess)                                                    \
      return ::cqc::Status::fail(CQC_ERR_HIP, std::string(#expr) + ": " +  \
                                                  hipGetErrorString(e_));    \
  } while (0)

#define CQC_TRY(expr)                \
  do {                               \
    ::cqc::Status s_ = (expr);       \
    if (!s_.good()) return s_;       \
  } while (0)

// Kernel launch tracing.  When enabled, the start and stop events are part of
// the dispatch itself (recorded when the kernel begins and ends), so a traced
// duration is the kernel's own run time without the launch gap around it.
bool trace_on();
bool trace_events(hipEvent_t *start, hipEvent_t *stop);
void trace_push(const char *name, hipEvent_t start, hipEvent_t stop);

// Launch helper: traces when enabled, checks the launch error.
template <typename Kernel, typename... Args>
Status launch(const char *name, Kernel k, dim3 grid, dim3 block, size_t shmem,
              hipStream_t s, Args... args) {
  if (grid.x == 0 || grid.y == 0 || grid.z == 0) return Status::ok();
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (trace_on() && trace_events(&ev0, &ev1))
    hipExtLaunchKernelGGL(k, grid, block, (uint32_t)shmem, s, ev0, ev1, 0u, args...);
  else
    hipLaunchKernelGGL(k, grid, block, shmem, s, args...);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    if (ev0) {
      (void)hipEventDestroy(ev0);
      (void)hipEventDestroy(ev1);
    }
    return Status::fail(CQC_ERR_HIP, std::string("launch ") + name + ": " +
                                         hipGetErrorString(e));
  }
  if (ev0) trace_push(name, ev0, ev1);
  return Status::ok();
}

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Tiles per work-queue item of the batched small-term tile kernels (one
// counter increment and descriptor lookup per item instead of per tile);
// shared by the batch planner and the queue kernel.
constexpr int kSmallTilesPerItem = 4;

}  // namespace cqc
