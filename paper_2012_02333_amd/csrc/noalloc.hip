// cqc_reconstruct_fd_noalloc: the full-definition call with its workspace in a
// fixed device array of this library, for callers that cannot allocate.
//
// The array is a file-scope __device__ symbol: each GPU that loads the code
// object holds its own copy, at its own address, until the process ends.  On
// the host, `scratch` names a host-side shadow, never the device memory, so
// host code only ever passes the device address that hipGetSymbolAddress
// returned for the device the call runs on (looked up once per device, with
// that device current, and kept).
#include <mutex>
#include <vector>

#include "common.hpp"

namespace cqc {
namespace {

constexpr size_t kScratchBytes = CQC_NOALLOC_WORKSPACE_BYTES;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
std::vector<void *> g_ptr;   // per device ordinal: device address of `scratch`

// Device that `stream` executes on (the current device for the null stream).
Status stream_device(hipStream_t stream, int *dev) {
  CQC_HIP_TRY(hipGetDevice(dev));
  if (stream) {
    hipDevice_t d = 0;
    CQC_HIP_TRY(hipStreamGetDevice(stream, &d));
    *dev = (int)d;
  }
  return Status::ok();
}

Status scratch_on(int dev, void **out) {
  std::lock_guard<std::mutex> g(g_mu);
  if ((size_t)dev < g_ptr.size() && g_ptr[dev]) {
    *out = g_ptr[dev];
    return Status::ok();
  }
  int cur = 0;
  CQC_HIP_TRY(hipGetDevice(&cur));
  if (cur != dev) CQC_HIP_TRY(hipSetDevice(dev));
  void *p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (cur != dev) (void)hipSetDevice(cur);
  if (e != hipSuccess || !p)
    return Status::fail(CQC_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  if (reinterpret_cast<uintptr_t>(p) % 256)
    return Status::fail(CQC_ERR_HIP, "static workspace is not 256-byte aligned");
  if (g_ptr.size() <= (size_t)dev) g_ptr.resize(dev + 1, nullptr);
  g_ptr[dev] = p;
  *out = p;
  return Status::ok();
}

}  // namespace
}  // namespace cqc

using namespace cqc;

extern "C" {

int cqc_reconstruct_fd_noalloc(const cqc_instance *inst, int32_t n_inst, cqc_dtype in_t,
                               cqc_dtype out_t, cqc_precision prec, hipStream_t stream) {
  size_t need = 0;
  int rc = cqc_fd_workspace_size(inst, n_inst, in_t, out_t, prec, &need);
  if (rc != CQC_OK) return rc;
  if (need > kScratchBytes)
    return Status::fail(CQC_ERR_WORKSPACE, "this call needs " + std::to_string(need) +
                                               " bytes of workspace; the static workspace holds " +
                                               std::to_string(kScratchBytes)).code;
  int dev = 0;
  Status st = stream_device(stream, &dev);
  if (!st.good()) return st.code;
  void *ws = nullptr;
  st = scratch_on(dev, &ws);
  if (!st.good()) return st.code;
  return cqc_reconstruct_fd(inst, n_inst, in_t, out_t, prec, ws, kScratchBytes, stream);
}

}  // extern "C"
