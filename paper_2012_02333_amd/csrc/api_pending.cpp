// Entry points whose kernels are not built yet: they validate nothing and
// report CQC_ERR_UNSUPPORTED.
#include "common.hpp"

extern "C" {

int cqc_backward_workspace_size(const cqc_instance *, int32_t, cqc_dtype, cqc_precision, size_t *) {
  return cqc::Status::fail(CQC_ERR_UNSUPPORTED, "backward not available").code;
}
int cqc_reconstruct_backward(const cqc_instance *, int32_t, cqc_dtype, cqc_precision,
                             const void *const *, void *const *const *, void *, size_t,
                             hipStream_t) {
  return cqc::Status::fail(CQC_ERR_UNSUPPORTED, "backward not available").code;
}
int cqc_autotune(const cqc_instance *, int32_t, cqc_dtype, cqc_dtype, cqc_precision, void *,
                 size_t, hipStream_t) {
  return cqc::Status::fail(CQC_ERR_UNSUPPORTED, "autotuner not available").code;
}
}
