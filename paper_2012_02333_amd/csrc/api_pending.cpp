// Entry points whose kernels are not built yet: they validate nothing and
// report CQC_ERR_UNSUPPORTED.
#include "common.hpp"

extern "C" {

int cqc_autotune(const cqc_instance *, int32_t, cqc_dtype, cqc_dtype, cqc_precision, void *,
                 size_t, hipStream_t) {
  return cqc::Status::fail(CQC_ERR_UNSUPPORTED, "autotuner not available").code;
}
}
