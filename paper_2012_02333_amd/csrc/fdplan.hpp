// Per-instance plans of the full-definition path (shared by single and batched calls).
#pragma once

#include <vector>

#include "engine.hpp"

namespace cqc {

struct FdInstancePlan {
  CutInfo cut;
  NetLayout net;
  std::vector<size_t> conv_off;  // per entry: converted copy (or SIZE_MAX)
  size_t end = 0;
};

Status precision_acc(cqc_precision prec, Acc *acc);
Status check_dtype(cqc_dtype t);
// out_optional: inst.out may be NULL (a cross-entropy batch that does not
// keep p); every other pointer is required when need_ptrs is set.
Status plan_fd_instance(const cqc_instance &in, cqc_dtype in_t, Acc acc, size_t base, bool need_ptrs,
                        FdInstancePlan *out, bool out_optional = false);
Status fd_plans(const cqc_instance *inst, int32_t n_inst, cqc_dtype in_t, cqc_dtype out_t,
                cqc_precision prec, bool need_ptrs, std::vector<FdInstancePlan> *plans, Acc *acc_out,
                bool out_optional = false);

}  // namespace cqc
