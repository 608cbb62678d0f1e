// C ABI: full-definition reconstruction, cost model, MFMA self test.
#include <cmath>
#include <cstring>

#include "fdplan.hpp"

namespace cqc {


Status precision_acc(cqc_precision prec, Acc *acc) {
  switch (prec) {
    case CQC_PREC_FP64: *acc = Acc::F64; return Status::ok();
    case CQC_PREC_FP32: *acc = Acc::F32; return Status::ok();
    case CQC_PREC_BF16X6: *acc = Acc::BF16X6; return Status::ok();
    case CQC_PREC_BF16X3: *acc = Acc::BF16X3; return Status::ok();
    default: return Status::fail(CQC_ERR_INVALID_ARG, "unknown precision");
  }
}

Status check_dtype(cqc_dtype t) {
  if (t != CQC_F32 && t != CQC_F64) return Status::fail(CQC_ERR_INVALID_ARG, "unknown dtype");
  return Status::ok();
}

Status plan_fd_instance(const cqc_instance &in, cqc_dtype in_t, Acc acc, size_t base,
                               bool need_ptrs, FdInstancePlan *out, bool out_optional) {
  FdInstancePlan ip;
  CQC_TRY(validate_cut(&in.cut, CQC_MAX_FD_QUBITS, &ip.cut));
  if (need_ptrs) {
    if (!in.entries) return Status::fail(CQC_ERR_INVALID_ARG, "entries is NULL");
    for (int c = 0; c < ip.cut.nsub; ++c)
      if (!in.entries[c]) return Status::fail(CQC_ERR_INVALID_ARG, "entries[" + std::to_string(c) + "] is NULL");
    if (!in.out && !out_optional) return Status::fail(CQC_ERR_INVALID_ARG, "out is NULL");
  }
  std::vector<int> bitpos(ip.cut.n);
  for (int q = 0; q < ip.cut.n; ++q) bitpos[q] = ip.cut.n - 1 - q;
  Plan plan = make_plan(ip.cut, ip.cut.qubits, bitpos, ip.cut.n);
  const bool in_double = in_t == CQC_F64;
  const bool acc_double = acc == Acc::F64;
  size_t off = base;
  ip.conv_off.assign(ip.cut.nsub, SIZE_MAX);
  if (in_double != acc_double) {
    for (int c = 0; c < ip.cut.nsub; ++c) {
      off = align_up(off, 256);
      ip.conv_off[c] = off;
      off += (acc_double ? 8 : 4) * (size_t)plan.tensors[c].rows() * (size_t)plan.tensors[c].cols();
    }
  }
  ip.net = layout_net(plan, acc, off);
  ip.end = ip.net.bytes;
  *out = std::move(ip);
  return Status::ok();
}

Status fd_plans(const cqc_instance *inst, int32_t n_inst, cqc_dtype in_t, cqc_dtype out_t,
                       cqc_precision prec, bool need_ptrs, std::vector<FdInstancePlan> *plans,
                       Acc *acc_out, bool out_optional) {
  if (!inst) return Status::fail(CQC_ERR_INVALID_ARG, "inst is NULL");
  if (n_inst < 1) return Status::fail(CQC_ERR_INVALID_ARG, "n_inst < 1");
  CQC_TRY(check_dtype(in_t));
  CQC_TRY(check_dtype(out_t));
  Acc acc;
  CQC_TRY(precision_acc(prec, &acc));
  size_t off = 0;
  plans->clear();
  for (int32_t i = 0; i < n_inst; ++i) {
    FdInstancePlan ip;
    Status st = plan_fd_instance(inst[i], in_t, acc, off, need_ptrs, &ip, out_optional);
    if (!st.good()) {
      set_error("instance " + std::to_string(i) + ": " + error_detail());
      return st;
    }
    off = ip.end;
    plans->push_back(std::move(ip));
  }
  *acc_out = acc;
  return Status::ok();
}

size_t batch_workspace_bytes(const cqc_instance *inst, int32_t n_inst, cqc_dtype in_t, cqc_dtype out_t,
                             cqc_precision prec, Status *st);

}  // namespace cqc

using namespace cqc;

extern "C" {

int cqc_fd_workspace_size(const cqc_instance *inst, int32_t n_inst, cqc_dtype in_t,
                          cqc_dtype out_t, cqc_precision prec, size_t *bytes) {
  if (!bytes) return Status::fail(CQC_ERR_INVALID_ARG, "bytes is NULL").code;
  std::vector<FdInstancePlan> plans;
  Acc acc;
  Status st = fd_plans(inst, n_inst, in_t, out_t, prec, false, &plans, &acc);
  if (!st.good()) return st.code;
  *bytes = plans.back().end;
  if (n_inst > 1 && (out_t == CQC_F64) == (acc == Acc::F64)) {
    const size_t b = batch_workspace_bytes(inst, n_inst, in_t, out_t, prec, &st);
    if (!st.good()) return st.code;
    *bytes = b;
  }
  return CQC_OK;
}

int cqc_reconstruct_fd(const cqc_instance *inst, int32_t n_inst, cqc_dtype in_t,
                       cqc_dtype out_t, cqc_precision prec, void *workspace,
                       size_t ws_bytes, hipStream_t stream) {
  std::vector<FdInstancePlan> plans;
  Acc acc;
  Status st = fd_plans(inst, n_inst, in_t, out_t, prec, true, &plans, &acc);
  if (!st.good()) return st.code;
  const size_t need = plans.back().end;
  if (!workspace && need > 0) return Status::fail(CQC_ERR_WORKSPACE, "workspace is NULL").code;
  if (ws_bytes < need)
    return Status::fail(CQC_ERR_WORKSPACE, "workspace has " + std::to_string(ws_bytes) +
                                               " bytes, needs " + std::to_string(need)).code;
  if (reinterpret_cast<uintptr_t>(workspace) % 256)
    return Status::fail(CQC_ERR_WORKSPACE, "workspace must be 256-byte aligned").code;
  char *ws = static_cast<char *>(workspace);
  const bool in_double = in_t == CQC_F64, acc_double = acc == Acc::F64;
  if (n_inst > 1 && (out_t == CQC_F64) == acc_double) {
    // batched: one flag pass, one launch per step group, one mass pass
    cqc_batch b = nullptr;
    int rc = cqc_batch_create(inst, n_inst, in_t, out_t, prec, workspace, ws_bytes, stream, &b);
    if (rc != CQC_OK) return rc;
    rc = cqc_batch_run(b, stream);
    cqc_batch_destroy(b);
    return rc;
  }
  for (int32_t i = 0; i < n_inst; ++i) {
    const FdInstancePlan &ip = plans[i];
    std::vector<const void *> ents(ip.cut.nsub);
    for (int c = 0; c < ip.cut.nsub; ++c) {
      if (in_double != acc_double) {
        void *dst = ws + ip.conv_off[c];
        const auto &T = ip.net.plan.tensors[c];
        st = launch_convert(inst[i].entries[c], in_double, dst, acc_double, T.rows() * T.cols(), stream);
        if (!st.good()) return st.code;
        ents[c] = dst;
      } else {
        ents[c] = inst[i].entries[c];
      }
    }
    st = run_net(ip.net, ws, ents, inst[i].out, out_t == CQC_F64, inst[i].mass, true, stream);
    if (!st.good()) return st.code;
  }
  return CQC_OK;
}

int cqc_cost(const cqc_cut *cut, double *eq14_mults, double *plan_macs_out) {
  CutInfo ci;
  Status st = validate_cut(cut, CQC_MAX_DD_QUBITS, &ci);
  if (!st.good()) return st.code;
  std::vector<int> bitpos(ci.n);
  for (int q = 0; q < ci.n; ++q) bitpos[q] = ci.n - 1 - q;
  Plan p = make_plan(ci, ci.qubits, bitpos, ci.n);
  if (eq14_mults) *eq14_mults = eq14_cost(ci);
  if (plan_macs_out) *plan_macs_out = plan_macs(p);
  return CQC_OK;
}

int cqc_selftest_mfma(void *out, hipStream_t stream) {
  if (!out) return Status::fail(CQC_ERR_INVALID_ARG, "out is NULL").code;
  return launch_selftest_mfma(out, stream).code;
}

}  // extern "C"
