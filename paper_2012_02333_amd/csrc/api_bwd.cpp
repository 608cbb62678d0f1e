// C ABI: adjoint of the full-definition build (gradients of a loss on the
// reconstructed distribution with respect to every entry tensor).
//
// The forward intermediates are recomputed (all contraction steps but the
// last), then the steps are swept in reverse: the last step's dL/dZ is the
// given dL/dp (gathered into blocked order if the output order is not
// blocked) scaled by 2^-K, and every step sends gradients to its two
// operands - straight into the caller's gradient buffers for entry tensors,
// into workspace for intermediates.  Early termination is not applied here:
// the gradient of an all-zero row is in general not zero.
#include <cmath>
#include <cstring>

#include "bwd.hpp"

namespace cqc {

struct BwdInstancePlan {
  CutInfo cut;
  NetLayout net;
  std::vector<size_t> conv_off;   // converted entries (or SIZE_MAX)
  std::vector<size_t> dz_off;     // per tensor: dL/dZ buffer of intermediates (or SIZE_MAX)
  size_t g_off = SIZE_MAX;        // converted / gathered dL/dp (or SIZE_MAX: use caller's)
  bool g_convert = false, g_gather = false;
  size_t part_off = 0, part_bytes = 0;
  std::vector<BwdSide> sx, sy;    // per step
  size_t end = 0;
};

BwdSide choose_bwd_side(int64_t inner, int64_t rest, int64_t out_elems, int64_t dz_elems, size_t esz,
                        double min_budget, double dz_frac) {
  BwdSide s;
  const double budget = std::max(min_budget, dz_frac * (double)dz_elems * (double)esz);
  int64_t kc = 128;
  if (kc > inner) kc = (inner + 15) / 16 * 16;
  while (true) {
    const int64_t chunks = (inner + kc - 1) / kc;
    const int64_t P = rest * chunks;
    if ((double)P * (double)out_elems * (double)esz <= budget || kc >= inner) {
      s.kChunk = kc;
      s.kChunks = (int32_t)chunks;
      s.P = P;
      return s;
    }
    kc *= 2;
  }
}

static Status plan_bwd_instance(const cqc_instance &in, const void *gout, void *const *gents,
                                cqc_dtype in_t, Acc acc, size_t base, bool need_ptrs,
                                BwdInstancePlan *out) {
  BwdInstancePlan ip;
  CQC_TRY(validate_cut(&in.cut, CQC_MAX_FD_QUBITS, &ip.cut));
  if (need_ptrs) {
    if (!in.entries) return Status::fail(CQC_ERR_INVALID_ARG, "entries is NULL");
    if (!gout) return Status::fail(CQC_ERR_INVALID_ARG, "grad_out is NULL");
    if (!gents) return Status::fail(CQC_ERR_INVALID_ARG, "grad_entries is NULL");
    for (int c = 0; c < ip.cut.nsub; ++c)
      if (!in.entries[c] || !gents[c])
        return Status::fail(CQC_ERR_INVALID_ARG, "entry or gradient pointer " + std::to_string(c) + " is NULL");
  }
  std::vector<int> bitpos(ip.cut.n);
  for (int q = 0; q < ip.cut.n; ++q) bitpos[q] = ip.cut.n - 1 - q;
  Plan plan = make_plan(ip.cut, ip.cut.qubits, bitpos, ip.cut.n);
  const bool in_double = in_t == CQC_F64, acc_double = acc == Acc::F64;
  const size_t esz = acc_double ? 8 : 4;
  size_t off = base;
  ip.conv_off.assign(ip.cut.nsub, SIZE_MAX);
  if (in_double != acc_double)
    for (int c = 0; c < ip.cut.nsub; ++c) {
      off = align_up(off, 256);
      ip.conv_off[c] = off;
      off += esz * (size_t)plan.tensors[c].rows() * (size_t)plan.tensors[c].cols();
    }
  ip.net = layout_net(plan, acc, off);
  off = ip.net.bytes;
  const Step &last = plan.steps.back();
  ip.g_convert = in_double != acc_double;
  ip.g_gather = !is_blocked(plan, last);
  const size_t gbytes = esz * ((size_t)1 << ip.cut.n);
  if (ip.g_convert || ip.g_gather) {
    off = align_up(off, 256);
    ip.g_off = off;
    off += gbytes * (ip.g_convert && ip.g_gather ? 2 : 1);
  }
  ip.dz_off.assign(plan.tensors.size(), SIZE_MAX);
  for (size_t i = 0; i + 1 < plan.steps.size(); ++i) {
    const TensorSpec &Z = plan.tensors[plan.steps[i].z];
    off = align_up(off, 256);
    ip.dz_off[plan.steps[i].z] = off;
    off += esz * (size_t)Z.rows() * (size_t)Z.cols();
  }
  size_t part = 0;
  for (const Step &st : plan.steps) {
    const TensorSpec &X = plan.tensors[st.x], &Y = plan.tensors[st.y];
    const int64_t M = int64_t(1) << st.logM, N = int64_t(1) << st.logN;
    const int64_t dz = st.nbatch * M * N;
    const int64_t RXn = int64_t(1) << (2 * st.RX.size()), RYn = int64_t(1) << (2 * st.RY.size());
    BwdSide bx = choose_bwd_side(N, RYn, X.rows() * M, dz, esz, 32.0 * (1 << 20));
    BwdSide by = choose_bwd_side(M, RXn, Y.rows() * N, dz, esz, 32.0 * (1 << 20));
    ip.sx.push_back(bx);
    ip.sy.push_back(by);
    part = std::max(part, esz * (size_t)(bx.P * X.rows() * M));
    part = std::max(part, esz * (size_t)(by.P * Y.rows() * N));
  }
  off = align_up(off, 256);
  ip.part_off = off;
  ip.part_bytes = part;
  off += part;
  ip.end = align_up(off, 256);
  *out = std::move(ip);
  return Status::ok();
}

static Status bwd_plans(const cqc_instance *inst, int32_t n_inst, cqc_dtype in_t, cqc_precision prec,
                        const void *const *gout, void *const *const *gents, bool need_ptrs,
                        std::vector<BwdInstancePlan> *plans, Acc *acc) {
  if (!inst) return Status::fail(CQC_ERR_INVALID_ARG, "inst is NULL");
  if (n_inst < 1) return Status::fail(CQC_ERR_INVALID_ARG, "n_inst < 1");
  if (in_t != CQC_F32 && in_t != CQC_F64) return Status::fail(CQC_ERR_INVALID_ARG, "unknown dtype");
  switch (prec) {
    case CQC_PREC_FP64: *acc = Acc::F64; break;
    case CQC_PREC_FP32: *acc = Acc::F32; break;
    case CQC_PREC_BF16X6:
    case CQC_PREC_BF16X3: return Status::fail(CQC_ERR_UNSUPPORTED, "the split-BF16 forms are not available for the adjoint");
    default: return Status::fail(CQC_ERR_INVALID_ARG, "unknown precision");
  }
  if (need_ptrs && (!gout || !gents)) return Status::fail(CQC_ERR_INVALID_ARG, "gradient arrays are NULL");
  size_t off = 0;
  plans->clear();
  for (int32_t i = 0; i < n_inst; ++i) {
    BwdInstancePlan ip;
    Status st = plan_bwd_instance(inst[i], need_ptrs ? gout[i] : nullptr, need_ptrs ? gents[i] : nullptr,
                                  in_t, *acc, off, need_ptrs, &ip);
    if (!st.good()) {
      set_error("instance " + std::to_string(i) + ": " + error_detail());
      return st;
    }
    off = ip.end;
    plans->push_back(std::move(ip));
  }
  return Status::ok();
}

static Status run_bwd_instance(const BwdInstancePlan &ip, const cqc_instance &in, const void *gout,
                               void *const *gents, bool in_double, Acc acc, char *ws, hipStream_t s) {
  const bool acc_double = acc == Acc::F64;
  const Plan &p = ip.net.plan;
  std::vector<const void *> ents(ip.cut.nsub);
  for (int c = 0; c < ip.cut.nsub; ++c) {
    if (ip.conv_off[c] != SIZE_MAX) {
      const auto &T = p.tensors[c];
      CQC_TRY(launch_convert(in.entries[c], in_double, ws + ip.conv_off[c], acc_double, T.rows() * T.cols(), s));
      ents[c] = ws + ip.conv_off[c];
    } else {
      ents[c] = in.entries[c];
    }
  }
  // forward intermediates
  CQC_TRY(run_net(ip.net, ws, ents, nullptr, acc_double, nullptr, true, s, true));
  std::vector<const void *> tptr(p.tensors.size(), nullptr);
  for (size_t t = 0; t < p.tensors.size(); ++t)
    tptr[t] = p.tensors[t].entry >= 0 ? ents[p.tensors[t].entry] : ws + ip.net.t_off[t];
  // dL/dZ of the last step in blocked order, Acc dtype
  const Step &last = p.steps.back();
  const void *g = gout;
  const size_t gelems = (size_t)1 << ip.cut.n;
  if (ip.g_convert) {
    CQC_TRY(launch_convert(gout, in_double, ws + ip.g_off, acc_double, (int64_t)gelems, s));
    g = ws + ip.g_off;
  }
  if (ip.g_gather) {
    char *dst = ws + ip.g_off + (ip.g_convert ? gelems * (acc_double ? 8 : 4) : 0);
    const auto &X = p.tensors[last.x], &Y = p.tensors[last.y];
    const int nX = (int)X.bits.size(), nY = (int)Y.bits.size();
    std::vector<int> px(nX), py(nY);
    for (int j = 0; j < nX; ++j) px[j] = p.bitpos[X.bits[nX - 1 - j]];
    for (int j = 0; j < nY; ++j) py[j] = p.bitpos[Y.bits[nY - 1 - j]];
    CQC_TRY(launch_gather_blocked(acc, g, dst, last.logM, last.logN, pack_pos(px), pack_pos(py), s));
    g = dst;
  }
  void *part = ws + ip.part_off;
  for (int i = (int)p.steps.size() - 1; i >= 0; --i) {
    const Step &st = p.steps[i];
    const bool is_last = i + 1 == (int)p.steps.size();
    BwdArgs a;
    std::memset(&a, 0, sizeof(a));
    a.X = tptr[st.x];
    a.Y = tptr[st.y];
    a.dZ = is_last ? g : ws + ip.dz_off[st.z];
    a.part = part;
    a.logM = st.logM;
    a.logN = st.logN;
    a.nS = (int)st.S.size();
    a.nRX = (int)st.RX.size();
    a.nRY = (int)st.RY.size();
    a.mx = to_dev(st.mx);
    a.my = to_dev(st.my);
    a.rowsX = p.tensors[st.x].rows();
    a.rowsY = p.tensors[st.y].rows();
    const double scale = is_last ? std::ldexp(1.0, -p.K) : 1.0;
    const int64_t M = int64_t(1) << st.logM, N = int64_t(1) << st.logN;
    for (int side = 0; side < 2; ++side) {
      const int t = side == 0 ? st.x : st.y;
      const TensorSpec &T = p.tensors[t];
      if (T.entry == -2) continue;  // unit tensor of a single subcircuit
      const BwdSide &bs = side == 0 ? ip.sx[i] : ip.sy[i];
      a.kChunk = bs.kChunk;
      a.kChunks = bs.kChunks;
      CQC_TRY(launch_bwd(acc, a, side == 1, s));
      const int64_t count = T.rows() * (side == 0 ? M : N);
      if (T.entry >= 0) {
        CQC_TRY(launch_bwd_reduce(acc, part, count, bs.P, scale, gents[T.entry], in_double, s));
      } else {
        CQC_TRY(launch_bwd_reduce(acc, part, count, bs.P, scale, ws + ip.dz_off[t], acc_double, s));
      }
    }
  }
  return Status::ok();
}

}  // namespace cqc

using namespace cqc;

extern "C" {

int cqc_backward_workspace_size(const cqc_instance *inst, int32_t n_inst, cqc_dtype in_t,
                                cqc_precision prec, size_t *bytes) {
  if (!bytes) return Status::fail(CQC_ERR_INVALID_ARG, "bytes is NULL").code;
  std::vector<BwdInstancePlan> plans;
  Acc acc;
  Status st = bwd_plans(inst, n_inst, in_t, prec, nullptr, nullptr, false, &plans, &acc);
  if (!st.good()) return st.code;
  *bytes = plans.back().end;
  return CQC_OK;
}

int cqc_reconstruct_backward(const cqc_instance *inst, int32_t n_inst, cqc_dtype in_t,
                             cqc_precision prec, const void *const *grad_out,
                             void *const *const *grad_entries, void *workspace,
                             size_t ws_bytes, hipStream_t stream) {
  std::vector<BwdInstancePlan> plans;
  Acc acc;
  Status st = bwd_plans(inst, n_inst, in_t, prec, grad_out, grad_entries, true, &plans, &acc);
  if (!st.good()) return st.code;
  const size_t need = plans.back().end;
  if (!workspace || ws_bytes < need)
    return Status::fail(CQC_ERR_WORKSPACE, "workspace needs " + std::to_string(need) + " bytes").code;
  if (reinterpret_cast<uintptr_t>(workspace) % 256)
    return Status::fail(CQC_ERR_WORKSPACE, "workspace must be 256-byte aligned").code;
  for (int32_t i = 0; i < n_inst; ++i) {
    st = run_bwd_instance(plans[i], inst[i], grad_out[i], grad_entries[i], in_t == CQC_F64, acc,
                          static_cast<char *>(workspace), stream);
    if (!st.good()) return st.code;
  }
  return CQC_OK;
}

}  // extern "C"
