// C ABI: the device-resident dynamic-definition query (Algorithm 1,
// Section 4.3).
//
// The host-driven query (api_dd.cpp) reads every round's candidates back to
// choose the next bin.  Here the choice is a kernel: a run enqueues, for each
// recursion k, the refill of the window the previous pick emptied (a top-T
// request whose parameters the pick left in device memory), the pick of k,
// and then the merge, term sum, FP64 mass and top-T of every depth k could
// have - each launch gated on the depth the pick wrote, so exactly one of
// them does the work.  The records and the recursion count are written to
// device memory; nothing is read back, and a run can be captured in a graph.
// A zoom depth's plan does not depend on the chosen bins (only the zoomed
// values do, and the merge reads those from the query state), so every
// launch's arguments are fixed when the query is created.
#include <cmath>
#include <cstring>

#include "ddplan.hpp"

struct cqc_dd_query_s {
  std::shared_ptr<const cqc::DdPlan> plan;
  std::vector<const void *> entries;
  bool in_double = false;
  char *bins = nullptr;
  cqc_dd_record *records = nullptr;
  int32_t *n_done = nullptr;
  char *ws = nullptr;
  cqc::DdqState *st = nullptr;
};

namespace cqc {

static size_t ddq_state_off(const DdPlan &d) { return align_up(d.bytes, 256); }
static size_t ddq_bytes(const DdPlan &d) { return ddq_state_off(d) + align_up(ddq_state_bytes(d.R), 256); }

static Status ddq_plan(const cqc_instance *inst, cqc_dtype in_t, cqc_precision prec, const cqc_dd_params *p,
                       std::shared_ptr<const DdPlan> *out) {
  CQC_TRY(cached_dd(inst, in_t, prec, p, out));
  const DdPlan &d = **out;
  if (d.per_round != 1)
    return Status::fail(CQC_ERR_UNSUPPORTED, "the device-resident query expands one bin per recursion "
                                             "(bins_per_round 0 or 1)");
  if ((int)d.depths.size() > kDdqMaxDepths)
    return Status::fail(CQC_ERR_UNSUPPORTED, "more zoom depths than the device-resident query holds");
  return Status::ok();
}

static Status ddq_create(const cqc_instance *inst, cqc_dtype in_t, cqc_precision prec, const cqc_dd_params *p,
                         void *bins, cqc_dd_record *records, int32_t *n_done, void *workspace, size_t ws_bytes,
                         hipStream_t s, cqc_dd_query_s **out) {
  std::shared_ptr<const DdPlan> plan;
  CQC_TRY(ddq_plan(inst, in_t, prec, p, &plan));
  const DdPlan &d = *plan;
  if (!bins || !records || !n_done) return Status::fail(CQC_ERR_INVALID_ARG, "bins, records or n_done is NULL");
  if (!inst->entries) return Status::fail(CQC_ERR_INVALID_ARG, "entries is NULL");
  for (int c = 0; c < d.cut.nsub; ++c)
    if (!inst->entries[c]) return Status::fail(CQC_ERR_INVALID_ARG, "entries[" + std::to_string(c) + "] is NULL");
  const size_t need = ddq_bytes(d);
  if (!workspace || ws_bytes < need)
    return Status::fail(CQC_ERR_WORKSPACE, "workspace needs " + std::to_string(need) + " bytes");
  if (reinterpret_cast<uintptr_t>(workspace) % 256)
    return Status::fail(CQC_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  char *ws = static_cast<char *>(workspace);
  // the static tables of the state (the per-recursion part is reset by every run)
  std::vector<char> img(sizeof(DdqState), 0);
  DdqState &h = *reinterpret_cast<DdqState *>(img.data());
  h.R = d.R;
  h.D = (int)d.depths.size();
  h.n = d.cut.n;
  h.nsub = d.cut.nsub;
  h.strategy = d.strategy;
  int off = 0;
  for (int c = 0; c < d.cut.nsub; ++c) {
    h.f[c] = d.cut.f[c];
    for (int j = 0; j < d.cut.f[c]; ++j) h.qubit[off + j] = (int8_t)d.cut.qubits[c][j];
    off += d.cut.f[c];
  }
  for (size_t k = 0; k < d.depths.size(); ++k) {
    const DepthPlan &dp = d.depths[k];
    h.depth[k].n_active = (int32_t)dp.active.size();
    h.depth[k].has_merged = dp.has_merged ? 1 : 0;
    for (size_t t = 0; t < dp.active.size(); ++t) h.depth[k].active[t] = (int8_t)dp.active[t];
  }
  h.records = records;
  h.n_done = n_done;
  DdqState *st = reinterpret_cast<DdqState *>(ws + ddq_state_off(d));
  hipError_t e = hipMemcpyAsync(st, img.data(), img.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return Status::fail(CQC_ERR_HIP, std::string("uploading the query tables: ") + hipGetErrorString(e));
  auto *q = new cqc_dd_query_s();
  q->plan = plan;
  q->entries.assign(inst->entries, inst->entries + d.cut.nsub);
  q->in_double = in_t == CQC_F64;
  q->bins = static_cast<char *>(bins);
  q->records = records;
  q->n_done = n_done;
  q->ws = ws;
  q->st = st;
  *out = q;
  return Status::ok();
}

// Enqueues recursions [k0, k1); k0 = 0 starts a new search (state reset),
// k0 > 0 continues the one the query state holds.
static Status ddq_run(const cqc_dd_query_s *q, int k0, int k1, hipStream_t s) {
  const DdPlan &d = *q->plan;
  const bool acc_double = d.acc == Acc::F64;
  const int64_t stride = int64_t(1) << d.a;
  const size_t bin_size = d.bins_f32 ? 4 : 8;
  DdqState *st = q->st;
  char *ws = q->ws;
  const int D = (int)d.depths.size();
  if (k0 == 0) CQC_TRY(launch_ddq_init(st, s));
  for (int k = k0; k < k1; ++k) {
    if (k > 0) {
      CQC_TRY(launch_topk_req(q->bins, d.bins_f32, stride, stride, ws + d.topk_off, &st->refill, s));
      CQC_TRY(launch_ddq_pick(st, k, s));
    }
    char *brow = q->bins + (size_t)k * (size_t)stride * bin_size;
    const int32_t *gate = &st->rec[k].depth;
    // the depths recursion k can have: 0 for the first; a child of a
    // recursion j < k is one deeper than j, and only depths below the last
    // have merged qubits to refine
    const int d_lo = k == 0 ? 0 : 1, d_hi = k == 0 ? 0 : std::min(k, D - 1);
    for (int dd = d_lo; dd <= d_hi; ++dd) {
      const DepthPlan &dp = d.depths[dd];
      const int64_t *zoom_dev[CQC_MAX_SUB];
      for (int c = 0; c < d.cut.nsub; ++c) zoom_dev[c] = &st->rec[k].zoom[c];
      MergeArgs ma;
      int64_t blocks = 0;
      std::vector<const void *> merged;
      dd_merge_args(d, dp, q->entries.data(), ws, q->in_double, nullptr, zoom_dev, &ma, &blocks, &merged);
      ma.gate = gate;
      ma.gate_val = dd;
      if (ma.n > 0) CQC_TRY(launch_dd_merge(ma, blocks, q->in_double, acc_double, s));
      CQC_TRY(run_net(dp.net, ws, merged, brow, !d.bins_f32, &q->records[k].mass, true, s, false, gate, dd));
      if (dp.has_merged && k + 1 < d.R)
        CQC_TRY(launch_topk(brow, d.bins_f32, int64_t(1) << dp.active.size(), kTopT, ws + d.topk_off,
                            &st->rec[k].top, INFINITY, -1, s, gate, dd));
    }
  }
  return Status::ok();
}

}  // namespace cqc

using namespace cqc;

extern "C" {

int cqc_dd_query_workspace_size(const cqc_instance *inst, cqc_dtype in_t, cqc_precision prec,
                                const cqc_dd_params *p, size_t *bytes) {
  if (!bytes) return Status::fail(CQC_ERR_INVALID_ARG, "bytes is NULL").code;
  std::shared_ptr<const DdPlan> plan;
  Status st = ddq_plan(inst, in_t, prec, p, &plan);
  if (!st.good()) return st.code;
  *bytes = ddq_bytes(*plan);
  return CQC_OK;
}

int cqc_dd_query_create(const cqc_instance *inst, cqc_dtype in_t, cqc_precision prec, const cqc_dd_params *p,
                        void *bins, cqc_dd_record *records, int32_t *n_done, void *workspace, size_t ws_bytes,
                        hipStream_t stream, cqc_dd_query *out) {
  if (!out) return Status::fail(CQC_ERR_INVALID_ARG, "out is NULL").code;
  cqc_dd_query_s *q = nullptr;
  Status st = ddq_create(inst, in_t, prec, p, bins, records, n_done, workspace, ws_bytes, stream, &q);
  if (!st.good()) return st.code;
  *out = q;
  return CQC_OK;
}

int cqc_dd_query_run(cqc_dd_query q, hipStream_t stream) {
  if (!q) return Status::fail(CQC_ERR_INVALID_ARG, "query is NULL").code;
  return ddq_run(q, 0, q->plan->R, stream).code;
}

int cqc_dd_query_run_range(cqc_dd_query q, int32_t first, int32_t count, hipStream_t stream) {
  if (!q) return Status::fail(CQC_ERR_INVALID_ARG, "query is NULL").code;
  if (first < 0 || count < 0 || (int64_t)first + count > q->plan->R)
    return Status::fail(CQC_ERR_INVALID_ARG, "recursion range outside [0, n_recursions)").code;
  return ddq_run(q, first, first + count, stream).code;
}

int cqc_dd_query_destroy(cqc_dd_query q) {
  delete q;
  return CQC_OK;
}

}  // extern "C"
