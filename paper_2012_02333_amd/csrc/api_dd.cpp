// C ABI: dynamic definition (Algorithm 1, Section 4.3), host-driven.
//
// The qubit roles of a recursion depend only on its depth in the zoom tree
// (depth 1: the first active set; depth d+1: the depth-d zoomed and active
// qubits are zoomed, the next n_active un-zoomed qubits in output order are
// active), never on which bin was chosen - only the zoomed VALUES depend on
// the data.  So every depth's contraction plan and workspace are known before
// anything runs; per recursion the host only learns which bin to refine.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>

#include "dd.hpp"

namespace cqc {

struct DepthPlan {
  std::vector<int> active;                   // ascending qubit ids
  std::vector<char> zoomed;                  // per qubit
  bool has_merged = false;
  std::vector<std::vector<int>> act_local;   // per subcircuit: active local bits j (ascending)
  std::vector<std::vector<int>> mrg_local;   // per subcircuit: merged local bits j
  NetLayout net;
  std::vector<size_t> merged_off;
  size_t end = 0;
};

struct DdPlan {
  CutInfo cut;
  Acc acc;
  int a = 0, R = 0;
  std::vector<DepthPlan> depths;
  size_t topk_off = 0, out_off = 0, bytes = 0;
};

static Status build_dd(const cqc_instance *inst, cqc_dtype in_t, cqc_precision prec,
                       const cqc_dd_params *p, DdPlan *out) {
  if (!inst) return Status::fail(CQC_ERR_INVALID_ARG, "inst is NULL");
  if (!p) return Status::fail(CQC_ERR_INVALID_ARG, "params is NULL");
  if (in_t != CQC_F32 && in_t != CQC_F64) return Status::fail(CQC_ERR_INVALID_ARG, "unknown dtype");
  DdPlan d;
  switch (prec) {
    case CQC_PREC_FP64: d.acc = Acc::F64; break;
    case CQC_PREC_FP32: d.acc = Acc::F32; break;
    case CQC_PREC_BF16X6: d.acc = Acc::BF16X6; break;
    default: return Status::fail(CQC_ERR_INVALID_ARG, "unknown precision");
  }
  CQC_TRY(validate_cut(&inst->cut, CQC_MAX_DD_QUBITS, &d.cut));
  const int n = d.cut.n;
  if (p->strategy != 0) return Status::fail(CQC_ERR_UNSUPPORTED, "only strategy 0 (heaviest bin) is implemented");
  if (p->n_active < 1 || p->n_active > 30) return Status::fail(CQC_ERR_INVALID_ARG, "n_active must be in [1, 30]");
  if (p->n_recursions < 1) return Status::fail(CQC_ERR_INVALID_ARG, "n_recursions must be >= 1");
  if (n < 1) return Status::fail(CQC_ERR_SHAPE, "dynamic definition needs at least one qubit");
  d.a = std::min(p->n_active, n);
  d.R = p->n_recursions;
  std::vector<int> first;
  if (p->first_active) {
    if (p->n_active > n) return Status::fail(CQC_ERR_INVALID_ARG, "first_active longer than n_qubits");
    std::vector<char> seen(n, 0);
    for (int i = 0; i < p->n_active; ++i) {
      const int q = p->first_active[i];
      if (q < 0 || q >= n) return Status::fail(CQC_ERR_INVALID_ARG, "first_active names a qubit out of range");
      if (seen[q]++) return Status::fail(CQC_ERR_INVALID_ARG, "first_active repeats a qubit");
      first.push_back(q);
    }
    std::sort(first.begin(), first.end());
  } else {
    for (int q = 0; q < d.a; ++q) first.push_back(q);
  }
  // depth plans
  std::vector<char> zoomed(n, 0);
  std::vector<int> active = first;
  size_t esz = d.acc == Acc::F64 ? 8 : 4;
  for (int depth = 0; depth < d.R && !active.empty(); ++depth) {
    DepthPlan dp;
    dp.active = active;
    dp.zoomed = zoomed;
    std::vector<char> is_act(n, 0);
    for (int q : active) is_act[q] = 1;
    int n_merged = 0;
    for (int q = 0; q < n; ++q) n_merged += !is_act[q] && !zoomed[q];
    dp.has_merged = n_merged > 0;
    std::vector<std::vector<int>> cols(d.cut.nsub);
    dp.act_local.assign(d.cut.nsub, {});
    dp.mrg_local.assign(d.cut.nsub, {});
    for (int c = 0; c < d.cut.nsub; ++c)
      for (int j = 0; j < d.cut.f[c]; ++j) {
        const int q = d.cut.qubits[c][j];
        if (is_act[q]) {
          dp.act_local[c].push_back(j);
          cols[c].push_back(q);
        } else if (!zoomed[q]) {
          dp.mrg_local[c].push_back(j);
        }
      }
    const int ad = (int)active.size();
    std::vector<int> bitpos(n, 0);
    for (int r = 0; r < ad; ++r) bitpos[active[r]] = ad - 1 - r;
    Plan plan = make_plan(d.cut, cols, bitpos, ad);
    size_t off = 0;
    dp.merged_off.assign(d.cut.nsub, 0);
    for (int c = 0; c < d.cut.nsub; ++c) {
      off = align_up(off, 256);
      dp.merged_off[c] = off;
      off += esz * (size_t)plan.tensors[c].rows() * ((size_t)1 << dp.act_local[c].size());
    }
    dp.net = layout_net(plan, d.acc, off);
    dp.end = dp.net.bytes;
    d.depths.push_back(std::move(dp));
    // next depth
    if (n_merged == 0) break;
    for (int q : active) zoomed[q] = 1;
    active.clear();
    for (int q = 0; q < n && (int)active.size() < d.a; ++q)
      if (!zoomed[q]) active.push_back(q);
  }
  size_t end = 0;
  for (auto &dp : d.depths) end = std::max(end, dp.end);
  d.topk_off = align_up(end, 256);
  d.out_off = align_up(d.topk_off + topk_scratch_bytes(int64_t(1) << d.a, kTopT), 256);
  d.bytes = align_up(d.out_off + sizeof(TopOut) + 8, 256);
  *out = std::move(d);
  return Status::ok();
}

namespace {
struct RecState {
  int depth = 0;
  std::map<int, int> zoomval;        // qubit -> 0/1
  std::vector<std::pair<double, int64_t>> cands;
  size_t consumed = 0;
  bool exhausted = false;
  bool has_merged = false;
  int64_t nbins = 0;
};
}  // namespace

}  // namespace cqc

using namespace cqc;

extern "C" {

int cqc_dd_workspace_size(const cqc_instance *inst, cqc_dtype in_t, cqc_precision prec,
                          const cqc_dd_params *p, size_t *bytes) {
  if (!bytes) return Status::fail(CQC_ERR_INVALID_ARG, "bytes is NULL").code;
  DdPlan d;
  Status st = build_dd(inst, in_t, prec, p, &d);
  if (!st.good()) return st.code;
  *bytes = d.bytes;
  return CQC_OK;
}

int cqc_reconstruct_dd(const cqc_instance *inst, cqc_dtype in_t, cqc_precision prec,
                       const cqc_dd_params *p, double *bins, cqc_dd_record *records,
                       int32_t *n_done, void *workspace, size_t ws_bytes, hipStream_t stream) {
  DdPlan d;
  Status st = build_dd(inst, in_t, prec, p, &d);
  if (!st.good()) return st.code;
  if (!bins || !records || !n_done) return Status::fail(CQC_ERR_INVALID_ARG, "bins, records or n_done is NULL").code;
  if (!inst->entries) return Status::fail(CQC_ERR_INVALID_ARG, "entries is NULL").code;
  for (int c = 0; c < d.cut.nsub; ++c)
    if (!inst->entries[c]) return Status::fail(CQC_ERR_INVALID_ARG, "entries[" + std::to_string(c) + "] is NULL").code;
  if (!workspace || ws_bytes < d.bytes)
    return Status::fail(CQC_ERR_WORKSPACE, "workspace needs " + std::to_string(d.bytes) + " bytes").code;
  if (reinterpret_cast<uintptr_t>(workspace) % 256)
    return Status::fail(CQC_ERR_WORKSPACE, "workspace must be 256-byte aligned").code;
  char *ws = static_cast<char *>(workspace);
  const int n = d.cut.n;
  const bool in_double = in_t == CQC_F64, acc_double = d.acc == Acc::F64;
  const int64_t stride = int64_t(1) << d.a;
  TopOut *dev_top = reinterpret_cast<TopOut *>(ws + d.out_off);
  double *dev_mass = reinterpret_cast<double *>(ws + d.out_off + sizeof(TopOut));
  std::vector<RecState> recs;
  *n_done = 0;

  auto fetch = [&](TopOut *top, double *mass) -> Status {
    struct {
      TopOut t;
      double m;
    } host;
    CQC_HIP_TRY(hipMemcpyAsync(&host, dev_top, sizeof(TopOut) + 8, hipMemcpyDeviceToHost, stream));
    CQC_HIP_TRY(hipStreamSynchronize(stream));
    if (top) *top = host.t;
    if (mass) *mass = host.m;
    return Status::ok();
  };
  auto refill = [&](int k) -> Status {
    RecState &rs = recs[k];
    double av = INFINITY;
    int64_t ai = -1;
    if (!rs.cands.empty()) {
      av = rs.cands.back().first;
      ai = rs.cands.back().second;
    }
    CQC_TRY(launch_topk(bins + (int64_t)k * stride, rs.nbins, kTopT, ws + d.topk_off, dev_top, av, ai, stream));
    TopOut top;
    CQC_TRY(fetch(&top, nullptr));
    int got = 0;
    for (int t = 0; t < kTopT; ++t)
      if (top.index[t] != INT64_MAX) {
        rs.cands.push_back({top.value[t], top.index[t]});
        ++got;
      }
    if (got < kTopT) rs.exhausted = true;
    return Status::ok();
  };

  for (int r = 0; r < d.R; ++r) {
    RecState rs;
    int parent = -1;
    int64_t pbin = -1;
    if (r > 0) {
      int best = -1;
      for (int k = 0; k < (int)recs.size(); ++k) {
        RecState &ck = recs[k];
        if (!ck.has_merged) continue;
        if (ck.consumed == ck.cands.size() && !ck.exhausted) {
          st = refill(k);
          if (!st.good()) return st.code;
        }
        if (ck.consumed == ck.cands.size()) continue;
        if (best < 0 || ck.cands[ck.consumed].first > recs[best].cands[recs[best].consumed].first) best = k;
      }
      if (best < 0) break;
      parent = best;
      pbin = recs[best].cands[recs[best].consumed].second;
      recs[best].consumed++;
      const RecState &pr = recs[best];
      rs.depth = pr.depth + 1;
      rs.zoomval = pr.zoomval;
      const auto &pact = d.depths[pr.depth].active;
      const int pa = (int)pact.size();
      for (int t = 0; t < pa; ++t) rs.zoomval[pact[t]] = (int)((pbin >> (pa - 1 - t)) & 1);
    }
    if (rs.depth >= (int)d.depths.size()) break;
    const DepthPlan &dp = d.depths[rs.depth];
    // ---- merge (FP64 accumulate) the entries over the merged qubits
    MergeArgs ma;
    std::memset(&ma, 0, sizeof(ma));
    ma.n = d.cut.nsub;
    int64_t blocks = 0;
    std::vector<const void *> merged(d.cut.nsub);
    for (int c = 0; c < d.cut.nsub; ++c) {
      MergeDesc &md = ma.d[c];
      const int f = d.cut.f[c];
      md.src = inst->entries[c];
      md.dst = ws + dp.merged_off[c];
      merged[c] = md.dst;
      md.rows = int64_t(1) << (2 * d.cut.inc[c].size());
      md.f = f;
      md.n_active = (int)dp.act_local[c].size();
      md.n_merged = (int)dp.mrg_local[c].size();
      std::vector<int> apos, mpos;
      for (int k = md.n_active - 1; k >= 0; --k) apos.push_back(f - 1 - dp.act_local[c][k]);
      for (int k = md.n_merged - 1; k >= 0; --k) mpos.push_back(f - 1 - dp.mrg_local[c][k]);
      md.active_pos = pack_pos(apos);
      md.merged_pos = pack_pos(mpos);
      md.merged_low_contig = 1;
      for (int k = 0; k < md.n_merged; ++k)
        if (mpos[k] != k) md.merged_low_contig = 0;
      int64_t zv = 0;
      for (int j = 0; j < f; ++j) {
        const int q = d.cut.qubits[c][j];
        auto it = rs.zoomval.find(q);
        if (it != rs.zoomval.end() && it->second) zv |= int64_t(1) << (f - 1 - j);
      }
      md.zoom_value = zv;
      md.block_start = blocks;
      const int64_t nout = md.rows << md.n_active;
      blocks += md.n_merged >= 6 ? (nout + 3) / 4 : (nout + 255) / 256;
    }
    st = launch_dd_merge(ma, blocks, in_double, acc_double, stream);
    if (!st.good()) return st.code;
    // ---- term sum onto the 2^#active bins (FP64 output and FP64 bin mass)
    double *brow = bins + (int64_t)r * stride;
    st = run_net(dp.net, ws, merged, brow, true, dev_mass, true, stream);
    if (!st.good()) return st.code;
    rs.has_merged = dp.has_merged;
    rs.nbins = int64_t(1) << dp.active.size();
    // ---- candidates for later zooming
    double mass = 0.0;
    if (dp.has_merged && r + 1 < d.R) {
      st = launch_topk(brow, rs.nbins, kTopT, ws + d.topk_off, dev_top, INFINITY, -1, stream);
      if (!st.good()) return st.code;
      TopOut top;
      st = fetch(&top, &mass);
      if (!st.good()) return st.code;
      int got = 0;
      for (int t = 0; t < kTopT; ++t)
        if (top.index[t] != INT64_MAX) {
          rs.cands.push_back({top.value[t], top.index[t]});
          ++got;
        }
      rs.exhausted = got < kTopT;
    } else {
      st = fetch(nullptr, &mass);
      if (!st.good()) return st.code;
      rs.exhausted = true;
    }
    // ---- record
    cqc_dd_record &rec = records[r];
    std::memset(&rec, 0, sizeof(rec));
    rec.parent_rec = parent;
    rec.parent_bin = pbin;
    rec.n_active = (int32_t)dp.active.size();
    rec.mass = mass;
    for (int q = 0; q < n; ++q) rec.role[q] = -1;
    for (auto &kv : rs.zoomval) rec.role[kv.first] = (int8_t)kv.second;
    for (int q : dp.active) rec.role[q] = -2;
    recs.push_back(std::move(rs));
    *n_done = r + 1;
  }
  return CQC_OK;
}

}  // extern "C"
