// C ABI: dynamic definition (Algorithm 1, Section 4.3), host-driven.
//
// The qubit roles of a recursion depend only on its depth in the zoom tree
// (depth 1: the first active set; depth d+1: the depth-d zoomed and active
// qubits are zoomed, the next n_active un-zoomed qubits in output order are
// active), never on which bin was chosen - only the zoomed VALUES depend on
// the data.  So every depth's contraction plan and workspace are known before
// anything runs; per recursion the host only learns which bin to refine.
//
// Recursions run in rounds: a round picks up to bins_per_round bins from the
// recursions that existed when it began (in the order of the search strategy,
// restricted to the first pick's depth for BFS and to its recursion for DFS),
// enqueues every picked recursion's merge, term sum and top-T back to back,
// and reads all their candidates and masses with one copy and one sync.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>

#include "ddplan.hpp"

namespace cqc {

// >= 0 when pos[j] == pos[0] + j for every j (bit j of a packed index lands at
// position shift + j), -1 otherwise; 0 for an empty list
static int contiguous_shift(const std::vector<int> &pos) {
  for (size_t j = 1; j < pos.size(); ++j)
    if (pos[j] != pos[0] + (int)j) return -1;
  return pos.empty() ? 0 : pos[0];
}

void dd_merge_args(const DdPlan &d, const DepthPlan &dp, const void *const *entries, char *ws, bool in_double,
                   const int64_t *zoom, const int64_t *const *zoom_dev, MergeArgs *ma, int64_t *blocks,
                   std::vector<const void *> *merged) {
  const bool acc_double = d.acc == Acc::F64;
  std::memset(ma, 0, sizeof(*ma));
  *blocks = 0;
  merged->assign(d.cut.nsub, nullptr);
  for (int c = 0; c < d.cut.nsub; ++c) {
    const int f = d.cut.f[c];
    // every bit active, in local order, and no conversion: the merged
    // tensor is the entry tensor itself
    if (dp.mrg_local[c].empty() && (int)dp.act_local[c].size() == f && in_double == acc_double) {
      (*merged)[c] = entries[c];
      continue;
    }
    MergeDesc &md = ma->d[ma->n++];
    md.src = entries[c];
    md.dst = ws + dp.merged_off[c];
    (*merged)[c] = md.dst;
    md.rows = int64_t(1) << (2 * d.cut.inc[c].size());
    md.f = f;
    md.n_active = (int)dp.act_local[c].size();
    md.n_merged = (int)dp.mrg_local[c].size();
    std::vector<int> apos, mpos;
    for (int k = md.n_active - 1; k >= 0; --k) apos.push_back(f - 1 - dp.act_local[c][k]);
    for (int k = md.n_merged - 1; k >= 0; --k) mpos.push_back(f - 1 - dp.mrg_local[c][k]);
    md.active_pos = pack_pos(apos);
    md.merged_pos = pack_pos(mpos);
    md.active_shift = contiguous_shift(apos);
    md.merged_shift = contiguous_shift(mpos);
    md.log_chunks = merge_log_chunks(md.n_merged);
    md.seg = merge_segmented(md.n_merged, md.active_shift, md.merged_shift) ? 1 : 0;
    md.part = md.log_chunks > 0 ? reinterpret_cast<double *>(ws + dp.part_off[c]) : nullptr;
    md.zoom_value = zoom ? zoom[c] : 0;
    md.zoom_dev = zoom_dev ? zoom_dev[c] : nullptr;
    md.block_start = *blocks;
    *blocks += merge_blocks(md.rows << md.n_active, md.n_merged, md.seg != 0);
  }
}

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
    case CQC_PREC_BF16X3: d.acc = Acc::BF16X3; break;
    default: return Status::fail(CQC_ERR_INVALID_ARG, "unknown precision");
  }
  CQC_TRY(validate_cut(&inst->cut, CQC_MAX_DD_QUBITS, &d.cut));
  const int n = d.cut.n;
  if (p->strategy < CQC_DD_HEAVIEST || p->strategy > CQC_DD_BFS)
    return Status::fail(CQC_ERR_INVALID_ARG, "unknown strategy");
  if (p->bins_per_round < 0 || p->bins_per_round > kDdMaxPerRound)
    return Status::fail(CQC_ERR_INVALID_ARG, "bins_per_round must be in [0, 64]");
  d.strategy = p->strategy;
  d.per_round = std::max(1, (int)p->bins_per_round);
  if (p->n_active < 1 || p->n_active > 36) return Status::fail(CQC_ERR_INVALID_ARG, "n_active must be in [1, 36]");
  if (p->bins_f32 != 0 && p->bins_f32 != 1) return Status::fail(CQC_ERR_INVALID_ARG, "bins_f32 must be 0 or 1");
  d.bins_f32 = p->bins_f32 == 1;
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
    dp.part_off.assign(d.cut.nsub, SIZE_MAX);
    for (int c = 0; c < d.cut.nsub; ++c) {
      const size_t nout = (size_t)plan.tensors[c].rows() * ((size_t)1 << dp.act_local[c].size());
      off = align_up(off, 256);
      dp.merged_off[c] = off;
      off += esz * nout;
      const int lc = merge_log_chunks((int)dp.mrg_local[c].size());
      if (lc > 0) {
        off = align_up(off, 256);
        dp.part_off[c] = off;
        off += sizeof(double) * (nout << lc);
      }
    }
    dp.net = layout_net(plan, d.acc, off);
    // a recursion's steps are small (2^a bins at most): prefer more, smaller
    // register tiles so the grid covers the chip (64 x 256 tiles leave most
    // CUs idle below 2^22 outputs)
    for (size_t i = 0; i < dp.net.tile.size(); ++i) {
      const Step &st = dp.net.plan.steps[i];
      const int64_t M = int64_t(1) << st.logM, N = int64_t(1) << st.logN;
      if (dp.net.tile[i] == kTileL && M * N * st.nbatch < (int64_t(1) << 22) && M >= 32 && N >= 128) {
        dp.net.tile[i] = kTileM;
        const TileShape sh = tile_shape(kTileM);
        dp.net.nblocks[i] = ((M + sh.bm - 1) / sh.bm) * ((N + sh.bn - 1) / sh.bn) * st.nbatch;
      }
    }
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
  d.bytes = align_up(d.out_off + sizeof(DdSlot) * (size_t)d.per_round, 256);
  *out = std::move(d);
  return Status::ok();
}

namespace {
// Page-locked host buffers for the per-round read-back of the selected bins:
// a device-to-host copy into pinned memory goes straight to its destination,
// without the runtime's staging copy for pageable memory.  One buffer per
// concurrent query, taken from a process-wide free list and returned when
// the query ends; the buffers are kept until the process exits.
class PinnedSlots {
 public:
  PinnedSlots() {
    {
      std::lock_guard<std::mutex> g(mu());
      if (!pool().empty()) {
        p_ = pool().back();
        pool().pop_back();
        return;
      }
    }
    void *v = nullptr;
    if (hipHostMalloc(&v, sizeof(DdSlot) * kDdMaxPerRound, hipHostMallocDefault) == hipSuccess) {
      p_ = static_cast<DdSlot *>(v);
    } else {
      (void)hipGetLastError();
      fallback_.resize(kDdMaxPerRound);   // pageable: slower read-back, same results
    }
  }
  ~PinnedSlots() {
    if (!p_) return;
    std::lock_guard<std::mutex> g(mu());
    pool().push_back(p_);
  }
  PinnedSlots(const PinnedSlots &) = delete;
  PinnedSlots &operator=(const PinnedSlots &) = delete;
  DdSlot &operator[](size_t i) { return p_ ? p_[i] : fallback_[i]; }
  DdSlot *data() { return p_ ? p_ : fallback_.data(); }

 private:
  static std::mutex &mu() {
    static std::mutex m;
    return m;
  }
  static std::vector<DdSlot *> &pool() {
    static auto *v = new std::vector<DdSlot *>();   // never destroyed: used until exit
    return *v;
  }
  DdSlot *p_ = nullptr;
  std::vector<DdSlot> fallback_;
};

struct RecState {
  int depth = 0;
  int round = 0;
  std::map<int, int> zoomval;        // qubit -> 0/1
  std::vector<std::pair<double, int64_t>> cands;
  size_t consumed = 0;
  bool exhausted = false;
  bool has_merged = false;
  int64_t nbins = 0;
};
}  // namespace

// Plans of recent calls, keyed by every input that determines them (the cut,
// dtypes, precision and parameters): a repeated query skips re-planning every
// depth.  Only successful builds are stored; the cache is bounded and guarded.
static bool dd_key(const cqc_instance *inst, cqc_dtype in_t, cqc_precision prec, const cqc_dd_params *p,
                   std::vector<int64_t> *key) {
  if (!inst || !p) return false;
  const cqc_cut &c = inst->cut;
  if (c.n_qubits < 0 || c.n_qubits > CQC_MAX_DD_QUBITS || c.n_sub < 0 || c.n_sub > CQC_MAX_SUB || c.n_cuts < 0 ||
      c.n_cuts > CQC_MAX_CUTS || !c.f || !c.out_qubit || (c.n_cuts > 0 && (!c.edge_up || !c.edge_down)))
    return false;
  if (p->n_active < 1 || p->n_active > 36 || (p->first_active && p->n_active > c.n_qubits)) return false;
  key->assign({c.n_qubits, c.n_sub, c.n_cuts, (int64_t)in_t, (int64_t)prec, p->n_active, p->n_recursions,
               p->strategy, p->bins_per_round, p->bins_f32, p->first_active ? 1 : 0});
  for (int i = 0; i < c.n_sub; ++i) key->push_back(c.f[i]);
  for (int e = 0; e < c.n_cuts; ++e) {
    key->push_back(c.edge_up[e]);
    key->push_back(c.edge_down[e]);
  }
  for (int q = 0; q < c.n_qubits; ++q) key->push_back(c.out_qubit[q]);
  if (p->first_active)
    for (int i = 0; i < p->n_active; ++i) key->push_back(p->first_active[i]);
  return true;
}

Status cached_dd(const cqc_instance *inst, cqc_dtype in_t, cqc_precision prec, const cqc_dd_params *p,
                 std::shared_ptr<const DdPlan> *out) {
  static std::mutex mu;
  static std::map<std::vector<int64_t>, std::shared_ptr<const DdPlan>> cache;
  std::vector<int64_t> key;
  const bool keyed = dd_key(inst, in_t, prec, p, &key);
  if (keyed) {
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(key);
    if (it != cache.end()) {
      *out = it->second;
      return Status::ok();
    }
  }
  auto plan = std::make_shared<DdPlan>();
  CQC_TRY(build_dd(inst, in_t, prec, p, plan.get()));
  if (keyed) {
    std::lock_guard<std::mutex> g(mu);
    if (cache.size() >= 64) cache.clear();
    cache[key] = plan;
  }
  *out = std::move(plan);
  return Status::ok();
}

}  // namespace cqc

using namespace cqc;

extern "C" {

int cqc_dd_workspace_size(const cqc_instance *inst, cqc_dtype in_t, cqc_precision prec,
                          const cqc_dd_params *p, size_t *bytes) {
  if (!bytes) return Status::fail(CQC_ERR_INVALID_ARG, "bytes is NULL").code;
  std::shared_ptr<const DdPlan> plan;
  Status st = cached_dd(inst, in_t, prec, p, &plan);
  if (!st.good()) return st.code;
  *bytes = plan->bytes;
  return CQC_OK;
}

int cqc_reconstruct_dd(const cqc_instance *inst, cqc_dtype in_t, cqc_precision prec,
                       const cqc_dd_params *p, void *bins_v, cqc_dd_record *records,
                       int32_t *n_done, void *workspace, size_t ws_bytes, hipStream_t stream) {
  std::shared_ptr<const DdPlan> plan;
  Status st = cached_dd(inst, in_t, prec, p, &plan);
  if (!st.good()) return st.code;
  const DdPlan &d = *plan;
  if (!bins_v || !records || !n_done) return Status::fail(CQC_ERR_INVALID_ARG, "bins, records or n_done is NULL").code;
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
  const size_t bin_size = d.bins_f32 ? 4 : 8;
  char *bins = static_cast<char *>(bins_v);
  auto bin_row = [&](int64_t r) { return bins + (size_t)r * (size_t)stride * bin_size; };
  DdSlot *dev_slots = reinterpret_cast<DdSlot *>(ws + d.out_off);
  PinnedSlots host_slots;   // d.per_round <= kDdMaxPerRound slots
  std::vector<RecState> recs;
  *n_done = 0;

  auto fetch = [&](int count) -> Status {
    CQC_HIP_TRY(hipMemcpyAsync(host_slots.data(), dev_slots, sizeof(DdSlot) * count, hipMemcpyDeviceToHost,
                               stream));
    CQC_HIP_TRY(hipStreamSynchronize(stream));
    return Status::ok();
  };
  auto take = [&](RecState &rs, const TopOut &top) {
    int got = 0;
    for (int t = 0; t < kTopT; ++t)
      if (top.index[t] != INT64_MAX) {
        rs.cands.push_back({top.value[t], top.index[t]});
        ++got;
      }
    rs.exhausted = got < kTopT;
  };
  // the next candidates of recursion k, ranked after the ones already taken
  auto refill = [&](int k) -> Status {
    RecState &rs = recs[k];
    const double av = rs.cands.back().first;
    const int64_t ai = rs.cands.back().second;
    CQC_TRY(launch_topk(bin_row(k), d.bins_f32, rs.nbins, kTopT, ws + d.topk_off, &dev_slots[0].top, av, ai,
                        stream));
    CQC_TRY(fetch(1));
    take(rs, host_slots[0].top);
    return Status::ok();
  };
  // does recursion k (of the round's first `start`) have a candidate left?
  auto available = [&](int k, Status &err) -> bool {
    RecState &rk = recs[k];
    if (!rk.has_merged) return false;
    if (rk.consumed == rk.cands.size() && !rk.exhausted) {
      err = refill(k);
      if (!err.good()) return false;
    }
    return rk.consumed < rk.cands.size();
  };
  auto top_of = [&](int k) { return recs[k].cands[recs[k].consumed].first; };
  // the strategy's next pick among recursions [0, start), or -1
  auto choose = [&](int start, int restrict_val, Status &err) -> int {
    int best = -1;
    if (d.strategy == CQC_DD_DFS) {
      // the latest round with a candidate, and in it the earliest pick
      // (rounds never decrease along the records)
      for (int k = start - 1; k >= 0; --k) {
        if (best >= 0 && recs[k].round < recs[best].round) break;
        if (restrict_val >= 0 && k != restrict_val) continue;
        if (available(k, err)) best = k;
        if (!err.good()) return -1;
      }
      return best;
    }
    int best_depth = INT_MAX;
    for (int k = 0; k < start; ++k) {
      if (d.strategy == CQC_DD_BFS && restrict_val >= 0 && recs[k].depth != restrict_val) continue;
      if (!available(k, err)) {
        if (!err.good()) return -1;
        continue;
      }
      const int dk = d.strategy == CQC_DD_BFS ? recs[k].depth : 0;
      if (best < 0 || dk < best_depth || (dk == best_depth && top_of(k) > top_of(best))) {
        best = k;
        best_depth = dk;
      }
    }
    return best;
  };

  int r = 0, round = 0;
  while (r < d.R) {
    // ---- picks of this round
    std::vector<std::pair<int, int64_t>> picks;
    if (r == 0) {
      picks.push_back({-1, -1});
    } else {
      const int start = (int)recs.size();
      const int lim = std::min(d.per_round, d.R - r);
      int restrict_val = -1;
      while ((int)picks.size() < lim) {
        Status err = Status::ok();
        const int k = choose(start, restrict_val, err);
        if (!err.good()) return err.code;
        if (k < 0) break;
        picks.push_back({k, recs[k].cands[recs[k].consumed].second});
        recs[k].consumed++;
        if (restrict_val < 0 && d.strategy == CQC_DD_DFS) restrict_val = k;
        if (restrict_val < 0 && d.strategy == CQC_DD_BFS) restrict_val = recs[k].depth;
      }
      if (picks.empty()) break;
    }
    // ---- enqueue every picked recursion
    std::vector<RecState> fresh;
    for (size_t i = 0; i < picks.size(); ++i) {
      RecState rs;
      rs.round = round;
      const int parent = picks[i].first;
      const int64_t pbin = picks[i].second;
      if (parent >= 0) {
        const RecState &pr = recs[parent];
        rs.depth = pr.depth + 1;
        rs.zoomval = pr.zoomval;
        const auto &pact = d.depths[pr.depth].active;
        const int pa = (int)pact.size();
        for (int t = 0; t < pa; ++t) rs.zoomval[pact[t]] = (int)((pbin >> (pa - 1 - t)) & 1);
      }
      if (rs.depth >= (int)d.depths.size())
        return Status::fail(CQC_ERR_UNSUPPORTED, "dynamic definition: no plan for a picked depth").code;
      const DepthPlan &dp = d.depths[rs.depth];
      // merge (FP64 accumulate) the entries over the merged qubits
      MergeArgs ma;
      int64_t blocks = 0;
      std::vector<const void *> merged;
      std::vector<int64_t> zoomv(d.cut.nsub, 0);
      for (int c = 0; c < d.cut.nsub; ++c) {
        const int f = d.cut.f[c];
        for (int j = 0; j < f; ++j) {
          auto it = rs.zoomval.find(d.cut.qubits[c][j]);
          if (it != rs.zoomval.end() && it->second) zoomv[c] |= int64_t(1) << (f - 1 - j);
        }
      }
      dd_merge_args(d, dp, inst->entries, ws, in_double, zoomv.data(), nullptr, &ma, &blocks, &merged);
      st = launch_dd_merge(ma, blocks, in_double, acc_double, stream);
      if (!st.good()) return st.code;
      // term sum onto the 2^#active bins (FP64 or FP32 output, FP64 bin mass)
      char *brow = bin_row(r + (int64_t)i);
      st = run_net(dp.net, ws, merged, brow, !d.bins_f32, &dev_slots[i].mass, true, stream);
      if (!st.good()) return st.code;
      rs.has_merged = dp.has_merged;
      rs.nbins = int64_t(1) << dp.active.size();
      // candidates for later zooming
      if (dp.has_merged && r + (int)i + 1 < d.R) {
        st = launch_topk(brow, d.bins_f32, rs.nbins, kTopT, ws + d.topk_off, &dev_slots[i].top, INFINITY, -1,
                         stream);
        if (!st.good()) return st.code;
      } else {
        rs.exhausted = true;
      }
      fresh.push_back(std::move(rs));
    }
    // ---- one read-back for the round
    st = fetch((int)picks.size());
    if (!st.good()) return st.code;
    for (size_t i = 0; i < picks.size(); ++i) {
      RecState &rs = fresh[i];
      const DepthPlan &dp = d.depths[rs.depth];
      if (!rs.exhausted) take(rs, host_slots[i].top);
      cqc_dd_record &rec = records[r + i];
      std::memset(&rec, 0, sizeof(rec));
      rec.parent_rec = picks[i].first;
      rec.parent_bin = picks[i].second;
      rec.n_active = (int32_t)dp.active.size();
      rec.mass = host_slots[i].mass;
      for (int q = 0; q < n; ++q) rec.role[q] = -1;
      for (auto &kv : rs.zoomval) rec.role[kv.first] = (int8_t)kv.second;
      for (int q : dp.active) rec.role[q] = -2;
      recs.push_back(std::move(rs));
    }
    r += (int)picks.size();
    ++round;
    *n_done = r;
  }
  return CQC_OK;
}

}  // extern "C"
