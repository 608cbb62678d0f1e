// C ABI: adjoint of a prepared batch - gradients of a loss on every
// instance's reconstructed distribution with respect to its entry tensors -
// in a fixed handful of launches.
//
// The forward operands are the ones the batch's last run left in its
// workspace (converted entries and intermediates), so nothing is recomputed.
// Adjoint steps are taken in reverse plan order as levels (level 0: every
// instance's last step).  Within a level the dX and dY work of all instances
// is grouped by kernel shape, and each group is one persistent launch
// draining an atomic (step, block) queue, largest steps first; then one
// launch per level adds every step's split-K partials in a fixed order,
// straight into the caller's gradient buffers for entry tensors and into this
// workspace for intermediates (the dL/dZ of the next level).  A first launch
// zeroes the queue counters and gathers dL/dp of the instances whose output
// order is not blocked.  The tables are uploaded once by
// cqc_batch_backward_create; cqc_batch_backward_run only enqueues kernels.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <tuple>

#include "batch.hpp"
#include "bwd.hpp"

struct cqc_batch_bwd_s {
  cqc::Acc acc = cqc::Acc::F32;
  const cqc::BwdGatherDesc *gather = nullptr;
  const int64_t *gather_start = nullptr;
  int32_t n_gather = 0;
  int64_t gather_blocks = 0;
  unsigned long long *counters = nullptr;
  int32_t n_counters = 0;
  struct Level {
    std::vector<cqc::BwdQueue> queues;
    const cqc::BwdReduceDesc *red = nullptr;
    const int64_t *red_start = nullptr;
    int32_t n_red = 0;
    int64_t red_blocks = 0;
  };
  std::vector<Level> levels;
};

namespace cqc {

static constexpr uint32_t kBwdQueueGrid = 2048;
// Smallest split-K partials budget per step side: a batch already has its
// parallelism across instances, so small steps are not split further.
static constexpr double kBatchBwdMinBudget = 1.0 * (1 << 20);
// Partials budget per step side as a fraction of its dL/dZ bytes.  Measured
// on the 256-instance training step: the dX launches took 0.65 ms at 1/4,
// 0.59 at 1/16 (longer inner chunks, fewer partial sums to write and add),
// 0.88 at 1/32 (too few blocks); the dY launches were fastest at 1/4 (0.54 ms
// against 0.59 at 1/2 and 0.56 at 1/16).
static constexpr double kBatchBwdFracX = 1.0 / 16, kBatchBwdFracY = 0.25;

struct BwdBuild {
  size_t bytes = 0, tables_off = 0;
  std::vector<BwdGatherDesc> gathers;
  struct QG {
    int level;
    bool y, dual;
    int sb;
    std::vector<std::pair<int64_t, BwdArgs>> steps;   // (blocks, args)
  };
  std::vector<QG> groups;
  std::vector<std::vector<BwdReduceDesc>> red;         // per level
  size_t gather_off = 0, gstart_off = 0, counter_off = 0;
  std::vector<size_t> desc_off, prefix_off, red_off, rstart_off;
};

static int64_t blocks_of(int64_t elems) { return (elems + 255) / 256; }

// Sizes and (with need_ptrs) addresses of one batch's adjoint; pointers are
// relative to `ws` (nullptr: sizes only).
static Status build_bwd(const cqc_batch_s *bt, const void *const *gout, void *const *const *gents,
                        bool need_ptrs, char *ws, BwdBuild *out) {
  BwdBuild B;
  const Acc acc = bt->acc == Acc::F64 ? Acc::F64 : Acc::F32;   // BF16X6 batches: FP32 adjoint
  const bool acc_double = acc == Acc::F64;
  const size_t esz = acc_double ? 8 : 4;
  size_t off = 0;
  std::map<std::tuple<int, int, int>, size_t> gidx;
  for (size_t i = 0; i < bt->plans.size(); ++i) {
    const FdInstancePlan &ip = bt->plans[i];
    const NetLayout &L = ip.net;
    const Plan &p = L.plan;
    const std::string who = "instance " + std::to_string(i) + ": ";
    if (need_ptrs) {
      if (!gout[i]) return Status::fail(CQC_ERR_INVALID_ARG, who + "grad_out is NULL");
      if (!gents[i]) return Status::fail(CQC_ERR_INVALID_ARG, who + "grad_entries is NULL");
      for (int c = 0; c < ip.cut.nsub; ++c)
        if (!gents[i][c]) return Status::fail(CQC_ERR_INVALID_ARG, who + "gradient " + std::to_string(c) + " is NULL");
    }
    // forward operands, as the batch's run left them
    std::vector<const void *> tptr(p.tensors.size(), nullptr);
    for (size_t t = 0; t < p.tensors.size(); ++t) {
      const auto &T = p.tensors[t];
      if (T.entry >= 0)
        tptr[t] = ip.conv_off[T.entry] != SIZE_MAX ? bt->ws + ip.conv_off[T.entry] : bt->entry_src[i][T.entry];
      else
        tptr[t] = bt->ws + L.t_off[t];
    }
    // dL/dp of the last step in blocked order
    const Step &last = p.steps.back();
    const void *g = need_ptrs ? gout[i] : nullptr;
    if (!is_blocked(p, last)) {
      off = align_up(off, 256);
      BwdGatherDesc d;
      std::memset(&d, 0, sizeof(d));
      d.src = g;
      d.dst = ws + off;
      d.logM = last.logM;
      d.logN = last.logN;
      const auto &X = p.tensors[last.x], &Y = p.tensors[last.y];
      const int nX = (int)X.bits.size(), nY = (int)Y.bits.size();
      std::vector<int> px(nX), py(nY);
      for (int j = 0; j < nX; ++j) px[j] = p.bitpos[X.bits[nX - 1 - j]];
      for (int j = 0; j < nY; ++j) py[j] = p.bitpos[Y.bits[nY - 1 - j]];
      d.px = pack_pos(px);
      d.py = pack_pos(py);
      B.gathers.push_back(d);
      g = ws + off;
      off += esz * ((size_t)1 << ip.cut.n);
    }
    // dL/dZ of the intermediates
    std::vector<size_t> dz_off(p.tensors.size(), SIZE_MAX);
    for (size_t s = 0; s + 1 < p.steps.size(); ++s) {
      const TensorSpec &Z = p.tensors[p.steps[s].z];
      off = align_up(off, 256);
      dz_off[p.steps[s].z] = off;
      off += esz * (size_t)Z.rows() * (size_t)Z.cols();
    }
    // split-K choice per step side, and one partials region per side sized for
    // the largest step (levels run one after the other)
    std::vector<BwdSide> sx, sy;
    std::vector<char> dual;
    size_t px_bytes = 0, py_bytes = 0;
    for (const Step &st : p.steps) {
      const TensorSpec &X = p.tensors[st.x], &Y = p.tensors[st.y];
      const int64_t M = int64_t(1) << st.logM, N = int64_t(1) << st.logN;
      const int64_t dz = st.nbatch * M * N;
      const int64_t RXn = int64_t(1) << (2 * st.RX.size()), RYn = int64_t(1) << (2 * st.RY.size());
      // steps of at most 16 labels: both sides in one pass over dL/dZ
      const bool d2 = bwd_dual_ok((int)st.S.size(), M, N, !acc_double) && X.entry != -2 && Y.entry != -2;
      dual.push_back(d2);
      if (d2) {
        BwdSide bx, by;
        bx.kChunk = std::min<int64_t>(N, kDualChunk);
        bx.kChunks = (int32_t)((N + bx.kChunk - 1) / bx.kChunk);
        bx.P = RYn * bx.kChunks;
        by.kChunk = kDualRows;
        by.kChunks = (int32_t)((M + kDualRows - 1) / kDualRows);
        by.P = RXn * by.kChunks;
        sx.push_back(bx);
        sy.push_back(by);
      } else {
        sx.push_back(choose_bwd_side(N, RYn, X.rows() * M, dz, esz, kBatchBwdMinBudget, kBatchBwdFracX));
        sy.push_back(choose_bwd_side(M, RXn, Y.rows() * N, dz, esz, kBatchBwdMinBudget, kBatchBwdFracY));
      }
      px_bytes = std::max(px_bytes, esz * (size_t)(sx.back().P * X.rows() * M));
      py_bytes = std::max(py_bytes, esz * (size_t)(sy.back().P * Y.rows() * N));
    }
    off = align_up(off, 256);
    const size_t px_off = off;
    off = align_up(off + px_bytes, 256);
    const size_t py_off = off;
    off = align_up(off + py_bytes, 256);
    for (int s = (int)p.steps.size() - 1; s >= 0; --s) {
      const Step &st = p.steps[s];
      const bool is_last = s + 1 == (int)p.steps.size();
      const int level = (int)p.steps.size() - 1 - s;
      if ((int)B.red.size() <= level) B.red.resize(level + 1);
      BwdArgs a;
      std::memset(&a, 0, sizeof(a));
      a.X = tptr[st.x];
      a.Y = tptr[st.y];
      a.dZ = is_last ? g : ws + dz_off[st.z];
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
      if (dual[s]) {
        a.part = ws + px_off;
        a.kChunk = sx[s].kChunk;
        a.kChunks = sx[s].kChunks;
        a.part2 = ws + py_off;
        a.kChunks2 = sy[s].kChunks;
        const auto key = std::make_tuple(level, 2, 1);
        auto it = gidx.find(key);
        if (it == gidx.end()) {
          it = gidx.emplace(key, B.groups.size()).first;
          BwdBuild::QG q;
          q.level = level;
          q.y = false;
          q.dual = true;
          q.sb = 1;
          B.groups.push_back(q);
        }
        B.groups[it->second].steps.push_back({bwd_dual_blocks(a, st.nbatch), a});
      }
      for (int side = 0; side < 2; ++side) {
        const int t = side == 0 ? st.x : st.y;
        const TensorSpec &T = p.tensors[t];
        if (T.entry == -2) continue;   // unit tensor of a single subcircuit
        const BwdSide &bs = side == 0 ? sx[s] : sy[s];
        if (!dual[s]) {
          a.part = ws + (side == 0 ? px_off : py_off);
          a.kChunk = bs.kChunk;
          a.kChunks = bs.kChunks;
          const auto key = std::make_tuple(level, side, bwd_sb(a.nS, side == 1, !acc_double));
          auto it = gidx.find(key);
          if (it == gidx.end()) {
            it = gidx.emplace(key, B.groups.size()).first;
            BwdBuild::QG q;
            q.level = level;
            q.y = side == 1;
            q.dual = false;
            q.sb = bwd_sb(a.nS, side == 1, !acc_double);
            B.groups.push_back(q);
          }
          B.groups[it->second].steps.push_back({bwd_blocks(a, side == 1, !acc_double), a});
        }
        BwdReduceDesc r;
        std::memset(&r, 0, sizeof(r));
        r.part = ws + (side == 0 ? px_off : py_off);
        r.count = T.rows() * (side == 0 ? M : N);
        r.P = bs.P;
        r.scale = scale;
        if (T.entry >= 0) {
          r.out = need_ptrs ? gents[i][T.entry] : nullptr;
          r.out_double = bt->in_double ? 1 : 0;
        } else {
          r.out = ws + dz_off[t];
          r.out_double = acc_double ? 1 : 0;
        }
        r.vec = !acc_double && r.count % 4 == 0 && reinterpret_cast<uintptr_t>(r.out) % 16 == 0 ? 1 : 0;
        B.red[level].push_back(r);
      }
    }
  }
  std::stable_sort(B.groups.begin(), B.groups.end(),
                   [](const BwdBuild::QG &x, const BwdBuild::QG &y) { return x.level < y.level; });
  for (auto &q : B.groups)
    std::stable_sort(q.steps.begin(), q.steps.end(),
                     [](const std::pair<int64_t, BwdArgs> &x, const std::pair<int64_t, BwdArgs> &y) {
                       return x.first > y.first;
                     });
  if (B.groups.size() > 256) return Status::fail(CQC_ERR_UNSUPPORTED, "too many distinct adjoint step shapes");
  // tables after the instance regions
  off = align_up(off, 256);
  B.tables_off = off;
  B.gather_off = off;
  off = align_up(off + sizeof(BwdGatherDesc) * B.gathers.size(), 256);
  B.gstart_off = off;
  off = align_up(off + sizeof(int64_t) * (B.gathers.size() + 1), 256);
  B.counter_off = off;
  off = align_up(off + sizeof(unsigned long long) * std::max<size_t>(1, B.groups.size()), 256);
  for (auto &q : B.groups) {
    B.desc_off.push_back(off);
    off = align_up(off + sizeof(BwdArgs) * q.steps.size(), 256);
    B.prefix_off.push_back(off);
    off = align_up(off + sizeof(int64_t) * (q.steps.size() + 1), 256);
  }
  for (auto &r : B.red) {
    B.red_off.push_back(off);
    off = align_up(off + sizeof(BwdReduceDesc) * r.size(), 256);
    B.rstart_off.push_back(off);
    off = align_up(off + sizeof(int64_t) * (r.size() + 1), 256);
  }
  B.bytes = off;
  *out = std::move(B);
  return Status::ok();
}

static Status bwd_create(cqc_batch_s *bt, const void *const *gout, void *const *const *gents, void *workspace,
                         size_t ws_bytes, hipStream_t s, cqc_batch_bwd_s **out) {
  if (!gout || !gents) return Status::fail(CQC_ERR_INVALID_ARG, "gradient arrays are NULL");
  char *ws = static_cast<char *>(workspace);
  BwdBuild B;
  CQC_TRY(build_bwd(bt, gout, gents, true, ws, &B));
  if (!workspace || ws_bytes < B.bytes)
    return Status::fail(CQC_ERR_WORKSPACE, "workspace needs " + std::to_string(B.bytes) + " bytes");
  if (reinterpret_cast<uintptr_t>(workspace) % 256)
    return Status::fail(CQC_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  std::vector<char> img(B.bytes - B.tables_off, 0);
  auto put = [&](size_t off, const void *src, size_t n) {
    if (n) std::memcpy(img.data() + (off - B.tables_off), src, n);
  };
  auto *h = new cqc_batch_bwd_s();
  h->acc = bt->acc == Acc::F64 ? Acc::F64 : Acc::F32;
  // gathers
  std::vector<int64_t> gstart(1, 0);
  for (auto &d : B.gathers) gstart.push_back(gstart.back() + blocks_of(int64_t(1) << (d.logM + d.logN)));
  put(B.gather_off, B.gathers.data(), sizeof(BwdGatherDesc) * B.gathers.size());
  put(B.gstart_off, gstart.data(), sizeof(int64_t) * gstart.size());
  h->gather = reinterpret_cast<const BwdGatherDesc *>(ws + B.gather_off);
  h->gather_start = reinterpret_cast<const int64_t *>(ws + B.gstart_off);
  h->n_gather = (int32_t)B.gathers.size();
  h->gather_blocks = gstart.back();
  h->counters = reinterpret_cast<unsigned long long *>(ws + B.counter_off);
  h->n_counters = (int32_t)B.groups.size();
  h->levels.resize(B.red.size());
  for (size_t q = 0; q < B.groups.size(); ++q) {
    const auto &G = B.groups[q];
    std::vector<BwdArgs> descs;
    std::vector<int64_t> prefix(1, 0);
    for (auto &st : G.steps) {
      descs.push_back(st.second);
      prefix.push_back(prefix.back() + st.first);
    }
    put(B.desc_off[q], descs.data(), sizeof(BwdArgs) * descs.size());
    put(B.prefix_off[q], prefix.data(), sizeof(int64_t) * prefix.size());
    BwdQueue bq;
    bq.y = G.y;
    bq.dual = G.dual;
    bq.sb = G.sb;
    bq.descs = reinterpret_cast<const BwdArgs *>(ws + B.desc_off[q]);
    bq.prefix = reinterpret_cast<const int64_t *>(ws + B.prefix_off[q]);
    bq.ndesc = (int)descs.size();
    bq.queue = h->counters + q;
    bq.total = prefix.back();
    bq.grid = (uint32_t)std::min<int64_t>(bq.total, kBwdQueueGrid);
    h->levels[G.level].queues.push_back(bq);
  }
  for (size_t l = 0; l < B.red.size(); ++l) {
    std::vector<int64_t> rstart(1, 0);
    for (auto &r : B.red[l]) rstart.push_back(rstart.back() + bwd_reduce_blocks(r));
    put(B.red_off[l], B.red[l].data(), sizeof(BwdReduceDesc) * B.red[l].size());
    put(B.rstart_off[l], rstart.data(), sizeof(int64_t) * rstart.size());
    h->levels[l].red = reinterpret_cast<const BwdReduceDesc *>(ws + B.red_off[l]);
    h->levels[l].red_start = reinterpret_cast<const int64_t *>(ws + B.rstart_off[l]);
    h->levels[l].n_red = (int32_t)B.red[l].size();
    h->levels[l].red_blocks = rstart.back();
  }
  hipError_t e = hipMemcpyAsync(ws + B.tables_off, img.data(), img.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    delete h;
    return Status::fail(CQC_ERR_HIP, std::string("uploading adjoint tables: ") + hipGetErrorString(e));
  }
  *out = h;
  return Status::ok();
}

static Status bwd_run(const cqc_batch_bwd_s *h, hipStream_t s) {
  CQC_TRY(launch_bwd_prep(h->acc, h->gather, h->gather_start, h->n_gather, h->gather_blocks, h->counters,
                          h->n_counters, s));
  for (const auto &L : h->levels) {
    for (const auto &q : L.queues) CQC_TRY(launch_bwd_queue(h->acc, q, s));
    CQC_TRY(launch_bwd_reduce_table(h->acc, L.red, L.red_start, L.n_red, L.red_blocks, s));
  }
  return Status::ok();
}

}  // namespace cqc

using namespace cqc;

extern "C" {

int cqc_batch_backward_workspace_size(cqc_batch batch, size_t *bytes) {
  if (!batch) return Status::fail(CQC_ERR_INVALID_ARG, "batch is NULL").code;
  if (!bytes) return Status::fail(CQC_ERR_INVALID_ARG, "bytes is NULL").code;
  BwdBuild B;
  Status st = build_bwd(batch, nullptr, nullptr, false, nullptr, &B);
  if (!st.good()) return st.code;
  *bytes = B.bytes;
  return CQC_OK;
}

int cqc_batch_backward_create(cqc_batch batch, const void *const *grad_out, void *const *const *grad_entries,
                              void *workspace, size_t ws_bytes, hipStream_t stream, cqc_batch_bwd *out) {
  if (!batch) return Status::fail(CQC_ERR_INVALID_ARG, "batch is NULL").code;
  if (!out) return Status::fail(CQC_ERR_INVALID_ARG, "out is NULL").code;
  cqc_batch_bwd_s *h = nullptr;
  Status st = bwd_create(batch, grad_out, grad_entries, workspace, ws_bytes, stream, &h);
  if (!st.good()) return st.code;
  *out = h;
  return CQC_OK;
}

int cqc_batch_backward_run(cqc_batch_bwd b, hipStream_t stream) {
  if (!b) return Status::fail(CQC_ERR_INVALID_ARG, "handle is NULL").code;
  return bwd_run(b, stream).code;
}

int cqc_batch_backward_destroy(cqc_batch_bwd b) {
  delete b;
  return CQC_OK;
}

}  // extern "C"
