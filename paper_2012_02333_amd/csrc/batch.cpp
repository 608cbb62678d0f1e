// Batched full-definition reconstruction: many independent instances of
// uneven shape in a handful of launches.
//
// All steps of all instances are grouped by (plan level, kernel variant,
// output mode, tile shape).  Intermediate levels run first, then the final
// steps; every group is one persistent launch draining an atomic (step, tile)
// queue whose steps are ordered most expensive first.  One launch computes the
// entry row flags of every instance (and zeroes the queue counters), one adds
// up every instance's FP64 mass.  The descriptor tables live in the caller's
// workspace and are uploaded once by cqc_batch_create; cqc_batch_run only
// enqueues kernels, so it can be captured in a HIP graph and replayed.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <tuple>

#include "batch.hpp"

namespace cqc {

static constexpr int kFinalLevel = 1 << 20;

// Cross-entropy binding of a batch (cqc_batch_create_xent): per instance the
// target, the gradient buffer and an optional loss (host arrays of device
// pointers).
struct XentBind {
  const void *const *targets;
  void *const *grads;
  double *const *losses;
};
static constexpr uint32_t kQueueGrid = 2048;

struct BatchBuild {
  std::vector<FdInstancePlan> plans;
  Acc acc;
  size_t tables_off = 0, bytes = 0;
  // host images of the tables
  std::vector<FlagDesc> flags;
  int64_t flag_blocks = 0;
  std::vector<MassDesc> mass;
  struct G {
    int level, mode, cfg;
    bool small, strip;
    int xent;
    Acc acc;
    std::vector<std::pair<double, ContractArgs>> steps;  // (cost, args)
  };
  std::vector<G> groups;
  size_t flag_off = 0, mass_off = 0, counter_off = 0;
  std::vector<size_t> desc_off, prefix_off, bprefix_off;
};

// Tile of a step in a batched launch: the autotuner's choice for the step's
// shape class (the cache single calls consult) where a queue kernel has that
// tile and the operands fit it, else the built-in rule.  The queue kernels
// have no 256 x 16 form; its steps take the 16 x 64 tile.
// In a work-queue launch the wide kernel's tiles share the launch with those
// of every other step of its group, so a step with few tiles does not leave
// the chip idle (which is why a single call keeps the register kernel below
// 2^22 outputs): FP32 steps of three or more shared cuts with both operands at
// least 128 wide take the wide kernel from 2^kBatchWideLog outputs.  Measured
// on the 256-instance training step: 4.01 ms per step with 2^22, 3.97 with
// 2^20, 3.94 with 2^19, 3.96 with 2^17 and 2^18.  Such a step's outputs then
// differ from the single call's by FP32 rounding (another product order).
static constexpr int kBatchWideLog = 19;
static int queue_cfg(Acc acc, const Step &st, int mode, bool out_double) {
  const Acc sa = step_acc(acc, st.wide_ok(), (int)st.S.size());
  const int nS = (int)st.S.size();
  int c = choose_tile(sa, nS, st.logM, st.logN, st.wide_ok(), st.nbatch);
  if (sa == Acc::F32 && st.wide_ok() && nS >= 3 && st.logM >= 7 && st.logN >= 7 &&
      (int64_t(1) << (st.logM + st.logN)) * st.nbatch >= (int64_t(1) << kBatchWideLog))
    c = kTileW;
  int tc = 0, xcd = 0;
  if (tuned_choice(sa, mode, nS <= 2, st.logM, st.logN, nS, out_double, &tc, &xcd) && tile_ok(sa, tc) &&
      (tc != kTileW || st.wide_ok()))
    c = tc;
  return c == kTileT ? kTileS : c;
}

// Builds the groups with pointers relative to `ws` (nullptr: sizes only).
static Status build_batch(const cqc_instance *inst, int32_t n_inst, cqc_dtype in_t, cqc_dtype out_t,
                          cqc_precision prec, bool need_ptrs, char *ws, BatchBuild *out,
                          const XentBind *xent = nullptr) {
  BatchBuild B;
  CQC_TRY(fd_plans(inst, n_inst, in_t, out_t, prec, need_ptrs, &B.plans, &B.acc, xent != nullptr));
  if (xent && need_ptrs) {
    if (!xent->targets || !xent->grads) return Status::fail(CQC_ERR_INVALID_ARG, "targets or grads is NULL");
    for (int32_t i = 0; i < n_inst; ++i) {
      const std::string who = "instance " + std::to_string(i) + ": ";
      if (!xent->targets[i] || !xent->grads[i])
        return Status::fail(CQC_ERR_INVALID_ARG, who + "target or gradient pointer is NULL");
      if (xent->losses && xent->losses[i] && inst[i].mass)
        return Status::fail(CQC_ERR_INVALID_ARG, who + "a loss and a mass cannot both be asked for");
    }
  }
  const bool acc_double = B.acc == Acc::F64;
  if ((out_t == CQC_F64) != acc_double)
    return Status::fail(CQC_ERR_UNSUPPORTED, "batched calls need the output dtype of the precision");
  std::map<std::tuple<int, int, int, int, int, int>, size_t> gidx;
  for (int32_t i = 0; i < n_inst; ++i) {
    const FdInstancePlan &ip = B.plans[i];
    const NetLayout &L = ip.net;
    const Plan &p = L.plan;
    std::vector<const void *> tptr(p.tensors.size(), nullptr);
    for (size_t t = 0; t < p.tensors.size(); ++t) {
      const auto &T = p.tensors[t];
      if (T.entry >= 0)
        tptr[t] = ip.conv_off[T.entry] != SIZE_MAX ? ws + ip.conv_off[T.entry]
                                                     : (need_ptrs ? inst[i].entries[T.entry] : nullptr);
      else
        tptr[t] = ws + L.t_off[t];
    }
    // flag descriptors of this instance's entries, for instances whose
    // one-instance call computes row flags (the others run without them, as
    // that call does)
    const bool inst_flags = needs_flags(L, false);
    for (size_t t = 0; t < p.tensors.size() && inst_flags; ++t) {
      const auto &T = p.tensors[t];
      if (T.entry < 0) continue;
      FlagDesc d;
      std::memset(&d, 0, sizeof(d));
      d.ptr = tptr[t];
      d.rows = T.rows();
      d.cols = T.cols();
      d.flags = reinterpret_cast<int32_t *>(ws + L.f_off[t]);
      d.block_start = B.flag_blocks;
      if (p.single && T.entry == 0) {
        d.unit = ws + L.t_off[1];
        d.unit_flag = reinterpret_cast<int32_t *>(ws + L.f_off[1]);
      }
      B.flag_blocks += T.rows() * flag_chunks(T.cols());
      B.flags.push_back(d);
    }
    for (size_t s = 0; s < p.steps.size(); ++s) {
      const Step &st = p.steps[s];
      const bool last = s + 1 == p.steps.size();
      ContractArgs a;
      std::memset(&a, 0, sizeof(a));
      a.X = tptr[st.x];
      a.Y = tptr[st.y];
      if (inst_flags) {
        a.flagX = reinterpret_cast<const int32_t *>(ws + L.f_off[st.x]);
        a.flagY = reinterpret_cast<const int32_t *>(ws + L.f_off[st.y]);
      }
      a.nchX = p.tensors[st.x].entry >= 0 ? (int)flag_chunks(p.tensors[st.x].cols()) : 1;
      a.nchY = p.tensors[st.y].entry >= 0 ? (int)flag_chunks(p.tensors[st.y].cols()) : 1;
      a.logM = st.logM;
      a.logN = st.logN;
      a.nS = (int)st.S.size();
      a.nRX = (int)st.RX.size();
      a.nRY = (int)st.RY.size();
      const int step_mode = !last ? kModeIntermediate : (is_blocked(p, st) ? kModeFinalBlocked : kModeFinalDeposit);
      const int cfg = queue_cfg(B.acc, st, step_mode, acc_double);
      const TileShape sh = tile_shape(cfg);
      a.tilesM = (int)(((int64_t(1) << st.logM) + sh.bm - 1) / sh.bm);
      a.tilesN = (int)(((int64_t(1) << st.logN) + sh.bn - 1) / sh.bn);
      a.nblocks = (int64_t)a.tilesM * a.tilesN * st.nbatch;
      a.mx = to_dev(st.mx);
      a.my = to_dev(st.my);
      set_lists(L, s, ws, &a);
      int level = (int)s;
      if (!last) {
        a.mode = kModeIntermediate;
        a.Z = ws + L.t_off[st.z];
        a.flagZ = reinterpret_cast<int32_t *>(ws + L.f_off[st.z]);
        a.scale = 1.0;
      } else {
        level = kFinalLevel;
        a.Z = need_ptrs ? inst[i].out : nullptr;
        a.scale = std::ldexp(1.0, -p.K);
        if (is_blocked(p, st)) {
          a.mode = kModeFinalBlocked;
        } else {
          a.mode = kModeFinalDeposit;
          const auto &X = p.tensors[st.x], &Y = p.tensors[st.y];
          const int nX = (int)X.bits.size(), nY = (int)Y.bits.size();
          std::vector<int> px(nX), py(nY);
          for (int j = 0; j < nX; ++j) px[j] = p.bitpos[X.bits[nX - 1 - j]];
          for (int j = 0; j < nY; ++j) py[j] = p.bitpos[Y.bits[nY - 1 - j]];
          a.posX = pack_pos(px);
          a.posY = pack_pos(py);
        }
        double *sum_to = need_ptrs ? inst[i].mass : nullptr;
        if (xent && need_ptrs) {
          a.xt = xent->targets[i];
          a.xg = xent->grads[i];
          if (xent->losses && xent->losses[i]) sum_to = xent->losses[i];
        }
        if (sum_to) {
          // per-tile partials live in this instance's (resized) partials slot
          a.partials = reinterpret_cast<double *>(ws + L.partials_off);
          MassDesc md;
          md.partials = a.partials;
          md.count = kPartialsPerTile * a.nblocks;
          md.mass = sum_to;
          B.mass.push_back(md);
        }
      }
      const bool small = a.nS <= 2;
      const Acc sa = step_acc(B.acc, st.wide_ok(), (int)st.S.size());
      // FP32 small-term steps over whole 64 x 256 tiles in pairs of rows run as
      // two-tile strips with every term kept (dead terms add exact zeros) -
      // for instances whose one-instance call computes no row flags, so the
      // outputs stay bitwise those of that call
      const bool strip = small && sa == Acc::F32 && cfg == kTileL && st.logM >= 7 && st.logN >= 8 &&
                         (a.mode == kModeFinalBlocked || a.mode == kModeIntermediate) && !inst_flags;
      if (strip) a.flagX = a.flagY = nullptr;
      // cross-entropy form of the final step: 1 gradient, 2 gradient and loss
      const int xe = xent == nullptr || !last ? 0 : (xent->losses && xent->losses[i] ? 2 : 1);
      auto key = std::make_tuple(level, (int)a.mode, cfg, (int)small * 2 + (int)strip, (int)sa, xe);
      auto it = gidx.find(key);
      if (it == gidx.end()) {
        it = gidx.emplace(key, B.groups.size()).first;
        BatchBuild::G g;
        g.level = level;
        g.mode = a.mode;
        g.cfg = cfg;
        g.small = small;
        g.strip = strip;
        g.xent = xe;
        g.acc = sa;
        B.groups.push_back(g);
      }
      const double cost = (double)a.nblocks * std::ldexp(1.0, 2 * a.nS) * sh.bm * sh.bn;
      B.groups[it->second].steps.push_back({cost, a});
    }
  }
  std::stable_sort(B.groups.begin(), B.groups.end(), [](const BatchBuild::G &x, const BatchBuild::G &y) {
    return x.level < y.level;
  });
  for (auto &g : B.groups)
    std::stable_sort(g.steps.begin(), g.steps.end(),
                     [](const std::pair<double, ContractArgs> &x, const std::pair<double, ContractArgs> &y) {
                       return x.first > y.first;
                     });
  // tables after the instance regions
  size_t off = align_up(B.plans.back().end, 256);
  B.tables_off = off;
  B.flag_off = off;
  off = align_up(off + sizeof(FlagDesc) * B.flags.size(), 256);
  B.mass_off = off;
  off = align_up(off + sizeof(MassDesc) * B.plans.size(), 256);   // room for every instance's mass
  B.counter_off = off;
  off = align_up(off + sizeof(unsigned long long) * std::max<size_t>(1, B.groups.size()), 256);
  for (auto &g : B.groups) {
    B.desc_off.push_back(off);
    off = align_up(off + sizeof(ContractArgs) * g.steps.size(), 256);
    B.prefix_off.push_back(off);
    off = align_up(off + sizeof(int64_t) * (g.steps.size() + 1), 256);
    B.bprefix_off.push_back(off);
    if (g.cfg == kTileW) off = align_up(off + sizeof(int64_t) * (g.steps.size() + 1), 256);
  }
  B.bytes = off;
  if (B.groups.size() > 256)
    return Status::fail(CQC_ERR_UNSUPPORTED, "too many distinct step shapes in one batch");
  *out = std::move(B);
  return Status::ok();
}

size_t batch_workspace_bytes(const cqc_instance *inst, int32_t n_inst, cqc_dtype in_t, cqc_dtype out_t,
                             cqc_precision prec, Status *st) {
  BatchBuild B;
  *st = build_batch(inst, n_inst, in_t, out_t, prec, false, nullptr, &B);
  return st->good() ? B.bytes : 0;
}

static Status batch_run(cqc_batch_s *b, hipStream_t s) {
  const bool acc_double = b->acc == Acc::F64;
  for (size_t i = 0; i < b->plans.size(); ++i) {
    const FdInstancePlan &ip = b->plans[i];
    for (int c = 0; c < ip.cut.nsub; ++c)
      if (ip.conv_off[c] != SIZE_MAX) {
        const auto &T = ip.net.plan.tensors[c];
        CQC_TRY(launch_convert(b->entry_src[i][c], b->in_double, b->ws + ip.conv_off[c], acc_double,
                               T.rows() * T.cols(), s));
      }
  }
  CQC_TRY(launch_row_flags_table(b->flag_descs, b->n_flag, b->flag_blocks, acc_double, b->counters,
                                 (int32_t)b->groups.size(), s));
  for (size_t g = 0; g < b->groups.size(); ++g) {
    const auto &G = b->groups[g];
    QueueLaunch q;
    q.descs = G.descs;
    q.prefix = G.prefix;
    q.ndesc = G.ndesc;
    q.queue = b->counters + g;
    q.total = G.total;
    q.grid = (uint32_t)std::min<int64_t>(G.total, kQueueGrid);
    q.bprefix = G.bprefix;
    q.btotal = G.btotal;
    q.xent = G.xent;
    if (G.strip) CQC_TRY(launch_contract_strip_queue(G.mode, q, s));
    else CQC_TRY(launch_contract_queue(G.acc, G.mode, G.cfg, G.small, q, s));
  }
  if (b->n_mass > 0) CQC_TRY(launch_mass_table(b->mass_descs, b->n_mass, s));
  return Status::ok();
}

static Status batch_create(const cqc_instance *inst, int32_t n_inst, cqc_dtype in_t, cqc_dtype out_t,
                           cqc_precision prec, void *workspace, size_t ws_bytes, hipStream_t s,
                           cqc_batch_s **out, const XentBind *xent = nullptr) {
  BatchBuild B;
  char *ws = static_cast<char *>(workspace);
  if (n_inst < 2) return Status::fail(CQC_ERR_INVALID_ARG, "a prepared batch needs at least two instances");
  CQC_TRY(build_batch(inst, n_inst, in_t, out_t, prec, true, ws, &B, xent));
  if (!workspace || ws_bytes < B.bytes)
    return Status::fail(CQC_ERR_WORKSPACE, "workspace needs " + std::to_string(B.bytes) + " bytes");
  if (reinterpret_cast<uintptr_t>(workspace) % 256)
    return Status::fail(CQC_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  // host image of the table region, uploaded once
  std::vector<char> img(B.bytes - B.tables_off, 0);
  auto put = [&](size_t off, const void *src, size_t n) { std::memcpy(img.data() + (off - B.tables_off), src, n); };
  if (!B.flags.empty()) put(B.flag_off, B.flags.data(), sizeof(FlagDesc) * B.flags.size());
  if (!B.mass.empty()) put(B.mass_off, B.mass.data(), sizeof(MassDesc) * B.mass.size());
  auto *b = new cqc_batch_s();
  b->plans = B.plans;
  b->acc = B.acc;
  b->in_double = in_t == CQC_F64;
  b->ws = ws;
  for (int32_t i = 0; i < n_inst; ++i)
    b->entry_src.emplace_back(inst[i].entries, inst[i].entries + B.plans[i].cut.nsub);
  b->flag_descs = reinterpret_cast<const FlagDesc *>(ws + B.flag_off);
  b->n_flag = (int32_t)B.flags.size();
  b->flag_blocks = B.flag_blocks;
  b->mass_descs = reinterpret_cast<const MassDesc *>(ws + B.mass_off);
  b->n_mass = (int32_t)B.mass.size();
  b->counters = reinterpret_cast<unsigned long long *>(ws + B.counter_off);
  for (size_t g = 0; g < B.groups.size(); ++g) {
    const auto &G = B.groups[g];
    std::vector<ContractArgs> descs;
    std::vector<int64_t> prefix(1, 0), bprefix(1, 0);
    for (auto &st : G.steps) {
      descs.push_back(st.second);
      const int64_t nb = st.second.nblocks;
      prefix.push_back(prefix.back() + (G.strip   ? nb / kStripRows
                                        : G.small ? (nb + kSmallTilesPerItem - 1) / kSmallTilesPerItem
                                                  : nb));
      bprefix.push_back(bprefix.back() + st.second.nbatch);
    }
    put(B.desc_off[g], descs.data(), sizeof(ContractArgs) * descs.size());
    put(B.prefix_off[g], prefix.data(), sizeof(int64_t) * prefix.size());
    if (G.cfg == kTileW) put(B.bprefix_off[g], bprefix.data(), sizeof(int64_t) * bprefix.size());
    cqc_batch_s::Group bg;
    bg.level = G.level;
    bg.mode = G.mode;
    bg.cfg = G.cfg;
    bg.small = G.small;
    bg.strip = G.strip;
    bg.xent = G.xent;
    bg.acc = G.acc;
    bg.descs = reinterpret_cast<const ContractArgs *>(ws + B.desc_off[g]);
    bg.prefix = reinterpret_cast<const int64_t *>(ws + B.prefix_off[g]);
    bg.ndesc = (int32_t)descs.size();
    bg.total = prefix.back();
    bg.bprefix = G.cfg == kTileW ? reinterpret_cast<const int64_t *>(ws + B.bprefix_off[g]) : nullptr;
    bg.btotal = G.cfg == kTileW ? bprefix.back() : 0;
    b->groups.push_back(bg);
  }
  hipError_t e = hipMemcpyAsync(ws + B.tables_off, img.data(), img.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    delete b;
    return Status::fail(CQC_ERR_HIP, std::string("uploading batch tables: ") + hipGetErrorString(e));
  }
  *out = b;
  return Status::ok();
}

}  // namespace cqc

using namespace cqc;

extern "C" {

int cqc_batch_create(const cqc_instance *inst, int32_t n_inst, cqc_dtype in_t, cqc_dtype out_t,
                     cqc_precision prec, void *workspace, size_t ws_bytes, hipStream_t stream,
                     cqc_batch *out) {
  if (!out) return Status::fail(CQC_ERR_INVALID_ARG, "out is NULL").code;
  cqc_batch_s *b = nullptr;
  Status st = batch_create(inst, n_inst, in_t, out_t, prec, workspace, ws_bytes, stream, &b);
  if (!st.good()) return st.code;
  *out = b;
  return CQC_OK;
}

int cqc_batch_create_xent(const cqc_instance *inst, int32_t n_inst, cqc_dtype in_t, cqc_dtype out_t,
                          cqc_precision prec, const void *const *targets, void *const *grads,
                          double *const *losses, void *workspace, size_t ws_bytes, hipStream_t stream,
                          cqc_batch *out) {
  if (!out) return Status::fail(CQC_ERR_INVALID_ARG, "out is NULL").code;
  const XentBind xb{targets, grads, losses};
  cqc_batch_s *b = nullptr;
  Status st = batch_create(inst, n_inst, in_t, out_t, prec, workspace, ws_bytes, stream, &b, &xb);
  if (!st.good()) return st.code;
  *out = b;
  return CQC_OK;
}

int cqc_batch_run(cqc_batch b, hipStream_t stream) {
  if (!b) return Status::fail(CQC_ERR_INVALID_ARG, "batch is NULL").code;
  return batch_run(b, stream).code;
}

int cqc_batch_destroy(cqc_batch b) {
  delete b;
  return CQC_OK;
}

}  // extern "C"
