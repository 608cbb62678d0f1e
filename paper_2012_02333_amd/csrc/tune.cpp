// Tile autotuner and its process-wide cache.
//
// Every contraction step belongs to a shape class (arithmetic, output mode,
// kernel variant, log2 of both operand widths, shared labels, output dtype).
// cqc_autotune times every candidate tile shape and block-to-XCD mapping of
// each class the given instances need, on the device, and records the
// fastest; the planner consults the cache before its built-in rule.  The cache
// can persist in a text file named by CQC_TUNE_CACHE (one class per line);
// with CQC_TUNE_VERBOSE set, every candidate's time is printed to stderr.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

#include "fdplan.hpp"

namespace cqc {

namespace {
using Key = std::tuple<int, int, int, int, int, int, int>;  // acc, mode, small, logM, logN, nS, out_double
struct Choice {
  int cfg;
  int xcd;
  double us;
};
struct Cache {
  std::mutex mu;
  std::map<Key, Choice> map;
  bool loaded = false;
};
Cache &cache() {
  static Cache c;
  return c;
}

void load_locked(Cache &c) {
  if (c.loaded) return;
  c.loaded = true;
  const char *path = std::getenv("CQC_TUNE_CACHE");
  if (!path) return;
  FILE *f = std::fopen(path, "r");
  if (!f) return;
  int k[7], cfg, xcd;
  double us;
  while (std::fscanf(f, "%d %d %d %d %d %d %d %d %d %lf", &k[0], &k[1], &k[2], &k[3], &k[4], &k[5], &k[6],
                     &cfg, &xcd, &us) == 10) {
    if (cfg < 0 || cfg >= kTileCount || (xcd != 0 && xcd != 1)) continue;
    c.map[Key(k[0], k[1], k[2], k[3], k[4], k[5], k[6])] = Choice{cfg, xcd, us};
  }
  std::fclose(f);
}

void save_locked(Cache &c) {
  const char *path = std::getenv("CQC_TUNE_CACHE");
  if (!path) return;
  FILE *f = std::fopen(path, "w");
  if (!f) return;
  for (auto &kv : c.map) {
    const Key &k = kv.first;
    std::fprintf(f, "%d %d %d %d %d %d %d %d %d %.3f\n", std::get<0>(k), std::get<1>(k), std::get<2>(k),
                 std::get<3>(k), std::get<4>(k), std::get<5>(k), std::get<6>(k), kv.second.cfg, kv.second.xcd,
                 kv.second.us);
  }
  std::fclose(f);
}
}  // namespace

bool tuned_choice(Acc acc, int mode, bool small, int logM, int logN, int nS, bool out_double, int *cfg,
                  int *xcd) {
  Cache &c = cache();
  std::lock_guard<std::mutex> g(c.mu);
  load_locked(c);
  auto it = c.map.find(Key((int)acc, mode, (int)small, logM, logN, nS, (int)out_double));
  if (it == c.map.end()) return false;
  *cfg = it->second.cfg;
  *xcd = it->second.xcd;
  return true;
}

static void record(const Key &k, Choice ch) {
  Cache &c = cache();
  std::lock_guard<std::mutex> g(c.mu);
  load_locked(c);
  c.map[k] = ch;
}

static void persist() {
  Cache &c = cache();
  std::lock_guard<std::mutex> g(c.mu);
  save_locked(c);
}

// Times one contraction step with every candidate (tile, XCD mapping), `reps`
// launches each, and records the fastest.
static Status tune_step(const NetLayout &L, size_t si, char *ws, const std::vector<const void *> &ents, void *out,
                        bool out_double, hipStream_t s) {
  const Plan &p = L.plan;
  const Step &st = p.steps[si];
  const bool last = si + 1 == p.steps.size();
  ContractArgs a;
  std::memset(&a, 0, sizeof(a));
  std::vector<const void *> tptr(p.tensors.size());
  for (size_t t = 0; t < p.tensors.size(); ++t)
    tptr[t] = p.tensors[t].entry >= 0 ? ents[p.tensors[t].entry] : ws + L.t_off[t];
  a.X = tptr[st.x];
  a.Y = tptr[st.y];
  if (needs_flags(L, false)) {
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
  a.mx = to_dev(st.mx);
  a.my = to_dev(st.my);
  set_lists(L, si, ws, &a);
  bool od = L.acc == Acc::F64;
  if (!last) {
    a.mode = kModeIntermediate;
    a.Z = ws + L.t_off[st.z];
    a.scale = 1.0;
  } else {
    a.Z = out;
    od = out_double;
    a.scale = std::ldexp(1.0, -p.K);
    a.mode = is_blocked(p, st) ? kModeFinalBlocked : kModeFinalDeposit;
    if (a.mode == kModeFinalDeposit) {
      const auto &X = p.tensors[st.x], &Y = p.tensors[st.y];
      const int nX = (int)X.bits.size(), nY = (int)Y.bits.size();
      std::vector<int> px(nX), py(nY);
      for (int j = 0; j < nX; ++j) px[j] = p.bitpos[X.bits[nX - 1 - j]];
      for (int j = 0; j < nY; ++j) py[j] = p.bitpos[Y.bits[nY - 1 - j]];
      a.posX = pack_pos(px);
      a.posY = pack_pos(py);
    }
  }
  const Acc sa = step_acc(L.acc, st.wide_ok(), (int)st.S.size());
  const int64_t work = (int64_t(1) << (st.logM + st.logN)) * st.nbatch;
  const int reps = work >= (int64_t(1) << 24) ? 10 : 30;
  struct Events {  // destroyed on every return path
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Events() {
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
    }
  } ev;
  CQC_HIP_TRY(hipEventCreate(&ev.e0));
  CQC_HIP_TRY(hipEventCreate(&ev.e1));
  hipEvent_t e0 = ev.e0, e1 = ev.e1;
  Choice best{-1, 0, 1e30};
  for (int cfg = 0; cfg < kTileCount; ++cfg) {
    if (!tile_ok(sa, cfg)) continue;
    const TileShape sh = tile_shape(cfg);
    const int64_t M = int64_t(1) << st.logM, N = int64_t(1) << st.logN;
    // skip shapes that would leave most of every tile empty
    if ((M < sh.bm || N < sh.bn) && cfg != kTileS && cfg != choose_tile(sa, a.nS, st.logM, st.logN, st.wide_ok(), st.nbatch)) continue;
    if (cfg == kTileW && !st.wide_ok()) continue;
    for (int xcd = 0; xcd < 2; ++xcd) {
      a.tilesM = (int)((M + sh.bm - 1) / sh.bm);
      a.tilesN = (int)((N + sh.bn - 1) / sh.bn);
      a.nblocks = (int64_t)a.tilesM * a.tilesN * st.nbatch;
      if (xcd && a.nblocks % 8) continue;
      a.xcd_remap = xcd;
      CQC_TRY(launch_contract(sa, od, cfg, a, s));  // warm-up
      CQC_HIP_TRY(hipEventRecord(e0, s));
      for (int r = 0; r < reps; ++r) CQC_TRY(launch_contract(sa, od, cfg, a, s));
      CQC_HIP_TRY(hipEventRecord(e1, s));
      CQC_HIP_TRY(hipEventSynchronize(e1));
      float ms = 0.f;
      CQC_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      const double us = 1000.0 * ms / reps;
      if (std::getenv("CQC_TUNE_VERBOSE"))
        std::fprintf(stderr, "cqc_autotune step %zu acc %d mode %d logM %d logN %d nS %d batches %lld: tile %d xcd %d %.2f us\n",
                     si, (int)L.acc, a.mode, st.logM, st.logN, a.nS, (long long)st.nbatch, cfg, xcd, us);
      if (us < best.us) best = Choice{cfg, xcd, us};
    }
  }
  if (best.cfg >= 0)
    record(Key((int)sa, a.mode, (int)(a.nS <= 2), st.logM, st.logN, a.nS, (int)od), best);
  return Status::ok();
}

}  // namespace cqc

using namespace cqc;

extern "C" {

int cqc_autotune(const cqc_instance *inst, int32_t n_inst, cqc_dtype in_t, cqc_dtype out_t,
                 cqc_precision prec, void *workspace, size_t ws_bytes, hipStream_t stream) {
  std::vector<FdInstancePlan> plans;
  Acc acc;
  Status st = fd_plans(inst, n_inst, in_t, out_t, prec, true, &plans, &acc);
  if (!st.good()) return st.code;
  const size_t need = plans.back().end;
  if (!workspace || ws_bytes < need)
    return Status::fail(CQC_ERR_WORKSPACE, "workspace needs " + std::to_string(need) + " bytes").code;
  char *ws = static_cast<char *>(workspace);
  const bool in_double = in_t == CQC_F64, acc_double = acc == Acc::F64;
  for (int32_t i = 0; i < n_inst; ++i) {
    const FdInstancePlan &ip = plans[i];
    std::vector<const void *> ents(ip.cut.nsub);
    for (int c = 0; c < ip.cut.nsub; ++c) {
      if (ip.conv_off[c] != SIZE_MAX) {
        const auto &T = ip.net.plan.tensors[c];
        st = launch_convert(inst[i].entries[c], in_double, ws + ip.conv_off[c], acc_double, T.rows() * T.cols(),
                            stream);
        if (!st.good()) return st.code;
        ents[c] = ws + ip.conv_off[c];
      } else {
        ents[c] = inst[i].entries[c];
      }
    }
    // one full run computes the flags and every intermediate
    st = run_net(ip.net, ws, ents, inst[i].out, out_t == CQC_F64, nullptr, true, stream);
    if (!st.good()) return st.code;
    for (size_t s = 0; s < ip.net.plan.steps.size(); ++s) {
      st = tune_step(ip.net, s, ws, ents, inst[i].out, out_t == CQC_F64, stream);
      if (!st.good()) return st.code;
    }
  }
  persist();
  return CQC_OK;
}

int cqc_tune_reset(void) {
  Cache &c = cache();
  std::lock_guard<std::mutex> g(c.mu);
  c.map.clear();
  c.loaded = false;
  return CQC_OK;
}

}  // extern "C"
