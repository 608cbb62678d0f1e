// Workspace layout and enqueue of a contraction plan.
#include "engine.hpp"

#include <cstring>

namespace cqc {

NetLayout layout_net(const Plan &plan, Acc acc, size_t base) {
  NetLayout L;
  L.plan = plan;
  L.acc = acc;
  L.esz = acc == Acc::F32 ? 4 : 8;
  size_t off = align_up(base, 256);
  const size_t nt = plan.tensors.size();
  L.t_off.assign(nt, 0);
  L.f_off.assign(nt, 0);
  for (size_t t = 0; t < nt; ++t) {
    L.f_off[t] = off;
    off = align_up(off + sizeof(int32_t) * (size_t)plan.tensors[t].rows(), 256);
  }
  const int last = (int)plan.steps.size() - 1;
  for (size_t t = 0; t < nt; ++t) {
    const auto &T = plan.tensors[t];
    bool is_out = last >= 0 && (int)t == plan.steps[last].z;
    if (T.entry == -1 && !is_out) {
      L.t_off[t] = off;
      off = align_up(off + L.esz * (size_t)T.rows() * (size_t)T.cols(), 256);
    } else if (T.entry == -2) {
      L.t_off[t] = off;
      off = align_up(off + 8, 256);
    }
  }
  int64_t max_final_blocks = 1;
  for (const auto &st : plan.steps) {
    int cfg = choose_tile(st.logM, st.logN);
    TileShape sh = tile_shape(cfg);
    int64_t tm = ((int64_t(1) << st.logM) + sh.bm - 1) / sh.bm;
    int64_t tn = ((int64_t(1) << st.logN) + sh.bn - 1) / sh.bn;
    L.tile.push_back(cfg);
    L.nblocks.push_back(tm * tn * st.nbatch);
  }
  if (last >= 0) max_final_blocks = L.nblocks[last];
  L.partials_off = off;
  off = align_up(off + 8 * (size_t)max_final_blocks, 256);
  L.counter_off = off;
  off = align_up(off + 8, 256);
  L.bytes = off;
  return L;
}

static DigitMapDev to_dev(const DigitMap &m) {
  DigitMapDev d;
  std::memset(&d, 0, sizeof(d));
  d.n = m.n;
  for (int i = 0; i < m.n; ++i) {
    d.src[i] = m.src[i];
    d.shift[i] = m.shift[i];
  }
  return d;
}

Status run_net(const NetLayout &L, char *ws, const std::vector<const void *> &entries,
               void *out, bool out_double, double *mass, bool compute_entry_flags,
               hipStream_t s) {
  const Plan &p = L.plan;
  const size_t nt = p.tensors.size();
  std::vector<const void *> tptr(nt, nullptr);
  for (size_t t = 0; t < nt; ++t) {
    const auto &T = p.tensors[t];
    if (T.entry >= 0) tptr[t] = entries[T.entry];
    else tptr[t] = ws + L.t_off[t];
  }
  uint32_t *counter = reinterpret_cast<uint32_t *>(ws + L.counter_off);
  if (compute_entry_flags) {
    FlagArgs fa;
    std::memset(&fa, 0, sizeof(fa));
    int64_t rows = 0;
    int n = 0;
    for (size_t t = 0; t < nt; ++t) {
      const auto &T = p.tensors[t];
      if (T.entry < 0) continue;
      FlagDesc &d = fa.d[n++];
      d.ptr = tptr[t];
      d.rows = T.rows();
      d.cols = T.cols();
      d.flags = reinterpret_cast<int32_t *>(ws + L.f_off[t]);
      d.row_start = rows;
      rows += T.rows();
    }
    fa.n = n;
    fa.is_double = L.acc == Acc::F64;
    fa.counter = counter;
    if (p.single) {
      fa.unit = ws + L.t_off[1];
      fa.unit_flag = reinterpret_cast<int32_t *>(ws + L.f_off[1]);
    }
    CQC_TRY(launch_row_flags(fa, rows, s));
  }
  for (size_t i = 0; i < p.steps.size(); ++i) {
    const Step &st = p.steps[i];
    const bool last = i + 1 == p.steps.size();
    ContractArgs a;
    std::memset(&a, 0, sizeof(a));
    a.X = tptr[st.x];
    a.Y = tptr[st.y];
    a.flagX = reinterpret_cast<const int32_t *>(ws + L.f_off[st.x]);
    a.flagY = reinterpret_cast<const int32_t *>(ws + L.f_off[st.y]);
    a.logM = st.logM;
    a.logN = st.logN;
    a.nS = (int)st.S.size();
    a.nRX = (int)st.RX.size();
    a.nRY = (int)st.RY.size();
    TileShape sh = tile_shape(L.tile[i]);
    a.tilesM = (int)(((int64_t(1) << st.logM) + sh.bm - 1) / sh.bm);
    a.tilesN = (int)(((int64_t(1) << st.logN) + sh.bn - 1) / sh.bn);
    a.nblocks = L.nblocks[i];
    a.mx = to_dev(st.mx);
    a.my = to_dev(st.my);
    if (!last) {
      a.mode = kModeIntermediate;
      a.Z = ws + L.t_off[st.z];
      a.flagZ = reinterpret_cast<int32_t *>(ws + L.f_off[st.z]);
      a.scale = 1.0;
      CQC_TRY(launch_contract(L.acc, L.acc == Acc::F64, L.tile[i], a, s));
    } else {
      a.Z = out;
      a.scale = std::ldexp(1.0, -p.K);
      if (is_blocked(p, st)) {
        a.mode = kModeFinalBlocked;
      } else {
        a.mode = kModeFinalDeposit;
        const auto &X = p.tensors[st.x], &Y = p.tensors[st.y];
        const int nX = (int)X.bits.size(), nY = (int)Y.bits.size();
        for (int j = 0; j < nX; ++j) a.posX[j] = (int8_t)p.bitpos[X.bits[nX - 1 - j]];
        for (int j = 0; j < nY; ++j) a.posY[j] = (int8_t)p.bitpos[Y.bits[nY - 1 - j]];
      }
      if (mass) {
        a.partials = reinterpret_cast<double *>(ws + L.partials_off);
        a.counter = counter;
        a.mass = mass;
      }
      CQC_TRY(launch_contract(L.acc, out_double, L.tile[i], a, s));
    }
  }
  return Status::ok();
}

}  // namespace cqc
