// Workspace layout and enqueue of a contraction plan.
#include "engine.hpp"

#include <algorithm>
#include <cstring>

namespace cqc {

NetLayout layout_net(const Plan &plan, Acc acc, size_t base) {
  NetLayout L;
  L.plan = plan;
  L.acc = acc;
  L.esz = acc == Acc::F64 ? 8 : 4;
  size_t off = align_up(base, 256);
  const size_t nt = plan.tensors.size();
  L.t_off.assign(nt, 0);
  L.f_off.assign(nt, 0);
  for (size_t t = 0; t < nt; ++t) {
    L.f_off[t] = off;
    const auto &T = plan.tensors[t];
    // entry tensors carry chunk flags; intermediates one flag per row
    const int64_t nch = T.entry >= 0 ? flag_chunks(T.cols()) : 1;
    off = align_up(off + sizeof(int32_t) * (size_t)(T.rows() * nch), 256);
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
    int cfg = choose_tile(step_acc(acc, st.wide_ok(), (int)st.S.size()), (int)st.S.size(), st.logM, st.logN,
                          st.wide_ok(), st.nbatch);
    TileShape sh = tile_shape(cfg);
    int64_t tm = ((int64_t(1) << st.logM) + sh.bm - 1) / sh.bm;
    int64_t tn = ((int64_t(1) << st.logN) + sh.bn - 1) / sh.bn;
    L.tile.push_back(cfg);
    L.nblocks.push_back(tm * tn * st.nbatch);
  }
  if (last >= 0) {
    // room for the per-tile partials of any tile shape the last step may run
    // with (tuned choices and the batched path may pick another shape)
    const Step &st = plan.steps[last];
    for (int cfg = 0; cfg < kTileCount; ++cfg) {
      const TileShape sh = tile_shape(cfg);
      const int64_t t = (((int64_t(1) << st.logM) + sh.bm - 1) / sh.bm) *
                        (((int64_t(1) << st.logN) + sh.bn - 1) / sh.bn) * st.nbatch;
      max_final_blocks = std::max(max_final_blocks, t);
    }
  }
  L.partials_off = off;
  off = align_up(off + 8 * (size_t)kPartialsPerTile * (size_t)max_final_blocks, 256);
  // label lists of every step that may run on the wide kernel
  L.list_off.assign(plan.steps.size(), SIZE_MAX);
  if (acc != Acc::F64) {
    for (size_t i = 0; i < plan.steps.size(); ++i) {
      const Step &st = plan.steps[i];
      L.list_off[i] = off;
      off = align_up(off + wide_list_bytes((int)st.S.size(), st.nbatch), 256);
    }
  }
  // bfloat16 parts of the operands of split-form wide steps (split once per
  // call, not once per tile)
  L.xs_off.assign(plan.steps.size(), SIZE_MAX);
  L.ys_off.assign(plan.steps.size(), SIZE_MAX);
  if (is_split(acc)) {
    for (size_t i = 0; i < plan.steps.size(); ++i) {
      const Step &st = plan.steps[i];
      if (!is_split(step_acc(acc, st.wide_ok(), (int)st.S.size()))) continue;
      const size_t parts = (size_t)split_parts(acc);
      const TensorSpec &X = plan.tensors[st.x], &Y = plan.tensors[st.y];
      L.xs_off[i] = off;
      off = align_up(off + parts * 2 * (size_t)(X.rows() * X.cols()), 256);
      L.ys_off[i] = off;
      off = align_up(off + parts * 2 * (size_t)(Y.rows() * Y.cols()), 256);
    }
  }
  L.bytes = off;
  return L;
}

bool needs_flags(const NetLayout &L, bool skip_final) {
  const Plan &p = L.plan;
  if (p.single) return true;   // the flag pass also writes the unit operand
  for (size_t i = 0; i < p.steps.size(); ++i) {
    if (i + 1 == p.steps.size() && skip_final) break;
    if (p.steps[i].S.size() > 2 || L.tile[i] == kTileW) return true;
  }
  return false;
}

void set_lists(const NetLayout &L, size_t step, char *ws, ContractArgs *a) {
  const Step &st = L.plan.steps[step];
  a->nbatch = st.nbatch;
  if (L.list_off.empty() || L.list_off[step] == SIZE_MAX) return;
  a->list_ld = wide_list_ld((int)st.S.size());
  a->lists = reinterpret_cast<int32_t *>(ws + L.list_off[step]);
  a->counts = reinterpret_cast<int32_t *>(ws + L.list_off[step] + (size_t)st.nbatch * a->list_ld * 8);
}

DigitMapDev to_dev(const DigitMap &m) {
  DigitMapDev d;
  std::memset(&d, 0, sizeof(d));
  d.n = m.n;
  for (int i = 0; i < m.n; ++i) {
    if (m.src[i]) d.srcmask |= 1u << i;
    d.shifts[i / 10] |= (uint64_t)(m.shift[i] & 63) << (6 * (i % 10));
  }
  return d;
}

BitPos pack_pos(const std::vector<int> &pos) {
  BitPos b;
  std::memset(&b, 0, sizeof(b));
  for (size_t j = 0; j < pos.size(); ++j) b.w[j / 10] |= (uint64_t)(pos[j] & 63) << (6 * (j % 10));
  return b;
}

Status run_net(const NetLayout &L, char *ws, const std::vector<const void *> &entries,
               void *out, bool out_double, double *mass, bool compute_entry_flags,
               hipStream_t s, bool skip_final, const int32_t *gate, int32_t gate_val) {
  const Plan &p = L.plan;
  const size_t nt = p.tensors.size();
  std::vector<const void *> tptr(nt, nullptr);
  for (size_t t = 0; t < nt; ++t) {
    const auto &T = p.tensors[t];
    if (T.entry >= 0) tptr[t] = entries[T.entry];
    else tptr[t] = ws + L.t_off[t];
  }
  const bool need_flags = needs_flags(L, skip_final);
  if (compute_entry_flags && need_flags) {
    FlagArgs fa;
    std::memset(&fa, 0, sizeof(fa));
    int64_t blocks = 0;
    int n = 0;
    for (size_t t = 0; t < nt; ++t) {
      const auto &T = p.tensors[t];
      if (T.entry < 0) continue;
      FlagDesc &d = fa.d[n++];
      d.ptr = tptr[t];
      d.rows = T.rows();
      d.cols = T.cols();
      d.flags = reinterpret_cast<int32_t *>(ws + L.f_off[t]);
      d.block_start = blocks;
      blocks += T.rows() * flag_chunks(T.cols());
    }
    fa.n = n;
    fa.is_double = L.acc == Acc::F64;
    fa.gate = gate;
    fa.gate_val = gate_val;
    if (p.single) {
      fa.d[0].unit = ws + L.t_off[1];
      fa.d[0].unit_flag = reinterpret_cast<int32_t *>(ws + L.f_off[1]);
    }
    CQC_TRY(launch_row_flags(fa, blocks, s));
  }
  for (size_t i = 0; i < p.steps.size(); ++i) {
    const Step &st = p.steps[i];
    const bool last = i + 1 == p.steps.size();
    if (last && skip_final) break;
    ContractArgs a;
    std::memset(&a, 0, sizeof(a));
    a.X = tptr[st.x];
    a.Y = tptr[st.y];
    a.gate = gate;
    a.gate_val = gate_val;
    if (need_flags) {
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
    set_lists(L, i, ws, &a);
    const int mode = !last ? kModeIntermediate : (is_blocked(p, st) ? kModeFinalBlocked : kModeFinalDeposit);
    const bool od = last ? out_double : L.acc == Acc::F64;
    const Acc sa = step_acc(L.acc, st.wide_ok(), (int)st.S.size());
    int cfg = L.tile[i], xcd = 0;
    // a cached choice is keyed by shape class, which does not fix the operand
    // heights: the wide tile also needs this step's operands to fit it
    if (!tuned_choice(sa, mode, a.nS <= 2, st.logM, st.logN, a.nS, od, &cfg, &xcd) || !tile_ok(sa, cfg) ||
        (cfg == kTileW && !st.wide_ok())) {
      cfg = L.tile[i];
      // the wide kernel's tiles of one operand row block share that block's
      // operand columns: keep them on one XCD (and its L2)
      xcd = cfg == kTileW ? 1 : 0;
    }
    const TileShape sh = tile_shape(cfg);
    a.tilesM = (int)(((int64_t(1) << st.logM) + sh.bm - 1) / sh.bm);
    a.tilesN = (int)(((int64_t(1) << st.logN) + sh.bn - 1) / sh.bn);
    a.nblocks = (int64_t)a.tilesM * a.tilesN * st.nbatch;
    a.xcd_remap = (xcd && a.nblocks % 8 == 0) ? 1 : 0;
    if (cfg == kTileW && is_split(sa) && L.xs_off[i] != SIZE_MAX && !gate) {
      // split both operands into their bfloat16 parts once, for every tile
      const TensorSpec &X = p.tensors[st.x], &Y = p.tensors[st.y];
      a.xplane = X.rows() * X.cols();
      a.yplane = Y.rows() * Y.cols();
      a.Xs = ws + L.xs_off[i];
      a.Ys = ws + L.ys_off[i];
      CQC_TRY(launch_presplit(split_parts(sa), static_cast<const float *>(a.X), ws + L.xs_off[i], a.xplane,
                              a.xplane, s));
      CQC_TRY(launch_presplit(split_parts(sa), static_cast<const float *>(a.Y), ws + L.ys_off[i], a.yplane,
                              a.yplane, s));
    }
    if (!last) {
      a.mode = kModeIntermediate;
      a.Z = ws + L.t_off[st.z];
      a.flagZ = reinterpret_cast<int32_t *>(ws + L.f_off[st.z]);
      a.scale = 1.0;
      CQC_TRY(launch_contract(sa, L.acc == Acc::F64, cfg, a, s));
    } else {
      a.Z = out;
      a.scale = std::ldexp(1.0, -p.K);
      if (mode == kModeFinalBlocked) {
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
      if (mass) a.partials = reinterpret_cast<double *>(ws + L.partials_off);
      CQC_TRY(launch_contract(sa, out_double, cfg, a, s));
      if (mass) CQC_TRY(launch_mass_final(a.partials, kPartialsPerTile * a.nblocks, mass, s, gate, gate_val));
    }
  }
  return Status::ok();
}

}  // namespace cqc
