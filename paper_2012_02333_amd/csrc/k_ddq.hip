// Control kernels of the device-resident dynamic-definition query (Algorithm 1,
// Section 4.3): the choice of the bin each recursion refines is made on the
// device from the candidate windows the top-T passes leave in the query
// state, so every recursion can be enqueued before the first one runs.
//
// A recursion's candidates are kept as a window of the kTopT best bins not yet
// taken, ranked (value descending, index ascending).  Taking the last bin of a
// full window schedules a refill (the next kTopT bins ranked after it) that
// the next round's top-T request pass performs before its pick.
#include <climits>
#include <cstddef>

#include "kdev.hpp"
#include "ddplan.hpp"

namespace cqc {

// The static part of the query state (sizes, qubit tables, depth table) is
// copied into LDS by the whole block first: the pick is a chain of dependent
// decisions taken by one thread, and every table lookup it makes from global
// memory would be a full memory round trip.
constexpr int kDdqStaticBytes = (int)offsetof(DdqState, refill);
static_assert(kDdqStaticBytes % 4 == 0, "copied in 4-byte words");

__device__ __forceinline__ const DdqState *stage_static(const DdqState *st, uint32_t *lds) {
  const uint32_t *src = reinterpret_cast<const uint32_t *>(st);
  for (int i = threadIdx.x; i < (kDdqStaticBytes + 3) / 4; i += blockDim.x) lds[i] = src[i];
  __syncthreads();
  return reinterpret_cast<const DdqState *>(lds);
}

__device__ __forceinline__ void take_window(DdqRec &r) {
  int c = 0;
#pragma unroll
  for (int t = 0; t < kTopT; ++t) c += r.top.index[t] != INT64_MAX;
  r.ncand = c;
  r.consumed = 0;
  r.exhausted = c < kTopT;
}

// Roles of record k (every lane a share of the qubits): zoomed qubits carry
// their value, the depth's active qubits -2, the others -1 (merged); the
// entries past n stay 0.
__device__ __forceinline__ void write_roles(const DdqState *cs, const DdqRec &r, cqc_dd_record &rec) {
  const DdqDepth &dp = cs->depth[r.depth];
  for (int q = threadIdx.x; q < CQC_MAX_DD_QUBITS; q += blockDim.x) {
    int8_t v = 0;
    if (q < cs->n) {
      const uint64_t bit = uint64_t(1) << (q & 63);
      v = (r.zmask[q >> 6] & bit) ? (int8_t)((r.zbits[q >> 6] & bit) ? 1 : 0) : (int8_t)-1;
    }
    rec.role[q] = v;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < dp.n_active; t += blockDim.x) rec.role[dp.active[t]] = -2;
}

// Start of a run: recursion 0 (depth 0, nothing zoomed) is the only one set up.
__global__ __launch_bounds__(64) void k_ddq_init(DdqState *st) {
  __shared__ uint32_t lds[(kDdqStaticBytes + 3) / 4];
  const DdqState *cs = stage_static(st, lds);
  for (int k = threadIdx.x; k < cs->R; k += blockDim.x) st->rec[k].depth = -1;
  __syncthreads();
  if (threadIdx.x == 0) {
    st->stop = 0;
    st->refill.active = 0;
    DdqRec &r = st->rec[0];
    r.depth = 0;
    r.parent = -1;
    r.parent_bin = -1;
    r.ncand = r.consumed = r.exhausted = 0;
    r.zmask[0] = r.zmask[1] = r.zbits[0] = r.zbits[1] = 0;
    for (int c = 0; c < CQC_MAX_SUB; ++c) r.zoom[c] = 0;
    cqc_dd_record &rec = st->records[0];
    rec.parent_rec = -1;
    rec.parent_bin = -1;
    rec.n_active = cs->depth[0].n_active;
    *st->n_done = 1;
  }
  __syncthreads();
  write_roles(cs, st->rec[0], st->records[0]);
}

// The pick of recursion k >= 1.  Candidates: the bins of the windows of
// recursions 0..k-1 whose depth still has merged qubits.
//   heaviest (Algorithm 1): the largest value; ties to the lowest recursion
//   BFS: the shallowest depth, then the largest value, then the lowest recursion
//   DFS: the latest recursion that has a candidate (one recursion per round)
// With no candidate the search stops: recursion k and every later one stay
// unrun (their depth -1 gates their kernels off).
// Recursions whose candidate heads are loaded in parallel into LDS before the
// (serial, order-sensitive) scan; beyond this the one thread reads them from
// global memory itself.
constexpr int kPickScan = 1024;

__global__ __launch_bounds__(64) void k_ddq_pick(DdqState *st, int k) {
  __shared__ int s_go, s_stop;
  __shared__ uint32_t lds[(kDdqStaticBytes + 3) / 4];
  __shared__ double cand_v[kPickScan];
  __shared__ int cand_d[kPickScan];   // depth of recursion j's head candidate, -1: none
  const DdqState *cs = stage_static(st, lds);
  if (threadIdx.x == 0) {
    s_stop = st->stop;
    if (!s_stop) {
      DdqRec &prev = st->rec[k - 1];
      // the previous recursion's window (its top-T ran only if its depth has
      // merged qubits), and a refill performed since the last pick
      if (prev.depth >= 0) {
        if (cs->depth[prev.depth].has_merged) take_window(prev);
        else prev.ncand = prev.consumed = 0, prev.exhausted = 1;
      }
      if (st->refill.active) {
        take_window(st->rec[st->refill.row]);
        st->refill.active = 0;
      }
    }
  }
  __syncthreads();
  if (s_stop) return;
  // every recursion's head candidate (its depth and value), loaded by all lanes
  const bool par = k <= kPickScan;
  if (par)
    for (int j = threadIdx.x; j < k; j += blockDim.x) {
      const DdqRec &r = st->rec[j];
      const int d = r.depth;
      const bool ok = d >= 0 && cs->depth[d].has_merged && r.consumed < r.ncand;
      cand_d[j] = ok ? d : -1;
      cand_v[j] = ok ? r.top.value[r.consumed] : 0.0;
    }
  __syncthreads();
  if (threadIdx.x == 0) {
    int go = 0;
    {
      int best = -1, best_depth = INT_MAX;
      double best_v = 0.0;
      for (int j = 0; j < k; ++j) {
        int d;
        double v;
        if (par) {
          d = cand_d[j];
          v = cand_v[j];
        } else {
          const DdqRec &r = st->rec[j];
          d = r.depth >= 0 && cs->depth[r.depth].has_merged && r.consumed < r.ncand ? r.depth : -1;
          v = d >= 0 ? r.top.value[r.consumed] : 0.0;
        }
        if (d < 0) continue;
        if (cs->strategy == CQC_DD_DFS) {
          best = j;
          continue;
        }
        const int dj = cs->strategy == CQC_DD_BFS ? d : 0;
        if (best < 0 || dj < best_depth || (dj == best_depth && v > best_v)) {
          best = j;
          best_depth = dj;
          best_v = v;
        }
      }
      if (best < 0) {
        st->stop = 1;
      } else {
        DdqRec &p = st->rec[best];
        const int64_t bin = p.top.index[p.consumed];
        p.consumed++;
        const DdqDepth &pd = cs->depth[p.depth];
        if (p.consumed == p.ncand && !p.exhausted) {
          TopReq &q = st->refill;
          q.row = best;
          q.count = int64_t(1) << pd.n_active;
          q.after_v = p.top.value[kTopT - 1];
          q.after_i = p.top.index[kTopT - 1];
          q.out = &p.top;
          q.active = 1;
        }
        DdqRec &r = st->rec[k];
        r.depth = p.depth + 1;
        r.parent = best;
        r.parent_bin = bin;
        r.ncand = r.consumed = r.exhausted = 0;
        // masks in registers while they are built (r is global memory)
        uint64_t zm[2] = {p.zmask[0], p.zmask[1]}, zb[2] = {p.zbits[0], p.zbits[1]};
        // the parent's active qubits are zoomed to the bits of the bin
        // (first active qubit = most significant bin bit)
        for (int t = 0; t < pd.n_active; ++t) {
          const int q = pd.active[t];
          const uint64_t bit = uint64_t(1) << (q & 63);
          zm[q >> 6] |= bit;
          if ((bin >> (pd.n_active - 1 - t)) & 1) zb[q >> 6] |= bit;
        }
        r.zmask[0] = zm[0];
        r.zmask[1] = zm[1];
        r.zbits[0] = zb[0];
        r.zbits[1] = zb[1];
        int off = 0;
        for (int c = 0; c < cs->nsub; ++c) {
          const int f = cs->f[c];
          int64_t zv = 0;
          for (int j = 0; j < f; ++j) {
            const int q = cs->qubit[off + j];
            if ((zb[q >> 6] >> (q & 63)) & 1) zv |= int64_t(1) << (f - 1 - j);
          }
          r.zoom[c] = zv;
          off += f;
        }
        cqc_dd_record &rec = st->records[k];
        rec.parent_rec = best;
        rec.parent_bin = bin;
        rec.n_active = cs->depth[r.depth].n_active;
        *st->n_done = k + 1;
        go = 1;
      }
    }
    s_go = go;
  }
  __syncthreads();
  if (!s_go) return;
  write_roles(cs, st->rec[k], st->records[k]);
}

Status launch_ddq_init(DdqState *st, hipStream_t s) {
  return launch("ddq_init", k_ddq_init, dim3(1), dim3(64), 0, s, st);
}

Status launch_ddq_pick(DdqState *st, int k, hipStream_t s) {
  return launch("ddq_pick", k_ddq_pick, dim3(1), dim3(64), 0, s, st, k);
}

}  // namespace cqc
