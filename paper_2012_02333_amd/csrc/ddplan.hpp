// Dynamic definition: host plans of a query (one per zoom depth), shared by the
// host-driven query and the device-resident one, and the device-resident
// query's state.
#pragma once

#include <memory>
#include <vector>

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
  std::vector<size_t> part_off;              // chunk sums of long merges (SIZE_MAX: none)
  size_t end = 0;
};

// what a round of the host-driven query reads back per recursion: its top-T
// candidates and its mass
struct DdSlot {
  TopOut top;
  double mass;
};

constexpr int kDdMaxPerRound = 64;

struct DdPlan {
  CutInfo cut;
  Acc acc;
  int a = 0, R = 0, strategy = 0, per_round = 1;
  bool bins_f32 = false;
  std::vector<DepthPlan> depths;
  size_t topk_off = 0, out_off = 0, bytes = 0;
};

// The plan of a query (validated, cached across calls with equal inputs).
Status cached_dd(const cqc_instance *inst, cqc_dtype in_t, cqc_precision prec, const cqc_dd_params *p,
                 std::shared_ptr<const DdPlan> *out);

// Merge descriptors of one recursion at depth dp: zoom values from the host
// (zoom[c]) or read by the kernels from device memory (zoom_dev[c]); merged[c]
// is the operand the term sum reads (the entry tensor itself where nothing is
// merged).
void dd_merge_args(const DdPlan &d, const DepthPlan &dp, const void *const *entries, char *ws, bool in_double,
                   const int64_t *zoom, const int64_t *const *zoom_dev, MergeArgs *ma, int64_t *blocks,
                   std::vector<const void *> *merged);

// ---- device-resident query: every decision of Algorithm 1 is taken by a
// kernel, so all recursions are enqueued at once (no host round trip) and the
// whole query can be captured in a graph.
constexpr int kDdqMaxDepths = 64;

struct DdqRec {             // one recursion of the query, in device memory
  int32_t depth;            // -1: not run (the search stopped before it)
  int32_t parent;           // -1 for the first recursion
  int64_t parent_bin;
  int32_t ncand;            // valid candidates in `top` (the current window)
  int32_t consumed;         // of them, already expanded
  int32_t exhausted;        // no candidate ranks after the window
  int32_t pad;
  TopOut top;               // candidate window, best first
  int64_t zoom[CQC_MAX_SUB];        // per subcircuit: zoom value at its local bit positions
  uint64_t zmask[2], zbits[2];      // zoomed global qubits and their values
};

struct DdqDepth {           // static description of one zoom depth
  int32_t n_active;
  int32_t has_merged;
  int8_t active[40];        // ascending qubit ids (n_active <= 36)
};

struct DdqState {           // in the workspace; tables written once at creation
  int32_t R, D, n, nsub, strategy, stop;
  int32_t f[CQC_MAX_SUB];
  int8_t qubit[CQC_MAX_DD_QUBITS];  // global qubit of local bit j of subcircuit c, concatenated over c
  DdqDepth depth[kDdqMaxDepths];
  TopReq refill;            // next round's refill of the window it emptied
  cqc_dd_record *records;   // caller's (device) records and recursion count
  int32_t *n_done;
  DdqRec rec[1];            // [R]
};
inline size_t ddq_state_bytes(int R) { return sizeof(DdqState) + sizeof(DdqRec) * (size_t)(R - 1); }

// Launchers of the query's control kernels.
Status launch_ddq_init(DdqState *st, hipStream_t s);
Status launch_ddq_pick(DdqState *st, int k, hipStream_t s);

}  // namespace cqc
