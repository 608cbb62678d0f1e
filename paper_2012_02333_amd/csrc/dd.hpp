// Dynamic definition: device argument blocks and host planning helpers.
#pragma once

#include <vector>

#include "engine.hpp"

namespace cqc {

constexpr int kTopT = 8;  // candidates kept per recursion and refill step

struct MergeDesc {
  const void *src;        // E_c, input dtype, [rows][2^f]
  void *dst;              // E'_c, Acc dtype, [rows][2^n_active]
  int64_t rows;
  int32_t f;
  int32_t n_active, n_merged;
  int32_t active_shift;   // >= 0: active bit j sits at local position active_shift + j
  int32_t merged_shift;   // >= 0: merged bit j sits at local position merged_shift + j
  int32_t log_chunks;     // long merges: 2^log_chunks chunks per output, one wave each
  double *part;           // [outputs][2^log_chunks] chunk sums (log_chunks > 0)
  int64_t chunk_block_start;  // first block of this descriptor in the second pass (set by the launcher)
  int32_t seg;            // short merge over the lowest bits with the active bits right above:
                          //   a row's outputs are consecutive runs of 2^n_merged elements
  int64_t zoom_value;     // fixed bits of the zoomed qubits at their local positions
  const int64_t *zoom_dev;  // if set: the zoom value is read from device memory instead
  BitPos active_pos;      // active bit j (from least significant) -> local position
  BitPos merged_pos;
  int64_t block_start;
};

struct MergeArgs {
  MergeDesc d[CQC_MAX_SUB];
  int32_t n;
  const int32_t *gate;    // device-side predicate, as in ContractArgs
  int32_t gate_val;
};

struct TopOut {
  double value[kTopT];
  int64_t index[kTopT];
};

// Merged combinations per wave and chunk of a long merge.
constexpr int kMergeLogChunk = 12;
// Chunks per output of a merge over 2^n_merged combinations (log2).
inline int merge_log_chunks(int n_merged) { return n_merged > kMergeLogChunk ? n_merged - kMergeLogChunk : 0; }
// Whether a short merge can take the segmented path (see k_dd_merge).
inline bool merge_segmented(int n_merged, int active_shift, int merged_shift) {
  return n_merged >= 1 && n_merged < 6 && merged_shift == 0 && active_shift == n_merged;
}
// Blocks of one descriptor in the merge grid (2048 elements per segmented block).
inline int64_t merge_blocks(int64_t nout, int n_merged, bool seg) {
  if (n_merged >= 6) return ((nout << merge_log_chunks(n_merged)) + 3) / 4;
  if (seg) return ((nout << n_merged) + 2047) / 2048;
  return (nout + 255) / 256;
}
// blocks: sum of merge_blocks over the descriptors.  Long merges write chunk
// sums to their `part` area, then a second pass adds them in chunk order.
Status launch_dd_merge(const MergeArgs &a, int64_t blocks, bool in_double, bool out_double,
                       hipStream_t s);
size_t topk_scratch_bytes(int64_t count, int t);
// Best t bins ranked strictly after (after_v, after_i) in the order
// (value descending, index ascending); missing places get index INT64_MAX.
// gate / gate_val: an optional device-side predicate (see ContractArgs).
Status launch_topk(const void *bins, bool bins_f32, int64_t count, int t, void *scratch, TopOut *out,
                   double after_v, int64_t after_i, hipStream_t s, const int32_t *gate = nullptr,
                   int32_t gate_val = 0);
// A top-kTopT request whose parameters live in device memory (written by an
// earlier kernel of the same stream): when active, rank row `row` of the bins
// (row * stride elements in), its first `count` bins, strictly after
// (after_v, after_i), into *out.
struct TopReq {
  int32_t active;
  int32_t row;
  int64_t count;
  double after_v;
  int64_t after_i;
  TopOut *out;
};
// Scratch and grid are sized for max_count bins (any count the request may carry).
Status launch_topk_req(const void *bins, bool bins_f32, int64_t stride, int64_t max_count, void *scratch,
                       const TopReq *req, hipStream_t s);

}  // namespace cqc
