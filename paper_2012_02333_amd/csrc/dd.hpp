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
  int64_t zoom_value;     // fixed bits of the zoomed qubits at their local positions
  BitPos active_pos;      // active bit j (from least significant) -> local position
  BitPos merged_pos;
  int64_t block_start;
};

struct MergeArgs {
  MergeDesc d[CQC_MAX_SUB];
  int32_t n;
};

struct TopOut {
  double value[kTopT];
  int64_t index[kTopT];
};

Status launch_dd_merge(const MergeArgs &a, int64_t blocks, bool in_double, bool out_double,
                       hipStream_t s);
size_t topk_scratch_bytes(int64_t count, int t);
// Best t bins ranked strictly after (after_v, after_i) in the order
// (value descending, index ascending); missing places get index INT64_MAX.
Status launch_topk(const double *bins, int64_t count, int t, void *scratch, TopOut *out,
                   double after_v, int64_t after_i, hipStream_t s);

}  // namespace cqc
