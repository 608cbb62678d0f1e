// Adjoint of the contraction plan: device argument block and launchers.
#pragma once

#include "engine.hpp"

namespace cqc {

struct BwdArgs {
  const void *X;       // forward operands (Acc dtype)
  const void *Y;
  const void *dZ;      // dL/dZ, row-major per batch [(rX,rY)][M][N]
  void *part;          // partial sums [P][rows][cols]
  int32_t logM, logN;
  int32_t nS, nRX, nRY;
  DigitMapDev mx, my;
  int64_t kChunk;      // inner-dimension chunk per partial (multiple of 16)
  int32_t kChunks;     // chunks per rest-label value
  int64_t rowsX, rowsY;
  // both sides in one pass (k_bwd_dual_queue): the X side's partials go to
  // part with column chunks of kChunk (kChunks per rY), the Y side's to part2
  // with row tiles of kDualRows (kChunks2 per rX)
  void *part2;
  int32_t kChunks2;
};

// Both sides of a step from one read of dL/dZ (steps of at most 16 labels,
// FP32, both operands at least kDualMin wide): row tile and column sub-tile
// of the staged dL/dZ, and the column chunk of one block.
constexpr int kDualRows = 128, kDualCols = 64, kDualChunk = 1024, kDualMin = 64;
inline bool bwd_dual_ok(int nS, int64_t M, int64_t N, bool f32) {
  return f32 && nS <= 2 && M >= kDualMin && N >= kDualMin;
}
inline int64_t bwd_dual_blocks(const BwdArgs &a, int64_t nbatch) {
  return nbatch * (int64_t)a.kChunks2 * (int64_t)a.kChunks;
}

// Split-K choice of one side of an adjoint step: inner-dimension chunk, chunks
// per rest-label value and partial count P = rest * chunks, the smallest
// chunk (from 128) whose partials fit max(min_budget, dz_frac * dz bytes).
struct BwdSide {
  int64_t kChunk = 16;
  int32_t kChunks = 1;
  int64_t P = 1;
};
BwdSide choose_bwd_side(int64_t inner, int64_t rest, int64_t out_elems, int64_t dz_elems, size_t esz,
                        double min_budget, double dz_frac = 0.25);

// Batched adjoint tables (device memory).
struct BwdReduceDesc {    // out[i] = scale * sum_{p < P} part[p][i], i < count
  const void *part;       // [P][count], Acc dtype
  void *out;              // [count], FP64 if out_double else FP32
  int64_t count, P;
  double scale;
  int32_t out_double;
  int32_t vec;            // FP32 partials, count % 4 == 0, out 16-byte aligned: four outputs per thread
};
// Blocks of the batched reduce for one descriptor (256 threads each).
inline int64_t bwd_reduce_blocks(const BwdReduceDesc &r) {
  return r.vec ? (r.count + 1023) / 1024 : (r.count + 255) / 256;
}
struct BwdGatherDesc {    // dst[m * N + n] = src[rowoff(m) + coloff(n)], Acc dtype
  const void *src;
  void *dst;
  int32_t logM, logN;
  BitPos px, py;
};
struct BwdQueue {         // one persistent launch over many steps of one kernel shape
  bool y;                 // dY side (else dX)
  bool dual = false;      // both sides in one pass (k_bwd_dual_queue; y and sb unused)
  int sb;                 // label blocks of 16 per block tile (bwd_sb)
  const BwdArgs *descs;
  const int64_t *prefix;  // [ndesc + 1] first item of each step
  int ndesc;
  unsigned long long *queue;   // zeroed by the run's prep launch
  int64_t total;
  uint32_t grid;
};

int bwd_sb(int nS, bool y, bool f32);
int64_t bwd_blocks(const BwdArgs &a, bool which_y, bool f32);
Status launch_bwd(Acc acc, const BwdArgs &a, bool which_y, hipStream_t s);
Status launch_bwd_queue(Acc acc, const BwdQueue &q, hipStream_t s);
Status launch_bwd_reduce_table(Acc acc, const BwdReduceDesc *descs, const int64_t *start, int ndesc,
                               int64_t blocks, hipStream_t s);
Status launch_bwd_prep(Acc acc, const BwdGatherDesc *descs, const int64_t *start, int ndesc, int64_t blocks,
                       unsigned long long *counters, int ncounters, hipStream_t s);
Status launch_bwd_reduce(Acc acc, const void *part, int64_t count, int64_t P, double scale,
                         void *out, bool out_double, hipStream_t s);
Status launch_gather_blocked(Acc acc, const void *src, void *dst, int logM, int logN,
                             const BitPos &px, const BitPos &py, hipStream_t s);

}  // namespace cqc
