// Kernel argument blocks and host launchers of the gfx950 kernels.
#pragma once

#include <cstdint>

#include "common.hpp"

namespace cqc {

// Row-index map of one operand, packed into scalars so the kernel never indexes
// a kernel-argument array with a runtime index (that turns into dependent
// vector loads from the argument segment).  Digit i (most significant first)
// takes source (srcmask >> i) & 1 (0: shared index s, 1: rest index r) and
// shift (shifts[i / 10] >> 6 (i % 10)) & 63.
struct DigitMapDev {
  int32_t n;
  uint32_t srcmask;
  uint64_t shifts[2];
};

// Output-bit positions of the column bits of an operand (bit j counted from
// the least significant), 6 bits each, 10 per word.
struct BitPos {
  uint64_t w[5];
};

// One pairwise contraction step (see plan.hpp), executed as a batched GEMM
//   C_b[m][n] = sum_{s live} X[rowX(s, rX)][m] * Y[rowY(s, rY)][n],  b = (rX, rY)
enum ContractMode : int32_t {
  kModeIntermediate = 0,  // Z[b][m][n] row-major, Acc dtype, row flags of Z written
  kModeFinalBlocked = 1,  // out[m * N + n] * scale
  kModeFinalDeposit = 2   // out[rowoff(m) + coloff(n)] * scale, per-bit positions
};

struct ContractArgs {
  const void *X;
  const void *Y;
  const int32_t *flagX;   // [rows][nchX] chunk flags
  const int32_t *flagY;
  int32_t nchX, nchY;
  int32_t *flagZ;
  void *Z;
  int32_t logM, logN;
  int32_t nS, nRX, nRY;
  int32_t tilesM, tilesN;
  int32_t mode;
  int32_t xcd_remap;  // 1: keep consecutive logical tiles on one XCD
  int64_t nblocks;
  double scale;
  DigitMapDev mx, my;
  BitPos posX, posY;  // deposit mode: column bit -> output bit position
  double *partials;  // [nblocks] per-block FP64 sums of the written outputs, or null
  // wide kernel only: live-label lists of every batch entry (written by the
  // label-list pass of the same step)
  int32_t *lists;    // [nbatch][2][list_ld] byte offsets of the live terms' X rows, then of
                     //   their Y rows, ascending s; padding 0
  int32_t *counts;   // [nbatch] live labels
  int32_t list_ld;   // pairs per batch entry: 4^nS rounded up to a multiple of 32
  int64_t nbatch;
  // device-side predicate: when gate is set, the launch does nothing unless
  // *gate == gate_val (a dynamic-definition query enqueues the kernels of
  // every depth a recursion can have, and runs only the one its pick chose)
  const int32_t *gate;
  int32_t gate_val;
  // split-BF16 wide steps: the operands already split into bfloat16 parts,
  // part p of X at Xs + p * xplane elements (same layout as X), or null (the
  // wide kernel splits while staging)
  const void *Xs;
  const void *Ys;
  int64_t xplane, yplane;
  // cross-entropy form of a final step (batched queue kernels): xt is the
  // target t in output order; every output p gets dL/dp = -t/p (0 where p <=
  // 1e-30) written to xg at its position, p itself is written only if Z is
  // set, and the partial sums add the loss terms -t log max(p, 1e-30) (kernel
  // form with the loss) or p
  const void *xt;
  void *xg;
};

// FP64 mass partials: every wave of a final-step tile (four per block) stores
// the FP64 sum of the outputs it wrote at partials[kPartialsPerTile * tile +
// wave], so no block barrier stands between a tile's stores and the next
// tile; the final pass adds them in index order.
constexpr int kPartialsPerTile = 4;

// Workspace of the label lists of a step run by the wide kernel.
// Operands of the wide kernel are addressed with 32-bit byte offsets.
constexpr int64_t kWideMaxOperandElems = int64_t(1) << 30;
inline int32_t wide_list_ld(int nS) { return (int32_t)((((int64_t)1 << (2 * nS)) + 31) / 32 * 32); }
inline size_t wide_list_bytes(int nS, int64_t nbatch) {
  return (size_t)nbatch * (size_t)wide_list_ld(nS) * 8 + (size_t)nbatch * 4;
}

// Row flags are kept per (row, chunk of kFlagChunk columns): flag[r * nch + c]
// says whether chunk c of row r has a non-zero element; a row is live if any
// of its chunk flags is set.  Splitting rows lets the flag pass run with many
// small blocks instead of one block per long row.
constexpr int kFlagChunk = 2048;
__host__ __device__ inline int64_t flag_chunks(int64_t cols) { return (cols + kFlagChunk - 1) / kFlagChunk; }

struct FlagDesc {
  const void *ptr;
  int64_t rows;
  int64_t cols;
  int32_t *flags;      // [rows][flag_chunks(cols)]
  int64_t block_start; // first block of this tensor
  void *unit;          // if non-null: a unit operand (Acc-typed 1.0) is written here
  int32_t *unit_flag;  //   and its row flag set
};

struct FlagArgs {
  FlagDesc d[CQC_MAX_SUB + 1];
  int32_t n;
  int32_t is_double;
  const int32_t *gate;   // as in ContractArgs
  int32_t gate_val;
};

// Arithmetic of a plan.  BF16X6 and BF16X3 keep every tensor in FP32 and
// split the operands into three (two) bfloat16 parts inside the wide kernel.
enum class Acc { F32, F64, BF16X6, BF16X3 };
inline bool is_split(Acc a) { return a == Acc::BF16X6 || a == Acc::BF16X3; }
// bfloat16 parts per operand of the wide kernel's form (0: FP32)
inline int split_parts(Acc a) { return a == Acc::BF16X6 ? 3 : a == Acc::BF16X3 ? 2 : 0; }

// Tile configurations of the contraction kernels: L, M, S, T select the
// register-operand kernel (FP32 and FP64), W the LDS-staged wide kernel
// (FP32 and the split forms; the only one the split forms run on).
enum TileCfg : int32_t { kTileL = 0, kTileM = 1, kTileS = 2, kTileT = 3, kTileW = 4, kTileCount = 5 };
struct TileShape { int bm, bn; };
TileShape tile_shape(int cfg);
// Built-in rule (the autotuner's cache takes precedence where it has an entry).
// wide_ok: both operands fit the wide kernel's addressing (wide_fits).
// nbatch: batch entries of the step (the wide kernel needs enough 128 x 128
// tiles over all of them to fill the chip).
int choose_tile(Acc acc, int nS, int logM, int logN, bool wide_ok, int64_t nbatch);
// Whether the arithmetic has a kernel with this tile configuration.
bool tile_ok(Acc acc, int cfg);
// Arithmetic a step of a plan runs in.  A split-form step runs the FP32 form
// where the split has nothing to win: an operand the wide kernel cannot take
// (one column: a matrix-vector product), or at most 16 terms (nS <= 2 shared
// cuts; such a step is bound by its output writes, and FP32 products are at
// least as accurate as the BF16 ones).
inline Acc step_acc(Acc acc, bool wide_ok, int nS) {
  return is_split(acc) && (!wide_ok || nS <= 2) ? Acc::F32 : acc;
}

Status launch_row_flags(const FlagArgs &a, int64_t total_blocks, hipStream_t s);
Status launch_mass_final(const double *partials, int64_t count, double *mass, hipStream_t s,
                         const int32_t *gate = nullptr, int32_t gate_val = 0);

// One launch over many contraction steps of the same kernel configuration:
// descs[d] in device memory, prefix[d] = first queue item of step d (items of
// step d are its tiles), queue = zeroed counter.
struct QueueLaunch {
  const ContractArgs *descs;
  const int64_t *prefix;
  int32_t ndesc;
  unsigned long long *queue;
  int64_t total;
  uint32_t grid;
  const int64_t *bprefix;  // wide kernel: bprefix[d] = first batch entry of step d over the table
  int64_t btotal;          //   and the total (one label-list block per batch entry)
  int xent = 0;            // final steps of the cross-entropy form (ContractArgs::xt):
                           //   1 gradient (partials sum p), 2 gradient and loss
};
Status launch_contract_queue(Acc acc, int mode, int cfg, bool small, const QueueLaunch &q, hipStream_t s);
// Two-tile strips of the 64 x 256 FP32 small-term kernel (FP32 output, blocked
// or intermediate mode, no row flags): a step of nblocks tiles is nblocks /
// kStripRows queue items.
constexpr int kStripRows = 2;
Status launch_contract_strip_queue(int mode, const QueueLaunch &q, hipStream_t s);

// Batched row flags (descriptor table in device memory, block_start = prefix)
// and per-instance mass reductions; the flag pass also zeroes `counters`.
struct MassDesc {
  const double *partials;
  int64_t count;
  double *mass;
};
Status launch_row_flags_table(const FlagDesc *descs, int32_t n, int64_t total_blocks, bool is_double,
                              unsigned long long *counters, int32_t n_counters, hipStream_t s);
Status launch_mass_table(const MassDesc *descs, int32_t n, hipStream_t s);
Status launch_contract(Acc acc, bool out_double, int cfg, const ContractArgs &a, hipStream_t s);
Status launch_contract_wide(int parts, bool out_double, const ContractArgs &a, hipStream_t s);
// Splits `count` floats (a multiple of 4) into `parts` bfloat16 planes of
// `plane` elements each (the same split as the wide kernel's staging).
Status launch_presplit(int parts, const float *src, void *dst, int64_t count, int64_t plane, hipStream_t s);
// Whether both operands of a step are within the wide kernel's 2^30-element addressing.
bool wide_fits(const ContractArgs &a);
Status launch_contract_wide_queue(int parts, int mode, const QueueLaunch &q, hipStream_t s);
Status launch_convert(const void *src, bool src_double, void *dst, bool dst_double,
                      int64_t count, hipStream_t s);
Status launch_selftest_mfma(void *out, hipStream_t s);

}  // namespace cqc
