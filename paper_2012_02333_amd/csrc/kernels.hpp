// Kernel argument blocks and host launchers of the gfx950 kernels.
#pragma once

#include <cstdint>

#include "common.hpp"

namespace cqc {

struct DigitMapDev {
  int8_t n;
  int8_t src[CQC_MAX_K_SUB + 4];
  int8_t shift[CQC_MAX_K_SUB + 4];
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
  const int32_t *flagX;
  const int32_t *flagY;
  int32_t *flagZ;
  void *Z;
  int32_t logM, logN;
  int32_t nS, nRX, nRY;
  int32_t tilesM, tilesN;
  int32_t mode;
  int64_t nblocks;
  double scale;
  DigitMapDev mx, my;
  int8_t posX[48];   // column bit j (from the least significant) of X -> output bit position
  int8_t posY[48];
  double *partials;  // per-block FP64 sum of written outputs (final mode) or null
  uint32_t *counter; // last-block counter, zeroed by the row-flag kernel
  double *mass;      // FP64 total (final mode) or null
};

struct FlagDesc {
  const void *ptr;
  int64_t rows;
  int64_t cols;
  int32_t *flags;
  int64_t row_start;
};

struct FlagArgs {
  FlagDesc d[CQC_MAX_SUB + 1];
  int32_t n;
  int32_t is_double;
  uint32_t *counter;    // zeroed (may be null)
  void *unit;           // if non-null: one Acc-typed 1.0 written here, unit_flag = 1
  int32_t *unit_flag;
};

enum class Acc { F32, F64 };

// Tile configurations of the contraction kernel.
enum TileCfg : int32_t { kTileL = 0, kTileM = 1, kTileS = 2, kTileT = 3, kTileCount = 4 };
struct TileShape { int bm, bn; };
TileShape tile_shape(int cfg);
int choose_tile(int logM, int logN);

Status launch_row_flags(const FlagArgs &a, int64_t total_rows, hipStream_t s);
Status launch_contract(Acc acc, bool out_double, int cfg, const ContractArgs &a, hipStream_t s);
Status launch_convert(const void *src, bool src_double, void *dst, bool dst_double,
                      int64_t count, hipStream_t s);
Status launch_selftest_mfma(void *out, hipStream_t s);

}  // namespace cqc
