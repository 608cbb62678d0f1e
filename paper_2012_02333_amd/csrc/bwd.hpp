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
};

Status launch_bwd(Acc acc, const BwdArgs &a, bool which_y, hipStream_t s);
Status launch_bwd_reduce(Acc acc, const void *part, int64_t count, int64_t P, double scale,
                         void *out, bool out_double, hipStream_t s);
Status launch_gather_blocked(Acc acc, const void *src, void *dst, int logM, int logN,
                             const BitPos &px, const BitPos &py, hipStream_t s);

}  // namespace cqc
