// On-device entry construction: device argument block and launcher.
#pragma once

#include "common.hpp"

namespace cqc {

constexpr int kEntryMaxIn = 3;    // incoming (initialised) cuts per subcircuit
constexpr int kEntryMaxOut = 4;   // outgoing (measured) cuts per subcircuit

struct EntryArgs {
  const void *V;   // [4^k_in][3^k_out][2^f][2^k_out]
  void *E;         // [4^k][2^f]
  int32_t f, k_in, k_out, k;
  int32_t p3;      // 3^k_out
  int32_t vec;     // FP32 variants 16-byte aligned: measured-bit strings read with 16-byte loads
  int32_t eigen;   // entry form: 0 Pauli (Eq. 1 and 3), 1 eigen (Eq. 2)
  int32_t in_pos[kEntryMaxIn];    // digit of the i-th incoming cut in the row number (0: most significant)
  int32_t out_pos[kEntryMaxOut];  // same for the outgoing cuts
};

Status launch_build_entries(const EntryArgs &a, bool in_double, bool out_double, hipStream_t s);

}  // namespace cqc
