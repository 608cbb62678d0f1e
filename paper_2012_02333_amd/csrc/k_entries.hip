// On-device entry construction (Sections 3.1-3.2, Pauli form): E_c of a
// subcircuit from the stacked distributions of its variants.
//
// One thread per (outgoing-label combination, output column x): for every
// initialisation combination it adds the measured cut bits of the basis
// combination its outgoing labels select, signed by Eq. 3 (FP64), then
// applies the incoming cuts' initialisation weights one cut at a time as
// 4 x 4 mode products on the per-thread vector of initialisation
// combinations, and writes one entry per incoming-label combination.
// Consecutive threads take consecutive x: every read of a measured-bit string
// and every entry write is coalesced across the wave.  The tensor is read
// about once per outgoing label that shares its basis combination (I and Z
// share the computational basis) and written once: memory-bound.
#include <algorithm>
#include <string>

#include "entries.hpp"

namespace cqc {

// Pauli-form initialisation weights w[label][init] over (|0>, |1>, |+>, |+i>).
__device__ __forceinline__ double init_weight(int label, int init) {
  switch (label) {
    case 0: return init < 2 ? 1.0 : 0.0;                                  // I: q0 + q1
    case 3: return init == 0 ? 1.0 : (init == 1 ? -1.0 : 0.0);            // Z: q0 - q1
    case 1: return init < 2 ? -1.0 : (init == 2 ? 2.0 : 0.0);             // X: 2 q+ - q0 - q1
    default: return init < 2 ? -1.0 : (init == 3 ? 2.0 : 0.0);            // Y: 2 q+i - q0 - q1
  }
}

template <typename TI, typename TO, int KIN>
__global__ __launch_bounds__(256) void k_build_entries(const EntryArgs a) {
  constexpr int NI = 1 << (2 * KIN);
  const int64_t nx = int64_t(1) << a.f;
  const int kout = a.k_out;
  const int64_t total = (int64_t(1) << (2 * kout)) * nx;
  const int nb = 1 << kout;
  const TI *V = static_cast<const TI *>(a.V);
  TO *E = static_cast<TO *>(a.E);
  for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < total;
       id += (int64_t)gridDim.x * blockDim.x) {
    const int64_t x = id & (nx - 1);
    const int lo = (int)(id >> a.f);   // outgoing labels, first outgoing cut most significant
    int bi = 0;                        // basis combination, base 3
    uint32_t mask = 0;                 // measured bits whose label is not I flip the sign
    int64_t rowo = 0;                  // the outgoing labels' part of the row number
    for (int t = 0; t < kout; ++t) {
      const int l = (lo >> (2 * (kout - 1 - t))) & 3;
      bi = 3 * bi + (l == 1 ? 1 : (l == 2 ? 2 : 0));
      if (l != 0) mask |= 1u << (kout - 1 - t);
      rowo += (int64_t)l << (2 * (a.k - 1 - a.out_pos[t]));
    }
    double u[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      const TI *v = V + (((int64_t)i * a.p3 + bi) * nx + x) * nb;
      double s = 0.0;
      if (sizeof(TI) == 4 && a.vec && nb >= 4) {
        // the thread's measured-bit string is nb contiguous floats: 16-byte loads
        for (int b = 0; b < nb; b += 4) {
          const float4 q = *reinterpret_cast<const float4 *>(v + b);
          const float w4[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const double w = (double)w4[e];
            s += (__popc((uint32_t)(b + e) & mask) & 1) ? -w : w;
          }
        }
      } else {
        for (int b = 0; b < nb; ++b) {
          const double w = (double)v[b];
          s += (__popc((uint32_t)b & mask) & 1) ? -w : w;
        }
      }
      u[i] = s;
    }
    // initialisation weights, one incoming cut (base-4 digit t) at a time
#pragma unroll
    for (int t = 0; t < KIN; ++t) {
      const int sh = 2 * (KIN - 1 - t);
#pragma unroll
      for (int rest = 0; rest < NI / 4; ++rest) {
        // index with digit t cleared: low digits below t stay, high digits shift up
        const int lowmask = (1 << sh) - 1;
        const int base = ((rest & ~lowmask) << 2) | (rest & lowmask);
        const double u0 = u[base], u1 = u[base | (1 << sh)], u2 = u[base | (2 << sh)], u3 = u[base | (3 << sh)];
#pragma unroll
        for (int l = 0; l < 4; ++l)
          u[base | (l << sh)] = init_weight(l, 0) * u0 + init_weight(l, 1) * u1 + init_weight(l, 2) * u2 +
                                init_weight(l, 3) * u3;
      }
    }
#pragma unroll
    for (int li = 0; li < NI; ++li) {
      int64_t row = rowo;
#pragma unroll
      for (int t = 0; t < KIN; ++t) row += (int64_t)((li >> (2 * (KIN - 1 - t))) & 3) << (2 * (a.k - 1 - a.in_pos[t]));
      E[row * nx + x] = (TO)u[li];
    }
  }
}

template <typename TI, typename TO>
static Status launch_entries_t(const EntryArgs &a, hipStream_t s) {
  const int64_t total = (int64_t(1) << (2 * a.k_out)) << a.f;
  const dim3 g((unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 65536))), b(256);
  switch (a.k_in) {
    case 0: return launch("build_entries", k_build_entries<TI, TO, 0>, g, b, 0, s, a);
    case 1: return launch("build_entries", k_build_entries<TI, TO, 1>, g, b, 0, s, a);
    case 2: return launch("build_entries", k_build_entries<TI, TO, 2>, g, b, 0, s, a);
    case 3: return launch("build_entries", k_build_entries<TI, TO, 3>, g, b, 0, s, a);
    default: return Status::fail(CQC_ERR_UNSUPPORTED, "more than 3 incoming cuts");
  }
}

Status launch_build_entries(const EntryArgs &a, bool in_double, bool out_double, hipStream_t s) {
  if (in_double)
    return out_double ? launch_entries_t<double, double>(a, s) : launch_entries_t<double, float>(a, s);
  return out_double ? launch_entries_t<float, double>(a, s) : launch_entries_t<float, float>(a, s);
}

}  // namespace cqc
