// On-device entry construction (Sections 3.1-3.2, Pauli form): E_c of a
// subcircuit from the stacked distributions of its variants.
//
// One thread per (outgoing-label combination, output column x): for every
// initialisation combination it adds the measured cut bits of the basis
// combination its outgoing labels select, weighted per bit by the labels
// (Eq. 3 in the Pauli form: +1, or +1 / -1; Eq. 2's eigen form: 2 / 0, 0 / 2,
// +1 / -1) in FP64, then applies the incoming cuts' initialisation weights one
// cut at a time as 4 x 4 mode products on the per-thread vector of
// initialisation combinations, and writes one entry per incoming-label
// combination.  The form is a template parameter, so the weights are
// compile-time constants.
// Consecutive threads take consecutive x: every read of a measured-bit string
// and every entry write is coalesced across the wave.  The tensor is read
// about once per outgoing label that shares its basis combination (I and Z
// share the computational basis) and written once: memory-bound.
#include <algorithm>
#include <string>

#include "entries.hpp"

namespace cqc {

// Initialisation weight of |0>, |1>, |+>, |+i> (init 0..3) for an incoming
// label: Pauli form I: q0 + q1, X: 2 q+ - q0 - q1, Y: 2 q+i - q0 - q1,
// Z: q0 - q1; eigen form A1: q0, A2: q1, A3, A4 as X, Y.
template <int EIGEN>
__device__ __forceinline__ constexpr double init_weight(int label, int init) {
  if (EIGEN) {
    if (label == 0) return init == 0 ? 1.0 : 0.0;
    if (label == 1) return init == 1 ? 1.0 : 0.0;
  } else {
    if (label == 0) return init < 2 ? 1.0 : 0.0;
    if (label == 3) return init == 0 ? 1.0 : (init == 1 ? -1.0 : 0.0);
  }
  const int plus = EIGEN ? (label == 2 ? 2 : 3) : (label == 1 ? 2 : 3);   // X-like: |+>, Y-like: |+i>
  return init < 2 ? -1.0 : (init == plus ? 2.0 : 0.0);
}

template <typename TI, typename TO, int KIN, int EIGEN>
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
    // weight of measured bit string b: 0 unless (b & zmask) == zval, else
    // scale * (-1)^popcount(b & smask).  Pauli form: I weighs both outcomes
    // +1, X, Y, Z weigh 0 / 1 as +1 / -1.  Eigen form: A1 (A2) keeps only
    // outcome 0 (1) with weight 2, A3, A4 weigh +1 / -1.
    int bi = 0;                        // basis combination, base 3
    int64_t rowo = 0;                  // the outgoing labels' part of the row number
    uint32_t zmask = 0, zval = 0, smask = 0;
    double scale = 1.0;
    for (int t = 0; t < kout; ++t) {
      const int l = (lo >> (2 * (kout - 1 - t))) & 3;
      const uint32_t bit = 1u << (kout - 1 - t);
      rowo += (int64_t)l << (2 * (a.k - 1 - a.out_pos[t]));
      if (EIGEN) {
        bi = 3 * bi + (l < 2 ? 0 : l - 1);
        if (l < 2) {
          zmask |= bit;
          if (l == 1) zval |= bit;
          scale *= 2.0;
        } else {
          smask |= bit;
        }
      } else {
        bi = 3 * bi + (l == 1 ? 1 : (l == 2 ? 2 : 0));
        if (l != 0) smask |= bit;
      }
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
            const uint32_t bb = (uint32_t)(b + e);
            const double w = (double)w4[e];
            if ((bb & zmask) == zval) s += (__popc(bb & smask) & 1) ? -w : w;
          }
        }
      } else {
        for (int b = 0; b < nb; ++b) {
          const double w = (double)v[b];
          if (((uint32_t)b & zmask) == zval) s += (__popc((uint32_t)b & smask) & 1) ? -w : w;
        }
      }
      u[i] = scale * s;
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
          u[base | (l << sh)] = init_weight<EIGEN>(l, 0) * u0 + init_weight<EIGEN>(l, 1) * u1 +
                                init_weight<EIGEN>(l, 2) * u2 + init_weight<EIGEN>(l, 3) * u3;
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
  if (a.eigen) {
    switch (a.k_in) {
      case 0: return launch("build_entries", k_build_entries<TI, TO, 0, 1>, g, b, 0, s, a);
      case 1: return launch("build_entries", k_build_entries<TI, TO, 1, 1>, g, b, 0, s, a);
      case 2: return launch("build_entries", k_build_entries<TI, TO, 2, 1>, g, b, 0, s, a);
      case 3: return launch("build_entries", k_build_entries<TI, TO, 3, 1>, g, b, 0, s, a);
      default: return Status::fail(CQC_ERR_UNSUPPORTED, "more than 3 incoming cuts");
    }
  }
  switch (a.k_in) {
    case 0: return launch("build_entries", k_build_entries<TI, TO, 0, 0>, g, b, 0, s, a);
    case 1: return launch("build_entries", k_build_entries<TI, TO, 1, 0>, g, b, 0, s, a);
    case 2: return launch("build_entries", k_build_entries<TI, TO, 2, 0>, g, b, 0, s, a);
    case 3: return launch("build_entries", k_build_entries<TI, TO, 3, 0>, g, b, 0, s, a);
    default: return Status::fail(CQC_ERR_UNSUPPORTED, "more than 3 incoming cuts");
  }
}

Status launch_build_entries(const EntryArgs &a, bool in_double, bool out_double, hipStream_t s) {
  if (in_double)
    return out_double ? launch_entries_t<double, double>(a, s) : launch_entries_t<double, float>(a, s);
  return out_double ? launch_entries_t<float, double>(a, s) : launch_entries_t<float, float>(a, s);
}

}  // namespace cqc
