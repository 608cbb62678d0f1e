// Device helpers shared by the contraction kernels (gfx950 only).
#pragma once

#include <cmath>

#include "kernels.hpp"

namespace cqc {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct MfmaOp;
// Accumulator layout of one 16x16 block (measured by k_selftest_mfma):
//   FP32: lane l, register r holds row 4*(l/16) + r   (4 consecutive rows)
//   FP64: lane l, register r holds row (l/16) + 4*r   (rows strided by 4)
// of column l%16, where "row" is the index contributed by the A operand.
template <> struct MfmaOp<float> {
  using V = f32x4;
  static constexpr bool kConsecutive = true;
  static __device__ __forceinline__ V run(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct MfmaOp<double> {
  using V = f64x4;
  static constexpr bool kConsecutive = false;
  static __device__ __forceinline__ V run(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

__device__ __forceinline__ int row_of(const DigitMapDev &m, int s, int r) {
  int row = 0;
#pragma unroll 1
  for (int i = 0; i < m.n; ++i) {
    const int v = ((m.srcmask >> i) & 1u) ? r : s;
    const uint64_t w = i < 10 ? m.shifts[0] : m.shifts[1];
    const int sh = (int)((w >> (6 * (i < 10 ? i : i - 10))) & 63);
    row = (row << 2) | ((v >> sh) & 3);
  }
  return row;
}

__device__ inline int64_t deposit(int64_t v, const BitPos &pos, int nbits) {
  int64_t out = 0;
#pragma unroll 1
  for (int j = 0; j < nbits; ++j) {
    const uint64_t w = pos.w[0] * (j / 10 == 0) + pos.w[1] * (j / 10 == 1) + pos.w[2] * (j / 10 == 2) +
                       pos.w[3] * (j / 10 == 3) + pos.w[4] * (j / 10 == 4);
    out |= ((v >> j) & 1) << ((w >> (6 * (j % 10))) & 63);
  }
  return out;
}

// A launch whose device-side predicate is set and false does nothing.
__device__ __forceinline__ bool gated_off(const int32_t *gate, int32_t val) { return gate && *gate != val; }

// A row is live if any of its chunk flags is set.
__device__ __forceinline__ int row_live(const int32_t *flags, int nch, int row) {
  int any = 0;
  for (int c = 0; c < nch; ++c) any |= flags[(int64_t)row * nch + c];
  return any != 0;
}

// Spread consecutive logical blocks over one XCD: hardware dispatches block i
// to XCD i % 8, so logical tile t lands on XCD t / (nblocks / 8) and tiles that
// share an X row block share that XCD's L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t nblocks) {
  if (nblocks % 8) return bid;
  return (bid % 8) * (nblocks / 8) + bid / 8;
}

template <typename T> __device__ __forceinline__ void load4(const T *p, T *v);
template <> __device__ __forceinline__ void load4<float>(const float *p, float *v) {
  float4 t = *reinterpret_cast<const float4 *>(p);
  v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
}
template <> __device__ __forceinline__ void load4<double>(const double *p, double *v) {
  double2 a = reinterpret_cast<const double2 *>(p)[0];
  double2 b = reinterpret_cast<const double2 *>(p)[1];
  v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}

template <typename T> __device__ __forceinline__ void store4(T *p, const T *v);
template <> __device__ __forceinline__ void store4<float>(float *p, const float *v) {
  *reinterpret_cast<float4 *>(p) = make_float4(v[0], v[1], v[2], v[3]);
}
template <> __device__ __forceinline__ void store4<double>(double *p, const double *v) {
  reinterpret_cast<double2 *>(p)[0] = make_double2(v[0], v[1]);
  reinterpret_cast<double2 *>(p)[1] = make_double2(v[2], v[3]);
}

// Gradient of the cross-entropy L = -sum_x t_x log max(p_x, 1e-30) with respect
// to p_x: -t_x / p_x above the floor, 0 at or below it (flat there).  The floor
// test is made on p widened to FP64, the division in T.
constexpr double kXentFloor = 1e-30;
template <typename T>
__device__ __forceinline__ T xent_grad_of(T p, T t) {
  return (double)p > kXentFloor ? -t / p : T(0);
}

// Partial-sum contribution of one output p of a cross-entropy final step
// (ContractArgs::xt): the loss term -t log max(p, 1e-30) when the loss is
// asked for, else p itself (the mass).  The logarithm is taken in the output
// precision (FP32 outputs: an FP32 logarithm, relative error about 1e-7 per
// term, no larger than what FP32 rounding of p itself leaves in the term;
// the FP64 logarithm is several times the code of the whole store path and
// keeps the epilogues from being unrolled); terms are summed in FP64.
__device__ __forceinline__ double xent_log_floor(float p) {
  return (double)logf((double)p > kXentFloor ? p : (float)kXentFloor);
}
__device__ __forceinline__ double xent_log_floor(double p) { return log(p > kXentFloor ? p : kXentFloor); }
template <typename T>
__device__ __forceinline__ double xent_part(T p, T t, bool loss) {
  return loss ? -(double)t * xent_log_floor(p) : (double)p;
}

// One output p of a cross-entropy final step at element o of the output order:
// gradient to xg, p to z if set; returns the partial-sum contribution.
template <typename T>
__device__ __forceinline__ double xent_put1(const ContractArgs &a, int64_t o, T p, bool loss) {
  const T t = static_cast<const T *>(a.xt)[o];
  if (a.Z) static_cast<T *>(a.Z)[o] = p;
  static_cast<T *>(a.xg)[o] = xent_grad_of(p, t);
  return xent_part(p, t, loss);
}

// Four consecutive outputs at elements o..o+3 (o a multiple of 4): vector
// accesses; the contributions go to c[].
template <typename T>
__device__ __forceinline__ void xent_put4(const ContractArgs &a, int64_t o, const T (&v)[4], double (&c)[4],
                                          bool loss) {
  T t[4], g[4];
  load4<T>(static_cast<const T *>(a.xt) + o, t);
  if (a.Z) store4<T>(static_cast<T *>(a.Z) + o, v);
#pragma unroll
  for (int r = 0; r < 4; ++r) g[r] = xent_grad_of(v[r], t[r]);
  store4<T>(static_cast<T *>(a.xg) + o, g);
#pragma unroll
  for (int r = 0; r < 4; ++r) c[r] = xent_part(v[r], t[r], loss);
}

// FP32 forms with the targets loaded ahead.  A wait for a load also waits for
// every memory access issued before it (loads and stores retire through one
// in-order counter), so a final step that loaded t next to each store would
// wait for its own earlier stores every time: the kernels load the targets of
// a whole tile before its first store instead.  Targets are read once and
// gradients written once: non-temporal accesses.
__device__ __forceinline__ f32x4 xent_t4(const ContractArgs &a, int64_t o) {
  return __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(static_cast<const float *>(a.xt) + o));
}
__device__ __forceinline__ void xent_emit4(const ContractArgs &a, int64_t o, const float (&v)[4], const f32x4 &t,
                                           double (&c)[4], bool loss) {
  if (a.Z) store4<float>(static_cast<float *>(a.Z) + o, v);
  f32x4 g;
#pragma unroll
  for (int r = 0; r < 4; ++r) g[r] = xent_grad_of(v[r], t[r]);
  __builtin_nontemporal_store(g, reinterpret_cast<f32x4 *>(static_cast<float *>(a.xg) + o));
#pragma unroll
  for (int r = 0; r < 4; ++r) c[r] = xent_part(v[r], t[r], loss);
}

// Wave-wide FP64 sum in a fixed order (butterfly); every lane gets the total.
__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Largest d with prefix[d] <= item (the step a work-queue item belongs to).
// The table is written before the launch and only read during it, and the
// item is the same for the whole block: the search runs on scalar loads
// through the constant address space, which wait on the scalar counter - not
// behind this wave's outstanding vector loads and output stores, as a chain
// of dependent vector loads would.
__device__ __forceinline__ int find_desc(const int64_t *prefix, int n, int64_t item) {
  using cp = const __attribute__((address_space(4))) int64_t *;
  const cp tab = (cp)(const __attribute__((address_space(1))) int64_t *)prefix;
  const int64_t it = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(item >> 32)) << 32) |
                               (uint32_t)__builtin_amdgcn_readfirstlane((int32_t)item));
  int lo = 0, hi = __builtin_amdgcn_readfirstlane(n - 1);   // largest d with prefix[d] <= it
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tab[mid] <= it) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

}  // namespace cqc
