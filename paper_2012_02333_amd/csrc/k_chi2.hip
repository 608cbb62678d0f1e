// Chi-square distance of two distributions (Eq. 16): sum over i with
// a_i + b_i > 0 of (a_i - b_i)^2 / (a_i + b_i), in FP64.
//
// Two launches with a fixed split: block g of G adds the terms of a
// contiguous range whose start is a multiple of 1024 elements, each thread
// taking groups of four consecutive elements (16-byte loads when both inputs
// are 16-byte aligned, the same groups by scalar loads otherwise, two groups in
// flight per iteration), then the block tree; a single block then adds the G
// partials in block order.  The split and every thread's order of terms depend
// only on n, so a result is bitwise reproducible and independent of alignment.
#include <algorithm>
#include <cstdint>
#include <string>

#include "common.hpp"

namespace cqc {

constexpr int kChi2MaxBlocks = 1024;

typedef float cf4 __attribute__((ext_vector_type(4)));

// every element is read once: non-temporal loads for the FP32 stream
template <bool VEC, typename T>
__device__ __forceinline__ void load4(const T *p, int64_t i, double (&v)[4]) {
  if constexpr (VEC && sizeof(T) == 4) {
    const cf4 q = __builtin_nontemporal_load(reinterpret_cast<const cf4 *>(p + i));
    v[0] = q[0], v[1] = q[1], v[2] = q[2], v[3] = q[3];
  } else if constexpr (VEC) {
    const double2 q0 = *reinterpret_cast<const double2 *>(p + i);
    const double2 q1 = *reinterpret_cast<const double2 *>(p + i + 2);
    v[0] = q0.x, v[1] = q0.y, v[2] = q1.x, v[3] = q1.y;
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = (double)p[i + k];
  }
}

__device__ __forceinline__ double chi2_term(double x, double y) {
  const double t = x + y;
  return t > 0.0 ? (x - y) * (x - y) / t : 0.0;
}

template <bool VEC, typename TA, typename TB>
__global__ __launch_bounds__(256) void k_chi2_part(const TA *a, const TB *b, int64_t n, int64_t per,
                                                   double *part) {
  __shared__ double red[4];
  const int64_t i0 = (int64_t)blockIdx.x * per, i1 = n < i0 + per ? n : i0 + per;
  double s = 0.0;
  int64_t i = i0 + 4 * (int64_t)threadIdx.x;
  for (; i + 1024 + 4 <= i1; i += 2048) {
    double x0[4], y0[4], x1[4], y1[4];
    load4<VEC>(a, i, x0);
    load4<VEC>(b, i, y0);
    load4<VEC>(a, i + 1024, x1);
    load4<VEC>(b, i + 1024, y1);
#pragma unroll
    for (int k = 0; k < 4; ++k) s += chi2_term(x0[k], y0[k]);
#pragma unroll
    for (int k = 0; k < 4; ++k) s += chi2_term(x1[k], y1[k]);
  }
  if (i + 4 <= i1) {
    double x0[4], y0[4];
    load4<VEC>(a, i, x0);
    load4<VEC>(b, i, y0);
#pragma unroll
    for (int k = 0; k < 4; ++k) s += chi2_term(x0[k], y0[k]);
    i += 1024;
  }
  for (int k = 0; k < 4 && i + k < i1; ++k) s += chi2_term((double)a[i + k], (double)b[i + k]);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ __launch_bounds__(256) void k_chi2_final(const double *part, int g, double *out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < g; i += 256) s += part[i];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = ((red[0] + red[1]) + red[2]) + red[3];
}

template <typename TA, typename TB>
static Status launch_chi2_t(const void *a, const void *b, int64_t n, double *part, double *out, hipStream_t s) {
  // per is a multiple of 1024 so every block (and, with aligned inputs,
  // every group of four) starts on a 16-byte boundary
  const int64_t g = n == 0 ? 0 : std::min<int64_t>(kChi2MaxBlocks, (n + 4095) / 4096);
  const int64_t per = g == 0 ? 0 : ((n + g - 1) / g + 1023) / 1024 * 1024;
  const bool vec = (reinterpret_cast<uintptr_t>(a) % 16 == 0) && (reinterpret_cast<uintptr_t>(b) % 16 == 0);
  if (g > 0) {
    const TA *pa = static_cast<const TA *>(a);
    const TB *pb = static_cast<const TB *>(b);
    CQC_TRY(vec ? launch("chi2_part", k_chi2_part<true, TA, TB>, dim3((unsigned)g), dim3(256), 0, s, pa, pb, n, per,
                         part)
                : launch("chi2_part", k_chi2_part<false, TA, TB>, dim3((unsigned)g), dim3(256), 0, s, pa, pb, n,
                         per, part));
  }
  return launch("chi2_final", k_chi2_final, dim3(1), dim3(256), 0, s, part, (int)g, out);
}

Status launch_chi2(const void *a, bool a_double, const void *b, bool b_double, int64_t n, double *part,
                   double *out, hipStream_t s) {
  if (a_double)
    return b_double ? launch_chi2_t<double, double>(a, b, n, part, out, s)
                    : launch_chi2_t<double, float>(a, b, n, part, out, s);
  return b_double ? launch_chi2_t<float, double>(a, b, n, part, out, s)
                  : launch_chi2_t<float, float>(a, b, n, part, out, s);
}

}  // namespace cqc

using namespace cqc;

extern "C" {

int cqc_chi2(const void *a, cqc_dtype a_t, const void *b, cqc_dtype b_t, int64_t n, double *out,
             void *workspace, size_t ws_bytes, hipStream_t stream) {
  if ((a_t != CQC_F32 && a_t != CQC_F64) || (b_t != CQC_F32 && b_t != CQC_F64))
    return Status::fail(CQC_ERR_INVALID_ARG, "unknown dtype").code;
  if (n < 0) return Status::fail(CQC_ERR_INVALID_ARG, "n < 0").code;
  if (!out) return Status::fail(CQC_ERR_INVALID_ARG, "out is NULL").code;
  if (n > 0 && (!a || !b)) return Status::fail(CQC_ERR_INVALID_ARG, "a or b is NULL").code;
  if (!workspace || ws_bytes < sizeof(double) * kChi2MaxBlocks)
    return Status::fail(CQC_ERR_WORKSPACE, "workspace needs " + std::to_string(sizeof(double) * kChi2MaxBlocks) +
                                               " bytes")
        .code;
  return launch_chi2(a, a_t == CQC_F64, b, b_t == CQC_F64, n, static_cast<double *>(workspace), out, stream).code;
}

}  // extern "C"
