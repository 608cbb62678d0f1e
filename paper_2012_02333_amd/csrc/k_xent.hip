// Cross-entropy against a target distribution over reconstructed outputs, and
// its gradient, in one pass: L = -sum_x t_x log max(p_x, 1e-30) and
// dL/dp_x = -t_x / p_x where p_x > 1e-30, else 0 (the floor is flat there).
// This is the loss the adjoint of the reconstruction is driven by; the
// floor test is made on p widened exactly to FP64.
//
// Each block takes a contiguous range that starts on a multiple of 1024
// elements; each thread takes groups of four consecutive elements (16-byte
// loads and stores for aligned FP32 buffers, the same groups by scalar access
// otherwise).  With the loss requested, every block leaves its FP64 partial
// and one block adds the partials in block order, so the loss is bitwise
// reproducible for a given n.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>

#include "kdev.hpp"

namespace cqc {

constexpr int kXentMaxBlocks = 1024;

typedef float xf4 __attribute__((ext_vector_type(4)));

// every element is touched once: non-temporal loads and stores
template <bool VEC, typename T>
__device__ __forceinline__ void xload4(const T *p, int64_t i, T (&v)[4]) {
  if constexpr (VEC && sizeof(T) == 4) {
    const xf4 q = __builtin_nontemporal_load(reinterpret_cast<const xf4 *>(p + i));
    v[0] = q[0], v[1] = q[1], v[2] = q[2], v[3] = q[3];
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = p[i + k];
  }
}

template <bool VEC, typename T>
__device__ __forceinline__ void xstore4(T *p, int64_t i, const T (&v)[4]) {
  if constexpr (VEC && sizeof(T) == 4) {
    __builtin_nontemporal_store(xf4{v[0], v[1], v[2], v[3]}, reinterpret_cast<xf4 *>(p + i));
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) p[i + k] = v[k];
  }
}

template <bool LOSS, typename T>
__device__ __forceinline__ T xent_one(T p, T t, double &loss) {
  if constexpr (LOSS) loss -= (double)t * log((double)p > kXentFloor ? (double)p : kXentFloor);
  return xent_grad_of(p, t);
}

template <bool VEC, bool LOSS, typename T>
__global__ __launch_bounds__(256) void k_xent(const T *p, const T *t, int64_t n, int64_t per, T *g,
                                              double *part) {
  const int64_t i0 = (int64_t)blockIdx.x * per, i1 = n < i0 + per ? n : i0 + per;
  double loss = 0.0;
  int64_t i = i0 + 4 * (int64_t)threadIdx.x;
  // with the loss (FP64 logarithms: arithmetic-heavy) four groups per thread
  // at a time, all loads issued before the first use; each thread still takes
  // its groups in increasing order, so the loss sums in the same order as one
  // group at a time.  Without it one group at a time streams faster.
  if constexpr (LOSS) {
    for (; i + 3 * 1024 + 4 <= i1; i += 4 * 1024) {
      T pv[4][4], tv[4][4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        xload4<VEC>(p, i + u * 1024, pv[u]);
        xload4<VEC>(t, i + u * 1024, tv[u]);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        T gv[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) gv[k] = xent_one<LOSS>(pv[u][k], tv[u][k], loss);
        xstore4<VEC>(g, i + u * 1024, gv);
      }
    }
  }
  for (; i + 4 <= i1; i += 1024) {
    T pv[4], tv[4], gv[4];
    xload4<VEC>(p, i, pv);
    xload4<VEC>(t, i, tv);
#pragma unroll
    for (int k = 0; k < 4; ++k) gv[k] = xent_one<LOSS>(pv[k], tv[k], loss);
    xstore4<VEC>(g, i, gv);
  }
  for (int k = 0; k < 4 && i + k < i1; ++k) g[i + k] = xent_one<LOSS>(p[i + k], t[i + k], loss);
  if constexpr (LOSS) {
    __shared__ double red[4];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) loss += __shfl_xor(loss, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = loss;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
  }
}

__global__ __launch_bounds__(256) void k_xent_final(const double *part, int g, double *out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < g; i += 256) s += part[i];
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = ((red[0] + red[1]) + red[2]) + red[3];
}

template <typename T>
static Status launch_xent_t(const void *p, const void *t, int64_t n, void *g, double *loss, double *part,
                            hipStream_t s) {
  const int64_t blocks = n == 0 ? 0 : std::min<int64_t>(kXentMaxBlocks, (n + 4095) / 4096);
  const int64_t per = blocks == 0 ? 0 : ((n + blocks - 1) / blocks + 1023) / 1024 * 1024;
  const bool vec = sizeof(T) == 4 && reinterpret_cast<uintptr_t>(p) % 16 == 0 &&
                   reinterpret_cast<uintptr_t>(t) % 16 == 0 && reinterpret_cast<uintptr_t>(g) % 16 == 0;
  const T *pp = static_cast<const T *>(p), *tp = static_cast<const T *>(t);
  T *gp = static_cast<T *>(g);
  const dim3 grid((unsigned)blocks), block(256);
  if (blocks > 0) {
    if (loss)
      CQC_TRY(vec ? launch("xent", k_xent<true, true, T>, grid, block, 0, s, pp, tp, n, per, gp, part)
                  : launch("xent", k_xent<false, true, T>, grid, block, 0, s, pp, tp, n, per, gp, part));
    else
      CQC_TRY(vec ? launch("xent", k_xent<true, false, T>, grid, block, 0, s, pp, tp, n, per, gp, part)
                  : launch("xent", k_xent<false, false, T>, grid, block, 0, s, pp, tp, n, per, gp, part));
  }
  if (loss) return launch("xent_final", k_xent_final, dim3(1), dim3(256), 0, s, part, (int)blocks, loss);
  return Status::ok();
}

}  // namespace cqc

using namespace cqc;

extern "C" {

int cqc_xent_grad(const void *p, const void *t, cqc_dtype dt, int64_t n, void *grad, double *loss,
                  void *workspace, size_t ws_bytes, hipStream_t stream) {
  if (dt != CQC_F32 && dt != CQC_F64) return Status::fail(CQC_ERR_INVALID_ARG, "unknown dtype").code;
  if (n < 0) return Status::fail(CQC_ERR_INVALID_ARG, "n < 0").code;
  if (n > 0 && (!p || !t || !grad)) return Status::fail(CQC_ERR_INVALID_ARG, "p, t or grad is NULL").code;
  if (loss && (!workspace || ws_bytes < sizeof(double) * kXentMaxBlocks))
    return Status::fail(CQC_ERR_WORKSPACE, "the loss needs a workspace of " +
                                               std::to_string(sizeof(double) * kXentMaxBlocks) + " bytes")
        .code;
  double *part = static_cast<double *>(workspace);
  return (dt == CQC_F64 ? launch_xent_t<double>(p, t, n, grad, loss, part, stream)
                        : launch_xent_t<float>(p, t, n, grad, loss, part, stream))
      .code;
}

}  // extern "C"
