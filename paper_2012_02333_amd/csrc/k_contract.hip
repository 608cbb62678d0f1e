// Pairwise contraction kernel of the FD/DD term sum on CDNA4 matrix cores.
//
// One launch executes one contraction step of the plan as a batched GEMM with
// gathered operand rows:
//     C_b[m][n] = sum_{s live} X[rowX(s, rX)][m] * Y[rowY(s, rY)][n]
// Both operands are "k-major" (a label row is a contiguous vector over output
// columns), so every LDS stage loads whole row segments with 16-byte loads.
// The inner index s enumerates the assignments of the shared cut labels; a
// term whose X row or Y row is entirely zero is dropped before it reaches the
// matrix cores (early termination, Section 4.2).  Live terms are compacted
// per 256-label chunk in ascending s, so the accumulation order is fixed.
//
// Matrix-core mapping (16x16x4, one block): MFMA row i <-> output column n,
// MFMA column j <-> output row m.  In FP32 each lane ends with 4 consecutive n
// of one m and stores them as one 16-byte vector (16 lanes cover 64 contiguous
// bytes of an output row); the FP64 accumulator strides its rows by 4, so the
// FP64 form stores element by element.  The last step scales by 2^-K (exact) and reduces
// the FP64 sum of everything it wrote: per-block partials, then the last
// block to finish adds the partials in block order.
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
    int v = m.src[i] ? r : s;
    row = (row << 2) | ((v >> m.shift[i]) & 3);
  }
  return row;
}

__device__ __forceinline__ int64_t deposit(int64_t v, const int8_t *pos, int nbits) {
  int64_t out = 0;
#pragma unroll 1
  for (int j = 0; j < nbits; ++j) out |= ((v >> j) & 1) << pos[j];
  return out;
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

__device__ __forceinline__ double atomic_load_f64(const double *p) {
  unsigned long long u = __hip_atomic_load(reinterpret_cast<const unsigned long long *>(p),
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return __longlong_as_double((long long)u);
}

// Block-wide FP64 sum in a fixed order (wave butterfly, then waves 0..3).
__device__ __forceinline__ double block_sum_f64(double v, double *red) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) t = ((red[0] + red[1]) + red[2]) + red[3];
  __syncthreads();
  return t;
}

// Last block of the grid adds all per-block partials in block order.
__device__ void finish_mass(const ContractArgs &a, int64_t my_block, double block_total,
                            double *red) {
  __shared__ int is_last;
  if (threadIdx.x == 0) {
    a.partials[my_block] = block_total;
    __threadfence();
    unsigned prev = atomicAdd(a.counter, 1u);
    is_last = (prev == (unsigned)(a.nblocks - 1));
  }
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  double v = 0.0;
  for (int64_t i = threadIdx.x; i < a.nblocks; i += blockDim.x) v += atomic_load_f64(&a.partials[i]);
  // fixed-order tree over the 256 thread sums
  __shared__ double tsum[256];
  tsum[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) tsum[threadIdx.x] += tsum[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (a.mass) a.mass[0] = tsum[0];
    *a.counter = 0u;
  }
  (void)red;
}

template <typename T, typename O, int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(256) void k_contract(const ContractArgs a) {
  constexpr int BK = 16;
  constexpr int TM = BM / WM, TN = BN / WN;
  constexpr int BMB = TM / 16, BNB = TN / 16;
  constexpr int PAD = sizeof(T) == 4 ? 16 : 8;
  static_assert(WM * WN == 4, "four waves");
  static_assert(BMB >= 1 && BNB >= 1, "wave tile at least 16x16");
  using Op = MfmaOp<T>;
  using V = typename Op::V;

  __shared__ T Xs[BK][BM + PAD];
  __shared__ T Ys[BK][BN + PAD];
  __shared__ int2 lst[256];
  __shared__ int wcnt[4];
  __shared__ double red[4];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t blk = xcd_remap(blockIdx.x, a.nblocks);
  const int64_t tiles = (int64_t)a.tilesM * a.tilesN;
  const int64_t batch = blk / tiles;
  const int64_t t = blk - batch * tiles;
  const int tm = (int)(t / a.tilesN), tn = (int)(t - (int64_t)tm * a.tilesN);
  const int rX = (int)(batch >> (2 * a.nRY));
  const int rY = (int)(batch & ((int64_t(1) << (2 * a.nRY)) - 1));
  const int64_t M = int64_t(1) << a.logM, N = int64_t(1) << a.logN;
  const int64_t m0 = (int64_t)tm * BM, n0 = (int64_t)tn * BN;
  const int wm0 = (wave / WN) * TM, wn0 = (wave % WN) * TN;
  const T *X = static_cast<const T *>(a.X);
  const T *Y = static_cast<const T *>(a.Y);

  V acc[BMB][BNB];
#pragma unroll
  for (int i = 0; i < BMB; ++i)
#pragma unroll
    for (int j = 0; j < BNB; ++j) acc[i][j] = V{0, 0, 0, 0};

  const int nSv = 1 << (2 * a.nS);
  int total_live = 0;
  for (int s0 = 0; s0 < nSv; s0 += 256) {
    // ---- compact the live labels of this chunk, ascending s
    const int s = s0 + tid;
    int live = 0, rx = 0, ry = 0;
    if (s < nSv) {
      rx = row_of(a.mx, s, rX);
      ry = row_of(a.my, s, rY);
      live = (a.flagX[rx] != 0) && (a.flagY[ry] != 0);
    }
    const unsigned long long bal = __ballot(live);
    const int pre = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wcnt[wave] = __popcll(bal);
    __syncthreads();
    int base = 0;
    for (int w = 0; w < wave; ++w) base += wcnt[w];
    const int cnt = wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
    if (live) lst[base + pre] = make_int2(rx, ry);
    __syncthreads();
    total_live += cnt;

    for (int k0 = 0; k0 < cnt; k0 += BK) {
      // ---- stage BK gathered rows of X (BM wide) and Y (BN wide) in LDS
      for (int idx = tid * 4; idx < BK * BM; idx += 1024) {
        const int r = idx / BM, c = idx - r * BM;
        T v[4] = {0, 0, 0, 0};
        if (k0 + r < cnt) {
          const T *src = X + (int64_t)lst[k0 + r].x * M + m0 + c;
          if (m0 + c + 3 < M) load4<T>(src, v);
          else
            for (int e = 0; e < 4; ++e)
              if (m0 + c + e < M) v[e] = src[e];
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) Xs[r][c + e] = v[e];
      }
      for (int idx = tid * 4; idx < BK * BN; idx += 1024) {
        const int r = idx / BN, c = idx - r * BN;
        T v[4] = {0, 0, 0, 0};
        if (k0 + r < cnt) {
          const T *src = Y + (int64_t)lst[k0 + r].y * N + n0 + c;
          if (n0 + c + 3 < N) load4<T>(src, v);
          else
            for (int e = 0; e < 4; ++e)
              if (n0 + c + e < N) v[e] = src[e];
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) Ys[r][c + e] = v[e];
      }
      __syncthreads();
      // ---- matrix cores
#pragma unroll
      for (int kq = 0; kq < BK; kq += 4) {
        const int kr = kq + (lane >> 4);
        T bx[BMB], ay[BNB];
#pragma unroll
        for (int i = 0; i < BMB; ++i) bx[i] = Xs[kr][wm0 + i * 16 + (lane & 15)];
#pragma unroll
        for (int j = 0; j < BNB; ++j) ay[j] = Ys[kr][wn0 + j * 16 + (lane & 15)];
#pragma unroll
        for (int i = 0; i < BMB; ++i)
#pragma unroll
          for (int j = 0; j < BNB; ++j) acc[i][j] = Op::run(ay[j], bx[i], acc[i][j]);
      }
      __syncthreads();
    }
  }

  // ---- epilogue
  double msum = 0.0;
  const bool final_mode = a.mode != kModeIntermediate;
  const O scale = (O)a.scale;
#pragma unroll
  for (int i = 0; i < BMB; ++i) {
    const int64_t m = m0 + wm0 + i * 16 + (lane & 15);
    if (m >= M) continue;
#pragma unroll
    for (int j = 0; j < BNB; ++j) {
      const int64_t nb = n0 + wn0 + j * 16;
      if (Op::kConsecutive) {
        const int64_t n = nb + 4 * (lane >> 4);
        if (n >= N) continue;
        if (a.mode == kModeIntermediate) {
          T *Z = static_cast<T *>(a.Z) + batch * M * N + m * N + n;
          T w[4] = {acc[i][j][0], acc[i][j][1], acc[i][j][2], acc[i][j][3]};
          if (n + 3 < N) store4<T>(Z, w);
          else
            for (int r = 0; r < 4; ++r)
              if (n + r < N) Z[r] = w[r];
        } else {
          O v[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) v[r] = (O)acc[i][j][r] * scale;
          if (a.mode == kModeFinalBlocked) {
            O *Z = static_cast<O *>(a.Z) + m * N + n;
            if (n + 3 < N) store4<O>(Z, v);
            else
              for (int r = 0; r < 4; ++r)
                if (n + r < N) Z[r] = v[r];
          } else {
            O *Z = static_cast<O *>(a.Z);
            const int64_t ro = deposit(m, a.posX, a.logM);
            for (int r = 0; r < 4; ++r)
              if (n + r < N) Z[ro + deposit(n + r, a.posY, a.logN)] = v[r];
          }
          for (int r = 0; r < 4; ++r)
            if (n + r < N) msum += (double)v[r];
        }
      } else {
        // rows strided by 4: one element per register
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t n = nb + (lane >> 4) + 4 * r;
          if (n >= N) continue;
          if (a.mode == kModeIntermediate) {
            static_cast<T *>(a.Z)[batch * M * N + m * N + n] = acc[i][j][r];
          } else {
            const O v = (O)acc[i][j][r] * scale;
            if (a.mode == kModeFinalBlocked)
              static_cast<O *>(a.Z)[m * N + n] = v;
            else
              static_cast<O *>(a.Z)[deposit(m, a.posX, a.logM) + deposit(n, a.posY, a.logN)] = v;
            msum += (double)v;
          }
        }
      }
    }
  }
  (void)final_mode;
  if (a.mode == kModeIntermediate) {
    if (a.flagZ && tm == 0 && tn == 0 && tid == 0) a.flagZ[batch] = total_live > 0;
    return;
  }
  if (a.partials) {
    const double tot = block_sum_f64(msum, red);
    finish_mass(a, blockIdx.x, tot, red);
  }
}

// ---------------------------------------------------------------------------
// Row flags of the entry tensors: flag[r] = row r has a non-zero element.
__global__ __launch_bounds__(256) void k_row_flags(const FlagArgs a) {
  const int64_t bid = blockIdx.x;
  int i = 0;
  while (i + 1 < a.n && bid >= a.d[i + 1].row_start) ++i;
  const FlagDesc &d = a.d[i];
  const int64_t r = bid - d.row_start;
  int any = 0;
  if (a.is_double) {
    const double *p = static_cast<const double *>(d.ptr) + r * d.cols;
    for (int64_t c = threadIdx.x; c < d.cols; c += blockDim.x) any |= (p[c] != 0.0);
  } else {
    const float *p = static_cast<const float *>(d.ptr) + r * d.cols;
    for (int64_t c = threadIdx.x; c < d.cols; c += blockDim.x) any |= (p[c] != 0.0f);
  }
  any = __syncthreads_or(any);
  if (threadIdx.x == 0) {
    d.flags[r] = any ? 1 : 0;
    if (bid == 0) {
      if (a.counter) *a.counter = 0u;
      if (a.unit) {
        if (a.is_double) *static_cast<double *>(a.unit) = 1.0;
        else *static_cast<float *>(a.unit) = 1.0f;
        *a.unit_flag = 1;
      }
    }
  }
}

template <typename S, typename D>
__global__ __launch_bounds__(256) void k_convert(const S *src, D *dst, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (D)src[i];
}

// Lane-layout probe: D = A * B for one 16x16x4 block with A[i][k] = i + 16 k,
// B[k][j] = 1 + k + 4 j (exact in FP32), stored as D[i][j] by the accumulator
// layouts the contraction kernel relies on (MfmaOp above).
__global__ void k_selftest_mfma(float *outf, double *outd) {
  const int lane = threadIdx.x;
  const int i = lane & 15, k = lane >> 4, j = lane & 15;
  f32x4 cf = {0, 0, 0, 0};
  cf = __builtin_amdgcn_mfma_f32_16x16x4f32((float)(i + 16 * k), (float)(1 + k + 4 * j), cf, 0, 0, 0);
  f64x4 cd = {0, 0, 0, 0};
  cd = __builtin_amdgcn_mfma_f64_16x16x4f64((double)(i + 16 * k), (double)(1 + k + 4 * j), cd, 0, 0, 0);
  for (int r = 0; r < 4; ++r) {
    const int col = lane & 15;
    outf[(4 * (lane >> 4) + r) * 16 + col] = cf[r];
    outd[((lane >> 4) + 4 * r) * 16 + col] = cd[r];
  }
}

// ---------------------------------------------------------------------------
TileShape tile_shape(int cfg) {
  switch (cfg) {
    case kTileL: return {64, 256};
    case kTileM: return {32, 128};
    case kTileS: return {16, 64};
    default: return {256, 16};
  }
}

int choose_tile(int logM, int logN) {
  const int64_t M = int64_t(1) << logM, N = int64_t(1) << logN;
  if (M >= 64 && N >= 256) return kTileL;
  if (N < 64 && M >= 256) return kTileT;
  if (M >= 32 && N >= 128) return kTileM;
  return kTileS;
}

template <typename T, typename O>
static Status launch_contract_t(int cfg, const ContractArgs &a, hipStream_t s) {
  const dim3 grid((unsigned)a.nblocks), block(256);
  switch (cfg) {
    case kTileL: return launch("contract_64x256", k_contract<T, O, 64, 256, 1, 4>, grid, block, 0, s, a);
    case kTileM: return launch("contract_32x128", k_contract<T, O, 32, 128, 1, 4>, grid, block, 0, s, a);
    case kTileS: return launch("contract_16x64", k_contract<T, O, 16, 64, 1, 4>, grid, block, 0, s, a);
    default: return launch("contract_256x16", k_contract<T, O, 256, 16, 4, 1>, grid, block, 0, s, a);
  }
}

Status launch_contract(Acc acc, bool out_double, int cfg, const ContractArgs &a, hipStream_t s) {
  if (acc == Acc::F32)
    return out_double ? launch_contract_t<float, double>(cfg, a, s)
                      : launch_contract_t<float, float>(cfg, a, s);
  return out_double ? launch_contract_t<double, double>(cfg, a, s)
                    : launch_contract_t<double, float>(cfg, a, s);
}

Status launch_row_flags(const FlagArgs &a, int64_t total_rows, hipStream_t s) {
  return launch("row_flags", k_row_flags, dim3((unsigned)total_rows), dim3(256), 0, s, a);
}

Status launch_convert(const void *src, bool src_double, void *dst, bool dst_double,
                      int64_t count, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>((count + 255) / 256, 4096);
  if (blocks == 0) return Status::ok();
  if (src_double && !dst_double)
    return launch("convert_f64_f32", k_convert<double, float>, dim3((unsigned)blocks), dim3(256), 0, s,
                  static_cast<const double *>(src), static_cast<float *>(dst), count);
  if (!src_double && dst_double)
    return launch("convert_f32_f64", k_convert<float, double>, dim3((unsigned)blocks), dim3(256), 0, s,
                  static_cast<const float *>(src), static_cast<double *>(dst), count);
  return Status::fail(CQC_ERR_INVALID_ARG, "convert: same dtype");
}

Status launch_selftest_mfma(void *out, hipStream_t s) {
  float *of = static_cast<float *>(out);
  double *od = reinterpret_cast<double *>(of + 256);
  return launch("selftest_mfma", k_selftest_mfma, dim3(1), dim3(64), 0, s, of, od);
}

}  // namespace cqc
