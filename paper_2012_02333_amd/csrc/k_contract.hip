// Pairwise contraction kernel of the FD/DD term sum on CDNA4 matrix cores.
//
// One launch executes one contraction step of the plan as a batched GEMM with
// gathered operand rows:
//     C_b[m][n] = sum_{s live} X[rowX(s, rX)][m] * Y[rowY(s, rY)][n]
// Both operands are "k-major" (a label row is a contiguous vector over output
// columns) and small next to the output, so every wave loads its operands
// straight from L2 into registers in the matrix-core lane layout (16 lanes read
// 16 consecutive columns of one label row) and runs independently of the other
// waves: no LDS staging and no barrier inside the term loop.  The inner index
// s enumerates the assignments of the shared cut labels; a term whose X row or
// Y row is entirely zero is dropped before it reaches the matrix cores (early
// termination, Section 4.2).  Live terms are compacted per 256-label chunk in
// ascending s into a per-block gather list, so the accumulation order is fixed.
//
// Matrix-core mapping (16x16x4, one block): MFMA row i <-> output column n,
// MFMA column j <-> output row m.  In FP32 each lane ends with 4 consecutive n
// of one m and stores them as one 16-byte vector (16 lanes cover 64 contiguous
// bytes of an output row).  The FP64 accumulator strides its rows by 4, so the
// FP64 form swaps the operands (MFMA row <-> m): 16 lanes then hold 16
// consecutive n of one row and store 128 contiguous bytes per register.
// The last step scales by 2^-K (exact) and reduces the FP64 sum of everything
// it wrote: per-block partials, added in block order by k_mass_final.
#include <type_traits>

#include "kdev.hpp"

namespace cqc {

// Cross-entropy form (XE) of four consecutive outputs o..o+3: with the FP32
// target prefetched (pre) or loaded here.
template <typename O>
__device__ __forceinline__ void xent4_at(const ContractArgs &a, int64_t o, const O (&v)[4], bool pre,
                                         const f32x4 &t, double (&c)[4], bool loss) {
  if constexpr (std::is_same<O, float>::value) {
    if (pre) {
      xent_emit4(a, o, v, t, c, loss);
      return;
    }
  }
  xent_put4<O>(a, o, v, c, loss);
}

// FP64 mass: every block of the last step stores the FP64 sum of what it
// wrote; k_mass_final then adds the partials in block order.  (A completion
// counter in the contraction kernel would need a device-scope release fence
// per block, which on a multi-XCD part writes back the L2 - full of freshly
// written outputs - once per block.)
__global__ __launch_bounds__(1024) void k_mass_final(const double *partials, int64_t count,
                                                     double *mass, const int32_t *gate, int32_t gate_val) {
  if (gated_off(gate, gate_val)) return;
  // thread t adds partials t + 1024 (16 q + u) into accumulator u (sixteen
  // loads in flight per thread, missing ones read as zero), then the
  // accumulators, the lanes of each wave (a fixed butterfly) and the sixteen
  // waves are combined in fixed trees: the same order for every call of the
  // same count, with one block barrier
  constexpr int U = 16;
  __shared__ double wsum[16];
  double v[U];
#pragma unroll
  for (int u = 0; u < U; ++u) v[u] = 0.0;
  int64_t i = threadIdx.x;
  for (; i + (U - 1) * 1024 < count; i += U * 1024) {
    double x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) x[u] = partials[i + u * 1024];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] += x[u];
  }
  if (i < count) {
    double x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) x[u] = i + u * 1024 < count ? partials[i + u * 1024] : 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] += x[u];
  }
#pragma unroll
  for (int w = U / 2; w >= 1; w >>= 1)
#pragma unroll
    for (int u = 0; u < w; ++u) v[u] += v[u + w];
  double t = v[0];
  t = wave_sum_f64(t);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x < 64) {
    double w = threadIdx.x < 16 ? wsum[threadIdx.x] : 0.0;
#pragma unroll
    for (int o = 8; o >= 1; o >>= 1) w += __shfl_xor(w, o, 64);
    if (threadIdx.x == 0) mass[0] = w;
  }
}

template <typename T, typename O, int BM, int BN, int WM, int WN, int MODE, int XE = 0>
__device__ __forceinline__ void contract_tile(const ContractArgs &a, uint32_t blk_in) {
  constexpr int TM = BM / WM, TN = BN / WN;     // wave tile
  constexpr int BMB = TM / 16, BNB = TN / 16;    // 16x16 blocks per wave
  constexpr int KG = 4;                          // k-quads per register group (16 terms)
  static_assert(WM * WN == 4, "four waves");
  static_assert(BMB >= 1 && BNB >= 1, "wave tile at least 16x16");
  using Op = MfmaOp<T>;
  using V = typename Op::V;

  __shared__ int2 lst[256 + 16];
  __shared__ int wcnt[4];
  __shared__ int64_t rowoff[MODE == kModeFinalDeposit ? BM : 1];
  __shared__ int64_t coloff[MODE == kModeFinalDeposit ? BN : 1];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t blk = blk_in;
  const int64_t tiles = (int64_t)a.tilesM * a.tilesN;
  const int64_t batch = blk / tiles;
  const int64_t t = blk - batch * tiles;
  const int tm = (int)(t / a.tilesN), tn = (int)(t - (int64_t)tm * a.tilesN);
  const int rX = (int)(batch >> (2 * a.nRY));
  const int rY = (int)(batch & ((int64_t(1) << (2 * a.nRY)) - 1));
  const int64_t M = int64_t(1) << a.logM, N = int64_t(1) << a.logN;
  const int64_t mw = (int64_t)tm * BM + (wave / WN) * TM;   // this wave's first m
  const int64_t nw = (int64_t)tn * BN + (wave % WN) * TN;   // this wave's first n
  const T *X = static_cast<const T *>(a.X);
  const T *Y = static_cast<const T *>(a.Y);
  const int l16 = lane & 15, lg = lane >> 4;
  if (MODE == kModeFinalDeposit) {
    // output offsets of this block's rows and columns (bit deposit, once)
    for (int r = tid; r < BM; r += 256)
      rowoff[r] = (int64_t)tm * BM + r < M ? deposit((int64_t)tm * BM + r, a.posX, a.logM) : 0;
    for (int c = tid; c < BN; c += 256)
      coloff[c] = (int64_t)tn * BN + c < N ? deposit((int64_t)tn * BN + c, a.posY, a.logN) : 0;
  }

  // column offsets of this lane's operands (masked where the tile overhangs)
  int64_t xcol[BMB], ycol[BNB];
  bool xok[BMB], yok[BNB];
#pragma unroll
  for (int i = 0; i < BMB; ++i) { xcol[i] = mw + i * 16 + l16; xok[i] = xcol[i] < M; }
#pragma unroll
  for (int j = 0; j < BNB; ++j) { ycol[j] = nw + j * 16 + l16; yok[j] = ycol[j] < N; }

  V acc[BMB][BNB];
#pragma unroll
  for (int i = 0; i < BMB; ++i)
#pragma unroll
    for (int j = 0; j < BNB; ++j) acc[i][j] = V{0, 0, 0, 0};

  const int nSv = 1 << (2 * a.nS);
  int total_live = 0;
  for (int s0 = 0; s0 < nSv; s0 += 256) {
    // ---- compact the live labels of this chunk, ascending s (zero-padded to 16)
    const int s = s0 + tid;
    int live = 0, rx = 0, ry = 0;
    if (s < nSv) {
      rx = row_of(a.mx, s, rX);
      ry = row_of(a.my, s, rY);
      live = a.flagX ? row_live(a.flagX, a.nchX, rx) & row_live(a.flagY, a.nchY, ry) : 1;
    }
    const unsigned long long bal = __ballot(live);
    const int pre = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wcnt[wave] = __popcll(bal);
    __syncthreads();
    int base = 0;
    for (int w = 0; w < wave; ++w) base += wcnt[w];
    const int cnt = wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
    if (live) lst[base + pre] = make_int2(rx, ry);
    if (tid < 16) lst[cnt + tid] = make_int2(-1, -1);
    __syncthreads();
    total_live += cnt;

    // ---- term sum: operands straight from L2 into registers, 16 terms at a time
    for (int k0 = 0; k0 < cnt; k0 += 4 * KG) {
      T bx[KG][BMB], ay[KG][BNB];
#pragma unroll
      for (int q = 0; q < KG; ++q) {
        const int2 rr = lst[k0 + 4 * q + lg];
        const bool kok = rr.x >= 0;
        const T *xr = X + (int64_t)(kok ? rr.x : 0) * M;
        const T *yr = Y + (int64_t)(kok ? rr.y : 0) * N;
#pragma unroll
        for (int i = 0; i < BMB; ++i) bx[q][i] = (kok && xok[i]) ? xr[xcol[i]] : (T)0;
#pragma unroll
        for (int j = 0; j < BNB; ++j) ay[q][j] = (kok && yok[j]) ? yr[ycol[j]] : (T)0;
      }
#pragma unroll
      for (int q = 0; q < KG; ++q)
#pragma unroll
        for (int i = 0; i < BMB; ++i)
#pragma unroll
          for (int j = 0; j < BNB; ++j)
            acc[i][j] = Op::kConsecutive ? Op::run(ay[q][j], bx[q][i], acc[i][j])
                                         : Op::run(bx[q][i], ay[q][j], acc[i][j]);
    }
    __syncthreads();   // lst is rewritten by the next chunk
  }

  // ---- epilogue
  double msum = 0.0;
  const O scale = (O)a.scale;
  // cross-entropy form: the targets of the whole wave tile before its first store
  constexpr bool kPre = XE && MODE == kModeFinalBlocked && Op::kConsecutive;
  const bool pre = kPre && mw + TM <= M && nw + TN <= N;
  f32x4 tv[kPre ? BMB * BNB : 1];
  if constexpr (kPre) {
    if (pre)
#pragma unroll
      for (int i = 0; i < BMB; ++i)
#pragma unroll
        for (int j = 0; j < BNB; ++j) tv[i * BNB + j] = xent_t4(a, (mw + i * 16 + l16) * N + nw + j * 16 + 4 * lg);
  }
#pragma unroll
  for (int i = 0; i < BMB; ++i) {
#pragma unroll
    for (int j = 0; j < BNB; ++j) {
      const int64_t nb = nw + j * 16;
      if (Op::kConsecutive) {
        const int64_t m = mw + i * 16 + l16;
        const int64_t n = nb + 4 * lg;
        if (m >= M || n >= N) continue;
        if (MODE == kModeIntermediate) {
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
          if constexpr (XE) {
            if (MODE == kModeFinalBlocked && n + 3 < N) {
              double c[4];
              xent4_at<O>(a, m * N + n, v, pre, tv[kPre ? i * BNB + j : 0], c, XE == 2);
              for (int r = 0; r < 4; ++r) msum += c[r];
            } else {
              for (int r = 0; r < 4; ++r)
                if (n + r < N)
                  msum += xent_put1<O>(a, MODE == kModeFinalBlocked ? m * N + n + r
                                                                   : rowoff[m - (int64_t)tm * BM] +
                                                                         coloff[n + r - (int64_t)tn * BN],
                                       v[r], XE == 2);
            }
          } else {
            if (MODE == kModeFinalBlocked) {
              O *Z = static_cast<O *>(a.Z) + m * N + n;
              if (n + 3 < N) store4<O>(Z, v);
              else
                for (int r = 0; r < 4; ++r)
                  if (n + r < N) Z[r] = v[r];
            } else {
              O *Z = static_cast<O *>(a.Z);
              const int64_t ro = rowoff[m - (int64_t)tm * BM];
              for (int r = 0; r < 4; ++r)
                if (n + r < N) Z[ro + coloff[n + r - (int64_t)tn * BN]] = v[r];
            }
            for (int r = 0; r < 4; ++r)
              if (n + r < N) msum += (double)v[r];
          }
        }
      } else {
        // FP64: operands swapped (MFMA row <-> m), so register r of lane l holds
        // output row mb + l/16 + 4r at column nb + l%16: 16 lanes store 128
        // contiguous bytes of one row.
        const int64_t n = nb + l16;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t m = mw + i * 16 + lg + 4 * r;
          if (m >= M || n >= N) continue;
          if (MODE == kModeIntermediate) {
            static_cast<T *>(a.Z)[batch * M * N + m * N + n] = acc[i][j][r];
          } else {
            const O v = (O)acc[i][j][r] * scale;
            const int64_t o = MODE == kModeFinalBlocked
                                  ? m * N + n
                                  : rowoff[m - (int64_t)tm * BM] + coloff[n - (int64_t)tn * BN];
            if constexpr (XE) {
              msum += xent_put1<O>(a, o, v, XE == 2);
            } else {
              static_cast<O *>(a.Z)[o] = v;
              msum += (double)v;
            }
          }
        }
      }
    }
  }
  if (MODE == kModeIntermediate) {
    if (a.flagZ && tm == 0 && tn == 0 && tid == 0) a.flagZ[batch] = total_live > 0;
    return;
  }
  if (a.partials) {
    const double tot = wave_sum_f64(msum);
    if (lane == 0) a.partials[kPartialsPerTile * blk + wave] = tot;
  }
}

// Variant for at most 16 live terms (4^|S| <= 16): the Y operands of every
// term stay in registers, and each 16-row block of the wave tile is written
// as soon as its matrix-core products are done, so stores start early and
// few registers are live (all blocks of a launch fit on the chip at once).
template <typename T, typename O, int BM, int BN, int WM, int WN, int MODE, int XE = 0>
__device__ __forceinline__ void contract_small_tile(const ContractArgs &a, uint32_t blk_in) {
  constexpr int TM = BM / WM, TN = BN / WN;
  constexpr int BMB = TM / 16, BNB = TN / 16;
  static_assert(WM * WN == 4, "four waves");
  using Op = MfmaOp<T>;
  using V = typename Op::V;

  __shared__ int2 lst[16];
  // FP32 store staging: one 16 x TN slice per wave, so each store instruction
  // writes whole TN-wide row segments instead of 64-byte pieces.
  constexpr bool kStage = Op::kConsecutive && sizeof(O) == 4 && MODE != kModeFinalDeposit && TN >= 32;
  constexpr int SLD = TN + 4;
  __shared__ float stage[kStage ? 4 * 16 * SLD : 1];
  __shared__ int64_t rowoff[MODE == kModeFinalDeposit ? BM : 1];
  __shared__ int64_t coloff[MODE == kModeFinalDeposit ? BN : 1];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t blk = blk_in;
  const uint32_t tiles = (uint32_t)a.tilesM * (uint32_t)a.tilesN;
  const uint32_t batch = blk / tiles;
  const uint32_t t = blk - batch * tiles;
  const uint32_t tm = t / (uint32_t)a.tilesN, tn = t - tm * (uint32_t)a.tilesN;
  const int rX = (int)(batch >> (2 * a.nRY));
  const int rY = (int)(batch & ((1u << (2 * a.nRY)) - 1u));
  const int64_t M = int64_t(1) << a.logM, N = int64_t(1) << a.logN;
  const int64_t mw = (int64_t)tm * BM + (wave / WN) * TM;
  const int64_t nw = (int64_t)tn * BN + (wave % WN) * TN;
  const T *X = static_cast<const T *>(a.X);
  const T *Y = static_cast<const T *>(a.Y);
  const int l16 = lane & 15, lg = lane >> 4;

  if (MODE == kModeFinalDeposit) {
    for (int r = tid; r < BM; r += 256)
      rowoff[r] = (int64_t)tm * BM + r < M ? deposit((int64_t)tm * BM + r, a.posX, a.logM) : 0;
    for (int c = tid; c < BN; c += 256)
      coloff[c] = (int64_t)tn * BN + c < N ? deposit((int64_t)tn * BN + c, a.posY, a.logN) : 0;
  }
  // Operands are loaded for the full term list s = 0..4^|S|-1 at once (term
  // s = 4q + lane/16 in quad q), in parallel with the row-flag check; only if
  // some term turns out dead are they reloaded from the compacted live list.
  // Without row flags (flagX null) every term is kept: a term whose operand
  // slices are zero in this tile adds exact zeros, and at most 16 terms cost
  // nothing next to the output writes.
  const int nSv = 1 << (2 * a.nS);
  int2 rrq[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int sq = 4 * q + lg;
    rrq[q] = sq < nSv ? make_int2(row_of(a.mx, sq, rX), row_of(a.my, sq, rY)) : make_int2(-1, -1);
  }
  T ay[4][BNB], bxa[BMB][4];
  auto load_ops = [&]() {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const bool kok = rrq[q].x >= 0;
      const T *yr = Y + (int64_t)(kok ? rrq[q].y : 0) * N;
      const T *xr = X + (int64_t)(kok ? rrq[q].x : 0) * M;
#pragma unroll
      for (int j = 0; j < BNB; ++j) {
        const int64_t c = nw + j * 16 + l16;
        ay[q][j] = (kok && c < N) ? yr[c] : (T)0;
      }
#pragma unroll
      for (int i = 0; i < BMB; ++i) {
        const int64_t c = mw + i * 16 + l16;
        bxa[i][q] = (kok && c < M) ? xr[c] : (T)0;
      }
    }
  };
  load_ops();
  __shared__ int cnt_sh;
  if (!a.flagX) {
    if (tid == 0) cnt_sh = nSv;
  } else if (wave == 0) {
    int live = 0, rx = 0, ry = 0;
    if (lane < nSv) {
      rx = row_of(a.mx, lane, rX);
      ry = row_of(a.my, lane, rY);
      live = row_live(a.flagX, a.nchX, rx) & row_live(a.flagY, a.nchY, ry);
    }
    const unsigned long long bal = __ballot(live);
    const int pre = __popcll(bal & ((1ull << lane) - 1ull));
    const int cnt = __popcll(bal);
    if (live) lst[pre] = make_int2(rx, ry);
    if (lane >= cnt && lane < 16) lst[lane] = make_int2(-1, -1);
    if (lane == 0) cnt_sh = cnt;
  }
  __syncthreads();
  if (cnt_sh != nSv) {       // early termination: drop the dead terms
#pragma unroll
    for (int q = 0; q < 4; ++q) rrq[q] = lst[4 * q + lg];
    load_ops();
  }

  double msum = 0.0;
  const O scale = (O)a.scale;
  // cross-entropy form: the targets of the whole wave tile before its first
  // store, in the layout of the staged row stores (else of the lanes' own runs)
  constexpr bool kPre = XE && MODE == kModeFinalBlocked && Op::kConsecutive;
  constexpr int kLPR = TN >= 32 ? TN / 4 : 1, kRPI = 64 / kLPR, kTQ = kStage ? 16 / kRPI : BNB;
  const bool pre = kPre && mw + TM <= M && nw + TN <= N;
  f32x4 tv[kPre ? BMB * kTQ : 1];
  if constexpr (kPre) {
    if (pre)
#pragma unroll
      for (int i = 0; i < BMB; ++i)
#pragma unroll
        for (int q = 0; q < kTQ; ++q)
          tv[i * kTQ + q] = kStage ? xent_t4(a, (mw + i * 16 + q * kRPI + lane / kLPR) * N + nw + (lane % kLPR) * 4)
                                   : xent_t4(a, (mw + i * 16 + l16) * N + nw + q * 16 + 4 * lg);
  }
#pragma unroll
  for (int i = 0; i < BMB; ++i) {
    const T *bx = bxa[i];
    V acc[BNB];
#pragma unroll
    for (int j = 0; j < BNB; ++j) acc[j] = V{0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int j = 0; j < BNB; ++j)
        acc[j] = Op::kConsecutive ? Op::run(ay[q][j], bx[q], acc[j]) : Op::run(bx[q], ay[q][j], acc[j]);
    if (kStage && mw + i * 16 + 16 <= M && nw + TN <= N) {
      float *st = stage + wave * 16 * SLD;
      const float sc = MODE == kModeIntermediate ? 1.0f : (float)a.scale;
#pragma unroll
      for (int j = 0; j < BNB; ++j)
        *reinterpret_cast<float4 *>(st + l16 * SLD + j * 16 + 4 * lg) =
            make_float4((float)acc[j][0] * sc, (float)acc[j][1] * sc, (float)acc[j][2] * sc, (float)acc[j][3] * sc);
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
      constexpr int LPR = TN / 4, RPI = 64 / LPR;
      const int64_t mrow = mw + i * 16;
      O *Zb = MODE == kModeIntermediate ? static_cast<O *>(a.Z) + (int64_t)batch * M * N : static_cast<O *>(a.Z);
#pragma unroll
      for (int rr = 0; rr < 16; rr += RPI) {
        const int row = rr + lane / LPR, col = (lane % LPR) * 4;
        const float4 v = *reinterpret_cast<const float4 *>(st + row * SLD + col);
        if constexpr (XE) {
          const float w[4] = {v.x, v.y, v.z, v.w};
          double c[4];
          xent4_at<float>(a, (mrow + row) * N + nw + col, w, pre, tv[kPre ? i * kTQ + rr / RPI : 0], c, XE == 2);
          msum += (c[0] + c[1]) + (c[2] + c[3]);
        } else {
          *reinterpret_cast<float4 *>(Zb + (mrow + row) * N + nw + col) = v;
          if (MODE != kModeIntermediate) msum += ((double)v.x + (double)v.y) + ((double)v.z + (double)v.w);
        }
      }
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
      continue;
    }
#pragma unroll
    for (int j = 0; j < BNB; ++j) {
      const int64_t nb = nw + j * 16;
      if (Op::kConsecutive) {
        const int64_t m = mw + i * 16 + l16;
        const int64_t n = nb + 4 * lg;
        if (m >= M || n >= N) continue;
        if (MODE == kModeIntermediate) {
          T *Z = static_cast<T *>(a.Z) + (int64_t)batch * M * N + m * N + n;
          T w[4] = {acc[j][0], acc[j][1], acc[j][2], acc[j][3]};
          if (n + 3 < N) store4<T>(Z, w);
          else
            for (int r = 0; r < 4; ++r)
              if (n + r < N) Z[r] = w[r];
        } else {
          O v[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) v[r] = (O)acc[j][r] * scale;
          if constexpr (XE) {
            if (MODE == kModeFinalBlocked && n + 3 < N) {
              double c[4];
              xent4_at<O>(a, m * N + n, v, pre, tv[kPre && !kStage ? i * BNB + j : 0], c, XE == 2);
              for (int r = 0; r < 4; ++r) msum += c[r];
            } else {
              for (int r = 0; r < 4; ++r)
                if (n + r < N)
                  msum += xent_put1<O>(a, MODE == kModeFinalBlocked ? m * N + n + r
                                                                   : rowoff[m - (int64_t)tm * BM] +
                                                                         coloff[n + r - (int64_t)tn * BN],
                                       v[r], XE == 2);
            }
          } else {
            if (MODE == kModeFinalBlocked) {
              O *Z = static_cast<O *>(a.Z) + m * N + n;
              if (n + 3 < N) store4<O>(Z, v);
              else
                for (int r = 0; r < 4; ++r)
                  if (n + r < N) Z[r] = v[r];
            } else {
              O *Z = static_cast<O *>(a.Z);
              const int64_t ro = rowoff[m - (int64_t)tm * BM];
              for (int r = 0; r < 4; ++r)
                if (n + r < N) Z[ro + coloff[n + r - (int64_t)tn * BN]] = v[r];
            }
            for (int r = 0; r < 4; ++r)
              if (n + r < N) msum += (double)v[r];
          }
        }
      } else {
        const int64_t n = nb + l16;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t m = mw + i * 16 + lg + 4 * r;
          if (m >= M || n >= N) continue;
          if (MODE == kModeIntermediate) {
            static_cast<T *>(a.Z)[(int64_t)batch * M * N + m * N + n] = acc[j][r];
          } else {
            const O v = (O)acc[j][r] * scale;
            const int64_t o = MODE == kModeFinalBlocked
                                  ? m * N + n
                                  : rowoff[m - (int64_t)tm * BM] + coloff[n - (int64_t)tn * BN];
            if constexpr (XE) {
              msum += xent_put1<O>(a, o, v, XE == 2);
            } else {
              static_cast<O *>(a.Z)[o] = v;
              msum += (double)v;
            }
          }
        }
      }
    }
  }
  if (MODE == kModeIntermediate) {
    if (a.flagZ && tm == 0 && tn == 0 && tid == 0) a.flagZ[batch] = cnt_sh > 0;
    return;
  }
  if (a.partials) {
    const double tot = wave_sum_f64(msum);
    if (lane == 0) a.partials[kPartialsPerTile * blk + wave] = tot;
  }
}


// Two-tile strips for the 64 x 256 FP32 tile with FP32 output and every term
// kept (no row flags): a block takes two vertically adjacent tiles, loads the Y operands
// once and issues the X loads of the second tile before the first tile's
// output stores, so that wait never covers stores.  Half as many blocks
// start together, which spreads the operand fetch at the start of the launch
// over the first tile's stores.  One partial mass per tile, as in the
// one-tile kernel.

template <typename O, int MODE, int XE = 0>
__device__ __forceinline__ void contract_small_strip(const ContractArgs &a, uint32_t strip) {
  static_assert(sizeof(O) == 4, "staged float4 stores: FP32 output only");
  constexpr int R = kStripRows, BM = 64, BN = 256, TN = 64, SLD = TN + 4;
  using Op = MfmaOp<float>;
  using V = typename Op::V;
  __shared__ float stage[4 * 16 * SLD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t tilesN = (uint32_t)a.tilesN, groups = (uint32_t)a.tilesM / R;
  const uint32_t per_batch = groups * tilesN;
  const uint32_t batch = strip / per_batch;
  const uint32_t rem = strip - batch * per_batch;
  const uint32_t g = rem / tilesN, tn = rem - g * tilesN;
  const int rX = (int)(batch >> (2 * a.nRY));
  const int rY = (int)(batch & ((1u << (2 * a.nRY)) - 1u));
  const int64_t M = int64_t(1) << a.logM, N = int64_t(1) << a.logN;
  const int64_t nw = (int64_t)tn * BN + wave * TN;
  const float *X = static_cast<const float *>(a.X);
  const float *Y = static_cast<const float *>(a.Y);
  const int l16 = lane & 15, lg = lane >> 4;
  const int nSv = 1 << (2 * a.nS);
  int2 rrq[4];   // term 4q + lane/16 (rows -1: past the term count)
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int sq = 4 * q + lg;
    rrq[q] = sq < nSv ? make_int2(row_of(a.mx, sq, rX), row_of(a.my, sq, rY)) : make_int2(-1, -1);
  }
  float ay[4][4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const bool kok = rrq[q].x >= 0;
    const float *yr = Y + (int64_t)(kok ? rrq[q].y : 0) * N;
#pragma unroll
    for (int j = 0; j < 4; ++j) ay[q][j] = kok ? yr[nw + j * 16 + l16] : 0.f;
  }
  float bx[R][4][4];
  auto load_x = [&](int r) {
    const int64_t mw = (int64_t)(g * R + r) * BM;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const bool kok = rrq[q].x >= 0;
      const float *xr = X + (int64_t)(kok ? rrq[q].x : 0) * M;
#pragma unroll
      for (int i = 0; i < 4; ++i) bx[r][i][q] = kok ? xr[mw + i * 16 + l16] : 0.f;
    }
  };
  load_x(0);
  float *st = stage + wave * 16 * SLD;
  const float sc = MODE == kModeIntermediate ? 1.0f : (float)a.scale;
  O *Zb = MODE == kModeIntermediate ? static_cast<O *>(a.Z) + (int64_t)batch * M * N : static_cast<O *>(a.Z);
  // cross-entropy form: the targets of a whole tile, loaded before its first
  // store (strips cover whole tiles)
  f32x4 tv[XE ? 16 : 1];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const uint32_t tm = g * R + r;
    const int64_t mw = (int64_t)tm * BM;
    if constexpr (XE)
#pragma unroll
      for (int q = 0; q < 16; ++q)
        tv[q] = xent_t4(a, (mw + (q >> 2) * 16 + (q & 3) * 4 + lane / 16) * N + nw + (lane % 16) * 4);
    if (r + 1 < R) load_x(r + 1);
    double msum = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      V acc[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[j] = V{0, 0, 0, 0};
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] = Op::run(ay[q][j], bx[r][i][q], acc[j]);
      // stage the 16 x 64 slice, then write whole 256-byte row segments
#pragma unroll
      for (int j = 0; j < 4; ++j)
        *reinterpret_cast<float4 *>(st + l16 * SLD + j * 16 + 4 * lg) =
            make_float4(acc[j][0] * sc, acc[j][1] * sc, acc[j][2] * sc, acc[j][3] * sc);
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
#pragma unroll
      for (int rr = 0; rr < 16; rr += 4) {
        const int row = rr + lane / 16, col = (lane % 16) * 4;
        const float4 v = *reinterpret_cast<const float4 *>(st + row * SLD + col);
        if constexpr (XE) {
          const float w[4] = {v.x, v.y, v.z, v.w};
          double c[4];
          xent_emit4(a, (mw + i * 16 + row) * N + nw + col, w, tv[XE ? 4 * i + rr / 4 : 0], c, XE == 2);
          msum += (c[0] + c[1]) + (c[2] + c[3]);
        } else {
          *reinterpret_cast<float4 *>(Zb + (mw + i * 16 + row) * N + nw + col) = v;
          if (MODE != kModeIntermediate) msum += ((double)v.x + (double)v.y) + ((double)v.z + (double)v.w);
        }
      }
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    }
    if (MODE == kModeIntermediate) {
      if (a.flagZ && tm == 0 && tn == 0 && tid == 0) a.flagZ[batch] = nSv > 0;
    } else if (a.partials) {
      const double tot = wave_sum_f64(msum);
      const int64_t tile = (int64_t)batch * a.tilesM * a.tilesN + (int64_t)tm * tilesN + tn;
      if (lane == 0) a.partials[kPartialsPerTile * tile + wave] = tot;
    }
  }
}

template <int MODE, int XE>
__global__ __launch_bounds__(256) void k_contract_strip_queue(const ContractArgs *descs, const int64_t *prefix,
                                                              int ndesc, unsigned long long *queue, int64_t total) {
  __shared__ int64_t item;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) item = (int64_t)atomicAdd(queue, 1ull);
    __syncthreads();
    const int64_t it = item;
    if (it >= total) return;
    const int d = find_desc(prefix, ndesc, it);
    contract_small_strip<float, MODE, XE>(descs[d], (uint32_t)(it - prefix[d]));
  }
}

template <typename O, int MODE>
__global__ __launch_bounds__(256) void k_contract_strip(const ContractArgs a) {
  if (gated_off(a.gate, a.gate_val)) return;
  const int64_t ns = a.nblocks / kStripRows;
  const uint32_t s = a.xcd_remap ? (uint32_t)xcd_remap(blockIdx.x, ns) : blockIdx.x;
  contract_small_strip<O, MODE>(a, s);
}

// ---- launch wrappers: one step per launch, or a work queue over many steps
template <typename T, typename O, int BM, int BN, int WM, int WN, int MODE, bool SMALL>
__global__ __launch_bounds__(256) void k_contract(const ContractArgs a) {
  if (gated_off(a.gate, a.gate_val)) return;
  const uint32_t blk = a.xcd_remap ? (uint32_t)xcd_remap(blockIdx.x, a.nblocks) : blockIdx.x;
  if (SMALL) contract_small_tile<T, O, BM, BN, WM, WN, MODE>(a, blk);
  else contract_tile<T, O, BM, BN, WM, WN, MODE>(a, blk);
}


// Persistent blocks take (step, tile) items from an atomic queue until it
// runs dry; steps are laid out most expensive first, so large instances start
// early and small ones fill the tail.  Every block leaves once the counter
// passes `total`.
template <typename T, typename O, int BM, int BN, int WM, int WN, int MODE, bool SMALL, int XE>
__global__ __launch_bounds__(256) void k_contract_queue(const ContractArgs *descs, const int64_t *prefix,
                                                        int ndesc, unsigned long long *queue, int64_t total) {
  __shared__ int64_t item;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) item = (int64_t)atomicAdd(queue, 1ull);
    __syncthreads();
    const int64_t it = item;
    if (it >= total) return;
    const int d = find_desc(prefix, ndesc, it);
    if (SMALL) {
      // kSmallTilesPerItem consecutive tiles of one step per item
      const ContractArgs &a = descs[d];
      const int64_t t0 = (it - prefix[d]) * kSmallTilesPerItem;
      for (int j = 0; j < kSmallTilesPerItem && t0 + j < a.nblocks; ++j) {
        if (j) __syncthreads();
        contract_small_tile<T, O, BM, BN, WM, WN, MODE, XE>(a, (uint32_t)(t0 + j));
      }
    } else {
      contract_tile<T, O, BM, BN, WM, WN, MODE, XE>(descs[d], (uint32_t)(it - prefix[d]));
    }
  }
}

// ---------------------------------------------------------------------------
// Row flags of the entry tensors: one block per (row, chunk of kFlagChunk
// columns) writes whether that chunk has a non-zero element.  The first block
// of a tensor that carries a unit operand (single-subcircuit plans) also
// writes that operand's value 1 and its flag.
__device__ __forceinline__ void flags_chunk(const FlagDesc &d, int64_t rc, bool is_double) {
  const int64_t nch = flag_chunks(d.cols);
  const int64_t r = rc / nch, ch = rc - r * nch;
  const int64_t c0 = ch * kFlagChunk;
  const int64_t c1 = d.cols < c0 + kFlagChunk ? d.cols : c0 + kFlagChunk;
  int any = 0;
  if (is_double) {
    const double *p = static_cast<const double *>(d.ptr) + r * d.cols;
    if (d.cols % 2 == 0) {
      const double2 *q = reinterpret_cast<const double2 *>(p);
#pragma unroll 4
      for (int64_t c = c0 / 2 + threadIdx.x; c < c1 / 2; c += blockDim.x) {
        const double2 v = q[c];
        any |= (v.x != 0.0) | (v.y != 0.0);
      }
    } else {
      for (int64_t c = c0 + threadIdx.x; c < c1; c += blockDim.x) any |= (p[c] != 0.0);
    }
  } else {
    const float *p = static_cast<const float *>(d.ptr) + r * d.cols;
    if (d.cols % 4 == 0) {
      const float4 *q = reinterpret_cast<const float4 *>(p);
#pragma unroll 2
      for (int64_t c = c0 / 4 + threadIdx.x; c < c1 / 4; c += blockDim.x) {
        const float4 v = q[c];
        any |= (v.x != 0.0f) | (v.y != 0.0f) | (v.z != 0.0f) | (v.w != 0.0f);
      }
    } else {
      for (int64_t c = c0 + threadIdx.x; c < c1; c += blockDim.x) any |= (p[c] != 0.0f);
    }
  }
  any = __syncthreads_or(any);
  if (threadIdx.x == 0) {
    d.flags[rc] = any ? 1 : 0;
    if (rc == 0 && d.unit) {
      if (is_double) *static_cast<double *>(d.unit) = 1.0;
      else *static_cast<float *>(d.unit) = 1.0f;
      *d.unit_flag = 1;
    }
  }
}

__global__ __launch_bounds__(256) void k_row_flags(const FlagArgs a) {
  if (gated_off(a.gate, a.gate_val)) return;
  const int64_t bid = blockIdx.x;
  int i = 0;
  while (i + 1 < a.n && bid >= a.d[i + 1].block_start) ++i;
  flags_chunk(a.d[i], bid - a.d[i].block_start, a.is_double != 0);
}

__global__ __launch_bounds__(256) void k_row_flags_table(const FlagDesc *descs, int32_t n, int32_t is_double,
                                                         unsigned long long *counters, int32_t n_counters) {
  const int64_t bid = blockIdx.x;
  if (bid == 0 && (int)threadIdx.x < n_counters) counters[threadIdx.x] = 0ull;
  if (n == 0) return;   // a batch without row flags: the counters only
  // the table is only read during the launch: scalar loads (see find_desc)
  using cd = const __attribute__((address_space(4))) FlagDesc *;
  const cd tab = (cd)(const __attribute__((address_space(1))) FlagDesc *)descs;
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tab[mid].block_start <= bid) lo = mid;
    else hi = mid - 1;
  }
  flags_chunk(descs[lo], bid - tab[lo].block_start, is_double != 0);
}

// One block per instance: its FP64 mass from the per-tile partials, in order.
__global__ __launch_bounds__(256) void k_mass_table(const MassDesc *descs) {
  const MassDesc &d = descs[blockIdx.x];
  __shared__ double tsum[256];
  double v = 0.0;
  for (int64_t i = threadIdx.x; i < d.count; i += blockDim.x) v += d.partials[i];
  tsum[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) tsum[threadIdx.x] += tsum[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) d.mass[0] = tsum[0];
}

template <typename S, typename D>
__global__ __launch_bounds__(256) void k_convert(const S *src, D *dst, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (D)src[i];
}

// Lane-layout probe: D = A * B for one 16x16x4 block with A[i][k] = i + 16 k,
// B[k][j] = 1 + k + 4 j (exact in FP32), stored as D[i][j] by the accumulator
// layouts the contraction kernels rely on (MfmaOp above); and one 16x16x32
// bfloat16 block with A[i][k] = (i + 3k) % 7 - 3, B[k][j] = (2k + j) % 5 - 2,
// where lane l supplies A[l % 16][8 (l / 16) + e] and B[8 (l / 16) + e][l % 16]
// (the operand layout of the wide kernel's BF16X6 form).
__global__ void k_selftest_mfma(float *outf, double *outd, float *outb) {
  typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
  const int lane = threadIdx.x;
  const int i = lane & 15, k = lane >> 4, j = lane & 15;
  f32x4 cf = {0, 0, 0, 0};
  cf = __builtin_amdgcn_mfma_f32_16x16x4f32((float)(i + 16 * k), (float)(1 + k + 4 * j), cf, 0, 0, 0);
  f64x4 cd = {0, 0, 0, 0};
  cd = __builtin_amdgcn_mfma_f64_16x16x4f64((double)(i + 16 * k), (double)(1 + k + 4 * j), cd, 0, 0, 0);
  bf16x8 ab, bb;
  for (int e = 0; e < 8; ++e) {
    const int kk = 8 * (lane >> 4) + e;
    ab[e] = (__bf16)(float)((i + 3 * kk) % 7 - 3);
    bb[e] = (__bf16)(float)((2 * kk + j) % 5 - 2);
  }
  f32x4 cb = {0, 0, 0, 0};
  cb = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ab, bb, cb, 0, 0, 0);
  for (int r = 0; r < 4; ++r) {
    const int col = lane & 15;
    outf[(4 * (lane >> 4) + r) * 16 + col] = cf[r];
    outd[((lane >> 4) + 4 * r) * 16 + col] = cd[r];
    outb[(4 * (lane >> 4) + r) * 16 + col] = cb[r];
  }
}

// ---------------------------------------------------------------------------
TileShape tile_shape(int cfg) {
  switch (cfg) {
    case kTileL: return {64, 256};
    case kTileM: return {32, 128};
    case kTileS: return {16, 64};
    case kTileW: return {128, 128};
    default: return {256, 16};
  }
}

bool tile_ok(Acc acc, int cfg) {
  if (cfg < 0 || cfg >= kTileCount) return false;
  if (is_split(acc)) return cfg == kTileW;
  if (acc == Acc::F64) return cfg != kTileW;
  return true;
}

int choose_tile(Acc acc, int nS, int logM, int logN, bool wide_ok, int64_t nbatch) {
  const int64_t M = int64_t(1) << logM, N = int64_t(1) << logN;
  if (is_split(acc)) return kTileW;
  // long term sums over large tiles are compute-bound: LDS-staged operands, on
  // steps with at least 256 tiles of 128 x 128 (fewer leave most of the chip
  // idle on the persistent kernel: the 64 x 256 register kernel then wins, e.g.
  // 2^20 dynamic-definition bins, measured 25% faster per query)
  if (acc == Acc::F32 && wide_ok && nS >= 3 && M >= 128 && N >= 128 && M * N * nbatch >= (int64_t(1) << 22))
    return kTileW;
  if (M >= 64 && N >= 256) return kTileL;
  if (N < 64 && M >= 256) return kTileT;
  if (M >= 32 && N >= 128) return kTileM;
  return kTileS;
}

template <typename T, typename O, int MODE, bool SMALL>
static Status launch_contract_ms(int cfg, const ContractArgs &a, hipStream_t s) {
  const dim3 grid((unsigned)a.nblocks), block(256);
  if constexpr (SMALL && std::is_same<T, float>::value && std::is_same<O, float>::value &&
                MODE != kModeFinalDeposit) {
    // every term kept and whole tiles in pairs of rows: two-tile strips
    if (cfg == kTileL && !a.flagX && a.logN >= 8 && a.logM >= 7)
      return launch("contract_small_strip_64x256", k_contract_strip<O, MODE>,
                    dim3((unsigned)(a.nblocks / kStripRows)), block, 0, s, a);
  }
  switch (cfg) {
    case kTileL: return launch(SMALL ? "contract_small_64x256" : "contract_64x256", k_contract<T, O, 64, 256, 1, 4, MODE, SMALL>, grid, block, 0, s, a);
    case kTileM: return launch(SMALL ? "contract_small_32x128" : "contract_32x128", k_contract<T, O, 32, 128, 1, 4, MODE, SMALL>, grid, block, 0, s, a);
    case kTileS: return launch(SMALL ? "contract_small_16x64" : "contract_16x64", k_contract<T, O, 16, 64, 1, 4, MODE, SMALL>, grid, block, 0, s, a);
    default: return launch(SMALL ? "contract_small_256x16" : "contract_256x16", k_contract<T, O, 256, 16, 4, 1, MODE, SMALL>, grid, block, 0, s, a);
  }
}

template <typename T, typename O, int MODE>
static Status launch_contract_m(int cfg, const ContractArgs &a, hipStream_t s) {
  if (a.nS <= 2) return launch_contract_ms<T, O, MODE, true>(cfg, a, s);
  return launch_contract_ms<T, O, MODE, false>(cfg, a, s);
}

template <typename T, int MODE, bool SMALL, int XE>
static Status launch_queue_x(int cfg, const QueueLaunch &q, hipStream_t s) {
  const dim3 grid(q.grid), block(256);
  const char *nm = XE == 2 ? (SMALL ? "contract_small_queue_xent_loss" : "contract_queue_xent_loss")
                   : XE ? (SMALL ? "contract_small_queue_xent" : "contract_queue_xent")
                        : (SMALL ? "contract_small_queue" : "contract_queue");
  switch (cfg) {
    case kTileL: return launch(nm, k_contract_queue<T, T, 64, 256, 1, 4, MODE, SMALL, XE>, grid, block, 0, s, q.descs, q.prefix, q.ndesc, q.queue, q.total);
    case kTileM: return launch(nm, k_contract_queue<T, T, 32, 128, 1, 4, MODE, SMALL, XE>, grid, block, 0, s, q.descs, q.prefix, q.ndesc, q.queue, q.total);
    default: return launch(nm, k_contract_queue<T, T, 16, 64, 1, 4, MODE, SMALL, XE>, grid, block, 0, s, q.descs, q.prefix, q.ndesc, q.queue, q.total);
  }
}

template <typename T, int MODE, bool SMALL>
static Status launch_queue_t(int cfg, const QueueLaunch &q, hipStream_t s) {
  if constexpr (MODE != kModeIntermediate) {
    if (q.xent == 1) return launch_queue_x<T, MODE, SMALL, 1>(cfg, q, s);
    if (q.xent == 2) return launch_queue_x<T, MODE, SMALL, 2>(cfg, q, s);
  }
  return launch_queue_x<T, MODE, SMALL, 0>(cfg, q, s);
}

Status launch_contract_strip_queue(int mode, const QueueLaunch &q, hipStream_t s) {
  const dim3 grid(q.grid), block(256);
  if (mode == kModeIntermediate)
    return launch("contract_strip_queue", k_contract_strip_queue<kModeIntermediate, 0>, grid, block, 0, s,
                  q.descs, q.prefix, q.ndesc, q.queue, q.total);
  if (mode == kModeFinalBlocked && q.xent == 1)
    return launch("contract_strip_queue_xent", k_contract_strip_queue<kModeFinalBlocked, 1>, grid, block, 0, s,
                  q.descs, q.prefix, q.ndesc, q.queue, q.total);
  if (mode == kModeFinalBlocked && q.xent == 2)
    return launch("contract_strip_queue_xent_loss", k_contract_strip_queue<kModeFinalBlocked, 2>, grid, block, 0,
                  s, q.descs, q.prefix, q.ndesc, q.queue, q.total);
  if (mode == kModeFinalBlocked)
    return launch("contract_strip_queue", k_contract_strip_queue<kModeFinalBlocked, 0>, grid, block, 0, s,
                  q.descs, q.prefix, q.ndesc, q.queue, q.total);
  return Status::fail(CQC_ERR_UNSUPPORTED, "two-tile strips need blocked or intermediate output");
}

template <typename T, int MODE>
static Status launch_queue_m(int cfg, bool small, const QueueLaunch &q, hipStream_t s) {
  return small ? launch_queue_t<T, MODE, true>(cfg, q, s) : launch_queue_t<T, MODE, false>(cfg, q, s);
}

Status launch_contract_queue(Acc acc, int mode, int cfg, bool small, const QueueLaunch &q, hipStream_t s) {
  if (!tile_ok(acc, cfg)) return Status::fail(CQC_ERR_INVALID_ARG, "tile configuration not available for this arithmetic");
  if (cfg == kTileW) return launch_contract_wide_queue(split_parts(acc), mode, q, s);
  if (acc == Acc::F32) {
    if (mode == kModeIntermediate) return launch_queue_m<float, kModeIntermediate>(cfg, small, q, s);
    if (mode == kModeFinalBlocked) return launch_queue_m<float, kModeFinalBlocked>(cfg, small, q, s);
    return launch_queue_m<float, kModeFinalDeposit>(cfg, small, q, s);
  }
  if (mode == kModeIntermediate) return launch_queue_m<double, kModeIntermediate>(cfg, small, q, s);
  if (mode == kModeFinalBlocked) return launch_queue_m<double, kModeFinalBlocked>(cfg, small, q, s);
  return launch_queue_m<double, kModeFinalDeposit>(cfg, small, q, s);
}

template <typename T, typename O>
static Status launch_contract_t(int cfg, const ContractArgs &a, hipStream_t s) {
  if (a.mode == kModeFinalBlocked) return launch_contract_m<T, O, kModeFinalBlocked>(cfg, a, s);
  if (a.mode == kModeFinalDeposit) return launch_contract_m<T, O, kModeFinalDeposit>(cfg, a, s);
  return launch_contract_m<T, T, kModeIntermediate>(cfg, a, s);
}

Status launch_contract(Acc acc, bool out_double, int cfg, const ContractArgs &a, hipStream_t s) {
  if (!tile_ok(acc, cfg)) return Status::fail(CQC_ERR_INVALID_ARG, "tile configuration not available for this arithmetic");
  if (cfg == kTileW) return launch_contract_wide(split_parts(acc), out_double, a, s);
  if (acc == Acc::F32)
    return out_double ? launch_contract_t<float, double>(cfg, a, s)
                      : launch_contract_t<float, float>(cfg, a, s);
  return out_double ? launch_contract_t<double, double>(cfg, a, s)
                    : launch_contract_t<double, float>(cfg, a, s);
}

Status launch_mass_final(const double *partials, int64_t count, double *mass, hipStream_t s,
                         const int32_t *gate, int32_t gate_val) {
  return launch("mass_final", k_mass_final, dim3(1), dim3(1024), 0, s, partials, count, mass, gate, gate_val);
}

Status launch_row_flags_table(const FlagDesc *descs, int32_t n, int64_t total_blocks, bool is_double,
                              unsigned long long *counters, int32_t n_counters, hipStream_t s) {
  // at least one block: the pass also zeroes the queue counters
  return launch("row_flags_table", k_row_flags_table, dim3((unsigned)std::max<int64_t>(1, total_blocks)), dim3(256),
                0, s, descs, n,
                (int32_t)is_double, counters, n_counters);
}

Status launch_mass_table(const MassDesc *descs, int32_t n, hipStream_t s) {
  return launch("mass_table", k_mass_table, dim3((unsigned)n), dim3(256), 0, s, descs);
}

Status launch_row_flags(const FlagArgs &a, int64_t total_blocks, hipStream_t s) {
  return launch("row_flags", k_row_flags, dim3((unsigned)total_blocks), dim3(256), 0, s, a);
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
  float *ob = reinterpret_cast<float *>(od + 256);
  return launch("selftest_mfma", k_selftest_mfma, dim3(1), dim3(64), 0, s, of, od, ob);
}

}  // namespace cqc
