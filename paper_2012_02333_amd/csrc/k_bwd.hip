// Adjoint kernels of one contraction step
//     Z[(rX,rY)][m][n] = sum_s X[rowX(s,rX)][m] * Y[rowY(s,rY)][n]
// given dZ = dL/dZ (row-major per batch):
//     dX[rowX(s,rX)][m] = sum_{rY} sum_n dZ[(rX,rY)][m][n] * Y[rowY(s,rY)][n]    (k_bwd_x)
//     dY[rowY(s,rY)][n] = sum_{rX} sum_m X[rowX(s,rX)][m] * dZ[(rX,rY)][m][n]    (k_bwd_y)
// Both are GEMMs with a long inner dimension (output columns of the other
// operand, and its rest labels), run split-K: every block owns one chunk of
// the inner dimension and writes its partial sums; k_bwd_reduce then adds the
// partials in chunk order (fixed, so results are bitwise reproducible) and
// applies the scale.  Matrix-core row i <-> label s, column j <-> the output
// column, k <-> the inner index; each lane takes 4 consecutive inner indices
// with one 16-byte load and feeds them to 4 MFMAs (inner index 4*(lane/16)+t
// in MFMA t, the same for both operands).  FP32 tiles of 64 labels run their
// products split into bfloat16 parts on the BF16 matrix cores (six products,
// FP32 accumulation, FP32-level accuracy); see bwd_block_staged.
#include <algorithm>

#include "bwd.hpp"
#include "kdev.hpp"

namespace cqc {


template <typename T> struct BOp;
template <> struct BOp<float> {
  using V = f32x4;
  static constexpr bool kConsecutive = true;  // register r <-> row 4*(l/16)+r
  static __device__ __forceinline__ V run(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct BOp<double> {
  using V = f64x4;
  static constexpr bool kConsecutive = false;  // register r <-> row (l/16)+4r
  static __device__ __forceinline__ V run(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

template <typename T>
__device__ __forceinline__ void load4m(const T *p, int64_t c, int64_t lim, T *v) {
  // v[t] = p[c + t] for c + t < lim, else 0 (c is a multiple of 4)
  if (c + 3 < lim) {
    if (sizeof(T) == 4) {
      const float4 q = *reinterpret_cast<const float4 *>(p + c);
      v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    } else {
      const double2 a = *reinterpret_cast<const double2 *>(p + c);
      const double2 b = *reinterpret_cast<const double2 *>(p + c + 2);
      v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
    }
  } else {
#pragma unroll
    for (int t = 0; t < 4; ++t) v[t] = c + t < lim ? p[c + t] : (T)0;
  }
}

// Operand prefetch (two register sets) where the registers allow it: FP32
// with up to 4 label blocks; occupancy targets of four waves per SIMD for the
// one-label-block form, two for the others (no constraint without prefetch).
template <typename T, int SB> struct BwdCfg {
  static constexpr bool kPF = sizeof(T) == 4 && SB <= 4;
  static constexpr int kWaves = sizeof(T) == 4 && SB == 16 ? 2 : (!kPF ? 1 : (SB == 1 ? 4 : 2));
};

// grid: x = (((p * RXn + rX) * sSuper + ss) * mTiles + mt), p = (rY, k-chunk)
template <typename T, int SB, int MB>
__device__ __forceinline__ void bwd_x_block(const BwdArgs &a, int64_t blk) {
  constexpr bool PF = BwdCfg<T, SB>::kPF;
  using Op = BOp<T>;
  using V = typename Op::V;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, lg = lane >> 4;
  const int64_t M = int64_t(1) << a.logM, N = int64_t(1) << a.logN;
  const int RYn = 1 << (2 * a.nRY), RXn = 1 << (2 * a.nRX), SN = 1 << (2 * a.nS);
  const int sSuper = (SN + 16 * SB - 1) / (16 * SB);
  const int64_t mTiles = (M + 64 * MB - 1) / (64 * MB);
  int64_t b = blk;
  const int64_t mt = b % mTiles; b /= mTiles;
  const int ss = (int)(b % sSuper); b /= sSuper;
  const int rX = (int)(b % RXn); b /= RXn;
  const int64_t p = b;                       // partial index = rY * kChunks + kc
  const int rY = (int)(p / a.kChunks), kc = (int)(p % a.kChunks);
  const int64_t k0 = (int64_t)kc * a.kChunk;
  const int64_t k1 = N < k0 + a.kChunk ? N : k0 + a.kChunk;
  const int64_t mw = mt * 64 * MB + wave * 16 * MB;
  const T *X = static_cast<const T *>(a.X);  (void)X;
  const T *Y = static_cast<const T *>(a.Y);
  const T *dZ = static_cast<const T *>(a.dZ) + ((int64_t)rX * RYn + rY) * M * N;
  int yrow[SB];
  bool sok[SB];
#pragma unroll
  for (int sb = 0; sb < SB; ++sb) {
    const int s = (ss * SB + sb) * 16 + l16;
    sok[sb] = s < SN;
    yrow[sb] = sok[sb] ? row_of(a.my, s, rY) : 0;
  }
  V acc[SB][MB];
#pragma unroll
  for (int i = 0; i < SB; ++i)
#pragma unroll
    for (int j = 0; j < MB; ++j) acc[i][j] = V{0, 0, 0, 0};
  // operands of the next 16 inner indices are loaded while the current ones
  // are on the matrix cores (two register sets, alternating)
  T av[PF ? 2 : 1][SB][4], bv[PF ? 2 : 1][MB][4];
  auto load = [&](int buf, int64_t n0) {
    const int64_t c = n0 + 4 * lg;
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) {
      if (sok[sb]) load4m<T>(Y + (int64_t)yrow[sb] * N, c, k1, av[buf][sb]);
      else
        for (int t = 0; t < 4; ++t) av[buf][sb][t] = 0;
    }
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      const int64_t m = mw + mb * 16 + l16;
      if (m < M) load4m<T>(dZ + m * N, c, k1, bv[buf][mb]);
      else
        for (int t = 0; t < 4; ++t) bv[buf][mb][t] = 0;
    }
  };
  auto mfma = [&](int buf) {
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int sb = 0; sb < SB; ++sb)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) acc[sb][mb] = Op::run(av[buf][sb][t], bv[buf][mb][t], acc[sb][mb]);
  };
  if constexpr (PF) {
    if (k0 < k1) load(0, k0);
    for (int64_t n0 = k0; n0 < k1; n0 += 32) {
      const bool two = n0 + 16 < k1;
      if (two) load(PF ? 1 : 0, n0 + 16);
      mfma(0);
      if (n0 + 32 < k1) load(0, n0 + 32);
      if (two) mfma(PF ? 1 : 0);
    }
  } else {
    for (int64_t n0 = k0; n0 < k1; n0 += 16) {
      load(0, n0);
      mfma(0);
    }
  }
  T *part = static_cast<T *>(a.part) + p * a.rowsX * M;
#pragma unroll
  for (int sb = 0; sb < SB; ++sb)
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      const int64_t m = mw + mb * 16 + l16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int s = (ss * SB + sb) * 16 + (Op::kConsecutive ? 4 * lg + r : lg + 4 * r);
        if (s < SN && m < M) part[(int64_t)row_of(a.mx, s, rX) * M + m] = acc[sb][mb][r];
      }
    }
}

// grid: x = (((p * RYn + rY) * sSuper + ss) * nTiles + nt), p = (rX, k-chunk over m)
template <typename T, int SB, int NB>
__device__ __forceinline__ void bwd_y_block(const BwdArgs &a, int64_t blk) {
  constexpr bool PF = BwdCfg<T, SB>::kPF;
  using Op = BOp<T>;
  using V = typename Op::V;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, lg = lane >> 4;
  const int64_t M = int64_t(1) << a.logM, N = int64_t(1) << a.logN;
  const int RYn = 1 << (2 * a.nRY), SN = 1 << (2 * a.nS);
  const int sSuper = (SN + 16 * SB - 1) / (16 * SB);
  const int64_t nTiles = (N + 64 * NB - 1) / (64 * NB);
  int64_t b = blk;
  const int64_t nt = b % nTiles; b /= nTiles;
  const int ss = (int)(b % sSuper); b /= sSuper;
  const int rY = (int)(b % RYn); b /= RYn;
  const int64_t p = b;                       // partial index = rX * kChunks + kc
  const int rX = (int)(p / a.kChunks), kc = (int)(p % a.kChunks);
  const int64_t k0 = (int64_t)kc * a.kChunk;
  const int64_t k1 = M < k0 + a.kChunk ? M : k0 + a.kChunk;
  const int64_t nw = nt * 64 * NB + wave * 16 * NB;
  const T *X = static_cast<const T *>(a.X);
  const T *dZ = static_cast<const T *>(a.dZ) + ((int64_t)rX * RYn + rY) * M * N;
  int xrow[SB];
  bool sok[SB];
#pragma unroll
  for (int sb = 0; sb < SB; ++sb) {
    const int s = (ss * SB + sb) * 16 + l16;
    sok[sb] = s < SN;
    xrow[sb] = sok[sb] ? row_of(a.mx, s, rX) : 0;
  }
  V acc[SB][NB];
#pragma unroll
  for (int i = 0; i < SB; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = V{0, 0, 0, 0};
  T av[PF ? 2 : 1][SB][4], bv[PF ? 2 : 1][NB][4];
  auto load = [&](int buf, int64_t m0) {
    const int64_t c = m0 + 4 * lg;
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) {
      if (sok[sb]) load4m<T>(X + (int64_t)xrow[sb] * M, c, k1, av[buf][sb]);
      else
        for (int t = 0; t < 4; ++t) av[buf][sb][t] = 0;
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int64_t n = nw + nb * 16 + l16;
#pragma unroll
      for (int t = 0; t < 4; ++t) bv[buf][nb][t] = (n < N && c + t < k1) ? dZ[(c + t) * N + n] : (T)0;
    }
  };
  auto mfma = [&](int buf) {
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int sb = 0; sb < SB; ++sb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[sb][nb] = Op::run(av[buf][sb][t], bv[buf][nb][t], acc[sb][nb]);
  };
  if constexpr (PF) {
    if (k0 < k1) load(0, k0);
    for (int64_t m0 = k0; m0 < k1; m0 += 32) {
      const bool two = m0 + 16 < k1;
      if (two) load(PF ? 1 : 0, m0 + 16);
      mfma(0);
      if (m0 + 32 < k1) load(0, m0 + 32);
      if (two) mfma(PF ? 1 : 0);
    }
  } else {
    for (int64_t m0 = k0; m0 < k1; m0 += 16) {
      load(0, m0);
      mfma(0);
    }
  }
  T *part = static_cast<T *>(a.part) + p * a.rowsY * N;
#pragma unroll
  for (int sb = 0; sb < SB; ++sb)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int64_t n = nw + nb * 16 + l16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int s = (ss * SB + sb) * 16 + (Op::kConsecutive ? 4 * lg + r : lg + 4 * r);
        if (s < SN && n < N) part[(int64_t)row_of(a.my, s, rY) * N + n] = acc[sb][nb][r];
      }
    }
}

// 16 SB label rows x 64 OB outputs per block (four waves of 16 OB: 64 x 256,
// 128 x 128 or 256 x 64), the label rows' 32-index slices staged in LDS once per block
// (double-buffered) instead of loaded by every wave; the dL/dZ operand per
// wave from global memory, one 16-index half ahead.  Y: the dY side (label rows of X over m, dZ columns);
// else the dX side (label rows of Y over n, dZ rows).
// FAST: inner extent at least 16, so every chunk is a multiple of 16 and a
// 16-index group never straddles its end; all loads are unconditional global
// loads from clamped addresses, and nothing consumes a loaded value before
// its use (a select right after a load would wait for it there).
constexpr int kStagedLd = 36;
// Split form of the 64- and 128-label FP32 tiles (FAST, SB = 4 or 8): the
// label slices are staged as three bfloat16 part planes [2][3][16 SB][kSplitLd]
// (pitch 48: the 16-byte operand reads of 16 rows x 2 lane groups fall on
// distinct 16-byte slots modulo 512 bytes).
constexpr int kSplitLd = 48;
template <int SB> struct StagedLds {
  static constexpr int kF32 = 2 * 16 * SB * kStagedLd;
  static constexpr int kSplit = SB == 4 || SB == 8 ? 2 * 3 * 16 * SB * kSplitLd / 2 : 0;
  static constexpr int kFloats = kF32 > kSplit ? kF32 : kSplit;
};
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
// a = h + m + l, each part the round-to-nearest bfloat16 of what is left (the
// remainders are exact in FP32, so the parts carry 24 significand bits)
__device__ __forceinline__ void split_bf16(float a, __bf16 &h, __bf16 &m, __bf16 &l) {
  h = (__bf16)a;
  const float r1 = a - (float)h;
  m = (__bf16)r1;
  l = (__bf16)(r1 - (float)m);
}
template <bool YS, bool FAST, int SB = 4, int OB = 4>
__device__ __forceinline__ void bwd_block_staged(const BwdArgs &a, int64_t blk, float (*ls)[16 * SB][kStagedLd]) {
  // Pitch 36 floats.  The 16-byte fragment reads conflict on LDS banks at this
  // pitch (a 40-float pitch removes that, measured) - but the kernel measured
  // 8% slower with the conflict-free pitch, so the conflicts are not what
  // bounds it
  constexpr int KS = 32;
  static_assert(kStagedLd == KS + 4, "staging pitch");
  constexpr int RPT = SB / 4;   // label rows staged per thread
  // Split form: every label and dL/dZ value a = a0 + a1 + a2 in bfloat16
  // parts, and the six products a_i b_j with i + j <= 2 accumulated in FP32 on
  // v_mfma_f32_16x16x32_bf16, smallest first (the dropped products and the
  // split's remainder are below 2^-24 of |a b|: FP32-level products at the
  // bfloat16 matrix-core rate).  A lane feeds the inner indices 8 (l / 16)
  // .. + 7 of a 32-index step; both operands use that order.
  constexpr bool SPL = FAST && ((SB == 4 && OB == 4) || (SB == 8 && OB == 2));
  constexpr int LR = 16 * SB;   // label rows of a tile
  // dX side (dL/dZ rows along the inner index): a lane's eight inner indices
  // are 4 (l / 16) + t and 16 + 4 (l / 16) + t, so that each load instruction
  // reads 64 contiguous bytes per row; the label parts are staged in the same
  // order (slot 8 (l / 16) + e holds that lane's e-th index)
  constexpr bool PERM = SPL && !YS;
  using Op = BOp<float>;
  using V = typename Op::V;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, lg = lane >> 4;
  const int64_t M = int64_t(1) << a.logM, N = int64_t(1) << a.logN;
  const int RYn = 1 << (2 * a.nRY), RXn = 1 << (2 * a.nRX), SN = 1 << (2 * a.nS);
  const int sSuper = (SN + 16 * SB - 1) / (16 * SB);
  const int64_t OUT = YS ? N : M, INNER = YS ? M : N;
  const int64_t oTiles = (OUT + 64 * OB - 1) / (64 * OB);
  int64_t b = blk;
  const int64_t ot = b % oTiles; b /= oTiles;
  const int ss = (int)(b % sSuper); b /= sSuper;
  const int rO = (int)(b % (YS ? RYn : RXn)); b /= (YS ? RYn : RXn);
  const int64_t p = b;
  const int rI = (int)(p / a.kChunks), kc = (int)(p % a.kChunks);
  const int rX = YS ? rI : rO, rY = YS ? rO : rI;
  const int64_t k0 = (int64_t)kc * a.kChunk;
  const int64_t k1 = INNER < k0 + a.kChunk ? INNER : k0 + a.kChunk;
  const int64_t ow = ot * 64 * OB + wave * 16 * OB;
  const float *L = static_cast<const float *>(YS ? a.X : a.Y);
  const float *dZ = static_cast<const float *>(a.dZ) + ((int64_t)rX * RYn + rY) * M * N;
  // staging: thread t owns label rows t / 4 + 64 r, eight inner indices at
  // 8 (t % 4)
  const int sr = tid >> 2, sq = tid & 3;
  bool st_ok[RPT];
  const float *lrow[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int s_st = ss * 16 * SB + sr + 64 * r;
    st_ok[r] = s_st < SN;
    lrow[r] = L + (int64_t)(st_ok[r] ? row_of(YS ? a.mx : a.my, s_st, YS ? rX : rY) : 0) * INNER;
  }
  float g[RPT][8];
  // FAST: the label slice's halves past the chunk end (chunks of 16) are
  // zeroed when staged; a label past 4^nS reads row 0 and feeds only MFMA rows
  // that are never stored
  bool gok[2] = {true, true};
  auto gload = [&](int64_t n0) {
    const int64_t c = n0 + 8 * sq;
    if constexpr (FAST) {
      using gfv = const __attribute__((address_space(1))) f32x4 *;
      gok[0] = c < k1;
      gok[1] = c + 4 < k1;
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const f32x4 q0 = *(gfv)(lrow[r] + (gok[0] ? c : 0));
        const f32x4 q1 = *(gfv)(lrow[r] + (gok[1] ? c + 4 : 0));
#pragma unroll
        for (int t = 0; t < 4; ++t) g[r][t] = q0[t], g[r][4 + t] = q1[t];
      }
    } else {
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        load4m<float>(lrow[r], c, k1, g[r]);
        load4m<float>(lrow[r], c + 4, k1, g[r] + 4);
        if (!st_ok[r])
          for (int e = 0; e < 8; ++e) g[r][e] = 0.f;
      }
    }
  };
  auto sstore = [&](int buf) {
    if constexpr (SPL) {
      // three part planes; values past the chunk end are zero
      __bf16 *lb = reinterpret_cast<__bf16 *>(ls);
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
      bf16x8 ph, pm, pl;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float x = gok[e >> 2] ? g[r][e] : 0.f;
        __bf16 h, m, l;
        split_bf16(x, h, m, l);
        ph[e] = h, pm[e] = m, pl[e] = l;
      }
      __bf16 *d = lb + ((buf * 3) * LR + sr + 64 * r) * kSplitLd;
      if constexpr (PERM) {
        // inner index i sits at slot 8 ((i % 16) / 4) + 4 (i / 16) + i % 4
        typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
        const int sa = 8 * ((8 * sq & 15) >> 2) + 4 * (8 * sq >> 4);
        const int sbb = 8 * (((8 * sq + 4) & 15) >> 2) + 4 * ((8 * sq + 4) >> 4);
        const bf16x8 *pp[3] = {&ph, &pm, &pl};
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const bf16x8 v = *pp[q];
          *reinterpret_cast<bf16x4 *>(d + q * LR * kSplitLd + sa) = bf16x4{v[0], v[1], v[2], v[3]};
          *reinterpret_cast<bf16x4 *>(d + q * LR * kSplitLd + sbb) = bf16x4{v[4], v[5], v[6], v[7]};
        }
      } else {
        *reinterpret_cast<bf16x8 *>(d + 8 * sq) = ph;
        *reinterpret_cast<bf16x8 *>(d + 8 * sq + LR * kSplitLd) = pm;
        *reinterpret_cast<bf16x8 *>(d + 8 * sq + 2 * LR * kSplitLd) = pl;
      }
      }
      return;
    }
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      float *d = &ls[buf][sr + 64 * r][8 * sq];
      if constexpr (FAST) {
        const float z = 0.f;
        *reinterpret_cast<float4 *>(d) =
            gok[0] ? make_float4(g[r][0], g[r][1], g[r][2], g[r][3]) : make_float4(z, z, z, z);
        *reinterpret_cast<float4 *>(d + 4) =
            gok[1] ? make_float4(g[r][4], g[r][5], g[r][6], g[r][7]) : make_float4(z, z, z, z);
      } else {
        *reinterpret_cast<float4 *>(d) = make_float4(g[r][0], g[r][1], g[r][2], g[r][3]);
        *reinterpret_cast<float4 *>(d + 4) = make_float4(g[r][4], g[r][5], g[r][6], g[r][7]);
      }
    }
  };
  float bv[2][OB][4];
  // dY side, FAST, four output blocks, at least four columns: block ob of a
  // wave takes the columns ow + 4 j + ob (j the MFMA column), so a lane's four
  // blocks are four adjacent columns of one dL/dZ row and come in one 16-byte
  // load per inner index (a 256-byte row segment per 16 lanes) instead of four
  // strided element loads
  constexpr bool kVecY = YS && FAST && OB == 4;
  const bool vecy = kVecY && OUT >= 4;
  const int64_t o4 = ow + 4 * l16, oc4 = o4 < OUT ? o4 : 0;
  auto bload = [&](int h, int64_t n0) {
    const int64_t c = n0 + 4 * lg;
    if constexpr (kVecY) {
      if (vecy) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const f32x4 q = *(const __attribute__((address_space(1))) f32x4 *)(dZ + (c + t) * N + oc4);
#pragma unroll
          for (int ob = 0; ob < OB; ++ob) bv[h][ob][t] = q[ob];
        }
        return;
      }
    }
#pragma unroll
    for (int ob = 0; ob < OB; ++ob) {
      const int64_t o = ow + ob * 16 + l16;
      if constexpr (FAST) {
        // c + 3 < k1 always (groups of 16 inside a chunk); an output column
        // past OUT reads a clamped address and lands in an MFMA column that is
        // never stored
        const int64_t oc = o < OUT ? o : 0;
        if (!YS) {
          const f32x4 q = *(const __attribute__((address_space(1))) f32x4 *)(dZ + oc * N + c);
#pragma unroll
          for (int t = 0; t < 4; ++t) bv[h][ob][t] = q[t];
        } else {
          const __attribute__((address_space(1))) float *q =
              (const __attribute__((address_space(1))) float *)dZ + c * N + oc;
#pragma unroll
          for (int t = 0; t < 4; ++t) bv[h][ob][t] = q[t * N];
        }
      } else if (!YS) {
        if (o < OUT) load4m<float>(dZ + o * N, c, k1, bv[h][ob]);
        else
          for (int t = 0; t < 4; ++t) bv[h][ob][t] = 0.f;
      } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) bv[h][ob][t] = (o < OUT && c + t < k1) ? dZ[(c + t) * N + o] : 0.f;
      }
    }
  };
  V acc[SB][OB];
#pragma unroll
  for (int i = 0; i < SB; ++i)
#pragma unroll
    for (int j = 0; j < OB; ++j) acc[i][j] = V{0, 0, 0, 0};
  auto half = [&](int cur, int h) {
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) {
      const float4 q = *reinterpret_cast<const float4 *>(&ls[cur][sb * 16 + l16][16 * h + 4 * lg]);
      const float av[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int ob = 0; ob < OB; ++ob) acc[sb][ob] = Op::run(av[t], bv[h][ob][t], acc[sb][ob]);
    }
  };
  // split form: dL/dZ operands of the step at s0 (inner indices s0 + 8 lg +
  // 4 hh + t, or s0 + 16 hh + 4 lg + t on the dX side); with only 16 indices
  // left (full false) the loads past them read first-half addresses, and their
  // values are zeroed before use
  auto spl_load = [&](float (&dst)[2][OB][4], int64_t s0, bool full) {
    const int64_t c = s0 + (PERM ? 4 * lg : 8 * lg - (full || lg < 2 ? 0 : 16));
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
      const int64_t cc = PERM ? c + (full ? 16 * hh : 0) : c + 4 * hh;
      if constexpr (kVecY) {
        if (vecy) {
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const f32x4 q = *(const __attribute__((address_space(1))) f32x4 *)(dZ + (cc + t) * N + oc4);
#pragma unroll
            for (int ob = 0; ob < OB; ++ob) dst[hh][ob][t] = q[ob];
          }
          continue;
        }
      }
#pragma unroll
      for (int ob = 0; ob < OB; ++ob) {
        const int64_t o = ow + ob * 16 + l16;
        const int64_t oc = o < OUT ? o : 0;
        if (!YS) {
          const f32x4 q = *(const __attribute__((address_space(1))) f32x4 *)(dZ + oc * N + cc);
#pragma unroll
          for (int t = 0; t < 4; ++t) dst[hh][ob][t] = q[t];
        } else {
          const __attribute__((address_space(1))) float *q =
              (const __attribute__((address_space(1))) float *)dZ + cc * N + oc;
#pragma unroll
          for (int t = 0; t < 4; ++t) dst[hh][ob][t] = q[t * N];
        }
      }
    }
  };
  // the parts of a step's dL/dZ operands, split once when they arrive (the
  // lanes past a 16-index last step get zeros)
  bf16x8 dp[SPL ? OB : 1][3];
  auto spl_split = [&](const float (&src)[2][OB][4], bool full) {
    const bool hv = full || lg < 2;
#pragma unroll
    for (int ob = 0; ob < (SPL ? OB : 0); ++ob)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const bool ok = PERM ? full || e < 4 : hv;
        const float x = ok ? src[e >> 2][ob][e & 3] : 0.f;
        __bf16 h, m, l;
        split_bf16(x, h, m, l);
        dp[ob][0][e] = h, dp[ob][1][e] = m, dp[ob][2][e] = l;
      }
  };
  auto spl_step = [&](int cur) {
    const __bf16 *lb = reinterpret_cast<const __bf16 *>(ls) + (cur * 3) * LR * kSplitLd;
#pragma unroll
    for (int sb = 0; sb < SB; ++sb) {
      bf16x8 lp[3];
#pragma unroll
      for (int q = 0; q < 3; ++q)
        lp[q] = *reinterpret_cast<const bf16x8 *>(lb + (q * LR + sb * 16 + l16) * kSplitLd + 8 * lg);
      // (label part, dL/dZ part), smallest first
      constexpr int kPi[6] = {0, 2, 1, 0, 1, 0}, kPj[6] = {2, 0, 1, 1, 0, 0};
#pragma unroll
      for (int u = 0; u < 6; ++u)
#pragma unroll
        for (int ob = 0; ob < (SPL ? OB : 0); ++ob)
          acc[sb][ob] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(lp[kPi[u]], dp[ob][kPj[u]], acc[sb][ob], 0, 0, 0);
    }
  };
  if constexpr (FAST) {
    // every operand of step n0 + KS (label slice and both dL/dZ halves) is
    // loaded at the top of step n0 into a second register set; step n0 reads
    // only registers loaded one step earlier, so its matrix-core work never
    // waits on the loads in flight
    float bn[2][OB][4];
    if (k0 < k1) {
      gload(k0);
      sstore(0);
      if constexpr (SPL) {
        spl_load(bn, k0, k0 + 16 < k1);
        spl_split(bn, k0 + 16 < k1);
      } else {
        bload(0, k0);
        if (k0 + 16 < k1) bload(1, k0 + 16);
      }
    }
    __syncthreads();
    int cur = 0;
    for (int64_t n0 = k0; n0 < k1; n0 += KS) {
      const bool more = n0 + KS < k1;
      const bool h1 = n0 + 16 < k1;
      const bool h1n = n0 + KS + 16 < k1;
      if (SPL && more) {
        gload(n0 + KS);
        spl_load(bn, n0 + KS, h1n);
      } else if (more) {
        gload(n0 + KS);
        const int64_t c = n0 + KS + 4 * lg;
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          if constexpr (kVecY) {
            if (vecy) {
              const int64_t cc = hh == 0 || h1n ? c + 16 * hh : c;
#pragma unroll
              for (int t = 0; t < 4; ++t) {
                const f32x4 q = *(const __attribute__((address_space(1))) f32x4 *)(dZ + (cc + t) * N + oc4);
#pragma unroll
                for (int ob = 0; ob < OB; ++ob) bn[hh][ob][t] = q[ob];
              }
              continue;
            }
          }
#pragma unroll
          for (int ob = 0; ob < OB; ++ob) {
            const int64_t o = ow + ob * 16 + l16;
            const int64_t oc = o < OUT ? o : 0;
            // the second half of the last step may lie past the chunk: it
            // reads the first half's address and is never used
            const int64_t cc = hh == 0 || h1n ? c + 16 * hh : c;
            if (!YS) {
              const f32x4 q = *(const __attribute__((address_space(1))) f32x4 *)(dZ + oc * N + cc);
#pragma unroll
              for (int t = 0; t < 4; ++t) bn[hh][ob][t] = q[t];
            } else {
              const __attribute__((address_space(1))) float *q =
                  (const __attribute__((address_space(1))) float *)dZ + cc * N + oc;
#pragma unroll
              for (int t = 0; t < 4; ++t) bn[hh][ob][t] = q[t * N];
            }
          }
        }
      }
      // keep the loads above the matrix-core work (the scheduler would sink
      // them next to their use to save registers, and the work would wait)
      __builtin_amdgcn_sched_barrier(0);
      if constexpr (SPL) {
        spl_step(cur);
        if (more) {
          sstore(cur ^ 1);
          spl_split(bn, h1n);
        }
        __syncthreads();
        cur ^= 1;
        continue;
      } else {
        half(cur, 0);
        if (h1) half(cur, 1);
      }
      if (more) {
        sstore(cur ^ 1);
#pragma unroll
        for (int hh = 0; hh < 2; ++hh)
#pragma unroll
          for (int ob = 0; ob < OB; ++ob)
#pragma unroll
            for (int t = 0; t < 4; ++t) bv[hh][ob][t] = bn[hh][ob][t];
      }
      __syncthreads();
      cur ^= 1;
    }
  } else {
    if (k0 < k1) {
      gload(k0);
      sstore(0);
      bload(0, k0);
    }
    __syncthreads();
    int cur = 0;
    for (int64_t n0 = k0; n0 < k1; n0 += KS) {
      const bool more = n0 + KS < k1;
      const bool h1 = n0 + 16 < k1;
      if (more) gload(n0 + KS);
      if (h1) bload(1, n0 + 16);
      half(cur, 0);
      if (more) bload(0, n0 + KS);
      if (h1) half(cur, 1);
      if (more) sstore(cur ^ 1);
      __syncthreads();
      cur ^= 1;
    }
  }
  float *part = static_cast<float *>(a.part) + p * (YS ? a.rowsY : a.rowsX) * OUT;
  if constexpr (kVecY) {
    if (vecy) {
      // a lane's four output blocks are four adjacent columns (OUT, a power
      // of two of at least four, holds whole groups of four): one 16-byte
      // store per label row
#pragma unroll
      for (int sb = 0; sb < SB; ++sb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int s = (ss * SB + sb) * 16 + 4 * lg + r;
          if (s < SN && o4 < OUT)
            *reinterpret_cast<float4 *>(part + (int64_t)row_of(a.my, s, rO) * OUT + o4) =
                make_float4(acc[sb][0][r], acc[sb][1][r], acc[sb][2][r], acc[sb][3][r]);
        }
      return;
    }
  }
#pragma unroll
  for (int sb = 0; sb < SB; ++sb)
#pragma unroll
    for (int ob = 0; ob < OB; ++ob) {
      const int64_t o = ow + ob * 16 + l16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int s = (ss * SB + sb) * 16 + 4 * lg + r;
        if (s < SN && o < OUT) part[(int64_t)row_of(YS ? a.my : a.mx, s, rO) * OUT + o] = acc[sb][ob][r];
      }
    }
}

template <typename T, int SB, int MB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(BwdCfg<T, SB>::kWaves, 8)))
void k_bwd_x(const BwdArgs a) {
  if constexpr (sizeof(T) == 4 && ((SB == 4 && MB == 4) || (SB == 8 && MB == 2) || (SB == 16 && MB == 1))) {
    __shared__ __attribute__((aligned(16))) float lsraw[StagedLds<SB>::kFloats];
    auto ls = reinterpret_cast<float (*)[16 * SB][kStagedLd]>(lsraw);
    if (a.logN >= 4) bwd_block_staged<false, true, SB, MB>(a, blockIdx.x, ls);
    else bwd_block_staged<false, false, SB, MB>(a, blockIdx.x, ls);
  } else {
    bwd_x_block<T, SB, MB>(a, blockIdx.x);
  }
}

template <typename T, int SB, int NB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(BwdCfg<T, SB>::kWaves, 8)))
void k_bwd_y(const BwdArgs a) {
  if constexpr (sizeof(T) == 4 && ((SB == 4 && NB == 4) || (SB == 16 && NB == 1))) {
    __shared__ __attribute__((aligned(16))) float lsraw[StagedLds<SB>::kFloats];
    auto ls = reinterpret_cast<float (*)[16 * SB][kStagedLd]>(lsraw);
    if (a.logM >= 4) bwd_block_staged<true, true, SB, NB>(a, blockIdx.x, ls);
    else bwd_block_staged<true, false, SB, NB>(a, blockIdx.x, ls);
  } else {
    bwd_y_block<T, SB, NB>(a, blockIdx.x);
  }
}

// Many adjoint steps of one shape in one persistent launch: blocks take
// (step, block) items from an atomic counter; descs[d] in device memory,
// prefix[d] = first item of step d, queue zeroed before the launch.
template <typename T, int SB, int MB, bool Y>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(BwdCfg<T, SB>::kWaves, 8)))
void k_bwd_queue(const BwdArgs *descs, const int64_t *prefix, int ndesc, unsigned long long *queue,
                 int64_t total) {
  __shared__ int64_t item;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) item = (int64_t)atomicAdd(queue, 1ull);
    __syncthreads();
    const int64_t it = item;
    if (it >= total) return;
    const int d = find_desc(prefix, ndesc, it);
    if constexpr (sizeof(T) == 4 && ((SB == 4 && MB == 4) || (SB == 8 && MB == 2) || (SB == 16 && MB == 1))) {
      __shared__ __attribute__((aligned(16))) float lsraw[StagedLds<SB>::kFloats];
      auto ls = reinterpret_cast<float (*)[16 * SB][kStagedLd]>(lsraw);
      const BwdArgs &a = descs[d];
      if ((Y ? a.logM : a.logN) >= 4) bwd_block_staged<Y, true, SB, MB>(a, it - prefix[d], ls);
      else bwd_block_staged<Y, false, SB, MB>(a, it - prefix[d], ls);
    } else {
      if (Y) bwd_y_block<T, SB, MB>(descs[d], it - prefix[d]);
      else bwd_x_block<T, SB, MB>(descs[d], it - prefix[d]);
    }
  }
}

// ---- Both sides of a step with at most 16 labels from one read of dL/dZ.
// A block takes one batch entry b = (rX, rY), a tile of kDualRows rows of
// dZ_b and a chunk of kDualChunk columns, and streams the chunk through LDS in
// sub-tiles of kDualRows x kDualCols (double-buffered: the next sub-tile's
// loads are in flight while the current one is on the matrix cores).  Both
// products take their dL/dZ operand from the staged sub-tile:
//   dX[rowX(s,rX)][m] (+)= sum_n Y[rowY(s,rY)][n] dZ_b[m][n]: wave w owns rows
//     32 w .. 32 w + 31 of the tile and accumulates over the whole chunk;
//   dY[rowY(s,rY)][n] (+)= sum_m X[rowX(s,rX)][m] dZ_b[m][n]: wave w owns
//     columns 16 w .. 16 w + 15 of each sub-tile and sums over the tile's rows.
// Two product forms:
//   16 labels (two shared cuts): 16 x 16 x 4 products, label s is MFMA row
//     l % 16; lane l feeds the inner indices 4 (l / 16) + t of a 16-index
//     group to MFMA t;
//   at most 4 labels (one shared cut or none, ONE): the 16-block 4 x 4 x 1
//     product, in which lane 4 q + i feeds element i of block q's A column and
//     B row, and lane 4 q + j, register r receives block q's C[r][j].  For dX,
//     block q takes column 16 c + q of the sub-tile, rows 4 g + i and label j;
//     for dY, block q = 4 h + c takes row 4 k + h, label i and column 4 c + j
//     of the wave's 16.  The blocks' sums are added across lanes (over q for
//     dX at the end of the chunk, over h for dY per sub-tile), so all of the
//     products' work is useful instead of a quarter of it.
// Labels >= 4^nS are zero rows or never-stored outputs.  The label operands of
// the next sub-tile are loaded with its dL/dZ, so no wait inside the
// matrix-core loop covers the staging loads.  Partials (fixed order, added by
// the reduce pass): X side part[(rY kChunks + column chunk)][row][m], Y side
// part2[(rX kChunks2 + row tile)][row][n].
constexpr int kDualLd = kDualCols + 4;
template <bool ONE>
__device__ __forceinline__ void bwd_dual_block(const BwdArgs &a, int64_t blk, float (*gs)[kDualRows][kDualLd]) {
  constexpr int TR = kDualRows, TC = kDualCols;
  using V = f32x4;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int l16 = lane & 15, lg = lane >> 4;
  const int q4 = lane >> 2, i4 = lane & 3;   // 4 x 4 x 1 block and element
  const int64_t M = int64_t(1) << a.logM, N = int64_t(1) << a.logN;
  const int RYn = 1 << (2 * a.nRY), SN = 1 << (2 * a.nS);
  int64_t b = blk;
  const int kc = (int)(b % a.kChunks); b /= a.kChunks;
  const int mt = (int)(b % a.kChunks2); b /= a.kChunks2;
  const int rX = (int)(b / RYn), rY = (int)(b % RYn);
  const int64_t m0 = (int64_t)mt * TR;
  const int64_t n0 = (int64_t)kc * a.kChunk;
  const int64_t n1 = N < n0 + a.kChunk ? N : n0 + a.kChunk;
  const float *X = static_cast<const float *>(a.X);
  const float *Y = static_cast<const float *>(a.Y);
  const float *dZ = static_cast<const float *>(a.dZ) + ((int64_t)rX * RYn + rY) * M * N;
  // Every load below is an unconditional global load: the column sub-tiles
  // are always whole (N >= 64, both powers of two), and a row past M (tiles of
  // M = 64) or a label past 4^nS reads a clamped in-range address.  Rows past
  // M are zeroed when staged (they are summed over for dY); a label past 4^nS
  // only feeds MFMA outputs that are never stored.  Nothing consumes a loaded
  // value before the staging point, so no wait sits between the loads and the
  // matrix-core work they overlap.
  auto ld = [](const float *p) {
    const f32x4 v = *(const __attribute__((address_space(1))) f32x4 *)p;
    return make_float4(v[0], v[1], v[2], v[3]);
  };
  auto ld1 = [](const float *p) { return *(const __attribute__((address_space(1))) float *)p; };
  auto sel = [](bool ok, float4 v) {
    return make_float4(ok ? v.x : 0.f, ok ? v.y : 0.f, ok ? v.z : 0.f, ok ? v.w : 0.f);
  };
  // this lane's label as an MFMA operand row: l % 16 (16-label form), i4 (ONE)
  const int lab = ONE ? i4 : l16;
  const bool sok = lab < SN;
  const float *xl = X + (int64_t)(sok ? row_of(a.mx, lab, rX) : 0) * M;
  const float *yl = Y + (int64_t)(sok ? row_of(a.my, lab, rY) : 0) * N;
  // X operands of the tile's rows, once per block: rows m0 + 16 kr + 4 lg + t
  // (16-label form) or m0 + 4 k + lg (ONE: the dY block's row phase h = lg)
  float xa[TR / 4];
  if constexpr (ONE) {
#pragma unroll
    for (int k = 0; k < TR / 4; ++k) {
      const int64_t m = m0 + 4 * k + lg;
      const float v = ld1(xl + (m < M ? m : 0));
      xa[k] = m < M ? v : 0.f;
    }
  } else {
#pragma unroll
    for (int kr = 0; kr < TR / 16; ++kr) {
      const int64_t m = m0 + 16 * kr + 4 * lg;
      const float4 v = sel(m < M, ld(xl + (m < M ? m : 0)));
      xa[4 * kr] = v.x, xa[4 * kr + 1] = v.y, xa[4 * kr + 2] = v.z, xa[4 * kr + 3] = v.w;
    }
  }
  // staging: thread t loads rows t / 16 + 16 j, columns 4 (t % 16) + 0..3;
  // label operands of a sub-tile: columns 16 kq + 4 lg + 0..3 (16-label form)
  // or column 16 kq + q4 (ONE)
  float4 gr[TR / 16];
  float4 yn[TC / 16];
  float yn1[TC / 16];
  auto load_sub = [&](int64_t c0) {
#pragma unroll
    for (int j = 0; j < TR / 16; ++j) {
      const int64_t m = m0 + (tid >> 4) + 16 * j;
      gr[j] = ld(dZ + (m < M ? m : 0) * N + c0 + 4 * (tid & 15));
    }
#pragma unroll
    for (int kq = 0; kq < TC / 16; ++kq) {
      if constexpr (ONE) yn1[kq] = ld1(yl + c0 + 16 * kq + q4);
      else yn[kq] = ld(yl + c0 + 16 * kq + 4 * lg);
    }
  };
  auto store_sub = [&](int buf) {
#pragma unroll
    for (int j = 0; j < TR / 16; ++j)
      *reinterpret_cast<float4 *>(&gs[buf][(tid >> 4) + 16 * j][4 * (tid & 15)]) =
          sel(m0 + (tid >> 4) + 16 * j < M, gr[j]);
  };
  V ax[ONE ? 8 : 2];
#pragma unroll
  for (int r = 0; r < (ONE ? 8 : 2); ++r) ax[r] = V{0, 0, 0, 0};
  float4 yc[TC / 16];
  float yc1[TC / 16];
  auto next_y = [&]() {
#pragma unroll
    for (int kq = 0; kq < TC / 16; ++kq) {
      if constexpr (ONE) yc1[kq] = yn1[kq];
      else yc[kq] = yn[kq];
    }
  };
  const int nsub = (int)((n1 - n0) / TC);
  load_sub(n0);
  store_sub(0);
  next_y();
  __syncthreads();
  __attribute__((address_space(1))) float *part2 =
      (__attribute__((address_space(1))) float *)static_cast<float *>(a.part2) +
      ((int64_t)rX * a.kChunks2 + mt) * a.rowsY * N;
  // dY output rows: labels 4 lg + r (16-label form, register r) or lg (ONE:
  // after the sum over row phases each lane stores the label of its phase)
  int yrow[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int sr = ONE ? lg : 4 * lg + r;
    yrow[r] = sr < SN ? row_of(a.my, sr, rY) : -1;
  }
  for (int i = 0; i < nsub; ++i) {
    const int cur = i & 1;
    const int64_t c0 = n0 + (int64_t)i * TC;
    const bool more = i + 1 < nsub;
    if (more) load_sub(c0 + TC);
    if constexpr (ONE) {
      // dX: rows 32 w + 4 g + i4 at column 16 kq + q4, against label i4
#pragma unroll
      for (int kq = 0; kq < TC / 16; ++kq)
#pragma unroll
        for (int g = 0; g < 8; ++g)
          ax[g] = __builtin_amdgcn_mfma_f32_4x4x1f32(gs[cur][32 * wave + 4 * g + i4][16 * kq + q4], yc1[kq],
                                                     ax[g], 0, 0, 0);
      // dY: rows 4 k + lg (row phase h = lg), columns 16 w + 4 c + i4 (c = q4 % 4)
      V ay[4] = {V{0, 0, 0, 0}, V{0, 0, 0, 0}, V{0, 0, 0, 0}, V{0, 0, 0, 0}};
#pragma unroll
      for (int k = 0; k < TR / 4; ++k)
        ay[k & 3] = __builtin_amdgcn_mfma_f32_4x4x1f32(xa[k], gs[cur][4 * k + lg][16 * wave + l16], ay[k & 3], 0, 0,
                                                       0);
      float v[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        v[r] = (ay[0][r] + ay[1][r]) + (ay[2][r] + ay[3][r]);
        v[r] += __shfl_xor(v[r], 16, 64);
        v[r] += __shfl_xor(v[r], 32, 64);
      }
      // lane (h, c, j) stores label h of column 16 w + 4 c + j
      const float out = lg == 0 ? v[0] : lg == 1 ? v[1] : lg == 2 ? v[2] : v[3];
      if (yrow[0] >= 0) part2[(int64_t)yrow[0] * N + c0 + 16 * wave + l16] = out;
    } else {
      // dX: rows 32 w + 16 mb + l16 against the sub-tile's 64 columns
#pragma unroll
      for (int kq = 0; kq < TC / 16; ++kq)
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
          const float4 g = *reinterpret_cast<const float4 *>(&gs[cur][32 * wave + 16 * mb + l16][16 * kq + 4 * lg]);
          const float gv[4] = {g.x, g.y, g.z, g.w};
          const float yv[4] = {yc[kq].x, yc[kq].y, yc[kq].z, yc[kq].w};
#pragma unroll
          for (int t = 0; t < 4; ++t) ax[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(yv[t], gv[t], ax[mb], 0, 0, 0);
        }
      // dY: columns 16 w + l16 over the tile's rows
      V ay = V{0, 0, 0, 0};
#pragma unroll
      for (int kr = 0; kr < TR / 16; ++kr)
#pragma unroll
        for (int t = 0; t < 4; ++t)
          ay = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[4 * kr + t], gs[cur][16 * kr + 4 * lg + t][16 * wave + l16], ay,
                                                    0, 0, 0);
      const int64_t n = c0 + 16 * wave + l16;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (yrow[r] >= 0) part2[(int64_t)yrow[r] * N + n] = ay[r];
    }
    if (more) {
      store_sub(cur ^ 1);
      next_y();
    }
    __syncthreads();
  }
  __attribute__((address_space(1))) float *part =
      (__attribute__((address_space(1))) float *)static_cast<float *>(a.part) +
      ((int64_t)rY * a.kChunks + kc) * a.rowsX * M;
  if constexpr (ONE) {
    // sum the 16 column phases (blocks q4); lane (q4 < 8, j) then stores rows
    // 32 w + 4 q4 .. + 3 of label j as one 16-byte store
    float4 o = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int g = 0; g < 8; ++g) {
      float v[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        v[r] = ax[g][r];
#pragma unroll
        for (int s = 4; s <= 32; s <<= 1) v[r] += __shfl_xor(v[r], s, 64);
      }
      if (q4 == g) o = make_float4(v[0], v[1], v[2], v[3]);
    }
    const int64_t m = m0 + 32 * wave + 4 * q4;
    if (q4 < 8 && sok && m < M) {
      const int64_t row = row_of(a.mx, i4, rX);
      *reinterpret_cast<__attribute__((address_space(1))) f32x4 *>(part + row * M + m) = f32x4{o.x, o.y, o.z, o.w};
    }
  } else {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int sr = 4 * lg + r;
      if (sr >= SN) continue;
      const int64_t row = row_of(a.mx, sr, rX);
#pragma unroll
      for (int mb = 0; mb < 2; ++mb) {
        const int64_t m = m0 + 32 * wave + 16 * mb + l16;
        if (m < M) part[row * M + m] = ax[mb][r];
      }
    }
  }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8))) void k_bwd_dual_queue(const BwdArgs *descs, const int64_t *prefix, int ndesc,
                                                        unsigned long long *queue, int64_t total) {
  __shared__ int64_t item;
  __shared__ float gs[2][kDualRows][kDualLd];
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) item = (int64_t)atomicAdd(queue, 1ull);
    __syncthreads();
    const int64_t it = item;
    if (it >= total) return;
    const int d = find_desc(prefix, ndesc, it);
    const BwdArgs &a = descs[d];
    if (a.nS <= 1) bwd_dual_block<true>(a, it - prefix[d], gs);
    else bwd_dual_block<false>(a, it - prefix[d], gs);
  }
}

// out[i] = scale * sum_{p < P} part[p][i].  With G = 8, eight threads share
// an output: thread g adds the g-th of eight consecutive ranges of partials in
// ascending p, then the range sums are added in range order (for few outputs
// and many partials: eight times the loads in flight); with G = 1 one thread
// adds all P in ascending p.  Either order is fixed for a given P.
template <typename T, typename O, int G>
__global__ __launch_bounds__(256) void k_bwd_reduce(const T *part, int64_t count, int64_t P,
                                                    double scale, O *out) {
  constexpr int W = 256 / G;   // outputs per block and pass
  __shared__ T sums[G][W + 1];
  const int g = threadIdx.x / W, j = threadIdx.x % W;
  const int64_t per = (P + G - 1) / G;
  const int64_t p0 = g * per, p1 = P < p0 + per ? P : p0 + per;
  for (int64_t base = (int64_t)blockIdx.x * W; base < count; base += (int64_t)gridDim.x * W) {
    const int64_t i = base + j;
    T s = 0;
    if (i < count) {
      int64_t p = p0;
      for (; p + 4 <= p1; p += 4) {
        const T v0 = part[p * count + i], v1 = part[(p + 1) * count + i];
        const T v2 = part[(p + 2) * count + i], v3 = part[(p + 3) * count + i];
        s += v0; s += v1; s += v2; s += v3;
      }
      for (; p < p1; ++p) s += part[p * count + i];
    }
    if (G == 1) {
      if (i < count) out[i] = (O)(s * (T)scale);
      continue;
    }
    sums[g][j] = s;
    __syncthreads();
    if (g == 0 && i < count) {
      T t = sums[0][j];
#pragma unroll
      for (int q = 1; q < G; ++q) t += sums[q][j];
      out[i] = (O)(t * (T)scale);
    }
    __syncthreads();
  }
}

// Gather a globally ordered vector into blocked [m][n] order:
// dst[m * N + n] = src[rowoff(m) + coloff(n)].
template <typename T>
__global__ __launch_bounds__(256) void k_gather_blocked(const T *src, T *dst, int logM, int logN,
                                                        BitPos px, BitPos py) {
  const int64_t total = int64_t(1) << (logM + logN);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = i >> logN, n = i & ((int64_t(1) << logN) - 1);
    int64_t addr = 0;
    for (int j = 0; j < logM; ++j) {
      const uint64_t w = px.w[j / 10];
      addr |= ((m >> j) & 1) << ((w >> (6 * (j % 10))) & 63);
    }
    for (int j = 0; j < logN; ++j) {
      const uint64_t w = py.w[j / 10];
      addr |= ((n >> j) & 1) << ((w >> (6 * (j % 10))) & 63);
    }
    dst[i] = src[addr];
  }
}

// Batched adjoint: every reduction of one level in one launch.  Block b
// belongs to descriptor d with start[d] <= b < start[d + 1]; its 256 threads
// each add one output's P partials in ascending p (a fixed order).
template <typename T>
__global__ __launch_bounds__(256) void k_bwd_reduce_table(const BwdReduceDesc *descs, const int64_t *start,
                                                          int ndesc, int64_t blocks) {
  for (int64_t b = blockIdx.x; b < blocks; b += gridDim.x) {
    const int d = find_desc(start, ndesc, b);
    const BwdReduceDesc &D = descs[d];
    if constexpr (sizeof(T) == 4) {
      if (D.vec) {
        // four consecutive outputs per thread, eight partials' loads in flight;
        // each output still adds its partials in ascending p
        const int64_t i = ((b - start[d]) * 256 + threadIdx.x) * 4;
        if (i >= D.count) continue;
        using gv = const __attribute__((address_space(1))) f32x4 *;
        const float *part = static_cast<const float *>(D.part) + i;
        f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
        int64_t p = 0;
        for (; p + 8 <= D.P; p += 8) {
          f32x4 v[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) v[u] = *(gv)(part + (p + u) * D.count);
#pragma unroll
          for (int u = 0; u < 8; ++u) acc += v[u];
        }
        for (; p < D.P; ++p) acc += *(gv)(part + p * D.count);
        const float sc = (float)D.scale;
        if (D.out_double) {
          double *o = static_cast<double *>(D.out) + i;
          reinterpret_cast<double2 *>(o)[0] = make_double2((double)(acc[0] * sc), (double)(acc[1] * sc));
          reinterpret_cast<double2 *>(o)[1] = make_double2((double)(acc[2] * sc), (double)(acc[3] * sc));
        } else {
          *reinterpret_cast<f32x4 *>(static_cast<float *>(D.out) + i) = acc * sc;
        }
        continue;
      }
    }
    const int64_t i = (b - start[d]) * 256 + threadIdx.x;
    if (i >= D.count) continue;
    const T *part = static_cast<const T *>(D.part);
    T acc = 0;
    int64_t p = 0;
    for (; p + 4 <= D.P; p += 4) {
      const T v0 = part[p * D.count + i], v1 = part[(p + 1) * D.count + i];
      const T v2 = part[(p + 2) * D.count + i], v3 = part[(p + 3) * D.count + i];
      acc += v0; acc += v1; acc += v2; acc += v3;
    }
    for (; p < D.P; ++p) acc += part[p * D.count + i];
    const T v = acc * (T)D.scale;
    if (D.out_double) static_cast<double *>(D.out)[i] = (double)v;
    else static_cast<float *>(D.out)[i] = (float)v;
  }
}

// First launch of a batched adjoint run: zeroes the queue counters of the
// run's persistent launches (a kernel, not a memset, so the run can be
// captured in a graph) and gathers every instance's dL/dp that is not in
// blocked order: dst[m * N + n] = src[rowoff(m) + coloff(n)].
template <typename T>
__global__ __launch_bounds__(256) void k_bwd_prep(const BwdGatherDesc *descs, const int64_t *start, int ndesc,
                                                  int64_t blocks, unsigned long long *counters, int ncounters) {
  if (blockIdx.x == 0 && (int)threadIdx.x < ncounters) counters[threadIdx.x] = 0ull;
  for (int64_t b = blockIdx.x; b < blocks; b += gridDim.x) {
    const int d = find_desc(start, ndesc, b);
    const BwdGatherDesc &D = descs[d];
    const int64_t i = (b - start[d]) * 256 + threadIdx.x;
    if (i >= (int64_t(1) << (D.logM + D.logN))) continue;
    const int64_t m = i >> D.logN, n = i & ((int64_t(1) << D.logN) - 1);
    int64_t addr = 0;
    for (int j = 0; j < D.logM; ++j) {
      const uint64_t w = D.px.w[j / 10];
      addr |= ((m >> j) & 1) << ((w >> (6 * (j % 10))) & 63);
    }
    for (int j = 0; j < D.logN; ++j) {
      const uint64_t w = D.py.w[j / 10];
      addr |= ((n >> j) & 1) << ((w >> (6 * (j % 10))) & 63);
    }
    static_cast<T *>(D.dst)[i] = static_cast<const T *>(D.src)[addr];
  }
}

// Label blocks of 16 per block tile.  Three shared cuts take 64 labels per
// tile, four take 128 on the dX side (two output blocks per wave, so dL/dZ is
// read twice) and 64 on the dY side; in FP32 these tiles run the split
// products.  Measured in C5: the split 64-label dX tiles at four cuts were
// faster than FP32 256-label ones (0.79 -> 0.70 ms for the dX launches,
// although they read dL/dZ four times instead of once) and 128-label split
// tiles faster still (0.65 ms); on the dY side 128 labels with two output
// blocks measured 0.64 ms against 0.54 ms for 64 with four (its dL/dZ loads
// then cover two adjacent columns per lane instead of four).  Five and more
// cuts take 256 (dL/dZ would otherwise be read 16 times; the 256 label rows of
// a 32-index slice are staged in LDS once per block).  (An earlier 256-label
// form in which every wave loaded the same 256 operand rows itself was 1.5x
// slower than 64.)
static int sb_for(int nS, bool y, bool f32) {
  if (nS <= 2) return 1;
  if (nS == 3) return 4;
  if (nS == 4) return f32 && !y ? 8 : 4;
  return 16;
}
// output blocks of 16 per wave for a label-block count
static int ob_for(int SB) { return SB == 16 ? 1 : SB == 8 ? 2 : 4; }

template <typename T>
static Status launch_bwd_t(const BwdArgs &a, bool which_y, hipStream_t s) {
  const int SN = 1 << (2 * a.nS);
  const int SB = sb_for(a.nS, which_y, sizeof(T) == 4);
  const int sSuper = (SN + 16 * SB - 1) / (16 * SB);
  const int64_t M = int64_t(1) << a.logM, N = int64_t(1) << a.logN;
  const int RXn = 1 << (2 * a.nRX), RYn = 1 << (2 * a.nRY);
  if (!which_y) {
    const int MB = ob_for(SB);
    const int64_t tiles = (M + 64 * MB - 1) / (64 * MB);
    const int64_t P = (int64_t)RYn * a.kChunks;
    const dim3 g((unsigned)(P * RXn * sSuper * tiles)), b(256);
    if (SB == 1) return launch("bwd_x", k_bwd_x<T, 1, 4>, g, b, 0, s, a);
    if (SB == 4) return launch("bwd_x", k_bwd_x<T, 4, 4>, g, b, 0, s, a);
    if constexpr (sizeof(T) == 4)
      if (SB == 8) return launch("bwd_x", k_bwd_x<T, 8, 2>, g, b, 0, s, a);
    return launch("bwd_x", k_bwd_x<T, 16, 1>, g, b, 0, s, a);
  }
  const int NB = ob_for(SB);
  const int64_t tiles = (N + 64 * NB - 1) / (64 * NB);
  const int64_t P = (int64_t)RXn * a.kChunks;
  const dim3 g((unsigned)(P * RYn * sSuper * tiles)), b(256);
  if (SB == 1) return launch("bwd_y", k_bwd_y<T, 1, 4>, g, b, 0, s, a);
  if (SB == 4) return launch("bwd_y", k_bwd_y<T, 4, 4>, g, b, 0, s, a);
  return launch("bwd_y", k_bwd_y<T, 16, 1>, g, b, 0, s, a);
}

Status launch_bwd(Acc acc, const BwdArgs &a, bool which_y, hipStream_t s) {
  return acc == Acc::F32 ? launch_bwd_t<float>(a, which_y, s) : launch_bwd_t<double>(a, which_y, s);
}

int bwd_sb(int nS, bool y, bool f32) { return sb_for(nS, y, f32); }

int64_t bwd_blocks(const BwdArgs &a, bool which_y, bool f32) {
  const int SN = 1 << (2 * a.nS);
  const int SB = sb_for(a.nS, which_y, f32);
  const int sSuper = (SN + 16 * SB - 1) / (16 * SB);
  const int64_t M = int64_t(1) << a.logM, N = int64_t(1) << a.logN;
  const int64_t RXn = int64_t(1) << (2 * a.nRX), RYn = int64_t(1) << (2 * a.nRY);
  const int B = ob_for(SB);
  if (!which_y) return (RYn * a.kChunks) * RXn * sSuper * ((M + 64 * B - 1) / (64 * B));
  return (RXn * a.kChunks) * RYn * sSuper * ((N + 64 * B - 1) / (64 * B));
}

template <typename T>
static Status launch_bwd_queue_t(const BwdQueue &q, hipStream_t s) {
  const dim3 g(q.grid), b(256);
  const char *nm = q.y ? "bwd_y_queue" : "bwd_x_queue";
  if (q.y) {
    if (q.sb == 1) return launch(nm, k_bwd_queue<T, 1, 4, true>, g, b, 0, s, q.descs, q.prefix, q.ndesc, q.queue, q.total);
    if (q.sb == 4) return launch(nm, k_bwd_queue<T, 4, 4, true>, g, b, 0, s, q.descs, q.prefix, q.ndesc, q.queue, q.total);
    return launch(nm, k_bwd_queue<T, 16, 1, true>, g, b, 0, s, q.descs, q.prefix, q.ndesc, q.queue, q.total);
  }
  if (q.sb == 1) return launch(nm, k_bwd_queue<T, 1, 4, false>, g, b, 0, s, q.descs, q.prefix, q.ndesc, q.queue, q.total);
  if (q.sb == 4) return launch(nm, k_bwd_queue<T, 4, 4, false>, g, b, 0, s, q.descs, q.prefix, q.ndesc, q.queue, q.total);
  if constexpr (sizeof(T) == 4)
    if (q.sb == 8) return launch(nm, k_bwd_queue<T, 8, 2, false>, g, b, 0, s, q.descs, q.prefix, q.ndesc, q.queue, q.total);
  return launch(nm, k_bwd_queue<T, 16, 1, false>, g, b, 0, s, q.descs, q.prefix, q.ndesc, q.queue, q.total);
}

Status launch_bwd_queue(Acc acc, const BwdQueue &q, hipStream_t s) {
  if (q.total <= 0) return Status::ok();
  if (q.dual) {
    if (acc != Acc::F32) return Status::fail(CQC_ERR_INVALID_ARG, "the two-sided adjoint pass is FP32 only");
    return launch("bwd_dual_queue", k_bwd_dual_queue, dim3(q.grid), dim3(256), 0, s, q.descs, q.prefix, q.ndesc,
                  q.queue, q.total);
  }
  return acc == Acc::F32 ? launch_bwd_queue_t<float>(q, s) : launch_bwd_queue_t<double>(q, s);
}

Status launch_bwd_reduce_table(Acc acc, const BwdReduceDesc *descs, const int64_t *start, int ndesc,
                               int64_t blocks, hipStream_t s) {
  if (blocks <= 0) return Status::ok();
  const dim3 g((unsigned)std::min<int64_t>(blocks, 16384)), b(256);
  if (acc == Acc::F32)
    return launch("bwd_reduce_table", k_bwd_reduce_table<float>, g, b, 0, s, descs, start, ndesc, blocks);
  return launch("bwd_reduce_table", k_bwd_reduce_table<double>, g, b, 0, s, descs, start, ndesc, blocks);
}

Status launch_bwd_prep(Acc acc, const BwdGatherDesc *descs, const int64_t *start, int ndesc, int64_t blocks,
                       unsigned long long *counters, int ncounters, hipStream_t s) {
  if (ncounters > 256) return Status::fail(CQC_ERR_UNSUPPORTED, "too many queue counters");
  const dim3 g((unsigned)std::max<int64_t>(1, std::min<int64_t>(blocks, 16384))), b(256);
  if (acc == Acc::F32)
    return launch("bwd_prep", k_bwd_prep<float>, g, b, 0, s, descs, start, ndesc, blocks, counters, ncounters);
  return launch("bwd_prep", k_bwd_prep<double>, g, b, 0, s, descs, start, ndesc, blocks, counters, ncounters);
}

template <typename T, typename O>
static Status launch_reduce_t(const void *part, int64_t count, int64_t P, double scale, void *out, hipStream_t s) {
  const T *pp = static_cast<const T *>(part);
  O *o = static_cast<O *>(out);
  const dim3 b(256);
  if (count < (int64_t(1) << 18) && P >= 16) {
    const dim3 g((unsigned)std::max<int64_t>(1, std::min<int64_t>((count + 31) / 32, 16384)));
    return launch("bwd_reduce", k_bwd_reduce<T, O, 8>, g, b, 0, s, pp, count, P, scale, o);
  }
  const dim3 g((unsigned)std::max<int64_t>(1, std::min<int64_t>((count + 255) / 256, 16384)));
  return launch("bwd_reduce", k_bwd_reduce<T, O, 1>, g, b, 0, s, pp, count, P, scale, o);
}

Status launch_bwd_reduce(Acc acc, const void *part, int64_t count, int64_t P, double scale,
                         void *out, bool out_double, hipStream_t s) {
  if (acc == Acc::F32)
    return out_double ? launch_reduce_t<float, double>(part, count, P, scale, out, s)
                      : launch_reduce_t<float, float>(part, count, P, scale, out, s);
  return out_double ? launch_reduce_t<double, double>(part, count, P, scale, out, s)
                    : launch_reduce_t<double, float>(part, count, P, scale, out, s);
}

Status launch_gather_blocked(Acc acc, const void *src, void *dst, int logM, int logN,
                             const BitPos &px, const BitPos &py, hipStream_t s) {
  const int64_t total = int64_t(1) << (logM + logN);
  const dim3 g((unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 16384))), b(256);
  if (acc == Acc::F32)
    return launch("gather_blocked", k_gather_blocked<float>, g, b, 0, s, static_cast<const float *>(src),
                  static_cast<float *>(dst), logM, logN, px, py);
  return launch("gather_blocked", k_gather_blocked<double>, g, b, 0, s, static_cast<const double *>(src),
                static_cast<double *>(dst), logM, logN, px, py);
}

}  // namespace cqc
