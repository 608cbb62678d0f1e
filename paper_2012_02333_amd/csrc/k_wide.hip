// Wide contraction kernel: LDS-staged operands for steps whose term sums are
// long enough to make the step compute-bound (many shared cut labels), in two
// arithmetic forms of the same tile program.
//
//   FP32    float operands on v_mfma_f32_32x32x2f32, FP32 accumulation (on
//           this part it sustains about 20% more than the 16x16x4 form).
//   BF16X6  every float operand a is split into three bfloat16 parts
//           a = a0 + a1 + a2 (a0 = a rounded to bfloat16, a1 = the remainder
//           rounded, a2 = the next remainder rounded; the remainders are exact
//           in FP32, so the three parts carry 24 significand bits), and the six
//           products a_i b_j with i + j <= 2 are accumulated in FP32 by
//           v_mfma_f32_16x16x32_bf16, smallest first.  The three dropped
//           products are below 2^-24 of |a b|, so the result keeps FP32
//           accuracy at the bfloat16 matrix-core rate (6 products at 16x the
//           FP32 rate: 2.7x the FP32 form's arithmetic throughput).
//   BF16X3  two parts a = a0 + a1 (16 significand bits) and the three products
//           a_i b_j with i + j <= 1, smallest first: half the BF16X6 matrix-core
//           work, with the dropped part and product up to 2^-15 of
//           |a b| per product - the speed end of the same split.
//
// A label-list pass first compacts, for every batch entry of the step, the
// live terms (both operand rows non-zero: early termination, Section 4.2) in
// ascending label order into the workspace.  The contraction itself runs on
// persistent blocks of four waves (2 x 2), each owning a 128 x 128 output tile
// at a time and walking a sequence of tiles (a contiguous range per XCD, so
// the tiles that share operand columns share an L2; or an atomic work queue
// over many steps).  Terms are consumed 32 at a time: each wave loads 16 terms
// of one operand, each lane two adjacent columns of them, two chunks ahead -
// across tile boundaries, so the next tile's first operands are in flight
// while the current tile computes and stores - and writes them to LDS with
// the term index fastest, so that each lane fetches a whole matrix-core
// operand with one 16-byte LDS read.  The epilogue stages each 16-row slice of
// a wave tile through LDS and writes whole 256-byte row segments.
#include <algorithm>
#include <map>
#include <mutex>
#include <type_traits>

#include "kdev.hpp"

namespace cqc {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

namespace {
constexpr int kWB = 128;        // block tile edge (m and n)
constexpr int kWT = 64;         // wave tile edge
constexpr int kWC = 32;         // terms per staged chunk
constexpr int kF32Ld = 36;      // floats per LDS operand column (FP32 form): 32 terms + pad
constexpr int kB16Ld = 40;      // bfloat16 per LDS operand column and part (BF16X6 form)
constexpr int kStLd = kWT + 4;  // floats per row of an epilogue staging slice
}  // namespace

// a = h + m (+ l) with each part the round-to-nearest bfloat16 of what is left.
__device__ __forceinline__ void split3(float a, __bf16 *h, __bf16 *m, __bf16 *l) {
  const __bf16 p0 = (__bf16)a;
  const float r1 = a - (float)p0;
  const __bf16 p1 = (__bf16)r1;
  const float r2 = r1 - (float)p1;
  *h = p0;
  *m = p1;
  *l = (__bf16)r2;
}

// ---- label lists: one block per batch entry of a step; per batch entry the
// byte offsets of the live terms' X rows, then of their Y rows (operands hold
// at most 2^30 elements)
__device__ __forceinline__ void label_list(const ContractArgs &a, int64_t batch) {
  __shared__ int wcnt[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rX = (int)(batch >> (2 * a.nRY));
  const int rY = (int)(batch & ((int64_t(1) << (2 * a.nRY)) - 1));
  uint32_t *Lx = reinterpret_cast<uint32_t *>(a.lists) + batch * 2 * a.list_ld;   // X row offsets
  uint32_t *Ly = Lx + a.list_ld;                                                     // Y row offsets
  const int nSv = 1 << (2 * a.nS);
  int total = 0;
  for (int s0 = 0; s0 < nSv; s0 += 256) {
    const int s = s0 + tid;
    int live = 0, rx = 0, ry = 0;
    if (s < nSv) {
      rx = row_of(a.mx, s, rX);
      ry = row_of(a.my, s, rY);
      // without row flags (plans whose other steps need none) every term is live
      live = a.flagX ? row_live(a.flagX, a.nchX, rx) & row_live(a.flagY, a.nchY, ry) : 1;
    }
    const unsigned long long bal = __ballot(live);
    const int pre = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wcnt[wave] = __popcll(bal);
    __syncthreads();
    int base = 0;
    for (int w = 0; w < wave; ++w) base += wcnt[w];
    const int cnt = wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
    if (live) {
      Lx[total + base + pre] = (uint32_t)rx << (a.logM + 2);
      Ly[total + base + pre] = (uint32_t)ry << (a.logN + 2);
    }
    total += cnt;
    __syncthreads();   // wcnt is rewritten by the next chunk
  }
  // pad to whole chunks (one chunk of padding if nothing is live) with row 0
  // (a valid address; the terms are masked by the count)
  const int padded = total == 0 ? kWC : (total + kWC - 1) / kWC * kWC;
  for (int k = total + tid; k < padded; k += 256) Lx[k] = Ly[k] = 0u;
  if (tid == 0) {
    a.counts[batch] = total;
    if (a.flagZ) a.flagZ[batch] = total > 0;
  }
}

__global__ __launch_bounds__(256) void k_label_list(const ContractArgs a) {
  if (gated_off(a.gate, a.gate_val)) return;
  label_list(a, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_label_list_table(const ContractArgs *descs, const int64_t *bprefix,
                                                          int ndesc) {
  const int d = find_desc(bprefix, ndesc, blockIdx.x);
  label_list(descs[d], (int64_t)blockIdx.x - bprefix[d]);
}

// Values the compiler cannot prove wave-uniform (loaded through pointers the
// kernel could in principle write) moved to scalar registers.
__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni(int64_t v) {
  return (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int32_t)(uint32_t)v) |
         ((int64_t)__builtin_amdgcn_readfirstlane((int32_t)(v >> 32)) << 32);
}
template <typename T> __device__ __forceinline__ T *uni(T *p) {
  return reinterpret_cast<T *>(uni((int64_t)reinterpret_cast<uintptr_t>(p)));
}
__device__ __forceinline__ double uni(double v) { return __builtin_bit_cast(double, uni(__builtin_bit_cast(int64_t, v))); }
// Global-address-space view of a pointer (a pointer that went through an
// integer is generic to the compiler, which would emit flat accesses).
template <typename T> using gptr = __attribute__((address_space(1))) T *;
template <typename T> __device__ __forceinline__ gptr<T> gbl(T *p) { return (gptr<T>)p; }
// Constant-address-space view of data that no wave writes during the kernel
// (label lists and counts, written by the preceding label-list pass): uniform
// loads through it become scalar loads, which are waited for on the scalar
// counter - not behind this wave's outstanding output stores.
template <typename T> using cptr = __attribute__((address_space(4))) const T *;
template <typename T> __device__ __forceinline__ cptr<T> cst(const T *p) { return (cptr<T>)gbl(p); }

// ---- a tile of a step: its block index and chunk count; the geometry is
// recomputed from the step's arguments where it is needed (few scalars live)
struct WideTile {
  uint32_t blk;
  int nch;   // chunks of kWC terms (at least one)
  int cnt;   // live terms
  int d;     // step of the tile (work-queue launches; 0 otherwise)
};

struct WideGeom {
  int64_t M, N, m0, n0, batch;
  int logM, logN;
};

__device__ __forceinline__ WideGeom wide_geom(const ContractArgs &a, uint32_t blk) {
  WideGeom g;
  const uint32_t tilesN = (uint32_t)uni(a.tilesN);
  const uint32_t tiles = (uint32_t)uni(a.tilesM) * tilesN;
  const uint32_t batch = blk / tiles;
  const uint32_t r = blk - batch * tiles;
  const uint32_t tm = r / tilesN, tn = r - tm * tilesN;
  g.logM = uni(a.logM);
  g.logN = uni(a.logN);
  g.M = int64_t(1) << g.logM;
  g.N = int64_t(1) << g.logN;
  g.m0 = (int64_t)tm * kWB;
  g.n0 = (int64_t)tn * kWB;
  g.batch = batch;
  return g;
}

__device__ __forceinline__ WideTile wide_decode(const ContractArgs &a, uint32_t blk) {
  const WideGeom g = wide_geom(a, blk);
  const int cnt = cst(uni(a.counts))[g.batch];
  return WideTile{blk, cnt == 0 ? 1 : (cnt + kWC - 1) / kWC, cnt, 0};
}

// Tile sequences of a block.  Strided: one step, tiles of a contiguous range
// per XCD (hardware places block b on XCD b % 8).  Queue: many steps; a new
// tile is fetched by thread 0 into one of two LDS slots (alternating) before a
// barrier, and decoded by every thread after it.
struct StridedSeq {
  const ContractArgs &a;
  int64_t pos, end, stride;
  __device__ StridedSeq(const ContractArgs &args) : a(args) {
    const int64_t T = a.nblocks, G = gridDim.x, b = blockIdx.x;
    if (a.xcd_remap && G % 8 == 0 && T % 8 == 0 && G <= T) {
      const int64_t per = T / 8;
      pos = (b % 8) * per + b / 8;
      end = (b % 8) * per + per;
      stride = G / 8;
    } else {
      pos = b;
      end = T;
      stride = G;
    }
  }
  __device__ bool first(WideTile *t) {
    if (pos >= end) return false;
    *t = wide_decode(a, (uint32_t)pos);
    return true;
  }
  __device__ void fetch(int) {}
  __device__ bool next(WideTile *t, int) {
    pos += stride;
    if (pos >= end) return false;
    *t = wide_decode(a, (uint32_t)pos);
    return true;
  }
  __device__ const ContractArgs &args(const WideTile &) const { return a; }
};

struct QueueSeq {
  const ContractArgs *descs;
  const int64_t *prefix;
  int ndesc;
  unsigned long long *queue;
  int64_t total;
  int64_t *slot;    // [2] fetched queue items, in LDS
  __device__ int64_t read_slot(int sp) const {
    const int64_t v = slot[sp];
    return (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v) |
           ((int64_t)__builtin_amdgcn_readfirstlane((int)(v >> 32)) << 32);
  }
  __device__ bool decode_item(int64_t item, WideTile *t) {
    if (item >= total) return false;
    const int d = uni(find_desc(prefix, ndesc, item));
    *t = wide_decode(descs[d], (uint32_t)(item - uni(prefix[d])));
    t->d = d;
    return true;
  }
  __device__ bool first(WideTile *t) {
    if (threadIdx.x == 0) slot[0] = (int64_t)atomicAdd(queue, 1ull);
    __syncthreads();
    return decode_item(read_slot(0), t);
  }
  // by every thread, before the barrier that precedes next(sp)
  __device__ void fetch(int sp) {
    if (threadIdx.x == 0) slot[sp] = (int64_t)atomicAdd(queue, 1ull);
  }
  __device__ bool next(WideTile *t, int sp) { return decode_item(read_slot(sp), t); }
  __device__ const ContractArgs &args(const WideTile &t) const { return descs[t.d]; }
};

// NP: bfloat16 parts per operand (3: BF16X6, 2: BF16X3), 0 for the FP32 form.
// PS (split forms): the operands come already split into bfloat16 part planes
// (ContractArgs::Xs, Ys), so staging only repacks them; otherwise every tile
// splits the FP32 operands it stages.
// XE: final steps of the cross-entropy form (ContractArgs::xt): 1 gradient,
// 2 gradient and loss.
template <int NP, typename O, int MODE, bool PS, int XE, class Seq>
__device__ __forceinline__ void wide_run(Seq &seq) {
  static_assert(!PS || NP > 0, "pre-split operands are for the split forms");
  static_assert(NP == 0 || NP == 2 || NP == 3, "FP32, BF16X3 or BF16X6");
  // operand staging area: FP32 [256 columns][kF32Ld]; split forms [NP parts][256][kB16Ld]
  constexpr int kOpBytes = NP ? NP * 2 * kWB * kB16Ld * 2 : 2 * kWB * kF32Ld * 4;
  static_assert(kOpBytes >= 4 * 16 * kStLd * 4, "epilogue staging fits in the operand area");
  static_assert(NP != 0 || kOpBytes >= 4 * 32 * kStLd * 4, "32-row staging slices fit in the operand area");
  __shared__ __attribute__((aligned(16))) unsigned char smem[kOpBytes];
  __shared__ int64_t rowoff[MODE == kModeFinalDeposit ? kWB : 1];
  __shared__ int64_t coloff[MODE == kModeFinalDeposit ? kWB : 1];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int l16 = lane & 15, lg = lane >> 4;
  // staging role of the wave (wave-uniform): waves 0 and 2 stage X, 1 and 3
  // stage Y; waves 0 and 1 the first 16 terms of a chunk, 2 and 3 the last 16;
  // lane l owns the two adjacent operand columns 2l and 2l + 1 of the tile
  const int wv = uni(wave);
  const bool roleX = (wv & 1) == 0;
  const int half = wv >> 1;

  // accumulators: split forms 4 x 4 blocks of 16 x 16 (f32x4 per lane); the
  // FP32 form 2 x 2 blocks of 32 x 32 (f32x16 per lane: lane l, register r
  // holds row n = (r % 4) + 8 (r / 4) + 4 (l / 32), column m = l % 32)
  f32x4 acc[4][4];
  f32x16 acc2[2][2];
  auto zero_acc = [&]() {
    if constexpr (NP == 0) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int r = 0; r < 16; ++r) acc2[i][j][r] = 0.f;
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
  };
  zero_acc();

  // Branch-free prefetch: every lane loads (padding and overhanging columns
  // read element 0), so all kWC loads of a chunk are in flight together; the
  // invalid ones are zeroed only when the chunk is written to LDS.
  constexpr int kH = kWC / 2;      // terms per staging wave and chunk
  float pre[2][PS ? 1 : kH][2];
  uint32_t pre16[2][PS ? kH : 1][PS ? NP : 1];   // pre-split: parts of the lane's two columns, per term
  uint32_t okrow[2] = {0u, 0u};    // wave-uniform: term k of this wave's half is live
  bool colok[2][2] = {{true, true}, {true, true}};   // this lane's two columns lie inside the operand
  auto gload = [&](auto B, const ContractArgs &a, const WideTile &t, int ch) {
    constexpr int b = decltype(B)::value;
    const WideGeom g = wide_geom(a, t.blk);
    // the row offsets of this wave's terms come in by scalar loads; each load
    // is a scalar base plus a 32-bit lane offset and fetches two columns
    // (one wave instruction: 512 contiguous bytes of an operand row)
    const int32_t ld32 = uni(a.list_ld);
    const cptr<uint32_t> offs = cst(reinterpret_cast<const uint32_t *>(uni(a.lists))) +
                                (g.batch * 2 + (roleX ? 0 : 1)) * ld32 + ch * kWC + half * kH;
    const char *srcb = reinterpret_cast<const char *>(roleX ? uni(a.X) : uni(a.Y));
    const int64_t ld = roleX ? g.M : g.N;
    const int64_t colv = (roleX ? g.m0 : g.n0) + 2 * lane;
    colok[b][0] = colv < ld;
    colok[b][1] = colv + 1 < ld;
    const int nv = t.cnt - ch * kWC - half * kH;   // live terms of this wave's half (uniform)
    okrow[b] = nv >= kH ? 0xffffu : (nv <= 0 ? 0u : (1u << nv) - 1u);
    // ld is a power of two >= 2 (steps with a one-column operand do not run
    // here): both columns are inside or both outside
    if constexpr (PS) {
      // part p of the two columns: 4 bytes at plane p, row offset / 2 (the
      // list holds FP32 byte offsets)
      const char *pb = reinterpret_cast<const char *>(roleX ? uni(a.Xs) : uni(a.Ys));
      const int64_t plane2 = 2 * (roleX ? uni(a.xplane) : uni(a.yplane));
      const uint32_t col2 = colok[b][1] ? (uint32_t)colv * 2u : 0u;
#pragma unroll
      for (int k = 0; k < kH; ++k)
#pragma unroll
        for (int p = 0; p < NP; ++p)
          pre16[b][k][p] = *(gptr<const uint32_t>)(gbl(pb) + p * plane2 + ((offs[k] >> 1) + col2));
    } else {
      const uint32_t col4 = colok[b][1] ? (uint32_t)colv * 4u : 0u;
#pragma unroll
      for (int k = 0; k < kH; ++k) {
        const f32x2 v = *(gptr<const f32x2>)(gbl(srcb) + (offs[k] + col4));
        pre[b][k][0] = v[0];
        pre[b][k][1] = v[1];
      }
    }
  };
  auto stage = [&](auto B) {
    constexpr int b = decltype(B)::value;
    auto val = [&](int k, int j) { return (colok[b][j] && ((okrow[b] >> k) & 1u)) ? pre[b][k][j] : 0.0f; };
    const int col0 = (roleX ? 0 : kWB) + 2 * lane;   // first of this lane's two LDS operand columns
    if constexpr (NP == 0) {
      // term 2 s + h of an 8-term group sits at 4 h + s, so the half-wave h of
      // a 32 x 32 x 2 product reads its terms {h, h+2, h+4, h+6} of the group
      // at once; this wave's 16 terms are groups 2 half and 2 half + 1
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        float *cp = reinterpret_cast<float *>(smem) + (col0 + j) * kF32Ld + 16 * half;
#pragma unroll
        for (int g8 = 0; g8 < 2; ++g8)
#pragma unroll
          for (int h = 0; h < 2; ++h)
            *reinterpret_cast<float4 *>(cp + 8 * g8 + 4 * h) =
                make_float4(val(8 * g8 + h, j), val(8 * g8 + 2 + h, j), val(8 * g8 + 4 + h, j), val(8 * g8 + 6 + h, j));
      }
    } else if constexpr (PS) {
      // repack: the 8 terms of column j of one part, two terms per 32 bits
      // (low half = column 2 lane, high half = column 2 lane + 1 in the
      // loaded words); dead terms and outside columns give zeros
      __bf16 *bp = reinterpret_cast<__bf16 *>(smem);
      auto w = [&](int k, int p) -> uint32_t {
        return (colok[b][0] && ((okrow[b] >> k) & 1u)) ? pre16[b][k][p] : 0u;
      };
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int o = 0; o < 2; ++o) {
          const int pos = 16 * half + 8 * o;
#pragma unroll
          for (int p = 0; p < NP; ++p) {
            uint32_t q[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const uint32_t lo = w(8 * o + 2 * u, p), hi = w(8 * o + 2 * u + 1, p);
              q[u] = j == 0 ? ((lo & 0xffffu) | (hi << 16)) : ((lo >> 16) | (hi & 0xffff0000u));
            }
            *reinterpret_cast<uint4 *>(bp + (p * 2 * kWB + col0 + j) * kB16Ld + pos) = make_uint4(q[0], q[1], q[2], q[3]);
          }
        }
    } else {
      __bf16 *bp = reinterpret_cast<__bf16 *>(smem);
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int o = 0; o < 2; ++o) {
          bf16x8 h, m, l;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            __bf16 x0, x1, x2;
            split3(val(8 * o + e, j), &x0, &x1, &x2);
            h[e] = x0;
            m[e] = x1;
            l[e] = x2;
          }
          const int pos = 16 * half + 8 * o;
          *reinterpret_cast<bf16x8 *>(bp + (0 * 2 * kWB + col0 + j) * kB16Ld + pos) = h;
          *reinterpret_cast<bf16x8 *>(bp + (1 * 2 * kWB + col0 + j) * kB16Ld + pos) = m;
          if constexpr (NP == 3) *reinterpret_cast<bf16x8 *>(bp + (2 * 2 * kWB + col0 + j) * kB16Ld + pos) = l;
        }
    }
  };
  // MFMA mapping: A operand = Y (MFMA row <-> n), B operand = X (MFMA column
  // <-> m), so lane (l16, lg) accumulates 4 consecutive n of output row l16.
  auto compute = [&]() {
    if constexpr (NP == 0) {
      // lane (i = l % 32, h = l / 32) feeds operand row/column i and term
      // 2 s + h of each 8-term group to the s-th product of the group
      const int i32 = lane & 31, h = lane >> 5;
      const float *px = reinterpret_cast<const float *>(smem) + (wm * kWT + i32) * kF32Ld + 4 * h;
      const float *py = reinterpret_cast<const float *>(smem) + (kWB + wn * kWT + i32) * kF32Ld + 4 * h;
#pragma unroll
      for (int g = 0; g < kWC / 8; ++g) {
        float xa[2][4], yb[2][4];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const float4 v = *reinterpret_cast<const float4 *>(px + b * 32 * kF32Ld + 8 * g);
          xa[b][0] = v.x; xa[b][1] = v.y; xa[b][2] = v.z; xa[b][3] = v.w;
          const float4 w = *reinterpret_cast<const float4 *>(py + b * 32 * kF32Ld + 8 * g);
          yb[b][0] = w.x; yb[b][1] = w.y; yb[b][2] = w.z; yb[b][3] = w.w;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
              acc2[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(yb[j][q], xa[i][q], acc2[i][j], 0, 0, 0);
      }
    } else {
      const __bf16 *bp = reinterpret_cast<const __bf16 *>(smem);
      bf16x8 xv[4][NP];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int p = 0; p < NP; ++p)
          xv[i][p] = *reinterpret_cast<const bf16x8 *>(bp + (p * 2 * kWB + wm * kWT + i * 16 + l16) * kB16Ld + 8 * lg);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        bf16x8 yv[NP];
#pragma unroll
        for (int p = 0; p < NP; ++p)
          yv[p] = *reinterpret_cast<const bf16x8 *>(bp + (p * 2 * kWB + kWB + wn * kWT + j * 16 + l16) * kB16Ld +
                                                    8 * lg);
        // (part of Y, part of X) for the six (three) products, smallest first
        if constexpr (NP == 3) {
#pragma unroll
          for (int i = 0; i < 4; ++i) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yv[0], xv[i][NP - 1], acc[i][j], 0, 0, 0);
#pragma unroll
          for (int i = 0; i < 4; ++i) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yv[NP - 1], xv[i][0], acc[i][j], 0, 0, 0);
#pragma unroll
          for (int i = 0; i < 4; ++i) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yv[1], xv[i][1], acc[i][j], 0, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yv[0], xv[i][1], acc[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yv[1], xv[i][0], acc[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yv[0], xv[i][0], acc[i][j], 0, 0, 0);
      }
    }
  };
  // Writes the finished tile (all threads; the operand area is free).
  auto epilogue = [&](const ContractArgs &a, const WideTile &t) {
    const WideGeom g = wide_geom(a, t.blk);
    const int64_t M = g.M, N = g.N;
    if (MODE == kModeFinalDeposit) {
      if (tid < kWB) rowoff[tid] = g.m0 + tid < M ? deposit(g.m0 + tid, a.posX, g.logM) : 0;
      else coloff[tid - kWB] = g.n0 + (tid - kWB) < N ? deposit(g.n0 + (tid - kWB), a.posY, g.logN) : 0;
      __syncthreads();
    }
    double msum = 0.0;
    const int64_t mw = g.m0 + wm * kWT, nw = g.n0 + wn * kWT;
    const gptr<O> Zb = gbl(uni(static_cast<O *>(a.Z))) + (MODE == kModeIntermediate ? g.batch * M * N : 0);
    constexpr bool kStage = sizeof(O) == 4 && MODE != kModeFinalDeposit;
    // cross-entropy form: the targets of the whole wave tile (64 rows, in the
    // staged stores' layout: row 4 q + lane / 16, columns 4 (lane % 16) + 0..3)
    // are loaded before its first store (see xent_emit4)
    constexpr bool kPre = XE && MODE == kModeFinalBlocked && kStage;
    const bool pre = kPre && mw + kWT <= M && nw + kWT <= N;
    f32x4 tv[kPre ? 16 : 1];
    const gptr<float> XT = gbl(uni(static_cast<float *>(const_cast<void *>(a.xt))));
    const gptr<float> XG = gbl(uni(static_cast<float *>(a.xg)));
    const gptr<float> XZ = gbl(uni(static_cast<float *>(a.Z)));
    constexpr bool xloss = XE == 2;
    if constexpr (kPre) {
      if (pre)
#pragma unroll
        for (int q = 0; q < 16; ++q)
          tv[q] = __builtin_nontemporal_load((gptr<f32x4>)(XT + (mw + 4 * q + lg) * N + nw + 4 * l16));
    }
    const double sc64 = uni(a.scale);
    const float scf = MODE == kModeIntermediate ? 1.0f : (float)sc64;
    const O scale = (O)sc64;
    // a run of 4 consecutive n of output row m, written element-wise (edge
    // tiles, FP64 output, bit-deposit order)
    auto write_run = [&](int64_t m, int64_t n, const f32x4 &vals) {
      if (m >= M || n >= N) return;
      if (MODE == kModeIntermediate) {
        const gptr<float> Z = (gptr<float>)Zb + m * N + n;
        if (n + 3 < N) *(gptr<f32x4>)Z = vals;
        else
          for (int r = 0; r < 4; ++r)
            if (n + r < N) Z[r] = vals[r];
      } else {
        O v[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = (O)vals[r] * scale;
        if constexpr (XE) {
          for (int r = 0; r < 4; ++r)
            if (n + r < N)
              msum += xent_put1<O>(a, MODE == kModeFinalBlocked ? m * N + n + r
                                                               : rowoff[m - g.m0] + coloff[n + r - g.n0],
                                   v[r], XE == 2);
        } else {
          if (MODE == kModeFinalBlocked) {
            const gptr<O> Z = Zb + m * N + n;
            for (int r = 0; r < 4; ++r)
              if (n + r < N) Z[r] = v[r];
          } else {
            const int64_t ro = rowoff[m - g.m0];
            for (int r = 0; r < 4; ++r)
              if (n + r < N) Zb[ro + coloff[n + r - g.n0]] = v[r];
          }
          for (int r = 0; r < 4; ++r)
            if (n + r < N) msum += (double)v[r];
        }
      }
    };
    // a staged slice of `rows` output rows x 64 columns (this wave's LDS
    // slice, already written): 16 lanes per 64-float row, 4 rows per store
    // instruction.  The stores are non-temporal: the output is written once
    // and never read here, so it should not evict the operands from L2
    // (measured 5% faster for BF16X6, and the L2 holds fewer dirty lines at
    // the end)
    auto store_slice = [&](const float *st, auto rows_c, int64_t m0) {
      constexpr int rows = decltype(rows_c)::value;
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
#pragma unroll
      for (int rr = 0; rr < rows; rr += 4) {
        const int row = rr + lg, c4 = l16 * 4;
        const float4 v = *reinterpret_cast<const float4 *>(st + row * kStLd + c4);
        if constexpr (XE) {
          const float w[4] = {v.x, v.y, v.z, v.w};
          const int64_t o = (m0 + row) * N + nw + c4;
          double c[4];
          if (pre) {
            const f32x4 t = tv[kPre ? (int)((m0 - mw) / 4) + rr / 4 : 0];
            if (XZ) *(gptr<f32x4>)(XZ + o) = f32x4{w[0], w[1], w[2], w[3]};
            f32x4 gv;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              gv[r] = xent_grad_of(w[r], t[r]);
              c[r] = xent_part(w[r], t[r], xloss);
            }
            __builtin_nontemporal_store(gv, (gptr<f32x4>)(XG + o));
          } else {
            xent_put4<float>(a, o, w, c, xloss);
          }
          msum += (c[0] + c[1]) + (c[2] + c[3]);
        } else {
          __builtin_nontemporal_store(f32x4{v.x, v.y, v.z, v.w},
                                      (gptr<f32x4>)((gptr<float>)Zb + (m0 + row) * N + nw + c4));
          if (MODE != kModeIntermediate) msum += ((double)v.x + (double)v.y) + ((double)v.z + (double)v.w);
        }
      }
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    };
    if constexpr (NP == 0) {
      // 32 x 32 blocks: lane l holds, for output row m = mb + l % 32, the runs
      // n = 32 bj + 8 q + 4 (l / 32) + {0..3} in registers 4 q .. 4 q + 3
      const int i32 = lane & 31, h = lane >> 5;
#pragma unroll
      for (int bi = 0; bi < 2; ++bi) {
        const int64_t mb = mw + bi * 32;
        if (kStage && mb + 32 <= M && nw + kWT <= N) {
          float *st = reinterpret_cast<float *>(smem) + wave * 32 * kStLd;
#pragma unroll
          for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int q = 0; q < 4; ++q)
              *reinterpret_cast<float4 *>(st + i32 * kStLd + bj * 32 + 8 * q + 4 * h) =
                  make_float4(acc2[bi][bj][4 * q] * scf, acc2[bi][bj][4 * q + 1] * scf,
                              acc2[bi][bj][4 * q + 2] * scf, acc2[bi][bj][4 * q + 3] * scf);
          store_slice(st, std::integral_constant<int, 32>{}, mb);
          continue;
        }
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
          for (int q = 0; q < 4; ++q)
            write_run(mb + i32, nw + bj * 32 + 8 * q + 4 * h,
                      f32x4{acc2[bi][bj][4 * q], acc2[bi][bj][4 * q + 1], acc2[bi][bj][4 * q + 2],
                            acc2[bi][bj][4 * q + 3]});
      }
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (kStage && mw + i * 16 + 16 <= M && nw + kWT <= N) {
          float *st = reinterpret_cast<float *>(smem) + wave * 16 * kStLd;
#pragma unroll
          for (int j = 0; j < 4; ++j)
            *reinterpret_cast<float4 *>(st + l16 * kStLd + j * 16 + 4 * lg) =
                make_float4(acc[i][j][0] * scf, acc[i][j][1] * scf, acc[i][j][2] * scf, acc[i][j][3] * scf);
          store_slice(st, std::integral_constant<int, 16>{}, mw + i * 16);
          continue;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) write_run(mw + i * 16 + l16, nw + j * 16 + 4 * lg, acc[i][j]);
      }
    }
    double *partials = uni(a.partials);
    if (MODE != kModeIntermediate && partials) {
      const double tot = wave_sum_f64(msum);
      if (lane == 0) gbl(partials)[kPartialsPerTile * t.blk + wave] = tot;
    }
  };

  // ---- the pipelined item sequence.  An item is (tile, chunk); the operands
  // of item q+2 are loaded while item q is on the matrix cores, into the
  // register set item q has just left.  Loads are issued on every item (a
  // repeat of the current item's past the end of the sequence), so the wait
  // for an item's operands always has the next item's loads and a whole item
  // of matrix-core work after it - any output stores of the tile before have
  // drained by then, instead of being waited for (loads and stores share one
  // in-order completion counter).
  struct Item { WideTile t; int c; bool ok; };
  Item q0;
  if (!seq.first(&q0.t)) return;
  q0.c = 0;
  q0.ok = true;
  int sp = 1;   // next fetch slot (the first tile came through slot 0)
  auto item_args = [&](const Item &x) -> const ContractArgs & { return seq.args(x.t); };
  gload(std::integral_constant<int, 0>{}, item_args(q0), q0.t, 0);
  Item q1 = q0;
  if (q1.c + 1 < q1.t.nch) {
    ++q1.c;
  } else {
    seq.fetch(sp);
    __syncthreads();
    q1.ok = seq.next(&q1.t, sp);
    sp ^= 1;
    q1.c = 0;
  }
  {
    const WideTile lt = q1.ok ? q1.t : q0.t;   // one load site (a repeat past the end)
    gload(std::integral_constant<int, 1>{}, seq.args(lt), lt, q1.ok ? q1.c : q0.c);
  }
  Item q2 = q1;   // advanced to item q+2 inside each step
  // Items are taken in pairs (register set 0, then 1) and the sequence may
  // only end after the second: a block with an odd item count finishes with
  // an empty item (q0.ok false) that loads a repeat and computes nothing.
  // An exit after the first would join the loop header on a path where only
  // set 0's loads are in flight, and the compiler would then drain every load
  // before staging set 0 on every iteration.
  auto step = [&](auto B) -> bool {
    // advancing q2 starts a new tile: fetch it before the barrier
    const bool new_tile = q2.ok && q2.c + 1 == q2.t.nch;
    if (new_tile) seq.fetch(sp);
    __syncthreads();   // the operand area (and staging slices) are free
    stage(B);
    __syncthreads();
    if (q2.ok) {
      if (new_tile) {
        q2.ok = seq.next(&q2.t, sp);
        sp ^= 1;
        q2.c = 0;
      } else {
        ++q2.c;
      }
    }
    const WideTile lt = q2.ok ? q2.t : q0.t;     // one load site (a repeat past the end)
    gload(B, seq.args(lt), lt, q2.ok ? q2.c : q0.c);
    if (q0.ok) compute();
    if (q0.ok && q0.c == q0.t.nch - 1) {
      __syncthreads();   // every wave is done reading operands: stage the outputs
      epilogue(item_args(q0), q0.t);
      zero_acc();
    }
    if (decltype(B)::value == 1 && !q1.ok) return false;
    if (q1.ok) q0 = q1;
    else q0.ok = false;   // keeps the last real tile for the empty item's loads
    q1 = q2;
    return true;
  };
  for (;;) {
    step(std::integral_constant<int, 0>{});
    if (!step(std::integral_constant<int, 1>{})) break;
  }
}

// Occupancy target: two blocks per CU (8 waves).  Three FP32 blocks would fit
// the LDS but not the registers without spilling, and measure slower.
template <int NP> struct WideOcc { static constexpr int kWaves = 2; };

template <int NP, typename O, int MODE, bool PS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WideOcc<NP>::kWaves, WideOcc<NP>::kWaves)))
void k_wide(const ContractArgs a) {
  if (gated_off(a.gate, a.gate_val)) return;
  StridedSeq seq(a);
  wide_run<NP, O, MODE, PS, 0>(seq);
}

template <int NP, int MODE, int XE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WideOcc<NP>::kWaves, WideOcc<NP>::kWaves)))
void k_wide_queue(const ContractArgs *__restrict__ descs,
                                                    const int64_t *__restrict__ prefix, int ndesc,
                                                    unsigned long long *queue, int64_t total) {
  __shared__ int64_t slot[2];
  QueueSeq seq{descs, prefix, ndesc, queue, total, slot};
  wide_run<NP, float, MODE, false, XE>(seq);
}

// The split of the wide kernel's staging (split3), once per operand element:
// part p of element i at dst[p * plane + i].  Four elements per thread.
template <int NP, bool VEC>
__global__ __launch_bounds__(256) void k_presplit(const float *src, __bf16 *dst, int64_t count, int64_t plane) {
  const int64_t n4 = count >> 2;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x) {
    float v[4];
    if constexpr (VEC) {
      const float4 q = reinterpret_cast<const float4 *>(src)[i];
      v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] = src[4 * i + e];
    }
    __bf16 part[3][4];
#pragma unroll
    for (int e = 0; e < 4; ++e) split3(v[e], &part[0][e], &part[1][e], &part[2][e]);
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
      bf16x4 o;
#pragma unroll
      for (int e = 0; e < 4; ++e) o[e] = part[p][e];
      *reinterpret_cast<bf16x4 *>(dst + p * plane + 4 * i) = o;
    }
  }
}
// ---------------------------------------------------------------------------
bool wide_fits(const ContractArgs &a) {
  const int64_t x = (int64_t)2 * (a.nS + a.nRX) + a.logM, y = (int64_t)2 * (a.nS + a.nRY) + a.logN;
  return x <= 30 && y <= 30 && a.logM >= 1 && a.logN >= 1;
}

// Blocks of a kernel that fit on the current device at once (cached).
static int64_t resident_blocks(const void *kernel) {
  static std::mutex mu;
  static std::map<std::pair<const void *, int>, int64_t> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  std::lock_guard<std::mutex> g(mu);
  auto it = cache.find({kernel, dev});
  if (it != cache.end()) return it->second;
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  const int64_t v = (int64_t)(per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
  cache[{kernel, dev}] = v;
  return v;
}

template <typename K>
static Status launch_persistent(const char *nm, K kernel, const ContractArgs &a, hipStream_t s) {
  int64_t G = resident_blocks(reinterpret_cast<const void *>(kernel));
  if (G <= 0) return Status::fail(CQC_ERR_HIP, "occupancy query failed");
  G = std::min<int64_t>(G, a.nblocks);
  if (G >= 8) G -= G % 8;   // whole per-XCD ranges
  return launch(nm, kernel, dim3((unsigned)G), dim3(256), 0, s, a);
}

template <int NP> struct WideNames;
template <> struct WideNames<0> {
  static constexpr const char *fin = "wide_f32_final", *mid = "wide_f32_inter", *queue = "wide_f32_queue",
                              *qx = "wide_f32_queue_xent";
};
template <> struct WideNames<2> {
  static constexpr const char *fin = "wide_bf16x3_final", *mid = "wide_bf16x3_inter", *queue = "wide_bf16x3_queue",
                              *qx = "wide_bf16x3_queue_xent";
};
template <> struct WideNames<3> {
  static constexpr const char *fin = "wide_bf16x6_final", *mid = "wide_bf16x6_inter", *queue = "wide_bf16x6_queue",
                              *qx = "wide_bf16x6_queue_xent";
};

template <int NP, typename O, bool PS>
static Status launch_wide_ps(const ContractArgs &a, hipStream_t s) {
  if (a.mode == kModeFinalBlocked) return launch_persistent(WideNames<NP>::fin, k_wide<NP, O, kModeFinalBlocked, PS>, a, s);
  if (a.mode == kModeFinalDeposit) return launch_persistent(WideNames<NP>::fin, k_wide<NP, O, kModeFinalDeposit, PS>, a, s);
  return launch_persistent(WideNames<NP>::mid, k_wide<NP, float, kModeIntermediate, PS>, a, s);
}

template <int NP, typename O>
static Status launch_wide_t(const ContractArgs &a, hipStream_t s) {
  CQC_TRY(launch("label_list", k_label_list, dim3((unsigned)a.nbatch), dim3(256), 0, s, a));
  if constexpr (NP > 0) {
    if (a.Xs && a.Ys) return launch_wide_ps<NP, O, true>(a, s);
  }
  return launch_wide_ps<NP, O, false>(a, s);
}

template <int NP>
static Status launch_wide_np(bool out_double, const ContractArgs &a, hipStream_t s) {
  return out_double ? launch_wide_t<NP, double>(a, s) : launch_wide_t<NP, float>(a, s);
}

Status launch_contract_wide(int parts, bool out_double, const ContractArgs &a, hipStream_t s) {
  if (!a.lists || !a.counts || a.nbatch < 1 || a.list_ld < wide_list_ld(a.nS))
    return Status::fail(CQC_ERR_INVALID_ARG, "wide contraction without label-list workspace");
  if (!wide_fits(a))
    return Status::fail(CQC_ERR_UNSUPPORTED, "wide contraction: an operand has one column or exceeds 2^30 elements");
  switch (parts) {
    case 0: return launch_wide_np<0>(out_double, a, s);
    case 2: return launch_wide_np<2>(out_double, a, s);
    case 3: return launch_wide_np<3>(out_double, a, s);
    default: return Status::fail(CQC_ERR_INVALID_ARG, "wide contraction: unknown operand split");
  }
}

Status launch_presplit(int parts, const float *src, void *dst, int64_t count, int64_t plane, hipStream_t s) {
  if (count % 4 || plane < count) return Status::fail(CQC_ERR_INVALID_ARG, "presplit: bad element count");
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((count / 4 + 255) / 256, 8192));
  const bool vec = (reinterpret_cast<uintptr_t>(src) & 15) == 0;
  __bf16 *d = static_cast<__bf16 *>(dst);
  const dim3 g((unsigned)blocks), b(256);
  switch (parts) {
    case 2: return vec ? launch("presplit", k_presplit<2, true>, g, b, 0, s, src, d, count, plane)
                       : launch("presplit", k_presplit<2, false>, g, b, 0, s, src, d, count, plane);
    case 3: return vec ? launch("presplit", k_presplit<3, true>, g, b, 0, s, src, d, count, plane)
                       : launch("presplit", k_presplit<3, false>, g, b, 0, s, src, d, count, plane);
    default: return Status::fail(CQC_ERR_INVALID_ARG, "presplit: parts must be 2 or 3");
  }
}

template <int NP>
static Status launch_wide_queue_t(int mode, const QueueLaunch &q, hipStream_t s) {
  const dim3 grid(q.grid), block(256);
  const char *nm = WideNames<NP>::queue;
  CQC_TRY(launch("label_list_table", k_label_list_table, dim3((unsigned)q.btotal), block, 0, s, q.descs, q.bprefix,
                 q.ndesc));
  const char *nx = WideNames<NP>::qx;
  if (mode != kModeIntermediate && q.xent) {
    if (mode == kModeFinalBlocked)
      return q.xent == 2 ? launch(nx, k_wide_queue<NP, kModeFinalBlocked, 2>, grid, block, 0, s, q.descs, q.prefix, q.ndesc, q.queue, q.total)
                         : launch(nx, k_wide_queue<NP, kModeFinalBlocked, 1>, grid, block, 0, s, q.descs, q.prefix, q.ndesc, q.queue, q.total);
    return q.xent == 2 ? launch(nx, k_wide_queue<NP, kModeFinalDeposit, 2>, grid, block, 0, s, q.descs, q.prefix, q.ndesc, q.queue, q.total)
                       : launch(nx, k_wide_queue<NP, kModeFinalDeposit, 1>, grid, block, 0, s, q.descs, q.prefix, q.ndesc, q.queue, q.total);
  }
  if (mode == kModeFinalBlocked)
    return launch(nm, k_wide_queue<NP, kModeFinalBlocked, 0>, grid, block, 0, s, q.descs, q.prefix, q.ndesc, q.queue, q.total);
  if (mode == kModeFinalDeposit)
    return launch(nm, k_wide_queue<NP, kModeFinalDeposit, 0>, grid, block, 0, s, q.descs, q.prefix, q.ndesc, q.queue, q.total);
  return launch(nm, k_wide_queue<NP, kModeIntermediate, 0>, grid, block, 0, s, q.descs, q.prefix, q.ndesc, q.queue, q.total);
}

Status launch_contract_wide_queue(int parts, int mode, const QueueLaunch &q, hipStream_t s) {
  if (!q.bprefix || q.btotal < 1) return Status::fail(CQC_ERR_INVALID_ARG, "wide queue without label-list table");
  switch (parts) {
    case 0: return launch_wide_queue_t<0>(mode, q, s);
    case 2: return launch_wide_queue_t<2>(mode, q, s);
    case 3: return launch_wide_queue_t<3>(mode, q, s);
    default: return Status::fail(CQC_ERR_INVALID_ARG, "wide queue: unknown operand split");
  }
}

}  // namespace cqc
