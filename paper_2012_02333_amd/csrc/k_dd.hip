// Dynamic-definition kernels (Algorithm 1, Section 4.3): merging subcircuit
// entries over their merged qubits, and selecting the heaviest bins.
#include "kdev.hpp"
#include "dd.hpp"

namespace cqc {

// E'_c[r][a] = sum_m E_c[r][dep(a, active) | zoom | dep(m, merged)], summed in
// FP64.  With >= 64 merged combinations one wave takes each (output, chunk of
// 2^kMergeLogChunk combinations): lanes strided over the chunk with eight
// accumulators each, combined in a fixed tree and a fixed butterfly; an
// output with one chunk is written directly, otherwise its chunk sums go to
// `part` and k_dd_merge_chunks adds them in chunk order.  With fewer merged
// combinations one thread takes each output, in ascending m.
template <typename I, typename O>
__global__ __launch_bounds__(256) void k_dd_merge(const MergeArgs a) {
  if (gated_off(a.gate, a.gate_val)) return;
  const int64_t bid = blockIdx.x;
  int i = 0;
  while (i + 1 < a.n && bid >= a.d[i + 1].block_start) ++i;
  const MergeDesc &d = a.d[i];
  const I *E = static_cast<const I *>(d.src);
  O *Out = static_cast<O *>(d.dst);
  const int64_t nout = d.rows << d.n_active;
  const int64_t nmerge = int64_t(1) << d.n_merged;
  const int64_t f = int64_t(1) << d.f;
  const int ash = d.active_shift, msh = d.merged_shift;
  const int64_t zoom = d.zoom_dev ? *d.zoom_dev : d.zoom_value;
  if (nmerge >= 64) {
    const int lc = d.log_chunks;
    const int64_t w = (bid - d.block_start) * 4 + (threadIdx.x >> 6);
    if (w >= (nout << lc)) return;
    const int64_t o = w >> lc, ch = w & ((int64_t(1) << lc) - 1);
    const int64_t clen = nmerge >> lc;
    const int lane = threadIdx.x & 63;
    const int64_t r = o >> d.n_active, av = o & ((int64_t(1) << d.n_active) - 1);
    const int64_t base = (ash >= 0 ? av << ash : deposit(av, d.active_pos, d.n_active)) | zoom;
    const I *row = E + r * f;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int64_t m1 = (ch + 1) * clen;
    for (int64_t m0 = ch * clen + lane; m0 < m1; m0 += 8 * 64) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t m = m0 + u * 64;
        v[u] = m < m1 ? (double)row[base | (msh >= 0 ? m << msh : deposit(m, d.merged_pos, d.n_merged))] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] += v[u];
    }
    double s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
#pragma unroll
    for (int k = 32; k >= 1; k >>= 1) s += __shfl_xor(s, k, 64);
    if (lane == 0) {
      if (lc == 0) Out[o] = (O)s;
      else d.part[w] = s;
    }
  } else if (d.seg) {
    // a row's merged runs are consecutive: element g of the stream (row r,
    // offset e = av * nmerge + m) sits at row r, zoom | e.  Lanes read
    // consecutive elements (eight loads in flight), and each aligned group of
    // nmerge lanes adds its run by a butterfly within the group.
    const int nm = d.n_merged;
    const int64_t rowlen = int64_t(1) << (d.n_active + nm);
    const int64_t total = nout << nm;
    const int64_t g0 = (bid - d.block_start) * 2048 + threadIdx.x;
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t g = g0 + u * 256;
      v[u] = g < total ? (double)E[(g / rowlen) * f + (zoom | (g % rowlen))] : 0.0;
    }
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      double s = v[u];
      for (int k = (1 << nm) >> 1; k >= 1; k >>= 1) s += __shfl_xor(s, k, 64);
      const int64_t g = g0 + u * 256;
      if ((lane & ((1 << nm) - 1)) == 0 && g < total) Out[g >> nm] = (O)s;
    }
  } else {
    const int64_t o = (bid - d.block_start) * 256 + threadIdx.x;
    if (o >= nout) return;
    const int64_t r = o >> d.n_active, av = o & ((int64_t(1) << d.n_active) - 1);
    const int64_t base = (ash >= 0 ? av << ash : deposit(av, d.active_pos, d.n_active)) | zoom;
    const I *row = E + r * f;
    double s = 0.0;
    for (int64_t m = 0; m < nmerge; ++m)
      s += (double)row[base | (msh >= 0 ? m << msh : deposit(m, d.merged_pos, d.n_merged))];
    Out[o] = (O)s;
  }
}

// Second pass of long merges: one thread per output adds its chunk sums in
// chunk order.  Descriptors without chunks have no blocks here.
template <typename O>
__global__ __launch_bounds__(256) void k_dd_merge_chunks(const MergeArgs a) {
  if (gated_off(a.gate, a.gate_val)) return;
  const int64_t bid = blockIdx.x;
  int i = 0;
  while (i + 1 < a.n && bid >= a.d[i + 1].chunk_block_start) ++i;
  const MergeDesc &d = a.d[i];
  const int64_t o = (bid - d.chunk_block_start) * 256 + threadIdx.x;
  const int64_t nout = d.rows << d.n_active;
  if (d.log_chunks == 0 || o >= nout) return;
  const int64_t nc = int64_t(1) << d.log_chunks;
  const double *p = d.part + o * nc;
  double s = 0.0;
  for (int64_t c = 0; c < nc; ++c) s += p[c];
  static_cast<O *>(d.dst)[o] = (O)s;
}

// ---- top-T of FP64 bins, ordered by (value descending, index ascending)
struct Cand {
  double v;
  int64_t i;
};
__device__ __forceinline__ bool better(const Cand &a, const Cand &b) {
  return a.v > b.v || (a.v == b.v && a.i < b.i);
}
// NaN never wins: it compares false both ways, so treat it as -inf.
__device__ __forceinline__ double key(double v) { return v != v ? -__builtin_inf() : v; }

constexpr Cand kNoCand{-__builtin_inf(), INT64_MAX};

// Eight candidates at a time: compare-and-swap (better first) on values,
// a 19-exchange sorting network for eight, and the best eight of two sorted
// lists by one bitonic step (elementwise best of one list and the other
// reversed) plus a bitonic sort - 39 exchanges per eight candidates where
// eight insertions into a full list take 64.
static_assert(kTopT == 8, "the sorting network and merge are for eight");
__device__ __forceinline__ void cas(Cand &a, Cand &b) {
  const bool s = better(b, a);
  const double av = a.v, bv = b.v;
  const int64_t ai = a.i, bi = b.i;
  a.v = s ? bv : av;
  a.i = s ? bi : ai;
  b.v = s ? av : bv;
  b.i = s ? ai : bi;
}
__device__ __forceinline__ void sort8(Cand (&c)[8]) {
  cas(c[0], c[2]); cas(c[1], c[3]); cas(c[4], c[6]); cas(c[5], c[7]);
  cas(c[0], c[4]); cas(c[1], c[5]); cas(c[2], c[6]); cas(c[3], c[7]);
  cas(c[0], c[1]); cas(c[2], c[3]); cas(c[4], c[5]); cas(c[6], c[7]);
  cas(c[2], c[4]); cas(c[3], c[5]);
  cas(c[1], c[4]); cas(c[3], c[6]);
  cas(c[1], c[2]); cas(c[3], c[4]); cas(c[5], c[6]);
}
// m and c sorted best first; m becomes the best eight of both, sorted
__device__ __forceinline__ void keep_better(Cand &a, const Cand &b) {
  const bool s = better(b, a);
  const double av = a.v, bv = b.v;
  const int64_t ai = a.i, bi = b.i;
  a.v = s ? bv : av;
  a.i = s ? bi : ai;
}
__device__ __forceinline__ void merge8(Cand (&m)[kTopT], Cand (&c)[8]) {
  keep_better(m[0], c[7]); keep_better(m[1], c[6]); keep_better(m[2], c[5]); keep_better(m[3], c[4]);
  keep_better(m[4], c[3]); keep_better(m[5], c[2]); keep_better(m[6], c[1]); keep_better(m[7], c[0]);
  cas(m[0], m[4]); cas(m[1], m[5]); cas(m[2], m[6]); cas(m[3], m[7]);
  cas(m[0], m[2]); cas(m[1], m[3]); cas(m[4], m[6]); cas(m[5], m[7]);
  cas(m[0], m[1]); cas(m[2], m[3]); cas(m[4], m[5]); cas(m[6], m[7]);
}

// Block-wide best kTopT of the per-thread rankings, in kTopT rounds.  A round
// finds each wave's winner - the largest head value by a butterfly over values
// only, then the lowest index among the lanes holding it (one lane in the
// usual case, read directly) - and combines the NW wave winners in LDS; the
// thread holding the overall winner pops it.  Bin indices are unique, so
// exactly one thread pops.  The wave winners alternate between two LDS rows,
// so one barrier per round suffices: a wave can only rewrite a row after the
// next round's barrier, which every wave reaches after reading that row.
template <int NW>
__device__ __forceinline__ void block_top(Cand (&m)[kTopT], Cand *out) {
  __shared__ Cand wbest[2][NW];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll 1
  for (int k = 0; k < kTopT; ++k) {
    double mv = m[0].v;   // keys are never NaN
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      const double x = __shfl_xor(mv, o, 64);
      mv = x > mv ? x : mv;
    }
    const bool hold = m[0].v == mv;
    const unsigned long long hit = __ballot(hold);   // never empty
    Cand c;
    c.v = mv;
    if (__popcll(hit) == 1) {
      c.i = __shfl(m[0].i, __ffsll((long long)hit) - 1, 64);
    } else {
      int64_t ci = hold ? m[0].i : INT64_MAX;
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        const int64_t x = (int64_t)__shfl_xor((long long)ci, o, 64);
        ci = x < ci ? x : ci;
      }
      c.i = ci;
    }
    Cand *wb = wbest[k & 1];
    if (lane == 0) wb[wave] = c;
    __syncthreads();
    Cand w = wb[0];
#pragma unroll
    for (int j = 1; j < NW; ++j)
      if (better(wb[j], w)) w = wb[j];
    if (threadIdx.x == 0) out[k] = w;
    if (w.i != INT64_MAX && m[0].i == w.i) {
#pragma unroll
      for (int j = 0; j + 1 < kTopT; ++j) m[j] = m[j + 1];
      m[kTopT - 1] = kNoCand;
    }
  }
}

// Stage 1: each block ranks a contiguous range of bins, keeping only the
// candidates ranked strictly after `after` (so a consumed prefix of the
// ranking can be skipped when more candidates are needed).
template <typename B>
__global__ __launch_bounds__(256) void k_topk_stage1(const B *bins, int64_t count, int64_t per_block,
                                                     Cand *partial, double after_v, int64_t after_i,
                                                     const int32_t *gate, int32_t gate_val, const TopReq *req,
                                                     int64_t stride) {
  if (gated_off(gate, gate_val)) return;
  if (req) {   // parameters from device memory; the grid covers the largest count
    if (!req->active) return;
    bins += (int64_t)req->row * stride;
    count = req->count;
    per_block = (count + gridDim.x - 1) / gridDim.x;
    after_v = req->after_v;
    after_i = req->after_i;
  }
  Cand m[kTopT];
#pragma unroll
  for (int k = 0; k < kTopT; ++k) m[k] = kNoCand;
  const Cand after{after_v, after_i};
  const int64_t b0 = (int64_t)blockIdx.x * per_block;
  const int64_t b1 = count < b0 + per_block ? count : b0 + per_block;
  // chunks of 2048 bins: a thread's eight loads are all in flight before it
  // ranks them
  for (int64_t c0 = b0; c0 < b1; c0 += 8 * 256) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t i = c0 + u * 256 + threadIdx.x;
      v[u] = i < b1 ? (double)bins[i] : 0.0;
    }
    Cand c[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t i = c0 + u * 256 + threadIdx.x;
      const Cand x{key(v[u]), i};
      const bool ok = i < b1 && better(after, x);   // selects on values: the lists stay in registers
      c[u].v = ok ? x.v : kNoCand.v;
      c[u].i = ok ? x.i : kNoCand.i;
    }
    sort8(c);
    merge8(m, c);
  }
  block_top<4>(m, partial + (int64_t)blockIdx.x * kTopT);
}

// Stage 2: one block of 256 threads ranks all stage-1 candidates (at most
// 1024 blocks x kTopT), eight loads in flight per thread at a time, and
// writes the best t.  Four waves keep the block-wide rounds cheap.
__global__ __launch_bounds__(256) void k_topk_stage2(const Cand *partial, int64_t count, int t, TopOut *out,
                                                     const int32_t *gate, int32_t gate_val, const TopReq *req) {
  if (gated_off(gate, gate_val)) return;
  if (req) {
    if (!req->active) return;
    out = req->out;
  }
  __shared__ Cand res[kTopT];
  Cand m[kTopT];
#pragma unroll
  for (int k = 0; k < kTopT; ++k) m[k] = kNoCand;
  for (int64_t c0 = 0; c0 < count; c0 += 8 * 256) {
    Cand v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t i = c0 + u * 256 + threadIdx.x;
      v[u] = i < count ? partial[i] : kNoCand;
    }
    sort8(v);
    merge8(m, v);
  }
  block_top<4>(m, res);
  __syncthreads();
  if ((int)threadIdx.x < t) {
    out->value[threadIdx.x] = res[threadIdx.x].v;
    out->index[threadIdx.x] = res[threadIdx.x].i;
  }
}

Status launch_dd_merge(const MergeArgs &a, int64_t blocks, bool in_double, bool out_double,
                       hipStream_t s) {
  const dim3 g((unsigned)blocks), b(256);
  if (in_double)
    CQC_TRY(out_double ? launch("dd_merge", k_dd_merge<double, double>, g, b, 0, s, a)
                       : launch("dd_merge", k_dd_merge<double, float>, g, b, 0, s, a));
  else
    CQC_TRY(out_double ? launch("dd_merge", k_dd_merge<float, double>, g, b, 0, s, a)
                       : launch("dd_merge", k_dd_merge<float, float>, g, b, 0, s, a));
  // second pass over the descriptors with chunked merges (the others get an
  // empty block range)
  MergeArgs c = a;
  int64_t nb = 0;
  for (int i = 0; i < c.n; ++i) {
    c.d[i].chunk_block_start = nb;
    if (c.d[i].log_chunks > 0) nb += ((c.d[i].rows << c.d[i].n_active) + 255) / 256;
  }
  if (nb == 0) return Status::ok();
  const dim3 g2((unsigned)nb);
  return out_double ? launch("dd_merge_chunks", k_dd_merge_chunks<double>, g2, b, 0, s, c)
                    : launch("dd_merge_chunks", k_dd_merge_chunks<float>, g2, b, 0, s, c);
}

size_t topk_scratch_bytes(int64_t count, int t) {
  (void)t;
  const int64_t blocks = std::min<int64_t>(1024, (count + 2047) / 2048);
  return sizeof(Cand) * (size_t)(blocks * kTopT);
}

Status launch_topk(const void *bins, bool bins_f32, int64_t count, int t, void *scratch, TopOut *out,
                   double after_v, int64_t after_i, hipStream_t s, const int32_t *gate, int32_t gate_val) {
  if (count < 1) return Status::fail(CQC_ERR_INVALID_ARG, "top-k over no bins");
  const int64_t blocks = std::min<int64_t>(1024, (count + 2047) / 2048);
  const int64_t per_block = (count + blocks - 1) / blocks;
  if (t < 1 || t > kTopT) return Status::fail(CQC_ERR_INVALID_ARG, "top-k count out of range");
  Cand *partial = static_cast<Cand *>(scratch);
  if (bins_f32)
    CQC_TRY(launch("topk_stage1", k_topk_stage1<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                   static_cast<const float *>(bins), count, per_block, partial, after_v, after_i, gate, gate_val,
                   (const TopReq *)nullptr, (int64_t)0));
  else
    CQC_TRY(launch("topk_stage1", k_topk_stage1<double>, dim3((unsigned)blocks), dim3(256), 0, s,
                   static_cast<const double *>(bins), count, per_block, partial, after_v, after_i, gate, gate_val,
                   (const TopReq *)nullptr, (int64_t)0));
  return launch("topk_stage2", k_topk_stage2, dim3(1), dim3(256), 0, s, static_cast<const Cand *>(partial),
                blocks * kTopT, t, out, gate, gate_val, (const TopReq *)nullptr);
}

Status launch_topk_req(const void *bins, bool bins_f32, int64_t stride, int64_t max_count, void *scratch,
                       const TopReq *req, hipStream_t s) {
  if (max_count < 1) return Status::fail(CQC_ERR_INVALID_ARG, "top-k over no bins");
  const int64_t blocks = std::min<int64_t>(1024, (max_count + 2047) / 2048);
  Cand *partial = static_cast<Cand *>(scratch);
  const int32_t *no_gate = nullptr;
  if (bins_f32)
    CQC_TRY(launch("topk_req_stage1", k_topk_stage1<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                   static_cast<const float *>(bins), max_count, (int64_t)0, partial, 0.0, (int64_t)0, no_gate, 0,
                   req, stride));
  else
    CQC_TRY(launch("topk_req_stage1", k_topk_stage1<double>, dim3((unsigned)blocks), dim3(256), 0, s,
                   static_cast<const double *>(bins), max_count, (int64_t)0, partial, 0.0, (int64_t)0, no_gate, 0,
                   req, stride));
  return launch("topk_req_stage2", k_topk_stage2, dim3(1), dim3(256), 0, s, static_cast<const Cand *>(partial),
                blocks * kTopT, kTopT, (TopOut *)nullptr, no_gate, 0, req);
}

}  // namespace cqc
