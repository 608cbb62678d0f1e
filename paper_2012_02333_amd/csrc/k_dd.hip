// Dynamic-definition kernels (Algorithm 1, Section 4.3): merging subcircuit
// entries over their merged qubits, and selecting the heaviest bins.
#include "kernels.hpp"
#include "dd.hpp"

namespace cqc {

__device__ __forceinline__ int64_t dep_bits(int64_t v, const BitPos &pos, int nbits) {
  int64_t out = 0;
#pragma unroll 1
  for (int j = 0; j < nbits; ++j) {
    const uint64_t w = pos.w[0] * (j / 10 == 0) + pos.w[1] * (j / 10 == 1) + pos.w[2] * (j / 10 == 2) +
                       pos.w[3] * (j / 10 == 3) + pos.w[4] * (j / 10 == 4);
    out |= ((v >> j) & 1) << ((w >> (6 * (j % 10))) & 63);
  }
  return out;
}

// E'_c[r][a] = sum_m E_c[r][dep(a, active) | zoom | dep(m, merged)], summed in
// FP64 in ascending m (one wave per output when there are >= 64 merged
// combinations, lanes strided over m and combined by a fixed butterfly; one
// thread per output otherwise).
template <typename I, typename O>
__global__ __launch_bounds__(256) void k_dd_merge(const MergeArgs a) {
  const int64_t bid = blockIdx.x;
  int i = 0;
  while (i + 1 < a.n && bid >= a.d[i + 1].block_start) ++i;
  const MergeDesc &d = a.d[i];
  const I *E = static_cast<const I *>(d.src);
  O *Out = static_cast<O *>(d.dst);
  const int64_t nout = d.rows << d.n_active;
  const int64_t nmerge = int64_t(1) << d.n_merged;
  const int64_t f = int64_t(1) << d.f;
  const bool low_contig = d.merged_low_contig;
  if (nmerge >= 64) {
    const int64_t o = (bid - d.block_start) * 4 + (threadIdx.x >> 6);
    if (o >= nout) return;
    const int lane = threadIdx.x & 63;
    const int64_t r = o >> d.n_active, av = o & ((int64_t(1) << d.n_active) - 1);
    const int64_t base = dep_bits(av, d.active_pos, d.n_active) | d.zoom_value;
    const I *row = E + r * f;
    double s = 0.0;
    for (int64_t m = lane; m < nmerge; m += 64)
      s += (double)row[base | (low_contig ? m : dep_bits(m, d.merged_pos, d.n_merged))];
#pragma unroll
    for (int w = 32; w >= 1; w >>= 1) s += __shfl_xor(s, w, 64);
    if (lane == 0) Out[o] = (O)s;
  } else {
    const int64_t o = (bid - d.block_start) * 256 + threadIdx.x;
    if (o >= nout) return;
    const int64_t r = o >> d.n_active, av = o & ((int64_t(1) << d.n_active) - 1);
    const int64_t base = dep_bits(av, d.active_pos, d.n_active) | d.zoom_value;
    const I *row = E + r * f;
    double s = 0.0;
    for (int64_t m = 0; m < nmerge; ++m)
      s += (double)row[base | (low_contig ? m : dep_bits(m, d.merged_pos, d.n_merged))];
    Out[o] = (O)s;
  }
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

// Block-wide selection of the best `t` candidates from per-thread sorted
// lists (best first) of length <= kTopT.
__device__ void block_select(Cand (&mine)[kTopT], int nmine, int t, Cand *out, Cand *lds) {
  int head = 0;
  for (int k = 0; k < t; ++k) {
    Cand c = head < nmine ? mine[head] : Cand{-__builtin_inf(), INT64_MAX};
    lds[threadIdx.x] = c;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
      if ((int)threadIdx.x < w && better(lds[threadIdx.x + w], lds[threadIdx.x]))
        lds[threadIdx.x] = lds[threadIdx.x + w];
      __syncthreads();
    }
    const Cand win = lds[0];
    if (threadIdx.x == 0) out[k] = win;
    if (head < nmine && mine[head].i == win.i && mine[head].v == win.v) ++head;
    __syncthreads();
  }
}

__device__ void insert_cand(Cand (&mine)[kTopT], int &n, int t, Cand c) {
  if (n == t && !better(c, mine[t - 1])) return;
  int p = n < t ? n++ : t - 1;
  while (p > 0 && better(c, mine[p - 1])) {
    mine[p] = mine[p - 1];
    --p;
  }
  mine[p] = c;
}

// Stage 1: each block reduces a contiguous range of bins to its best t among
// the candidates ranked strictly after `after` (so a consumed prefix of the
// ranking can be skipped when more candidates are needed).
__global__ __launch_bounds__(256) void k_topk_stage1(const double *bins, int64_t count, int t,
                                                     int64_t per_block, Cand *partial, double after_v,
                                                     int64_t after_i) {
  __shared__ Cand lds[256];
  Cand mine[kTopT];
  int n = 0;
  const Cand after{after_v, after_i};
  const int64_t b0 = (int64_t)blockIdx.x * per_block;
  const int64_t b1 = count < b0 + per_block ? count : b0 + per_block;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += blockDim.x) {
    const Cand c{key(bins[i]), i};
    if (better(after, c)) insert_cand(mine, n, t, c);
  }
  block_select(mine, n, t, partial + (int64_t)blockIdx.x * t, lds);
}

// Stage 2: one block reduces all stage-1 candidates to the best t.
__global__ __launch_bounds__(256) void k_topk_stage2(const Cand *partial, int64_t count, int t,
                                                     TopOut *out) {
  __shared__ Cand lds[256];
  __shared__ Cand res[kTopT];
  Cand mine[kTopT];
  int n = 0;
  for (int64_t i = threadIdx.x; i < count; i += blockDim.x) insert_cand(mine, n, t, partial[i]);
  block_select(mine, n, t, res, lds);
  if (threadIdx.x < t) {
    out->value[threadIdx.x] = res[threadIdx.x].v;
    out->index[threadIdx.x] = res[threadIdx.x].i;
  }
}

Status launch_dd_merge(const MergeArgs &a, int64_t blocks, bool in_double, bool out_double,
                       hipStream_t s) {
  const dim3 g((unsigned)blocks), b(256);
  if (in_double)
    return out_double ? launch("dd_merge", k_dd_merge<double, double>, g, b, 0, s, a)
                      : launch("dd_merge", k_dd_merge<double, float>, g, b, 0, s, a);
  return out_double ? launch("dd_merge", k_dd_merge<float, double>, g, b, 0, s, a)
                    : launch("dd_merge", k_dd_merge<float, float>, g, b, 0, s, a);
}

size_t topk_scratch_bytes(int64_t count, int t) {
  const int64_t blocks = std::min<int64_t>(1024, (count + 2047) / 2048);
  return sizeof(Cand) * (size_t)(blocks * t);
}

Status launch_topk(const double *bins, int64_t count, int t, void *scratch, TopOut *out,
                   double after_v, int64_t after_i, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>(1024, (count + 2047) / 2048);
  const int64_t per_block = (count + blocks - 1) / blocks;
  Cand *partial = static_cast<Cand *>(scratch);
  CQC_TRY(launch("topk_stage1", k_topk_stage1, dim3((unsigned)blocks), dim3(256), 0, s, bins, count, t,
                 per_block, partial, after_v, after_i));
  return launch("topk_stage2", k_topk_stage2, dim3(1), dim3(256), 0, s,
                static_cast<const Cand *>(partial), blocks * t, t, out);
}

}  // namespace cqc
