/* Plain FP64 CPU twin of the oracle's full-definition build and of the
 * dynamic definition's merge, for timing.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests and by the benchmark's CPU
 * baseline; the reconstruction library never links or calls it.
 *
 * For every requested output x it evaluates the definition of the FD build
 * (Section 3.2.3; 4^K Kronecker products scaled by 2^-K, Section 3.3):
 *     p(x) = 2^-K * sum_{l} prod_c E_c[row_c(l)][x_c]
 * summing the terms sequentially in ascending l (cut 0 = most significant
 * base-4 digit) in double precision.  row_c(l) is the base-4 number formed by
 * the labels of the cuts incident to c in ascending cut id; x_c takes the bits
 * of x (qubit q = bit n-1-q) on c's output qubits, local bit 0 most
 * significant.  Outputs are independent, so OpenMP splits them over threads.
 */
#include <stdint.h>
#include <stdlib.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int cqo_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Returns 0 on success, -1 on bad arguments / allocation failure. */
int cqo_fd(int n, int n_sub, int K, const int *f, const int *edge_up,
           const int *edge_down, const int *out_qubit,
           const double *const *entries, const int64_t *xs, int64_t n_x,
           double *out, int threads) {
  if (n < 0 || n > 62 || n_sub < 1 || K < 0 || K > 15) return -1;
  int64_t n_terms = (int64_t)1 << (2 * K);
  int64_t total = xs ? n_x : ((int64_t)1 << n);
  /* row table: row_c(l) for every subcircuit and term */
  int32_t *row = (int32_t *)malloc(sizeof(int32_t) * (size_t)n_sub * (size_t)n_terms);
  int *qoff = (int *)malloc(sizeof(int) * (size_t)(n_sub + 1));
  if (!row || !qoff) { free(row); free(qoff); return -1; }
  qoff[0] = 0;
  for (int c = 0; c < n_sub; ++c) qoff[c + 1] = qoff[c] + f[c];
  for (int c = 0; c < n_sub; ++c) {
    for (int64_t l = 0; l < n_terms; ++l) {
      int32_t r = 0;
      for (int e = 0; e < K; ++e) {
        if (edge_up[e] == c || edge_down[e] == c) {
          int digit = (int)((l >> (2 * (K - 1 - e))) & 3);
          r = r * 4 + digit;
        }
      }
      row[(size_t)c * (size_t)n_terms + (size_t)l] = r;
    }
  }
  double scale = ldexp(1.0, -K);
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
#endif
#pragma omp parallel
  {
    int64_t xc[64];
#pragma omp for schedule(static)
    for (int64_t i = 0; i < total; ++i) {
      int64_t x = xs ? xs[i] : i;
      for (int c = 0; c < n_sub; ++c) {
        int64_t v = 0;
        for (int j = 0; j < f[c]; ++j) {
          int q = out_qubit[qoff[c] + j];
          v = (v << 1) | ((x >> (n - 1 - q)) & 1);
        }
        xc[c] = v;
      }
      double acc = 0.0;
      for (int64_t l = 0; l < n_terms; ++l) {
        double t = 1.0;
        for (int c = 0; c < n_sub; ++c) {
          int64_t width = (int64_t)1 << f[c];
          t *= entries[c][(int64_t)row[(size_t)c * (size_t)n_terms + (size_t)l] * width + xc[c]];
        }
        acc += t;
      }
      out[i] = acc * scale;
    }
  }
  free(row);
  free(qoff);
  return 0;
}

/* Dynamic definition (Algorithm 1, Section 4.3): the merge of one subcircuit's
 * entries over its merged output qubits, zoomed qubits held at their values:
 *     out[r][a] = sum over merged bit strings m (ascending) of E[r][x(a, m)]
 * where x places the bits of a on the active local bits, the zoom values on
 * the zoomed ones and the bits of m on the merged ones (all in local order,
 * local bit 0 most significant).  role[j] per local bit: -2 active, -1
 * merged, 0/1 zoomed to that value.  The additions run in ascending x (the
 * merged bits fill x in order), from 0.0, in double precision.  Rows are
 * independent, so OpenMP splits them over threads.  Returns 0, or -1 on bad
 * arguments. */
int cqo_dd_merge(int f, int64_t rows, const double *entries, const signed char *role, double *out,
                 int threads) {
  if (f < 0 || f > 40 || rows < 0) return -1;
  int n_act = 0, n_mer = 0;
  int act[64], mer[64];
  int64_t zoom = 0;
  for (int j = 0; j < f; ++j) {
    const int bit = f - 1 - j; /* local bit j is bit f-1-j of x */
    if (role[j] == -2) act[n_act++] = bit;
    else if (role[j] == -1) mer[n_mer++] = bit;
    else if (role[j] == 0 || role[j] == 1) zoom |= (int64_t)role[j] << bit;
    else return -1;
  }
  const int64_t width = (int64_t)1 << f, na = (int64_t)1 << n_act, nm = (int64_t)1 << n_mer;
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
#endif
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < rows; ++r) {
    for (int64_t a = 0; a < na; ++a) {
      int64_t base = zoom;
      for (int t = 0; t < n_act; ++t) base |= ((a >> (n_act - 1 - t)) & 1) << act[t];
      double acc = 0.0;
      for (int64_t m = 0; m < nm; ++m) {
        int64_t x = base;
        for (int t = 0; t < n_mer; ++t) x |= ((m >> (n_mer - 1 - t)) & 1) << mer[t];
        acc += entries[r * width + x];
      }
      out[r * na + a] = acc;
    }
  }
  return 0;
}

/* Chi-square distance of two distributions (Eq. 16), in double precision:
 * the sum over i with a_i + b_i > 0 of (a_i - b_i)^2 / (a_i + b_i).  Each
 * thread sums a contiguous range in ascending i; the thread sums are then
 * added in thread order. */
double cqo_chi2(const double *a, const double *b, int64_t n, int threads) {
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
  const int nt = omp_get_max_threads();
#else
  const int nt = 1;
#endif
  double part[256];
  const int T = nt < 256 ? nt : 256;
  for (int t = 0; t < T; ++t) part[t] = 0.0;
#pragma omp parallel num_threads(T)
  {
#ifdef _OPENMP
    const int t = omp_get_thread_num();
#else
    const int t = 0;
#endif
    const int64_t lo = n * t / T, hi = n * (t + 1) / T;
    double s = 0.0;
    for (int64_t i = lo; i < hi; ++i) {
      const double u = a[i] + b[i];
      if (u > 0.0) {
        const double d = a[i] - b[i];
        s += d * d / u;
      }
    }
    part[t] = s;
  }
  double tot = 0.0;
  for (int t = 0; t < T; ++t) tot += part[t];
  return tot;
}
