/* Plain FP64 CPU twin of the oracle's full-definition build, for timing.
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
