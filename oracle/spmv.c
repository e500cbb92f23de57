/*
 * Block-sparse matrix-vector products of the oracle's assembled DG operator
 * (test infrastructure only; the product path never links this file).
 *
 * A DG operator on a structured mesh has one block row per cell with at most
 * seven nonzero blocks: the cell itself and its six face neighbours (the
 * element-blocked structure of Section 1 and Section 3.1). Block (e, s) is
 * blocks[cls[e*7+s]] (n x n, row-major), its column block nbr[e*7+s] (-1:
 * absent). y = A x is the plain definition: y_e = sum_s B_(e,s) x_nbr(e,s),
 * rows in a fixed order, block rows split over OpenMP threads (static).
 */
#include <stdint.h>

void oracle_bsr_matvec(int64_t nelem, int32_t n, const int64_t* nbr, const int64_t* cls, const double* blocks,
                       const double* x, double* y, int32_t nthreads) {
#pragma omp parallel for schedule(static) num_threads(nthreads)
  for (int64_t e = 0; e < nelem; ++e) {
    double* ye = y + e * n;
    for (int32_t i = 0; i < n; ++i) ye[i] = 0.0;
    for (int s = 0; s < 7; ++s) {
      const int64_t c = nbr[e * 7 + s];
      if (c < 0) continue;
      const double* B = blocks + cls[e * 7 + s] * (int64_t)n * n;
      const double* xc = x + c * n;
      for (int32_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int32_t j = 0; j < n; ++j) acc += B[(int64_t)i * n + j] * xc[j];
        ye[i] += acc;
      }
    }
  }
}
