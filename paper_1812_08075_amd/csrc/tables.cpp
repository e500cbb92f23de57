// 1D quadrature and basis tables of the sum-factorized kernels (host side).
//
// The cell rule is the tensor product of 1D Gauss-Legendre rules of maximal
// order (Section 2.1); the 1D basis matrices A^(i) (basis values at the
// quadrature points) and D^(i) (derivatives) are the factors of the Kronecker
// form of Section 2.2. The nodal basis is the Lagrange basis at the k+1
// Gauss-Legendre points.
//
// Nodes: eigenvalues of the Jacobi matrix of the Legendre recurrence
// (Golub-Welsch), located by Sturm-sequence bisection. Weights: Christoffel
// numbers 1 / sum_j pt_j(x)^2 of the orthonormal Legendre polynomials pt_j.
// Lagrange values and derivatives: barycentric formulas.
#include <cmath>
#include <cfloat>
#include <stdexcept>

#include "internal.h"

namespace dgi {

namespace {
using ld = long double;

// Number of eigenvalues of the m x m symmetric tridiagonal matrix
// (zero diagonal, off-diagonal b[1..m-1]) smaller than x (Sturm count).
int sturm_count(int m, const ld* b, ld x) {
  int count = 0;
  ld q = -x;  // d_0 - x with zero diagonal
  if (q < 0) ++count;
  for (int i = 1; i < m; ++i) {
    ld denom = (q == 0) ? 1e-300L : q;
    q = -x - b[i] * b[i] / denom;
    if (q < 0) ++count;
  }
  return count;
}
}  // namespace

void gauss_legendre_golub_welsch(int m, double* x, double* w) {
  if (m < 1 || m > PMAX) throw std::invalid_argument("Gauss-Legendre: unsupported number of points");
  // Legendre: x P_n = (n+1)/(2n+1) P_{n+1} + n/(2n+1) P_{n-1}; Jacobi matrix
  // off-diagonal b_n = n / sqrt(4 n^2 - 1), zero diagonal, spectrum in (-1, 1).
  ld b[PMAX];
  b[0] = 0;
  for (int n = 1; n < m; ++n) b[n] = (ld)n / std::sqrt((ld)(4 * n * n - 1));
  for (int i = 0; i < m; ++i) {
    // i-th smallest eigenvalue: the x where the Sturm count steps from i to i+1
    ld lo = -1, hi = 1;
    for (int it = 0; it < 200; ++it) {
      ld mid = (lo + hi) / 2;
      if (sturm_count(m, b, mid) > i) hi = mid; else lo = mid;
      if (hi - lo <= 4 * LDBL_EPSILON * (std::fabs(lo) + std::fabs(hi) + LDBL_MIN)) break;
    }
    ld t = (lo + hi) / 2;
    // Christoffel number: 1 / sum_{j<m} pt_j(t)^2, pt_j = sqrt((2j+1)/2) P_j
    ld p0 = 1, p1 = t, s = 0.5L;  // pt_0^2 = 1/2
    if (m > 1) s += 1.5L * t * t;
    for (int j = 2; j < m; ++j) {
      ld p2 = ((2 * j - 1) * t * p1 - (j - 1) * p0) / j;
      s += (2 * j + 1) / 2.0L * p2 * p2;
      p0 = p1;
      p1 = p2;
    }
    x[i] = (double)((1 + t) / 2);
    w[i] = (double)(1.0L / s / 2);
  }
}

namespace {
// Barycentric weights lambda_j = 1 / prod_{k != j} (x_j - x_k).
void bary_weights(int p, const ld* xn, ld* lam) {
  for (int j = 0; j < p; ++j) {
    ld prod = 1;
    for (int k = 0; k < p; ++k)
      if (k != j) prod *= (xn[j] - xn[k]);
    lam[j] = 1 / prod;
  }
}

// l_j(t) and l_j'(t) for all j at a point t.
void lagrange_at(int p, const ld* xn, const ld* lam, ld t, ld* val, ld* der) {
  int hit = -1;
  for (int j = 0; j < p; ++j)
    if (t == xn[j]) hit = j;
  if (hit >= 0) {
    // at a node: l_j = delta; l_j'(x_h) = (lam_j/lam_h)/(x_h - x_j), diagonal by
    // the vanishing row sum of the differentiation matrix
    ld diag = 0;
    for (int j = 0; j < p; ++j) {
      val[j] = (j == hit) ? 1 : 0;
      if (j != hit) {
        der[j] = (lam[j] / lam[hit]) / (xn[hit] - xn[j]);
        diag -= der[j];
      }
    }
    der[hit] = diag;
    return;
  }
  // second (true) barycentric form; l_j'(t) = l_j(t) * sum_{k != j} 1/(t - x_k)
  ld denom = 0;
  for (int k = 0; k < p; ++k) denom += lam[k] / (t - xn[k]);
  for (int j = 0; j < p; ++j) {
    val[j] = (lam[j] / (t - xn[j])) / denom;
    ld s = 0;
    for (int k = 0; k < p; ++k)
      if (k != j) s += 1 / (t - xn[k]);
    der[j] = val[j] * s;
  }
}
}  // namespace

Tables1D make_tables(int p, int m) {
  if (p < 1 || p > PMAX || m < 1 || m > PMAX) throw std::invalid_argument("unsupported table size");
  Tables1D T;
  T.p = p;
  T.m = m;
  double wtmp[PMAX];
  gauss_legendre_golub_welsch(p, T.xn, wtmp);
  gauss_legendre_golub_welsch(m, T.xq, T.wq);
  ld xn[PMAX], lam[PMAX], val[PMAX], der[PMAX];
  for (int j = 0; j < p; ++j) xn[j] = T.xn[j];
  bary_weights(p, xn, lam);
  for (int q = 0; q < m; ++q) {
    lagrange_at(p, xn, lam, (ld)T.xq[q], val, der);
    for (int j = 0; j < p; ++j) {
      T.A[q][j] = (double)val[j];
      T.D[q][j] = (double)der[j];
    }
  }
  for (int s = 0; s < 2; ++s) {
    lagrange_at(p, xn, lam, (ld)s, val, der);
    for (int j = 0; j < p; ++j) {
      T.e[s][j] = (double)val[j];
      T.de[s][j] = (double)der[j];
    }
  }
  return T;
}

}  // namespace dgi
