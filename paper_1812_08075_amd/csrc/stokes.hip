// DG Stokes operator on trilinear hexahedra, sum-factorized (gfx950, FP64).
//
// Operator (Section 5.3, eq. stokes_weak, linear part, mu = 1):
//   cells: (grad u, grad v) - (p, div v) - (div u, q)
//   interior and Dirichlet faces: -({grad u} n, [v]) + theta ([u], {grad v} n)
//     + gamma_F ([u], [v]) + ({p}, [v].n) + ([u].n, {q})
// with the garbled second face term read as theta ([u], {grad v} n), velocity
// Q_k^3 in the nodal Gauss-Legendre basis (m = k+1 points, collocated) and
// pressure Q_{k-1} in the nodal basis at the k Gauss-Legendre points.
//
// Cells are images of the reference cube under the trilinear map of their
// vertices, so J, det J and J^{-1} are evaluated at every quadrature point
// from the 8 corners (Algorithm 1, part 2 with the geometry mu_T).
//
// Work decomposition: one wave (64 threads) per cell.
//  1. volume: thread = quadrature point. The nine reference derivatives
//     d_a u_c are 1D contractions with D along a (Algorithm 1, part 1); the
//     pressure at the point is the tensor interpolation A_p (x) A_p (x) A_p.
//     The pointwise stage forms R_{c,a} = w |det J| (J^{-1} (J^{-T} g_c) -
//     p J^{-1} e_c)_a and R_p = -w |det J| div u; the transposed
//     contractions (part 3) give the cell residual of node i.
//  2. faces (element-centric, all six at once): thread = face point. The own
//     trace of u and of every reference derivative is the line's dot product
//     with l_j(s) (normal direction first, Section 2.2). The neighbour's
//     velocity trace and normal derivative come from its line in global
//     memory; its tangential derivatives are D-contractions of its trace
//     across the face points (through LDS). Flux at the face point, then the
//     test functions of the own cell: value, normal derivative and the two
//     tangential derivatives (D^T across face points), pressure by
//     e_p (x) A_p^T (x) A_p^T.
// Every output entry has one writer; no atomics; bitwise reproducible.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <stdexcept>
#include <vector>

#include "internal.h"

namespace dgi {
namespace {

constexpr int NT = 64;

// Trilinear map of the 8 corners X[c][a] (corner c = c0 + 2 c1 + 4 c2):
// J[a][b] = d x_a / d xi_b at reference point xi.
__device__ __forceinline__ void jacobian(const double* X, const double xi[3], double J[3][3]) {
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) J[a][b] = 0.0;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int c0 = c & 1, c1 = (c >> 1) & 1, c2 = (c >> 2) & 1;
    const double f0 = c0 ? xi[0] : 1.0 - xi[0];
    const double f1 = c1 ? xi[1] : 1.0 - xi[1];
    const double f2 = c2 ? xi[2] : 1.0 - xi[2];
    const double d0 = (c0 ? 1.0 : -1.0) * f1 * f2;
    const double d1 = f0 * (c1 ? 1.0 : -1.0) * f2;
    const double d2 = f0 * f1 * (c2 ? 1.0 : -1.0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double x = X[3 * c + a];
      J[a][0] = fma(d0, x, J[a][0]);
      J[a][1] = fma(d1, x, J[a][1]);
      J[a][2] = fma(d2, x, J[a][2]);
    }
  }
}

// det J and J^{-1} (adjugate / det).
__device__ __forceinline__ double invert(const double J[3][3], double Ji[3][3]) {
  const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
  const double id = 1.0 / det;
  Ji[0][0] = c00 * id;
  Ji[1][0] = c01 * id;
  Ji[2][0] = c02 * id;
  Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
  Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
  Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
  Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
  Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
  Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
  return det;
}

struct StokesGeom {
  const double* vertices;  // (nz+1)(ny+1)(nx+1) x 3
  const double* gamma;     // per-face penalties, direction d at offset goff[d]
  int64_t goff[3];
};

__device__ __forceinline__ void load_corners(const StokesGeom& g, const StokesArgs& a, int ex, int ey, int ez,
                                             double* X, int t) {
  if (t < 24) {
    const int c = t / 3, k = t - 3 * c;
    const int i = ex + (c & 1), j = ey + ((c >> 1) & 1), l = ez + ((c >> 2) & 1);
    const int64_t v = i + (int64_t)(a.n[0] + 1) * (j + (int64_t)(a.n[1] + 1) * l);
    X[t] = g.vertices[3 * v + k];
  }
}

template <int P>
__global__ void __launch_bounds__(NT) k_stokes_apply(const double* __restrict__ x, double* __restrict__ y,
                                                     const StokesArgs a, const StokesGeom geo) {
  constexpr int KP = P - 1;
  constexpr int N = P * P * P, NQ = KP * KP * KP, L = P * P;
  constexpr int NB = 3 * N + NQ;      // DOFs per cell
  constexpr int NF = 6 * L;           // face points of the cell
  __shared__ double su[3 * N];        // velocity
  __shared__ double sp[NQ];           // pressure
  __shared__ double sX[24];           // own corners
  __shared__ double nX[6][24];        // neighbour corners
  __shared__ double np_[6][NQ];       // neighbour pressure
  __shared__ double sG[9 * N];        // reference gradients G[c*3+a][i]
  __shared__ double sR[9 * N];        // cell residual coefficients of d_a v_c
  __shared__ double sRp[N];           // cell residual coefficient of q
  __shared__ double fUN[3][NF];       // neighbour velocity traces
  __shared__ double fDN[3][NF];       // neighbour normal reference derivatives
  __shared__ double fV[3][NF];        // face coefficients of v_c
  __shared__ double fG[9][NF];        // face coefficients of d_a v_c
  __shared__ double fQ[NF];           // face coefficients of q

  const int t = threadIdx.x;
  const int e = blockIdx.x;
  const int nx = a.n[0], ny = a.n[1], nz = a.n[2];
  const int ec[3] = {e % nx, (e / nx) % ny, e / (nx * ny)};
  const int64_t base = (int64_t)e * NB;
  const int64_t estr[3] = {1, nx, (int64_t)nx * ny};

  // ---- loads ---------------------------------------------------------------
  for (int i = t; i < 3 * N; i += NT) su[i] = x[base + i];
  for (int i = t; i < NQ; i += NT) sp[i] = x[base + 3 * N + i];
  load_corners(geo, a, ec[0], ec[1], ec[2], sX, t);
  for (int f = 0; f < 6; ++f) {
    const int d = f >> 1, s = f & 1;
    int nc[3] = {ec[0], ec[1], ec[2]};
    nc[d] += s ? 1 : -1;
    if (nc[d] < 0 || nc[d] >= a.n[d]) continue;
    load_corners(geo, a, nc[0], nc[1], nc[2], nX[f], t);
    const int64_t nb = (int64_t)e + (s ? estr[d] : -estr[d]);
    for (int i = t; i < NQ; i += NT) np_[f][i] = x[nb * NB + 3 * N + i];
  }
  __syncthreads();

  // ---- volume, pointwise --------------------------------------------------
  for (int i = t; i < N; i += NT) {
    const int i0 = i % P, i1 = (i / P) % P, i2 = i / L;
    double g[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double* uc = su + c * N;
      double g0 = 0, g1 = 0, g2 = 0;
#pragma unroll
      for (int j = 0; j < P; ++j) {
        g0 = fma(a.D[i0 * P + j], uc[j + P * i1 + L * i2], g0);
        g1 = fma(a.D[i1 * P + j], uc[i0 + P * j + L * i2], g1);
        g2 = fma(a.D[i2 * P + j], uc[i0 + P * i1 + L * j], g2);
      }
      g[c][0] = g0;
      g[c][1] = g1;
      g[c][2] = g2;
      sG[(3 * c + 0) * N + i] = g0;
      sG[(3 * c + 1) * N + i] = g1;
      sG[(3 * c + 2) * N + i] = g2;
    }
    double pq = 0.0;
#pragma unroll
    for (int j2 = 0; j2 < KP; ++j2)
#pragma unroll
      for (int j1 = 0; j1 < KP; ++j1) {
        const double w12 = a.Ap[i1 * KP + j1] * a.Ap[i2 * KP + j2];
#pragma unroll
        for (int j0 = 0; j0 < KP; ++j0) pq = fma(a.Ap[i0 * KP + j0] * w12, sp[j0 + KP * (j1 + KP * j2)], pq);
      }
    const double xi[3] = {a.xq[i0], a.xq[i1], a.xq[i2]};
    double J[3][3], Ji[3][3];
    jacobian(sX, xi, J);
    const double det = invert(J, Ji);
    const double wd = a.w[i0] * a.w[i1] * a.w[i2] * fabs(det);
    double div = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double gp[3];  // physical gradient J^{-T} g
#pragma unroll
      for (int jj = 0; jj < 3; ++jj) gp[jj] = Ji[0][jj] * g[c][0] + Ji[1][jj] * g[c][1] + Ji[2][jj] * g[c][2];
      div += gp[c];
#pragma unroll
      for (int aa = 0; aa < 3; ++aa)
        sR[(3 * c + aa) * N + i] =
            wd * (Ji[aa][0] * gp[0] + Ji[aa][1] * gp[1] + Ji[aa][2] * gp[2] - pq * Ji[aa][c]);
    }
    sRp[i] = -wd * div;
  }

  // ---- faces, phase 1: neighbour traces ----------------------------------
  for (int fp = t; fp < NF; fp += NT) {
    const int f = fp / L, pt = fp - f * L;
    const int d = f >> 1, s = f & 1;
    int nc[3] = {ec[0], ec[1], ec[2]};
    nc[d] += s ? 1 : -1;
    if (nc[d] < 0 || nc[d] >= a.n[d]) continue;
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    const int pa = pt % P, pb = pt / P;
    int off = 0, str = 1;
    {
      int idx[3];
      idx[t1] = pa;
      idx[t2] = pb;
      idx[d] = 0;
      off = idx[0] + P * idx[1] + L * idx[2];
      str = d == 0 ? 1 : (d == 1 ? P : L);
    }
    const int64_t nb = (int64_t)e + (s ? estr[d] : -estr[d]);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double uN = 0, dN = 0;
#pragma unroll
      for (int j = 0; j < P; ++j) {
        const double v = x[nb * NB + c * N + off + j * str];
        uN = fma(a.e[1 - s][j], v, uN);
        dN = fma(a.de[1 - s][j], v, dN);
      }
      fUN[c][fp] = uN;
      fDN[c][fp] = dN;
    }
  }
  __syncthreads();

  // ---- faces, phase 2: flux at every face point ---------------------------
  for (int fp = t; fp < NF; fp += NT) {
    const int f = fp / L, pt = fp - f * L;
    const int d = f >> 1, s = f & 1;
    int nc[3] = {ec[0], ec[1], ec[2]};
    nc[d] += s ? 1 : -1;
    const bool has_nb = nc[d] >= 0 && nc[d] < a.n[d];
    const bool dir = (a.mask >> f) & 1u;
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    const int pa = pt % P, pb = pt / P;
    if (!has_nb && !dir) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        fV[c][fp] = 0.0;
        for (int aa = 0; aa < 3; ++aa) fG[3 * c + aa][fp] = 0.0;
      }
      fQ[fp] = 0.0;
      continue;
    }
    int idx[3];
    idx[t1] = pa;
    idx[t2] = pb;
    idx[d] = 0;
    const int off = idx[0] + P * idx[1] + L * idx[2];
    const int str = d == 0 ? 1 : (d == 1 ? P : L);
    // own traces of u_c and of all reference derivatives
    double uT[3], gT[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double u = 0, dn = 0, ga = 0, gb = 0;
#pragma unroll
      for (int j = 0; j < P; ++j) {
        const int node = off + j * str;
        u = fma(a.e[s][j], su[c * N + node], u);
        dn = fma(a.de[s][j], su[c * N + node], dn);
        ga = fma(a.e[s][j], sG[(3 * c + t1) * N + node], ga);
        gb = fma(a.e[s][j], sG[(3 * c + t2) * N + node], gb);
      }
      uT[c] = u;
      gT[c][d] = dn;
      gT[c][t1] = ga;
      gT[c][t2] = gb;
    }
    // own pressure trace: e_p(s) along d, A_p at the tangential nodes
    double pT = 0.0;
#pragma unroll
    for (int jd = 0; jd < KP; ++jd)
#pragma unroll
      for (int ja = 0; ja < KP; ++ja)
#pragma unroll
        for (int jb = 0; jb < KP; ++jb) {
          int pj[3];
          pj[d] = jd;
          pj[t1] = ja;
          pj[t2] = jb;
          pT = fma(a.ep[s][jd] * a.Ap[pa * KP + ja] * a.Ap[pb * KP + jb], sp[pj[0] + KP * (pj[1] + KP * pj[2])], pT);
        }
    // geometry from the own cell: normal (outward) and area element
    double xi[3];
    xi[d] = (double)s;
    xi[t1] = a.xq[pa];
    xi[t2] = a.xq[pb];
    double J[3][3], Ji[3][3];
    jacobian(sX, xi, J);
    const double det = invert(J, Ji);
    const double nn = sqrt(Ji[d][0] * Ji[d][0] + Ji[d][1] * Ji[d][1] + Ji[d][2] * Ji[d][2]);
    const double sg = s ? 1.0 : -1.0;
    const double nu[3] = {sg * Ji[d][0] / nn, sg * Ji[d][1] / nn, sg * Ji[d][2] / nn};
    const double dA = fabs(det) * nn * a.w[pa] * a.w[pb];
    // J^{-1} nu: reference components of the test-gradient direction
    const double Jn[3] = {Ji[0][0] * nu[0] + Ji[0][1] * nu[1] + Ji[0][2] * nu[2],
                          Ji[1][0] * nu[0] + Ji[1][1] * nu[1] + Ji[1][2] * nu[2],
                          Ji[2][0] * nu[0] + Ji[2][1] * nu[1] + Ji[2][2] * nu[2]};
    double gradT_n[3];  // (grad u_T,c) . nu
#pragma unroll
    for (int c = 0; c < 3; ++c) gradT_n[c] = Jn[0] * gT[c][0] + Jn[1] * gT[c][1] + Jn[2] * gT[c][2];
    const int plane = ec[d] + s;
    const int ct1 = ec[t1], ct2 = ec[t2];
    const double gam = geo.gamma[geo.goff[d] + plane + (int64_t)(a.n[d] + 1) * (ct1 + (int64_t)a.n[t1] * ct2)];
    double Rv[3], Rg[3], Rq = 0.0;
    if (has_nb) {
      // neighbour's full reference gradient at the same physical point
      double xin[3];
      xin[d] = (double)(1 - s);
      xin[t1] = a.xq[pa];
      xin[t2] = a.xq[pb];
      double JN[3][3], JiN[3][3];
      jacobian(nX[f], xin, JN);
      invert(JN, JiN);
      const double JnN[3] = {JiN[0][0] * nu[0] + JiN[0][1] * nu[1] + JiN[0][2] * nu[2],
                             JiN[1][0] * nu[0] + JiN[1][1] * nu[1] + JiN[1][2] * nu[2],
                             JiN[2][0] * nu[0] + JiN[2][1] * nu[1] + JiN[2][2] * nu[2]};
      const int fb = f * L;
      double pN = 0.0;
#pragma unroll
      for (int jd = 0; jd < KP; ++jd)
#pragma unroll
        for (int ja = 0; ja < KP; ++ja)
#pragma unroll
          for (int jb = 0; jb < KP; ++jb) {
            int pj[3];
            pj[d] = jd;
            pj[t1] = ja;
            pj[t2] = jb;
            pN = fma(a.ep[1 - s][jd] * a.Ap[pa * KP + ja] * a.Ap[pb * KP + jb],
                     np_[f][pj[0] + KP * (pj[1] + KP * pj[2])], pN);
          }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double gN[3];
        gN[d] = fDN[c][fp];
        double ga = 0, gb = 0;
#pragma unroll
        for (int j = 0; j < P; ++j) {
          ga = fma(a.D[pa * P + j], fUN[c][fb + j + P * pb], ga);
          gb = fma(a.D[pb * P + j], fUN[c][fb + pa + P * j], gb);
        }
        gN[t1] = ga;
        gN[t2] = gb;
        const double gradN_n = JnN[0] * gN[0] + JnN[1] * gN[1] + JnN[2] * gN[2];
        const double jump = uT[c] - fUN[c][fp];
        Rv[c] = dA * (-0.5 * (gradT_n[c] + gradN_n) + gam * jump + 0.5 * (pT + pN) * nu[c]);
        Rg[c] = dA * 0.5 * a.theta * jump;
        Rq += dA * 0.5 * jump * nu[c];
      }
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        Rv[c] = dA * (-gradT_n[c] + gam * uT[c] + pT * nu[c]);
        Rg[c] = dA * a.theta * uT[c];
        Rq += dA * uT[c] * nu[c];
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      fV[c][fp] = Rv[c];
#pragma unroll
      for (int aa = 0; aa < 3; ++aa) fG[3 * c + aa][fp] = Rg[c] * Jn[aa];
    }
    fQ[fp] = Rq;
  }
  __syncthreads();

  // ---- test functions: cell terms (part 3) plus the six faces --------------
  for (int i = t; i < N; i += NT) {
    const int ii[3] = {i % P, (i / P) % P, i / L};
    double acc[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < P; ++q) {
        s = fma(a.D[q * P + ii[0]], sR[(3 * c + 0) * N + q + P * ii[1] + L * ii[2]], s);
        s = fma(a.D[q * P + ii[1]], sR[(3 * c + 1) * N + ii[0] + P * q + L * ii[2]], s);
        s = fma(a.D[q * P + ii[2]], sR[(3 * c + 2) * N + ii[0] + P * ii[1] + L * q], s);
      }
      acc[c] = s;
    }
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      const int d = f >> 1, s = f & 1;
      const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
      const int j = ii[d], pa = ii[t1], pb = ii[t2];
      const int fb = f * L;
      const double es = a.e[s][j], des = a.de[s][j];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double tv = fV[c][fb + pa + P * pb];
#pragma unroll
        for (int q = 0; q < P; ++q) {
          tv = fma(a.D[q * P + pa], fG[3 * c + t1][fb + q + P * pb], tv);
          tv = fma(a.D[q * P + pb], fG[3 * c + t2][fb + pa + P * q], tv);
        }
        acc[c] = fma(es, tv, fma(des, fG[3 * c + d][fb + pa + P * pb], acc[c]));
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) y[base + c * N + i] = acc[c];
  }
  for (int i = t; i < NQ; i += NT) {
    const int jj[3] = {i % KP, (i / KP) % KP, i / (KP * KP)};
    double s = 0.0;
    for (int q = 0; q < N; ++q) {
      const int q0 = q % P, q1 = (q / P) % P, q2 = q / L;
      s = fma(a.Ap[q0 * KP + jj[0]] * a.Ap[q1 * KP + jj[1]] * a.Ap[q2 * KP + jj[2]], sRp[q], s);
    }
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      const int d = f >> 1, sd = f & 1;
      const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
      const double epv = a.ep[sd][jj[d]];
      const int fb = f * L;
      double fs = 0.0;
      for (int pt = 0; pt < L; ++pt) {
        const int pa = pt % P, pb = pt / P;
        fs = fma(a.Ap[pa * KP + jj[t1]] * a.Ap[pb * KP + jj[t2]], fQ[fb + pt], fs);
      }
      s = fma(epv, fs, s);
    }
    y[base + 3 * N + i] = s;
  }
}

// Host-side trilinear geometry for the penalties.
void host_jacobian(const double X[8][3], const double xi[3], double J[3][3]) {
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) J[a][b] = 0.0;
  for (int c = 0; c < 8; ++c) {
    const int cb[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
    double f[3], df[3];
    for (int d = 0; d < 3; ++d) {
      f[d] = cb[d] ? xi[d] : 1.0 - xi[d];
      df[d] = cb[d] ? 1.0 : -1.0;
    }
    const double dN[3] = {df[0] * f[1] * f[2], f[0] * df[1] * f[2], f[0] * f[1] * df[2]};
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) J[a][b] += dN[b] * X[c][a];
  }
}

double host_det(const double J[3][3]) {
  return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
         J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

}  // namespace

void cell_corners(const dg_mesh& M, int64_t e, double X[8][3]);

void stokes_setup(dg_mesh& M) {
  const int P = M.p, KP = M.kp;
  if (P != 3 && P != 4) throw std::runtime_error("Stokes is built for k = 2 and k = 3");
  StokesArgs& a = M.st;
  std::memset(&a, 0, sizeof(a));
  const Tables1D& T = M.tab;
  for (int q = 0; q < P; ++q)
    for (int j = 0; j < P; ++j) a.D[q * P + j] = T.D[q][j];
  for (int s = 0; s < 2; ++s)
    for (int j = 0; j < P; ++j) {
      a.e[s][j] = T.e[s][j];
      a.de[s][j] = T.de[s][j];
    }
  for (int q = 0; q < P; ++q) {
    a.w[q] = T.wq[q];
    a.xq[q] = T.xq[q];
  }
  const Tables1D TP = make_tables(KP, M.m);  // pressure basis at the quadrature points
  for (int q = 0; q < P; ++q)
    for (int j = 0; j < KP; ++j) a.Ap[q * KP + j] = TP.A[q][j];
  for (int s = 0; s < 2; ++s)
    for (int j = 0; j < KP; ++j) a.ep[s][j] = TP.e[s][j];
  a.theta = M.desc.theta;
  a.n[0] = M.desc.nx;
  a.n[1] = M.desc.ny;
  a.n[2] = M.desc.nz;
  a.nelem = (int32_t)M.nelem;
  a.mask = M.desc.dirichlet_mask;

  // vertices (regular grid when none were given)
  const int nx = M.desc.nx, ny = M.desc.ny, nz = M.desc.nz;
  if (M.vertices.empty()) {
    M.vertices.resize((size_t)(nx + 1) * (ny + 1) * (nz + 1) * 3);
    for (int l = 0; l <= nz; ++l)
      for (int j = 0; j <= ny; ++j)
        for (int i = 0; i <= nx; ++i) {
          double* v = &M.vertices[3 * (i + (size_t)(nx + 1) * (j + (size_t)(ny + 1) * l))];
          v[0] = (double)i / nx;
          v[1] = (double)j / ny;
          v[2] = (double)l / nz;
        }
  }
  // cell volumes |T| and face penalties gamma_F = coef |F| / min |T| by the m-point rules
  const double coef = M.desc.penalty_form == 0 ? M.desc.alpha * M.desc.k * (M.desc.k + 1)
                                               : M.desc.alpha * M.desc.k * (M.desc.k + 2);
  const int m = M.m;
  std::vector<double> vol(M.nelem);
  for (int64_t e = 0; e < M.nelem; ++e) {
    double X[8][3];
    cell_corners(M, e, X);
    double v = 0;
    for (int q2 = 0; q2 < m; ++q2)
      for (int q1 = 0; q1 < m; ++q1)
        for (int q0 = 0; q0 < m; ++q0) {
          const double xi[3] = {T.xq[q0], T.xq[q1], T.xq[q2]};
          double J[3][3];
          host_jacobian(X, xi, J);
          v += T.wq[q0] * T.wq[q1] * T.wq[q2] * std::fabs(host_det(J));
        }
    vol[e] = v;
  }
  const int n[3] = {nx, ny, nz};
  std::vector<double> gam;
  for (int d = 0; d < 3; ++d) {
    M.gamma_off[d] = (int64_t)gam.size();
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    const int64_t nfaces = (int64_t)(n[d] + 1) * n[t1] * n[t2];
    gam.resize(gam.size() + nfaces);
    for (int c2 = 0; c2 < n[t2]; ++c2)
      for (int c1 = 0; c1 < n[t1]; ++c1)
        for (int pl = 0; pl <= n[d]; ++pl) {
          // the face is side 0 of cell `hi` (pl < n_d) or side 1 of cell `lo` (pl > 0)
          int ch[3], cl[3];
          ch[d] = pl;
          cl[d] = pl - 1;
          ch[t1] = cl[t1] = c1;
          ch[t2] = cl[t2] = c2;
          const bool has_hi = pl < n[d], has_lo = pl > 0;
          const int64_t ehi = has_hi ? ch[0] + (int64_t)nx * (ch[1] + (int64_t)ny * ch[2]) : -1;
          const int64_t elo = has_lo ? cl[0] + (int64_t)nx * (cl[1] + (int64_t)ny * cl[2]) : -1;
          const int64_t eref = has_hi ? ehi : elo;
          const double side = has_hi ? 0.0 : 1.0;
          double X[8][3];
          cell_corners(M, eref, X);
          double area = 0;
          for (int qb = 0; qb < m; ++qb)
            for (int qa = 0; qa < m; ++qa) {
              double xi[3];
              xi[d] = side;
              xi[t1] = T.xq[qa];
              xi[t2] = T.xq[qb];
              double J[3][3];
              host_jacobian(X, xi, J);
              // |cof(J) e_d| = |det J| |row d of J^{-1}|
              const double det = host_det(J);
              double r[3];
              for (int k = 0; k < 3; ++k) {
                const int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
                const int d1 = (d + 1) % 3, d2 = (d + 2) % 3;
                r[k] = (J[k1][d1] * J[k2][d2] - J[k1][d2] * J[k2][d1]);  // cofactor C[k][d]
              }
              (void)det;
              area += T.wq[qa] * T.wq[qb] * std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
            }
          double vmin = 1e300;
          if (has_hi) vmin = std::min(vmin, vol[ehi]);
          if (has_lo) vmin = std::min(vmin, vol[elo]);
          gam[M.gamma_off[d] + pl + (int64_t)(n[d] + 1) * (c1 + (int64_t)n[t1] * c2)] = coef * area / vmin;
        }
  }
  if (hipMalloc(&M.d_vertices, sizeof(double) * M.vertices.size()) != hipSuccess ||
      hipMalloc(&M.d_gamma, sizeof(double) * gam.size()) != hipSuccess) {
    (void)hipGetLastError();
    throw std::runtime_error("device allocation failed (Stokes geometry)");
  }
  if (hipMemcpy(M.d_vertices, M.vertices.data(), sizeof(double) * M.vertices.size(), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(M.d_gamma, gam.data(), sizeof(double) * gam.size(), hipMemcpyHostToDevice) != hipSuccess)
    throw std::runtime_error("upload of the Stokes geometry failed");
}

hipError_t stokes_apply(const dg_mesh& M, const double* x, double* y, hipStream_t s) {
  StokesGeom g;
  g.vertices = M.d_vertices;
  g.gamma = M.d_gamma;
  for (int d = 0; d < 3; ++d) g.goff[d] = M.gamma_off[d];
  if (M.nelem > 0x7fffffff) return hipErrorInvalidValue;
  if (M.p == 4)
    hipLaunchKernelGGL(k_stokes_apply<4>, dim3((unsigned)M.nelem), dim3(NT), 0, s, x, y, M.st, g);
  else if (M.p == 3)
    hipLaunchKernelGGL(k_stokes_apply<3>, dim3((unsigned)M.nelem), dim3(NT), 0, s, x, y, M.st, g);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace dgi
