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

// Component c of the vector whose d-th entry is vd and whose two other entries,
// in increasing index order, are va and vb (selects; no indexed register arrays).
template <typename V>
__device__ __forceinline__ V place(int d, int c, V vd, V va, V vb) {
  if (c == 0) return d == 0 ? vd : va;
  if (c == 1) return d == 0 ? va : (d == 1 ? vd : vb);
  return d == 2 ? vd : vb;
}

// Index of pressure node (jd along d, ja along t1, jb along t2) in the cell block.
template <int KP>
__device__ __forceinline__ int pnode(int d, int jd, int ja, int jb) {
  return place(d, 0, jd, ja, jb) + KP * (place(d, 1, jd, ja, jb) + KP * place(d, 2, jd, ja, jb));
}

__device__ __forceinline__ void face_dirs(int d, int& t1, int& t2) {
  t1 = d == 0 ? 1 : 0;
  t2 = d == 2 ? 1 : 2;
}

template <int P>
__global__ void __launch_bounds__(NT) k_stokes_apply(const double* __restrict__ x, double* __restrict__ y,
                                                     const StokesArgs a, const StokesGeom geo) {
  constexpr int KP = P - 1;
  constexpr int N = P * P * P, NQ = KP * KP * KP, L = P * P;
  constexpr int NB = 3 * N + NQ;      // DOFs per cell
  constexpr int NF = 6 * L;           // face points of the cell
  constexpr int RA = (6 * NF > 10 * N) ? 6 * NF : 10 * N;
  // staging of the pressure contractions: cell stages s1 [P KP^2], s2 [P^2 KP] and
  // face-trace stages c1 [12 KP^2], c2 [12 P KP] live side by side; the test
  // stages (KP P^2 + 6 KP P + KP^2 P + 6 KP^2) reuse the space later. Both
  // run while the face coefficients are dead (before the faces' flux stage,
  // after the velocity test functions), so the staging shares their space.
  constexpr int TMP = P * KP * KP + P * P * KP + 12 * KP * KP + 12 * P * KP;
  static_assert(KP * P * P + 6 * KP * P + KP * KP * P + 6 * KP * KP <= TMP, "pressure staging");
  static_assert(TMP <= 9 * NF, "pressure staging inside the face coefficients");
  __shared__ double su[3 * N];        // velocity
  __shared__ double sp[NQ];           // pressure
  __shared__ double sX[24];           // own corners
  __shared__ double nX[6][24];        // neighbour corners
  __shared__ double npr[6][NQ];       // neighbour pressure
  __shared__ double spq[N];           // pressure at the quadrature points
  __shared__ double fpT[NF], fpN[NF]; // pressure traces (own, neighbour) at the face points
  __shared__ double regA[RA];         // faces: velocity traces fT[3][NF], fN[3][NF]; then cell residual sR[9][N], sRp[N]
  __shared__ double fcoef[9 * NF];    // fV, fRg, fJn (below); pressure staging `tmp` at other times
  __shared__ double fQ[NF];           // face coefficients of q
  double* fV = fcoef;                 // face coefficients of v_c
  double* fRg = fcoef + 3 * NF;       // face coefficients of grad v_c . nu
  double* fJn = fcoef + 6 * NF;       // J^{-1} nu at the face points
  double* tmp = fcoef;
  double* fT = regA;
  double* fN = regA + 3 * NF;
  double* sR = regA;
  double* sRp = regA + 9 * N;

  const int t = threadIdx.x;
  const int e = blockIdx.x;
  const int nx = a.n[0], ny = a.n[1];
  const int ec[3] = {e % nx, (e / nx) % ny, e / (nx * ny)};
  const int64_t base = (int64_t)e * NB;
  const int64_t estr[3] = {1, nx, (int64_t)nx * ny};
  unsigned hasn = 0;  // bit f: face f has a neighbour
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const int d = f >> 1, s = f & 1;
    const int c = ec[d] + (s ? 1 : -1);
    if (c >= 0 && c < a.n[d]) hasn |= 1u << f;
  }
  auto has_nb_of = [&](int f) { return ((hasn >> f) & 1u) != 0; };
  // runtime-direction helpers (selects instead of indexed register arrays)
  auto ecd = [&](int d) { return d == 0 ? ec[0] : (d == 1 ? ec[1] : ec[2]); };
  auto estrd = [&](int d) { return d == 0 ? estr[0] : (d == 1 ? estr[1] : estr[2]); };

  // ---- loads ---------------------------------------------------------------
  for (int i = t; i < 3 * N; i += NT) su[i] = x[base + i];
  for (int i = t; i < NQ; i += NT) sp[i] = x[base + 3 * N + i];
  load_corners(geo, a, ec[0], ec[1], ec[2], sX, t);
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    if (!has_nb_of(f)) continue;
    const int d = f >> 1, s = f & 1;
    int nc[3] = {ec[0], ec[1], ec[2]};
    nc[d] += s ? 1 : -1;
    load_corners(geo, a, nc[0], nc[1], nc[2], nX[f], t);
    const int64_t nb = (int64_t)e + (s ? estr[d] : -estr[d]);
    for (int i = t; i < NQ; i += NT) npr[f][i] = x[nb * NB + 3 * N + i];
  }
  __syncthreads();

  // ---- pressure by sum factorization: at the points, and face traces -------
  // cell: (A_p x A_p x A_p) P, one direction per stage
  double* s1 = tmp;              // [q0][j1][j2]
  double* s2 = tmp + P * KP * KP; // [q0][q1][j2]
  for (int i = t; i < P * KP * KP; i += NT) {
    const int q0 = i % P, j12 = i / P;
    double v = 0;
#pragma unroll
    for (int j0 = 0; j0 < KP; ++j0) v = fma(a.Ap[q0 * KP + j0], sp[j0 + KP * j12], v);
    s1[i] = v;
  }
  // faces, stage 1: contract the normal direction with e_p(side) (own: side s, neighbour: 1 - s)
  double* c1 = tmp + P * KP * KP + P * P * KP;  // [12][ja][jb]
  for (int i = t; i < 12 * KP * KP; i += NT) {
    const int fo = i / (KP * KP), r = i - fo * KP * KP;
    const int f = fo >> 1, o = fo & 1;  // o: 0 own, 1 neighbour
    const int d = f >> 1, s = f & 1;
    const int ja = r % KP, jb = r / KP;
    double v = 0;
    if (o == 0 || has_nb_of(f)) {
      const double* P_ = o ? npr[f] : sp;
      const int side = o ? 1 - s : s;
#pragma unroll
      for (int jd = 0; jd < KP; ++jd) v = fma(a.ep[side][jd], P_[pnode<KP>(d, jd, ja, jb)], v);
    }
    c1[i] = v;
  }
  __syncthreads();
  for (int i = t; i < P * P * KP; i += NT) {
    const int q0 = i % P, q1 = (i / P) % P, j2 = i / (P * P);
    double v = 0;
#pragma unroll
    for (int j1 = 0; j1 < KP; ++j1) v = fma(a.Ap[q1 * KP + j1], s1[q0 + P * (j1 + KP * j2)], v);
    s2[i] = v;
  }
  double* c2 = c1 + 12 * KP * KP;  // [12][pa][jb]
  for (int i = t; i < 12 * P * KP; i += NT) {
    const int fo = i / (P * KP), r = i - fo * P * KP;
    const int pa = r % P, jb = r / P;
    double v = 0;
#pragma unroll
    for (int ja = 0; ja < KP; ++ja) v = fma(a.Ap[pa * KP + ja], c1[fo * KP * KP + ja + KP * jb], v);
    c2[i] = v;
  }
  __syncthreads();
  for (int i = t; i < N; i += NT) {
    const int q01 = i % (P * P), q2 = i / (P * P);
    double v = 0;
#pragma unroll
    for (int j2 = 0; j2 < KP; ++j2) v = fma(a.Ap[q2 * KP + j2], s2[q01 + P * P * j2], v);
    spq[i] = v;
  }
  for (int i = t; i < 12 * L; i += NT) {
    const int fo = i / L, pt = i - fo * L;
    const int pa = pt % P, pb = pt / P;
    double v = 0;
#pragma unroll
    for (int jb = 0; jb < KP; ++jb) v = fma(a.Ap[pb * KP + jb], c2[fo * P * KP + pa + P * jb], v);
    const int f = fo >> 1, o = fo & 1;
    (o ? fpN : fpT)[f * L + pt] = v;
  }

  // ---- faces, phase 1: velocity traces and normal derivatives --------------
  double dnT[2][3], dnN[2][3];
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int fp = t + NT * r;
    if (fp >= NF) continue;
    const int f = fp / L, pt = fp - f * L;
    const int d = f >> 1, s = f & 1;
    const int pa = pt % P, pb = pt / P;
    const int off = d == 0 ? P * pa + L * pb : (d == 1 ? pa + L * pb : pa + P * pb);
    const int str = d == 0 ? 1 : (d == 1 ? P : L);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double u = 0, dn = 0;
#pragma unroll
      for (int j = 0; j < P; ++j) {
        const double v = su[c * N + off + j * str];
        u = fma(a.e[s][j], v, u);
        dn = fma(a.de[s][j], v, dn);
      }
      fT[c * NF + fp] = u;
      dnT[r][c] = dn;
    }
    if (has_nb_of(f)) {
      const int64_t nb = (int64_t)e + (s ? estrd(d) : -estrd(d));
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double u = 0, dn = 0;
#pragma unroll
        for (int j = 0; j < P; ++j) {
          const double v = x[nb * NB + c * N + off + j * str];
          u = fma(a.e[1 - s][j], v, u);
          dn = fma(a.de[1 - s][j], v, dn);
        }
        fN[c * NF + fp] = u;
        dnN[r][c] = dn;
      }
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        fN[c * NF + fp] = 0.0;
        dnN[r][c] = 0.0;
      }
    }
  }
  __syncthreads();

  // ---- faces, phase 2: flux at every face point ---------------------------
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int fp = t + NT * r;
    if (fp >= NF) continue;
    const int f = fp / L, pt = fp - f * L;
    const int d = f >> 1, s = f & 1;
    const int pa = pt % P, pb = pt / P;
    const bool has_nb = has_nb_of(f);
    const bool dir = (a.mask >> f) & 1u;
    if (!has_nb && !dir) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        fV[c * NF + fp] = 0.0;
        fRg[c * NF + fp] = 0.0;
        fJn[c * NF + fp] = 0.0;
      }
      fQ[fp] = 0.0;
      continue;
    }
    const int fb = f * L;
    // geometry at the face point from the own cell
    const double xs = (double)s, xa = a.xq[pa], xb = a.xq[pb];
    const double xi[3] = {place(d, 0, xs, xa, xb), place(d, 1, xs, xa, xb), place(d, 2, xs, xa, xb)};
    double J[3][3], Ji[3][3];
    jacobian(sX, xi, J);
    const double det = invert(J, Ji);
    // row d of J^{-1} (the gradient of xi_d): normal direction
    double rn[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) rn[k] = d == 0 ? Ji[0][k] : (d == 1 ? Ji[1][k] : Ji[2][k]);
    const double nn = sqrt(rn[0] * rn[0] + rn[1] * rn[1] + rn[2] * rn[2]);
    const double sg = s ? 1.0 : -1.0;
    const double nu[3] = {sg * rn[0] / nn, sg * rn[1] / nn, sg * rn[2] / nn};
    const double dA = fabs(det) * nn * a.w[pa] * a.w[pb];
    const double Jn[3] = {Ji[0][0] * nu[0] + Ji[0][1] * nu[1] + Ji[0][2] * nu[2],
                          Ji[1][0] * nu[0] + Ji[1][1] * nu[1] + Ji[1][2] * nu[2],
                          Ji[2][0] * nu[0] + Ji[2][1] * nu[1] + Ji[2][2] * nu[2]};
    // own full reference gradient along nu: normal part from phase 1, tangential
    // parts by D across the face points of the own trace
    double uT[3], gradT_n[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double ga = 0, gb = 0;
#pragma unroll
      for (int j = 0; j < P; ++j) {
        ga = fma(a.D[pa * P + j], fT[c * NF + fb + j + P * pb], ga);
        gb = fma(a.D[pb * P + j], fT[c * NF + fb + pa + P * j], gb);
      }
      const double dn = dnT[r][c];
      gradT_n[c] = Jn[0] * place(d, 0, dn, ga, gb) + Jn[1] * place(d, 1, dn, ga, gb) + Jn[2] * place(d, 2, dn, ga, gb);
      uT[c] = fT[c * NF + fp];
    }
    const double pT = fpT[fp];
    const int ct1 = d == 0 ? ec[1] : ec[0], ct2 = d == 2 ? ec[1] : ec[2];
    const int nd = d == 0 ? a.n[0] : (d == 1 ? a.n[1] : a.n[2]);
    const int nt1 = d == 0 ? a.n[1] : a.n[0];
    const int64_t goff = d == 0 ? geo.goff[0] : (d == 1 ? geo.goff[1] : geo.goff[2]);
    const double gam = geo.gamma[goff + (ecd(d) + s) + (int64_t)(nd + 1) * (ct1 + (int64_t)nt1 * ct2)];
    double Rv[3], Rg[3], Rq = 0.0;
    if (has_nb) {
      const double xn[3] = {place(d, 0, 1.0 - xs, xa, xb), place(d, 1, 1.0 - xs, xa, xb),
                            place(d, 2, 1.0 - xs, xa, xb)};
      double JN[3][3], JiN[3][3];
      jacobian(nX[f], xn, JN);
      invert(JN, JiN);
      const double JnN[3] = {JiN[0][0] * nu[0] + JiN[0][1] * nu[1] + JiN[0][2] * nu[2],
                             JiN[1][0] * nu[0] + JiN[1][1] * nu[1] + JiN[1][2] * nu[2],
                             JiN[2][0] * nu[0] + JiN[2][1] * nu[1] + JiN[2][2] * nu[2]};
      const double pN = fpN[fp];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double ga = 0, gb = 0;
#pragma unroll
        for (int j = 0; j < P; ++j) {
          ga = fma(a.D[pa * P + j], fN[c * NF + fb + j + P * pb], ga);
          gb = fma(a.D[pb * P + j], fN[c * NF + fb + pa + P * j], gb);
        }
        const double dn = dnN[r][c];
        const double gradN_n = JnN[0] * place(d, 0, dn, ga, gb) + JnN[1] * place(d, 1, dn, ga, gb) +
                               JnN[2] * place(d, 2, dn, ga, gb);
        const double jump = uT[c] - fN[c * NF + fp];
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
      fV[c * NF + fp] = Rv[c];
      fRg[c * NF + fp] = Rg[c];
      fJn[c * NF + fp] = Jn[c];
    }
    fQ[fp] = Rq;
  }
  __syncthreads();

  // ---- cell terms at the points (Algorithm 1, parts 1 and 2) ---------------
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
    }
    const double pq = spq[i];
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
      int t1, t2;
      face_dirs(d, t1, t2);
      const int j = ii[d], pa = ii[t1], pb = ii[t2];
      const int fb = f * L;
      const double es = a.e[s][j], des = a.de[s][j];
      const int fpt = fb + pa + P * pb;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double* Rg = fRg + c * NF;
        double tv = fV[c * NF + fpt];
#pragma unroll
        for (int q = 0; q < P; ++q) {
          const int f1 = fb + q + P * pb, f2 = fb + pa + P * q;
          tv = fma(a.D[q * P + pa], Rg[f1] * fJn[t1 * NF + f1], tv);
          tv = fma(a.D[q * P + pb], Rg[f2] * fJn[t2 * NF + f2], tv);
        }
        acc[c] = fma(es, tv, fma(des, Rg[fpt] * fJn[d * NF + fpt], acc[c]));
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) y[base + c * N + i] = acc[c];
  }
  // pressure test functions by sum factorization: cell (A_p^T x3) R_p and, per
  // face, e_p(s) (x) (A_p^T x A_p^T) Q_f; the staging overwrites the face
  // coefficients, read above by every thread
  __syncthreads();
  double* t1b = tmp;                      // [j0][q1][q2]
  double* u1 = tmp + KP * P * P;          // [f][ja][pb]
  for (int i = t; i < KP * P * P; i += NT) {
    const int j0 = i % KP, q12 = i / KP;
    double v = 0;
#pragma unroll
    for (int q0 = 0; q0 < P; ++q0) v = fma(a.Ap[q0 * KP + j0], sRp[q0 + P * q12], v);
    t1b[i] = v;
  }
  for (int i = t; i < 6 * KP * P; i += NT) {
    const int f = i / (KP * P), r = i - f * KP * P;
    const int ja = r % KP, pb = r / KP;
    double v = 0;
#pragma unroll
    for (int pa = 0; pa < P; ++pa) v = fma(a.Ap[pa * KP + ja], fQ[f * L + pa + P * pb], v);
    u1[i] = v;
  }
  __syncthreads();
  double* t2b = u1 + 6 * KP * P;          // [j0][j1][q2]
  double* u2 = t2b + KP * KP * P;         // [f][ja][jb]
  for (int i = t; i < KP * KP * P; i += NT) {
    const int j0 = i % KP, j1 = (i / KP) % KP, q2 = i / (KP * KP);
    double v = 0;
#pragma unroll
    for (int q1 = 0; q1 < P; ++q1) v = fma(a.Ap[q1 * KP + j1], t1b[j0 + KP * (q1 + P * q2)], v);
    t2b[i] = v;
  }
  for (int i = t; i < 6 * KP * KP; i += NT) {
    const int f = i / (KP * KP), r = i - f * KP * KP;
    const int ja = r % KP, jb = r / KP;
    double v = 0;
#pragma unroll
    for (int pb = 0; pb < P; ++pb) v = fma(a.Ap[pb * KP + jb], u1[f * KP * P + ja + KP * pb], v);
    u2[i] = v;
  }
  __syncthreads();
  for (int i = t; i < NQ; i += NT) {
    const int jj[3] = {i % KP, (i / KP) % KP, i / (KP * KP)};
    double v = 0;
#pragma unroll
    for (int q2 = 0; q2 < P; ++q2) v = fma(a.Ap[q2 * KP + jj[2]], t2b[jj[0] + KP * (jj[1] + KP * q2)], v);
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      const int d = f >> 1, s = f & 1;
      int t1, t2;
      face_dirs(d, t1, t2);
      v = fma(a.ep[s][jj[d]], u2[f * KP * KP + jj[t1] + KP * jj[t2]], v);
    }
    y[base + 3 * N + i] = v;
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
