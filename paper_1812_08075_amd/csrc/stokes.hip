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
// vertices, so the geometry is evaluated at every quadrature point
// (Algorithm 1, part 2 with the geometry mu_T).
//
// Geometry. The trilinear map of a cell is written in monomial form,
// x(xi) = a0 + a1 xi0 + a2 xi1 + a3 xi2 + a4 xi0 xi1 + a5 xi0 xi2 + a6 xi1 xi2
// + a7 xi0 xi1 xi2, with a1..a7 per cell computed once at setup from the
// corners; a column of J is then bilinear in the two other coordinates (three
// multiply-adds per entry). J^{-1} is never formed: with rho_a the cross
// product of the two other columns (rho_a = det J grad xi_a), the cell term
// at a point is (w / |det J|) (rho_a . rho_b) d_b u_c - p w sgn(det J)
// rho_a[c] and the divergence w sgn(det J) rho_a[c] d_a u_c. On a face of
// normal direction d both cells share the tangential columns t1, t2 of J (the
// face is the bilinear image of its four vertices), so n = t1 x t2, the area
// element |n| w_a w_b and the outward unit normal are common to both sides,
// and only the normal column differs; grad xi . nu follows from the Gram
// entries of (t1, t2) and the dot products of the normal column with them.
//
// Work decomposition: one wave (64 threads) per cell.
//  1. pressure: the cell's pressure at the points and the average of the two
//     pressure traces at every face point, by sum factorization.
//  2. volume: thread = quadrature point. The nine reference derivatives
//     d_a u_c are 1D contractions with D along a (Algorithm 1, part 1), then
//     the pointwise stage above; the transposed contractions (part 3) give
//     the cell part of the velocity residual of node i, kept in registers.
//  3. faces, in rounds of whole faces (64 points): thread = face point. The
//     own trace of u and its normal derivative are the line's dot products
//     with l_j(s), l'_j(s) (normal direction first, Section 2.2); the
//     neighbour's come from its line in global memory; tangential
//     derivatives are D-contractions across the face points. The flux gives,
//     per point, the coefficient of the test function's value and of its
//     gradient along nu; the tangential parts of the latter are contracted
//     across the face points (D^T) once per point, and every node then adds
//     l_j(s) and l'_j(s) times its face's two coefficients. At k = 3 a face's
//     16 points fill one 16-lane row, so both contractions across the face
//     points take their operands from the neighbouring lanes by DPP; at k = 2
//     (9 points per face) they go through LDS.
//  4. pressure test functions: the cell residual and the faces' [u].n terms
//     through A_p^T (x) A_p^T (x) A_p^T and e_p (x) A_p^T (x) A_p^T.
// Every output entry has one writer; no atomics; bitwise reproducible.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <stdexcept>
#include <vector>

#include "internal.h"
#include "lane_dpp.h"

namespace dgi {
namespace {

constexpr int NT = 64;
constexpr int GEO = 24;  // doubles per cell of the geometry table: a1..a7, 3 components each, padded

struct StokesGeom {
  const uint32_t* order;  // cell of every block
  const double* cellgeo;  // GEO doubles per cell: a_m component k at 3 (m - 1) + k
  const double* gamma;    // per-face penalties, direction d at offset goff[d]
  int64_t goff[3];
};

// Offsets in a cell's geometry record: the xi_b coefficient and the xi_b xi_o one.
__device__ __forceinline__ int g_lin(int b) { return 3 * b; }
__device__ __forceinline__ int g_pair(int b, int o) { return 9 + 3 * (b + o - 1); }
constexpr int G_TRI = 18;

// Index of pressure node (jd along d, ja along t1, jb along t2) in the cell block.
template <int KP>
__device__ __forceinline__ int pnode(int d, int jd, int ja, int jb) {
  const int i0 = d == 0 ? jd : ja, i1 = d == 1 ? jd : (d == 0 ? ja : jb), i2 = d == 2 ? jd : jb;
  return i0 + KP * (i1 + KP * i2);
}

__device__ __forceinline__ void face_dirs(int d, int& t1, int& t2) {
  t1 = d == 0 ? 1 : 0;
  t2 = d == 2 ? 1 : 2;
}

__device__ __forceinline__ void cross(const double* a, const double* b, double* c) {
  c[0] = fma(a[1], b[2], -a[2] * b[1]);
  c[1] = fma(a[2], b[0], -a[0] * b[2]);
  c[2] = fma(a[0], b[1], -a[1] * b[0]);
}

__device__ __forceinline__ double dot3(const double* a, const double* b) {
  return fma(a[0], b[0], fma(a[1], b[1], a[2] * b[2]));
}

// 1/x and 1/sqrt(x): the hardware estimate refined by two Newton steps
// (each squares the relative error) to the last bits of FP64.
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}

__device__ __forceinline__ double rsqrt_nr(double x) {
  double r = __builtin_amdgcn_rsq(x);
  r = fma(0.5 * r, fma(-x * r, r, 1.0), r);
  return fma(0.5 * r, fma(-x * r, r, 1.0), r);
}

// Per face of the cell (FG doubles): tangential columns t1 = al1 + be xi_t2,
// t2 = al2 + be xi_t1; the own normal column and the neighbour's, each
// g0 + g1 xi_t1 + g2 xi_t2 + g3 xi_t1 xi_t2 (component k of coefficient m
// at 3 m + k).
constexpr int FG = 33;
constexpr int FG_AL1 = 0, FG_AL2 = 3, FG_BE = 6, FG_OWN = 9, FG_NB = 21;

template <int P>
__device__ __forceinline__ void stokes_cell(const double* __restrict__ x, double* __restrict__ y, const StokesArgs& a,
                                            const StokesGeom& geo) {
  constexpr int KP = P - 1;
  constexpr int N = P * P * P, NQ = KP * KP * KP, L = P * P;
  constexpr int NB = 3 * N + NQ;                  // DOFs per cell
  constexpr int NF = 6 * L;                       // face points of the cell
  constexpr int FPR = NT / L;                     // whole faces per round
  constexpr int NR = (6 + FPR - 1) / FPR;         // rounds
  constexpr int RP = (FPR < 6 ? FPR : 6) * L;     // points of a full round
  static_assert(N <= NT && FPR >= 1, "one volume point and at least one face per thread round");
  // staging area X: pressure contractions (start), the cell residual sR[9][N]
  // (volume), two quantities of 3 components per face point of a round
  // (faces), pressure test contractions (end); the cell's pressure nodes and
  // then its pressure residual at the points live at XR
  constexpr int TMP0 = P * KP * KP + P * P * KP + 12 * KP * KP + 12 * P * KP;
  constexpr int TMP1 = KP * P * P + 6 * KP * P + KP * KP * P + 6 * KP * KP;
  constexpr int XR = (9 * N > 6 * RP) ? 9 * N : 6 * RP;
  static_assert(TMP0 <= XR && TMP1 <= XR && NQ <= N, "staging");
  __shared__ double tD[P * P], tE[2][P], tDE[2][P], tW[P], tX[P], tAp[P * KP], tEp[2][KP];
  __shared__ double su[3 * N];        // velocity
  __shared__ double fpA[NF];          // {p} at interior face points, p at boundary ones
  __shared__ double fQ_spq[NF > N ? NF : N];  // pressure at the points (volume); face coefficients of q (faces)
  __shared__ double fgeo[6 * FG];     // face geometry
  __shared__ int sNb[6];              // the cell across face f, -1 on the boundary
  __shared__ double X[XR + N];
  double* spq = fQ_spq;
  double* fQ = fQ_spq;
  double* spl = X + XR;               // the cell's pressure nodes, then its pressure residual sRp
  double* sRp = X + XR;

  const int t = threadIdx.x;
  const int e = (int)geo.order[blockIdx.x];  // the cell of this block (XCD-aware sweep table)
  const int nx = a.n[0], ny = a.n[1];
  const int ec[3] = {e % nx, (e / nx) % ny, e / (nx * ny)};
  const int64_t base = (int64_t)e * NB;
  unsigned hasn = 0;  // bit f: face f has a neighbour
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const int d = f >> 1, s = f & 1;
    const int c = ec[d] + (s ? 1 : -1);
    if (c >= 0 && c < a.n[d]) hasn |= 1u << f;
  }
  auto has_nb_of = [&](int f) { return ((hasn >> f) & 1u) != 0; };
  auto ecd = [&](int d) { return d == 0 ? ec[0] : (d == 1 ? ec[1] : ec[2]); };
  // the cell across face f (lane-varying f: a chain of selects of uniform values)
  const int nxy = nx * ny;
  auto nb_of = [&](int f) -> int64_t {
    int v = e + nxy;
    v = f == 4 ? e - nxy : v;
    v = f == 3 ? e + nx : v;
    v = f == 2 ? e - nx : v;
    v = f == 1 ? e + 1 : v;
    v = f == 0 ? e - 1 : v;
    return v;
  };
  const double* __restrict__ cg = geo.cellgeo + (int64_t)e * GEO;

  // ---- loads: every global load of the set-up is issued before the first
  // LDS write, so that their latencies overlap
  constexpr int NRU = (3 * N + NT - 1) / NT;
  double vu[NRU];
#pragma unroll
  for (int r = 0; r < NRU; ++r) {
    const int i = t + r * NT;
    vu[r] = i < 3 * N ? x[base + i] : 0.0;
  }
  const double vp = t < NQ ? x[base + 3 * N + t] : 0.0;
  const int tp = t < P ? t : 0, tq = t < KP ? t : 0;
  const double vD = a.D[t < P * P ? t : 0], vAp = a.Ap[t < P * KP ? t : 0];
  const double ve0 = a.e[0][tp], ve1 = a.e[1][tp], vd0 = a.de[0][tp], vd1 = a.de[1][tp];
  const double vw = a.w[tp], vx = a.xq[tp], vq0 = a.ep[0][tq], vq1 = a.ep[1][tq];
  // face geometry: thread = (face, component) for t < 18
  const int gf = t < 18 ? t / 3 : 0, gk = t - 3 * gf;
  const int gd = gf >> 1, gs = gf & 1;
  int g1, g2;
  face_dirs(gd, g1, g2);
  double go[7], gq[4] = {0.0, 0.0, 0.0, 0.0};
  if (t < 18) {
    go[0] = cg[g_lin(g1) + gk];
    go[1] = cg[g_pair(g1, gd) + gk];
    go[2] = cg[g_lin(g2) + gk];
    go[3] = cg[g_pair(g2, gd) + gk];
    go[4] = cg[g_pair(g1, g2) + gk];
    go[5] = cg[g_lin(gd) + gk];
    go[6] = cg[G_TRI + gk];
    if (has_nb_of(gf)) {
      const double* __restrict__ gn = geo.cellgeo + nb_of(gf) * GEO;
      gq[0] = gn[g_lin(gd) + gk];
      gq[1] = gn[g_pair(gd, g1) + gk];
      gq[2] = gn[g_pair(gd, g2) + gk];
      gq[3] = gn[G_TRI + gk];
    }
  }
  // the neighbours' pressure nodes on the shared faces: thread = (face, ja, jb)
  // for t < 6 KP^2, the KP nodes along the face normal
  const int pf = t < 6 * KP * KP ? t / (KP * KP) : 0, pr = t - pf * KP * KP;
  double vnp[KP];
#pragma unroll
  for (int jd = 0; jd < KP; ++jd) vnp[jd] = 0.0;
  if (t < 6 * KP * KP && has_nb_of(pf)) {
    const double* __restrict__ pn = x + nb_of(pf) * NB + 3 * N;
#pragma unroll
    for (int jd = 0; jd < KP; ++jd) vnp[jd] = pn[pnode<KP>(pf >> 1, jd, pr % KP, pr / KP)];
  }
  if (t < 6) sNb[t] = has_nb_of(t) ? (int)nb_of(t) : -1;
#pragma unroll
  for (int r = 0; r < NRU; ++r) {
    const int i = t + r * NT;
    if (i < 3 * N) su[i] = vu[r];
  }
  if (t < NQ) spl[t] = vp;
  if (t < P * P) tD[t] = vD;
  if (t < P * KP) tAp[t] = vAp;
  if (t < P) {
    tE[0][t] = ve0;
    tE[1][t] = ve1;
    tDE[0][t] = vd0;
    tDE[1][t] = vd1;
    tW[t] = vw;
    tX[t] = vx;
  }
  if (t < KP) {
    tEp[0][t] = vq0;
    tEp[1][t] = vq1;
  }
  if (t < 18) {
    const double sd = (double)gs;
    double* fg = fgeo + gf * FG;
    fg[FG_AL1 + gk] = fma(sd, go[1], go[0]);
    fg[FG_AL2 + gk] = fma(sd, go[3], go[2]);
    fg[FG_BE + gk] = fma(sd, go[6], go[4]);
    fg[FG_OWN + gk] = go[5];
    fg[FG_OWN + 3 + gk] = go[1];  // the xi_d xi_t1 and xi_d xi_t2 coefficients
    fg[FG_OWN + 6 + gk] = go[3];
    fg[FG_OWN + 9 + gk] = go[6];
#pragma unroll
    for (int m = 0; m < 4; ++m) fg[FG_NB + 3 * m + gk] = gq[m];
  }
  __syncthreads();

  // ---- 1. pressure by sum factorization: at the points, and face traces -----
  {
    double* s1 = X;                       // [q0][j1][j2]
    double* s2 = s1 + P * KP * KP;        // [q0][q1][j2]
    double* c1 = s2 + P * P * KP;         // [12][ja][jb]: (face, own / neighbour)
    double* c2 = c1 + 12 * KP * KP;       // [12][pa][jb]
    for (int i = t; i < P * KP * KP; i += NT) {
      const int q0 = i % P, j12 = i / P;
      double v = 0;
#pragma unroll
      for (int j0 = 0; j0 < KP; ++j0) v = fma(tAp[q0 * KP + j0], spl[j0 + KP * j12], v);
      s1[i] = v;
    }
    // faces: contract the normal direction with e_p(side) (own: side s, neighbour: 1 - s)
    if (t < 6 * KP * KP) {
      const int d = pf >> 1, s = pf & 1;
      double v = 0, vn = 0;
#pragma unroll
      for (int jd = 0; jd < KP; ++jd) {
        v = fma(tEp[s][jd], spl[pnode<KP>(d, jd, pr % KP, pr / KP)], v);
        vn = fma(tEp[1 - s][jd], vnp[jd], vn);
      }
      c1[(2 * pf) * KP * KP + pr] = v;
      c1[(2 * pf + 1) * KP * KP + pr] = vn;
    }
    __syncthreads();
    for (int i = t; i < P * P * KP; i += NT) {
      const int q0 = i % P, q1 = (i / P) % P, j2 = i / (P * P);
      double v = 0;
#pragma unroll
      for (int j1 = 0; j1 < KP; ++j1) v = fma(tAp[q1 * KP + j1], s1[q0 + P * (j1 + KP * j2)], v);
      s2[i] = v;
    }
    for (int i = t; i < 12 * P * KP; i += NT) {
      const int fo = i / (P * KP), r = i - fo * P * KP;
      const int pa = r % P, jb = r / P;
      double v = 0;
#pragma unroll
      for (int ja = 0; ja < KP; ++ja) v = fma(tAp[pa * KP + ja], c1[fo * KP * KP + ja + KP * jb], v);
      c2[i] = v;
    }
    __syncthreads();
    for (int i = t; i < N; i += NT) {
      const int q01 = i % (P * P), q2 = i / (P * P);
      double v = 0;
#pragma unroll
      for (int j2 = 0; j2 < KP; ++j2) v = fma(tAp[q2 * KP + j2], s2[q01 + P * P * j2], v);
      spq[i] = v;
    }
    for (int i = t; i < NF; i += NT) {
      const int f = i / L, pt = i - f * L;
      const int pa = pt % P, pb = pt / P;
      double vo = 0, vn = 0;
#pragma unroll
      for (int jb = 0; jb < KP; ++jb) {
        vo = fma(tAp[pb * KP + jb], c2[(2 * f) * P * KP + pa + P * jb], vo);
        vn = fma(tAp[pb * KP + jb], c2[(2 * f + 1) * P * KP + pa + P * jb], vn);
      }
      fpA[i] = has_nb_of(f) ? 0.5 * (vo + vn) : vo;
    }
    __syncthreads();
  }

  // ---- 2. cell terms at the points (Algorithm 1, parts 1 and 2) -------------
  double* sR = X;
  if (t < N) {
    const int i = t;
    const int i0 = i % P, i1 = (i / P) % P, i2 = i / L;
    double g[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) g[c][0] = g[c][1] = g[c][2] = 0.0;
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const double d0 = tD[i0 * P + j], d1 = tD[i1 * P + j], d2 = tD[i2 * P + j];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double* uc = su + c * N;
        g[c][0] = fma(d0, uc[j + P * i1 + L * i2], g[c][0]);
        g[c][1] = fma(d1, uc[i0 + P * j + L * i2], g[c][1]);
        g[c][2] = fma(d2, uc[i0 + P * i1 + L * j], g[c][2]);
      }
    }
    const double x0 = tX[i0], x1 = tX[i1], x2 = tX[i2];
    const double x01 = x0 * x1, x02 = x0 * x2, x12 = x1 * x2;
    double c0[3], c1[3], c2[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      c0[k] = fma(cg[G_TRI + k], x12, fma(cg[g_pair(0, 2) + k], x2, fma(cg[g_pair(0, 1) + k], x1, cg[g_lin(0) + k])));
      c1[k] = fma(cg[G_TRI + k], x02, fma(cg[g_pair(1, 2) + k], x2, fma(cg[g_pair(0, 1) + k], x0, cg[g_lin(1) + k])));
      c2[k] = fma(cg[G_TRI + k], x01, fma(cg[g_pair(1, 2) + k], x1, fma(cg[g_pair(0, 2) + k], x0, cg[g_lin(2) + k])));
    }
    double r0[3], r1[3], r2[3];
    cross(c1, c2, r0);
    cross(c2, c0, r1);
    cross(c0, c1, r2);
    const double det = dot3(c0, r0);
    const double wq = tW[i0] * tW[i1] * tW[i2];
    const double sc = wq * recip(fabs(det));
    const double wp = det < 0.0 ? -wq : wq;  // w sgn(det J)
    const double G00 = sc * dot3(r0, r0), G11 = sc * dot3(r1, r1), G22 = sc * dot3(r2, r2);
    const double G01 = sc * dot3(r0, r1), G02 = sc * dot3(r0, r2), G12 = sc * dot3(r1, r2);
    const double pw = spq[i] * wp;
    double div = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double ga = g[c][0], gb = g[c][1], gc = g[c][2];
      sR[(3 * c + 0) * N + i] = fma(G00, ga, fma(G01, gb, fma(G02, gc, -pw * r0[c])));
      sR[(3 * c + 1) * N + i] = fma(G01, ga, fma(G11, gb, fma(G12, gc, -pw * r1[c])));
      sR[(3 * c + 2) * N + i] = fma(G02, ga, fma(G12, gb, fma(G22, gc, -pw * r2[c])));
      div = fma(r0[c], ga, fma(r1[c], gb, fma(r2[c], gc, div)));
    }
    sRp[i] = -wp * div;
  }
  __syncthreads();

  // node of the thread for the test functions
  const int n0 = t % P, n1 = (t / P) % P, n2 = t / L;
  double acc[3] = {0.0, 0.0, 0.0};
  if (t < N) {  // cell terms, part 3
#pragma unroll
    for (int q = 0; q < P; ++q) {
      const double d0 = tD[q * P + n0], d1 = tD[q * P + n1], d2 = tD[q * P + n2];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        acc[c] = fma(d0, sR[(3 * c + 0) * N + q + P * n1 + L * n2], acc[c]);
        acc[c] = fma(d1, sR[(3 * c + 1) * N + n0 + P * q + L * n2], acc[c]);
        acc[c] = fma(d2, sR[(3 * c + 2) * N + n0 + P * n1 + L * q], acc[c]);
      }
    }
  }
  __syncthreads();

  // ---- 3. faces, in rounds of whole faces ----------------------------------
#pragma unroll
  for (int rd = 0; rd < NR; ++rd) {
    const int f = rd * FPR + t / L, pt = t % L;
    const bool valid = t < FPR * L && f < 6;
    const int d = f >> 1, s = f & 1;
    const int pa = pt % P, pb = pt / P;
    const int lb = (t / L) * L;  // first point of the thread's face in the round
    double* sT = X;               // own velocity traces [3][RP]
    double* sN = X + 3 * RP;      // neighbour's
    // k = 3: the tangential derivatives of the traces come from the face's
    // other lanes (DPP) instead of LDS reads along the face's lines
    constexpr bool LANES = P == 4;
    // row_ror:n gives lane i the value of lane i - n (mod 16) of its row, so
    // row_rot<4k> brings the value of point (pa, pb - k mod 4)
    int pbs[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) pbs[k] = (pb - k) & 3;
    double dnT[3] = {0.0, 0.0, 0.0}, dnN[3] = {0.0, 0.0, 0.0};
    const bool has_nb = valid && has_nb_of(f);
    if (valid) {
      const int off = d == 0 ? P * pa + L * pb : (d == 1 ? pa + L * pb : pa + P * pb);
      const int str = d == 0 ? 1 : (d == 1 ? P : L);
      double es[P], ds[P];
#pragma unroll
      for (int j = 0; j < P; ++j) {
        es[j] = tE[s][j];
        ds[j] = tDE[s][j];
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double u = 0, dn = 0;
#pragma unroll
        for (int j = 0; j < P; ++j) {
          const double v = su[c * N + off + j * str];
          u = fma(es[j], v, u);
          dn = fma(ds[j], v, dn);
        }
        sT[c * RP + t] = u;
        dnT[c] = dn;
      }
      if (has_nb) {
#pragma unroll
        for (int j = 0; j < P; ++j) {
          es[j] = tE[1 - s][j];
          ds[j] = tDE[1 - s][j];
        }
        const double* __restrict__ xn = x + (int64_t)sNb[f] * NB + off;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          double u = 0, dn = 0;
#pragma unroll
          for (int j = 0; j < P; ++j) {
            const double v = xn[c * N + j * str];
            u = fma(es[j], v, u);
            dn = fma(ds[j], v, dn);
          }
          sN[c * RP + t] = u;
          dnN[c] = dn;
        }
      } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) sN[c * RP + t] = 0.0;
      }
    }
    __syncthreads();

    // flux at the face point
    double Rv[3] = {0.0, 0.0, 0.0}, G[3] = {0.0, 0.0, 0.0}, RJ1[3] = {0.0, 0.0, 0.0}, RJ2[3] = {0.0, 0.0, 0.0};
    if (valid) {
      const int fp = f * L + pt;
      const bool dir = (a.mask >> f) & 1u;
      double Rq = 0.0;
      if (has_nb || dir) {
        const double* fg = fgeo + f * FG;
        const double xa = tX[pa], xb = tX[pb], xab = xa * xb;
        double ct1[3], ct2[3], cd[3], cn[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          ct1[k] = fma(fg[FG_BE + k], xb, fg[FG_AL1 + k]);
          ct2[k] = fma(fg[FG_BE + k], xa, fg[FG_AL2 + k]);
          cd[k] = fma(fg[FG_OWN + 9 + k], xab,
                      fma(fg[FG_OWN + 6 + k], xb, fma(fg[FG_OWN + 3 + k], xa, fg[FG_OWN + k])));
        }
        double n[3];
        cross(ct1, ct2, n);
        const double g11 = dot3(ct1, ct1), g22 = dot3(ct2, ct2), g12 = dot3(ct1, ct2);
        const double nn2 = dot3(n, n);
        const double detL = dot3(cd, n);
        // the neighbour's normal column (its tangential ones are the own)
        double detN = 1.0;
        if (has_nb) {
#pragma unroll
          for (int k = 0; k < 3; ++k)
            cn[k] = fma(fg[FG_NB + 9 + k], xab, fma(fg[FG_NB + 6 + k], xb, fma(fg[FG_NB + 3 + k], xa, fg[FG_NB + k])));
          detN = dot3(cn, n);
        }
        const double sg = (s ? 1.0 : -1.0) * (detL < 0.0 ? -1.0 : 1.0);
        const double rs = rsqrt_nr(nn2), srs = sg * rs;  // 1 / |n|, with the orientation
        const double z = recip(detL * detN);
        const double nu[3] = {srs * n[0], srs * n[1], srs * n[2]};
        const double dA = nn2 * rs * tW[pa] * tW[pb];
        // grad xi_(d, t1, t2) . nu of the own cell
        const double ka = srs * detN * z;
        const double q1 = dot3(cd, ct1), q2 = dot3(cd, ct2);
        const double Jd = ka * nn2, J1 = ka * fma(g12, q2, -g22 * q1), J2 = ka * fma(g12, q1, -g11 * q2);
        // own normal derivative: tangential parts by D across the face points
        double gT[3], uT[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          double ga = 0, gb = 0;
          if constexpr (LANES) {
            uT[c] = sT[c * RP + t];
            grid4_rows(tD, pa, pb, uT[c], ga, gb);
          } else {
#pragma unroll
            for (int j = 0; j < P; ++j) {
              ga = fma(tD[pa * P + j], sT[c * RP + lb + j + P * pb], ga);
              gb = fma(tD[pb * P + j], sT[c * RP + lb + pa + P * j], gb);
            }
            uT[c] = sT[c * RP + t];
          }
          gT[c] = fma(Jd, dnT[c], fma(J1, ga, J2 * gb));
        }
        const double pA = fpA[fp];
        int t1, t2;
        face_dirs(d, t1, t2);
        const int ct1i = ecd(t1), ct2i = ecd(t2);
        const int nd = a.n[d], nt1 = a.n[t1];
        const int64_t goff = d == 0 ? geo.goff[0] : (d == 1 ? geo.goff[1] : geo.goff[2]);
        const double gam = geo.gamma[goff + (ecd(d) + s) + (int64_t)(nd + 1) * (ct1i + (int64_t)nt1 * ct2i)];
        double Rg[3];
        if (has_nb) {
          const double kb = srs * detL * z;
          const double p1 = dot3(cn, ct1), p2 = dot3(cn, ct2);
          const double Nd = kb * nn2, N1 = kb * fma(g12, p2, -g22 * p1), N2 = kb * fma(g12, p1, -g11 * p2);
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            double ga = 0, gb = 0, uN;
            if constexpr (LANES) {
              uN = sN[c * RP + t];
              grid4_rows(tD, pa, pb, uN, ga, gb);
            } else {
#pragma unroll
              for (int j = 0; j < P; ++j) {
                ga = fma(tD[pa * P + j], sN[c * RP + lb + j + P * pb], ga);
                gb = fma(tD[pb * P + j], sN[c * RP + lb + pa + P * j], gb);
              }
              uN = sN[c * RP + t];
            }
            const double gN = fma(Nd, dnN[c], fma(N1, ga, N2 * gb));
            const double jump = uT[c] - uN;
            Rv[c] = dA * (fma(-0.5, gT[c] + gN, gam * jump) + pA * nu[c]);
            Rg[c] = dA * 0.5 * a.theta * jump;
            Rq = fma(dA * 0.5 * jump, nu[c], Rq);
          }
        } else {
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            Rv[c] = dA * (fma(gam, uT[c], -gT[c]) + pA * nu[c]);
            Rg[c] = dA * a.theta * uT[c];
            Rq = fma(dA * uT[c], nu[c], Rq);
          }
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          G[c] = Rg[c] * Jd;
          RJ1[c] = Rg[c] * J1;
          RJ2[c] = Rg[c] * J2;
        }
      }
      fQ[fp] = Rq;
    }
    __syncthreads();
    double* sJ1 = X;            // Rg (grad xi_t1 . nu) [3][RP]
    double* sJ2 = X + 3 * RP;   // Rg (grad xi_t2 . nu)
    if (!LANES && valid) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        sJ1[c * RP + t] = RJ1[c];
        sJ2[c * RP + t] = RJ2[c];
      }
    }
    __syncthreads();
    // coefficient of the test function's value: Rv plus the tangential parts
    // of the gradient term, contracted across the face points
    if (valid) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double v = Rv[c];
        if constexpr (LANES) {
          v = fma(tD[0 * 4 + pa], quad_bcast<0>(RJ1[c]), v);
          v = fma(tD[pbs[0] * 4 + pb], RJ2[c], v);
          v = fma(tD[1 * 4 + pa], quad_bcast<1>(RJ1[c]), v);
          v = fma(tD[pbs[1] * 4 + pb], row_rot<4>(RJ2[c]), v);
          v = fma(tD[2 * 4 + pa], quad_bcast<2>(RJ1[c]), v);
          v = fma(tD[pbs[2] * 4 + pb], row_rot<8>(RJ2[c]), v);
          v = fma(tD[3 * 4 + pa], quad_bcast<3>(RJ1[c]), v);
          v = fma(tD[pbs[3] * 4 + pb], row_rot<12>(RJ2[c]), v);
        } else {
#pragma unroll
          for (int q = 0; q < P; ++q) {
            v = fma(tD[q * P + pa], sJ1[c * RP + lb + q + P * pb], v);
            v = fma(tD[q * P + pb], sJ2[c * RP + lb + pa + P * q], v);
          }
        }
        Rv[c] = v;
      }
    }
    __syncthreads();
    double* sV = X;            // value coefficient [3][RP]
    double* sG = X + 3 * RP;   // normal-derivative coefficient
    if (valid) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        sV[c * RP + t] = Rv[c];
        sG[c * RP + t] = G[c];
      }
    }
    __syncthreads();
    if (t < N) {
#pragma unroll
      for (int lf = 0; lf < FPR; ++lf) {
        const int ff = rd * FPR + lf;
        if (ff >= 6) break;
        const int fd = ff >> 1, fs = ff & 1;
        const int j = fd == 0 ? n0 : (fd == 1 ? n1 : n2);
        const int qa = fd == 0 ? n1 : n0, qb = fd == 2 ? n1 : n2;
        const int idx = lf * L + qa + P * qb;
        const double es = tE[fs][j], ds = tDE[fs][j];
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c] = fma(es, sV[c * RP + idx], fma(ds, sG[c * RP + idx], acc[c]));
      }
    }
    __syncthreads();
  }
  if (t < N) {
#pragma unroll
    for (int c = 0; c < 3; ++c) y[base + c * N + t] = acc[c];
  }

  // ---- 4. pressure test functions by sum factorization: cell (A_p^T x3) R_p
  // and, per face, e_p(s) (x) (A_p^T x A_p^T) Q_f
  double* t1b = X;                        // [j0][q1][q2]
  double* u1 = t1b + KP * P * P;          // [f][ja][pb]
  double* t2b = u1 + 6 * KP * P;          // [j0][j1][q2]
  double* u2 = t2b + KP * KP * P;         // [f][ja][jb]
  for (int i = t; i < KP * P * P; i += NT) {
    const int j0 = i % KP, q12 = i / KP;
    double v = 0;
#pragma unroll
    for (int q0 = 0; q0 < P; ++q0) v = fma(tAp[q0 * KP + j0], sRp[q0 + P * q12], v);
    t1b[i] = v;
  }
  for (int i = t; i < 6 * KP * P; i += NT) {
    const int f = i / (KP * P), r = i - f * KP * P;
    const int ja = r % KP, pb = r / KP;
    double v = 0;
#pragma unroll
    for (int pa = 0; pa < P; ++pa) v = fma(tAp[pa * KP + ja], fQ[f * L + pa + P * pb], v);
    u1[i] = v;
  }
  __syncthreads();
  for (int i = t; i < KP * KP * P; i += NT) {
    const int j0 = i % KP, j1 = (i / KP) % KP, q2 = i / (KP * KP);
    double v = 0;
#pragma unroll
    for (int q1 = 0; q1 < P; ++q1) v = fma(tAp[q1 * KP + j1], t1b[j0 + KP * (q1 + P * q2)], v);
    t2b[i] = v;
  }
  for (int i = t; i < 6 * KP * KP; i += NT) {
    const int f = i / (KP * KP), r = i - f * KP * KP;
    const int ja = r % KP, jb = r / KP;
    double v = 0;
#pragma unroll
    for (int pb = 0; pb < P; ++pb) v = fma(tAp[pb * KP + jb], u1[f * KP * P + ja + KP * pb], v);
    u2[i] = v;
  }
  __syncthreads();
  for (int i = t; i < NQ; i += NT) {
    const int jj[3] = {i % KP, (i / KP) % KP, i / (KP * KP)};
    double v = 0;
#pragma unroll
    for (int q2 = 0; q2 < P; ++q2) v = fma(tAp[q2 * KP + jj[2]], t2b[jj[0] + KP * (jj[1] + KP * q2)], v);
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      const int d = f >> 1, s = f & 1;
      int t1, t2;
      face_dirs(d, t1, t2);
      v = fma(tEp[s][jj[d]], u2[f * KP * KP + jj[t1] + KP * jj[t2]], v);
    }
    y[base + 3 * N + i] = v;
  }
}

// k = 3: at most 168 VGPRs (three wavefronts per SIMD; the 10 KB of LDS per
// cell allow fifteen per CU), enough to keep the DPP face contractions free
// of spills
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3)))
    k_stokes_apply_q3(const double* __restrict__ x, double* __restrict__ y, const StokesArgs a, const StokesGeom geo) {
  stokes_cell<4>(x, y, a, geo);
}

__global__ void __launch_bounds__(NT)
    k_stokes_apply_q2(const double* __restrict__ x, double* __restrict__ y, const StokesArgs a, const StokesGeom geo) {
  stokes_cell<3>(x, y, a, geo);
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
  // monomial coefficients a1..a7 of every cell's trilinear map (corner c =
  // c0 + 2 c1 + 4 c2; a_m is the alternating sum of the corners over the
  // face, edge or cell spanned by the coordinates of the monomial)
  std::vector<double> cgeo((size_t)M.nelem * GEO, 0.0);
  for (int64_t e = 0; e < M.nelem; ++e) {
    double X[8][3];
    cell_corners(M, e, X);
    double* g = &cgeo[(size_t)e * GEO];
    for (int k = 0; k < 3; ++k) {
      g[0 + k] = X[1][k] - X[0][k];
      g[3 + k] = X[2][k] - X[0][k];
      g[6 + k] = X[4][k] - X[0][k];
      g[9 + k] = X[3][k] - X[2][k] - X[1][k] + X[0][k];
      g[12 + k] = X[5][k] - X[4][k] - X[1][k] + X[0][k];
      g[15 + k] = X[6][k] - X[4][k] - X[2][k] + X[0][k];
      g[18 + k] = X[7][k] - X[6][k] - X[5][k] + X[4][k] - X[3][k] + X[2][k] + X[1][k] - X[0][k];
    }
  }
  // Sweep order: the hardware dispatches block b to XCD b mod 8 and each XCD
  // has its own L2. XCD x takes the x-th of 8 slabs of the mesh (along z, or
  // along y when nz < 8), and inside a slab the cells run y-outermost, then z,
  // then x, so that the cells in flight on an XCD and their y- and
  // z-neighbours form a compact window of the slab.
  const int64_t G = M.nelem;
  std::vector<uint32_t> order;
  order.reserve((size_t)G);
  const bool zsplit = nz >= 8;
  const int ns = zsplit ? nz : ny;
  for (int r = 0; r < 8; ++r) {
    const int s0 = (int)((int64_t)ns * r / 8), s1 = (int)((int64_t)ns * (r + 1) / 8);
    const int z0 = zsplit ? s0 : 0, z1 = zsplit ? s1 : nz, y0 = zsplit ? 0 : s0, y1 = zsplit ? ny : s1;
    for (int ey = y0; ey < y1; ++ey)
      for (int ez = z0; ez < z1; ++ez)
        for (int ex = 0; ex < nx; ++ex) order.push_back((uint32_t)(ex + (int64_t)nx * (ey + (int64_t)ny * ez)));
  }
  if ((int64_t)order.size() != G) throw std::runtime_error("Stokes sweep order");
  std::vector<uint32_t> tab((size_t)G);
  {
    const int64_t q = G >> 3, rm = G & 7;
    for (int64_t b = 0; b < G; ++b) {
      const int64_t xcd = b & 7;
      tab[(size_t)b] = order[(size_t)(xcd * q + std::min(xcd, rm) + (b >> 3))];
    }
  }
  if (hipMalloc(&M.d_vertices, sizeof(double) * M.vertices.size()) != hipSuccess ||
      hipMalloc(&M.d_gamma, sizeof(double) * gam.size()) != hipSuccess ||
      hipMalloc(&M.d_cellgeo, sizeof(double) * cgeo.size()) != hipSuccess ||
      hipMalloc(&M.d_stokes_order, sizeof(uint32_t) * tab.size()) != hipSuccess) {
    (void)hipGetLastError();
    throw std::runtime_error("device allocation failed (Stokes geometry)");
  }
  if (hipMemcpy(M.d_vertices, M.vertices.data(), sizeof(double) * M.vertices.size(), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(M.d_gamma, gam.data(), sizeof(double) * gam.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(M.d_cellgeo, cgeo.data(), sizeof(double) * cgeo.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(M.d_stokes_order, tab.data(), sizeof(uint32_t) * tab.size(), hipMemcpyHostToDevice) != hipSuccess)
    throw std::runtime_error("upload of the Stokes geometry failed");
}

hipError_t stokes_apply(const dg_mesh& M, const double* x, double* y, hipStream_t s) {
  StokesGeom g;
  g.order = M.d_stokes_order;
  g.cellgeo = M.d_cellgeo;
  g.gamma = M.d_gamma;
  for (int d = 0; d < 3; ++d) g.goff[d] = M.gamma_off[d];
  if (M.nelem > 0x7fffffff) return hipErrorInvalidValue;
  if (M.p == 4)
    hipLaunchKernelGGL(k_stokes_apply_q3, dim3((unsigned)M.nelem), dim3(NT), 0, s, x, y, M.st, g);
  else if (M.p == 3)
    hipLaunchKernelGGL(k_stokes_apply_q2, dim3((unsigned)M.nelem), dim3(NT), 0, s, x, y, M.st, g);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace dgi
