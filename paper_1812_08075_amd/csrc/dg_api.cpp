// C entry points of the DG library: descriptor validation, mesh setup and the
// operator calls. See include/dg.h for the contract of every function.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <initializer_list>
#include <utility>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "internal.h"

namespace {
thread_local std::string g_last_error;

struct DgError : std::runtime_error {
  dg_status st;
  DgError(dg_status s, const std::string& m) : std::runtime_error(m), st(s) {}
};

[[noreturn]] void fail(dg_status s, const std::string& m) { throw DgError(s, m); }

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) fail(DG_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

template <class F>
dg_status guarded(F&& f) {
  try {
    return f();
  } catch (const DgError& e) {
    g_last_error = e.what();
    return e.st;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return DG_ERR_ALLOC;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return DG_ERR_ARG;
  } catch (...) {
    g_last_error = "unknown error";
    return DG_ERR_ARG;
  }
}

int quad_points(const dg_mesh_desc& d) { return d.m == 0 ? d.k + 1 : d.m; }

// Checks everything that can be checked without a device.
void validate(const dg_mesh_desc* d) {
  if (!d) fail(DG_ERR_ARG, "desc is NULL");
  if (d->nx < 1 || d->ny < 1 || d->nz < 1) fail(DG_ERR_ARG, "nx, ny, nz must be >= 1");
  if (d->nx > 65535 || d->ny > 65535 || d->nz > 65535) fail(DG_ERR_ARG, "nx, ny, nz must be <= 65535");
  if (d->problem != DG_PROBLEM_DIFFREAC && d->problem != DG_PROBLEM_STOKES && d->problem != DG_PROBLEM_DIFFREAC_PAPER &&
      d->problem != DG_PROBLEM_NONLINEAR)
    fail(DG_ERR_ARG, "unknown problem");
  if (d->k < 1) fail(DG_ERR_ARG, "k must be >= 1");
  if (d->m < 0) fail(DG_ERR_ARG, "m must be >= 0");
  if (!std::isfinite(d->c) || !std::isfinite(d->alpha) || !std::isfinite(d->theta))
    fail(DG_ERR_ARG, "c, alpha and theta must be finite");
  if (d->alpha < 0) fail(DG_ERR_ARG, "alpha must be >= 0");
  if (d->penalty_form != 0 && d->penalty_form != 1) fail(DG_ERR_ARG, "penalty_form must be 0 or 1");
  if (d->dirichlet_mask > 0x3Fu) fail(DG_ERR_ARG, "dirichlet_mask has bits above the six sides");
  if (d->kappa_mode != DG_KAPPA_ONE && d->kappa_mode != DG_KAPPA_QP) fail(DG_ERR_ARG, "unknown kappa_mode");
  if (d->kappa_face != DG_KAPPA_FACE_TRACE && d->kappa_face != DG_KAPPA_FACE_ONE)
    fail(DG_ERR_ARG, "unknown kappa_face");
  const int64_t nelem = (int64_t)d->nx * d->ny * d->nz;
  if (nelem > (int64_t)1 << 31) fail(DG_ERR_ARG, "too many cells");
  if (d->k + 1 > dgi::PMAX) fail(DG_ERR_UNSUPPORTED, "degree k > 7 is not built");
  if (quad_points(*d) != d->k + 1)
    fail(DG_ERR_UNSUPPORTED, "only m = k + 1 (collocated Gauss-Legendre basis) is built");
  if (d->problem == DG_PROBLEM_DIFFREAC || d->problem == DG_PROBLEM_DIFFREAC_PAPER ||
      d->problem == DG_PROBLEM_NONLINEAR) {
    if (d->vertices) fail(DG_ERR_UNSUPPORTED, "diffusion-reaction runs on the regular (axis-aligned) grid only");
    if (d->problem == DG_PROBLEM_DIFFREAC_PAPER && d->kappa_mode != DG_KAPPA_ONE)
      fail(DG_ERR_ARG, "the paper's problem has its own coefficient tensor: kappa_mode must be DG_KAPPA_ONE");
    if (d->problem == DG_PROBLEM_NONLINEAR && d->kappa_mode != DG_KAPPA_ONE)
      fail(DG_ERR_ARG, "the nonlinear problem's coefficient is kappa(u): kappa_mode must be DG_KAPPA_ONE");
  } else {
    if (d->k < 2) fail(DG_ERR_UNSUPPORTED, "Stokes needs k >= 2");
    if (d->kappa_mode != DG_KAPPA_ONE) fail(DG_ERR_ARG, "Stokes has no kappa");
  }
  if (d->vertices) {
    const int64_t nv = (int64_t)(d->nx + 1) * (d->ny + 1) * (d->nz + 1) * 3;
    for (int64_t i = 0; i < nv; ++i)
      if (!std::isfinite(d->vertices[i])) fail(DG_ERR_ARG, "non-finite vertex coordinate");
  }
}

double penalty_coef(const dg_mesh_desc& d) {
  const double k = d.k;
  return d.penalty_form == 0 ? d.alpha * k * (k + 1) : d.alpha * k * (k + 2);
}

// Eigen decomposition of a symmetric n x n matrix by cyclic Jacobi rotations
// (long double): B = Q diag(lam) Q^T, Q orthogonal, columns the eigenvectors.
void symmetric_eigen(int n, long double B[dgi::PMAX][dgi::PMAX], long double Q[dgi::PMAX][dgi::PMAX],
                     long double* lam) {
  using ld = long double;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Q[i][j] = i == j ? 1 : 0;
  for (int sweep = 0; sweep < 64; ++sweep) {
    ld off = 0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += B[i][j] * B[i][j];
    if (off < 1e-60L) break;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) {
        if (B[i][j] == 0) continue;
        // rotation in the (i, j) plane that zeroes B[i][j]
        const ld tau = (B[j][j] - B[i][i]) / (2 * B[i][j]);
        const ld t = (tau >= 0 ? 1 : -1) / (std::fabs(tau) + std::sqrt(1 + tau * tau));
        const ld c = 1 / std::sqrt(1 + t * t), sn = t * c;
        for (int k = 0; k < n; ++k) {  // B <- B R
          const ld bi = B[k][i], bj = B[k][j];
          B[k][i] = c * bi - sn * bj;
          B[k][j] = sn * bi + c * bj;
        }
        for (int k = 0; k < n; ++k) {  // B <- R^T B
          const ld bi = B[i][k], bj = B[j][k];
          B[i][k] = c * bi - sn * bj;
          B[j][k] = sn * bi + c * bj;
        }
        for (int k = 0; k < n; ++k) {  // Q <- Q R
          const ld qi = Q[k][i], qj = Q[k][j];
          Q[k][i] = c * qi - sn * qj;
          Q[k][j] = sn * qi + c * qj;
        }
      }
  }
  for (int i = 0; i < n; ++i) lam[i] = B[i][i];
}

// Tables of the block-Jacobi preconditioner (see ScalarArgs::fdmV): the
// unscaled line operator K_d of each direction and side-type variant, built
// from the FP64 1D tables in long double, and its W-orthonormal eigenbasis.
// Valid for the symmetric operator (theta = -1) with kappa = 1.
template <typename T>
void build_fdm(const dg_mesh& M, dgi::ScalarArgs<T>& a) {
  using ld = long double;
  a.fdm_ok = 0;
  if (M.desc.problem != DG_PROBLEM_DIFFREAC || M.desc.kappa_mode != DG_KAPPA_ONE || M.desc.theta != -1.0) return;
  const dgi::Tables1D& tb = M.tab;
  const int p = M.p;
  const int n[3] = {M.desc.nx, M.desc.ny, M.desc.nz};
  const ld detJ = (ld)1 / n[0] / n[1] / n[2];
  const ld coef = penalty_coef(M.desc);
  bool ok = true;
  for (int d = 0; d < 3; ++d) {
    const ld h = (ld)1 / n[d];
    const ld vs = detJ / (h * h), fs = detJ / h;
    // face coefficients of the symmetric form (consistency and symmetry terms -1)
    const ld fA = -fs / 2, fG = fs * coef / h;
    const ld fB[2] = {fs / 2 / h, -fs / 2 / h};
    ld Kvol[dgi::PMAX][dgi::PMAX];
    for (int i = 0; i < p; ++i)
      for (int j = 0; j < p; ++j) {
        ld acc = 0;
        for (int q = 0; q < p; ++q) acc += (ld)tb.D[q][i] * vs * (ld)tb.wq[q] * (ld)tb.D[q][j];
        if (d == 0 && i == j) acc += (ld)M.desc.c * detJ * (ld)tb.wq[i];
        Kvol[i][j] = acc;
      }
    auto face = [&](int sd, int t, int i, int j) -> ld {
      if (t == 2) return 0;  // natural side: no terms
      const ld two = t == 1 ? 2 : 1;
      const ld sg = sd ? 1 : -1;
      return two * fA * (ld)tb.e[sd][i] * sg * (ld)tb.de[sd][j] / h + fG * (ld)tb.e[sd][i] * (ld)tb.e[sd][j] +
             two * fB[sd] * (ld)tb.de[sd][i] * (ld)tb.e[sd][j];
    };
    for (int t0 = 0; t0 < 3; ++t0)
      for (int t1 = 0; t1 < 3; ++t1) {
        const int v = 3 * t0 + t1;
        // B = W^-1/2 K W^-1/2, symmetrized against rounding
        ld B[dgi::PMAX][dgi::PMAX], Q[dgi::PMAX][dgi::PMAX], lam[dgi::PMAX];
        for (int i = 0; i < p; ++i)
          for (int j = 0; j < p; ++j) {
            const ld kij = Kvol[i][j] + face(0, t0, i, j) + face(1, t1, i, j);
            const ld kji = Kvol[j][i] + face(0, t0, j, i) + face(1, t1, j, i);
            B[i][j] = (kij + kji) / 2 / std::sqrt((ld)tb.wq[i] * (ld)tb.wq[j]);
          }
        symmetric_eigen(p, B, Q, lam);
        for (int i = 0; i < p; ++i) {
          for (int j = 0; j < p; ++j) a.fdmV[d][v][i * p + j] = (T)(Q[i][j] / std::sqrt((ld)tb.wq[i]));
          a.fdmL[d][v][i] = (T)lam[i];
        }
      }
  }
  // every cell's block must be positive definite: lam_x + lam_y + lam_z > 0
  // over the variants that occur (first, last and an interior position)
  ld lmin[3] = {1e300L, 1e300L, 1e300L};
  const uint32_t mask = M.desc.dirichlet_mask;
  for (int d = 0; d < 3; ++d) {
    const int pos[3] = {0, n[d] - 1, n[d] >= 3 ? 1 : 0};
    for (int k = 0; k < 3; ++k) {
      const int c = pos[k];
      const int t0 = c > 0 ? 0 : ((mask >> (2 * d)) & 1u ? 1 : 2);
      const int t1 = c < n[d] - 1 ? 0 : ((mask >> (2 * d + 1)) & 1u ? 1 : 2);
      for (int i = 0; i < p; ++i) lmin[d] = std::min(lmin[d], (ld)a.fdmL[d][3 * t0 + t1][i]);
    }
  }
  ok = ok && (lmin[0] + lmin[1] + lmin[2] > 0);
  a.fdm_ok = ok ? 1 : 0;
}

template <typename T>
void fill_scalar_args(const dg_mesh& M, dgi::ScalarArgs<T>& a) {
  const dgi::Tables1D& t = M.tab;
  const int p = M.p;
  std::memset(&a, 0, sizeof(a));
  for (int q = 0; q < p; ++q)
    for (int j = 0; j < p; ++j) a.D[q * p + j] = (T)t.D[q][j];
  for (int s = 0; s < 2; ++s)
    for (int j = 0; j < p; ++j) {
      a.e[s][j] = (T)t.e[s][j];
      a.de[s][j] = (T)t.de[s][j];
    }
  for (int q = 0; q < p; ++q) {
    a.w[q] = (T)t.wq[q];
    a.xi[q] = (T)t.xq[q];
  }
  const int n[3] = {M.desc.nx, M.desc.ny, M.desc.nz};
  double h[3];
  for (int d = 0; d < 3; ++d) h[d] = 1.0 / n[d];
  const double detJ = h[0] * h[1] * h[2];
  const double coef = penalty_coef(M.desc);
  for (int d = 0; d < 3; ++d) {
    a.vs[d] = (T)(detJ / (h[d] * h[d]));
    a.fs[d] = (T)(detJ / h[d]);
    a.hinv[d] = (T)(1.0 / h[d]);
    // |F| / min(|T-|, |T+|) = (|J| / h_d) / |J| on the regular grid, interior and boundary
    a.gam[d] = (T)(coef / h[d]);
    a.n[d] = n[d];
  }
  a.cmass = (T)(M.desc.c * detJ);
  a.p = p;
  for (int d = 0; d < 3; ++d) {
    a.hd[d] = h[d];
    a.gamd[d] = coef / h[d];
  }
  a.detJd = detJ;
  a.cd = M.desc.c;
  a.c_cons = (T)(-1.0);
  a.c_sym = (T)M.desc.theta;
  a.nelem = (int32_t)M.nelem;
  a.mask = M.desc.dirichlet_mask;
  a.kappa_face_one = M.desc.kappa_face == DG_KAPPA_FACE_ONE;
  for (int d = 0; d < 3; ++d) {
    const double vsd = detJ / (h[d] * h[d]);
    for (int q = 0; q < p; ++q)
      for (int j = 0; j < p; ++j) a.Dv[d][q * p + j] = (T)(vsd * t.wq[q] * t.D[q][j]);
    for (int s = 0; s < 2; ++s) {
      const double sg = s ? 1.0 : -1.0;
      for (int j = 0; j < p; ++j) {
        a.dno[d][s][j] = (T)(sg / h[d] * t.de[s][j]);
        a.dni[d][s][j] = (T)(-sg / h[d] * t.de[1 - s][j]);
      }
    }
    a.fG[d] = (T)(detJ / h[d] * coef / h[d]);
  }
  for (int i = 0; i < p; ++i) a.cw[i] = (T)(M.desc.c * detJ * t.wq[i]);
  // even-odd split (computed in FP64 from the 1D tables, then rounded)
  const int H = p / 2;
  for (int d = 0; d < 3; ++d) {
    dgi::EvenOdd<T>& o = a.eo[d];
    const double vsd = detJ / (h[d] * h[d]);
    auto Dv = [&](int q, int j) { return vsd * t.wq[q] * t.D[q][j]; };
    for (int q = 0; q < H; ++q) {
      for (int j = 0; j < H; ++j) {
        o.DvP[q * H + j] = (T)(0.5 * (Dv(q, j) + Dv(q, p - 1 - j)));
        o.DvM[q * H + j] = (T)(0.5 * (Dv(q, j) - Dv(q, p - 1 - j)));
      }
      if (p & 1) {
        o.DvC[q] = (T)Dv(q, H);
        o.DvR[q] = (T)Dv(H, q);
      }
    }
    o.fG = a.fG[d];
  }
  for (int i = 0; i < H; ++i) {
    for (int q = 0; q < H; ++q) {
      a.G2p[i * H + q] = (T)(t.D[q][i] + t.D[q][p - 1 - i]);
      a.G2m[i * H + q] = (T)(t.D[q][i] - t.D[q][p - 1 - i]);
    }
    if (p & 1) {
      a.Gh[i] = (T)t.D[H][i];
      a.G2c[i] = (T)(2.0 * t.D[i][H]);
    }
    a.Ep[i] = (T)(0.5 * (t.e[0][i] + t.e[0][p - 1 - i]));
    a.Em[i] = (T)(0.5 * (t.e[0][i] - t.e[0][p - 1 - i]));
    a.DEp[i] = (T)(0.5 * (t.de[0][i] + t.de[0][p - 1 - i]));
    a.DEm[i] = (T)(0.5 * (t.de[0][i] - t.de[0][p - 1 - i]));
    a.cwh[i] = (T)(0.5 * M.desc.c * detJ * t.wq[i]);
  }
  a.Eh = (T)((p & 1) ? t.e[0][H] : 0.0);
  a.DEh = (T)((p & 1) ? t.de[0][H] : 0.0);
  a.cwm = (T)((p & 1) ? M.desc.c * detJ * t.wq[H] : 0.0);
  dgi::derive_face_constants(a);
  build_fdm(M, a);
}

size_t elem_size(int prec) { return prec == DG_F64 ? sizeof(double) : sizeof(float); }

void check_prec(int prec) {
  if (prec != DG_F64 && prec != DG_F32) fail(DG_ERR_ARG, "precision must be DG_F64 or DG_F32");
}

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  if (!a || !b) return false;
  const char* pa = (const char*)a;
  const char* pb = (const char*)b;
  return pa < pb + nb && pb < pa + na;
}

// Every vector argument must be 16-byte aligned: the kernels read and write
// whole 16-byte groups of elements.
constexpr size_t kVecAlign = 16;

// Alignment of the pointers that are given, checked before anything else.
void check_align(std::initializer_list<std::pair<const void*, const char*>> ps) {
  for (const auto& pn : ps)
    if (pn.first && (uintptr_t)pn.first % kVecAlign)
      fail(DG_ERR_ARG, std::string(pn.second) + " is not 16-byte aligned");
}

void check_vec(const void* p, const char* name) {
  if (!p) fail(DG_ERR_ARG, std::string(name) + " is NULL");
  if ((uintptr_t)p % kVecAlign) fail(DG_ERR_ARG, std::string(name) + " is not 16-byte aligned");
}

hipStream_t as_stream(void* s) { return (hipStream_t)s; }
}  // namespace

void dg_set_error(const std::string& msg) { g_last_error = msg; }

template <typename T>
void dgi::derive_face_constants(ScalarArgs<T>& a) {
  for (int d = 0; d < 3; ++d) {
    const double fs = (double)a.fs[d], hi = (double)a.hinv[d];
    a.fA[d] = (T)(fs * 0.5 * (double)a.c_cons);
    for (int s = 0; s < 2; ++s) a.fB[d][s] = (T)(fs * 0.5 * (double)a.c_sym * (s ? 1.0 : -1.0) * hi);
    a.eo[d].fAh = (T)(-fs * 0.5 * (double)a.c_cons * hi);
    a.eo[d].fB0 = a.fB[d][0];
  }
  // 1D line operators (kappa = 1), in long double from the FP64 geometry
  using ld = long double;
  const int p = a.p;
  {
    // any degree: even/odd interior K, rank-2 neighbour rows, boundary corrections
    const ld cc = (ld)(double)a.c_cons, cs = (ld)(double)a.c_sym;
    const int H = p / 2;
    for (int d = 0; d < 3; ++d) {
      dgi::LineOp<T>& o = a.lo[d];
      const ld h = a.hd[d], detJ = a.detJd;
      const ld vs = detJ / (h * h), fs = detJ / h;
      const ld fA = fs * cc / 2, fG = fs * (ld)a.gamd[d];
      const ld fB[2] = {-fs * cs / 2 / h, fs * cs / 2 / h};
      ld e[2][dgi::PMAX], de[2][dgi::PMAX], nrm[2][dgi::PMAX];
      for (int s = 0; s < 2; ++s)
        for (int j = 0; j < p; ++j) {
          e[s][j] = (ld)(double)a.e[s][j];
          de[s][j] = (ld)(double)a.de[s][j];
          nrm[s][j] = (s ? 1 : -1) * de[s][j] / h;
        }
      ld K[dgi::PMAX][dgi::PMAX];
      for (int i = 0; i < p; ++i)
        for (int j = 0; j < p; ++j) {
          ld acc = 0;
          for (int q = 0; q < p; ++q)
            acc += (ld)(double)a.D[q * p + i] * vs * (ld)(double)a.w[q] * (ld)(double)a.D[q * p + j];
          if (d == 0 && i == j) acc += (ld)a.cd * detJ * (ld)(double)a.w[i];
          for (int s = 0; s < 2; ++s)
            acc += fA * e[s][i] * nrm[s][j] + fG * e[s][i] * e[s][j] + fB[s] * de[s][i] * e[s][j];
          K[i][j] = acc;
        }
      for (int i = 0; i < H; ++i) {
        for (int j = 0; j < H; ++j) {
          o.Kp[i * H + j] = (T)((K[i][j] + K[i][p - 1 - j]) / 2);
          o.Km[i * H + j] = (T)((K[i][j] - K[i][p - 1 - j]) / 2);
        }
        if (p & 1) {
          o.Kc[i] = (T)K[i][H];
          o.Kr[i] = (T)K[H][i];
        }
      }
      o.Kh = (T)((p & 1) ? K[H][H] : 0);
      for (int j = 0; j < p; ++j) {
        o.la[j] = (T)(-fA * nrm[1][j] - fG * e[1][j]);
        o.lb[j] = (T)(-fB[0] * e[1][j]);
      }
      for (int s = 0; s < 2; ++s) {
        const ld sg = s ? 1 : -1;
        // Dirichlet: the one-sided consistency and symmetry terms count twice
        o.bq[0][s][0] = (T)(fA * sg / h);
        o.bq[0][s][1] = (T)0;
        o.bq[0][s][2] = (T)fB[s];
        // natural: no face terms at all
        o.bq[1][s][0] = (T)(-fA * sg / h);
        o.bq[1][s][1] = (T)(-fG);
        o.bq[1][s][2] = (T)(-fB[s]);
      }
    }
  }
  if (p == 4) {
    const ld cc = (ld)(double)a.c_cons, cs = (ld)(double)a.c_sym;
    for (int d = 0; d < 3; ++d) {
      const ld h = a.hd[d], detJ = a.detJd;
      const ld vs = detJ / (h * h), fs = detJ / h;
      const ld fA = fs * cc / 2, fG = fs * (ld)a.gamd[d];
      const ld fB[2] = {-fs * cs / 2 / h, fs * cs / 2 / h};
      ld e[2][4], de[2][4], nrm[2][4];
      for (int s = 0; s < 2; ++s)
        for (int j = 0; j < 4; ++j) {
          e[s][j] = (ld)(double)a.e[s][j];
          de[s][j] = (ld)(double)a.de[s][j];
          nrm[s][j] = (s ? 1 : -1) * de[s][j] / h;  // outward normal derivative row of side s
        }
      ld Kvol[4][4];
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
          ld acc = 0;
          for (int q = 0; q < 4; ++q)
            acc += (ld)(double)a.D[q * 4 + i] * vs * (ld)(double)a.w[q] * (ld)(double)a.D[q * 4 + j];
          if (d == 0 && i == j) acc += (ld)a.cd * detJ * (ld)(double)a.w[i];
          Kvol[i][j] = acc;
        }
      // own-cell face terms of side s for side type t (0 interior, 1 Dirichlet, 2 none)
      auto face = [&](int s, int t, int i, int j) -> ld {
        if (t == 2) return 0;
        const ld two = t == 1 ? 2 : 1;
        return two * fA * e[s][i] * nrm[s][j] + fG * e[s][i] * e[s][j] + two * fB[s] * de[s][i] * e[s][j];
      };
      // rows divided by the weight of the output node along d: the line's
      // tangential weight times row i is the full tensor weight of node i
      // divided by w_i, so the kernel applies one tensor weight per node
      // after summing the three directions
      ld winv[4];
      for (int i = 0; i < 4; ++i) winv[i] = 1 / (ld)(double)a.w[i];
      for (int t0 = 0; t0 < 3; ++t0)
        for (int t1 = 0; t1 < 3; ++t1)
          for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j)
              a.Km[d][3 * t0 + t1][4 * i + j] =
                  (T)(winv[i] * (Kvol[i][j] + face(0, t0, i, j) + face(1, t1, i, j)));
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
          // neighbour across side 0 meets it with its side 1, across side 1 with its side 0
          a.Lm[d][4 * i + j] =
              (T)(winv[i] * (-fA * e[0][i] * nrm[1][j] - fG * e[0][i] * e[1][j] - fB[0] * de[0][i] * e[1][j]));
          a.Rm[d][4 * i + j] =
              (T)(winv[i] * (-fA * e[1][i] * nrm[0][j] - fG * e[1][i] * e[0][j] - fB[1] * de[1][i] * e[0][j]));
        }
    }
    for (int lane = 0; lane < 64; ++lane) {
      const int ai = 4 * (lane & 3) + (lane >> 4);
      for (int d = 0; d < 3; ++d) {
        a.lrec[lane][3 * d] = (double)a.Km[d][0][ai];
        a.lrec[lane][3 * d + 1] = (double)a.Lm[d][ai];
        a.lrec[lane][3 * d + 2] = (double)a.Rm[d][ai];
      }
      a.lrec[lane][9] = 0.0;
      // tensor weights of the two nodes (2h, i1, i2), (2h + 1, i1, i2) the lane
      // holds in the pair layout lane = h + 2 i1 + 8 cell + 16 i2
      const int h = lane & 1, i1 = (lane >> 1) & 3, i2 = lane >> 4;
      const ld wt = (ld)(double)a.w[i1] * (ld)(double)a.w[i2];
      a.lrec[lane][10] = (double)(wt * (ld)(double)a.w[2 * h]);
      a.lrec[lane][11] = (double)(wt * (ld)(double)a.w[2 * h + 1]);
    }
  }
}
template void dgi::derive_face_constants<double>(ScalarArgs<double>&);
template void dgi::derive_face_constants<float>(ScalarArgs<float>&);

// The host-side trilinear geometry used by the Stokes setup and dg_mesh_qpoints.
namespace dgi {
void cell_corners(const dg_mesh& M, int64_t e, double X[8][3]);
void stokes_setup(dg_mesh& M);
}  // namespace dgi

void dgi::cell_corners(const dg_mesh& M, int64_t e, double X[8][3]) {
  const int nx = M.desc.nx, ny = M.desc.ny;
  const int64_t ex = e % nx, ey = (e / nx) % ny, ez = e / ((int64_t)nx * ny);
  for (int c = 0; c < 8; ++c) {
    const int64_t i = ex + (c & 1), j = ey + ((c >> 1) & 1), l = ez + ((c >> 2) & 1);
    if (M.vertices.empty()) {
      X[c][0] = (double)i / M.desc.nx;
      X[c][1] = (double)j / M.desc.ny;
      X[c][2] = (double)l / M.desc.nz;
    } else {
      const int64_t v = i + (int64_t)(nx + 1) * (j + (int64_t)(ny + 1) * l);
      for (int a = 0; a < 3; ++a) X[c][a] = M.vertices[3 * v + a];
    }
  }
}

extern "C" {

const char* dg_last_error(void) { return g_last_error.c_str(); }

dg_status dg_mesh_desc_validate(const dg_mesh_desc* desc) {
  return guarded([&] {
    validate(desc);
    return DG_OK;
  });
}

dg_status dg_mesh_create(const dg_mesh_desc* desc, void* stream, dg_mesh** out) {
  return guarded([&]() -> dg_status {
    if (!out) fail(DG_ERR_ARG, "out is NULL");
    *out = nullptr;
    validate(desc);
    dg_mesh* M = new dg_mesh();
    try {
      M->desc = *desc;
      M->desc.vertices = nullptr;
      M->p = desc->k + 1;
      M->m = quad_points(*desc);
      M->kp = desc->k;
      M->nelem = (int64_t)desc->nx * desc->ny * desc->nz;
      M->N = desc->problem == DG_PROBLEM_STOKES ? 3 * (int64_t)M->p * M->p * M->p + (int64_t)M->kp * M->kp * M->kp
                                                : (int64_t)M->p * M->p * M->p;
      M->ndofs = M->nelem * M->N;
      M->nqp = M->nelem * (int64_t)M->m * M->m * M->m;
      M->axis_aligned = desc->vertices == nullptr;
      if (desc->vertices) {
        const size_t nv = (size_t)(desc->nx + 1) * (desc->ny + 1) * (desc->nz + 1) * 3;
        M->vertices.assign(desc->vertices, desc->vertices + nv);
      }
      M->tab = dgi::make_tables(M->p, M->m);
      hip_check(hipGetDevice(&M->device), "hipGetDevice");
      hip_check(hipDeviceGetAttribute(&M->num_cu, hipDeviceAttributeMultiprocessorCount, M->device),
                "hipDeviceGetAttribute");
      fill_scalar_args(*M, M->sd);
      fill_scalar_args(*M, M->sf);
      if (desc->problem != DG_PROBLEM_STOKES) {
        if (hipMalloc(&M->d_pd, sizeof(M->pd)) != hipSuccess || hipMalloc(&M->d_pf, sizeof(M->pf)) != hipSuccess) {
          (void)hipGetLastError();
          fail(DG_ERR_ALLOC, "device allocation failed (parameter blocks)");
        }
        hip_check(dgi::scalar_params_upload(*M), "upload");
        hip_check(dgi::mfma_setup(*M), "upload");
      }
      if (desc->problem == DG_PROBLEM_STOKES) dgi::stokes_setup(*M);
      hip_check(hipStreamSynchronize(as_stream(stream)), "hipStreamSynchronize");
    } catch (...) {
      dg_mesh_destroy(M);
      throw;
    }
    *out = M;
    return DG_OK;
  });
}

dg_status dg_mesh_destroy(dg_mesh* M) {
  return guarded([&] {
    if (!M) return DG_OK;
    if (M->d_vertices) (void)hipFree(M->d_vertices);
    if (M->d_gamma) (void)hipFree(M->d_gamma);
    if (M->d_cellgeo) (void)hipFree(M->d_cellgeo);
    if (M->d_stokes_order) (void)hipFree(M->d_stokes_order);
    if (M->d_pd) (void)hipFree(M->d_pd);
    if (M->d_pf) (void)hipFree(M->d_pf);
    if (M->d_blocks) (void)hipFree(M->d_blocks);
    for (uint32_t* w : M->d_waves)
      if (w) (void)hipFree(w);
    delete M;
    return DG_OK;
  });
}

dg_status dg_mesh_info(const dg_mesh* M, dg_mesh_info_t* out) {
  return guarded([&] {
    if (!M || !out) fail(DG_ERR_ARG, "mesh or out is NULL");
    std::memset(out, 0, sizeof(*out));
    out->nelem = M->nelem;
    out->ndofs = M->ndofs;
    out->dofs_per_elem = M->N;
    out->nqp = M->nqp;
    out->p = M->p;
    out->m = M->m;
    out->axis_aligned = M->axis_aligned ? 1 : 0;
    const double p = M->p, E = (double)M->nelem;
    const bool kap = M->desc.kappa_mode == DG_KAPPA_QP;
    if (M->desc.problem == DG_PROBLEM_DIFFREAC) {
      // per cell, all six faces interior: 3 directions x p^2 lines, each with
      // two p x p contractions (4p^2), pointwise scaling (p, 2p with kappa) and
      // two faces (own trace + normal derivative 4p, neighbour 4p, flux 12,
      // test rows 4p; kappa traces +4p); mass term 2p on the x lines; final
      // sum of the three directions 2 per DOF
      const double face = 12 * p + 12 + (kap ? 4 * p : 0);
      const double line = 4 * p * p + (kap ? 2 * p : p) + 2 * face;
      out->flops_apply = E * (3 * p * p * line + 2 * p * p * p + 2 * p * p * p);
      // adjoint: the transposed apply on g, plus the forward contractions of u
      // (2p^2 per line), volume dkappa products (3p), face dkappa terms
      // (u, g traces of the neighbour 8p, product 8, test rows 2p)
      const double adj_line = line + 2 * p * p + 3 * p + 2 * (12 * p + 8);
      out->flops_adjoint = E * (3 * p * p * adj_line + 4 * p * p * p);
      out->bytes_apply[0] = (double)M->ndofs * (16 + (kap ? 8 : 0));
      out->bytes_apply[1] = (double)M->ndofs * (8 + (kap ? 4 : 0));
      out->bytes_adjoint = (double)M->ndofs * 40;
    } else if (M->desc.problem == DG_PROBLEM_NONLINEAR) {
      // Jacobian action per cell: per direction and line, the D contractions
      // of u0 and z (4p^2), the pointwise flux (6p), D^T (2p^2), and at both
      // ends the own and neighbour traces and normal derivatives of both
      // inputs (16p), the flux (~20) and the test rows (4p); mass 3p^3
      const double line = 6 * p * p + 6 * p + 2 * (20 * p + 20);
      out->flops_apply = E * (3 * p * p * line + 3 * p * p * p + 2 * p * p * p);
      out->flops_adjoint = 0;
      out->bytes_apply[0] = (double)M->ndofs * 24;  // read u0 and z, write y
      out->bytes_apply[1] = (double)M->ndofs * 12;
    } else if (M->desc.problem == DG_PROBLEM_DIFFREAC_PAPER) {
      // per cell: three forward and three transposed contractions (12 p^4),
      // K(x) grad u and the mass term per point (~25 p^3), and per direction
      // and line both faces: own and neighbour traces and normal derivatives,
      // tangential derivatives of both traces, flux, tangential test
      // contractions and test rows (~48 p + 60 per line and direction)
      out->flops_apply = E * (12 * p * p * p * p + 25 * p * p * p + 3 * p * p * (48 * p + 60) + p * p * p);
      out->flops_adjoint = out->flops_apply;
      out->bytes_apply[0] = (double)M->ndofs * 16;
      out->bytes_apply[1] = (double)M->ndofs * 8;
    } else {
      const double kp = M->kp;
      // per cell: 3 components x 3 gradient contractions forward and back
      // (18 p^4), pressure interpolation forward and back (2 C_SF(p,kp)),
      // geometry and pointwise work per point (~220), faces per side with
      // full gradient traces (~ 3 x 10 p^3 + 30 p^2 per side)
      const double csf = 2 * (p * kp * kp * kp + p * p * kp * kp + p * p * p * kp);
      const double face = 3 * (10 * p * p * p) + 60 * p * p;
      out->flops_apply = E * (18 * p * p * p * p + 2 * csf + 220 * p * p * p + 6 * face);
      out->bytes_apply[0] = (double)M->ndofs * 16;
      out->bytes_apply[1] = (double)M->ndofs * 8;
    }
    return DG_OK;
  });
}

dg_status dg_apply(const dg_mesh* M, int precision, const void* x, void* y, const void* kappa, void* stream) {
  return guarded([&] {
    check_align({{x, "x"}, {y, "y"}, {kappa, "kappa"}});
    if (!M) fail(DG_ERR_ARG, "mesh is NULL");
    check_prec(precision);
    const size_t es = elem_size(precision);
    check_vec(x, "x");
    check_vec(y, "y");
    const size_t nb = (size_t)M->ndofs * es;
    if (overlap(x, nb, y, nb)) fail(DG_ERR_ARG, "x and y overlap");
    const bool kap = M->desc.kappa_mode == DG_KAPPA_QP;
    if (kap) {
      check_vec(kappa, "kappa");
      if (overlap(kappa, (size_t)M->nqp * es, y, nb)) fail(DG_ERR_ARG, "kappa and y overlap");
    }
    if (M->desc.problem == DG_PROBLEM_STOKES) {
      if (precision != DG_F64) fail(DG_ERR_UNSUPPORTED, "the Stokes operator is built for FP64 only");
      hip_check(dgi::stokes_apply(*M, (const double*)x, (double*)y, as_stream(stream)), "stokes apply launch");
      return DG_OK;
    }
    if (M->desc.problem == DG_PROBLEM_DIFFREAC_PAPER) {
      hip_check(dgi::tensor_apply(*M, precision, x, y, false, false, as_stream(stream)), "apply launch");
      return DG_OK;
    }
    if (M->desc.problem == DG_PROBLEM_NONLINEAR)
      fail(DG_ERR_UNSUPPORTED, "the nonlinear operator's Jacobian needs a linearization point: dg_apply_jacobian");
    hip_check(dgi::scalar_apply(*M, precision, x, y, kap ? kappa : nullptr, false, as_stream(stream)),
              "apply launch");
    return DG_OK;
  });
}

dg_status dg_apply_jacobian(const dg_mesh* M, int precision, const void* u0, const void* z, void* y, void* stream) {
  return guarded([&] {
    check_align({{u0, "u0"}, {z, "z"}, {y, "y"}});
    if (!M) fail(DG_ERR_ARG, "mesh is NULL");
    check_prec(precision);
    check_vec(u0, "u0");
    check_vec(z, "z");
    check_vec(y, "y");
    const size_t nb = (size_t)M->ndofs * elem_size(precision);
    if (overlap(u0, nb, y, nb) || overlap(z, nb, y, nb)) fail(DG_ERR_ARG, "y overlaps u0 or z");
    if (M->desc.problem != DG_PROBLEM_NONLINEAR)
      fail(DG_ERR_UNSUPPORTED, "dg_apply_jacobian is for DG_PROBLEM_NONLINEAR (the linear problems: dg_apply)");
    hip_check(dgi::nonlinear_apply(*M, precision, u0, z, y, true, as_stream(stream)), "Jacobian launch");
    return DG_OK;
  });
}

dg_status dg_precond_apply(const dg_mesh* M, int precision, const void* r, void* z, void* stream) {
  return guarded([&] {
    check_align({{r, "r"}, {z, "z"}});
    if (!M) fail(DG_ERR_ARG, "mesh is NULL");
    check_prec(precision);
    const size_t es = elem_size(precision);
    check_vec(r, "r");
    check_vec(z, "z");
    const size_t nb = (size_t)M->ndofs * es;
    if (overlap(r, nb, z, nb)) fail(DG_ERR_ARG, "r and z overlap");
    if (M->desc.problem != DG_PROBLEM_DIFFREAC || !dgi::block_jacobi_supported(*M))
      fail(DG_ERR_UNSUPPORTED,
           "the block-Jacobi preconditioner is built for diffusion-reaction with kappa = 1 and theta = -1");
    hip_check(dgi::block_jacobi(*M, precision, r, z, nullptr, as_stream(stream)), "preconditioner launch");
    return DG_OK;
  });
}

dg_status dg_apply_adjoint(const dg_mesh* M, int precision, const void* g, const void* u, const void* kappa,
                           void* ATg, void* dkappa, void* stream) {
  return guarded([&] {
    check_align({{g, "g"}, {u, "u"}, {kappa, "kappa"}, {ATg, "ATg"}, {dkappa, "dkappa"}});
    if (!M) fail(DG_ERR_ARG, "mesh is NULL");
    if (M->desc.problem != DG_PROBLEM_DIFFREAC && M->desc.problem != DG_PROBLEM_DIFFREAC_PAPER)
      fail(DG_ERR_UNSUPPORTED, "the adjoint is built for diffusion-reaction");
    if (M->desc.problem == DG_PROBLEM_DIFFREAC_PAPER && dkappa)
      fail(DG_ERR_UNSUPPORTED, "the paper's problem has no kappa to differentiate (dkappa must be NULL)");
    check_prec(precision);
    const size_t es = elem_size(precision);
    check_vec(g, "g");
    check_vec(ATg, "ATg");
    const size_t nb = (size_t)M->ndofs * es, nk = (size_t)M->nqp * es;
    const bool kap = M->desc.kappa_mode == DG_KAPPA_QP;
    if (kap) check_vec(kappa, "kappa");
    if (dkappa) {
      check_vec(dkappa, "dkappa");
      check_vec(u, "u");
      if (overlap(dkappa, nk, g, nb) || overlap(dkappa, nk, u, nb) || overlap(dkappa, nk, ATg, nb) ||
          (kap && overlap(dkappa, nk, kappa, nk)))
        fail(DG_ERR_ARG, "dkappa overlaps another argument");
      if (overlap(ATg, nb, u, nb)) fail(DG_ERR_ARG, "ATg and u overlap");
    }
    if (overlap(ATg, nb, g, nb)) fail(DG_ERR_ARG, "ATg and g overlap");
    if (kap && overlap(ATg, nb, kappa, nk)) fail(DG_ERR_ARG, "ATg and kappa overlap");
    hipStream_t s = as_stream(stream);
    if (M->desc.problem == DG_PROBLEM_DIFFREAC_PAPER) {
      hip_check(dgi::tensor_apply(*M, precision, g, ATg, true, false, s), "adjoint launch");
      return DG_OK;
    }
    if (!dkappa) {
      hip_check(dgi::scalar_apply(*M, precision, g, ATg, kap ? kappa : nullptr, true, s), "adjoint launch");
      return DG_OK;
    }
    hip_check(dgi::scalar_adjoint(*M, precision, g, u, kap ? kappa : nullptr, ATg, dkappa, s), "adjoint launch");
    return DG_OK;
  });
}

dg_status dg_residual(const dg_mesh* M, int precision, const void* u, void* r, void* stream) {
  return guarded([&] {
    check_align({{u, "u"}, {r, "r"}});
    if (!M) fail(DG_ERR_ARG, "mesh is NULL");
    check_prec(precision);
    check_vec(u, "u");
    check_vec(r, "r");
    const size_t nb = (size_t)M->ndofs * elem_size(precision);
    if (overlap(u, nb, r, nb)) fail(DG_ERR_ARG, "u and r overlap");
    if (M->desc.problem == DG_PROBLEM_NONLINEAR) {
      hip_check(dgi::nonlinear_apply(*M, precision, u, u, r, false, as_stream(stream)), "residual launch");
      return DG_OK;
    }
    if (M->desc.problem != DG_PROBLEM_DIFFREAC_PAPER)
      fail(DG_ERR_UNSUPPORTED,
           "dg_residual is for DG_PROBLEM_DIFFREAC_PAPER (with its data) and DG_PROBLEM_NONLINEAR");
    hip_check(dgi::tensor_apply(*M, precision, u, r, false, true, as_stream(stream)), "residual launch");
    return DG_OK;
  });
}

dg_status dg_mesh_qpoints(const dg_mesh* M, double* xyz) {
  return guarded([&] {
    if (!M || !xyz) fail(DG_ERR_ARG, "mesh or xyz is NULL");
    const int m = M->m;
    const double* xq = M->tab.xq;
    for (int64_t e = 0; e < M->nelem; ++e) {
      double X[8][3];
      dgi::cell_corners(*M, e, X);
      for (int q2 = 0; q2 < m; ++q2)
        for (int q1 = 0; q1 < m; ++q1)
          for (int q0 = 0; q0 < m; ++q0) {
            const double t[3] = {xq[q0], xq[q1], xq[q2]};
            double* o = xyz + 3 * (e * m * m * m + q0 + m * (q1 + m * q2));
            o[0] = o[1] = o[2] = 0;
            for (int c = 0; c < 8; ++c) {
              double wgt = 1;
              for (int d = 0; d < 3; ++d) wgt *= ((c >> d) & 1) ? t[d] : 1 - t[d];
              for (int a = 0; a < 3; ++a) o[a] += wgt * X[c][a];
            }
          }
    }
    return DG_OK;
  });
}

dg_status dg_load_vector(const dg_mesh* M, int precision, const void* fq, void* b, void* stream) {
  return guarded([&] {
    check_align({{fq, "fq"}, {b, "b"}});
    if (!M) fail(DG_ERR_ARG, "mesh is NULL");
    if (M->desc.problem == DG_PROBLEM_STOKES) fail(DG_ERR_UNSUPPORTED, "load vectors are built for diffusion-reaction");
    check_prec(precision);
    const size_t es = elem_size(precision);
    check_vec(fq, "fq");
    check_vec(b, "b");
    if (overlap(fq, (size_t)M->nqp * es, b, (size_t)M->ndofs * es)) fail(DG_ERR_ARG, "fq and b overlap");
    hip_check(dgi::scalar_load(*M, precision, fq, b, as_stream(stream)), "load vector launch");
    return DG_OK;
  });
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Variant selection (the autotuning counterpart of Section 4.2's choice among
// vectorization strategies: here among kernels and launch shapes of one
// operator, scored by measured time).

namespace {

struct Variant {
  int kind, param;
};

// Candidates for the apply of precision `prec` on this mesh, the cost
// model's default first.
std::vector<Variant> apply_candidates(const dg_mesh& M, int prec) {
  std::vector<Variant> v;
  const bool kap = M.desc.kappa_mode == DG_KAPPA_QP;
  const bool mc = M.desc.problem == DG_PROBLEM_DIFFREAC && M.p == 4 && !kap && M.d_waves[prec] != nullptr;
  if (mc) {
    const int r0 = dgi::mfma_default_rows(M.desc.nx, M.desc.ny, M.desc.nz);
    v.push_back({DG_VARIANT_MATRIX_CORE, r0});
    for (int r = 1; r <= 16; r *= 2)
      if (r != r0 && r <= M.desc.ny) v.push_back({DG_VARIANT_MATRIX_CORE, r});
  }
  v.push_back({DG_VARIANT_LINES, 0});
  v.push_back({DG_VARIANT_LINES, 1});
  if (prec == DG_F32 && M.p == 4 && M.desc.problem == DG_PROBLEM_DIFFREAC) {
    // FP32 lines of p = 4 with their contractions on the matrix cores
    v.push_back({DG_VARIANT_LINES, 2});
    v.push_back({DG_VARIANT_LINES, 3});
  }
  return v;
}

void set_variant(dg_mesh& M, int prec, const Variant& v) {
  if (v.kind == DG_VARIANT_MATRIX_CORE) {
    if (M.mfma_rows[prec] != v.param) hip_check(dgi::mfma_build(M, prec, v.param), "wavefront table");
    M.lines_forced[prec] = false;
  } else {
    M.lines_forced[prec] = M.d_waves[prec] != nullptr;
    if (prec == DG_F32) M.lines_mfma = (v.param & 2) != 0;
    if (M.sweep_linear != (v.param & 1)) hip_check(dgi::line_sweep_set(M, v.param & 1), "block table");
  }
}

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

struct Events {
  hipEvent_t a = nullptr, b = nullptr;
  ~Events() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

}  // namespace

extern "C" {

dg_status dg_mesh_set_variant(dg_mesh* M, int precision, int kind, int param) {
  return guarded([&] {
    if (!M) fail(DG_ERR_ARG, "mesh is NULL");
    check_prec(precision);
    if (M->desc.problem == DG_PROBLEM_STOKES) fail(DG_ERR_UNSUPPORTED, "the Stokes operator has one variant");
    const std::vector<Variant> c = apply_candidates(*M, precision);
    bool ok = false;
    for (const Variant& v : c) ok = ok || (v.kind == kind && (v.param == param || kind == DG_VARIANT_MATRIX_CORE));
    if (kind == DG_VARIANT_MATRIX_CORE && !(param >= 1 && param <= 16 && (param & (param - 1)) == 0)) ok = false;
    if (!ok) fail(DG_ERR_ARG, "no such variant for this mesh and precision");
    set_variant(*M, precision, {kind, param});
    return DG_OK;
  });
}

dg_status dg_mesh_tune(dg_mesh* M, int precision, int trials, void* stream, dg_tune_result* out) {
  return guarded([&] {
    if (!M || !out) fail(DG_ERR_ARG, "mesh and out must not be NULL");
    check_prec(precision);
    if (trials < 1 || trials > 100) fail(DG_ERR_ARG, "trials must be in 1..100");
    if (M->desc.problem == DG_PROBLEM_STOKES) fail(DG_ERR_UNSUPPORTED, "the Stokes operator has one variant");
    std::memset(out, 0, sizeof(*out));
    const std::vector<Variant> c = apply_candidates(*M, precision);
    if ((int)c.size() > DG_TUNE_MAX) fail(DG_ERR_UNSUPPORTED, "too many candidates");
    const hipStream_t s = as_stream(stream);
    const size_t es = elem_size(precision);
    const bool kap = M->desc.kappa_mode == DG_KAPPA_QP;
    DevBuf x, y, k;
    if (hipMalloc(&x.p, (size_t)M->ndofs * es) != hipSuccess || hipMalloc(&y.p, (size_t)M->ndofs * es) != hipSuccess ||
        (kap && hipMalloc(&k.p, (size_t)M->nqp * es) != hipSuccess)) {
      (void)hipGetLastError();
      fail(DG_ERR_ALLOC, "device allocation failed (tuning vectors)");
    }
    hip_check(hipMemsetAsync(x.p, 0, (size_t)M->ndofs * es, s), "hipMemsetAsync");
    if (kap) hip_check(hipMemsetAsync(k.p, 0, (size_t)M->nqp * es, s), "hipMemsetAsync");
    Events ev;
    hip_check(hipEventCreate(&ev.a), "hipEventCreate");
    hip_check(hipEventCreate(&ev.b), "hipEventCreate");
    constexpr int kReps = 10;
    auto run = [&] {
      if (M->desc.problem == DG_PROBLEM_DIFFREAC_PAPER)
        hip_check(dgi::tensor_apply(*M, precision, x.p, y.p, false, false, s), "apply");
      else if (M->desc.problem == DG_PROBLEM_NONLINEAR)
        hip_check(dgi::nonlinear_apply(*M, precision, x.p, x.p, y.p, true, s), "Jacobian");
      else
        hip_check(dgi::scalar_apply(*M, precision, x.p, y.p, kap ? k.p : nullptr, false, s), "apply");
    };
    int best = 0;
    for (size_t i = 0; i < c.size(); ++i) {
      set_variant(*M, precision, c[i]);
      for (int w = 0; w < 3; ++w) run();
      std::vector<float> t;
      for (int r = 0; r < trials; ++r) {
        hip_check(hipEventRecord(ev.a, s), "hipEventRecord");
        for (int j = 0; j < kReps; ++j) run();
        hip_check(hipEventRecord(ev.b, s), "hipEventRecord");
        hip_check(hipEventSynchronize(ev.b), "hipEventSynchronize");
        float ms = 0.0f;
        hip_check(hipEventElapsedTime(&ms, ev.a, ev.b), "hipEventElapsedTime");
        t.push_back(ms);
      }
      std::sort(t.begin(), t.end());
      out->kind[i] = c[i].kind;
      out->param[i] = c[i].param;
      out->us[i] = 1e3 * t[t.size() / 2] / kReps;
      if (out->us[i] < out->us[best]) best = (int)i;
    }
    out->ncand = (int)c.size();
    out->chosen = best;
    set_variant(*M, precision, c[best]);
    hip_check(hipStreamSynchronize(s), "hipStreamSynchronize");
    return DG_OK;
  });
}

}  // extern "C"
