// Matrix-free solvers of the SIPG system A x = b (diffusion-reaction, theta = -1,
// so A is symmetric positive definite): CG in FP64, and two refinement
// schemes whose CG applies the FP32 operator. Every CG runs either
// unpreconditioned or with the block-Jacobi preconditioner z = P r (the
// inverse diagonal cell blocks; PCG: alpha = r.z / p.Ap, beta = r_new.z_new /
// r.z, p = z + beta p; r.z comes out of the preconditioner kernel).
//
// Classic refinement (DG_SOLVE_IR_F32): r = b - A x in FP64 (FP64 apply),
// rhat = r / |r| rounded to FP32, a fresh inner CG on A_32 d = rhat with FP32
// vectors and FP64 inner products down to |rhat - A_32 d| <= inner_rtol, then
// x += |r| d in FP64.
//
// Refinement keeping the Krylov space (DG_SOLVE_RU_F32): one FP32 CG runs
// throughout on the correction; each time its recursive residual has dropped
// by the factor inner_rtol (in [1e-3, 1), else 0.1) since the last correction, its
// iterate is added to x in FP64 and its
// residual is replaced by the true FP64 b - A x (rounded to FP32) while the
// search direction is kept, so the convergence of the Krylov space is not
// restarted.
//
// Chebyshev-preconditioned CG (DG_SOLVE_CHEB_F32 / _F64): FP64 CG whose
// preconditioner is s steps of the Chebyshev iteration for A z = r (with the
// block-Jacobi inverse P: for P A z = P r) on the interval [b / ratio, b], run
// on the FP32 (or FP64) operator from z = 0. The map r -> z is a fixed
// polynomial in P A times P, symmetric and positive definite when the
// spectrum of P A lies in (0, b], so the outer iteration is ordinary PCG;
// the inner iteration takes no inner products, and FP32 rounding in it only
// perturbs the preconditioner. b is cheb_margin times the largest eigenvalue
// of the Lanczos matrix built from the step lengths and direction updates of
// the first FP64 CG iterations, which the solve runs first.
//
// Convergence is declared on the true FP64 residual |b - A x| <= rtol |b| in
// every mode.
//
// Device memory of a solve (vectors, per-block partial sums, the CG state) is
// one block laid out by `layout`: dg_solve allocates it per call, while
// dg_solve_noalloc takes it from a fixed device array of this file, for
// callers that cannot allocate.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <mutex>
#include <string>

#include "solver.h"

namespace {

struct DevMem {
  void* p = nullptr;
  ~DevMem() {
    if (p) (void)hipFree(p);
  }
};

struct HostPinned {
  void* p = nullptr;
  ~HostPinned() {
    if (p) (void)hipHostFree(p);
  }
};

struct SolveError {
  dg_status st;
  std::string msg;
};

void ck(hipError_t e, const char* what) {
  if (e != hipSuccess) throw SolveError{DG_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e)};
}

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = (const char*)a;
  const char* pb = (const char*)b;
  return pa < pb + nb && pb < pa + na;
}

// The device memory of one solve, carved out of one block.
struct Work {
  double* partial = nullptr;   // per-block partial sums
  double* partial2 = nullptr;  // second set (preconditioned CG: r.r beside r.z)
  dgi::CgState* state = nullptr;
  double* r = nullptr;         // FP64 residual b - A x
  double* q = nullptr;         // FP64 scratch (A x, A p)
  double* p = nullptr;         // FP64 CG: search direction
  double* z = nullptr;         // FP64 PCG: preconditioned residual
  float* f[5] = {};            // FP32 CG: residual, direction, A p, iterate, preconditioned residual;
                               // FP32 Chebyshev: right-hand side, iterate, step, A z
  double* d = nullptr;         // FP64 Chebyshev: step
  double* t = nullptr;         // FP64 Chebyshev: A z
  double* hist = nullptr;      // Lanczos coefficients (alpha, beta) of the first CG iterations
  float* k32 = nullptr;        // kappa rounded to FP32
};

constexpr int kMaxLanczos = 64;
constexpr int kMaxChebDegree = 64;

bool cheb_mode(int mode) { return mode == DG_SOLVE_CHEB_F32 || mode == DG_SOLVE_CHEB_F64; }

// Largest eigenvalue of the Lanczos matrix of k CG iterations with step
// lengths alpha_j and direction updates beta_j (hist[2j], hist[2j+1]): the
// symmetric tridiagonal T with T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1} and
// T_{j,j+1} = sqrt(beta_j)/alpha_j, whose eigenvalues are the Ritz values of
// the (preconditioned) operator on the Krylov space. Bisection on the Sturm
// count inside the Gershgorin interval. Returns 0 if a coefficient is not a
// positive finite number.
double lanczos_max(const double* hist, int k) {
  double dg[kMaxLanczos], off[kMaxLanczos];
  for (int j = 0; j < k; ++j) {
    const double al = hist[2 * j];
    if (!(al > 0.0) || !std::isfinite(al)) return 0.0;
    dg[j] = 1.0 / al;
    if (j > 0) dg[j] += hist[2 * j - 1] / hist[2 * j - 2];
    if (j + 1 < k) {
      const double be = hist[2 * j + 1];
      if (!(be >= 0.0) || !std::isfinite(be)) return 0.0;
      off[j] = std::sqrt(be) / al;
    }
  }
  double lo = 0.0, hi = 0.0;
  for (int j = 0; j < k; ++j) {
    const double r = (j > 0 ? off[j - 1] : 0.0) + (j + 1 < k ? off[j] : 0.0);
    hi = std::max(hi, dg[j] + r);
  }
  // number of eigenvalues of T smaller than x
  auto count_below = [&](double x) {
    int c = 0;
    double q = dg[0] - x;
    if (q < 0) ++c;
    for (int j = 1; j < k; ++j) {
      const double den = q != 0.0 ? q : 1e-300;
      q = dg[j] - x - off[j - 1] * off[j - 1] / den;
      if (q < 0) ++c;
    }
    return c;
  };
  for (int it = 0; it < 200 && hi - lo > 1e-14 * hi; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (count_below(mid) >= k) hi = mid; else lo = mid;
  }
  return hi;
}

// Lays out the memory of a solve from `base` (nullptr: only counts) and
// returns its size in bytes. Every piece starts on a 256-byte boundary.
size_t layout(const dg_mesh& M, int mode, bool pc, bool kap, char* base, Work* w) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    off = (off + 255) & ~(size_t)255;
    void* ptr = base ? base + off : nullptr;
    off += bytes > 0 ? bytes : 1;
    return ptr;
  };
  const size_t n = (size_t)M.ndofs;
  int64_t np = std::max(dgi::scalar_apply_blocks(M, DG_F64, kap), dgi::scalar_apply_blocks(M, DG_F32, kap));
  np = std::max<int64_t>(np, dgi::RED_BLOCKS);
  np = std::max<int64_t>(np, dgi::blas_cheb_blocks((int64_t)n));
  np = std::max(np, dgi::block_jacobi_blocks(M));
  w->partial = (double*)take(sizeof(double) * np);
  if (pc) w->partial2 = (double*)take(sizeof(double) * np);
  w->state = (dgi::CgState*)take(sizeof(dgi::CgState));
  w->r = (double*)take(sizeof(double) * n);
  w->q = (double*)take(sizeof(double) * n);
  if (mode == DG_SOLVE_CG_F64) {
    w->p = (double*)take(sizeof(double) * n);
    if (pc) w->z = (double*)take(sizeof(double) * n);
  } else if (cheb_mode(mode)) {
    w->hist = (double*)take(sizeof(double) * 4 * kMaxLanczos);  // two runs of (alpha, beta)
    w->p = (double*)take(sizeof(double) * n);
    if (pc || mode == DG_SOLVE_CHEB_F64) w->z = (double*)take(sizeof(double) * n);
    if (mode == DG_SOLVE_CHEB_F64) {
      w->d = (double*)take(sizeof(double) * n);
      w->t = (double*)take(sizeof(double) * n);
    } else {
      for (int i = 0; i < 4; ++i) w->f[i] = (float*)take(sizeof(float) * n);
      if (kap) w->k32 = (float*)take(sizeof(float) * (size_t)M.nqp);
    }
  } else {
    for (int i = 0; i < 4; ++i) w->f[i] = (float*)take(sizeof(float) * n);
    if (pc) w->f[4] = (float*)take(sizeof(float) * n);
    if (kap) w->k32 = (float*)take(sizeof(float) * (size_t)M.nqp);
  }
  return (off + 255) & ~(size_t)255;
}

class Solver {
 public:
  // host: where the state record is read back to (pinned or ordinary memory)
  Solver(const dg_mesh& M, const void* kappa, bool pc, const Work& w, dgi::CgState* host, hipStream_t s)
      : M_(M), kappa_(kappa), s_(s), n_(M.ndofs), pc_(pc), w_(w), host_(host) {
    ck(dgi::blas_state_zero(st(), s_), "state init");
  }

  dgi::CgState* st() { return w_.state; }
  double* partial() { return w_.partial; }

  dgi::CgState read() {
    ck(hipMemcpyAsync(host_, w_.state, sizeof(dgi::CgState), hipMemcpyDeviceToHost, s_), "state readback");
    ck(hipStreamSynchronize(s_), "hipStreamSynchronize");
    return *host_;
  }

  void apply(int prec, const void* x, void* y, const void* kappa) {
    ck(dgi::scalar_apply(M_, prec, x, y, kappa, false, s_), "apply");
  }

  // z = P r and r.z reduced into the state with `op` (OP_SET_RZ or OP_BETA_PC)
  void precond(int prec, const void* r, void* z, int op) {
    ck(dgi::block_jacobi(M_, prec, r, z, partial(), s_), "preconditioner");
    ck(dgi::blas_finalize(partial(), dgi::block_jacobi_blocks(M_), st(), op, s_), "r.z");
  }

  // first search direction of a (re)started CG: p = P r (with rz) or p = r
  void start_direction(int prec, const void* r, void* p, void* z) {
    if (pc_) {
      precond(prec, r, z, dgi::OP_SET_RZ);
      ck(dgi::blas_copy(z, p, prec, n_, s_), "p = z");
    } else {
      ck(dgi::blas_copy(r, p, prec, n_, s_), "p = r");
    }
  }

  // one CG iteration: q = A p (with p.q), r -= alpha q, then x += alpha p and
  // p = r + beta p in one pass (preconditioned: the residual update runs in
  // the preconditioner's pass, z = P r, p = z + beta p)
  void iterate(int prec, void* x, void* r, void* p, void* q, void* z, const void* kappa) {
    // q = A p with p.q reduced per block by the apply kernel itself
    ck(dgi::scalar_apply(M_, prec, p, q, kappa, false, s_, partial()), "apply");
    ck(dgi::blas_finalize(partial(), dgi::scalar_apply_blocks(M_, prec, kappa != nullptr), st(),
                          pc_ ? dgi::OP_ALPHA_PC : dgi::OP_ALPHA, s_),
       "p.Ap");
    if (pc_) {
      const double* alpha = reinterpret_cast<const double*>(reinterpret_cast<const char*>(st()) +
                                                            offsetof(dgi::CgState, alpha));
      const int64_t nb = dgi::block_jacobi_blocks(M_);
      ck(dgi::block_jacobi_update(M_, prec, r, q, alpha, z, partial(), w_.partial2, s_),
         "residual update and preconditioner");
      ck(dgi::blas_finalize(w_.partial2, nb, st(), dgi::OP_RR, s_), "r.r");
      ck(dgi::blas_finalize(partial(), nb, st(), dgi::OP_BETA_PC, s_), "r.z");
      ck(dgi::blas_xp_update(x, p, z, prec, n_, st(), s_), "x and p update");
    } else {
      ck(dgi::blas_r_update(r, q, prec, n_, partial(), st(), dgi::OP_BETA, s_), "residual update");
      ck(dgi::blas_xp_update(x, p, r, prec, n_, st(), s_), "x and p update");
    }
  }

  // z = C r: s steps of the Chebyshev iteration for (P) A z = (P) r from z = 0
  // on [lo, hi], in precision `prec` (rin: the right-hand side in that
  // precision; rd: the same in FP64, from which the last step reads it and
  // forms r.z), then r.z reduced into the state with `op`. With `fused`, the
  // steps k >= 1 run as one pass each (apply, residual, preconditioner and
  // update together) that writes the new iterate to the other of z and t.
  // Returns the vector that holds the result (z or t).
  void* cheb_precond(int prec, const void* rin, const double* rd, void* z, void* d, void* t, const void* kappa,
                     int s, double lo, double hi, int op, bool fused, int* applies) {
    const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
    double rho = 1.0 / sigma;
    int64_t nb = pc_ ? dgi::block_jacobi_blocks(M_) : dgi::blas_cheb_blocks(n_);
    for (int k = 0; k < s; ++k) {
      const bool first = k == 0, last = k == s - 1;
      double c1 = 0.0, c2 = 1.0 / theta;
      if (!first) {
        const double rho_new = 1.0 / (2.0 * sigma - rho);
        c1 = rho_new * rho;
        c2 = 2.0 * rho_new / delta;
        rho = rho_new;
        ++*applies;
        if (fused) {
          ck(dgi::cheb_apply(M_, prec, z, t, kappa, rin, last ? rd : nullptr, d, c1, c2, last, pc_, partial(), s_),
             "Chebyshev step");
          std::swap(z, t);
          if (last) nb = dgi::block_jacobi_blocks(M_);
          continue;
        }
        apply(prec, z, t, kappa);
      }
      if (pc_)
        ck(dgi::cheb_block_jacobi(M_, prec, rin, last ? rd : nullptr, t, d, z, c1, c2, first, last, partial(), s_),
           "Chebyshev step");
      else
        ck(dgi::blas_cheb_step(prec, rin, last ? rd : nullptr, t, d, z, c1, c2, first, last, n_, partial(), s_),
           "Chebyshev step");
    }
    ck(dgi::blas_finalize(partial(), nb, st(), op, s_), "r.z");
    return z;
  }

  // nrm2 = |b - A x|^2 with r = b - A x (q is scratch)
  double true_residual(const double* b, const double* x, double* r, double* q) {
    apply(DG_F64, x, q, kappa_);
    ck(dgi::blas_residual(b, q, r, n_, partial(), st(), s_), "residual");
    return read().nrm2;
  }

  // CG on A_prec z = rhs (r holds the initial residual rhs - A z, p the
  // first search direction from start_direction, st()->rr the square norm of
  // r). Runs until sqrt(rr) <= tol or `budget` iterations; returns the
  // iterations done. zp: preconditioned residual (preconditioned runs).
  int cg(int prec, void* z, void* r, void* p, void* q, void* zp, const void* kappa, double tol, int budget, int check,
         int* breakdown) {
    int it = 0;
    while (it < budget) {
      if (it % check == 0) {
        const dgi::CgState h = read();
        if (h.breakdown) {
          *breakdown = 1;
          return it;
        }
        if (std::sqrt(h.rr) <= tol) return it;
      }
      iterate(prec, z, r, p, q, zp, kappa);
      ++it;
    }
    const dgi::CgState h = read();
    if (h.breakdown) *breakdown = 1;
    return it;
  }

  int64_t n() const { return n_; }
  hipStream_t stream() const { return s_; }

 private:
  const dg_mesh& M_;
  const void* kappa_;
  hipStream_t s_;
  int64_t n_;
  bool pc_;
  const Work& w_;
  dgi::CgState* host_;
};

dg_status run(const dg_mesh* M, int mode, const double* b, double* x, const void* kappa, const dg_solve_params* prm,
              dg_solve_info* info, const Work& w, dgi::CgState* host, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  const bool pc = prm->precond == DG_PRECOND_BLOCK_JACOBI;
  Solver S(*M, kappa, pc, w, host, s);
  const int64_t n = S.n();
  const int check = prm->check_every > 0 ? prm->check_every : 10;
  double* r = w.r;
  double* q = w.q;
  ck(dgi::blas_dot(b, b, DG_F64, n, S.partial(), S.st(), dgi::OP_NORM, s), "b.b");
  const double bnorm = std::sqrt(S.read().nrm2);
  info->iterations = 0;
  info->outer = 0;
  info->rel_residual = 0.0;
  info->seconds = 0.0;
  info->inner_applies = 0;
  info->lanczos_iterations = 0;
  info->lambda_max = 0.0;
  dg_status status = DG_OK;
  if (bnorm == 0.0) {
    ck(dgi::blas_zero(x, DG_F64, n, s), "zero x");
    ck(hipStreamSynchronize(s), "hipStreamSynchronize");
    return DG_OK;
  }
  const double target = prm->rtol * bnorm;
  int breakdown = 0;
  double res = std::sqrt(S.true_residual(b, x, r, q));

  if (mode == DG_SOLVE_CG_F64) {
    double* p = w.p;
    double* zv = w.z;
    int total = 0;
    // restart from the true residual whenever the recursive one has converged but
    // the true one has not (residual replacement)
    while (res > target && total < prm->maxit && !breakdown) {
      ck(dgi::blas_state_from_norm(S.st(), s), "state");
      S.start_direction(DG_F64, r, p, zv);
      total += S.cg(DG_F64, x, r, p, q, zv, kappa, target, prm->maxit - total, check, &breakdown);
      res = std::sqrt(S.true_residual(b, x, r, q));
    }
    info->iterations = total;
  } else if (cheb_mode(mode)) {
    const bool f32 = mode == DG_SOLVE_CHEB_F32;
    const int ip = f32 ? DG_F32 : DG_F64;
    const int deg = prm->cheb_degree > 0 ? prm->cheb_degree : 8;
    const int nlz = prm->cheb_lanczos > 0 ? prm->cheb_lanczos : 20;
    const double ratio = prm->cheb_ratio > 0.0 ? prm->cheb_ratio : std::max(16.0, (double)deg * deg);
    double margin = prm->cheb_margin > 0.0 ? prm->cheb_margin : 1.1;
    double* p = w.p;
    double* zv = w.z;
    void* zc = f32 ? (void*)w.f[1] : (void*)w.z;  // the Chebyshev iterate
    void* dc = f32 ? (void*)w.f[2] : (void*)w.d;
    void* tc = f32 ? (void*)w.f[3] : (void*)w.t;
    float* r32 = w.f[0];
    const void* kapc = kappa;
    if (kappa && f32) {
      ck(dgi::blas_round_f32((const double*)kappa, w.k32, M->nqp, s), "kappa to FP32");
      kapc = w.k32;
    }
    // the inner steps fused into the line kernel, unless the operator runs
    // on the matrix-core kernel in this precision
    const bool fused = !dgi::mfma_apply_supported(*M, ip, kapc != nullptr) &&
                       !dgi::mfma_apply_f32_supported(*M, ip, kapc != nullptr);
    int total = 0, applies = 0, outer = 0;
    // 1. the spectrum, from two Lanczos matrices: (a) nlz (P)CG iterations in
    // the inner precision on a fixed pseudo-random right-hand side (every
    // eigenvector present; the iterate is not kept: the buffer of A p stands
    // in for it, its update landing after A p has been used), (b) the first
    // nlz FP64 (P)CG iterations of the solve itself (they advance x). From a
    // smooth b alone the Krylov space can miss the top of the spectrum, and a
    // polynomial of even degree is not positive above b; from the random start
    // alone the outer CG would begin on the raw residual, which the FP32 inner
    // iteration serves worse. Both Ritz values lie below the largest
    // eigenvalue; the larger one sets the interval.
    {
      void* er = f32 ? (void*)w.f[0] : (void*)r;
      void* ep = f32 ? (void*)w.f[2] : (void*)p;
      void* eq = f32 ? (void*)w.f[3] : (void*)q;
      void* ez = f32 ? (void*)w.f[1] : (void*)zv;
      ck(dgi::blas_random(er, ip, n, 0x2545F4914F6CDD1Dull, s), "random right-hand side");
      ck(dgi::blas_dot(er, er, ip, n, S.partial(), S.st(), dgi::OP_NORM, s), "r.r");
      ck(dgi::blas_state_from_norm(S.st(), s), "state");
      S.start_direction(ip, er, ep, ez);
      for (int j = 0; j < nlz; ++j) {
        S.iterate(ip, eq, er, ep, eq, ez, kapc);
        ck(dgi::blas_record(S.st(), w.hist, j, s), "record");
      }
    }
    info->lanczos_iterations = nlz;
    // r = b - A x again (in FP64 mode the estimate ran in r's buffer)
    (void)S.true_residual(b, x, r, q);
    ck(dgi::blas_state_from_norm(S.st(), s), "state");
    S.start_direction(DG_F64, r, p, zv);
    int nrec = 0;
    for (; nrec < nlz && total < prm->maxit; ++nrec, ++total) {
      S.iterate(DG_F64, x, r, p, q, zv, kappa);
      ck(dgi::blas_record(S.st(), w.hist, nlz + nrec, s), "record");
    }
    double hist[4 * kMaxLanczos];
    ck(hipMemcpyAsync(hist, w.hist, sizeof(double) * 2 * (nlz + nrec), hipMemcpyDeviceToHost, s),
       "Lanczos readback");
    (void)S.read();  // also waits for the coefficients
    // a CG that converged (or broke down) within its iterations leaves a zero
    // step length behind: each estimate uses the iterations before it
    auto ritz_max = [&](const double* h, int k) {
      int nval = 0;
      while (nval < k && h[2 * nval] > 0.0 && std::isfinite(h[2 * nval])) ++nval;
      return nval >= 1 ? lanczos_max(h, nval) : 0.0;
    };
    const double lmax = std::max(ritz_max(hist, nlz), ritz_max(hist + 2 * nlz, nrec));
    info->lambda_max = lmax;
    res = std::sqrt(S.true_residual(b, x, r, q));
    if (res > target && !(lmax > 0.0)) breakdown = 1;
    // 2. CG preconditioned by the Chebyshev polynomial; restarted from the
    // true residual when the recursive one has converged but the true one
    // has not, and with a wider interval if the polynomial lost definiteness
    int widen = 0;
    while (res > target && total < prm->maxit && !breakdown) {
      const double hi = margin * lmax, lo = hi / ratio;
      ck(dgi::blas_state_from_norm(S.st(), s), "state");
      if (f32) ck(dgi::blas_round_f32(r, r32, n, s), "r to FP32");
      void* zr = S.cheb_precond(ip, f32 ? (const void*)r32 : (const void*)r, r, zc, dc, tc, kapc, deg, lo, hi,
                                dgi::OP_SET_RZ, fused, &applies);
      if (f32) ck(dgi::blas_widen((const float*)zr, p, n, s), "p = z");
      else ck(dgi::blas_copy((const double*)zr, p, DG_F64, n, s), "p = z");
      const int cstep = std::max(1, check / deg);
      int it = 0, lost = 0;
      while (total < prm->maxit) {
        if (it % cstep == 0) {
          const dgi::CgState h = S.read();
          if (h.breakdown) {
            lost = 1;
            break;
          }
          if (std::sqrt(h.rr) <= target) break;
        }
        // q = A p and p.Ap; alpha = r.z / p.Ap
        ck(dgi::scalar_apply(*M, DG_F64, p, q, kappa, false, s, S.partial()), "apply");
        ck(dgi::blas_finalize(S.partial(), dgi::scalar_apply_blocks(*M, DG_F64, kappa != nullptr), S.st(),
                              dgi::OP_ALPHA_PC, s),
           "p.Ap");
        // r -= alpha q with r.r (and its FP32 copy)
        if (f32) ck(dgi::blas_r_update_round(r, q, r32, n, S.partial(), S.st(), dgi::OP_RR, s), "residual update");
        else ck(dgi::blas_r_update(r, q, DG_F64, n, S.partial(), S.st(), dgi::OP_RR, s), "residual update");
        // z = C r with r.z; beta = r.z / previous r.z
        zr = S.cheb_precond(ip, f32 ? (const void*)r32 : (const void*)r, r, zc, dc, tc, kapc, deg, lo, hi,
                            dgi::OP_BETA_PC, fused, &applies);
        // x += alpha p; p = z + beta p
        if (f32) ck(dgi::blas_xp_update_mixed(x, p, (const float*)zr, n, S.st(), s), "x and p update");
        else ck(dgi::blas_xp_update(x, p, zr, DG_F64, n, S.st(), s), "x and p update");
        ++it;
        ++total;
      }
      ++outer;
      res = std::sqrt(S.true_residual(b, x, r, q));
      if (lost && res > target) {
        // a polynomial that is not positive on the spectrum shows as
        // p.Ap <= 0 or r.z < 0: widen the interval and start again from x
        if (++widen > 3) breakdown = 1;
        margin *= 1.5;
      }
    }
    info->iterations = total;
    info->outer = outer;
    info->inner_applies = applies;
  } else if (mode == DG_SOLVE_RU_F32) {
    // one FP32 CG whose residual is replaced by the true FP64 residual (and its
    // iterate moved into x) each time it has dropped by RU_DROP since the last
    // replacement; the search direction is kept across replacements
    // below ~1e-3 per correction the FP32 recursion would run past FP32 accuracy
    const double RU_DROP = (prm->inner_rtol >= 1e-3 && prm->inner_rtol < 1.0) ? prm->inner_rtol : 0.1;
    float *rl = w.f[0], *pl = w.f[1], *ql = w.f[2], *xl = w.f[3], *zl = w.f[4];
    const void* kap32 = nullptr;
    if (kappa) {
      ck(dgi::blas_round_f32((const double*)kappa, w.k32, M->nqp, s), "kappa to FP32");
      kap32 = w.k32;
    }
    ck(dgi::blas_zero(xl, DG_F32, n, s), "xl = 0");
    ck(dgi::blas_round_f32(r, rl, n, s), "r to FP32");
    S.start_direction(DG_F32, rl, pl, zl);
    ck(dgi::blas_dot(rl, rl, DG_F32, n, S.partial(), S.st(), dgi::OP_SET_RR, s), "r.r");
    double last = std::sqrt(S.read().rr);
    double lowest = last;  // smallest recursive residual since the last correction
    double prev = last;    // recursive residual at the previous check
    int growth = 0;        // consecutive checks with a growing residual
    int total = 0, outer = 0, since_restart = 0;
    while (res > target && total < prm->maxit && !breakdown) {
      for (int it = 0; it < check && total < prm->maxit; ++it, ++total, ++since_restart)
        S.iterate(DG_F32, xl, rl, pl, ql, zl, kap32);
      const dgi::CgState h = S.read();
      const double cur = std::sqrt(h.rr);
      // The FP32 recursion can lose its footing once its residual has drifted
      // below FP32 accuracy: p.Ap turns non-positive, or, with p.Ap still
      // positive, the recursive residual starts to grow geometrically. Either
      // triggers a correction with a fresh search direction; a loss right after
      // such a restart is a real breakdown.
      // (CG residuals are not monotone and spike briefly: growth counts only
      // when it has lasted three check windows in a row and exceeds a factor 4
      // over the lowest value since the last correction)
      growth = cur > prev ? growth + 1 : 0;
      prev = cur;
      const bool diverging = !std::isfinite(cur) || (growth >= 3 && cur > 4.0 * lowest);
      const bool lost = h.breakdown != 0 || diverging;
      lowest = std::min(lowest, cur);
      if (h.breakdown != 0 && since_restart <= check) {
        breakdown = 1;
        break;
      }
      if (lost || cur <= RU_DROP * last || cur <= target || total >= prm->maxit) {
        // a non-finite FP32 iterate is dropped rather than added
        if (std::isfinite(cur)) ck(dgi::blas_accumulate(x, xl, n, s), "x += xl");
        else ck(dgi::blas_zero(xl, DG_F32, n, s), "xl = 0");
        ++outer;
        res = std::sqrt(S.true_residual(b, x, r, q));
        if (res <= target) break;
        ck(dgi::blas_round_f32(r, rl, n, s), "r to FP32");
        if (lost) {
          ck(dgi::blas_state_zero(S.st(), s), "state reset");
          S.start_direction(DG_F32, rl, pl, zl);
          since_restart = 0;
        } else if (pc) {
          // the kept direction continues with r.z of the replaced residual
          S.precond(DG_F32, rl, zl, dgi::OP_SET_RZ);
        }
        ck(dgi::blas_dot(rl, rl, DG_F32, n, S.partial(), S.st(), dgi::OP_SET_RR, s), "r.r");
        last = lowest = prev = std::sqrt(S.read().rr);
        growth = 0;
      }
    }
    info->iterations = total;
    info->outer = outer;
  } else {
    float *rh = w.f[0], *ph = w.f[1], *qh = w.f[2], *dh = w.f[3], *zh = w.f[4];
    const void* kap32 = nullptr;
    if (kappa) {
      ck(dgi::blas_round_f32((const double*)kappa, w.k32, M->nqp, s), "kappa to FP32");
      kap32 = w.k32;
    }
    int total = 0, outer = 0;
    while (res > target && outer < prm->max_outer && total < prm->maxit && !breakdown) {
      // S.true_residual left r = b - A x and nrm2 = |r|^2 on the device
      ck(dgi::blas_ir_start(r, rh, ph, dh, n, S.st(), s), "ir start");
      ck(dgi::blas_dot(rh, rh, DG_F32, n, S.partial(), S.st(), dgi::OP_SET_RR, s), "rhat.rhat");
      if (pc) S.start_direction(DG_F32, rh, ph, zh);  // blas_ir_start set p = rhat
      const double inner_tol = prm->inner_rtol * std::sqrt(S.read().rr0);
      int inner_lost = 0;
      const int its =
          S.cg(DG_F32, dh, rh, ph, qh, zh, kap32, inner_tol, prm->maxit - total, check, &inner_lost);
      total += its;
      // nrm2 still holds |r|^2 of this outer step
      ck(dgi::blas_ir_correct(x, dh, n, S.st(), s), "x += |r| d");
      ++outer;
      const double prev = res;
      res = std::sqrt(S.true_residual(b, x, r, q));
      // an inner breakdown (FP32 rounding) just ends that inner solve; it is a
      // real breakdown only when the correction made no progress
      if (inner_lost && !(res < prev)) breakdown = 1;
    }
    info->iterations = total;
    info->outer = outer;
  }
  ck(hipStreamSynchronize(s), "hipStreamSynchronize");
  if (!std::isfinite(res)) breakdown = 1;  // never report a NaN/Inf residual as converged
  info->rel_residual = res / bnorm;
  info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (breakdown) {
    dg_set_error("CG breakdown: p.Ap <= 0 or a non-finite value (is the operator SPD, theta = -1?)");
    status = DG_BREAKDOWN;
  } else if (res > target) {
    dg_set_error("not converged within maxit / max_outer");
    status = DG_NOT_CONVERGED;
  }
  return status;
}

// Checks the arguments of dg_solve / dg_solve_noalloc (before any HIP call).
dg_status check_args(const dg_mesh* M, int mode, const double* b, double* x, const void* kappa,
                     const dg_solve_params* prm, dg_solve_info* info) {
  if (((uintptr_t)b | (uintptr_t)x | (uintptr_t)kappa) % 16) {
    dg_set_error("b, x and kappa must be 16-byte aligned");
    return DG_ERR_ARG;
  }
  if (!M || !b || !x || !prm || !info) {
    dg_set_error("mesh, b, x, params and info must not be NULL");
    return DG_ERR_ARG;
  }
  if (M->desc.problem != DG_PROBLEM_DIFFREAC) {
    dg_set_error("dg_solve is built for the diffusion-reaction operator");
    return DG_ERR_UNSUPPORTED;
  }
  if (mode != DG_SOLVE_CG_F64 && mode != DG_SOLVE_IR_F32 && mode != DG_SOLVE_RU_F32 && !cheb_mode(mode)) {
    dg_set_error("unknown solve mode");
    return DG_ERR_ARG;
  }
  if (cheb_mode(mode) &&
      (prm->cheb_degree < 0 || prm->cheb_degree > kMaxChebDegree || prm->cheb_lanczos < 0 ||
       prm->cheb_lanczos == 1 || prm->cheb_lanczos > kMaxLanczos || !(prm->cheb_ratio == 0.0 || prm->cheb_ratio > 1.0) ||
       !(prm->cheb_margin == 0.0 || prm->cheb_margin >= 1.0))) {
    dg_set_error("Chebyshev parameters: degree 0..64, lanczos 0 or 2..64, ratio 0 or > 1, margin 0 or >= 1");
    return DG_ERR_ARG;
  }
  if (!(prm->rtol > 0) || prm->maxit < 1 || (mode == DG_SOLVE_IR_F32 && (!(prm->inner_rtol > 0) || prm->max_outer < 1))) {
    dg_set_error("rtol, inner_rtol must be > 0; maxit, max_outer >= 1");
    return DG_ERR_ARG;
  }
  if (prm->precond != DG_PRECOND_NONE && prm->precond != DG_PRECOND_BLOCK_JACOBI) {
    dg_set_error("unknown preconditioner");
    return DG_ERR_ARG;
  }
  if (prm->precond == DG_PRECOND_BLOCK_JACOBI && !dgi::block_jacobi_supported(*M)) {
    dg_set_error("the block-Jacobi preconditioner is built for kappa = 1 and theta = -1");
    return DG_ERR_UNSUPPORTED;
  }
  const bool kap = M->desc.kappa_mode == DG_KAPPA_QP;
  if (kap && !kappa) {
    dg_set_error("kappa is required for kappa_mode DG_KAPPA_QP");
    return DG_ERR_ARG;
  }
  const size_t nb = sizeof(double) * (size_t)M->ndofs;
  if (overlap(b, nb, x, nb) || (kap && overlap(kappa, sizeof(double) * (size_t)M->nqp, x, nb))) {
    dg_set_error("x overlaps b or kappa");
    return DG_ERR_ARG;
  }
  return DG_OK;
}

// The fixed workspace of dg_solve_noalloc: one copy per device, for the life
// of the process. Host code never uses this name as an address (it is a
// host-side stand-in); it uses the device address from hipGetSymbolAddress.
constexpr size_t kScratchBytes = (size_t)64 << 20;
__device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
char* scratch_on_current_device() {
  int dev = 0;
  ck(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) throw SolveError{DG_ERR_UNSUPPORTED, "device index beyond the workspace table"};
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    ck(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!ptr) throw SolveError{DG_ERR_DEVICE, "hipGetSymbolAddress(scratch) returned NULL"};
    g_scratch_ptr[dev] = (char*)ptr;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" dg_status dg_solve(const dg_mesh* M, int mode, const double* b, double* x, const void* kappa,
                              const dg_solve_params* prm, dg_solve_info* info, void* stream) {
  try {
    const dg_status st = check_args(M, mode, b, x, kappa, prm, info);
    if (st != DG_OK) return st;
    const bool kap = M->desc.kappa_mode == DG_KAPPA_QP;
    const bool pc = prm->precond == DG_PRECOND_BLOCK_JACOBI;
    Work w;
    const size_t bytes = layout(*M, mode, pc, kap, nullptr, &w);
    DevMem mem;
    if (hipMalloc(&mem.p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      throw SolveError{DG_ERR_ALLOC, "device allocation failed"};
    }
    layout(*M, mode, pc, kap, (char*)mem.p, &w);
    HostPinned host;
    if (hipHostMalloc(&host.p, sizeof(dgi::CgState)) != hipSuccess) {
      (void)hipGetLastError();
      throw SolveError{DG_ERR_ALLOC, "pinned host allocation failed"};
    }
    return run(M, mode, b, x, kap ? kappa : nullptr, prm, info, w, (dgi::CgState*)host.p, (hipStream_t)stream);
  } catch (const SolveError& e) {
    dg_set_error(e.msg);
    return e.st;
  } catch (...) {
    dg_set_error("dg_solve: unexpected exception");
    return DG_ERR_DEVICE;
  }
}

extern "C" dg_status dg_solve_noalloc(const dg_mesh* M, int mode, const double* b, double* x, const void* kappa,
                                      const dg_solve_params* prm, dg_solve_info* info, void* stream) {
  try {
    const dg_status st = check_args(M, mode, b, x, kappa, prm, info);
    if (st != DG_OK) return st;
    const bool kap = M->desc.kappa_mode == DG_KAPPA_QP;
    const bool pc = prm->precond == DG_PRECOND_BLOCK_JACOBI;
    Work w;
    const size_t bytes = layout(*M, mode, pc, kap, nullptr, &w);
    if (bytes > kScratchBytes) {
      dg_set_error("dg_solve_noalloc: this solve needs " + std::to_string(bytes) +
                   " bytes of workspace, more than its fixed " + std::to_string(kScratchBytes) +
                   " (use dg_solve)");
      return DG_ERR_ARG;
    }
    layout(*M, mode, pc, kap, scratch_on_current_device(), &w);
    dgi::CgState host{};  // ordinary host memory: no pinned allocation
    return run(M, mode, b, x, kap ? kappa : nullptr, prm, info, w, &host, (hipStream_t)stream);
  } catch (const SolveError& e) {
    dg_set_error(e.msg);
    return e.st;
  } catch (...) {
    dg_set_error("dg_solve_noalloc: unexpected exception");
    return DG_ERR_DEVICE;
  }
}
