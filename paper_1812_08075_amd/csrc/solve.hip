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
// Convergence is declared on the true FP64 residual |b - A x| <= rtol |b| in
// every mode.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
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

void dev_alloc(DevMem& m, size_t bytes) {
  if (hipMalloc(&m.p, bytes > 0 ? bytes : 1) != hipSuccess) {
    (void)hipGetLastError();
    throw SolveError{DG_ERR_ALLOC, "device allocation failed"};
  }
}

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char* pa = (const char*)a;
  const char* pb = (const char*)b;
  return pa < pb + nb && pb < pa + na;
}

class Solver {
 public:
  Solver(const dg_mesh& M, const void* kappa, bool pc, hipStream_t s)
      : M_(M), kappa_(kappa), s_(s), n_(M.ndofs), pc_(pc) {
    const bool kap = kappa != nullptr;
    const int64_t napply =
        std::max(dgi::scalar_apply_blocks(M, DG_F64, kap), dgi::scalar_apply_blocks(M, DG_F32, kap));
    int64_t np = std::max<int64_t>(dgi::RED_BLOCKS, napply);
    if (pc) np = std::max(np, dgi::block_jacobi_blocks(M));
    dev_alloc(partial_, sizeof(double) * np);
    if (pc) dev_alloc(partial2_, sizeof(double) * np);
    dev_alloc(state_, sizeof(dgi::CgState));
    if (hipHostMalloc(&host_.p, sizeof(dgi::CgState)) != hipSuccess) {
      (void)hipGetLastError();
      throw SolveError{DG_ERR_ALLOC, "pinned host allocation failed"};
    }
    ck(dgi::blas_state_zero(st(), s_), "state init");
  }

  dgi::CgState* st() { return (dgi::CgState*)state_.p; }
  double* partial() { return (double*)partial_.p; }

  dgi::CgState read() {
    ck(hipMemcpyAsync(host_.p, state_.p, sizeof(dgi::CgState), hipMemcpyDeviceToHost, s_), "state readback");
    ck(hipStreamSynchronize(s_), "hipStreamSynchronize");
    return *(dgi::CgState*)host_.p;
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
      ck(dgi::block_jacobi_update(M_, prec, r, q, alpha, z, partial(), (double*)partial2_.p, s_),
         "residual update and preconditioner");
      ck(dgi::blas_finalize((double*)partial2_.p, nb, st(), dgi::OP_RR, s_), "r.r");
      ck(dgi::blas_finalize(partial(), nb, st(), dgi::OP_BETA_PC, s_), "r.z");
      ck(dgi::blas_xp_update(x, p, z, prec, n_, st(), s_), "x and p update");
    } else {
      ck(dgi::blas_r_update(r, q, prec, n_, partial(), st(), dgi::OP_BETA, s_), "residual update");
      ck(dgi::blas_xp_update(x, p, r, prec, n_, st(), s_), "x and p update");
    }
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
  DevMem partial_, partial2_, state_;
  HostPinned host_;
};

dg_status run(const dg_mesh* M, int mode, const double* b, double* x, const void* kappa, const dg_solve_params* prm,
              dg_solve_info* info, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  const bool pc = prm->precond == DG_PRECOND_BLOCK_JACOBI;
  Solver S(*M, kappa, pc, s);
  const int64_t n = S.n();
  const int check = prm->check_every > 0 ? prm->check_every : 10;
  DevMem r, p, q;
  dev_alloc(r, sizeof(double) * n);
  dev_alloc(q, sizeof(double) * n);
  ck(dgi::blas_dot(b, b, DG_F64, n, S.partial(), S.st(), dgi::OP_NORM, s), "b.b");
  const double bnorm = std::sqrt(S.read().nrm2);
  info->iterations = 0;
  info->outer = 0;
  dg_status status = DG_OK;
  if (bnorm == 0.0) {
    ck(hipMemsetAsync(x, 0, sizeof(double) * n, s), "zero x");
    ck(hipStreamSynchronize(s), "hipStreamSynchronize");
    info->rel_residual = 0.0;
    return DG_OK;
  }
  const double target = prm->rtol * bnorm;
  int breakdown = 0;
  double res = std::sqrt(S.true_residual(b, x, (double*)r.p, (double*)q.p));

  if (mode == DG_SOLVE_CG_F64) {
    DevMem zv;
    dev_alloc(p, sizeof(double) * n);
    if (pc) dev_alloc(zv, sizeof(double) * n);
    int total = 0;
    // restart from the true residual whenever the recursive one has converged but
    // the true one has not (residual replacement)
    while (res > target && total < prm->maxit && !breakdown) {
      ck(dgi::blas_state_from_norm(S.st(), s), "state");
      S.start_direction(DG_F64, r.p, p.p, zv.p);
      total += S.cg(DG_F64, x, r.p, p.p, q.p, zv.p, kappa, target, prm->maxit - total, check, &breakdown);
      res = std::sqrt(S.true_residual(b, x, (double*)r.p, (double*)q.p));
    }
    info->iterations = total;
  } else if (mode == DG_SOLVE_RU_F32) {
    // one FP32 CG whose residual is replaced by the true FP64 residual (and its
    // iterate moved into x) each time it has dropped by RU_DROP since the last
    // replacement; the search direction is kept across replacements
    // below ~1e-3 per correction the FP32 recursion would run past FP32 accuracy
    const double RU_DROP = (prm->inner_rtol >= 1e-3 && prm->inner_rtol < 1.0) ? prm->inner_rtol : 0.1;
    DevMem rl, pl, ql, xl, zl, k32;
    dev_alloc(rl, sizeof(float) * n);
    dev_alloc(pl, sizeof(float) * n);
    dev_alloc(ql, sizeof(float) * n);
    dev_alloc(xl, sizeof(float) * n);
    if (pc) dev_alloc(zl, sizeof(float) * n);
    const void* kap32 = nullptr;
    if (kappa) {
      dev_alloc(k32, sizeof(float) * M->nqp);
      ck(dgi::blas_round_f32((const double*)kappa, (float*)k32.p, M->nqp, s), "kappa to FP32");
      kap32 = k32.p;
    }
    ck(dgi::blas_zero(xl.p, DG_F32, n, s), "xl = 0");
    ck(dgi::blas_round_f32((const double*)r.p, (float*)rl.p, n, s), "r to FP32");
    S.start_direction(DG_F32, rl.p, pl.p, zl.p);
    ck(dgi::blas_dot(rl.p, rl.p, DG_F32, n, S.partial(), S.st(), dgi::OP_SET_RR, s), "r.r");
    double last = std::sqrt(S.read().rr);
    double lowest = last;  // smallest recursive residual since the last correction
    double prev = last;    // recursive residual at the previous check
    int growth = 0;        // consecutive checks with a growing residual
    int total = 0, outer = 0, since_restart = 0;
    while (res > target && total < prm->maxit && !breakdown) {
      for (int it = 0; it < check && total < prm->maxit; ++it, ++total, ++since_restart)
        S.iterate(DG_F32, xl.p, rl.p, pl.p, ql.p, zl.p, kap32);
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
        if (std::isfinite(cur)) ck(dgi::blas_accumulate(x, (float*)xl.p, n, s), "x += xl");
        else ck(dgi::blas_zero(xl.p, DG_F32, n, s), "xl = 0");
        ++outer;
        res = std::sqrt(S.true_residual(b, x, (double*)r.p, (double*)q.p));
        if (res <= target) break;
        ck(dgi::blas_round_f32((const double*)r.p, (float*)rl.p, n, s), "r to FP32");
        if (lost) {
          ck(dgi::blas_state_zero(S.st(), s), "state reset");
          S.start_direction(DG_F32, rl.p, pl.p, zl.p);
          since_restart = 0;
        } else if (pc) {
          // the kept direction continues with r.z of the replaced residual
          S.precond(DG_F32, rl.p, zl.p, dgi::OP_SET_RZ);
        }
        ck(dgi::blas_dot(rl.p, rl.p, DG_F32, n, S.partial(), S.st(), dgi::OP_SET_RR, s), "r.r");
        last = lowest = prev = std::sqrt(S.read().rr);
        growth = 0;
      }
    }
    info->iterations = total;
    info->outer = outer;
  } else {
    DevMem rh, ph, qh, dh, zh, k32;
    dev_alloc(rh, sizeof(float) * n);
    dev_alloc(ph, sizeof(float) * n);
    dev_alloc(qh, sizeof(float) * n);
    dev_alloc(dh, sizeof(float) * n);
    if (pc) dev_alloc(zh, sizeof(float) * n);
    const void* kap32 = nullptr;
    if (kappa) {
      dev_alloc(k32, sizeof(float) * M->nqp);
      ck(dgi::blas_round_f32((const double*)kappa, (float*)k32.p, M->nqp, s), "kappa to FP32");
      kap32 = k32.p;
    }
    int total = 0, outer = 0;
    while (res > target && outer < prm->max_outer && total < prm->maxit && !breakdown) {
      // S.true_residual left r = b - A x and nrm2 = |r|^2 on the device
      ck(dgi::blas_ir_start((const double*)r.p, (float*)rh.p, (float*)ph.p, (float*)dh.p, n, S.st(), s), "ir start");
      ck(dgi::blas_dot(rh.p, rh.p, DG_F32, n, S.partial(), S.st(), dgi::OP_SET_RR, s), "rhat.rhat");
      if (pc) S.start_direction(DG_F32, rh.p, ph.p, zh.p);  // blas_ir_start set p = rhat
      const double inner_tol = prm->inner_rtol * std::sqrt(S.read().rr0);
      int inner_lost = 0;
      const int its =
          S.cg(DG_F32, dh.p, rh.p, ph.p, qh.p, zh.p, kap32, inner_tol, prm->maxit - total, check, &inner_lost);
      total += its;
      // nrm2 still holds |r|^2 of this outer step
      ck(dgi::blas_ir_correct(x, (const float*)dh.p, n, S.st(), s), "x += |r| d");
      ++outer;
      const double prev = res;
      res = std::sqrt(S.true_residual(b, x, (double*)r.p, (double*)q.p));
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

}  // namespace

extern "C" dg_status dg_solve(const dg_mesh* M, int mode, const double* b, double* x, const void* kappa,
                              const dg_solve_params* prm, dg_solve_info* info, void* stream) {
  try {
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
    if (mode != DG_SOLVE_CG_F64 && mode != DG_SOLVE_IR_F32 && mode != DG_SOLVE_RU_F32) {
      dg_set_error("unknown solve mode");
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
    return run(M, mode, b, x, kap ? kappa : nullptr, prm, info, (hipStream_t)stream);
  } catch (const SolveError& e) {
    dg_set_error(e.msg);
    return e.st;
  } catch (...) {
    dg_set_error("dg_solve: unexpected exception");
    return DG_ERR_DEVICE;
  }
}
