// Device state and vector kernels of the CG solvers.
#pragma once

#include "internal.h"

namespace dgi {

constexpr int RED_BLOCKS = 1024;  // fixed grid of the reductions (deterministic order)

// CG scalars kept on the device; the host reads the record every few iterations.
struct CgState {
  double rr;      // r.r of the current residual
  double rr0;     // r.r at the start of the run
  double pq;      // p.Ap
  double alpha;
  double beta;
  double nrm2;    // last norm computed with OP_NORM (outer residual of the refinement)
  double rz;      // r.z, z = P r (preconditioned CG)
  int32_t breakdown;
  int32_t pad;
};

// OP_SET_RR: rr = rr0 = s. OP_ALPHA: pq = s, alpha = rr / pq. OP_BETA: beta =
// s / rr, rr = s. OP_NORM: nrm2 = s. Preconditioned CG: OP_RR: rr = s;
// OP_SET_RZ: rz = s; OP_ALPHA_PC: pq = s, alpha = rz / pq; OP_BETA_PC:
// beta = s / rz, rz = s.
enum : int {
  OP_SET_RR = 0,
  OP_ALPHA = 1,
  OP_BETA = 2,
  OP_NORM = 3,
  OP_RR = 4,
  OP_SET_RZ = 5,
  OP_ALPHA_PC = 6,
  OP_BETA_PC = 7
};

// a.b (FP64 accumulation) reduced into the state with `op`.
hipError_t blas_dot(const void* a, const void* b, int prec, int64_t n, double* partial, CgState* st, int op,
                    hipStream_t s);
// Sums nb partial sums (fixed order) and applies `op` to the state.
hipError_t blas_finalize(const double* partial, int64_t nb, CgState* st, int op, hipStream_t s);
// r -= alpha q, then r.r reduced with `op` (OP_BETA or OP_RR).
hipError_t blas_r_update(void* r, const void* q, int prec, int64_t n, double* partial, CgState* st, int op,
                         hipStream_t s);
// x += alpha p, p = z + beta p in one pass.
hipError_t blas_xp_update(void* x, void* p, const void* z, int prec, int64_t n, CgState* st, hipStream_t s);
// r = b - Ax, nrm2 = r.r.
hipError_t blas_residual(const double* b, const double* Ax, double* r, int64_t n, double* partial, CgState* st,
                         hipStream_t s);
// rhat = r/|r| (FP32), p = rhat, d = 0, rr = 1.
hipError_t blas_ir_start(const double* r, float* rh, float* ph, float* d, int64_t n, CgState* st, hipStream_t s);
// x += |r| d.
hipError_t blas_ir_correct(double* x, const float* d, int64_t n, CgState* st, hipStream_t s);
hipError_t blas_copy(const void* a, void* b, int prec, int64_t n, hipStream_t s);
// x += xl (FP32 to FP64), xl = 0.
hipError_t blas_accumulate(double* x, float* xl, int64_t n, hipStream_t s);
hipError_t blas_zero(void* a, int prec, int64_t n, hipStream_t s);
hipError_t blas_round_f32(const double* a, float* b, int64_t n, hipStream_t s);
// b = a widened to FP64.
hipError_t blas_widen(const float* a, double* b, int64_t n, hipStream_t s);
// r -= alpha q (FP64), r.r reduced with `op`, and r32 = r rounded to FP32.
hipError_t blas_r_update_round(double* r, const double* q, float* r32, int64_t n, double* partial, CgState* st,
                               int op, hipStream_t s);
// x += alpha p, p = z + beta p with z in FP32 (x, p FP64).
hipError_t blas_xp_update_mixed(double* x, double* p, const float* z, int64_t n, CgState* st, hipStream_t s);
// One Chebyshev step without preconditioner (k_cheb_plain): w = r - t,
// d = c1 d + c2 w, z += d; the first step has t = d = z = 0; with rd (FP64
// right-hand side, read instead of r) the last step writes the partial sums of
// rd.z (blas_cheb_blocks(n) entries) and does not store d.
hipError_t blas_cheb_step(int prec, const void* r, const double* rd, const void* t, void* d, void* z, double c1,
                          double c2, bool first, bool last, int64_t n, double* partial, hipStream_t s);
int64_t blas_cheb_blocks(int64_t n);
// hist[2j] = alpha, hist[2j+1] = beta of the state.
hipError_t blas_record(const CgState* st, double* hist, int j, hipStream_t s);
// every field zero (a fresh state record).
hipError_t blas_state_zero(CgState* st, hipStream_t s);
// rr = rr0 = nrm2, alpha = beta = 0.
hipError_t blas_state_from_norm(CgState* st, hipStream_t s);
// a = pseudo-random values in [-1, 1), a function of the index and the seed only.
hipError_t blas_random(void* a, int prec, int64_t n, uint64_t seed, hipStream_t s);

}  // namespace dgi
