// Vector kernels of the conjugate-gradient solvers (gfx950).
//
// Every inner product accumulates in FP64, also for FP32 vectors, and is
// reduced in a fixed order: a fixed grid of RED_BLOCKS blocks writes one
// partial sum each (grid-stride loop, then a tree over the block), and a
// single-block kernel sums the partials in a fixed order. Results are
// therefore bitwise reproducible. The CG scalars (alpha, beta, r.r) stay on
// the device in a small state record read by the update kernels, so an
// iteration needs no host round trip.
#include "solver.h"

namespace dgi {
namespace {

constexpr int RT = 256;  // threads per reduction block

__device__ __forceinline__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int s = RT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  return sh[0];
}

template <typename T>
__global__ void __launch_bounds__(RT) k_dot(const T* __restrict__ a, const T* __restrict__ b, int64_t n,
                                            double* __restrict__ partial) {
  __shared__ double sh[RT];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x; i < n; i += (int64_t)gridDim.x * RT)
    acc = fma((double)a[i], (double)b[i], acc);
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Sums the partials (fixed order) and applies `op` to the CG state.
__global__ void __launch_bounds__(RT) k_finalize(const double* __restrict__ partial, int nb,
                                                 CgState* __restrict__ st, int op) {
  __shared__ double sh[RT];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += RT) acc += partial[i];
  const double s = block_sum(acc, sh);
  if (threadIdx.x != 0) return;
  switch (op) {
    case OP_SET_RR:
      st->rr = s;
      st->rr0 = s;
      break;
    case OP_ALPHA: {
      st->pq = s;
      const double alpha = (s > 0.0) ? st->rr / s : 0.0;
      // non-positive or non-finite p.Ap, or a step that would overflow FP32 vectors
      if (!(s > 0.0) || !isfinite(s) || !(alpha < 1e30)) {
        st->breakdown = 1;
        st->alpha = 0.0;
      } else {
        st->alpha = alpha;
      }
      break;
    }
    case OP_BETA:
      st->beta = (st->rr > 0.0) ? s / st->rr : 0.0;
      st->rr = s;
      if (!isfinite(s)) st->breakdown = 1;
      break;
    case OP_NORM:
      st->nrm2 = s;
      if (!isfinite(s)) st->breakdown = 1;
      break;
    case OP_RR:
      st->rr = s;
      if (!isfinite(s)) st->breakdown = 1;
      break;
    case OP_SET_RZ:
      st->rz = s;
      if (s < 0.0 || !isfinite(s)) st->breakdown = 1;  // P is SPD: r.z >= 0
      break;
    case OP_ALPHA_PC: {
      st->pq = s;
      const double alpha = (s > 0.0) ? st->rz / s : 0.0;
      if (!(s > 0.0) || !isfinite(s) || !(alpha < 1e30)) {
        st->breakdown = 1;
        st->alpha = 0.0;
      } else {
        st->alpha = alpha;
      }
      break;
    }
    case OP_BETA_PC:
      st->beta = (st->rz > 0.0) ? s / st->rz : 0.0;
      st->rz = s;
      if (!isfinite(s)) st->breakdown = 1;
      break;
  }
}

// r -= alpha q; partial sums of r.r
template <typename T>
__global__ void __launch_bounds__(RT) k_r_update(T* __restrict__ r, const T* __restrict__ q,
                                                 const CgState* __restrict__ st, int64_t n,
                                                 double* __restrict__ partial) {
  __shared__ double sh[RT];
  const T a = (T)st->alpha;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x; i < n; i += (int64_t)gridDim.x * RT) {
    const T ri = fma(-a, q[i], r[i]);
    r[i] = ri;
    acc = fma((double)ri, (double)ri, acc);
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// x += alpha p; p = z + beta p (z: the residual, or the preconditioned one)
template <typename T>
__global__ void __launch_bounds__(RT) k_xp_update(T* __restrict__ x, T* __restrict__ p, const T* __restrict__ z,
                                                  const CgState* __restrict__ st, int64_t n) {
  const T a = (T)st->alpha, b = (T)st->beta;
  for (int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x; i < n; i += (int64_t)gridDim.x * RT) {
    const T pi = p[i];
    x[i] = fma(a, pi, x[i]);
    p[i] = fma(b, pi, z[i]);
  }
}

// r = b - Ax (FP64); partial sums of r.r
__global__ void __launch_bounds__(RT) k_residual(const double* __restrict__ b, const double* __restrict__ Ax,
                                                 double* __restrict__ r, int64_t n, double* __restrict__ partial) {
  __shared__ double sh[RT];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x; i < n; i += (int64_t)gridDim.x * RT) {
    const double ri = b[i] - Ax[i];
    r[i] = ri;
    acc = fma(ri, ri, acc);
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Inner system of the refinement: rhat = r / |r| rounded to FP32; d = 0; p = rhat.
__global__ void __launch_bounds__(RT) k_ir_start(const double* __restrict__ r, const CgState* __restrict__ st,
                                                 float* __restrict__ rh, float* __restrict__ ph,
                                                 float* __restrict__ d, int64_t n) {
  const double inv = 1.0 / sqrt(st->nrm2);
  for (int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x; i < n; i += (int64_t)gridDim.x * RT) {
    const float v = (float)(r[i] * inv);
    rh[i] = v;
    ph[i] = v;
    d[i] = 0.0f;
  }
}

// x += |r| d (FP64 update with the FP32 correction)
__global__ void __launch_bounds__(RT) k_ir_correct(double* __restrict__ x, const float* __restrict__ d,
                                                   const CgState* __restrict__ st, int64_t n) {
  const double s = sqrt(st->nrm2);
  for (int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x; i < n; i += (int64_t)gridDim.x * RT)
    x[i] = fma(s, (double)d[i], x[i]);
}

// x += (FP64) xl; xl = 0 (the FP32 iterate of the refinement moves into x)
__global__ void __launch_bounds__(RT) k_accumulate(double* __restrict__ x, float* __restrict__ xl, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x; i < n; i += (int64_t)gridDim.x * RT) {
    x[i] += (double)xl[i];
    xl[i] = 0.0f;
  }
}

template <typename T>
__global__ void __launch_bounds__(RT) k_fill(T* __restrict__ a, T v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x; i < n; i += (int64_t)gridDim.x * RT) a[i] = v;
}

template <typename T>
__global__ void __launch_bounds__(RT) k_copy(const T* __restrict__ a, T* __restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x; i < n; i += (int64_t)gridDim.x * RT) b[i] = a[i];
}

__global__ void __launch_bounds__(RT) k_round_f32(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x; i < n; i += (int64_t)gridDim.x * RT) b[i] = (float)a[i];
}

// Sets the scalars of a fresh CG run (r.r taken from nrm2 or 1 for the
// normalized inner right-hand side).
__global__ void k_state_reset(CgState* st, int from_norm) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const double rr = from_norm ? st->nrm2 : 1.0;
    st->rr = rr;
    st->rr0 = rr;
    st->alpha = st->beta = st->pq = 0.0;
    st->breakdown = 0;
  }
}

// Zeroes every field of a freshly allocated state record.
__global__ void k_state_zero(CgState* st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->rr = st->rr0 = st->pq = st->alpha = st->beta = st->nrm2 = st->rz = 0.0;
    st->breakdown = 0;
    st->pad = 0;
  }
}

unsigned grid_for(int64_t n) {
  const int64_t g = (n + RT - 1) / RT;
  return (unsigned)(g < RED_BLOCKS ? (g > 0 ? g : 1) : RED_BLOCKS);
}
}  // namespace

hipError_t blas_dot(const void* a, const void* b, int prec, int64_t n, double* partial, CgState* st, int op,
                    hipStream_t s) {
  const unsigned g = grid_for(n);
  if (prec == DG_F64)
    hipLaunchKernelGGL(k_dot<double>, dim3(g), dim3(RT), 0, s, (const double*)a, (const double*)b, n, partial);
  else
    hipLaunchKernelGGL(k_dot<float>, dim3(g), dim3(RT), 0, s, (const float*)a, (const float*)b, n, partial);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(RT), 0, s, partial, (int)g, st, op);
  return hipGetLastError();
}

hipError_t blas_finalize(const double* partial, int64_t nb, CgState* st, int op, hipStream_t s) {
  if (nb < 1 || nb > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(RT), 0, s, partial, (int)nb, st, op);
  return hipGetLastError();
}

hipError_t blas_r_update(void* r, const void* q, int prec, int64_t n, double* partial, CgState* st, int op,
                         hipStream_t s) {
  const unsigned g = grid_for(n);
  if (prec == DG_F64)
    hipLaunchKernelGGL(k_r_update<double>, dim3(g), dim3(RT), 0, s, (double*)r, (const double*)q, st, n, partial);
  else
    hipLaunchKernelGGL(k_r_update<float>, dim3(g), dim3(RT), 0, s, (float*)r, (const float*)q, st, n, partial);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(RT), 0, s, partial, (int)g, st, op);
  return hipGetLastError();
}

hipError_t blas_xp_update(void* x, void* p, const void* z, int prec, int64_t n, CgState* st, hipStream_t s) {
  const unsigned g = grid_for(n);
  if (prec == DG_F64)
    hipLaunchKernelGGL(k_xp_update<double>, dim3(g), dim3(RT), 0, s, (double*)x, (double*)p, (const double*)z, st,
                       n);
  else
    hipLaunchKernelGGL(k_xp_update<float>, dim3(g), dim3(RT), 0, s, (float*)x, (float*)p, (const float*)z, st, n);
  return hipGetLastError();
}

hipError_t blas_residual(const double* b, const double* Ax, double* r, int64_t n, double* partial, CgState* st,
                         hipStream_t s) {
  const unsigned g = grid_for(n);
  hipLaunchKernelGGL(k_residual, dim3(g), dim3(RT), 0, s, b, Ax, r, n, partial);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(RT), 0, s, partial, (int)g, st, (int)OP_NORM);
  return hipGetLastError();
}

hipError_t blas_ir_start(const double* r, float* rh, float* ph, float* d, int64_t n, CgState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_ir_start, dim3(grid_for(n)), dim3(RT), 0, s, r, st, rh, ph, d, n);
  hipLaunchKernelGGL(k_state_reset, dim3(1), dim3(1), 0, s, st, 0);
  return hipGetLastError();
}

hipError_t blas_ir_correct(double* x, const float* d, int64_t n, CgState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_ir_correct, dim3(grid_for(n)), dim3(RT), 0, s, x, d, st, n);
  return hipGetLastError();
}

hipError_t blas_accumulate(double* x, float* xl, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_accumulate, dim3(grid_for(n)), dim3(RT), 0, s, x, xl, n);
  return hipGetLastError();
}

hipError_t blas_zero(void* a, int prec, int64_t n, hipStream_t s) {
  if (prec == DG_F64)
    hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(n)), dim3(RT), 0, s, (double*)a, 0.0, n);
  else
    hipLaunchKernelGGL(k_fill<float>, dim3(grid_for(n)), dim3(RT), 0, s, (float*)a, 0.0f, n);
  return hipGetLastError();
}

hipError_t blas_copy(const void* a, void* b, int prec, int64_t n, hipStream_t s) {
  if (prec == DG_F64)
    hipLaunchKernelGGL(k_copy<double>, dim3(grid_for(n)), dim3(RT), 0, s, (const double*)a, (double*)b, n);
  else
    hipLaunchKernelGGL(k_copy<float>, dim3(grid_for(n)), dim3(RT), 0, s, (const float*)a, (float*)b, n);
  return hipGetLastError();
}

hipError_t blas_round_f32(const double* a, float* b, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_round_f32, dim3(grid_for(n)), dim3(RT), 0, s, a, b, n);
  return hipGetLastError();
}

hipError_t blas_state_zero(CgState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_state_zero, dim3(1), dim3(1), 0, s, st);
  return hipGetLastError();
}

hipError_t blas_state_from_norm(CgState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_state_reset, dim3(1), dim3(1), 0, s, st, 1);
  return hipGetLastError();
}

}  // namespace dgi
