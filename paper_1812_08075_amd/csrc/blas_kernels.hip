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

// Sums the partials (fixed order) and applies `op` to the CG state. FT
// threads: thread i adds partial[i], partial[i + FT], ... in order, four
// independent loads at a time, then a tree over the block.
constexpr int FT = 1024;
__global__ void __launch_bounds__(FT) k_finalize(const double* __restrict__ partial, int nb,
                                                 CgState* __restrict__ st, int op) {
  __shared__ double sh[FT];
  double acc = 0.0;
  int i = threadIdx.x;
  for (; i + 3 * FT < nb; i += 4 * FT) {
    const double a0 = partial[i], a1 = partial[i + FT], a2 = partial[i + 2 * FT], a3 = partial[i + 3 * FT];
    acc += a0;
    acc += a1;
    acc += a2;
    acc += a3;
  }
  for (; i < nb; i += FT) acc += partial[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
#pragma unroll
  for (int s = FT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double s = sh[0];
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

// r -= alpha q (FP64) with partial sums of r.r, and r32 = r rounded to FP32
// (the right-hand side of the FP32 Chebyshev inner solve)
__global__ void __launch_bounds__(RT) k_r_update_round(double* __restrict__ r, const double* __restrict__ q,
                                                       float* __restrict__ r32, const CgState* __restrict__ st,
                                                       int64_t n, double* __restrict__ partial) {
  __shared__ double sh[RT];
  const double a = st->alpha;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x; i < n; i += (int64_t)gridDim.x * RT) {
    const double ri = fma(-a, q[i], r[i]);
    r[i] = ri;
    r32[i] = (float)ri;
    acc = fma(ri, ri, acc);
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// x += alpha p; p = z + beta p with the preconditioned residual z in FP32
__global__ void __launch_bounds__(RT) k_xp_update_mixed(double* __restrict__ x, double* __restrict__ p,
                                                        const float* __restrict__ z,
                                                        const CgState* __restrict__ st, int64_t n) {
  const double a = st->alpha, b = st->beta;
  for (int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x; i < n; i += (int64_t)gridDim.x * RT) {
    const double pi = p[i];
    x[i] = fma(a, pi, x[i]);
    p[i] = fma(b, pi, (double)z[i]);
  }
}

// One step of the Chebyshev iteration for A z = r without a preconditioner:
// w = r - t (t = A z; absent on the first step, where z = 0), d = c1 d + c2 w
// (d absent on the first step), z += d. The right-hand side is read from rd
// (FP64, rounded to T) when given, else from r; with rd the last step also
// writes the partial sums of rd.z (FP64) and skips the store of d.
template <typename T>
__global__ void __launch_bounds__(RT) k_cheb_plain(const T* __restrict__ r, const double* __restrict__ rd,
                                                   const T* __restrict__ t, T* __restrict__ d,
                                                   T* __restrict__ z, T c1, T c2, int first, int last,
                                                   int64_t n, double* __restrict__ partial) {
  __shared__ double sh[RT];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x; i < n; i += (int64_t)gridDim.x * RT) {
    const T ri = rd ? (T)rd[i] : r[i];
    const T wi = first ? ri : ri - t[i];
    const T di = first ? c2 * wi : fma(c1, d[i], c2 * wi);
    const T zi = first ? di : z[i] + di;
    if (!last) d[i] = di;
    z[i] = zi;
    if (last && rd) acc = fma(rd[i], (double)zi, acc);
  }
  if (last && rd) {
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
  }
}

// Records the step length and direction update of the CG iteration just done
// (the Lanczos coefficients of the spectral estimate).
__global__ void k_record(const CgState* __restrict__ st, double* __restrict__ hist, int j) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    hist[2 * j] = st->alpha;
    hist[2 * j + 1] = st->beta;
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

__global__ void __launch_bounds__(RT) k_widen(const float* __restrict__ a, double* __restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x; i < n; i += (int64_t)gridDim.x * RT) b[i] = (double)a[i];
}

__global__ void __launch_bounds__(RT) k_round_f32(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x; i < n; i += (int64_t)gridDim.x * RT) b[i] = (float)a[i];
}

// a[i] = a pseudo-random value in [-1, 1) from the counter i and the seed:
// the SplitMix64 output function (Steele, Lea and Flood, 2014) of
// seed + (i + 1) times the golden-ratio increment, top 53 bits.
template <typename T>
__global__ void __launch_bounds__(RT) k_random(T* __restrict__ a, int64_t n, uint64_t seed) {
  for (int64_t i = (int64_t)blockIdx.x * RT + threadIdx.x; i < n; i += (int64_t)gridDim.x * RT) {
    uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    a[i] = (T)(2.0 * ((double)(z >> 11) * 0x1.0p-53) - 1.0);
  }
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
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(FT), 0, s, partial, (int)g, st, op);
  return hipGetLastError();
}

hipError_t blas_finalize(const double* partial, int64_t nb, CgState* st, int op, hipStream_t s) {
  if (nb < 1 || nb > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(FT), 0, s, partial, (int)nb, st, op);
  return hipGetLastError();
}

hipError_t blas_r_update(void* r, const void* q, int prec, int64_t n, double* partial, CgState* st, int op,
                         hipStream_t s) {
  const unsigned g = grid_for(n);
  if (prec == DG_F64)
    hipLaunchKernelGGL(k_r_update<double>, dim3(g), dim3(RT), 0, s, (double*)r, (const double*)q, st, n, partial);
  else
    hipLaunchKernelGGL(k_r_update<float>, dim3(g), dim3(RT), 0, s, (float*)r, (const float*)q, st, n, partial);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(FT), 0, s, partial, (int)g, st, op);
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

hipError_t blas_r_update_round(double* r, const double* q, float* r32, int64_t n, double* partial, CgState* st,
                               int op, hipStream_t s) {
  const unsigned g = grid_for(n);
  hipLaunchKernelGGL(k_r_update_round, dim3(g), dim3(RT), 0, s, r, q, r32, st, n, partial);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(FT), 0, s, partial, (int)g, st, op);
  return hipGetLastError();
}

hipError_t blas_xp_update_mixed(double* x, double* p, const float* z, int64_t n, CgState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_xp_update_mixed, dim3(grid_for(n)), dim3(RT), 0, s, x, p, z, st, n);
  return hipGetLastError();
}

int64_t blas_cheb_blocks(int64_t n) { return grid_for(n); }

hipError_t blas_cheb_step(int prec, const void* r, const double* rd, const void* t, void* d, void* z, double c1,
                          double c2, bool first, bool last, int64_t n, double* partial, hipStream_t s) {
  const unsigned g = grid_for(n);
  if (prec == DG_F64)
    hipLaunchKernelGGL(k_cheb_plain<double>, dim3(g), dim3(RT), 0, s, (const double*)r, rd, (const double*)t,
                       (double*)d, (double*)z, c1, c2, (int)first, (int)last, n, partial);
  else
    hipLaunchKernelGGL(k_cheb_plain<float>, dim3(g), dim3(RT), 0, s, (const float*)r, rd, (const float*)t,
                       (float*)d, (float*)z, (float)c1, (float)c2, (int)first, (int)last, n, partial);
  return hipGetLastError();
}

hipError_t blas_record(const CgState* st, double* hist, int j, hipStream_t s) {
  hipLaunchKernelGGL(k_record, dim3(1), dim3(1), 0, s, st, hist, j);
  return hipGetLastError();
}

hipError_t blas_residual(const double* b, const double* Ax, double* r, int64_t n, double* partial, CgState* st,
                         hipStream_t s) {
  const unsigned g = grid_for(n);
  hipLaunchKernelGGL(k_residual, dim3(g), dim3(RT), 0, s, b, Ax, r, n, partial);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(FT), 0, s, partial, (int)g, st, (int)OP_NORM);
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

hipError_t blas_widen(const float* a, double* b, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_widen, dim3(grid_for(n)), dim3(RT), 0, s, a, b, n);
  return hipGetLastError();
}

hipError_t blas_random(void* a, int prec, int64_t n, uint64_t seed, hipStream_t s) {
  if (prec == DG_F64)
    hipLaunchKernelGGL(k_random<double>, dim3(grid_for(n)), dim3(RT), 0, s, (double*)a, n, seed);
  else
    hipLaunchKernelGGL(k_random<float>, dim3(grid_for(n)), dim3(RT), 0, s, (float*)a, n, seed);
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
