// Matrix-core apply of the SIPG diffusion-reaction operator for k = 3 (p = 4
// nodes per direction), kappa = 1, axis-aligned cells, on FP32 vectors
// (gfx950).
//
// Operator (Section 5.2, eq. diffreac_weak, linear part) as in the FP64
// matrix-core kernel: per direction the 1D line operator
//     out = K u + L u_left + R u_right
// of the line and of the matching lines of the two face neighbours, with row
// i of each operator divided by w_i on the host and the sum over the three
// directions multiplied by the node's tensor weight. The vectors are FP32;
// the arithmetic is FP64 on the same operator tables and in the same order
// as the FP64 kernel, so the result is the FP64 kernel's result for the
// FP32 input, rounded once to FP32.
//
// Design.
//  * A 16-byte load carries four FP32 values: a whole x-line of a cell. A
//    "quad layout" holds in one lane the four nodes i0 = 0..3 of one x-line:
//    lane = i1 + 4 c + 16 i2 for the z direction ("z-quad"), lane = i2 + 4 c
//    + 16 i1 for the y direction ("y-quad"), c the cell of the chunk of 4.
//    Converted to FP64, each of the four components is an operand of
//    v_mfma_f64_4x4x4f64, which contracts over lane bits 4-5 and keeps bits
//    0-3 as 16 independent lines: the lines of all four cells go through one
//    product.
//  * The x direction needs i0 in lane bits 4-5 ("x layout": lane = i1 + 4 i2
//    + 16 i0, one cell per register): the own cells are staged in LDS (FP64,
//    padded i1, i2 and cell strides 4, 18, 70) and read back in the x, y and
//    z layouts; the x-lines beyond both ends of the chunk are read from
//    global memory.
//  * A wavefront owns a chunk of 4 x-consecutive cells and marches along y
//    over the rows of its table entry (the table of the FP64 kernel). Two
//    LDS buffers hold rows y and y + 1: per step the wavefront reads from
//    global memory the row y + 1 and the two z-neighbour rows (one 16-byte
//    load each) and the two x-end lines, and takes the y-neighbour lines
//    from LDS, row y - 1 read before it is replaced.
//  * Results: x results to LDS, y results added in the y-quad layout, z
//    results added on reading them back in the z-quad layout, times the
//    tensor weight, rounded to FP32 and stored with one 16-byte
//    non-temporal store per lane.
#include "internal.h"

namespace dgi {
namespace {

constexpr int NC = 4;  // cells per step (consecutive along x)
// LDS node (i0, i1, i2) of cell c at c LCS + i2 LPS + i1 LIS + i0 (doubles)
constexpr int LIS = 4, LPS = 18, LCS = 70;
constexpr int T_INT = 0, T_DIR = 1, T_NONE = 2;

__device__ __forceinline__ double mfma(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int side_type(bool has, bool dirichlet) {
  return has ? T_INT : (dirichlet ? T_DIR : T_NONE);
}

typedef float fvec4 __attribute__((ext_vector_type(4)));
typedef double dvec2 __attribute__((ext_vector_type(2)));

struct Quad {
  double v[4];
};

// 16-byte load of one x-line (zeros when !ok), widened to FP64
__device__ __forceinline__ Quad load_quad(const float* p, bool ok) {
  fvec4 r = {0.0f, 0.0f, 0.0f, 0.0f};
  if (ok) r = *reinterpret_cast<const fvec4*>(p);
  Quad q;
  q.v[0] = (double)r.x;
  q.v[1] = (double)r.y;
  q.v[2] = (double)r.z;
  q.v[3] = (double)r.w;
  return q;
}

__device__ __forceinline__ Quad lds_quad(const double* p) {
  const dvec2 a = *reinterpret_cast<const dvec2*>(p);
  const dvec2 b = *reinterpret_cast<const dvec2*>(p + 2);
  Quad q;
  q.v[0] = a.x;
  q.v[1] = a.y;
  q.v[2] = b.x;
  q.v[3] = b.y;
  return q;
}

__device__ __forceinline__ void lds_store_quad(double* p, const Quad& q) {
  const dvec2 a = {q.v[0], q.v[1]};
  const dvec2 b = {q.v[2], q.v[3]};
  *reinterpret_cast<dvec2*>(p) = a;
  *reinterpret_cast<dvec2*>(p + 2) = b;
}

// one direction on a quad register: K u + L u_left + R u_right per component
__device__ __forceinline__ Quad quad_line(double K, double L, double R, const Quad& u, const Quad& ul,
                                          const Quad& ur, bool h0, bool h1) {
  Quad c;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    c.v[q] = mfma(K, u.v[q], 0.0);
    if (h0) c.v[q] = mfma(L, ul.v[q], c.v[q]);
    if (h1) c.v[q] = mfma(R, ur.v[q], c.v[q]);
  }
  return c;
}

// One wavefront per block; the wavefronts are independent. A wavefront
// handles NC cells along x in each of its rows along y, one row per step.
// DOT: each wavefront also writes the sum of x_i y_i over its cells (FP64,
// fixed order, of the FP32 values) to partial[block].
template <bool DOT>
__device__ __forceinline__ void apply_q3_wave_f32(const float* __restrict__ x, float* __restrict__ y,
                                                  const ScalarArgs<double>* __restrict__ ap,
                                                  const uint32_t* __restrict__ waves,
                                                  double* __restrict__ partial) {
  __shared__ __attribute__((aligned(16))) double su[2 * NC * LCS];  // own cells of rows y and y + 1
  __shared__ __attribute__((aligned(16))) double sr[NC * LCS];      // x results, then x + y results
  const ScalarArgs<double>& a = *ap;
  const int lane = threadIdx.x;
  const uint32_t w0 = waves[2 * blockIdx.x], w1 = waves[2 * blockIdx.x + 1];
  const int ex0 = (int)(w0 & 0xffffu), ey0 = (int)(w0 >> 16), ez = (int)(w1 & 0xffffu);
  const int nx = a.n[0], ny = a.n[1], nz = a.n[2];
  if (ex0 >= nx || ey0 >= ny) {
    if (DOT && lane == 0) partial[blockIdx.x] = 0.0;
    return;
  }
  double pq = 0.0;
  const int nvalid = min(NC, nx - ex0);
  const int nsteps = min((int)(w1 >> 16), ny - ey0);
  const bool hxl = ex0 > 0, hxr = ex0 + nvalid < nx;
  const size_t row0 = (size_t)nx * ((size_t)ey0 + (size_t)ny * ez);
  const size_t sy = (size_t)nx * 64, sz = (size_t)nx * ny * 64;  // neighbour strides in values
  const bool hz0 = ez > 0, hz1 = ez < nz - 1;

  // quad layouts: the lane's cell and x-line (i1, i2)
  const int c = (lane >> 2) & 3;
  const bool cval = c < nvalid;
  const int zi1 = lane & 3, zi2 = lane >> 4;  // z-quad
  const int yi2 = lane & 3, yi1 = lane >> 4;  // y-quad
  const int offz = 64 * c + 4 * zi1 + 16 * zi2;
  const int lz = LCS * c + LIS * zi1 + LPS * zi2;
  const int ly = LCS * c + LIS * yi1 + LPS * yi2;
  // x layout: lane = i1 + 4 i2 + 16 i0
  const int offx = (lane >> 4) + 4 * (lane & 3) + 16 * ((lane >> 2) & 3);
  const int lx = (lane >> 4) + LIS * (lane & 3) + LPS * ((lane >> 2) & 3);

  // A-operand entries of the interior operators (entry (lane % 4, lane / 16));
  // the tensor weights of the lane's four nodes come from the records of the
  // lanes that hold them in the FP64 kernel's pair layout
  const int ai = 4 * (lane & 3) + (lane >> 4);
  const double* rl = a.lrec[lane];
  const double Kx_int = rl[0], Lx = rl[1], Rx = rl[2];
  const double Ky_int = rl[3], Ly = rl[4], Ry = rl[5];
  double Kz = rl[6];
  const double Lz = rl[7], Rz = rl[8];
  double wq[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) wq[q] = a.lrec[(q >> 1) + 2 * zi1 + 16 * zi2][10 + (q & 1)];
  const uint32_t mask = a.mask;
  const int vz = 3 * side_type(hz0, mask & 16u) + side_type(hz1, mask & 32u);
  if (vz != 0) Kz = a.Km[2][vz][ai];

  // own row ey0 to buffer 0, row ey0 - 1 to buffer 1 (invalid or absent
  // cells as zeros)
  {
    const float* __restrict__ xc = x + (row0 + ex0) * 64;
    lds_store_quad(su + lz, load_quad(xc + offz, cval));
    lds_store_quad(su + NC * LCS + lz, load_quad(xc - sy + offz, cval && ey0 > 0));
  }

  for (int s = 0; s < nsteps; ++s) {
    const int ey = ey0 + s;
    const bool hy0 = ey > 0, hy1 = ey < ny - 1;
    const size_t row = row0 + (size_t)s * nx;
    const float* __restrict__ xc = x + (row + ex0) * 64;
    double* cur = su + (s & 1) * (NC * LCS);        // row y
    double* oth = su + ((s + 1) & 1) * (NC * LCS);  // row y - 1, then row y + 1

    const Quad nr = load_quad(xc + sy + offz, cval && hy1);
    const Quad zl = load_quad(xc - sz + offz, cval && hz0);
    const Quad zr = load_quad(xc + sz + offz, cval && hz1);
    const double xl = hxl ? (double)xc[offx - 64] : 0.0;
    const double xr = hxr ? (double)xc[64 * nvalid + offx] : 0.0;

    // row ey - 1 in the y layout, before the next row replaces it
    const Quad yl = lds_quad(oth + ly);
    __syncthreads();
    lds_store_quad(oth + lz, nr);
    __syncthreads();
    double ux[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) ux[k] = cur[LCS * k + lx];

#pragma unroll
    for (int k = 0; k < NC; ++k) {
      if (k < nvalid) {
        const int ex = ex0 + k;
        const bool hx0 = ex > 0, hx1 = ex < nx - 1;
        const double ul = k == 0 ? xl : ux[k > 0 ? k - 1 : 0];
        const double ur = k == nvalid - 1 ? xr : ux[k + 1 < NC ? k + 1 : k];
        double Kx = Kx_int;
        if (!(hx0 && hx1)) Kx = a.Km[0][3 * side_type(hx0, mask & 1u) + side_type(hx1, mask & 2u)][ai];
        double cx = mfma(Kx, ux[k], 0.0);
        if (hx0) cx = mfma(Lx, ul, cx);
        if (hx1) cx = mfma(Rx, ur, cx);
        sr[LCS * k + lx] = cx;
      }
    }
    __syncthreads();
    // y direction, added onto the x results
    {
      const int vy = 3 * side_type(hy0, mask & 4u) + side_type(hy1, mask & 8u);
      const double Ky = vy != 0 ? a.Km[1][vy][ai] : Ky_int;
      const Quad cy = quad_line(Ky, Ly, Ry, lds_quad(cur + ly), yl, lds_quad(oth + ly), hy0, hy1);
      Quad o = lds_quad(sr + ly);
#pragma unroll
      for (int q = 0; q < 4; ++q) o.v[q] = o.v[q] + cy.v[q];
      lds_store_quad(sr + ly, o);
    }
    __syncthreads();
    // z direction, the sum, the tensor weight, the store
    {
      const Quad uz = lds_quad(cur + lz);
      const Quad cz = quad_line(Kz, Lz, Rz, uz, zl, zr, hz0, hz1);
      const Quad o = lds_quad(sr + lz);
      fvec4 v;
      v.x = (float)(wq[0] * (o.v[0] + cz.v[0]));
      v.y = (float)(wq[1] * (o.v[1] + cz.v[1]));
      v.z = (float)(wq[2] * (o.v[2] + cz.v[2]));
      v.w = (float)(wq[3] * (o.v[3] + cz.v[3]));
      if (cval) {
        __builtin_nontemporal_store(v, reinterpret_cast<fvec4*>(y + (row + ex0) * 64 + offz));
        if (DOT) {
          pq = fma(uz.v[0], (double)v.x, pq);
          pq = fma(uz.v[1], (double)v.y, pq);
          pq = fma(uz.v[2], (double)v.z, pq);
          pq = fma(uz.v[3], (double)v.w, pq);
        }
      }
    }
  }
  if (DOT) {  // butterfly over the 64 lanes, then lane 0 writes
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) pq += __shfl_xor(pq, m, 64);
    if (lane == 0) partial[blockIdx.x] = pq;
  }
}

__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(5)))
    k_apply_q3_mfma_f32(const float* __restrict__ x, float* __restrict__ y,
                        const ScalarArgs<double>* __restrict__ ap, const uint32_t* __restrict__ waves) {
  apply_q3_wave_f32<false>(x, y, ap, waves, nullptr);
}

__global__ void __launch_bounds__(64)
    k_apply_q3_mfma_f32_dot(const float* __restrict__ x, float* __restrict__ y,
                            const ScalarArgs<double>* __restrict__ ap, const uint32_t* __restrict__ waves,
                            double* __restrict__ partial) {
  apply_q3_wave_f32<true>(x, y, ap, waves, partial);
}

}  // namespace

bool mfma_apply_f32_supported(const dg_mesh& M, int prec, bool kappa) {
  return M.p == 4 && prec == DG_F32 && !kappa && M.d_waves[DG_F32] != nullptr && !M.lines_forced[DG_F32];
}

hipError_t mfma_apply_f32(const dg_mesh& M, int variant, const float* x, float* y, double* partial,
                          hipStream_t s) {
  if (M.ndofs > 0xffffffffLL) return hipErrorInvalidValue;
  const int64_t G = M.nwaves[DG_F32];
  if (G < 1) return hipSuccess;
  if (partial)
    hipLaunchKernelGGL(k_apply_q3_mfma_f32_dot, dim3((unsigned)G), dim3(64), 0, s, x, y, M.d_pd + variant,
                       (const uint32_t*)M.d_waves[DG_F32], partial);
  else
    hipLaunchKernelGGL(k_apply_q3_mfma_f32, dim3((unsigned)G), dim3(64), 0, s, x, y, M.d_pd + variant,
                       (const uint32_t*)M.d_waves[DG_F32]);
  return hipGetLastError();
}

}  // namespace dgi
