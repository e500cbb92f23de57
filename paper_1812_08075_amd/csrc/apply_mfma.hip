// Matrix-core apply of the SIPG diffusion-reaction operator for k = 3 (p = 4
// nodes per direction), FP64, kappa = 1, axis-aligned cells (gfx950).
//
// Operator (Section 5.2, eq. diffreac_weak, linear part) evaluated with the
// sum-factorized structure of Algorithm 1 and the face treatment of Section
// 2.2 (m_d = 1 along the face normal). With the collocated Gauss-Legendre
// basis on a cell J = diag(h), the contribution of direction d to a line of
// p nodes along d is a fixed 1D operator of the line and of the matching
// lines of the two neighbours across the faces normal to d:
//     out = K u + L u_left + R u_right,
// times the line's tangential quadrature weight w_a w_b. K holds the volume
// term D^T diag(|J|/h_d^2 w) D (for d = 0 also the mass term c |J| diag(w))
// and the own-cell face terms, L and R the terms coupling to the neighbour
// (built on the host in long double, one K per pair of side types). The
// tangential weight times w_i is the node's tensor weight, so the host
// divides row i of each operator by w_i and the kernel multiplies the sum
// over the three directions by the tensor weight once per node.
//
// Design.
//  * The L2-to-register path issues one load instruction per 64 lanes at a
//    fixed cost, whatever the width, so cells are read two at a time with
//    16-byte loads. A "pair layout" holds two x-consecutive cells in one
//    double2 register: lane = h + 2 t + 8 c + 16 n, components the nodes
//    i0 = 2h and 2h + 1 of cell c; (t, n) = (i1, i2) for the z direction,
//    (i2, i1) for the y direction. v_mfma_f64_4x4x4f64 (four 4x4 blocks)
//    contracts over lane bits 4-5 and keeps bits 0-3 as 16 independent
//    lines, so each component of a pair register is a valid operand: the
//    lines of both cells go through one product.
//  * The x direction needs i0 in lane bits 4-5, one cell per register
//    ("x layout": lane = i1 + 4 i2 + 16 i0). The own cells are staged in LDS
//    in natural order and read back in the x and y layouts; the x-lines of
//    the cells beyond both ends of the chunk are read from global memory.
//  * Each wavefront owns NC = 4 x-consecutive cells and issues all of its
//    global reads first: the own cells and the z- and y-neighbour cells in
//    pairs, the two x-end lines, and its operator record. The A-operand
//    entries of the nine interior-cell operators and the two nodes' tensor
//    weights form one 96-byte record per lane; boundary cells read their
//    own K variant. Wavefronts are independent (one per block).
//  * Results: the x results are written to LDS in natural order, the y
//    results added to them in the y-pair layout, and the z results added on
//    reading them back in the z-pair layout; the sum times the tensor
//    weight is stored with 16-byte stores.
//  * Wavefronts walk the sweep order (slab of z-planes, y, z, x-chunk) with
//    an XCD-aware renumbering (table built on the host), so that the y- and
//    z-neighbour cells are served by the XCD's L2.
#include <algorithm>
#include <vector>

#include "internal.h"

namespace dgi {
namespace {

constexpr int NC = 4;            // cells per wavefront (consecutive along x): two pairs
constexpr int T_INT = 0, T_DIR = 1, T_NONE = 2;

__device__ __forceinline__ double mfma(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

// 16-byte load of two doubles (zeros when !v); a native vector type keeps it
// one dwordx4 load
typedef double dvec2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 load2(const double* p, bool v) {
  dvec2 r = {0.0, 0.0};
  if (v) r = *reinterpret_cast<const dvec2*>(p);
  return make_double2(r.x, r.y);
}

__device__ __forceinline__ int side_type(bool has, bool dirichlet) {
  return has ? T_INT : (dirichlet ? T_DIR : T_NONE);
}

// one direction on a pair register: K u + L u_left + R u_right per component
__device__ __forceinline__ double2 pair_line(double K, double L, double R, double2 u, double2 ul, double2 ur,
                                             bool h0, bool h1) {
  double2 c;
  c.x = mfma(K, u.x, 0.0);
  c.y = mfma(K, u.y, 0.0);
  if (h0) {
    c.x = mfma(L, ul.x, c.x);
    c.y = mfma(L, ul.y, c.y);
  }
  if (h1) {
    c.x = mfma(R, ur.x, c.x);
    c.y = mfma(R, ur.y, c.y);
  }
  return c;
}

// One wavefront per block; the wavefronts are independent.
__global__ void __launch_bounds__(64)
    k_apply_q3_mfma(const double* __restrict__ x, double* __restrict__ y, const ScalarArgs<double>* __restrict__ ap,
                    const uint32_t* __restrict__ waves) {
  __shared__ __attribute__((aligned(16))) double su[NC * 64];  // own cells, natural node order
  __shared__ __attribute__((aligned(16))) double sr[NC * 64];  // x results, then x + y results
  const ScalarArgs<double>& a = *ap;
  const int lane = threadIdx.x;
  const uint32_t w0 = waves[2 * blockIdx.x], w1 = waves[2 * blockIdx.x + 1];
  const int ex0 = (int)(w0 & 0xffffu), ey = (int)(w0 >> 16), ez = (int)w1;
  const int nx = a.n[0], ny = a.n[1], nz = a.n[2];
  const int nvalid = min(NC, nx - ex0);
  if (nvalid <= 0) return;

  const size_t c0 = (size_t)nx * ((size_t)ey + (size_t)ny * ez) + ex0;
  const size_t sy = (size_t)nx * 64, sz = (size_t)nx * ny * 64;  // neighbour strides in doubles
  const bool hy0 = ey > 0, hy1 = ey < ny - 1, hz0 = ez > 0, hz1 = ez < nz - 1;
  const bool hxl = ex0 > 0, hxr = ex0 + nvalid < nx;
  const double* __restrict__ xc = x + c0 * 64;

  // pair layouts: lane = h + 2 t + 8 c + 16 n; node offsets of the lane's first node
  const int h = lane & 1, t = (lane >> 1) & 3, pc = (lane >> 3) & 1, n = lane >> 4;
  const int offz = 2 * h + 4 * t + 16 * n + 64 * pc;  // node (2h, t, n) of cell pc
  const int offy = 2 * h + 16 * t + 4 * n + 64 * pc;  // node (2h, n, t) of cell pc
  // x layout: lane = i1 + 4 i2 + 16 i0
  const int offx = (lane >> 4) + 4 * (lane & 3) + 16 * ((lane >> 2) & 3);

  double2 uz[2], zl[2], zr[2], yl[2], yr[2];
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const bool v = 2 * p + pc < nvalid;
    const double* b = xc + 128 * p;
    uz[p] = load2(b + offz, v);
    zl[p] = load2(b - sz + offz, v && hz0);
    zr[p] = load2(b + sz + offz, v && hz1);
    yl[p] = load2(b - sy + offy, v && hy0);
    yr[p] = load2(b + sy + offy, v && hy1);
  }
  const double xl = hxl ? xc[offx - 64] : 0.0;
  const double xr = hxr ? xc[64 * nvalid + offx] : 0.0;
  double2 rec[6];
  const double2* lr = reinterpret_cast<const double2*>(a.lrec[lane]);
#pragma unroll
  for (int k = 0; k < 6; ++k) rec[k] = lr[k];

  const int ai = 4 * (lane & 3) + (lane >> 4);  // A operand: entry (lane % 4, lane / 16)
  const uint32_t mask = a.mask;
  const int vy = 3 * side_type(hy0, mask & 4u) + side_type(hy1, mask & 8u);
  const int vz = 3 * side_type(hz0, mask & 16u) + side_type(hz1, mask & 32u);
  const double Kx_int = rec[0].x, Lx = rec[0].y, Rx = rec[1].x;
  double Ky = rec[1].y;
  const double Ly = rec[2].x, Ry = rec[2].y;
  double Kz = rec[3].x;
  const double Lz = rec[3].y, Rz = rec[4].x;
  const double2 wn = rec[5];
  if (vy != 0) Ky = a.Km[1][vy][ai];
  if (vz != 0) Kz = a.Km[2][vz][ai];

  // own cells to LDS (invalid cells as zeros), back in the x and y layouts
#pragma unroll
  for (int p = 0; p < 2; ++p) *reinterpret_cast<double2*>(su + 128 * p + offz) = uz[p];
  __syncthreads();
  double ux[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) ux[k] = su[64 * k + offx];
  double2 uy[2];
#pragma unroll
  for (int p = 0; p < 2; ++p) uy[p] = *reinterpret_cast<const double2*>(su + 128 * p + offy);

  // x direction, one cell per product
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
      sr[64 * k + offx] = cx;
    }
  }
  __syncthreads();
  // y direction on pairs, added onto the x results
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    if (2 * p < nvalid) {
      const double2 c = pair_line(Ky, Ly, Ry, uy[p], yl[p], yr[p], hy0, hy1);
      double2* r = reinterpret_cast<double2*>(sr + 128 * p + offy);
      const double2 o = *r;
      *r = make_double2(o.x + c.x, o.y + c.y);
    }
  }
  __syncthreads();
  // z direction on pairs, the sum, the tensor weight, the store
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    if (2 * p < nvalid) {
      const double2 c = pair_line(Kz, Lz, Rz, uz[p], zl[p], zr[p], hz0, hz1);
      const double2 o = *reinterpret_cast<const double2*>(sr + 128 * p + offz);
      if (2 * p + pc < nvalid)
        *reinterpret_cast<double2*>(y + c0 * 64 + 128 * p + offz) = make_double2(wn.x * (o.x + c.x), wn.y * (o.y + c.y));
    }
  }
}

// XCD-aware renumbering of hardware blocks (block b runs on XCD b % 8).
int xcd_swizzle_host(int b, int G) {
  const int q = G >> 3, r = G & 7;
  const int xcd = b & 7, idx = b >> 3;
  return xcd * q + std::min(xcd, r) + idx;
}

}  // namespace

bool mfma_apply_supported(const dg_mesh& M, int prec, bool kappa) {
  return M.p == 4 && prec == DG_F64 && !kappa && M.d_waves != nullptr;
}

hipError_t mfma_setup(dg_mesh& M) {
  if (M.p != 4) return hipSuccess;
  const int nx = M.desc.nx, ny = M.desc.ny, nz = M.desc.nz;
  const int nc = (nx + NC - 1) / NC;
  const int64_t W = (int64_t)nc * ny * nz;
  if (W > 0x7fffffff / 2) return hipErrorInvalidValue;
  const int sz = nz >= 8 ? nz / 8 : 1;
  const int per_slab = nc * ny * sz;
  // logical wavefront t = chunk + nc (z in slab + hz y) + per_slab slab;
  // hardware block b (one wavefront) runs logical wavefront swizzle(b)
  const int G = (int)W;
  std::vector<uint32_t> tab(2 * (size_t)G, 0);
  for (int b = 0; b < G; ++b) {
    const int t = xcd_swizzle_host(b, G);
    const int slab = t / per_slab, rem = t - slab * per_slab;
    const int hz = std::min(sz, nz - slab * sz);
    const int ey = rem / (nc * hz), rem2 = rem - ey * nc * hz;
    const int ezi = rem2 / nc, chunk = rem2 - ezi * nc;
    tab[2 * (size_t)b] = (uint32_t)(chunk * NC) | ((uint32_t)ey << 16);
    tab[2 * (size_t)b + 1] = (uint32_t)(slab * sz + ezi);
  }
  hipError_t e = hipMalloc(&M.d_waves, sizeof(uint32_t) * tab.size());
  if (e != hipSuccess) return e;
  M.nwaves = G;
  return hipMemcpy(M.d_waves, tab.data(), sizeof(uint32_t) * tab.size(), hipMemcpyHostToDevice);
}

hipError_t mfma_apply(const dg_mesh& M, int variant, const double* x, double* y, hipStream_t s) {
  if (M.ndofs > 0xffffffffLL) return hipErrorInvalidValue;
  const int64_t G = M.nwaves;
  if (G < 1) return hipSuccess;
  hipLaunchKernelGGL(k_apply_q3_mfma, dim3((unsigned)G), dim3(64), 0, s, x, y, M.d_pd + variant,
                     (const uint32_t*)M.d_waves);
  return hipGetLastError();
}

}  // namespace dgi
