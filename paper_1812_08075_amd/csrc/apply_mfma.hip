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
// (built on the host in long double, one K per pair of side types).
//
// Design.
//  * One wavefront per cell and direction step: the cell's 64 values sit one
//    per lane in a "line layout" lane = line + 16 node (the 16 lines along d,
//    node index along d). v_mfma_f64_4x4x4f64 (four 4x4 blocks) multiplies
//    a 4x4 matrix held one entry per lane into all 16 lines at once, and its
//    result comes out in the same layout, so the three products of a
//    direction chain through the accumulator. The matrices cost one VGPR
//    pair each.
//  * Each wavefront owns NC consecutive cells of an x-row and issues all of
//    its global reads first: its cells once in natural node order (the z
//    layout), the x-lines of the cells beyond both ends, and the y- and
//    z-neighbour cells read directly in the layout they are used in (the
//    y-layout read is a permutation inside each 512-byte cell). The x and y
//    layouts of its own cells are formed with ds_bpermute (no LDS memory),
//    and the x-neighbours of the inner cells are these same values. The
//    wavefronts are independent: no barriers, no LDS allocation.
//  * Per lane, the A-operand entries of the nine interior-cell operators and
//    the line weight form one 80-byte record (five 16-byte reads); boundary
//    cells read their own K variant.
//  * The results of the x and y directions are brought to the natural node
//    order with ds_bpermute and summed with the z result; one coalesced
//    store per cell.
//  * Wavefronts walk the sweep order (slab of z-planes, y, z, x-chunk) with
//    an XCD-aware renumbering (table built on the host), so that the y- and
//    z-neighbour lines are served by the XCD's L2.
#include <algorithm>
#include <vector>

#include "internal.h"

namespace dgi {
namespace {

constexpr int NC = 4;            // cells per wavefront (consecutive along x)
constexpr int T_INT = 0, T_DIR = 1, T_NONE = 2;

__device__ __forceinline__ double mfma(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

// value of lane `src` (all lanes take part)
__device__ __forceinline__ double lane_read(double v, int src) {
  const int2 w = __builtin_bit_cast(int2, v);
  int2 r;
  r.x = __builtin_amdgcn_ds_bpermute(src << 2, w.x);
  r.y = __builtin_amdgcn_ds_bpermute(src << 2, w.y);
  return __builtin_bit_cast(double, r);
}

__device__ __forceinline__ int side_type(bool has, bool dirichlet) {
  return has ? T_INT : (dirichlet ? T_DIR : T_NONE);
}

// One wavefront per block; the wavefronts are independent.
__global__ void __launch_bounds__(64)
    k_apply_q3_mfma(const double* __restrict__ x, double* __restrict__ y, const ScalarArgs<double>* __restrict__ ap,
                    const uint32_t* __restrict__ waves) {
  const ScalarArgs<double>& a = *ap;
  const int lane = threadIdx.x;
  const uint32_t w0 = waves[2 * blockIdx.x], w1 = waves[2 * blockIdx.x + 1];
  const int ex0 = (int)(w0 & 0xffffu), ey = (int)(w0 >> 16), ez = (int)w1;
  const int nx = a.n[0], ny = a.n[1], nz = a.n[2];
  const int nvalid = min(NC, nx - ex0);
  if (nvalid <= 0) return;

  const uint32_t row = (uint32_t)nx * ((uint32_t)ey + (uint32_t)ny * ez);
  const uint32_t nxy = (uint32_t)nx * ny;
  const uint32_t c0 = row + ex0;
  const bool hy0 = ey > 0, hy1 = ey < ny - 1, hz0 = ez > 0, hz1 = ez < nz - 1;
  const bool hxl = ex0 > 0, hxr = ex0 + nvalid < nx;

  double2 rec[5];
  const double2* lr = reinterpret_cast<const double2*>(a.lrec[lane]);
#pragma unroll
  for (int k = 0; k < 5; ++k) rec[k] = lr[k];
  // line layouts: lane = l + 16 q, node q along the direction, line l = t1 + 4 t2
  const int q = lane >> 4, l = lane & 15, t1 = l & 3, t2 = l >> 2;
  const int nxl = q + 4 * t1 + 16 * t2;  // natural index of the x-layout lane
  const int nyl = t1 + 4 * q + 16 * t2;  // y-layout (the z-layout is the natural order)
  const int i0 = lane & 3, i1 = (lane >> 2) & 3, i2 = lane >> 4;
  const int srcx = i1 + 4 * i2 + 16 * i0, srcy = i0 + 4 * i2 + 16 * i1;  // lanes holding node `lane`
  const size_t b0 = (size_t)c0 * 64;
  // global reads: own cells (natural order), x-ends (x layout), y-neighbours (y layout), z-neighbours
  double uz[NC], xl, xr, uyl[NC], uyr[NC], uzl[NC], uzr[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) uz[k] = k < nvalid ? x[b0 + 64 * k + lane] : 0.0;
  xl = hxl ? x[b0 - 64 + nxl] : 0.0;
  xr = hxr ? x[b0 + 64 * nvalid + nxl] : 0.0;
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    uyl[k] = (k < nvalid && hy0) ? x[b0 - (size_t)nx * 64 + 64 * k + nyl] : 0.0;
    uyr[k] = (k < nvalid && hy1) ? x[b0 + (size_t)nx * 64 + 64 * k + nyl] : 0.0;
    uzl[k] = (k < nvalid && hz0) ? x[b0 - (size_t)nxy * 64 + 64 * k + lane] : 0.0;
    uzr[k] = (k < nvalid && hz1) ? x[b0 + (size_t)nxy * 64 + 64 * k + lane] : 0.0;
  }
  const int ai = 4 * (lane & 3) + (lane >> 4);  // A operand: entry (lane % 4, lane / 16)
  const uint32_t mask = a.mask;
  const int vy = 3 * side_type(hy0, mask & 4u) + side_type(hy1, mask & 8u);
  const int vz = 3 * side_type(hz0, mask & 16u) + side_type(hz1, mask & 32u);
  double Kx_int = rec[0].x, Lx = rec[0].y, Rx = rec[1].x, Ky = rec[1].y, Ly = rec[2].x, Ry = rec[2].y;
  double Kz = rec[3].x, Lz = rec[3].y, Rz = rec[4].x;
  const double wt = rec[4].y;
  if (vy != 0) Ky = a.Km[1][vy][ai];
  if (vz != 0) Kz = a.Km[2][vz][ai];
  // own cells in the x layout (the x-neighbours of the inner cells)
  double ux[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) ux[k] = lane_read(uz[k], nxl);
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
      double cy = mfma(Ky, lane_read(uz[k], nyl), 0.0);
      if (hy0) cy = mfma(Ly, uyl[k], cy);
      if (hy1) cy = mfma(Ry, uyr[k], cy);
      double cz = mfma(Kz, uz[k], 0.0);
      if (hz0) cz = mfma(Lz, uzl[k], cz);
      if (hz1) cz = mfma(Rz, uzr[k], cz);
      y[b0 + 64 * k + lane] = lane_read(wt * cx, srcx) + lane_read(wt * cy, srcy) + wt * cz;
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
