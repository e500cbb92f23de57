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
//    its loads first (own cells in the three line layouts, the x-line of
//    the cells before and after, the y- and z-neighbour lines), so that many
//    bytes are in flight per wavefront; the x-neighbour lines of interior
//    cells are the wavefront's own loads. The wavefronts are independent:
//    no block barriers.
//  * The results of the x and y directions are brought to the natural node
//    order with ds_bpermute and summed with the z result, which is already
//    natural; the cell is written with one coalesced store.
//  * Wavefronts walk the sweep order (slab of z-planes, y, z, x-chunk) with
//    an XCD-aware renumbering (table built on the host), so that the y- and
//    z-neighbour lines are served by the XCD's L2.
#include <algorithm>
#include <vector>

#include "internal.h"

namespace dgi {
namespace {

constexpr int NC = 4;            // cells per wavefront (consecutive along x)
constexpr int NSLOT = 5 * NC + 2;  // LDS cells per wavefront: own, two x-ends, four neighbour groups
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

// orders this wavefront's LDS writes before its later reads by other lanes
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int side_type(bool has, bool dirichlet) {
  return has ? T_INT : (dirichlet ? T_DIR : T_NONE);
}

// Reads `ncell` consecutive cells starting at cell `c` as 16-byte pieces
// (lane i takes pieces i and i + 64): one load instruction per two cells.
__device__ __forceinline__ void load_group(double2* r, const double2* __restrict__ x2, uint32_t c, int ncell,
                                           bool present, int lane) {
#pragma unroll
  for (int k = 0; k < NC / 2; ++k) {
    const int i = lane + 64 * k;
    r[k] = (present && i < 32 * ncell) ? x2[(size_t)c * 32 + i] : double2{0.0, 0.0};
  }
}
__device__ __forceinline__ void store_group(double* s, const double2* r, int lane) {
#pragma unroll
  for (int k = 0; k < NC / 2; ++k) reinterpret_cast<double2*>(s)[lane + 64 * k] = r[k];
}

// One wavefront per block: LDS is released as soon as the wavefront ends.
__global__ void __launch_bounds__(64)
    k_apply_q3_mfma(const double* __restrict__ x, double* __restrict__ y, const ScalarArgs<double>* __restrict__ ap,
                    const uint32_t* __restrict__ waves) {
  __shared__ double sb[NSLOT * 64];
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
  const double2* __restrict__ x2 = reinterpret_cast<const double2*>(x);

  // this lane's operator entries (interior cell) and line weight
  double2 rec[5];
  const double2* lr = reinterpret_cast<const double2*>(a.lrec[lane]);
#pragma unroll
  for (int k = 0; k < 5; ++k) rec[k] = lr[k];
  // all global reads first: own cells, the x-neighbours beyond both ends,
  // the y- and z-neighbour groups (each a run of consecutive cells)
  double2 rown[NC / 2], ryl[NC / 2], ryr[NC / 2], rzl[NC / 2], rzr[NC / 2], rend;
  load_group(rown, x2, c0, nvalid, true, lane);
  {
    const bool right = lane >= 32;
    const bool ok = right ? hxr : hxl;
    const uint32_t ce = right ? c0 + nvalid : c0 - 1;
    rend = ok ? x2[(size_t)ce * 32 + (lane & 31)] : double2{0.0, 0.0};
  }
  load_group(ryl, x2, c0 - nx, nvalid, hy0, lane);
  load_group(ryr, x2, c0 + nx, nvalid, hy1, lane);
  load_group(rzl, x2, c0 - nxy, nvalid, hz0, lane);
  load_group(rzr, x2, c0 + nxy, nvalid, hz1, lane);

  // LDS slots: 0..NC-1 own, NC left end, NC+1 right end, then y-left, y-right,
  // z-left, z-right groups of NC cells; natural node order inside a slot
  constexpr int S_END = NC, S_YL = NC + 2, S_YR = 2 * NC + 2, S_ZL = 3 * NC + 2, S_ZR = 4 * NC + 2;
  store_group(sb, rown, lane);
  reinterpret_cast<double2*>(sb + S_END * 64)[lane] = rend;
  store_group(sb + S_YL * 64, ryl, lane);
  store_group(sb + S_YR * 64, ryr, lane);
  store_group(sb + S_ZL * 64, rzl, lane);
  store_group(sb + S_ZR * 64, rzr, lane);
  wave_sync();

  // line layouts: lane = l + 16 q, node q along the direction, line l = t1 + 4 t2
  // over the two tangential indices in increasing dimension order
  const int q = lane >> 4, l = lane & 15, t1 = l & 3, t2 = l >> 2;
  const int nxl = q + 4 * t1 + 16 * t2;  // natural index of the x-layout lane
  const int nyl = t1 + 4 * q + 16 * t2;  // y-layout (the z-layout is the natural order)
  const int i0 = lane & 3, i1 = (lane >> 2) & 3, i2 = lane >> 4;
  const int srcx = i1 + 4 * i2 + 16 * i0, srcy = i0 + 4 * i2 + 16 * i1;  // lanes holding node `lane`
  const int ai = 4 * (lane & 3) + (lane >> 4);  // A operand: entry (lane % 4, lane / 16)

  const uint32_t mask = a.mask;
  const int vy = 3 * side_type(hy0, mask & 4u) + side_type(hy1, mask & 8u);
  const int vz = 3 * side_type(hz0, mask & 16u) + side_type(hz1, mask & 32u);
  double Kx_int = rec[0].x, Lx = rec[0].y, Rx = rec[1].x, Ky = rec[1].y, Ly = rec[2].x, Ry = rec[2].y;
  double Kz = rec[3].x, Lz = rec[3].y, Rz = rec[4].x;
  const double wt = rec[4].y;  // tangential weight of the lane's line
  if (vy != 0) Ky = a.Km[1][vy][ai];  // boundary rows and columns: other own-cell face terms
  if (vz != 0) Kz = a.Km[2][vz][ai];

  double out[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    out[k] = 0.0;
    if (k < nvalid) {
      const int ex = ex0 + k;
      const bool hx0 = ex > 0, hx1 = ex < nx - 1;
      const int sl = k == 0 ? S_END : k - 1;
      const int sr = k == nvalid - 1 ? S_END + 1 : k + 1;
      double Kx = Kx_int;
      if (!(hx0 && hx1)) Kx = a.Km[0][3 * side_type(hx0, mask & 1u) + side_type(hx1, mask & 2u)][ai];
      double cx = mfma(Kx, sb[k * 64 + nxl], 0.0);
      if (hx0) cx = mfma(Lx, sb[sl * 64 + nxl], cx);
      if (hx1) cx = mfma(Rx, sb[sr * 64 + nxl], cx);
      double cy = mfma(Ky, sb[k * 64 + nyl], 0.0);
      if (hy0) cy = mfma(Ly, sb[(S_YL + k) * 64 + nyl], cy);
      if (hy1) cy = mfma(Ry, sb[(S_YR + k) * 64 + nyl], cy);
      double cz = mfma(Kz, sb[k * 64 + lane], 0.0);
      if (hz0) cz = mfma(Lz, sb[(S_ZL + k) * 64 + lane], cz);
      if (hz1) cz = mfma(Rz, sb[(S_ZR + k) * 64 + lane], cz);
      out[k] = lane_read(wt * cx, srcx) + lane_read(wt * cy, srcy) + wt * cz;
    }
  }
  // results through the z-left slots (read above) and out as 16-byte pieces
  wave_sync();
#pragma unroll
  for (int k = 0; k < NC; ++k) sb[(S_ZL + k) * 64 + lane] = out[k];
  wave_sync();
  double2* __restrict__ y2 = reinterpret_cast<double2*>(y);
  const double2* so = reinterpret_cast<const double2*>(sb + S_ZL * 64);
#pragma unroll
  for (int k = 0; k < NC / 2; ++k) {
    const int i = lane + 64 * k;
    if (i < 32 * nvalid) y2[(size_t)c0 * 32 + i] = so[i];
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
  constexpr int WAVES = 1;  // wavefronts per block
  const int G = (int)((W + WAVES - 1) / WAVES);
  std::vector<uint32_t> tab(2 * (size_t)G * WAVES, 0);
  // logical wavefront t = chunk + nc (z in slab + hz y) + per_slab slab; hardware
  // wavefront WAVES b + v runs logical wavefront WAVES swizzle(b) + v
  for (int b = 0; b < G; ++b) {
    const int lb = xcd_swizzle_host(b, G);
    for (int v = 0; v < WAVES; ++v) {
      const int64_t t = (int64_t)lb * WAVES + v;
      const size_t hw = (size_t)b * WAVES + v;
      if (t >= W) {
        // past the end of the sweep: x index 65535 >= nx, so the wavefront has no cells
        tab[2 * hw] = 0xffffu;
        tab[2 * hw + 1] = 0;
        continue;
      }
      const int slab = (int)(t / per_slab), rem = (int)(t - (int64_t)slab * per_slab);
      const int hz = std::min(sz, nz - slab * sz);
      const int ey = rem / (nc * hz), rem2 = rem - ey * nc * hz;
      const int ezi = rem2 / nc, chunk = rem2 - ezi * nc;
      tab[2 * hw] = (uint32_t)(chunk * NC) | ((uint32_t)ey << 16);
      tab[2 * hw + 1] = (uint32_t)(slab * sz + ezi);
    }
  }
  hipError_t e = hipMalloc(&M.d_waves, sizeof(uint32_t) * tab.size());
  if (e != hipSuccess) return e;
  M.nwaves = (int64_t)G * WAVES;
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
