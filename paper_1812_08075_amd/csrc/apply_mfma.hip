// Matrix-core apply of the SIPG diffusion-reaction operator for k = 3 (p = 4
// nodes per direction), kappa = 1, axis-aligned cells (gfx950), on FP64 or
// FP32 vectors.
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
//    and read back in the x, y and z layouts; the x-lines of the cells beyond
//    both ends of the chunk are read from global memory. The LDS layout is
//    padded (i1, i2 and cell strides 4, 18, 70 doubles) against bank
//    conflicts of the three access layouts.
//  * A wavefront owns a chunk of NC = 4 x-consecutive cells and marches
//    along y over up to 16 rows of it (the count comes with its table
//    entry). Two LDS buffers hold the rows y and y + 1: per step the
//    wavefront reads from global memory only the row y + 1 (in the z
//    layout, into the buffer that held row y - 1), the z-neighbour cells
//    and the two x-end lines; the y-neighbour lines come from LDS, row
//    y - 1 read before it is replaced. That is 8 global loads per 4 cells
//    where reading the y-neighbours from L2 takes 12 (the load issue rate
//    bounded the kernel that read them from L2). Marches of odd
//    y-blocks run downwards (mirror image: the row behind is y + 1), so
//    that two neighbouring marches reach the rows of their shared boundary
//    at the same time. The A-operand entries
//    of the nine interior-cell operators and the two nodes' tensor weights
//    form one 96-byte record per lane, read once per wavefront; the K
//    variants of the chunk's boundary cells and of the boundary rows are
//    copied to LDS before the march. Wavefronts are independent (one per
//    block).
//  * Global memory is read and written through buffer resources over the
//    wavefront's window of x and y: absent values (missing neighbours,
//    cells beyond the mesh) come from out-of-range offsets as zeros, so a
//    step issues the same reads every time, in the order of use (the x-end
//    lines, the next row, the z-neighbour rows), and waits only for the
//    ones needed next: the next row arrives during the x stage, the
//    z-neighbour rows during the x and y stages.
//  * Results: the x results are written to LDS, the y results added to them
//    in the y-pair layout, and the z results added on reading them back in
//    the z-pair layout; the sum times the tensor weight is stored with
//    16-byte non-temporal stores, which keep the output from displacing
//    input cells that neighbours still need from L2.
//  * Each XCD (its own L2) sweeps one region of the mesh: x and z are split
//    so that the fewest cells are read across region boundaries, y is not
//    split, and inside a region the wavefronts run y-outermost, then z,
//    then x, so that the z-neighbour cells are still in the XCD's L2. The
//    hardware dispatches block b to XCD b mod 8; a table built on the host
//    maps blocks to wavefront positions accordingly.
//
// FP32 vectors. The arithmetic is FP64 on the same operator tables and in
// the same order, so the result is the FP64 kernel's result for the FP32
// input, rounded once to FP32. A 16-byte load carries four FP32 values: a
// whole x-line of a cell. The "quad layout" holds in one lane the four nodes
// i0 = 0..3 of one x-line: lane = i1 + 4 c + 16 i2 for the z direction, lane
// = i2 + 4 c + 16 i1 for the y direction, c the cell of the chunk; converted
// to FP64, each of the four components is an operand of the same product.
// Per step one 16-byte load each for row y + 1 and the two z-neighbour rows.
//
// The wavefront's march (the x direction, the LDS buffers, the order of the
// directions, the reduction) is one template; the layout of the y and z
// directions and of the loads and stores is a policy per precision
// (PairLanes, QuadLanes).
#include <algorithm>
#include <vector>

#include "internal.h"

namespace dgi {
namespace {

constexpr int NC = 4;            // cells per step (consecutive along x): two pairs
constexpr int NYMAX = 16;        // most rows along y per wavefront
// LDS node (i0, i1, i2) of cell c at c LCS + i2 LPS + i1 LIS + i0 (doubles):
// padded against bank conflicts of the three access layouts
constexpr int LIS = 4, LPS = 18, LCS = 70;
constexpr int T_INT = 0, T_DIR = 1, T_NONE = 2;

__device__ __forceinline__ double mfma(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Reads of a wavefront go through a buffer resource over the part of the
// input vector its march can touch (its window). A lane whose value is absent
// (a missing neighbour, a cell beyond the mesh) reads at an offset beyond the
// window and gets zeros from the hardware, without a branch: every step
// issues the same reads in the same order, so each wait covers only the
// reads needed next and the later ones stay in flight.
template <class T>
struct Window {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ Window(const T* base, uint32_t bytes)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base), (short)0, (int)bytes, 0x00020000)) {}
  static __device__ __forceinline__ uint32_t at(int64_t e, bool v) {
    return v ? (uint32_t)e * (uint32_t)sizeof(T) : 0x80000000u;
  }
  // 16 bytes at element e of the window (zeros when !v)
  __device__ __forceinline__ dvec2 load2(int64_t e, bool v) const {
    return __builtin_bit_cast(dvec2, __builtin_amdgcn_raw_buffer_load_b128(r, at(e, v), 0, 0));
  }
  __device__ __forceinline__ fvec4 load4(int64_t e, bool v) const {
    return __builtin_bit_cast(fvec4, __builtin_amdgcn_raw_buffer_load_b128(r, at(e, v), 0, 0));
  }
  // 16 bytes to element e, non-temporal (dropped when !v)
  __device__ __forceinline__ void store16(int64_t e, bool v, dvec2 d) const {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, d), r, at(e, v), 0, 2);
  }
  __device__ __forceinline__ void store16(int64_t e, bool v, fvec4 d) const {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, d), r, at(e, v), 0, 2);
  }
  // one value at element e (zero when !v)
  __device__ __forceinline__ double load1(int64_t e, bool v) const {
    if constexpr (sizeof(T) == 8)
      return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, at(e, v), 0, 0));
    else
      return (double)__builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, at(e, v), 0, 0));
  }
};

__device__ __forceinline__ int side_type(bool has, bool dirichlet) {
  return has ? T_INT : (dirichlet ? T_DIR : T_NONE);
}

struct Quad {
  double v[4];
};

// one FP32 x-line (zeros when !ok), widened to FP64
__device__ __forceinline__ Quad load_quad(const Window<float>& w, int64_t e, bool ok) {
  const fvec4 r = w.load4(e, ok);
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

// Operator entries of the lane (entry (lane % 4, lane / 16) of the x, y and
// z line operators of an interior cell: K, L, R each).
struct LineOps {
  double Kx, Lx, Rx, Ky, Ly, Ry, Kz, Lz, Rz;
};

// FP64 vectors, pair layout: lane = h + 2 t + 8 c + 16 n, the register's
// components the nodes i0 = 2h, 2h + 1 of cell c of a pair, (t, n) = (i1, i2)
// in the z layout and (i2, i1) in the y layout.
struct PairLanes {
  using T = double;
  struct Rows {
    double2 v[2];
  };
  int pc, offz, lz, ly;
  double2 wn;
  __device__ __forceinline__ PairLanes(int lane, const ScalarArgs<double>& a, int, LineOps& op) {
    const int h = lane & 1, t = (lane >> 1) & 3, n = lane >> 4;
    pc = (lane >> 3) & 1;
    offz = 2 * h + 4 * t + 16 * n + 64 * pc;
    lz = 2 * h + LIS * t + LPS * n + LCS * pc;
    ly = 2 * h + LPS * t + LIS * n + LCS * pc;
    double2 rec[6];
    const double2* lr = reinterpret_cast<const double2*>(a.lrec[lane]);
#pragma unroll
    for (int k = 0; k < 6; ++k) rec[k] = lr[k];
    op = LineOps{rec[0].x, rec[0].y, rec[1].x, rec[1].y, rec[2].x, rec[2].y, rec[3].x, rec[3].y, rec[4].x};
    wn = rec[5];
  }
  // the first row of the march (buffer cur) and the row behind it, at
  // offset back (buffer oth), of the chunk at element ec of the window
  __device__ __forceinline__ void first_rows(double* cur, double* oth, const Window<double>& w, int64_t ec,
                                             int64_t back, int nvalid, bool has_prev) const {
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const bool v = 2 * p + pc < nvalid;
      const dvec2 u0 = w.load2(ec + 128 * p + offz, v);
      const dvec2 um = w.load2(ec + back + 128 * p + offz, v && has_prev);
      *reinterpret_cast<dvec2*>(cur + 2 * LCS * p + lz) = u0;
      *reinterpret_cast<dvec2*>(oth + 2 * LCS * p + lz) = um;
    }
  }
  __device__ __forceinline__ Rows load_rows(const Window<double>& w, int64_t ec, int64_t off, int nvalid,
                                            bool ok) const {
    Rows r;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const dvec2 u = w.load2(ec + off + 128 * p + offz, ok && 2 * p + pc < nvalid);
      r.v[p] = make_double2(u.x, u.y);
    }
    return r;
  }
  __device__ __forceinline__ Rows lds_y(const double* b) const {
    Rows r;
#pragma unroll
    for (int p = 0; p < 2; ++p) r.v[p] = *reinterpret_cast<const double2*>(b + 2 * LCS * p + ly);
    return r;
  }
  __device__ __forceinline__ void store_z(double* b, const Rows& r) const {
#pragma unroll
    for (int p = 0; p < 2; ++p) *reinterpret_cast<double2*>(b + 2 * LCS * p + lz) = r.v[p];
  }
  // sr += the y lines of row cur; neighbours: yb (the row behind) and the
  // row in oth (the row ahead), on the y - 1 and y + 1 sides for an upward
  // march and the other way round for a downward one
  template <bool DOWN>
  __device__ __forceinline__ void y_stage(const double* cur, const double* oth, double* sr, const Rows& yb, double Ky,
                                          double Ly, double Ry, bool hy0, bool hy1, int nvalid) const {
    double2 uy[2], yr[2];
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      uy[p] = *reinterpret_cast<const double2*>(cur + 2 * LCS * p + ly);
      yr[p] = *reinterpret_cast<const double2*>(oth + 2 * LCS * p + ly);
    }
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      if (2 * p < nvalid) {
        const double2 c = DOWN ? pair_line(Ky, Ly, Ry, uy[p], yr[p], yb.v[p], hy0, hy1)
                               : pair_line(Ky, Ly, Ry, uy[p], yb.v[p], yr[p], hy0, hy1);
        double2* r = reinterpret_cast<double2*>(sr + 2 * LCS * p + ly);
        const double2 o = *r;
        *r = make_double2(o.x + c.x, o.y + c.y);
      }
    }
  }
  // the z lines, the sum of the three directions times the tensor weight, the store
  template <bool DOT>
  __device__ __forceinline__ void z_stage(const double* cur, const double* sr, const Rows& zl, const Rows& zr,
                                          double Kz, double Lz, double Rz, bool hz0, bool hz1, int nvalid,
                                          const Window<double>& yw, int64_t ec, double& pq) const {
    double2 uz[2];
#pragma unroll
    for (int p = 0; p < 2; ++p) uz[p] = *reinterpret_cast<const double2*>(cur + 2 * LCS * p + lz);
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      if (2 * p < nvalid) {
        const double2 c = pair_line(Kz, Lz, Rz, uz[p], zl.v[p], zr.v[p], hz0, hz1);
        const double2 o = *reinterpret_cast<const double2*>(sr + 2 * LCS * p + lz);
        const bool ok = 2 * p + pc < nvalid;
        const dvec2 v = {wn.x * (o.x + c.x), wn.y * (o.y + c.y)};
        yw.store16(ec + 128 * p + offz, ok, v);
        if (DOT && ok) pq = fma(uz[p].y, v.y, fma(uz[p].x, v.x, pq));
      }
    }
  }
};

// FP32 vectors, quad layout: one x-line of cell c per lane, lane = i1 + 4 c
// + 16 i2 (z layout) or i2 + 4 c + 16 i1 (y layout).
struct QuadLanes {
  using T = float;
  using Rows = Quad;
  int offz, lz, ly;
  bool cok;  // the lane's cell is in the chunk
  double wq[4];
  __device__ __forceinline__ QuadLanes(int lane, const ScalarArgs<double>& a, int nvalid, LineOps& op) {
    const int c = (lane >> 2) & 3;
    cok = c < nvalid;
    const int zi1 = lane & 3, zi2 = lane >> 4;  // z layout
    const int yi2 = lane & 3, yi1 = lane >> 4;  // y layout
    offz = 64 * c + 4 * zi1 + 16 * zi2;
    lz = LCS * c + LIS * zi1 + LPS * zi2;
    ly = LCS * c + LIS * yi1 + LPS * yi2;
    const double* rl = a.lrec[lane];
    op = LineOps{rl[0], rl[1], rl[2], rl[3], rl[4], rl[5], rl[6], rl[7], rl[8]};
    // the tensor weights of the lane's four nodes, from the records of the
    // lanes that hold them in the pair layout
#pragma unroll
    for (int q = 0; q < 4; ++q) wq[q] = a.lrec[(q >> 1) + 2 * zi1 + 16 * zi2][10 + (q & 1)];
  }
  __device__ __forceinline__ void first_rows(double* cur, double* oth, const Window<float>& w, int64_t ec,
                                             int64_t back, int, bool has_prev) const {
    lds_store_quad(cur + lz, load_quad(w, ec + offz, cok));
    lds_store_quad(oth + lz, load_quad(w, ec + back + offz, cok && has_prev));
  }
  __device__ __forceinline__ Rows load_rows(const Window<float>& w, int64_t ec, int64_t off, int, bool ok) const {
    return load_quad(w, ec + off + offz, cok && ok);
  }
  __device__ __forceinline__ Rows lds_y(const double* b) const { return lds_quad(b + ly); }
  __device__ __forceinline__ void store_z(double* b, const Rows& r) const { lds_store_quad(b + lz, r); }
  template <bool DOWN>
  __device__ __forceinline__ void y_stage(const double* cur, const double* oth, double* sr, const Rows& yb, double Ky,
                                          double Ly, double Ry, bool hy0, bool hy1, int) const {
    const Quad ya = lds_quad(oth + ly);
    const Quad cy = DOWN ? quad_line(Ky, Ly, Ry, lds_quad(cur + ly), ya, yb, hy0, hy1)
                         : quad_line(Ky, Ly, Ry, lds_quad(cur + ly), yb, ya, hy0, hy1);
    Quad o = lds_quad(sr + ly);
#pragma unroll
    for (int q = 0; q < 4; ++q) o.v[q] = o.v[q] + cy.v[q];
    lds_store_quad(sr + ly, o);
  }
  template <bool DOT>
  __device__ __forceinline__ void z_stage(const double* cur, const double* sr, const Rows& zl, const Rows& zr,
                                          double Kz, double Lz, double Rz, bool hz0, bool hz1, int,
                                          const Window<float>& yw, int64_t ec, double& pq) const {
    const Quad uz = lds_quad(cur + lz);
    const Quad cz = quad_line(Kz, Lz, Rz, uz, zl, zr, hz0, hz1);
    const Quad o = lds_quad(sr + lz);
    fvec4 v;
    v.x = (float)(wq[0] * (o.v[0] + cz.v[0]));
    v.y = (float)(wq[1] * (o.v[1] + cz.v[1]));
    v.z = (float)(wq[2] * (o.v[2] + cz.v[2]));
    v.w = (float)(wq[3] * (o.v[3] + cz.v[3]));
    yw.store16(ec + offz, cok, v);
    if (DOT && cok) {
      pq = fma(uz.v[0], (double)v.x, pq);
      pq = fma(uz.v[1], (double)v.y, pq);
      pq = fma(uz.v[2], (double)v.z, pq);
      pq = fma(uz.v[3], (double)v.w, pq);
    }
  }
};

// One wavefront per block; the wavefronts are independent. A wavefront
// handles NC cells along x in each of its rows along y, one row per step.
// DOT: each wavefront also writes the sum of x_i y_i over its cells (FP64,
// fixed order) to partial[block]: the p.Ap of a conjugate-gradient iteration.
template <bool D>
struct MarchDir {
  static constexpr bool value = D;
};

template <class Lanes, bool DOT>
__device__ __forceinline__ void apply_q3_wave(const typename Lanes::T* __restrict__ x, typename Lanes::T* __restrict__ y,
                                              const ScalarArgs<double>* __restrict__ ap,
                                              const uint32_t* __restrict__ waves, double* __restrict__ partial) {
  using T = typename Lanes::T;
  __shared__ __attribute__((aligned(16))) double su[2 * NC * LCS];  // own cells of rows y and y + 1
  __shared__ __attribute__((aligned(16))) double sr[NC * LCS];      // x results, then x + y results
  __shared__ double sk[5][64];                                      // boundary operators
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
  const int nsteps = min((int)((w1 >> 16) & 0x7fffu), ny - ey0);
  const bool hxl = ex0 > 0, hxr = ex0 + nvalid < nx;
  const int64_t sy = (int64_t)nx * 64, sz = (int64_t)nx * ny * 64;  // neighbour strides in values
  const bool hz0 = ez > 0, hz1 = ez < nz - 1;
  // x layout: lane = i1 + 4 i2 + 16 i0, one cell per register
  const int offx = (lane >> 4) + 4 * (lane & 3) + 16 * ((lane >> 2) & 3);
  const int lx = (lane >> 4) + LIS * (lane & 3) + LPS * ((lane >> 2) & 3);

  LineOps op;
  const Lanes ln(lane, a, nvalid, op);
  const int ai = 4 * (lane & 3) + (lane >> 4);
  const uint32_t mask = a.mask;
  const int vz = 3 * side_type(hz0, mask & 16u) + side_type(hz1, mask & 32u);
  const double Kz = vz != 0 ? a.Km[2][vz][ai] : op.Kz;

  // the wavefront's window: every element its march may read (rows ey0 - 1
  // to ey0 + nsteps of the planes ez - 1 to ez + 1, cells ex0 - 1 to
  // ex0 + NC), clipped to the vector
  const int ylo = max(ey0 - 1, 0), yhi = min(ey0 + nsteps, ny - 1);
  const int zlo = max(ez - 1, 0), zhi = min(ez + 1, nz - 1);
  const int64_t wlo = ((int64_t)nx * (ylo + (int64_t)ny * zlo) + max(ex0 - 1, 0)) * 64;
  const int64_t whi = ((int64_t)nx * (yhi + (int64_t)ny * zhi) + min(ex0 + NC + 1, nx)) * 64;
  const Window<T> win(x + wlo, (uint32_t)((whi - wlo) * (int64_t)sizeof(T)));
  const Window<T> yw(y + wlo, (uint32_t)((whi - wlo) * (int64_t)sizeof(T)));  // the same range of y
  // Boundary operators in LDS, read before the march: the x operators of the
  // chunk's first and last cells (the cells between are interior) and the y
  // operators of the first row, the last row and a single row. A global
  // read of them inside a step would sit in a branch, and the wait after it
  // would also drain the step's z-neighbour reads still in flight.
  const int exl = ex0 + nvalid - 1;
  const bool f0 = ex0 > 0, f1 = ex0 < nx - 1, l0 = exl > 0, l1 = exl < nx - 1;
  const int yb0 = 3 * side_type(false, mask & 4u), yb1 = side_type(false, mask & 8u);
  sk[0][lane] = a.Km[0][3 * side_type(f0, mask & 1u) + side_type(f1, mask & 2u)][ai];
  sk[1][lane] = a.Km[0][3 * side_type(l0, mask & 1u) + side_type(l1, mask & 2u)][ai];
  sk[2][lane] = a.Km[1][yb0][ai];
  sk[3][lane] = a.Km[1][yb1][ai];
  sk[4][lane] = a.Km[1][yb0 + yb1][ai];

  // The march runs up (y increasing) or, where the table entry's top bit is
  // set, down: odd y-blocks run down, so that the two wavefronts next to a
  // y-block boundary read the boundary rows at the same time (at both ends
  // of their marches), from the XCD's L2 rather than twice from HBM.
  auto march = [&](auto dir) {
    constexpr bool DOWN = decltype(dir)::value;
    const int eyf = DOWN ? ey0 + nsteps - 1 : ey0;  // first row of the march
    const int64_t row0 = (int64_t)nx * ((int64_t)eyf + (int64_t)ny * ez);
    const int64_t ahead = DOWN ? -sy : sy;  // offset of the next row
    // first row to buffer 0, the row behind it to buffer 1 (invalid or
    // absent cells as zeros)
    ln.first_rows(su, su + NC * LCS, win, (row0 + ex0) * 64 - wlo, -ahead, nvalid, DOWN ? eyf < ny - 1 : eyf > 0);

    for (int s = 0; s < nsteps; ++s) {
      const int ey = DOWN ? eyf - s : eyf + s;
      const bool hy0 = ey > 0, hy1 = ey < ny - 1;
      const int64_t row = DOWN ? row0 - (int64_t)s * nx : row0 + (int64_t)s * nx;
      const int64_t ec = (row + ex0) * 64 - wlo;      // the chunk in the window
      double* cur = su + (s & 1) * (NC * LCS);        // row ey
      double* oth = su + ((s + 1) & 1) * (NC * LCS);  // the row behind, then the row ahead

      // in the order of use: the x-end lines (the x stage), the next row
      // (stored to LDS after the x stage), the z-neighbour rows (the z stage)
      // (empty asm statements with a memory clobber pin that order: the
      // wait for a read also waits for every read issued before it)
      const double xl = win.load1(ec + offx - 64, hxl);
      const double xr = win.load1(ec + 64 * nvalid + offx, hxr);
      asm volatile("" ::: "memory");
      const typename Lanes::Rows nr = ln.load_rows(win, ec, ahead, nvalid, DOWN ? hy0 : hy1);
      asm volatile("" ::: "memory");
      const typename Lanes::Rows zl = ln.load_rows(win, ec, -sz, nvalid, hz0);
      const typename Lanes::Rows zr = ln.load_rows(win, ec, sz, nvalid, hz1);

      // the row behind in the y layout, before the next row replaces it
      const typename Lanes::Rows yb = ln.lds_y(oth);
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
          double Kx = op.Kx;
          if (!(hx0 && hx1)) Kx = sk[k == 0 ? 0 : 1][lane];
          // without a neighbour the x-end line read zeros, and its term adds
          // zero: no branch, so the compiler keeps the x-end reads where they
          // are issued instead of sinking them into the branch
          double cx = mfma(Kx, ux[k], 0.0);
          cx = mfma(op.Lx, ul, cx);
          cx = mfma(op.Rx, ur, cx);
          sr[LCS * k + lx] = cx;
        }
      }
      // the next row replaces the row behind only now, so that its read
      // has the x stage to arrive
      ln.store_z(oth, nr);
      __syncthreads();
      const double Ky = hy0 && hy1 ? op.Ky : sk[hy1 ? 2 : (hy0 ? 3 : 4)][lane];
      ln.template y_stage<DOWN>(cur, oth, sr, yb, Ky, op.Ly, op.Ry, hy0, hy1, nvalid);
      __syncthreads();
      ln.template z_stage<DOT>(cur, sr, zl, zr, Kz, op.Lz, op.Rz, hz0, hz1, nvalid, yw, ec, pq);
    }
  };
  if (w1 >> 31)
    march(MarchDir<true>{});
  else
    march(MarchDir<false>{});
  if (DOT) {  // butterfly over the 64 lanes, then lane 0 writes
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) pq += __shfl_xor(pq, m, 64);
    if (lane == 0) partial[blockIdx.x] = pq;
  }
}

// The applies, with a register budget for five wavefronts per SIMD (the
// matrix-core results in architectural VGPRs), and the conjugate-gradient
// variants with the fused p.Ap.
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(5)))
    k_apply_q3_mfma(const double* __restrict__ x, double* __restrict__ y, const ScalarArgs<double>* __restrict__ ap,
                    const uint32_t* __restrict__ waves) {
  apply_q3_wave<PairLanes, false>(x, y, ap, waves, nullptr);
}

__global__ void __launch_bounds__(64)
    k_apply_q3_mfma_dot(const double* __restrict__ x, double* __restrict__ y,
                        const ScalarArgs<double>* __restrict__ ap, const uint32_t* __restrict__ waves,
                        double* __restrict__ partial) {
  apply_q3_wave<PairLanes, true>(x, y, ap, waves, partial);
}

__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(5)))
    k_apply_q3_mfma_f32(const float* __restrict__ x, float* __restrict__ y,
                        const ScalarArgs<double>* __restrict__ ap, const uint32_t* __restrict__ waves) {
  apply_q3_wave<QuadLanes, false>(x, y, ap, waves, nullptr);
}

__global__ void __launch_bounds__(64)
    k_apply_q3_mfma_f32_dot(const float* __restrict__ x, float* __restrict__ y,
                            const ScalarArgs<double>* __restrict__ ap, const uint32_t* __restrict__ waves,
                            double* __restrict__ partial) {
  apply_q3_wave<QuadLanes, true>(x, y, ap, waves, partial);
}

// XCD-aware renumbering of hardware blocks (block b runs on XCD b % 8).
int xcd_swizzle_host(int b, int G) {
  const int q = G >> 3, r = G & 7;
  const int xcd = b & 7, idx = b >> 3;
  return xcd * q + std::min(xcd, r) + idx;
}

}  // namespace

bool mfma_apply_supported(const dg_mesh& M, int prec, bool kappa) {
  return M.p == 4 && prec == DG_F64 && !kappa && M.d_waves[DG_F64] != nullptr && !M.lines_forced[DG_F64];
}

// Rows per wavefront: the most, up to NYMAX, that still leave at least 4096
// wavefronts (16 per CU), else one. Longer marches save more loads (8 global
// loads per 4 cells with the y-neighbours from LDS, against 12 for one row)
// but fewer, longer wavefronts fill the chip less evenly.
int mfma_default_rows(int nx, int ny, int nz) {
  const int nc = (nx + NC - 1) / NC;
  for (int r = NYMAX; r > 1; r /= 2)
    if ((int64_t)nc * ((ny + r - 1) / r) * nz >= 4096) return r;
  return 1;
}

// A wavefront's window (two planes and the march's rows around it) must stay
// below 2 GiB: its reads take 32-bit byte offsets, and the offsets above it
// mark the absent values.
static bool mfma_window_fits(int nx, int ny, int rows) {
  const int64_t cells = 2LL * nx * ny + (int64_t)(rows + 2) * nx + NC + 2;
  return cells * 64 * (int64_t)sizeof(double) < (1LL << 31);
}

hipError_t mfma_setup(dg_mesh& M) {
  if (M.p != 4) return hipSuccess;
  // meshes with larger planes run the line kernels
  if (!mfma_window_fits(M.desc.nx, M.desc.ny, NYMAX)) return hipSuccess;
  hipError_t e = mfma_build(M, DG_F64, 0);
  if (e != hipSuccess) return e;
  return mfma_build(M, DG_F32, 0);
}

hipError_t mfma_build(dg_mesh& M, int prec, int rows) {
  if (M.p != 4 || (prec != DG_F64 && prec != DG_F32)) return hipErrorInvalidValue;
  const int nx = M.desc.nx, ny = M.desc.ny, nz = M.desc.nz;
  const int nc = (nx + NC - 1) / NC;
  if (rows <= 0) rows = mfma_default_rows(nx, ny, nz);
  if (rows > NYMAX) return hipErrorInvalidValue;
  const int nyb = (ny + rows - 1) / rows;
  const int64_t W = (int64_t)nc * nyb * nz;
  if (W > 0x7fffffff / 2 || !mfma_window_fits(nx, ny, rows)) return hipErrorInvalidValue;
  // One region of the mesh per XCD: the split (rx, ry, rz), rx ry rz = 8, that
  // reads the fewest cells across region boundaries (each XCD has its own
  // L2, so a neighbour cell of another region is fetched again).
  int best[3] = {1, 1, 8};
  double best_cost = -1;
  const int ext[3] = {nc, nyb, nz};
  // The y direction is not split: the sweep runs along y, and its front (the
  // region's x-z cross-section) is the same for every (rx, rz).
  for (int rx = 1; rx <= 8; rx *= 2)
    for (int ry = 1; ry == 1; ry *= 2) {
      const int rz = 8 / (rx * ry);
      const int r[3] = {rx, ry, rz};
      bool ok = true;
      for (int d = 0; d < 3; ++d) ok = ok && r[d] <= ext[d];
      if (!ok) continue;
      const double cost = (double)(rx - 1) * ny * nz + (double)(ry - 1) * nx * nz + (double)(rz - 1) * nx * ny;
      if (best_cost < 0 || cost < best_cost) {
        best_cost = cost;
        best[0] = rx;
        best[1] = ry;
        best[2] = rz;
      }
    }
  if (best_cost < 0) best[0] = best[1] = best[2] = 1;  // tiny meshes: one region
  // region bounds (x in whole chunks)
  auto bound = [](int n, int r, int i) { return (int)(((int64_t)n * i) / r); };
  const int G = (int)W;
  std::vector<uint32_t> order(2 * (size_t)G, 0);
  size_t t = 0;
  for (int gz = 0; gz < best[2]; ++gz)
    for (int gy = 0; gy < best[1]; ++gy)
      for (int gx = 0; gx < best[0]; ++gx) {
        const int c0 = bound(nc, best[0], gx), c1 = bound(nc, best[0], gx + 1);
        const int y0 = bound(nyb, best[1], gy), y1 = bound(nyb, best[1], gy + 1);
        const int z0 = bound(nz, best[2], gz), z1 = bound(nz, best[2], gz + 1);
        // inside a region: y outermost, then z, then the x chunks
        for (int yy = y0; yy < y1; ++yy)
          for (int zz = z0; zz < z1; ++zz)
            for (int cc = c0; cc < c1; ++cc) {
              const int ey0 = yy * rows;
              order[2 * t] = (uint32_t)(cc * NC) | ((uint32_t)ey0 << 16);
              order[2 * t + 1] = (uint32_t)zz | ((uint32_t)std::min(rows, ny - ey0) << 16) |
                                 ((yy & 1) ? 0x80000000u : 0u);
              ++t;
            }
      }
  if (t != (size_t)G) return hipErrorInvalidValue;
  // hardware block b (one wavefront) runs logical wavefront swizzle(b)
  std::vector<uint32_t> tab(2 * (size_t)G, 0);
  for (int b = 0; b < G; ++b) {
    const int l = xcd_swizzle_host(b, G);
    tab[2 * (size_t)b] = order[2 * (size_t)l];
    tab[2 * (size_t)b + 1] = order[2 * (size_t)l + 1];
  }
  uint32_t* d = nullptr;
  hipError_t e = hipMalloc(&d, sizeof(uint32_t) * tab.size());
  if (e != hipSuccess) return e;
  e = hipMemcpy(d, tab.data(), sizeof(uint32_t) * tab.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(d);
    return e;
  }
  // the old table may still be read by work queued on any stream
  if (M.d_waves[prec]) {
    e = hipDeviceSynchronize();
    if (e != hipSuccess) {
      (void)hipFree(d);
      return e;
    }
    (void)hipFree(M.d_waves[prec]);
  }
  M.d_waves[prec] = d;
  M.nwaves[prec] = G;
  M.mfma_rows[prec] = rows;
  return hipSuccess;
}

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

hipError_t mfma_apply(const dg_mesh& M, int variant, const double* x, double* y, double* partial, hipStream_t s) {
  if (M.ndofs > 0xffffffffLL) return hipErrorInvalidValue;
  const int64_t G = M.nwaves[DG_F64];
  if (G < 1) return hipSuccess;
  if (partial)
    hipLaunchKernelGGL(k_apply_q3_mfma_dot, dim3((unsigned)G), dim3(64), 0, s, x, y, M.d_pd + variant,
                       (const uint32_t*)M.d_waves[DG_F64], partial);
  else
    hipLaunchKernelGGL(k_apply_q3_mfma, dim3((unsigned)G), dim3(64), 0, s, x, y, M.d_pd + variant,
                       (const uint32_t*)M.d_waves[DG_F64]);
  return hipGetLastError();
}

}  // namespace dgi
