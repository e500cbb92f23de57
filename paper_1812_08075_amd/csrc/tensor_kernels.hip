// The SIPG diffusion-reaction operator with a full coefficient tensor at every
// quadrature point: Section 5.2's benchmark problem, -div(K grad u) + c u = f
// with K(x) = x x^T + I, f = -6 and Dirichlet data g(x) = |x|^2 on the unit
// cube (eq. diffreac_weak), on axis-aligned cells (gfx950).
//
// Unlike kappa I, a full tensor couples the three directions at every point,
// so the kernel follows Algorithm 1 as it stands:
//  part 1  the reference derivatives d_0 u, d_1 u, d_2 u at all points, one
//          1D contraction with D along each direction (collocation: the basis
//          matrix A is the identity, u at the points is the coefficients);
//  part 2  at every point the flux w |J| K(x) grad u and the mass term
//          w |J| c u (the residual also subtracts w |J| f);
//  part 3  the transposed contractions D^T of the three flux components.
// Faces (Section 2.2, m_d = 1): the normal direction is contracted first, for
// the own cell and for the neighbour across the face, giving each side's trace
// and normal derivative at the face points; the tangential derivatives, which
// K n . grad u needs as well, are D contractions of the traces on the face.
// The flux -{K grad u}.n [v] + theta [u] {K grad v}.n + gamma [u][v] (and on
// Dirichlet sides the data terms of g) is tested with the own cell's trace,
// normal-derivative and tangential-derivative rows only: element-centric, no
// atomics, one writer per output.
//
// Threads own 1D lines: p^2 threads per cell own its lines along x, along y,
// then along z; a block is a chunk of up to 128 / p^2 consecutive cells of one
// x-row (its cells are contiguous in memory), so x-neighbours inside the chunk
// come from LDS, the others from global memory (L2). Face work for the two
// sides of direction d runs on the d-lines, with the traces and the
// tangential test fluxes exchanged through small per-cell face buffers.
#include "line_common.h"

namespace dgi {
namespace {

// blocks of the 128-thread sweep grid (the adjoint's)
int64_t tensor_grid(const dg_mesh& M) {
  const ScalarArgs<double>& a = M.pd[SP_ADJOINT];
  return (int64_t)a.nchunk * a.n[1] * a.n[2];
}

template <int P>
struct TensorCells {
  static constexpr int value = (128 / (P * P)) > 0 ? (128 / (P * P)) : 1;
};

// Section 5.2's coefficient tensor: (K g)_r = x_r (x . g) + g_r.
template <typename T>
__device__ __forceinline__ T kx_row(const T* x, int r, T xg, T gr) {
  return fma(x[r], xg, gr);
}

// Physical coordinate along direction d of node index i in cell position c.
template <typename T>
__device__ __forceinline__ T coord(const ScalarArgs<T>& a, int c, T xi, int d) {
  return (T(c) + xi) / T(a.n[d]);
}

// Face work of the two sides of direction DIR for the thread's d-line
// (tangential node indices ta, tb). Adds the own-cell test contributions to
// `out`. `v`: the own line; `nb[s]`: the neighbour's line across side s (zero
// when absent); `fb`: this cell's face buffers, 8 arrays of p^2 values
// ([own trace, neighbour trace, tangential test flux a, b] per side).
// RESIDUAL adds the Dirichlet data terms of g. Called by every thread of the
// block (it synchronizes twice); inactive threads pass active = false.
// tD, tW, tX: the block's LDS copies of D, the weights and the nodes, for the
// reads whose index depends on the thread (from the parameter block each such
// read would be a vector load of its own).
template <int P, typename T, bool RESIDUAL, int DIR>
__device__ __forceinline__ void tensor_faces(const ScalarArgs<T>& a, bool active, const T* v, const T (*nb)[P],
                                             const bool* has, const int* cc, int ta, int tb, T* fb, T* out,
                                             const T* tD, const T* tW, const T* tX) {
  constexpr int L = P * P;
  constexpr int DA = DIR == 0 ? 1 : 0, DB = DIR == 2 ? 1 : 2;  // tangential directions
  const int pt = ta + P * tb;
  T To[2], Tn[2], No[2], Nn[2];
  if (active) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      T t0 = T(0), n0 = T(0), t1 = T(0), n1 = T(0);
#pragma unroll
      for (int j = 0; j < P; ++j) {
        t0 = fma(a.e[s][j], v[j], t0);
        n0 = fma(a.de[s][j], v[j], n0);
        t1 = fma(a.e[1 - s][j], nb[s][j], t1);
        n1 = fma(a.de[1 - s][j], nb[s][j], n1);
      }
      To[s] = t0;
      No[s] = n0;
      Tn[s] = t1;
      Nn[s] = n1;
      fb[(4 * s + 0) * L + pt] = t0;
      fb[(4 * s + 1) * L + pt] = t1;
    }
  }
  __syncthreads();
  T Rv[2] = {T(0), T(0)}, Rd[2] = {T(0), T(0)};
  if (active) {
    const T ha_inv = a.hinv[DA], hb_inv = a.hinv[DB], hd_inv = a.hinv[DIR];
    const T wF = tW[ta] * tW[tb] * a.fs[DIR];  // tangential weights x |F| / reference area
    T xF[3];
    xF[DA] = coord(a, cc[DA], tX[ta], DA);
    xF[DB] = coord(a, cc[DB], tX[tb], DB);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      T Ra = T(0), Rb = T(0);
      const bool dirichlet = (a.mask >> (2 * DIR + s)) & 1u;
      if (has[s] || dirichlet) {
        xF[DIR] = T(cc[DIR] + s) / T(a.n[DIR]);
        const T sg = s ? T(1) : T(-1);  // own cell is T- on side 1 (n_F = +e_d)
        // own physical gradient at the face point
        const T* fo = fb + (4 * s + 0) * L;
        T ga = T(0), gb = T(0);
#pragma unroll
        for (int j = 0; j < P; ++j) {
          ga = fma(tD[ta * P + j], fo[j + P * tb], ga);
          gb = fma(tD[tb * P + j], fo[ta + P * j], gb);
        }
        T g[3];
        g[DIR] = No[s] * hd_inv;
        g[DA] = ga * ha_inv;
        g[DB] = gb * hb_inv;
        const T xg = xF[0] * g[0] + xF[1] * g[1] + xF[2] * g[2];
        const T qo = kx_row(xF, DIR, xg, g[DIR]);  // (K grad u_own)_d
        T Kd[3];  // row d of K at the face point
#pragma unroll
        for (int b = 0; b < 3; ++b) Kd[b] = xF[DIR] * xF[b] + (b == DIR ? T(1) : T(0));
        T rv, rgrad;  // test value flux, and the factor of row d of K for the test gradient
        if (has[s]) {
          const T* fn = fb + (4 * s + 1) * L;
          T na = T(0), nbt = T(0);
#pragma unroll
          for (int j = 0; j < P; ++j) {
            na = fma(tD[ta * P + j], fn[j + P * tb], na);
            nbt = fma(tD[tb * P + j], fn[ta + P * j], nbt);
          }
          T h[3];
          h[DIR] = Nn[s] * hd_inv;
          h[DA] = na * ha_inv;
          h[DB] = nbt * hb_inv;
          const T xh = xF[0] * h[0] + xF[1] * h[1] + xF[2] * h[2];
          const T qn = kx_row(xF, DIR, xh, h[DIR]);
          const T avg = T(0.5) * (qo + qn);
          const T jump = sg * (To[s] - Tn[s]);
          rv = sg * fma(a.c_cons, avg, a.gam[DIR] * jump);
          rgrad = T(0.5) * a.c_sym * jump;
        } else {
          // Nitsche: [w] = {w} = w, outward normal sg e_d
          rv = fma(a.c_cons * sg, qo, a.gam[DIR] * To[s]);
          rgrad = a.c_sym * sg * To[s];
          if (RESIDUAL) {
            const T gD = xF[0] * xF[0] + xF[1] * xF[1] + xF[2] * xF[2];
            rv -= a.gam[DIR] * gD;
            rgrad -= a.c_sym * sg * gD;
          }
        }
        Rv[s] = wF * rv;
        Rd[s] = wF * rgrad * Kd[DIR] * hd_inv;
        Ra = wF * rgrad * Kd[DA] * ha_inv;
        Rb = wF * rgrad * Kd[DB] * hb_inv;
      }
      fb[(4 * s + 2) * L + pt] = Ra;
      fb[(4 * s + 3) * L + pt] = Rb;
    }
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      // tangential test derivatives: transposed D contractions on the face
      const T* ra = fb + (4 * s + 2) * L;
      const T* rb = fb + (4 * s + 3) * L;
      T tt = Rv[s];
#pragma unroll
      for (int j = 0; j < P; ++j) {
        tt = fma(tD[j * P + ta], ra[j + P * tb], tt);
        tt = fma(tD[j * P + tb], rb[ta + P * j], tt);
      }
#pragma unroll
      for (int i = 0; i < P; ++i) out[i] = fma(a.e[s][i], tt, fma(a.de[s][i], Rd[s], out[i]));
    }
  }
}

// y = A x (RESIDUAL = false: the Jacobian action, the u-independent terms
// dropped) or y = A x - b (RESIDUAL = true: the full residual with f and g).
template <int P, typename T, bool RESIDUAL>
__global__ void __launch_bounds__(TensorCells<P>::value * P * P)
    k_tensor_apply(const T* __restrict__ x, T* __restrict__ y, const ScalarArgs<T>* __restrict__ ap,
                   const uint32_t* __restrict__ blocks) {
  const ScalarArgs<T>& a = *ap;
  constexpr int EB = TensorCells<P>::value;
  constexpr int L = P * P, N = P * P * P;
  using Ly = Layout<P>;
  __shared__ T su[EB * Ly::NP];
  __shared__ T g0[EB * Ly::NP];  // d_0 u, then the flux component 0, then the x-line results (+= y)
  __shared__ T g1[EB * Ly::NP];  // d_1 u, then the flux component 1
  // The x-line results go where flux component 0 was: a thread writes them to
  // the positions of its own x-line, which it alone has read, and the flux is
  // not read again (one LDS array less: six blocks per CU instead of five).
  T* const sy = g0;
  __shared__ T sf[EB * 8 * L];   // face buffers
  __shared__ T tD[P * P], tW[P], tX[P];  // D, weights, nodes (reads indexed by the thread's line)

  const BlockCoord bc = block_coord(blocks);
  const int nx = a.n[0], ny = a.n[1], nz = a.n[2];
  const int ex0 = bc.ex0;
  const int nvalid = min(EB, nx - ex0);
  const uint32_t row = (uint32_t)nx * ((uint32_t)bc.ey + (uint32_t)ny * bc.ez);
  const uint32_t gbase = (row + ex0) * N;
  const int le = threadIdx.x / L;
  const int li = threadIdx.x - le * L;
  const bool active = le < nvalid;
  const int ta = li % P, tb = li / P;
  const int ex = ex0 + le;
  const uint32_t e = row + ex;
  const int cc[3] = {ex, bc.ey, bc.ez};
  if (active) load_cell_column<P, T>(su, x, gbase, le, ta, tb);
  if (threadIdx.x < P * P) tD[threadIdx.x] = a.D[threadIdx.x];
  if (threadIdx.x < P) {
    tW[threadIdx.x] = a.w[threadIdx.x];
    tX[threadIdx.x] = a.xi[threadIdx.x];
  }
  __syncthreads();
  const T* sue = su + le * Ly::NP;
  T* fb = sf + le * 8 * L;
  T vx[P], vy[P], vz[P];
  T gz[P];
  // part 1: reference derivatives along x and y to LDS, along z in registers
  if (active) {
    lds_line<P, T, 0>(sue, ta, tb, vx);
    lds_line<P, T, 1>(sue, ta, tb, vy);
    lds_line<P, T, 2>(sue, ta, tb, vz);
    T d0[P], d1[P];
#pragma unroll
    for (int q = 0; q < P; ++q) {
      T s0 = T(0), s1 = T(0), s2 = T(0);
#pragma unroll
      for (int j = 0; j < P; ++j) {
        s0 = fma(a.D[q * P + j], vx[j], s0);
        s1 = fma(a.D[q * P + j], vy[j], s1);
        s2 = fma(a.D[q * P + j], vz[j], s2);
      }
      d0[q] = s0;
      d1[q] = s1;
      gz[q] = s2;
    }
    lds_store_line<P, T, 0>(g0 + le * Ly::NP, ta, tb, d0);
    lds_store_line<P, T, 1>(g1 + le * Ly::NP, ta, tb, d1);
  }
  __syncthreads();
  // part 2: pointwise flux on the thread's z-line (i0, i1) = (ta, tb); the
  // z component stays in registers, with the mass (and source) term
  T rz[P], oz[P];
  if (active) {
    const T detJ = a.vs[0] / (a.hinv[0] * a.hinv[0]);
    const T w01 = tW[ta] * tW[tb];
    const T x0 = coord(a, ex, tX[ta], 0), x1 = coord(a, bc.ey, tX[tb], 1);
    T* g0e = g0 + le * Ly::NP + ta + Ly::S1 * tb;
    T* g1e = g1 + le * Ly::NP + ta + Ly::S1 * tb;
#pragma unroll
    for (int q = 0; q < P; ++q) {
      const T wq = w01 * a.w[q] * detJ;
      T xq[3] = {x0, x1, coord(a, bc.ez, a.xi[q], 2)};
      const T gr[3] = {g0e[q * Ly::S2] * a.hinv[0], g1e[q * Ly::S2] * a.hinv[1], gz[q] * a.hinv[2]};
      const T xg = xq[0] * gr[0] + xq[1] * gr[1] + xq[2] * gr[2];
      g0e[q * Ly::S2] = wq * kx_row(xq, 0, xg, gr[0]) * a.hinv[0];
      g1e[q * Ly::S2] = wq * kx_row(xq, 1, xg, gr[1]) * a.hinv[1];
      rz[q] = wq * kx_row(xq, 2, xg, gr[2]) * a.hinv[2];
      T m = a.cmass * (w01 * a.w[q]) * vz[q];
      if (RESIDUAL) m = fma(wq, T(6), m);  // -(f, v) with f = -6
      oz[q] = m;
    }
  }
  __syncthreads();
  // part 3 and faces, direction by direction
  T nb[2][P];
  bool has[2];
  {  // x: volume D^T of flux 0, faces normal to x; result to LDS
    T o[P];
    if (active) {
      T r[P];
      lds_line<P, T, 0>(g0 + le * Ly::NP, ta, tb, r);
#pragma unroll
      for (int i = 0; i < P; ++i) {
        T s = T(0);
#pragma unroll
        for (int q = 0; q < P; ++q) s = fma(a.D[q * P + i], r[q], s);
        o[i] = s;
      }
      neighbor_lines<P, T, 0>(su, x, e, le, nvalid, ex, nx, 1u, ta, tb, nb, has);
    }
    tensor_faces<P, T, RESIDUAL, 0>(a, active, vx, nb, has, cc, ta, tb, fb, o, tD, tW, tX);
    if (active) lds_store_line<P, T, 0>(sy + le * Ly::NP, ta, tb, o);
  }
  {  // y
    T o[P];
    if (active) {
      T r[P];
      lds_line<P, T, 1>(g1 + le * Ly::NP, ta, tb, r);
#pragma unroll
      for (int i = 0; i < P; ++i) {
        T s = T(0);
#pragma unroll
        for (int q = 0; q < P; ++q) s = fma(a.D[q * P + i], r[q], s);
        o[i] = s;
      }
      neighbor_lines<P, T, 1>(su, x, e, le, nvalid, bc.ey, ny, (uint32_t)nx, ta, tb, nb, has);
    }
    // the faces synchronize before the update below, after the x results are stored
    tensor_faces<P, T, RESIDUAL, 1>(a, active, vy, nb, has, cc, ta, tb, fb, o, tD, tW, tX);
    if (active) {
#pragma unroll
      for (int i = 0; i < P; ++i) sy[le * Ly::NP + ta + Ly::S1 * i + Ly::S2 * tb] += o[i];
    }
  }
  {  // z: registers, then the final sum
    if (active) {
#pragma unroll
      for (int i = 0; i < P; ++i) {
        T s = oz[i];
#pragma unroll
        for (int q = 0; q < P; ++q) s = fma(a.D[q * P + i], rz[q], s);
        oz[i] = s;
      }
      neighbor_lines<P, T, 2>(su, x, e, le, nvalid, bc.ez, nz, (uint32_t)nx * ny, ta, tb, nb, has);
    }
    tensor_faces<P, T, RESIDUAL, 2>(a, active, vz, nb, has, cc, ta, tb, fb, oz, tD, tW, tX);
    if (active) {
      const int lo = le * Ly::NP + ta + Ly::S1 * tb;
      T* __restrict__ ye = y + e * N + ta + P * tb;
#pragma unroll
      for (int j = 0; j < P; ++j) ye[j * L] = sy[lo + j * Ly::S2] + oz[j];
    }
  }
}

template <int P, typename T>
hipError_t launch_tensor(const dg_mesh& M, int variant, const T* x, T* y, bool residual, hipStream_t s) {
  constexpr int EB = TensorCells<P>::value;
  const ScalarArgs<double>& h = M.pd[variant];
  const int64_t G = (int64_t)((h.n[0] + EB - 1) / EB) * h.n[1] * h.n[2];
  // the sweep table of the 128-thread grid (chunks of 128 / p^2 cells)
  const uint32_t* blocks = M.pd[SP_ADJOINT].blocks;
  if (G > 0x7fffffff || M.ndofs > 0xffffffffLL || !blocks || G != tensor_grid(M)) return hipErrorInvalidValue;
  const ScalarArgs<T>* ap;
  if constexpr (sizeof(T) == 8) ap = M.d_pd + variant;
  else ap = M.d_pf + variant;
  if (residual)
    hipLaunchKernelGGL((k_tensor_apply<P, T, true>), dim3((unsigned)G), dim3(EB * P * P), 0, s, x, y, ap, blocks);
  else
    hipLaunchKernelGGL((k_tensor_apply<P, T, false>), dim3((unsigned)G), dim3(EB * P * P), 0, s, x, y, ap, blocks);
  return hipGetLastError();
}

template <typename T>
hipError_t dispatch_tensor(const dg_mesh& M, int variant, const T* x, T* y, bool residual, hipStream_t s) {
  switch (M.p) {
    case 2: return launch_tensor<2, T>(M, variant, x, y, residual, s);
    case 3: return launch_tensor<3, T>(M, variant, x, y, residual, s);
    case 4: return launch_tensor<4, T>(M, variant, x, y, residual, s);
    case 5: return launch_tensor<5, T>(M, variant, x, y, residual, s);
    case 6: return launch_tensor<6, T>(M, variant, x, y, residual, s);
    case 7: return launch_tensor<7, T>(M, variant, x, y, residual, s);
    case 8: return launch_tensor<8, T>(M, variant, x, y, residual, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t tensor_apply(const dg_mesh& M, int prec, const void* x, void* y, bool transpose, bool residual,
                        hipStream_t s) {
  const int v = transpose ? SP_APPLY_T : SP_APPLY;
  if (prec == DG_F64) return dispatch_tensor<double>(M, v, (const double*)x, (double*)y, residual, s);
  return dispatch_tensor<float>(M, v, (const float*)x, (float*)y, residual, s);
}

}  // namespace dgi
