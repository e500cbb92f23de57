// The nonlinear SIPG diffusion operator -div(kappa(u) grad u) + c u with
// kappa(u) = 1 + u^2 on axis-aligned cells (gfx950): its residual R(u) and
// the Jacobian action J(u0) z at a linearization point u0 (Section 2.1: for a
// nonlinear problem the action depends on the linearization point as well as
// on the direction).
//
// Residual (eq. diffreac_weak's SIPG form with the coefficient evaluated at
// the solution; homogeneous Dirichlet data on the masked sides):
//   (kappa(u) grad u, grad v) + (c u, v)
//   + sum_F -({kappa(u) grad u}.n, [v]) + theta ([u], {kappa(u) grad v}.n) + gamma ([u], [v]),
// with kappa on a face from each side's own trace of u. Jacobian action:
//   (kappa(u0) grad z + kappa'(u0) z grad u0, grad v) + (c z, v)
//   + sum_F -({kappa(u0) grad z + kappa'(u0) z grad u0}.n, [v])
//           + theta ([z], {kappa(u0) grad v}.n) + theta ([u0], {kappa'(u0) z grad v}.n)
//           + gamma ([z], [v]).
//
// Two-input fused evaluation (Section 3.1: kernels that evaluate both the
// solution and the linearization point): every 1D line of u0 and of z is
// contracted in the same thread, so the reference derivatives of both, the
// pointwise kappa(u0), kappa'(u0) and the face traces of both inputs come
// out of one pass over the two vectors. With the collocated Gauss-Legendre
// basis and J = diag(h), the volume term of direction d on a line is
//   D^T [ w |J| / h_d^2 (kappa(u0) D z + kappa'(u0) z D u0) ],
// and the faces normal to d sit at the two ends of the d-lines (normal
// direction contracted first): the own traces and outward normal
// derivatives of u0 and z, and the neighbour's from its matching line, give
// the flux per face point, tested with the own trace row and normal
// derivative row only (element-centric: one writer per output, no atomics).
// Threads own lines (p^2 per cell, x- then y- then z-lines) in chunks of up
// to 128 / p^2 consecutive cells of one x-row (the adjoint's sweep grid).
#include "line_common.h"

namespace dgi {
namespace {

template <int P>
struct NlCells {
  static constexpr int value = (128 / (P * P)) > 0 ? (128 / (P * P)) : 1;
};

// One d-line: volume and both faces of direction DIR, without the line's
// tangential weight. JAC: J(u0) z with v0 = u0's line and vz = z's line;
// otherwise R(u) with v0 = u's line (vz unused). n0[s], nz[s]: the
// neighbour's matching lines across side s (zero where there is none).
template <int P, typename T, bool JAC, int DIR>
__device__ __forceinline__ void nl_line(const T* v0, const T* vz, const T (*n0)[P], const T (*nz)[P],
                                        const bool* has, const ScalarArgs<T>& a, bool mass, T* out) {
  // volume: reference derivatives of both inputs at the points
  T fl[P];
  const T vs = a.vs[DIR];
#pragma unroll
  for (int q = 0; q < P; ++q) {
    T du = T(0), dz = T(0);
#pragma unroll
    for (int j = 0; j < P; ++j) {
      du = fma(a.D[q * P + j], v0[j], du);
      if (JAC) dz = fma(a.D[q * P + j], vz[j], dz);
    }
    const T u = v0[q];
    const T k = fma(u, u, T(1));
    const T wq = vs * a.w[q];
    fl[q] = JAC ? wq * fma(k, dz, (T(2) * u) * vz[q] * du) : wq * k * du;
  }
#pragma unroll
  for (int i = 0; i < P; ++i) {
    T s = mass ? a.cmass * a.w[i] * (JAC ? vz[i] : v0[i]) : T(0);
#pragma unroll
    for (int q = 0; q < P; ++q) s = fma(a.D[q * P + i], fl[q], s);
    out[i] = s;
  }
  // faces normal to DIR at both ends of the line
  const T hinv = a.hinv[DIR], fs = a.fs[DIR], gam = a.gam[DIR], th = a.c_sym;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const bool dirichlet = (a.mask >> (2 * DIR + s)) & 1u;
    if (!has[s] && !dirichlet) continue;
    const T sg = s ? T(1) : T(-1);  // outward normal sg e_d
    const T dsc = sg * hinv;        // reference derivative row -> outward normal derivative
    T uT = T(0), duT = T(0), zT = T(0), dzT = T(0);
#pragma unroll
    for (int j = 0; j < P; ++j) {
      uT = fma(a.e[s][j], v0[j], uT);
      duT = fma(a.de[s][j], v0[j], duT);
      if (JAC) {
        zT = fma(a.e[s][j], vz[j], zT);
        dzT = fma(a.de[s][j], vz[j], dzT);
      }
    }
    duT *= dsc;
    dzT *= dsc;
    const T kT = fma(uT, uT, T(1)), kpT = T(2) * uT;
    T cE, cD;  // coefficients of the own trace row and of the own outward normal derivative row
    if (has[s]) {
      // the neighbour meets this face with its side 1 - s; derivatives along the same outward normal
      T uN = T(0), duN = T(0), zN = T(0), dzN = T(0);
#pragma unroll
      for (int j = 0; j < P; ++j) {
        uN = fma(a.e[1 - s][j], n0[s][j], uN);
        duN = fma(a.de[1 - s][j], n0[s][j], duN);
        if (JAC) {
          zN = fma(a.e[1 - s][j], nz[s][j], zN);
          dzN = fma(a.de[1 - s][j], nz[s][j], dzN);
        }
      }
      duN *= dsc;
      dzN *= dsc;
      const T kN = fma(uN, uN, T(1));
      const T ju = uT - uN;
      if (JAC) {
        const T kpN = T(2) * uN;
        const T flux = T(0.5) * (fma(kT, dzT, kpT * zT * duT) + fma(kN, dzN, kpN * zN * duN));
        const T jz = zT - zN;
        cE = fma(gam, jz, -flux);
        cD = th * T(0.5) * fma(kT, jz, kpT * zT * ju);
      } else {
        const T flux = T(0.5) * fma(kT, duT, kN * duN);
        cE = fma(gam, ju, -flux);
        cD = th * T(0.5) * kT * ju;
      }
    } else {  // Dirichlet side, data 0: [w] = {w} = w
      if (JAC) {
        cE = fma(gam, zT, -fma(kT, dzT, kpT * zT * duT));
        cD = th * zT * fma(kpT, uT, kT);
      } else {
        cE = fma(gam, uT, -kT * duT);
        cD = th * kT * uT;
      }
    }
    cE *= fs;
    cD *= fs * dsc;
#pragma unroll
    for (int i = 0; i < P; ++i) out[i] = fma(cE, a.e[s][i], fma(cD, a.de[s][i], out[i]));
  }
}

template <int P, typename T, bool JAC, int DIR>
__device__ __forceinline__ void nl_direction(const T* su, const T* sz, const T* u0, const T* z, uint32_t e, int le,
                                             int nvalid, int ecd, int nd, uint32_t estride, int ta, int tb,
                                             const ScalarArgs<T>& a, T* out) {
  using Ly = Layout<P>;
  T v0[P], vz[P], n0[2][P], nz[2][P];
  bool has[2];
  lds_line<P, T, DIR>(su + le * Ly::NP, ta, tb, v0);
  neighbor_lines<P, T, DIR>(su, u0, e, le, nvalid, ecd, nd, estride, ta, tb, n0, has);
  if (JAC) {
    lds_line<P, T, DIR>(sz + le * Ly::NP, ta, tb, vz);
    neighbor_lines<P, T, DIR>(sz, z, e, le, nvalid, ecd, nd, estride, ta, tb, nz, has);
  }
  nl_line<P, T, JAC, DIR>(v0, vz, n0, nz, has, a, DIR == 0, out);
}

// y = J(u0) z (JAC) or y = R(u0) (z unused).
template <int P, typename T, bool JAC>
__global__ void __launch_bounds__(NlCells<P>::value * P * P)
    k_nonlinear(const T* __restrict__ u0, const T* __restrict__ z, T* __restrict__ y,
                const ScalarArgs<T>* __restrict__ ap, const uint32_t* __restrict__ blocks) {
  const ScalarArgs<T>& a = *ap;
  constexpr int EB = NlCells<P>::value;
  constexpr int L = P * P, N = P * P * P;
  using Ly = Layout<P>;
  __shared__ T su[EB * Ly::NP];
  __shared__ T sz[JAC ? EB * Ly::NP : 1];
  __shared__ T sy[EB * Ly::NP];

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
  if (active) {
    load_cell_column<P, T>(su, u0, gbase, le, ta, tb);
    if (JAC) load_cell_column<P, T>(sz, z, gbase, le, ta, tb);
  }
  __syncthreads();
  const T wt = a.wl[li];
  T o1[P], o2[P];
  if (active) {
    T o0[P];
    nl_direction<P, T, JAC, 0>(su, sz, u0, z, e, le, nvalid, ex, nx, 1u, ta, tb, a, o0);
    nl_direction<P, T, JAC, 1>(su, sz, u0, z, e, le, nvalid, bc.ey, ny, (uint32_t)nx, ta, tb, a, o1);
#pragma unroll
    for (int i = 0; i < P; ++i) sy[le * Ly::NP + i + Ly::S1 * ta + Ly::S2 * tb] = wt * o0[i];
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int i = 0; i < P; ++i) {
      T* yi = sy + le * Ly::NP + ta + Ly::S1 * i + Ly::S2 * tb;
      *yi = fma(wt, o1[i], *yi);
    }
    nl_direction<P, T, JAC, 2>(su, sz, u0, z, e, le, nvalid, bc.ez, nz, (uint32_t)nx * ny, ta, tb, a, o2);
  }
  __syncthreads();
  if (active) {
    const int lo = le * Ly::NP + ta + Ly::S1 * tb;
    T* __restrict__ ye = y + e * N + ta + P * tb;
#pragma unroll
    for (int j = 0; j < P; ++j) ye[j * L] = fma(wt, o2[j], sy[lo + j * Ly::S2]);
  }
}

template <int P, typename T>
hipError_t launch_nonlinear(const dg_mesh& M, const T* u0, const T* z, T* y, bool jac, hipStream_t s) {
  constexpr int EB = NlCells<P>::value;
  const ScalarArgs<double>& h = M.pd[SP_ADJOINT];
  const int64_t G = (int64_t)((h.n[0] + EB - 1) / EB) * h.n[1] * h.n[2];
  // the sweep table of the 128-thread grid (chunks of 128 / p^2 cells)
  const uint32_t* blocks = h.blocks;
  if (G > 0x7fffffff || M.ndofs > 0xffffffffLL || !blocks || G != (int64_t)h.nchunk * h.n[1] * h.n[2])
    return hipErrorInvalidValue;
  const ScalarArgs<T>* ap;
  if constexpr (sizeof(T) == 8) ap = M.d_pd + SP_APPLY;
  else ap = M.d_pf + SP_APPLY;
  if (jac)
    hipLaunchKernelGGL((k_nonlinear<P, T, true>), dim3((unsigned)G), dim3(EB * P * P), 0, s, u0, z, y, ap, blocks);
  else
    hipLaunchKernelGGL((k_nonlinear<P, T, false>), dim3((unsigned)G), dim3(EB * P * P), 0, s, u0, z, y, ap, blocks);
  return hipGetLastError();
}

template <typename T>
hipError_t dispatch_nonlinear(const dg_mesh& M, const T* u0, const T* z, T* y, bool jac, hipStream_t s) {
  switch (M.p) {
    case 2: return launch_nonlinear<2, T>(M, u0, z, y, jac, s);
    case 3: return launch_nonlinear<3, T>(M, u0, z, y, jac, s);
    case 4: return launch_nonlinear<4, T>(M, u0, z, y, jac, s);
    case 5: return launch_nonlinear<5, T>(M, u0, z, y, jac, s);
    case 6: return launch_nonlinear<6, T>(M, u0, z, y, jac, s);
    case 7: return launch_nonlinear<7, T>(M, u0, z, y, jac, s);
    case 8: return launch_nonlinear<8, T>(M, u0, z, y, jac, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t nonlinear_apply(const dg_mesh& M, int prec, const void* u0, const void* z, void* y, bool jac,
                           hipStream_t s) {
  if (prec == DG_F64) return dispatch_nonlinear<double>(M, (const double*)u0, (const double*)z, (double*)y, jac, s);
  return dispatch_nonlinear<float>(M, (const float*)u0, (const float*)z, (float*)y, jac, s);
}

}  // namespace dgi
