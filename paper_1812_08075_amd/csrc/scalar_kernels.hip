// Sum-factorized SIPG diffusion-reaction operator on axis-aligned hexahedra
// (gfx950).
//
// Operator (Section 5.2, eq. diffreac_weak, linear part; Jacobian action of
// Section 2.1): cell terms (kappa grad u, grad v) + (c u, v); on every interior
// face -({kappa grad u}.n, [v]) + theta ([u], {kappa grad v}.n) +
// gamma_F ([u], [v]); on Dirichlet sides the same with [w] = {w} = w.
//
// Design.
//  * Collocation: the nodal basis lives at the m = p Gauss-Legendre points, so
//    the basis matrix A of Section 2.2 is the identity and each derivative
//    is one 1D contraction with D along its direction (Algorithm 1, part 1);
//    the quadrature loop (part 2) is pointwise and the test-function
//    contraction (part 3) is D^T along the same direction.
//  * On axis-aligned cells J = diag(h), so the pointwise stage of direction d
//    only needs d_d u: kappa w |J| / h_d^2 * d_d u. Contraction, quadrature
//    and transposed contraction of one direction therefore run on one 1D
//    line of p values in one thread, with D from a device-resident parameter
//    block (wave-uniform scalar operands). A cell is handled by p^2 threads that
//    own, in turn, its p^2 lines along x, along y and along z.
//  * Faces normal to d (Section 2.2, m_d = 1, normal direction contracted
//    first) sit at the two ends of every d-line: the own trace u and its
//    normal derivative are dot products of the line with the rows
//    l_j(s), l_j'(s); the neighbour's trace comes from the neighbour's
//    matching line. The flux is formed per face point and multiplied back
//    with the same rows onto the own line only. Each face is thus evaluated
//    by both its cells (element-centric): every output value has exactly one
//    writer, there are no atomics, and results are bitwise reproducible.
//  * With kappa = 1 in FP64 the three stages of a direction and both face
//    terms are applied as fixed 1D line operators, out = K u + L u_left +
//    R u_right (K in even/odd form, L and R of rank 2; built on the host);
//    FP32 and kappa per point run the stages as above.
//  * A block is a chunk of up to EB consecutive cells of one x-row, so its
//    cells are contiguous in memory: each thread copies its own node column
//    of its cell into LDS (one load per z-plane, the lanes of a cell reading
//    one contiguous plane), and x-neighbours inside the chunk are read from
//    LDS. Each XCD sweeps one region of the mesh (x and z split to read the
//    fewest cells across region boundaries, y unsplit; inside a region y
//    outermost, then z, then x), so the y- and z-neighbour lines a block
//    reads were loaded shortly before by another block of the same XCD and
//    are served by its L2: HBM sees about one read of x (plus kappa) and one
//    write of y, plus the region boundaries.
//  * The x and y line results go through LDS (padded strides against bank
//    conflicts), the z line stays in registers; the sum is written once.
//  * The same kernel applies A^T: swapping the coefficients of the two
//    non-symmetric face terms (consistency term and theta term) transposes
//    the face bilinear form; the cell terms are symmetric. A template variant
//    also reduces x.y per block (the p.Ap of the conjugate-gradient solvers).
//  * Also here: the adjoint (A^T g and dL/dkappa in one pass), the
//    block-Jacobi preconditioner (each cell's diagonal block inverted by fast
//    diagonalization) and the load vector.
#include "line_common.h"

namespace dgi {
namespace {

template <int P>
struct CellsPerBlock {
  // about 256 threads per block, p^2 threads per cell
  static constexpr int value = (256 / (P * P)) > 0 ? (256 / (P * P)) : 1;
};

template <int P>
struct AdjCellsPerBlock {
  static constexpr int value = (128 / (P * P)) > 0 ? (128 / (P * P)) : 1;
};

// Face fluxes of the two ends of a d-line (general form): Rv[s] multiplies
// the trace row of side s, Sd[s] (times fB0) its derivative row.
template <int P, typename T, bool KAPPA, int DIR>
__device__ __forceinline__ void face_fluxes(const T* v, const T* kv, const T (*nb)[P], const T (*nk)[P],
                                            const bool* has_nb, const ScalarArgs<T>& a, T* Rv, T* Sd) {
  const EvenOdd<T>& dv = a.eo[DIR];
  // own traces and reference-coordinate derivatives at both ends: side 1 uses
  // the mirror image of the side-0 rows (the derivative row with a sign). They
  // are formed exactly as the neighbour across that face forms them (same rows,
  // same order), so both cells see bitwise the same face values and the
  // discrete operator stays symmetric in floating point (theta = -1).
  T uT[2] = {T(0), T(0)}, dT[2] = {T(0), T(0)};
#pragma unroll
  for (int j = 0; j < P; ++j) {
    uT[0] = fma(a.e[0][j], v[j], uT[0]);
    dT[0] = fma(a.de[0][j], v[j], dT[0]);
    uT[1] = fma(a.e[0][P - 1 - j], v[j], uT[1]);
    dT[1] = fma(a.de[0][P - 1 - j], v[j], dT[1]);
  }
  // (outward normal derivative = -(1/h) dT; the -1/h sits in fAh)
  const bool face_kappa = KAPPA && !a.kappa_face_one;
  T kT[2] = {T(1), T(1)};
  if (face_kappa) {
    kT[0] = kT[1] = T(0);
#pragma unroll
    for (int j = 0; j < P; ++j) {
      kT[0] = fma(a.e[0][j], kv[j], kT[0]);
      kT[1] = fma(a.e[0][P - 1 - j], kv[j], kT[1]);
    }
  }
  // face fluxes: Rv multiplies the trace row of side s, Sd (times fB0) its derivative row
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const bool dirichlet = (a.mask >> (2 * DIR + s)) & 1u;
    // the neighbour across side s meets it with its own side 1-s: trace row
    // e0 mirrored for s = 0, e0 for s = 1; derivative row likewise (no branch:
    // the neighbour line is zero where there is none)
    T uN = T(0), dN = T(0), kN = T(1);
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const int r = s == 0 ? P - 1 - j : j;
      uN = fma(a.e[0][r], nb[s][j], uN);
      dN = fma(a.de[0][r], nb[s][j], dN);
    }
    if (face_kappa) {
      kN = T(0);
#pragma unroll
      for (int j = 0; j < P; ++j) kN = fma(a.e[0][s == 0 ? P - 1 - j : j], nk[s][j], kN);
    }
    // interior: averages and jumps; Dirichlet: the one-sided terms count twice
    const T sel = has_nb[s] ? T(1) : (dirichlet ? T(2) : T(0));
    const T g = (has_nb[s] || dirichlet) ? dv.fG : T(0);
    const T jump = uT[s] - uN;
    Rv[s] = fma(sel * dv.fAh, kT[s] * dT[s] - kN * dN, g * jump);
    Sd[s] = sel * (kT[s] * jump);
  }
}

// Volume and face work of one 1D line of one cell in direction DIR, without
// the line's tangential quadrature weight w_a w_b, which the caller applies once.
//  v, kv: the line's values and kappa at its nodes; nb[s], nk[s]: the
//  neighbour's matching line across side s (zero where there is none);
//  mass: add the c |J| w u term (once per cell, on the x lines).
// The line is split into its even and odd parts about the cell centre (the
// even-odd tables of ScalarArgs): the contractions with D and D^T and the
// traces at both ends then each cost about half the multiplications.
template <int P, typename T, bool KAPPA, int DIR>
__device__ __forceinline__ void line_apply(const T* v, const T* kv, const T (*nb)[P], const T (*nk)[P],
                                           const bool* has_nb, const ScalarArgs<T>& a, bool mass, T* out) {
  constexpr int H = P / 2;
  constexpr bool ODD = (P & 1) != 0;
  const EvenOdd<T>& dv = a.eo[DIR];
  T ve[H], vo[H];
#pragma unroll
  for (int j = 0; j < H; ++j) {
    ve[j] = v[j] + v[P - 1 - j];
    vo[j] = v[j] - v[P - 1 - j];
  }
  const T vm = ODD ? v[H] : T(0);
  // cell: d = (|J|/h^2) w D v at the points, as d_q = se_q + so_q,
  // d_{p-1-q} = so_q - se_q (q < H) and the middle value dm
  T se[H], so[H];
#pragma unroll
  for (int q = 0; q < H; ++q) {
    T s0 = ODD ? dv.DvC[q] * vm : T(0), s1 = T(0);
#pragma unroll
    for (int j = 0; j < H; ++j) {
      s0 = fma(dv.DvP[q * H + j], ve[j], s0);
      s1 = fma(dv.DvM[q * H + j], vo[j], s1);
    }
    se[q] = s0;
    so[q] = s1;
  }
  T dm = T(0);
  if (ODD) {
#pragma unroll
    for (int j = 0; j < H; ++j) dm = fma(dv.DvR[j], vo[j], dm);
  }
  // r = kappa d as half sums re and half differences ro over mirrored points
  T re[H], ro[H], rm;
  T ks[H], kd[H];  // kappa_j + kappa_{p-1-j}, kappa_j - kappa_{p-1-j}
  if (KAPPA) {
#pragma unroll
    for (int q = 0; q < H; ++q) {
      ks[q] = kv[q] + kv[P - 1 - q];
      kd[q] = kv[q] - kv[P - 1 - q];
      const T ke = T(0.5) * ks[q], ko = T(0.5) * kd[q];
      re[q] = fma(ko, se[q], ke * so[q]);
      ro[q] = fma(ke, se[q], ko * so[q]);
    }
    rm = ODD ? kv[H] * dm : T(0);
  } else {
#pragma unroll
    for (int q = 0; q < H; ++q) {
      re[q] = so[q];
      ro[q] = se[q];
    }
    rm = dm;
  }
  // out = D^T r (+ mass) accumulated as half sums oe and half differences oo
  T oe[H], oo[H];
#pragma unroll
  for (int i = 0; i < H; ++i) {
    T t0 = mass ? a.cwh[i] * ve[i] : T(0);
    T t1 = mass ? a.cwh[i] * vo[i] : T(0);
#pragma unroll
    for (int q = 0; q < H; ++q) {
      t0 = fma(a.G2p[i * H + q], ro[q], t0);
      t1 = fma(a.G2m[i * H + q], re[q], t1);
    }
    if (ODD) t1 = fma(a.Gh[i], rm, t1);
    oe[i] = t0;
    oo[i] = t1;
  }
  T om = T(0);
  if (ODD) {
    om = mass ? a.cwm * vm : T(0);
#pragma unroll
    for (int q = 0; q < H; ++q) om = fma(a.G2c[q], ro[q], om);
  }
  T Rv[2], Sd[2];
  face_fluxes<P, T, KAPPA, DIR>(v, kv, nb, nk, has_nb, a, Rv, Sd);
  const T cE = Rv[0] + Rv[1], cO = Rv[0] - Rv[1];
  const T dE = dv.fB0 * (Sd[0] + Sd[1]), dO = dv.fB0 * (Sd[0] - Sd[1]);
#pragma unroll
  for (int i = 0; i < H; ++i) {
    oe[i] = fma(cE, a.Ep[i], fma(dE, a.DEp[i], oe[i]));
    oo[i] = fma(cO, a.Em[i], fma(dO, a.DEm[i], oo[i]));
  }
  if (ODD) om = fma(cE, a.Eh, fma(dE, a.DEh, om));
#pragma unroll
  for (int i = 0; i < H; ++i) {
    out[i] = oe[i] + oo[i];
    out[P - 1 - i] = oe[i] - oo[i];
  }
  if (ODD) out[H] = om;
}

// kappa = 1: the line's result is K u + L u_left + R u_right with the 1D
// line operators of ScalarArgs::lo (volume, mass for the x lines, and the
// SIPG face terms of both ends, built on the host). The interior K is
// centro-symmetric and applied in even/odd form; L and R have rank 2 (the
// neighbour's trace and normal derivative at the shared face), and a boundary
// side adds a rank-2 correction of K. The neighbour line is zero where there
// is none; the tangential weight is applied by the caller.
template <int P, typename T, int DIR>
__device__ __forceinline__ void line_apply_const(const T* v, const T (*nb)[P], const bool* has_nb,
                                                 const ScalarArgs<T>& a, T* out) {
  constexpr int H = P / 2;
  constexpr bool ODD = (P & 1) != 0;
  const LineOp<T>& o = a.lo[DIR];
  T ve[H], vo[H];
#pragma unroll
  for (int j = 0; j < H; ++j) {
    ve[j] = v[j] + v[P - 1 - j];
    vo[j] = v[j] - v[P - 1 - j];
  }
  const T vm = ODD ? v[H] : T(0);
  T oe[H], oo[H];
#pragma unroll
  for (int i = 0; i < H; ++i) {
    T t0 = ODD ? o.Kc[i] * vm : T(0), t1 = T(0);
#pragma unroll
    for (int j = 0; j < H; ++j) {
      t0 = fma(o.Kp[i * H + j], ve[j], t0);
      t1 = fma(o.Km[i * H + j], vo[j], t1);
    }
    oe[i] = t0;
    oo[i] = t1;
  }
  T om = T(0);
  if (ODD) {
    om = o.Kh * vm;
#pragma unroll
    for (int j = 0; j < H; ++j) om = fma(o.Kr[j], ve[j], om);
  }
  // coefficients of e0, de0 (side 0) and e1, de1 (side 1)
  T A0 = T(0), B0 = T(0), A1 = T(0), B1 = T(0);
#pragma unroll
  for (int j = 0; j < P; ++j) {
    A0 = fma(o.la[j], nb[0][j], A0);
    B0 = fma(o.lb[j], nb[0][j], B0);
    A1 = fma(o.la[P - 1 - j], nb[1][j], A1);
    B1 = fma(o.lb[P - 1 - j], nb[1][j], B1);
  }
  B1 = -B1;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    if (!has_nb[s]) {
      const int t = ((a.mask >> (2 * DIR + s)) & 1u) ? 0 : 1;
      T ev = T(0), dv = T(0);
#pragma unroll
      for (int j = 0; j < P; ++j) {
        const int r = s ? P - 1 - j : j;
        ev = fma(a.e[0][r], v[j], ev);
        dv = fma(a.de[0][r], v[j], dv);
      }
      if (s) dv = -dv;
      const T q1 = fma(o.bq[t][s][0], dv, o.bq[t][s][1] * ev), q2 = o.bq[t][s][2] * ev;
      if (s == 0) {
        A0 += q1;
        B0 += q2;
      } else {
        A1 += q1;
        B1 += q2;
      }
    }
  }
  const T cE = A0 + A1, cO = A0 - A1, dE = B0 - B1, dO = B0 + B1;
#pragma unroll
  for (int i = 0; i < H; ++i) {
    oe[i] = fma(cE, a.Ep[i], fma(dE, a.DEp[i], oe[i]));
    oo[i] = fma(cO, a.Em[i], fma(dO, a.DEm[i], oo[i]));
  }
  if (ODD) om = fma(cE, a.Eh, fma(dE, a.DEh, om));
#pragma unroll
  for (int i = 0; i < H; ++i) {
    out[i] = oe[i] + oo[i];
    out[P - 1 - i] = oe[i] - oo[i];
  }
  if (ODD) out[H] = om;
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 lines of p = 4 nodes on the matrix cores: v_mfma_f32_4x4x1_16b_f32
// computes, for each group of four lanes (a block), the outer product of the
// A values of its lanes (row i = lane % 4) and the B values (column j =
// lane % 4) into VGPR i of lane j. With B the lane's own line value k and A
// the table entry (lane % 4, k), four products accumulate sum_k T[i][k] v_k,
// i.e. the lane's own line times the 4 x 4 table, node i in VGPR i: a
// thread-per-line contraction with FP32 products and FP32 accumulation. The
// caller keeps the control flow uniform (the instruction works on all 64
// lanes). A[k] holds the lane's table entries, loaded once per thread.
__device__ __forceinline__ f32x4 mfma_line4(const float* A, const float* v) {
  f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int k = 0; k < 4; ++k) acc = __builtin_amdgcn_mfma_f32_4x4x1f32(A[k], v[k], acc, 0, 0, 0);
  return acc;
}

// Algorithm 1 on an FP32 line of p = 4 nodes with the two contractions on
// the matrix cores (the general form of line_apply: D contraction, the
// quadrature scaling w_q |J| / h_d^2 and pointwise kappa, D^T contraction,
// mass on the x-lines) and the same face fluxes as line_apply. AD[k] =
// D[lane % 4][k], ADt[k] = D[k][lane % 4]: the same for every direction.
template <bool KAPPA, int DIR>
__device__ __forceinline__ void line_apply_mfma4(const float* v, const float* kv, const float (*nb)[4],
                                                 const float (*nk)[4], const bool* has_nb,
                                                 const ScalarArgs<float>& a, bool mass, const float* AD,
                                                 const float* ADt, float* out) {
  constexpr int P = 4;
  const f32x4 d = mfma_line4(AD, v);
  const float vs = a.vs[DIR];
  float r[P] = {d.x * (vs * a.w[0]), d.y * (vs * a.w[1]), d.z * (vs * a.w[2]), d.w * (vs * a.w[3])};
  if (KAPPA) {
#pragma unroll
    for (int q = 0; q < P; ++q) r[q] *= kv[q];
  }
  const f32x4 o = mfma_line4(ADt, r);
  out[0] = o.x;
  out[1] = o.y;
  out[2] = o.z;
  out[3] = o.w;
  if (mass) {
#pragma unroll
    for (int i = 0; i < P; ++i) out[i] = fma(a.cw[i], v[i], out[i]);
  }
  float Rv[2], Sd[2];
  face_fluxes<P, float, KAPPA, DIR>(v, kv, nb, nk, has_nb, a, Rv, Sd);
  const float fB0 = a.eo[DIR].fB0;
#pragma unroll
  for (int i = 0; i < P; ++i) {
    const float t = fma(Rv[0], a.e[0][i], Rv[1] * a.e[0][P - 1 - i]);
    out[i] += fma(fB0 * Sd[0], a.de[0][i], fma(fB0 * Sd[1], a.de[0][P - 1 - i], t));
  }
}

// The line work of direction DIR: line operators for kappa = 1 in FP64, the
// general form otherwise (FP32 keeps the form whose face values are bitwise
// the same on both sides of a face); MC: FP32 lines of p = 4 with the
// contractions on the matrix cores.
template <int P, typename T, bool KAPPA, int DIR, bool MC>
__device__ __forceinline__ void line_work(const T* v, const T* kv, const T (*nb)[P], const T (*nk)[P],
                                          const bool* has_nb, const ScalarArgs<T>& a, bool mass, const T* AD,
                                          const T* ADt, T* out) {
  if constexpr (!KAPPA && sizeof(T) == 8) {
    line_apply_const<P, T, DIR>(v, nb, has_nb, a, out);
  } else if constexpr (MC) {
    static_assert(P == 4 && sizeof(T) == 4, "matrix-core lines: FP32, p = 4");
    line_apply_mfma4<KAPPA, DIR>(v, kv, nb, nk, has_nb, a, mass, AD, ADt, out);
  } else {
    line_apply<P, T, KAPPA, DIR>(v, kv, nb, nk, has_nb, a, mass, out);
  }
}

// ---------------------------------------------------------------------------
// Block-Jacobi preconditioner: z = B_T^-1 r on every cell T, B_T the diagonal
// block of the operator, by fast diagonalization (tables in
// ScalarArgs::fdmV, fdmL): the transposed eigenvector contractions along z,
// y and x, the division by lam_x + lam_y + lam_z on the x-lines, and the
// eigenvector contractions back along x, y and z. No neighbour data.

// side-type variant 3 t0 + t1 of a cell at position c of n along direction d
__device__ __forceinline__ int fdm_variant(int c, int n, uint32_t mask, int d) {
  const int t0 = c > 0 ? 0 : ((mask >> (2 * d)) & 1u ? 1 : 2);
  const int t1 = c < n - 1 ? 0 : ((mask >> (2 * d + 1)) & 1u ? 1 : 2);
  return 3 * t0 + t1;
}

// o = V^T v
template <int P, typename T>
__device__ __forceinline__ void fdm_forward(const T* __restrict__ V, const T* v, T* o) {
#pragma unroll
  for (int i = 0; i < P; ++i) {
    T acc = T(0);
#pragma unroll
    for (int j = 0; j < P; ++j) acc = fma(V[j * P + i], v[j], acc);
    o[i] = acc;
  }
}

// o = V t
template <int P, typename T>
__device__ __forceinline__ void fdm_backward(const T* __restrict__ V, const T* t, T* o) {
#pragma unroll
  for (int i = 0; i < P; ++i) {
    T acc = T(0);
#pragma unroll
    for (int j = 0; j < P; ++j) acc = fma(V[i * P + j], t[j], acc);
    o[i] = acc;
  }
}

// The x-line part of one cell with the tables (V, lam) of its x variant:
// forward, divide by lam_x + lam_y + lam_z, backward.
template <int P, typename T>
__device__ __forceinline__ void fdm_x(const T* V, const T* lam, T lyz, T* v) {
  T o[P];
  fdm_forward<P, T>(V, v, o);
#pragma unroll
  for (int j = 0; j < P; ++j) o[j] = o[j] / (lam[j] + lyz);
  fdm_backward<P, T>(V, o, v);
}

// Side-type variants of a block's cells for the preconditioner tables: y and
// z are block-uniform, x differs for the first and last cells of a row; the
// block's three possible x tables (its first cell's, the interior one, its
// last cell's) are staged in LDS.
struct FdmVariants {
  int vx, vy, vz, vfirst, vlast;
};

template <int P, typename T>
__device__ __forceinline__ FdmVariants fdm_setup(const ScalarArgs<T>& a, const BlockCoord& bc, int nvalid, int le,
                                                 T* sV, T* sL) {
  constexpr int L = P * P;
  const int nx = a.n[0], ny = a.n[1], nz = a.n[2];
  const uint32_t mask = a.mask;
  FdmVariants v;
  v.vx = fdm_variant(bc.ex0 + le, nx, mask, 0);
  // block-uniform (made explicit so that the tables are read with scalar loads)
  v.vy = __builtin_amdgcn_readfirstlane(fdm_variant(bc.ey, ny, mask, 1));
  v.vz = __builtin_amdgcn_readfirstlane(fdm_variant(bc.ez, nz, mask, 2));
  v.vfirst = __builtin_amdgcn_readfirstlane(fdm_variant(bc.ex0, nx, mask, 0));
  v.vlast = __builtin_amdgcn_readfirstlane(fdm_variant(bc.ex0 + nvalid - 1, nx, mask, 0));
  for (int i = threadIdx.x; i < 3 * (L + P); i += blockDim.x) {
    const int k = i / (L + P), e = i - k * (L + P);
    const int u = k == 0 ? v.vfirst : (k == 1 ? 0 : v.vlast);
    if (e < L) sV[k * L + e] = a.fdmV[0][u][e];
    else sL[k * P + e - L] = a.fdmL[0][u][e - L];
  }
  return v;
}

// o = B_T^-1 rv for the thread's column (ta, tb, 0..P-1) of its cell, by the
// five phases of fast diagonalization through the cell's LDS block sc. Every
// thread of the block calls it (it synchronizes); inactive threads pass
// active = false.
template <int P, typename T>
__device__ __forceinline__ void fdm_solve(const ScalarArgs<T>& a, T* sc, const T* sV, const T* sL,
                                          const FdmVariants& fv, bool active, int ta, int tb, const T* rv, T* o) {
  constexpr int L = P * P;
  T v[P], w[P];
  if (active) {  // z-lines: the thread's own column
    fdm_forward<P, T>(a.fdmV[2][fv.vz], rv, w);
    lds_store_line<P, T, 2>(sc, ta, tb, w);
  }
  __syncthreads();
  if (active) {  // y-lines (i0, i2) = (ta, tb)
    lds_line<P, T, 1>(sc, ta, tb, v);
    fdm_forward<P, T>(a.fdmV[1][fv.vy], v, w);
    lds_store_line<P, T, 1>(sc, ta, tb, w);
  }
  __syncthreads();
  if (active) {  // x-lines (i1, i2) = (ta, tb), the cell's x tables from LDS
    lds_line<P, T, 0>(sc, ta, tb, v);
    const int slot = fv.vx == fv.vfirst ? 0 : (fv.vx == fv.vlast ? 2 : 1);
    fdm_x<P, T>(sV + slot * L, sL + slot * P, a.fdmL[1][fv.vy][ta] + a.fdmL[2][fv.vz][tb], v);
    lds_store_line<P, T, 0>(sc, ta, tb, v);
  }
  __syncthreads();
  if (active) {
    lds_line<P, T, 1>(sc, ta, tb, v);
    fdm_backward<P, T>(a.fdmV[1][fv.vy], v, w);
    lds_store_line<P, T, 1>(sc, ta, tb, w);
  }
  __syncthreads();
  if (active) {
    lds_line<P, T, 2>(sc, ta, tb, v);
    fdm_backward<P, T>(a.fdmV[2][fv.vz], v, o);
  }
}

// Fixed-order tree sum of one value per thread over the block (NT threads,
// NT in [128, 256]) into out[slot]; sh: 256 doubles of LDS.
template <int NT>
__device__ __forceinline__ void block_sum_to(double val, double* sh, double* out, int64_t slot) {
  if (threadIdx.x + NT < 256) sh[threadIdx.x + NT] = 0.0;
  sh[threadIdx.x] = val;
  __syncthreads();
#pragma unroll
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[slot] = sh[0];
  __syncthreads();
}

// One step k >= 1 of the Chebyshev iteration fused into the apply (the
// epilogue of k_scalar_apply with EPI_CHEB / EPI_CHEB_BJ): with t = A z the
// apply's result, w = rhs - t (EPI_CHEB_BJ: w = P (rhs - t), the block-Jacobi
// inverse by fast diagonalization on the same cells and threads),
// d = c1 d + c2 w, and y = z + d (a second vector: neighbours still read z).
// The right-hand side is rd (FP64, rounded) when given, else r; with rd the
// last step also reduces rd.y per block and does not store d.
template <typename T>
struct ChebStep {
  const T* r;
  const double* rd;
  T* d;
  T c1, c2;
  int last;
};

enum : int { EPI_STORE = 0, EPI_CHEB = 1, EPI_CHEB_BJ = 2 };

// DOT: every block also writes the sum of x_i y_i over its cells (FP64, fixed
// order) to partial[block]: the p.Ap of a conjugate-gradient iteration.
// EPI: what happens to the result t = A x of a block's cells (ChebStep).
template <int P, typename T, bool KAPPA, bool DOT, bool MC, int EPI>
__global__ void __launch_bounds__(CellsPerBlock<P>::value * P * P)
    k_scalar_apply(const T* __restrict__ x, T* __restrict__ y, const T* __restrict__ kappa,
                   const ScalarArgs<T>* __restrict__ ap, double* __restrict__ partial, const ChebStep<T> cs) {
  const ScalarArgs<T>& a = *ap;
  constexpr int EB = CellsPerBlock<P>::value;
  constexpr int L = P * P, N = P * P * P, NT = EB * L;
  using Ly = Layout<P>;
  static_assert(EB * Ly::NP * sizeof(T) >= 256 * sizeof(double), "reduction scratch");
  static_assert(!(EPI == EPI_CHEB_BJ && KAPPA), "the block-Jacobi inverse is built for kappa = 1");
  // the chunk's cells; once every line has been read, the x-line results,
  // then += the y-line results (each thread keeps its own z-line, the cell
  // column it stands for, in registers)
  __shared__ __attribute__((aligned(16))) T sx[EB * Ly::NP];
  __shared__ T sk[KAPPA ? EB * Ly::NP : 1];
  __shared__ T sV[EPI == EPI_CHEB_BJ ? 3 * L : 1], sL[EPI == EPI_CHEB_BJ ? 3 * P : 1];

  const BlockCoord bc = block_coord(a.blocks);
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
  const uint32_t nxy = (uint32_t)nx * ny;
  T nb1[2][P], nk1[2][P], nb2[2][P], nk2[2][P];
  bool has1[2], has2[2];
  FdmVariants fv{};
  if constexpr (EPI == EPI_CHEB_BJ) fv = fdm_setup<P, T>(a, bc, nvalid, le, sV, sL);
  if (active) {
    load_cell_column<P, T>(sx, x, gbase, le, ta, tb);
    if (KAPPA) load_cell_column<P, T>(sk, kappa, gbase, le, ta, tb);
  }
  __syncthreads();

  const T wt = a.wl[li];  // tangential weight w_ta w_tb of this thread's lines
  const T* sxe = sx + le * Ly::NP;
  const T* ske = KAPPA ? sk + le * Ly::NP : nullptr;
  // With the matrix cores every lane runs the line work (the instruction
  // works on all 64 lanes, so it must not sit in divergent code); a lane of
  // a cell beyond the row (EB > nvalid) then works on its LDS slots and zero
  // neighbour lines, reads nothing from global memory and stores nothing.
  const bool work = MC || active;
  T AD[MC ? 4 : 1], ADt[MC ? 4 : 1];  // the lane's A operands of the two contractions
  if (MC) {
    const int r = threadIdx.x & 3;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      AD[k] = a.D[r * 4 + k];
      ADt[k] = a.D[k * 4 + r];
    }
  }
  T out0[P], out1[P], out2[P];
  T vz[P];  // the thread's own z-line: the input column (ta, tb, 0..P-1)
  if (work) {
    T v[P], kv[P];
    T nb[2][P], nk[2][P];
    bool has[2];
    // lines along x: (i1, i2) = (ta, tb)
    lds_line<P, T, 0>(sxe, ta, tb, v);
    if (KAPPA) lds_line<P, T, 0>(ske, ta, tb, kv);
    neighbor_lines<P, T, 0>(sx, x, e, le, nvalid, active ? ex : 0, active ? nx : 1, 1u, ta, tb, nb, has);
    if (KAPPA) neighbor_lines<P, T, 0>(sk, kappa, e, le, nvalid, active ? ex : 0, active ? nx : 1, 1u, ta, tb, nk, has);
    line_work<P, T, KAPPA, 0, MC>(v, kv, nb, nk, has, a, true, AD, ADt, out0);
    // lines along y: (i0, i2) = (ta, tb)
    lds_line<P, T, 1>(sxe, ta, tb, v);
    if (KAPPA) lds_line<P, T, 1>(ske, ta, tb, kv);
    neighbor_lines<P, T, 1>(sx, x, e, le, nvalid, active ? bc.ey : 0, active ? ny : 1, (uint32_t)nx, ta, tb, nb1, has1);
    if (KAPPA)
      neighbor_lines<P, T, 1>(sk, kappa, e, le, nvalid, active ? bc.ey : 0, active ? ny : 1, (uint32_t)nx, ta, tb, nk1,
                              has1);
    line_work<P, T, KAPPA, 1, MC>(v, kv, nb1, nk1, has1, a, false, AD, ADt, out1);
    lds_line<P, T, 2>(sxe, ta, tb, vz);
  }
  __syncthreads();  // every line of the cells has been read: sx takes the results
  if (work && active) {
#pragma unroll
    for (int i = 0; i < P; ++i) sx[le * Ly::NP + i + Ly::S1 * ta + Ly::S2 * tb] = wt * out0[i];
  }
  __syncthreads();
  if (work) {
    if (active) {
#pragma unroll
      for (int i = 0; i < P; ++i) {
        T* yi = sx + le * Ly::NP + ta + Ly::S1 * i + Ly::S2 * tb;
        *yi = fma(wt, out1[i], *yi);
      }
    }
    // lines along z: (i0, i1) = (ta, tb), kept in registers
    T kv[P];
    if (KAPPA) lds_line<P, T, 2>(ske, ta, tb, kv);
    neighbor_lines<P, T, 2>(sx, x, e, le, nvalid, active ? bc.ez : 0, active ? nz : 1, nxy, ta, tb, nb2, has2);
    if (KAPPA)
      neighbor_lines<P, T, 2>(sk, kappa, e, le, nvalid, active ? bc.ez : 0, active ? nz : 1, nxy, ta, tb, nk2, has2);
    line_work<P, T, KAPPA, 2, MC>(vz, kv, nb2, nk2, has2, a, false, AD, ADt, out2);
  }
  __syncthreads();
  double pq = 0.0;
  if constexpr (EPI == EPI_STORE) {
    if (active) {
      const int lo = le * Ly::NP + ta + Ly::S1 * tb;
      T* __restrict__ ye = y + e * N + ta + P * tb;
#pragma unroll
      for (int j = 0; j < P; ++j) {
        const T v = fma(wt, out2[j], sx[lo + j * Ly::S2]);
        ye[j * L] = v;
        if (DOT) pq = fma((double)vz[j], (double)v, pq);
      }
    }
  } else {
    // the Chebyshev step on the thread's column (ta, tb, 0..P-1): A z from sx,
    // z itself from the registers (the preconditioner then uses sx as scratch)
    const int lo = le * Ly::NP + ta + Ly::S1 * tb;
    const size_t col = (size_t)e * N + ta + P * tb;
    T w[P], zv[P], o[P];
#pragma unroll
    for (int j = 0; j < P; ++j) w[j] = zv[j] = T(0);
    if (active) {
#pragma unroll
      for (int j = 0; j < P; ++j) {
        const T t = fma(wt, out2[j], sx[lo + j * Ly::S2]);
        zv[j] = vz[j];
        const T ri = cs.rd ? (T)cs.rd[col + (size_t)j * L] : cs.r[col + (size_t)j * L];
        w[j] = ri - t;
      }
    }
    if constexpr (EPI == EPI_CHEB_BJ) {
      fdm_solve<P, T>(a, sx + le * Ly::NP, sV, sL, fv, active, ta, tb, w, o);
    } else {
#pragma unroll
      for (int j = 0; j < P; ++j) o[j] = w[j];
    }
    if (active) {
#pragma unroll
      for (int j = 0; j < P; ++j) {
        const size_t i = col + (size_t)j * L;
        const T dj = fma(cs.c1, cs.d[i], cs.c2 * o[j]);
        const T zj = zv[j] + dj;
        if (!cs.last) cs.d[i] = dj;
        y[i] = zj;
        if (cs.last && cs.rd) pq = fma(cs.rd[i], (double)zj, pq);
      }
    }
    if (cs.last && cs.rd) {
      __syncthreads();  // sx becomes the reduction scratch
      block_sum_to<NT>(pq, reinterpret_cast<double*>(sx), partial, chunk_slot(bc, a, EB));
    }
  }
  if (DOT) {  // fixed-order tree over the block (NT in [128, 256]), sx as scratch
    double* sh = reinterpret_cast<double*>(sx);
    __syncthreads();
    if (threadIdx.x + NT < 256) sh[threadIdx.x + NT] = 0.0;
    sh[threadIdx.x] = pq;
    __syncthreads();
#pragma unroll
    for (int st = 128; st > 0; st >>= 1) {
      if ((int)threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[chunk_slot(bc, a, EB)] = sh[0];
  }
}

// ---------------------------------------------------------------------------
// Adjoint: A^T g and dL/dkappa for L = g^T A(kappa) u.
//
// A^T g is the apply with the two non-symmetric face coefficients swapped.
// L = a(u_h, g_h) is linear in kappa. Per direction d and volume point q,
// kappa_q multiplies w_q |J| / h_d^2 (d_d u)(d_d g); on a face, kappa_T is the
// trace of the cell's interpolant of its point values, sum_j l_j(s) kappa_j
// along the normal line, so the face integrand's derivative at that face point
// is spread back onto the line with the same rows l_j(s). Per face point of
// cell T, with nu the outward normal of T and N the neighbour,
//   dI/dkappa_T = 1/2 (c_cons d_nu u_T (g_T - g_N) + c_sym (u_T - u_N) d_nu g_T)
// (c_cons = -1, c_sym = theta; on Dirichlet sides without the 1/2 and N).
template <int P, typename T, bool KAPPA, int DIR>
__device__ __forceinline__ void line_adjoint(const T* v, const T* uu, const T* kv, const T (*gn)[P],
                                             const T (*un)[P], const T (*kn)[P], const bool* has_nb, T wt,
                                             const ScalarArgs<T>& a, bool mass, T* outg, T* outk) {
  const T cf_cons = a.c_cons, cf_sym = a.c_sym;  // forward coefficients
  const T ca_cons = a.c_sym, ca_sym = a.c_cons;  // transposed apply
  const T vsw = a.vs[DIR] * wt;
  T r[P];
#pragma unroll
  for (int q = 0; q < P; ++q) {
    T dg = T(0), du = T(0);
#pragma unroll
    for (int j = 0; j < P; ++j) {
      dg = fma(a.D[q * P + j], v[j], dg);
      du = fma(a.D[q * P + j], uu[j], du);
    }
    const T sc = vsw * a.w[q];
    r[q] = KAPPA ? (sc * kv[q]) * dg : sc * dg;
    outk[q] = (sc * du) * dg;
  }
#pragma unroll
  for (int i = 0; i < P; ++i) {
    T s = T(0);
#pragma unroll
    for (int q = 0; q < P; ++q) s = fma(a.D[q * P + i], r[q], s);
    outg[i] = s;
  }
  if (mass) {
    const T cw = a.cmass * wt;
#pragma unroll
    for (int i = 0; i < P; ++i) outg[i] = fma(cw * a.w[i], v[i], outg[i]);
  }
  const T fw = wt * a.fs[DIR];
  const T hi = a.hinv[DIR];
  // kappa values on faces (traces) exist only with kappa per point; the face part of
  // dkappa exists whenever faces use the trace reading (kappa = 1 mode included)
  const bool face_kappa = KAPPA && !a.kappa_face_one;
  const bool face_dk = !a.kappa_face_one;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const bool dirichlet = (a.mask >> (2 * DIR + s)) & 1u;
    if (!has_nb[s] && !dirichlet) continue;
    T gT = T(0), dgT = T(0), uT = T(0), duT = T(0);
#pragma unroll
    for (int j = 0; j < P; ++j) {
      gT = fma(a.e[s][j], v[j], gT);
      dgT = fma(a.de[s][j], v[j], dgT);
      uT = fma(a.e[s][j], uu[j], uT);
      duT = fma(a.de[s][j], uu[j], duT);
    }
    T kT = T(1);
    if (face_kappa) {
      kT = T(0);
#pragma unroll
      for (int j = 0; j < P; ++j) kT = fma(a.e[s][j], kv[j], kT);
    }
    const T sg = s ? T(1) : T(-1);
    const T dnug = sg * hi * dgT, dnuu = sg * hi * duT;
    T Rv, Rdv, dI;
    if (has_nb[s]) {
      T gN = T(0), dgN = T(0), uN = T(0);
#pragma unroll
      for (int j = 0; j < P; ++j) {
        gN = fma(a.e[1 - s][j], gn[s][j], gN);
        dgN = fma(a.de[1 - s][j], gn[s][j], dgN);
        uN = fma(a.e[1 - s][j], un[s][j], uN);
      }
      T kN = T(1);
      if (face_kappa) {
        kN = T(0);
#pragma unroll
        for (int j = 0; j < P; ++j) kN = fma(a.e[1 - s][j], kn[s][j], kN);
      }
      const T dnugN = -sg * hi * dgN;
      const T jg = gT - gN;
      Rv = T(0.5) * ca_cons * (kT * dnug - kN * dnugN) + a.gam[DIR] * jg;
      Rdv = T(0.5) * ca_sym * kT * jg;
      dI = T(0.5) * (cf_cons * dnuu * jg + cf_sym * (uT - uN) * dnug);
    } else {
      Rv = ca_cons * kT * dnug + a.gam[DIR] * gT;
      Rdv = ca_sym * kT * gT;
      dI = cf_cons * dnuu * gT + cf_sym * uT * dnug;
    }
    Rv *= fw;
    Rdv *= fw * sg * hi;
#pragma unroll
    for (int i = 0; i < P; ++i) outg[i] = fma(Rv, a.e[s][i], fma(Rdv, a.de[s][i], outg[i]));
    if (face_dk) {
      dI *= fw;
#pragma unroll
      for (int j = 0; j < P; ++j) outk[j] = fma(dI, a.e[s][j], outk[j]);
    }
  }
}

template <int P, typename T, bool KAPPA, int DIR>
__device__ __forceinline__ void adjoint_direction(const T* sge, const T* sue, const T* ske, const T* sgb,
                                                  const T* sub, const T* skb, const T* __restrict__ g,
                                                  const T* __restrict__ u, const T* __restrict__ kappa, uint32_t e,
                                                  int le, int nvalid, int ecd, int nd, uint32_t estride, int ta,
                                                  int tb, T wt, const ScalarArgs<T>& a, bool mass, T* og, T* ok) {
  T v[P], uu[P], kv[P];
  T gn[2][P], un[2][P], kn[2][P];
  bool has[2];
  lds_line<P, T, DIR>(sge, ta, tb, v);
  lds_line<P, T, DIR>(sue, ta, tb, uu);
  if (KAPPA) lds_line<P, T, DIR>(ske, ta, tb, kv);
  neighbor_lines<P, T, DIR>(sgb, g, e, le, nvalid, ecd, nd, estride, ta, tb, gn, has);
  neighbor_lines<P, T, DIR>(sub, u, e, le, nvalid, ecd, nd, estride, ta, tb, un, has);
  if (KAPPA) neighbor_lines<P, T, DIR>(skb, kappa, e, le, nvalid, ecd, nd, estride, ta, tb, kn, has);
  line_adjoint<P, T, KAPPA, DIR>(v, uu, kv, gn, un, kn, has, wt, a, mass, og, ok);
}

template <int P, typename T, bool KAPPA>
__global__ void __launch_bounds__(AdjCellsPerBlock<P>::value * P * P)
    k_scalar_adjoint(const T* __restrict__ g, const T* __restrict__ u, const T* __restrict__ kappa,
                     T* __restrict__ ATg, T* __restrict__ dkappa, const ScalarArgs<T>* __restrict__ ap) {
  const ScalarArgs<T>& a = *ap;
  constexpr int EB = AdjCellsPerBlock<P>::value;
  constexpr int L = P * P, N = P * P * P;
  using Ly = Layout<P>;
  __shared__ T sg[EB * Ly::NP];
  __shared__ T su[EB * Ly::NP];
  __shared__ T sk[KAPPA ? EB * Ly::NP : 1];
  __shared__ T sy[EB * Ly::NP], sd[EB * Ly::NP];  // x-line results, then += y-line results

  const BlockCoord bc = block_coord(a.blocks);
  const int nx = a.n[0], ny = a.n[1], nz = a.n[2];
  const int ex0 = bc.ex0;
  const int nvalid = min(EB, nx - ex0);
  const uint32_t row = (uint32_t)nx * ((uint32_t)bc.ey + (uint32_t)ny * bc.ez);
  const uint32_t gbase = (row + ex0) * N;
  const int le = threadIdx.x / L;
  const int li = threadIdx.x - le * L;
  const bool active = le < nvalid;
  const int ta = li % P, tb = li / P;
  if (active) {
    load_cell_column<P, T>(sg, g, gbase, le, ta, tb);
    load_cell_column<P, T>(su, u, gbase, le, ta, tb);
    if (KAPPA) load_cell_column<P, T>(sk, kappa, gbase, le, ta, tb);
  }
  __syncthreads();
  const T wt = a.wl[li];
  const int ex = ex0 + le;
  const uint32_t e = row + ex;
  const T* sge = sg + le * Ly::NP;
  const T* sue = su + le * Ly::NP;
  const T* ske = KAPPA ? sk + le * Ly::NP : nullptr;
  // lines along x: each node is written by exactly one thread
  if (active) {
    T og[P], ok[P];
    adjoint_direction<P, T, KAPPA, 0>(sge, sue, ske, sg, su, sk, g, u, kappa, e, le, nvalid, ex, nx, 1u, ta, tb, wt,
                                      a, true, og, ok);
#pragma unroll
    for (int i = 0; i < P; ++i) {
      sy[le * Ly::NP + i + Ly::S1 * ta + Ly::S2 * tb] = og[i];
      sd[le * Ly::NP + i + Ly::S1 * ta + Ly::S2 * tb] = ok[i];
    }
  }
  __syncthreads();
  // lines along y are added in place (again one thread per node); lines along z stay in registers
  T og2[P], ok2[P];
  if (active) {
    T og[P], ok[P];
    adjoint_direction<P, T, KAPPA, 1>(sge, sue, ske, sg, su, sk, g, u, kappa, e, le, nvalid, bc.ey, ny,
                                      (uint32_t)nx, ta, tb, wt, a, false, og, ok);
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const int o = le * Ly::NP + ta + Ly::S1 * i + Ly::S2 * tb;
      sy[o] += og[i];
      sd[o] += ok[i];
    }
    adjoint_direction<P, T, KAPPA, 2>(sge, sue, ske, sg, su, sk, g, u, kappa, e, le, nvalid, bc.ez, nz,
                                      (uint32_t)nx * ny, ta, tb, wt, a, false, og2, ok2);
  }
  __syncthreads();
  if (active) {
    const int lo = le * Ly::NP + ta + Ly::S1 * tb;
    const uint32_t go = e * N + ta + P * tb;
#pragma unroll
    for (int j = 0; j < P; ++j) {
      ATg[go + j * L] = sy[lo + j * Ly::S2] + og2[j];
      dkappa[go + j * L] = sd[lo + j * Ly::S2] + ok2[j];
    }
  }
}

// With q != NULL the residual is first updated in place, r -= alpha q (alpha
// read from device memory), and partial sums of r.r go to partial_rr: one
// pass over r, q and z per conjugate-gradient iteration.
template <int P, typename T>
__global__ void __launch_bounds__(CellsPerBlock<P>::value * P * P) __attribute__((amdgpu_waves_per_eu(4)))
    k_block_jacobi(T* __restrict__ r, T* __restrict__ z, const ScalarArgs<T>* __restrict__ ap,
                   double* __restrict__ partial, const T* __restrict__ q, const double* __restrict__ alpha,
                   double* __restrict__ partial_rr) {
  const ScalarArgs<T>& a = *ap;
  constexpr int EB = CellsPerBlock<P>::value;
  constexpr int L = P * P, N = P * P * P, NT = EB * L;
  using Ly = Layout<P>;
  __shared__ T s[EB * Ly::NP];
  __shared__ T sV[3 * L], sL[3 * P];  // x tables: first cell, interior, last cell
  __shared__ double sh[256];

  const BlockCoord bc = block_coord(a.blocks);
  const int nx = a.n[0], ny = a.n[1];
  const int ex0 = bc.ex0;
  const int nvalid = min(EB, nx - ex0);
  const uint32_t row = (uint32_t)nx * ((uint32_t)bc.ey + (uint32_t)ny * bc.ez);
  const int le = threadIdx.x / L;
  const int li = threadIdx.x - le * L;
  const bool active = le < nvalid;
  const int ta = li % P, tb = li / P;
  const FdmVariants fv = fdm_setup<P, T>(a, bc, nvalid, le, sV, sL);
  // the thread's column (ta, tb, 0..P-1) is the z-line it owns first
  const size_t col = (size_t)(row + ex0 + le) * N + ta + P * tb;
  T rv[P], o[P];
  double rr = 0.0;
  if (active) {
    if (q) {
      const T al = (T)*alpha;
#pragma unroll
      for (int j = 0; j < P; ++j) {
        rv[j] = fma(-al, q[col + (size_t)j * L], r[col + (size_t)j * L]);
        r[col + (size_t)j * L] = rv[j];
        rr = fma((double)rv[j], (double)rv[j], rr);
      }
    } else {
#pragma unroll
      for (int j = 0; j < P; ++j) rv[j] = r[col + (size_t)j * L];
    }
  }
  fdm_solve<P, T>(a, s + le * Ly::NP, sV, sL, fv, active, ta, tb, rv, o);
  double rz = 0.0;
  if (active) {
#pragma unroll
    for (int j = 0; j < P; ++j) {
      z[col + (size_t)j * L] = o[j];
      rz = fma((double)rv[j], (double)o[j], rz);
    }
  }
  // block sums: r.z, then r.r
  if (partial) block_sum_to<NT>(rz, sh, partial, chunk_slot(bc, a, EB));
  if (q) block_sum_to<NT>(rr, sh, partial_rr, chunk_slot(bc, a, EB));
}

// One step of the Chebyshev iteration for B z = rhs preconditioned by the
// block-Jacobi inverse P: w = P (rhs - t) (t = A z; absent on the first
// step, where z = 0), d = c1 d + c2 w (d absent on the first step), z += d.
// The right-hand side is read from rd (FP64, rounded to T) when given, else
// from r; with rd the last step also writes the partial sums of rd.z (FP64,
// fixed order) and does not store d.
template <int P, typename T>
__global__ void __launch_bounds__(CellsPerBlock<P>::value * P * P)
    k_cheb_block_jacobi(const T* __restrict__ r, const double* __restrict__ rd, const T* __restrict__ t,
                        T* __restrict__ d, T* __restrict__ z, T c1, T c2, int first, int last,
                        const ScalarArgs<T>* __restrict__ ap, double* __restrict__ partial) {
  const ScalarArgs<T>& a = *ap;
  constexpr int EB = CellsPerBlock<P>::value;
  constexpr int L = P * P, N = P * P * P, NT = EB * L;
  using Ly = Layout<P>;
  __shared__ T s[EB * Ly::NP];
  __shared__ T sV[3 * L], sL[3 * P];
  __shared__ double sh[256];

  const BlockCoord bc = block_coord(a.blocks);
  const int nx = a.n[0], ny = a.n[1];
  const int ex0 = bc.ex0;
  const int nvalid = min(EB, nx - ex0);
  const uint32_t row = (uint32_t)nx * ((uint32_t)bc.ey + (uint32_t)ny * bc.ez);
  const int le = threadIdx.x / L;
  const int li = threadIdx.x - le * L;
  const bool active = le < nvalid;
  const int ta = li % P, tb = li / P;
  const FdmVariants fv = fdm_setup<P, T>(a, bc, nvalid, le, sV, sL);
  const size_t col = (size_t)(row + ex0 + le) * N + ta + P * tb;
  T wv[P], o[P];
  if (active) {
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const size_t i = col + (size_t)j * L;
      const T ri = rd ? (T)rd[i] : r[i];
      wv[j] = first ? ri : ri - t[i];
    }
  }
  fdm_solve<P, T>(a, s + le * Ly::NP, sV, sL, fv, active, ta, tb, wv, o);
  double rz = 0.0;
  if (active) {
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const size_t i = col + (size_t)j * L;
      const T di = first ? c2 * o[j] : fma(c1, d[i], c2 * o[j]);
      const T zi = first ? di : z[i] + di;
      if (!last) d[i] = di;
      z[i] = zi;
      if (last && rd) rz = fma(rd[i], (double)zi, rz);
    }
  }
  if (last && rd) block_sum_to<NT>(rz, sh, partial, chunk_slot(bc, a, EB));
}

// b_i = w_i |J| f_i: with collocation, phi_i(x_q) = delta_iq.
template <int P, typename T>
__global__ void k_scalar_load(const T* __restrict__ f, T* __restrict__ b, const ScalarArgs<T>* __restrict__ ap,
                              int64_t n) {
  const ScalarArgs<T>& a = *ap;
  constexpr int N = P * P * P;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int l = (int)(i % N);
  const int i0 = l % P, i1 = (l / P) % P, i2 = l / (P * P);
  const T detJ = a.vs[0] / (a.hinv[0] * a.hinv[0]);  // |J| = vs_0 h_0^2
  b[i] = (a.w[i0] * a.w[i1] * a.w[i2] * detJ) * f[i];
}

// Grid of the sweep: one block per x-chunk of eb cells of every (y, z) row.
template <typename T>
int64_t sweep_grid(ScalarArgs<T>& a, int eb) {
  a.nchunk = (a.n[0] + eb - 1) / eb;
  return (int64_t)a.nchunk * a.n[1] * a.n[2];
}

template <typename T>
const ScalarArgs<T>* host_params(const dg_mesh& M);
template <>
const ScalarArgs<double>* host_params<double>(const dg_mesh& M) { return M.pd; }
template <>
const ScalarArgs<float>* host_params<float>(const dg_mesh& M) { return M.pf; }
template <typename T>
const ScalarArgs<T>* device_params(const dg_mesh& M);
template <>
const ScalarArgs<double>* device_params<double>(const dg_mesh& M) { return M.d_pd; }
template <>
const ScalarArgs<float>* device_params<float>(const dg_mesh& M) { return M.d_pf; }

// Grid size of a parameter block whose sweep fields are already set.
template <typename T>
int64_t grid_of(const ScalarArgs<T>& a) {
  return (int64_t)a.nchunk * a.n[1] * a.n[2];
}

template <int P, typename T>
hipError_t launch_apply(const dg_mesh& M, int variant, const T* x, T* y, const T* kappa, double* partial,
                        hipStream_t s) {
  constexpr int EB = CellsPerBlock<P>::value;
  const int64_t G = grid_of(host_params<T>(M)[variant]);
  if (G > 0x7fffffff || M.ndofs > 0xffffffffLL) return hipErrorInvalidValue;
  const ScalarArgs<T>* ap = device_params<T>(M) + variant;
  const dim3 grid((unsigned)G), block(EB * P * P);
  const ChebStep<T> none{};
  constexpr bool MCOK = P == 4 && sizeof(T) == 4;  // FP32 lines of p = 4 may use the matrix cores
  if (MCOK && M.lines_mfma) {
    if (kappa && partial)
      hipLaunchKernelGGL((k_scalar_apply<P, T, true, true, MCOK, EPI_STORE>), grid, block, 0, s, x, y, kappa, ap,
                         partial, none);
    else if (kappa)
      hipLaunchKernelGGL((k_scalar_apply<P, T, true, false, MCOK, EPI_STORE>), grid, block, 0, s, x, y, kappa, ap,
                         partial, none);
    else if (partial)
      hipLaunchKernelGGL((k_scalar_apply<P, T, false, true, MCOK, EPI_STORE>), grid, block, 0, s, x, y, kappa, ap,
                         partial, none);
    else
      hipLaunchKernelGGL((k_scalar_apply<P, T, false, false, MCOK, EPI_STORE>), grid, block, 0, s, x, y, kappa, ap,
                         partial, none);
    return hipGetLastError();
  }
  if (kappa && partial)
    hipLaunchKernelGGL((k_scalar_apply<P, T, true, true, false, EPI_STORE>), grid, block, 0, s, x, y, kappa, ap,
                       partial, none);
  else if (kappa)
    hipLaunchKernelGGL((k_scalar_apply<P, T, true, false, false, EPI_STORE>), grid, block, 0, s, x, y, kappa, ap,
                       partial, none);
  else if (partial)
    hipLaunchKernelGGL((k_scalar_apply<P, T, false, true, false, EPI_STORE>), grid, block, 0, s, x, y, kappa, ap,
                       partial, none);
  else
    hipLaunchKernelGGL((k_scalar_apply<P, T, false, false, false, EPI_STORE>), grid, block, 0, s, x, y, kappa, ap,
                       partial, none);
  return hipGetLastError();
}

// One fused Chebyshev step (apply, residual, optional block-Jacobi inverse,
// update): reads z, writes zout (and d unless last).
template <int P, typename T>
hipError_t launch_cheb_apply(const dg_mesh& M, const T* z, T* zout, const T* kappa, const ChebStep<T>& cs, bool bj,
                             double* partial, hipStream_t s) {
  constexpr int EB = CellsPerBlock<P>::value;
  const int64_t G = grid_of(host_params<T>(M)[SP_APPLY]);
  if (G > 0x7fffffff || M.ndofs > 0xffffffffLL) return hipErrorInvalidValue;
  const ScalarArgs<T>* ap = device_params<T>(M) + SP_APPLY;
  const dim3 grid((unsigned)G), block(EB * P * P);
  if (bj)
    hipLaunchKernelGGL((k_scalar_apply<P, T, false, false, false, EPI_CHEB_BJ>), grid, block, 0, s, z, zout, kappa,
                       ap, partial, cs);
  else if (kappa)
    hipLaunchKernelGGL((k_scalar_apply<P, T, true, false, false, EPI_CHEB>), grid, block, 0, s, z, zout, kappa, ap,
                       partial, cs);
  else
    hipLaunchKernelGGL((k_scalar_apply<P, T, false, false, false, EPI_CHEB>), grid, block, 0, s, z, zout, kappa, ap,
                       partial, cs);
  return hipGetLastError();
}

template <typename T>
hipError_t dispatch_cheb_apply(const dg_mesh& M, const T* z, T* zout, const T* kappa, const ChebStep<T>& cs, bool bj,
                               double* partial, hipStream_t s) {
  switch (M.p) {
    case 2: return launch_cheb_apply<2, T>(M, z, zout, kappa, cs, bj, partial, s);
    case 3: return launch_cheb_apply<3, T>(M, z, zout, kappa, cs, bj, partial, s);
    case 4: return launch_cheb_apply<4, T>(M, z, zout, kappa, cs, bj, partial, s);
    case 5: return launch_cheb_apply<5, T>(M, z, zout, kappa, cs, bj, partial, s);
    case 6: return launch_cheb_apply<6, T>(M, z, zout, kappa, cs, bj, partial, s);
    case 7: return launch_cheb_apply<7, T>(M, z, zout, kappa, cs, bj, partial, s);
    case 8: return launch_cheb_apply<8, T>(M, z, zout, kappa, cs, bj, partial, s);
    default: return hipErrorInvalidValue;
  }
}

template <int P, typename T>
hipError_t launch_adjoint(const dg_mesh& M, const T* g, const T* u, const T* kappa, T* ATg, T* dk, hipStream_t s) {
  constexpr int EB = AdjCellsPerBlock<P>::value;
  const int64_t G = grid_of(host_params<T>(M)[SP_ADJOINT]);
  if (G > 0x7fffffff || M.ndofs > 0xffffffffLL) return hipErrorInvalidValue;
  const ScalarArgs<T>* ap = device_params<T>(M) + SP_ADJOINT;
  if (kappa)
    hipLaunchKernelGGL((k_scalar_adjoint<P, T, true>), dim3((unsigned)G), dim3(EB * P * P), 0, s, g, u, kappa, ATg,
                       dk, ap);
  else
    hipLaunchKernelGGL((k_scalar_adjoint<P, T, false>), dim3((unsigned)G), dim3(EB * P * P), 0, s, g, u, kappa,
                       ATg, dk, ap);
  return hipGetLastError();
}

template <int P, typename T>
hipError_t launch_block_jacobi(const dg_mesh& M, T* r, T* z, double* partial, const T* q, const double* alpha,
                               double* partial_rr, hipStream_t s) {
  constexpr int EB = CellsPerBlock<P>::value;
  static_assert(EB * P * P >= 128 && EB * P * P <= 256, "block reduction assumes 128..256 threads");
  const int64_t G = grid_of(host_params<T>(M)[SP_APPLY]);
  if (G > 0x7fffffff || M.ndofs > 0xffffffffLL) return hipErrorInvalidValue;
  const ScalarArgs<T>* ap = device_params<T>(M) + SP_APPLY;
  hipLaunchKernelGGL((k_block_jacobi<P, T>), dim3((unsigned)G), dim3(EB * P * P), 0, s, r, z, ap, partial, q, alpha,
                     partial_rr);
  return hipGetLastError();
}

template <int P, typename T>
hipError_t launch_cheb_block_jacobi(const dg_mesh& M, const T* r, const double* rd, const T* t, T* d, T* z, T c1,
                                    T c2, bool first, bool last, double* partial, hipStream_t s) {
  constexpr int EB = CellsPerBlock<P>::value;
  static_assert(EB * P * P >= 128 && EB * P * P <= 256, "block reduction assumes 128..256 threads");
  const int64_t G = grid_of(host_params<T>(M)[SP_APPLY]);
  if (G > 0x7fffffff || M.ndofs > 0xffffffffLL) return hipErrorInvalidValue;
  const ScalarArgs<T>* ap = device_params<T>(M) + SP_APPLY;
  hipLaunchKernelGGL((k_cheb_block_jacobi<P, T>), dim3((unsigned)G), dim3(EB * P * P), 0, s, r, rd, t, d, z, c1, c2,
                     (int)first, (int)last, ap, partial);
  return hipGetLastError();
}

// Cells per block of the apply and adjoint kernels for p nodes per direction.
int apply_cells_per_block(int p) { return 256 / (p * p) > 0 ? 256 / (p * p) : 1; }
int adjoint_cells_per_block(int p) { return 128 / (p * p) > 0 ? 128 / (p * p) : 1; }

#define DG_DISPATCH_P(P_, CALL)           \
  switch (P_) {                           \
    case 2: return CALL(2);               \
    case 3: return CALL(3);               \
    case 4: return CALL(4);               \
    case 5: return CALL(5);               \
    case 6: return CALL(6);               \
    case 7: return CALL(7);               \
    case 8: return CALL(8);               \
    default: return hipErrorInvalidValue; \
  }

template <typename T>
hipError_t dispatch_apply(const dg_mesh& M, int variant, const T* x, T* y, const T* kappa, double* partial,
                          hipStream_t s) {
#define DG_CALL(PP) launch_apply<PP, T>(M, variant, x, y, kappa, partial, s)
  DG_DISPATCH_P(M.p, DG_CALL)
#undef DG_CALL
}

template <typename T>
hipError_t dispatch_adjoint(const dg_mesh& M, const T* g, const T* u, const T* kappa, T* ATg, T* dk,
                            hipStream_t s) {
#define DG_CALL(PP) launch_adjoint<PP, T>(M, g, u, kappa, ATg, dk, s)
  DG_DISPATCH_P(M.p, DG_CALL)
#undef DG_CALL
}

template <typename T>
hipError_t dispatch_block_jacobi(const dg_mesh& M, T* r, T* z, double* partial, const T* q, const double* alpha,
                                 double* partial_rr, hipStream_t s) {
#define DG_CALL(PP) launch_block_jacobi<PP, T>(M, r, z, partial, q, alpha, partial_rr, s)
  DG_DISPATCH_P(M.p, DG_CALL)
#undef DG_CALL
}

template <typename T>
hipError_t dispatch_cheb_block_jacobi(const dg_mesh& M, const T* r, const double* rd, const T* t, T* d, T* z, T c1,
                                      T c2, bool first, bool last, double* partial, hipStream_t s) {
#define DG_CALL(PP) launch_cheb_block_jacobi<PP, T>(M, r, rd, t, d, z, c1, c2, first, last, partial, s)
  DG_DISPATCH_P(M.p, DG_CALL)
#undef DG_CALL
}

template <typename T>
hipError_t dispatch_load(const dg_mesh& M, const T* f, T* b, hipStream_t s) {
  const int64_t n = M.ndofs;
  const unsigned G = (unsigned)((n + 255) / 256);
  const ScalarArgs<T>* ap = device_params<T>(M) + SP_APPLY;
  switch (M.p) {
#define DG_LOAD_CASE(PP) \
  case PP: hipLaunchKernelGGL((k_scalar_load<PP, T>), dim3(G), dim3(256), 0, s, f, b, ap, n); break;
    DG_LOAD_CASE(2) DG_LOAD_CASE(3) DG_LOAD_CASE(4) DG_LOAD_CASE(5) DG_LOAD_CASE(6) DG_LOAD_CASE(7)
    DG_LOAD_CASE(8)
#undef DG_LOAD_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Hardware block b runs on XCD b % 8: give each XCD a contiguous range of
// the sweep so that its L2 holds the neighbours its blocks read.
int xcd_swizzle(int b, int G) {
  const int q = G >> 3, r = G & 7;
  const int xcd = b & 7, idx = b >> 3;
  return xcd * q + std::min(xcd, r) + idx;
}

// Block table of a sweep grid (chunks of eb cells of every x-row). Each XCD
// (its own L2) sweeps one region of the mesh: x (in whole chunks) and z are
// split so that the fewest cells are read across region boundaries, y is not
// split (the sweep front, the region's x-z cross-section, stays small), and
// inside a region the blocks run y-outermost, then z, then x. Hardware block
// b runs on XCD b % 8 and takes position swizzle(b) of that order.
// linear: the plain order (x chunks, then y, then z) with no XCD renumbering.
std::vector<uint32_t> block_table(int nx, int ny, int nz, int eb, bool linear) {
  const int nc = (nx + eb - 1) / eb;
  const int G = nc * ny * nz;
  if (linear) {
    std::vector<uint32_t> tab(2 * (size_t)G);
    size_t t = 0;
    for (int zz = 0; zz < nz; ++zz)
      for (int yy = 0; yy < ny; ++yy)
        for (int cc = 0; cc < nc; ++cc) {
          tab[2 * t] = (uint32_t)(cc * eb) | ((uint32_t)yy << 16);
          tab[2 * t + 1] = (uint32_t)zz;
          ++t;
        }
    return tab;
  }
  int best[2] = {1, 1};
  double best_cost = -1;
  for (int rx = 1; rx <= 8; rx *= 2) {
    const int rz = 8 / rx;
    if (rx > nc || rz > nz) continue;
    const double cost = (double)(rx - 1) * ny * nz + (double)(rz - 1) * nx * ny;
    if (best_cost < 0 || cost < best_cost) {
      best_cost = cost;
      best[0] = rx;
      best[1] = rz;
    }
  }
  auto bound = [](int n, int r, int i) { return (int)(((int64_t)n * i) / r); };
  std::vector<uint32_t> order(2 * (size_t)G);
  size_t t = 0;
  for (int gz = 0; gz < best[1]; ++gz)
    for (int gx = 0; gx < best[0]; ++gx) {
      const int c0 = bound(nc, best[0], gx), c1 = bound(nc, best[0], gx + 1);
      const int z0 = bound(nz, best[1], gz), z1 = bound(nz, best[1], gz + 1);
      for (int yy = 0; yy < ny; ++yy)
        for (int zz = z0; zz < z1; ++zz)
          for (int cc = c0; cc < c1; ++cc) {
            order[2 * t] = (uint32_t)(cc * eb) | ((uint32_t)yy << 16);
            order[2 * t + 1] = (uint32_t)zz;
            ++t;
          }
    }
  std::vector<uint32_t> tab(2 * (size_t)G);
  for (int b = 0; b < G; ++b) {
    const int l = xcd_swizzle(b, G);
    tab[2 * (size_t)b] = order[2 * (size_t)l];
    tab[2 * (size_t)b + 1] = order[2 * (size_t)l + 1];
  }
  return tab;
}

template <typename T>
void fill_params(const ScalarArgs<T>& base, const Tables1D& tab, int p, ScalarArgs<T>* out) {
  for (int v = 0; v < SP_COUNT; ++v) {
    ScalarArgs<T> a = base;
    if (v == SP_APPLY_T) {
      std::swap(a.c_cons, a.c_sym);
      derive_face_constants(a);
    }
    sweep_grid(a, v == SP_ADJOINT ? adjoint_cells_per_block(p) : apply_cells_per_block(p));
    for (int tb = 0; tb < p; ++tb)
      for (int ta = 0; ta < p; ++ta) {
        // rounded to T first, then multiplied in T, as the kernels' other weights
        a.wl[ta + p * tb] = (T)tab.wq[ta] * (T)tab.wq[tb];
      }
    out[v] = a;
  }
}

}  // namespace

hipError_t scalar_apply(const dg_mesh& M, int prec, const void* x, void* y, const void* kappa, bool transpose,
                        hipStream_t s, double* partial) {
  const int v = transpose ? SP_APPLY_T : SP_APPLY;
  if (mfma_apply_supported(M, prec, kappa != nullptr))
    return mfma_apply(M, v, (const double*)x, (double*)y, partial, s);
  if (mfma_apply_f32_supported(M, prec, kappa != nullptr))
    return mfma_apply_f32(M, v, (const float*)x, (float*)y, partial, s);
  if (prec == DG_F64)
    return dispatch_apply<double>(M, v, (const double*)x, (double*)y, (const double*)kappa, partial, s);
  return dispatch_apply<float>(M, v, (const float*)x, (float*)y, (const float*)kappa, partial, s);
}

int64_t scalar_apply_blocks(const dg_mesh& M, int prec, bool kappa) {
  if (mfma_apply_supported(M, prec, kappa) || mfma_apply_f32_supported(M, prec, kappa)) return M.nwaves[prec];
  return grid_of(M.pd[SP_APPLY]);
}

hipError_t scalar_adjoint(const dg_mesh& M, int prec, const void* g, const void* u, const void* kappa, void* ATg,
                          void* dkappa, hipStream_t s) {
  if (prec == DG_F64)
    return dispatch_adjoint<double>(M, (const double*)g, (const double*)u, (const double*)kappa, (double*)ATg,
                                    (double*)dkappa, s);
  return dispatch_adjoint<float>(M, (const float*)g, (const float*)u, (const float*)kappa, (float*)ATg,
                                 (float*)dkappa, s);
}

hipError_t block_jacobi(const dg_mesh& M, int prec, const void* r, void* z, double* partial, hipStream_t s) {
  // r is only read when no update is requested
  if (prec == DG_F64)
    return dispatch_block_jacobi<double>(M, (double*)r, (double*)z, partial, nullptr, nullptr, nullptr, s);
  return dispatch_block_jacobi<float>(M, (float*)r, (float*)z, partial, nullptr, nullptr, nullptr, s);
}

hipError_t block_jacobi_update(const dg_mesh& M, int prec, void* r, const void* q, const double* alpha, void* z,
                               double* partial_rz, double* partial_rr, hipStream_t s) {
  if (!q || !alpha || !partial_rz || !partial_rr) return hipErrorInvalidValue;
  if (prec == DG_F64)
    return dispatch_block_jacobi<double>(M, (double*)r, (double*)z, partial_rz, (const double*)q, alpha, partial_rr,
                                         s);
  return dispatch_block_jacobi<float>(M, (float*)r, (float*)z, partial_rz, (const float*)q, alpha, partial_rr, s);
}

int64_t block_jacobi_blocks(const dg_mesh& M) { return grid_of(M.pd[SP_APPLY]); }

hipError_t cheb_apply(const dg_mesh& M, int prec, const void* z, void* zout, const void* kappa, const void* r,
                      const double* rd, void* d, double c1, double c2, bool last, bool bj, double* partial,
                      hipStream_t s) {
  if ((last && rd && !partial) || (bj && kappa)) return hipErrorInvalidValue;
  if (prec == DG_F64) {
    const ChebStep<double> cs{(const double*)r, rd, (double*)d, c1, c2, last ? 1 : 0};
    return dispatch_cheb_apply<double>(M, (const double*)z, (double*)zout, (const double*)kappa, cs, bj, partial, s);
  }
  const ChebStep<float> cs{(const float*)r, rd, (float*)d, (float)c1, (float)c2, last ? 1 : 0};
  return dispatch_cheb_apply<float>(M, (const float*)z, (float*)zout, (const float*)kappa, cs, bj, partial, s);
}

hipError_t cheb_block_jacobi(const dg_mesh& M, int prec, const void* r, const double* rd, const void* t, void* d,
                             void* z, double c1, double c2, bool first, bool last, double* partial, hipStream_t s) {
  if (last && rd && !partial) return hipErrorInvalidValue;
  if (prec == DG_F64)
    return dispatch_cheb_block_jacobi<double>(M, (const double*)r, rd, (const double*)t, (double*)d, (double*)z, c1,
                                              c2, first, last, partial, s);
  return dispatch_cheb_block_jacobi<float>(M, (const float*)r, rd, (const float*)t, (float*)d, (float*)z, (float)c1,
                                           (float)c2, first, last, partial, s);
}

hipError_t scalar_load(const dg_mesh& M, int prec, const void* fq, void* b, hipStream_t s) {
  if (prec == DG_F64) return dispatch_load<double>(M, (const double*)fq, (double*)b, s);
  return dispatch_load<float>(M, (const float*)fq, (float*)b, s);
}

hipError_t scalar_params_upload(dg_mesh& M) {
  fill_params(M.sd, M.tab, M.p, M.pd);
  fill_params(M.sf, M.tab, M.p, M.pf);
  // block tables: apply grid, then adjoint grid
  const bool lin = M.sweep_linear != 0;
  const std::vector<uint32_t> ta =
      block_table(M.pd[SP_APPLY].n[0], M.pd[SP_APPLY].n[1], M.pd[SP_APPLY].n[2], apply_cells_per_block(M.p), lin);
  const std::vector<uint32_t> tj =
      block_table(M.pd[SP_ADJOINT].n[0], M.pd[SP_ADJOINT].n[1], M.pd[SP_ADJOINT].n[2],
                  adjoint_cells_per_block(M.p), lin);
  if (M.d_blocks) {  // a rebuild: the old table may still be read by queued work
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return e;
    (void)hipFree(M.d_blocks);
    M.d_blocks = nullptr;
  }
  hipError_t e = hipMalloc(&M.d_blocks, sizeof(uint32_t) * (ta.size() + tj.size()));
  if (e != hipSuccess) return e;
  e = hipMemcpy(M.d_blocks, ta.data(), sizeof(uint32_t) * ta.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  e = hipMemcpy(M.d_blocks + ta.size(), tj.data(), sizeof(uint32_t) * tj.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  for (int v = 0; v < SP_COUNT; ++v) {
    const uint32_t* t = v == SP_ADJOINT ? M.d_blocks + ta.size() : M.d_blocks;
    M.pd[v].blocks = t;
    M.pf[v].blocks = t;
  }
  e = hipMemcpy(M.d_pd, M.pd, sizeof(M.pd), hipMemcpyHostToDevice);
  if (e != hipSuccess) return e;
  return hipMemcpy(M.d_pf, M.pf, sizeof(M.pf), hipMemcpyHostToDevice);
}

hipError_t line_sweep_set(dg_mesh& M, int linear) {
  M.sweep_linear = linear ? 1 : 0;
  return scalar_params_upload(M);
}

}  // namespace dgi
