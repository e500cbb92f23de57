// Internal declarations of the DG library (host side and kernel launchers).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "dg.h"

namespace dgi {

constexpr int PMAX = 8;  // largest number of 1D nodes or points (degree 7)
constexpr int HMAX = PMAX / 2;

// 1D Gauss-Legendre rule on [0,1] and nodal Lagrange tables (Section 2.2: the
// basis matrices A^(i), D^(i) and the face rows used with m_d = 1).
struct Tables1D {
  int p = 0;   // basis nodes (k+1)
  int m = 0;   // quadrature points
  double xn[PMAX] = {};          // basis nodes = p-point Gauss-Legendre nodes
  double xq[PMAX] = {};          // quadrature nodes
  double wq[PMAX] = {};          // quadrature weights
  double A[PMAX][PMAX] = {};     // A[q][j] = l_j(xq_q)
  double D[PMAX][PMAX] = {};     // D[q][j] = l_j'(xq_q)
  double e[2][PMAX] = {};        // e[s][j] = l_j(s), s = 0, 1
  double de[2][PMAX] = {};       // de[s][j] = l_j'(s)
};

void gauss_legendre_golub_welsch(int m, double* x, double* w);
Tables1D make_tables(int p, int m);

// Even-odd volume tables of one direction (see ScalarArgs::eo).
template <typename T>
struct EvenOdd {
  T DvP[HMAX * HMAX];  // [q H + j] (Dv_qj + Dv_q,p-1-j) / 2
  T DvM[HMAX * HMAX];  // [q H + j] (Dv_qj - Dv_q,p-1-j) / 2
  T DvC[HMAX];         // Dv_qH (odd p)
  T DvR[HMAX];         // Dv_Hj (odd p): middle point, from the odd part
  T fAh;               // -|F| c_cons / (2 h): consistency term on reference-coordinate derivatives
  T fG;                // |F| gamma
  T fB0;               // |F| c_sym / 2 (-1/h): symmetry term of side 0
};

// 1D line operator of one direction for kappa = 1, any degree (see
// ScalarArgs::lo): out = K u + L u_left + R u_right along a line.
template <typename T>
struct LineOp {
  // interior K (both sides interior) is centro-symmetric: even/odd blocks
  T Kp[HMAX * HMAX];  // [i H + j] (K_ij + K_i,p-1-j) / 2
  T Km[HMAX * HMAX];  // [i H + j] (K_ij - K_i,p-1-j) / 2
  T Kc[HMAX];         // K_iH (odd p)
  T Kr[HMAX];         // K_Hj (odd p)
  T Kh;               // K_HH (odd p)
  // L = e0 la^T + de0 lb^T (rank 2); R = e1 ra^T + de1 rb^T with ra, rb the
  // mirror images of la, -lb
  T la[PMAX], lb[PMAX];
  // own-cell correction of K on a boundary side s of type t (0 Dirichlet,
  // 1 natural): e_s (cn d_s.u + ce e_s.u) + de_s (cb e_s.u), d_s = reference
  // derivative row of side s
  T bq[2][2][3];      // [t][s] {cn, ce, cb}
};

// Parameter block of the axis-aligned diffusion-reaction kernels. It lives in
// device memory (one copy per precision and kernel variant, written once at
// mesh creation) and the kernels take a pointer to it: every lane uses the
// same entry at the same time, so the reads are scalar loads issued where the
// entry is used. Passed by value instead, the whole block would be loaded into
// scalar registers at kernel entry and spilled.
template <typename T>
struct alignas(16) ScalarArgs {
  T D[PMAX * PMAX];    // D[q*P + j] = l_j'(x_q), collocated (m = p)
  T e[2][PMAX];        // face trace rows
  T de[2][PMAX];       // face derivative rows (reference coordinates)
  T w[PMAX];           // quadrature weights
  T xi[PMAX];          // nodes = quadrature points on [0, 1]
  T vs[3];             // |J| / h_d^2: volume diffusion scale of direction d
  T fs[3];             // |J| / h_d: face area element of faces normal to d
  T hinv[3];           // 1 / h_d
  T gam[3];            // gamma_F of faces normal to d
  T cmass;             // c |J|
  T c_cons, c_sym;     // face term coefficients: (-1, theta) forward, (theta, -1) adjoint
  int32_t n[3];
  int32_t nelem;
  uint32_t mask;       // Dirichlet sides, bit 2d+s
  int32_t kappa_face_one;
  // block order: a block is a chunk of up to EB consecutive cells of one x-row;
  // each XCD sweeps one region of the mesh (x and z split, y outermost inside)
  int32_t nchunk;      // chunks per x-row
  int32_t pad_sweep;
  // per hardware block: (first cell's x index | y << 16, z) of its chunk, in the
  // sweep order with the XCD renumbering applied (table written at mesh creation)
  const uint32_t* blocks;
  // Per-direction tables with the constant factors folded in; a line's
  // tangential weight w_a w_b multiplies its whole result once at the end.
  T Dv[3][PMAX * PMAX];  // (|J|/h_d^2) w_q l_j'(x_q): contraction to the points plus quadrature scaling
  T dno[3][2][PMAX];     // (2s-1)/h_d l_j'(s): outward normal derivative of the own trace at side s
  T dni[3][2][PMAX];     // -(2s-1)/h_d l_j'(1-s): the neighbour's outward normal derivative there
  T cw[PMAX];            // c |J| w_i: mass term
  T fA[3];               // |F_d| c_cons / 2
  T fG[3];               // |F_d| gamma_d
  T fB[3][2];            // |F_d| c_sym / 2 (2s-1)/h_d
  T wl[PMAX * PMAX];     // w_a w_b: tangential weight of the line a + p b
  LineOp<T> lo[3];     // per direction, kappa = 1
  // 1D line operators for kappa = 1 of the matrix-core apply (p = 4): along a
  // line of direction d, out = K u + L u_left + R u_right, where K holds the
  // volume term (and the mass term for d = 0) and the own-cell face terms,
  // L and R the neighbour face terms; row i is divided by w_i, so that the
  // sum over directions times the node's tensor weight is the result.
  // K has one variant per pair of side types (interior, Dirichlet, none):
  // index 3 t0 + t1. Row-major 4 x 4.
  T Km[3][9][16];
  T Lm[3][16];
  T Rm[3][16];
  // per lane of the matrix-core apply: the A operands of the interior cell
  // (Kx, Lx, Rx, Ky, Ly, Ry, Kz, Lz, Rz, entry (lane % 4, lane / 16)), a
  // zero, and the tensor weights of the two nodes the lane holds in the pair
  // layout: one 96-byte record per lane
  double lrec[64][12];
  int32_t p;           // nodes per direction
  // geometry in FP64 for the host-side table builders
  double hd[3], detJd, cd, gamd[3];
  // Even-odd split of the tables (H = p / 2, middle index H when p is odd).
  // The nodes are symmetric about the cell centre, so the derivative matrix
  // is centro-antisymmetric and the face rows of side 1 are the mirror images
  // of those of side 0 (the derivative row with a sign). A line v is carried
  // as ve_j = v_j + v_{p-1-j}, vo_j = v_j - v_{p-1-j} (j < H) and the middle
  // value; an output as half sums oe_i and half differences oo_i
  // (out_i = oe_i + oo_i, out_{p-1-i} = oe_i - oo_i) and the middle value.
  // Only the volume rows depend on the direction.
  EvenOdd<T> eo[3];
  T G2p[HMAX * HMAX];  // [i H + q] D_qi + D_q,p-1-i: transposed contraction of the odd part of r
  T G2m[HMAX * HMAX];  // [i H + q] D_qi - D_q,p-1-i: of the even part
  T Gh[HMAX];          // D_Hi (odd p)
  T G2c[HMAX];         // 2 D_qH (odd p): middle output
  T Ep[HMAX], Em[HMAX], Eh;     // (e0_j +- e0_{p-1-j}) / 2 and e0_H
  T DEp[HMAX], DEm[HMAX], DEh;  // the same of de0
  T cwh[HMAX], cwm;             // c |J| w_i / 2 and c |J| w_H (mass term)
  // Block-Jacobi preconditioner (kappa = 1, axis-aligned cells, theta = -1).
  // The diagonal block of a cell is sum_d W x W x K_d (K_d the unscaled line
  // operator of direction d for the cell's side types, W = diag(w) on the two
  // other directions), so with the generalized eigenpairs K_d V_d =
  // W V_d diag(lam_d), V_d^T W V_d = I, its inverse is
  // (V_z x V_y x V_x) diag(1 / (lam_x + lam_y + lam_z)) (V_z x V_y x V_x)^T.
  // Per direction and side-type variant 3 t0 + t1: fdmV[i p + j] = component
  // i of eigenvector j; fdmL[j] = lam_j.
  T fdmV[3][9][PMAX * PMAX];
  T fdmL[3][9][PMAX];
  int32_t fdm_ok;  // the tables are valid for this mesh
};

// Variants of the parameter block kept per mesh.
enum : int { SP_APPLY = 0, SP_APPLY_T = 1, SP_ADJOINT = 2, SP_COUNT = 3 };

// Kernel arguments of the Stokes kernels (general trilinear geometry).
struct StokesArgs {
  double D[PMAX * PMAX];   // velocity D at the velocity nodes (m = p)
  double Ap[PMAX * PMAX];  // pressure basis at the quadrature points, Ap[q*KP + j]
  double e[2][PMAX], de[2][PMAX];
  double ep[2][PMAX];      // pressure trace rows
  double w[PMAX];
  double xq[PMAX];         // quadrature points (= velocity nodes)
  double theta;
  int32_t n[3];
  int32_t nelem;
  uint32_t mask;
};

}  // namespace dgi

struct dg_mesh {
  dg_mesh_desc desc{};
  int p = 0, m = 0, kp = 0;    // velocity/scalar nodes, quadrature points, pressure nodes
  int64_t nelem = 0, N = 0, ndofs = 0, nqp = 0;
  bool axis_aligned = true;
  int device = 0;
  int num_cu = 0;                 // compute units of the device
  dgi::Tables1D tab;
  dgi::ScalarArgs<double> sd{};
  dgi::ScalarArgs<float> sf{};
  dgi::StokesArgs st{};
  std::vector<double> vertices;   // host copy (perturbed meshes)
  double* d_vertices = nullptr;   // device copy
  double* d_gamma = nullptr;      // per-face penalties [3][faces of direction d]
  double* d_cellgeo = nullptr;    // Stokes: coefficients of every cell's trilinear map
  uint32_t* d_stokes_order = nullptr;  // Stokes: the cell of every block (sweep order)
  // parameter blocks of the diffusion-reaction kernels (host copies and device copies)
  dgi::ScalarArgs<double> pd[dgi::SP_COUNT]{};
  dgi::ScalarArgs<float> pf[dgi::SP_COUNT]{};
  dgi::ScalarArgs<double>* d_pd = nullptr;
  dgi::ScalarArgs<float>* d_pf = nullptr;
  uint32_t* d_blocks = nullptr;  // block tables of the apply and adjoint grids (2 words per block)
  // wavefront tables of the matrix-core applies (2 words per wavefront), one per
  // precision [DG_F64, DG_F32], with their lengths and rows per wavefront
  uint32_t* d_waves[2] = {nullptr, nullptr};
  int64_t nwaves[2] = {0, 0};
  int mfma_rows[2] = {0, 0};
  // variant selection (dg_mesh_set_variant / dg_mesh_tune): the line kernels
  // serve this precision although a matrix-core kernel exists; order of the
  // line kernels' block sweep (0: one region per XCD, 1: linear)
  bool lines_forced[2] = {false, false};
  int sweep_linear = 0;
  // FP32 line kernel of p = 4: contractions on the matrix cores (else VALU)
  bool lines_mfma = false;
  int64_t gamma_off[3] = {0, 0, 0};
};

namespace dgi {
// Launchers (defined next to their kernels). They return the launch status.
// With partial != NULL the apply also writes one partial sum of x_i y_i per
// block (scalar_apply_blocks entries, fixed order): p.Ap for CG.
hipError_t scalar_apply(const dg_mesh& M, int prec, const void* x, void* y, const void* kappa,
                        bool transpose, hipStream_t s, double* partial = nullptr);
int64_t scalar_apply_blocks(const dg_mesh& M, int prec, bool kappa);
// Recomputes the face constants fA, fB of the folded tables from c_cons, c_sym.
template <typename T>
void derive_face_constants(ScalarArgs<T>& a);
hipError_t scalar_adjoint(const dg_mesh& M, int prec, const void* g, const void* u, const void* kappa,
                          void* ATg, void* dkappa, hipStream_t s);
hipError_t scalar_load(const dg_mesh& M, int prec, const void* fq, void* b, hipStream_t s);
// z = B^-1 r for the diagonal cell blocks B (requires the tables' fdm_ok);
// with `partial` != NULL also one partial sum of r.z per block
// (block_jacobi_blocks(M) entries, fixed order).
hipError_t block_jacobi(const dg_mesh& M, int prec, const void* r, void* z, double* partial, hipStream_t s);
// The same after the residual update r -= alpha q (alpha in device memory),
// with partial sums of r.z and of the updated r.r (one pass for PCG).
hipError_t block_jacobi_update(const dg_mesh& M, int prec, void* r, const void* q, const double* alpha, void* z,
                               double* partial_rz, double* partial_rr, hipStream_t s);
int64_t block_jacobi_blocks(const dg_mesh& M);
// One step of the Chebyshev iteration preconditioned by the block-Jacobi
// inverse P (k_cheb_block_jacobi): z += d, d = c1 d + c2 P (rhs - t); the first
// step has t = d = z = 0; the rhs is rd (FP64, rounded) when given, else r;
// with rd the last step writes the partial sums of rd.z
// (block_jacobi_blocks(M) entries) and does not store d.
hipError_t cheb_block_jacobi(const dg_mesh& M, int prec, const void* r, const double* rd, const void* t, void* d,
                             void* z, double c1, double c2, bool first, bool last, double* partial, hipStream_t s);
inline bool block_jacobi_supported(const dg_mesh& M) { return M.pd[SP_APPLY].fdm_ok != 0; }
// One step k >= 1 of the Chebyshev iteration in one pass over the cells (the
// line-kernel apply with the step as its epilogue): t = A z, w = rhs - t
// (bj: w = P (rhs - t)), d = c1 d + c2 w, zout = z + d; the rhs is rd (FP64,
// rounded) when given, else r; with rd the last step writes the partial sums
// of rd.zout (block_jacobi_blocks(M) entries) and does not store d. zout must
// not alias z. bj requires kappa == NULL.
hipError_t cheb_apply(const dg_mesh& M, int prec, const void* z, void* zout, const void* kappa, const void* r,
                      const double* rd, void* d, double c1, double c2, bool last, bool bj, double* partial,
                      hipStream_t s);
// Fills M.pd / M.pf from M.sd / M.sf (face constants per variant, sweep grid,
// line weights) and uploads them to M.d_pd / M.d_pf (allocated by the caller).
hipError_t scalar_params_upload(dg_mesh& M);
// Matrix-core apply of the p = 4, FP64, kappa = 1 operator (variant SP_APPLY or SP_APPLY_T).
bool mfma_apply_supported(const dg_mesh& M, int prec, bool kappa);
hipError_t mfma_apply(const dg_mesh& M, int variant, const double* x, double* y, double* partial, hipStream_t s);
// The same operator on FP32 vectors, computed in FP64 on the matrix cores (the
// FP64 kernel's result for the FP32 input, rounded to FP32).
bool mfma_apply_f32_supported(const dg_mesh& M, int prec, bool kappa);
hipError_t mfma_apply_f32(const dg_mesh& M, int variant, const float* x, float* y, double* partial,
                          hipStream_t s);
// Builds and uploads the wavefront tables of the matrix-core applies
// (M.d_waves) with the rows per wavefront of the cost model.
hipError_t mfma_setup(dg_mesh& M);
// Rebuilds the table of precision slot `prec` with `rows` rows per wavefront
// (0: the cost model's choice).
hipError_t mfma_build(dg_mesh& M, int prec, int rows);
// The cost model's rows per wavefront: the most, up to 16, that leave at
// least 4096 wavefronts (16 per CU), else 1.
int mfma_default_rows(int nx, int ny, int nz);
// Rebuilds the line kernels' block table in the given sweep order (0: one
// region of the mesh per XCD, 1: linear) and re-uploads the parameter blocks.
hipError_t line_sweep_set(dg_mesh& M, int linear);
hipError_t stokes_apply(const dg_mesh& M, const double* x, double* y, hipStream_t s);
// Section 5.2's benchmark operator (K = x x^T + I per point): y = A x (the
// Jacobian action), or with `residual` y = A x - b with its f and g terms.
hipError_t tensor_apply(const dg_mesh& M, int prec, const void* x, void* y, bool transpose, bool residual,
                        hipStream_t s);

// The nonlinear diffusion operator (kappa(u) = 1 + u^2): y = J(u0) z (jac)
// or y = R(u0) (z ignored).
hipError_t nonlinear_apply(const dg_mesh& M, int prec, const void* u0, const void* z, void* y, bool jac,
                           hipStream_t s);

// Vector kernels of the solvers (deterministic fixed-order reductions).
hipError_t blas_dot_partial(const void* a, const void* b, int prec, int64_t n, double* partial,
                            int nblk, hipStream_t s);
int blas_dot_blocks(int64_t n);
}  // namespace dgi

// Error reporting shared by the C entry points.
void dg_set_error(const std::string& msg);
