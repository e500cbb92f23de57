/*
 * dg.h - matrix-free application of interior-penalty DG operators on
 * hexahedral Q_k meshes by sum factorization, on AMD Instinct MI355X (gfx950).
 *
 * The operator is the Jacobian action A z of the DG residual (Section 2.1 of
 * Kempf, Hess, Muething, Bastian, "Automatic Code Generation for
 * High-Performance Discontinuous Galerkin Methods on Modern Architectures"):
 * for the linear problems here, the residual without its u-independent
 * terms. The problems:
 *
 *   DG_PROBLEM_DIFFREAC  -div(kappa grad u) + c u, symmetric interior penalty
 *                        (Section 5.2, eq. diffreac_weak), Nitsche terms on
 *                        the Dirichlet sides;
 *   DG_PROBLEM_STOKES    velocity Q_k^3 / pressure Q_{k-1} DG Stokes
 *                        (Section 5.3, eq. stokes_weak), mu = 1;
 *   DG_PROBLEM_DIFFREAC_PAPER  Section 5.2's benchmark problem: the same SIPG
 *                        form with the full tensor K(x) = x x^T + I evaluated
 *                        at every quadrature point, reaction c (the paper
 *                        uses 10), source f = -6 and Dirichlet data
 *                        g(x) = |x|^2 on the Dirichlet sides; dg_apply is its
 *                        Jacobian action, dg_residual its full residual;
 *   DG_PROBLEM_NONLINEAR -div(kappa(u) grad u) + c u with kappa(u) = 1 + u^2:
 *                        the same SIPG form with the coefficient evaluated at
 *                        the solution (kappa on a face from each side's own
 *                        trace), homogeneous Dirichlet data on the Dirichlet
 *                        sides; dg_residual is its residual R(u) (the source
 *                        term is a load vector, dg_load_vector), and
 *                        dg_apply_jacobian its Jacobian action J(u0) z at a
 *                        linearization point u0 (Section 2.1).
 *
 * Meshes are structured nx*ny*nz hexahedra of the unit cube, cell
 * e = ex + nx*(ey + ny*ez). Each cell is the image of [0,1]^3 under the
 * trilinear map of its 8 vertices (Section 2.1).
 *
 * Vector layout ("element-blocked, tensor-lexicographic"): a DOF vector holds
 * one contiguous block per cell, cells in increasing e. Inside a block, the
 * nodal coefficient at Gauss-Legendre node (i0, i1, i2) sits at
 * i0 + p*(i1 + p*i2), p = k+1 (x index fastest). A Stokes block is
 * [u_0 (p^3) | u_1 (p^3) | u_2 (p^3) | pressure (k^3)]. kappa and dkappa use
 * the same layout over the m^3 volume quadrature points of each cell.
 *
 * Conventions for every call:
 *  - Vectors are caller-owned DEVICE pointers (e.g. torch tensors' data_ptr()),
 *    contiguous, 16-byte aligned, of the element type selected by
 *    `precision` (DG_F64: double, DG_F32: float). The library never frees
 *    them. Outputs are overwritten, never accumulated into. Inputs and
 *    outputs must not overlap (DG_ERR_ARG).
 *  - `stream` is a hipStream_t (NULL = the null stream). dg_apply,
 *    dg_apply_adjoint and dg_load_vector only enqueue work and return;
 *    dg_solve and dg_mesh_create synchronize the stream before they return.
 *  - A negative status means the call had no effect; dg_last_error() then
 *    returns a message (thread-local, valid until the next call on the same
 *    thread). Argument checks run before any HIP call, so they are usable
 *    without a GPU. No C++ exception crosses this interface.
 */
#ifndef DG_H
#define DG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dg_mesh dg_mesh; /* opaque; owns its device-side tables */

typedef enum {
  DG_OK = 0,
  DG_ERR_ARG = -1,          /* invalid argument, null or overlapping pointers */
  DG_ERR_UNSUPPORTED = -2,  /* valid but not implemented (degree, rule, geometry) */
  DG_ERR_DEVICE = -3,       /* a HIP call failed; message from hipGetErrorString */
  DG_ERR_ALLOC = -4,        /* device or host allocation failed */
  DG_NOT_CONVERGED = 1,     /* dg_solve hit maxit; x and info are still filled */
  DG_BREAKDOWN = 2          /* dg_solve met p^T A p <= 0 or a non-finite value */
} dg_status;

enum { DG_PROBLEM_DIFFREAC = 0, DG_PROBLEM_STOKES = 1, DG_PROBLEM_DIFFREAC_PAPER = 2, DG_PROBLEM_NONLINEAR = 3 };
enum { DG_F64 = 0, DG_F32 = 1 };
enum { DG_KAPPA_ONE = 0, DG_KAPPA_QP = 1 };
enum { DG_KAPPA_FACE_TRACE = 0, DG_KAPPA_FACE_ONE = 1 };
enum { DG_SOLVE_CG_F64 = 0, DG_SOLVE_IR_F32 = 1, DG_SOLVE_RU_F32 = 2, DG_SOLVE_CHEB_F64 = 3,
       DG_SOLVE_CHEB_F32 = 4 };
enum { DG_PRECOND_NONE = 0, DG_PRECOND_BLOCK_JACOBI = 1 };
enum { DG_VARIANT_MATRIX_CORE = 0, DG_VARIANT_LINES = 1 };
enum { DG_TUNE_MAX = 16 };

/* Mesh and operator description (all fields are read by dg_mesh_create). */
typedef struct {
  int32_t nx, ny, nz;       /* cells per direction, 1 .. 65535 */
  int32_t k;                /* polynomial degree (velocity degree for Stokes) */
  int32_t m;                /* Gauss-Legendre points per direction; 0 -> k + 1 */
  int32_t problem;          /* DG_PROBLEM_* */
  double c;                 /* reaction coefficient (diffusion-reaction) */
  double alpha;             /* penalty parameter (the paper uses 3) */
  double theta;             /* -1: symmetric interior penalty (the paper's choice) */
  int32_t penalty_form;     /* 0: gamma_F = alpha k(k+1)|F|/min|T|,
                               1: gamma_F = alpha k(k+d-1)|F|/min|T| (Section 5.2) */
  uint32_t dirichlet_mask;  /* bit 2d+s: side s (0 low, 1 high) of direction d is
                               Dirichlet (Nitsche terms); other sides are natural */
  const double* vertices;   /* HOST pointer, (nz+1)(ny+1)(nx+1) x 3 coordinates,
                               x index fastest; NULL = regular grid i/n. Copied. */
  int32_t kappa_mode;       /* DG_KAPPA_ONE, or DG_KAPPA_QP: kappa per volume
                               quadrature point is passed to every apply */
  int32_t kappa_face;       /* DG_KAPPA_FACE_TRACE: kappa on a face is the cell's
                               interpolant of its point values; DG_KAPPA_FACE_ONE: 1 */
} dg_mesh_desc;

typedef struct {
  int64_t nelem;            /* cells */
  int64_t ndofs;            /* length of a DOF vector */
  int64_t dofs_per_elem;    /* p^3 (diffusion-reaction) or 3 p^3 + k^3 (Stokes) */
  int64_t nqp;              /* length of a kappa vector: nelem * m^3 */
  int32_t p, m;             /* 1D basis nodes and quadrature points */
  int32_t axis_aligned;     /* 1 when the mesh is the regular grid */
  double flops_apply;       /* algorithmic flops of one dg_apply (model of the kernels) */
  double flops_adjoint;     /* ... of one dg_apply_adjoint with dkappa */
  double bytes_apply[2];    /* compulsory HBM bytes of one dg_apply, [DG_F64, DG_F32] */
  double bytes_adjoint;     /* ... of one FP64 dg_apply_adjoint with dkappa */
} dg_mesh_info_t;

typedef struct {
  double rtol;              /* stop when ||b - A x||_2 <= rtol ||b||_2 (true FP64 residual) */
  double inner_rtol;        /* IR: relative residual target of each FP32 inner solve;
                               RU: residual drop between two corrections (0.1 unless in [1e-3, 1)) */
  int32_t maxit;            /* CG: iterations; IR: total inner iterations */
  int32_t max_outer;        /* IR: refinement steps */
  int32_t check_every;      /* read the residual norm to the host every n iterations */
  int32_t precond;          /* DG_PRECOND_*: preconditioner of every CG in the solve (FP64 CG
                               and the FP32 inner CG alike; CHEB: of the Chebyshev iteration) */
  int32_t cheb_degree;      /* CHEB: steps s of the inner Chebyshev iteration, 1..64 (0 -> 8) */
  int32_t cheb_lanczos;     /* CHEB: CG iterations on a pseudo-random right-hand side whose
                               Lanczos coefficients estimate the largest eigenvalue, 2..64 (0 -> 20) */
  double cheb_ratio;        /* CHEB: b / a of the Chebyshev interval [a, b], > 1 (0 -> max(s^2, 16)) */
  double cheb_margin;       /* CHEB: b = margin x the largest Ritz value, >= 1 (0 -> 1.1) */
} dg_solve_params;

typedef struct {
  int32_t iterations;       /* CG iterations (FP64 CG; CHEB: FP64 CG iterations, the first
                               cheb_lanczos unpreconditioned by the polynomial included)
                               or total inner iterations (IR, RU) */
  int32_t outer;            /* refinement steps / residual replacements (0 for FP64 CG) */
  double rel_residual;      /* true ||b - A x||_2 / ||b||_2 in FP64 at exit */
  double seconds;           /* wall time of the solve, host clock */
  int32_t inner_applies;    /* CHEB: operator applies of the inner Chebyshev iterations */
  int32_t lanczos_iterations; /* CHEB: CG iterations on the pseudo-random right-hand side
                                 (the estimate's own, not in iterations) */
  double lambda_max;        /* CHEB: the largest Ritz value of the estimate (of P A, or of A) */
} dg_solve_info;

/* Result of dg_mesh_tune: the candidates timed, in order, and the one chosen. */
typedef struct {
  int32_t ncand;                 /* candidates timed */
  int32_t chosen;                /* index of the fastest, now in use */
  int32_t kind[DG_TUNE_MAX];     /* DG_VARIANT_* */
  int32_t param[DG_TUNE_MAX];    /* MATRIX_CORE: rows per wavefront; LINES: sweep order */
  double us[DG_TUNE_MAX];        /* median microseconds per apply */
} dg_tune_result;

/* Checks a descriptor without touching the GPU (Section 2.1 restrictions:
 * cuboid meshes, isotropic degree). DG_OK, DG_ERR_ARG or DG_ERR_UNSUPPORTED. */
dg_status dg_mesh_desc_validate(const dg_mesh_desc* desc);

/* Builds the 1D Gauss-Legendre rule and nodal Lagrange tables (Section 2.2:
 * the basis matrices A and D and the face rows), geometry and penalties, and
 * uploads what the kernels need to the current device. Synchronous. */
dg_status dg_mesh_create(const dg_mesh_desc* desc, void* stream, dg_mesh** out);
dg_status dg_mesh_destroy(dg_mesh* mesh);
dg_status dg_mesh_info(const dg_mesh* mesh, dg_mesh_info_t* out);

/* y = A x: one matrix-free operator application by sum factorization
 * (Algorithm 1 for the cell integrals; facet integrals with the normal
 * direction contracted first, Section 2.2). kappa: device pointer, nqp values,
 * required iff kappa_mode == DG_KAPPA_QP, else ignored (may be NULL).
 * Each output entry is written exactly once; results are bitwise reproducible.
 * DG_F32: the vectors are float. For k = 3 with kappa_mode DG_KAPPA_ONE the
 * products run in FP64 (y is the FP64 result for the float x, rounded once to
 * float); otherwise the arithmetic is FP32 on tables rounded once from FP64. */
dg_status dg_apply(const dg_mesh* mesh, int precision, const void* x, void* y,
                   const void* kappa, void* stream);

/* ATg = A(kappa)^T g and, if dkappa != NULL, dkappa = dL/dkappa for
 * L = g^T A(kappa) u (the vector-Jacobian product of dg_apply). Diffusion-
 * reaction only; u is required iff dkappa != NULL. */
dg_status dg_apply_adjoint(const dg_mesh* mesh, int precision, const void* g, const void* u,
                           const void* kappa, void* ATg, void* dkappa, void* stream);

/* z = P r, P the block-Jacobi preconditioner: on every cell T, z_T = B_T^-1 r_T
 * with B_T the diagonal block of A (the cell's volume terms and its own face
 * terms). On the axis-aligned cells with kappa = 1, B_T is a sum of
 * Kronecker products of 1D operators and is inverted exactly by fast
 * diagonalization (the element block-Jacobi / fast diagonalization
 * preconditioners cited in Section 1): per direction, the generalized
 * eigenvectors of the 1D operator against the diagonal GL mass, contracted
 * along the three directions, a pointwise division, and the transposed
 * contractions. Diffusion-reaction with kappa_mode DG_KAPPA_ONE and
 * theta = -1 (else DG_ERR_UNSUPPORTED); FP64 or FP32. Asynchronous. */
dg_status dg_precond_apply(const dg_mesh* mesh, int precision, const void* r, void* z, void* stream);

/* Solves A x = b (diffusion-reaction, theta = -1, so A is SPD) by CG,
 * unpreconditioned or with the block-Jacobi preconditioner (params->precond,
 * same requirements as dg_precond_apply). Convergence is always judged on the true FP64
 * residual ||b - A x||_2 <= rtol ||b||_2.
 *  DG_SOLVE_CG_F64: FP64 throughout.
 *  DG_SOLVE_IR_F32: classic iterative refinement: outer residual b - A x in
 *    FP64, a fresh inner CG on the FP32 operator (FP32 vectors, FP64 inner
 *    products) to inner_rtol, FP64 solution update.
 *  DG_SOLVE_RU_F32: refinement that keeps the inner Krylov space: one FP32
 *    CG runs throughout; whenever its residual has dropped by inner_rtol
 *    since the last correction (checked every check_every iterations), the FP32
 *    iterate is added to x in FP64, the residual is replaced by the true
 *    FP64 b - A x and the search direction is kept.
 *  DG_SOLVE_CHEB_F32: FP64 CG preconditioned by a fixed polynomial of the
 *    FP32 operator: each CG iteration (FP64 apply, FP64 residual, inner
 *    products and update) solves A z = r approximately by s steps of the
 *    Chebyshev iteration on the FP32 operator (FP32 vectors, s - 1 FP32
 *    applies; with the block-Jacobi preconditioner P, the Chebyshev
 *    iteration of P A). The iteration has no inner products, so FP32
 *    rounding does not accumulate through a Krylov recursion. Its interval
 *    [b / cheb_ratio, b] comes from b = cheb_margin x the larger of two
 *    largest Ritz values: of cheb_lanczos (P)CG iterations in the inner
 *    precision on a fixed pseudo-random right-hand side (every eigenvector
 *    present: started from a smooth b alone the Krylov space can miss the
 *    top of the spectrum, and an even-degree polynomial is then indefinite
 *    there), and of the first cheb_lanczos FP64 (P)CG iterations of the
 *    solve (which advance x as well).
 *  DG_SOLVE_CHEB_F64: the same with the inner iteration in FP64 (the
 *    baseline that isolates the gain of the FP32 inner work).
 * b, x: device FP64 vectors; x holds the initial guess on entry. kappa as in
 * dg_apply (FP64 values; the FP32 operator rounds them). Synchronous. */
dg_status dg_solve(const dg_mesh* mesh, int mode, const double* b, double* x, const void* kappa,
                   const dg_solve_params* params, dg_solve_info* info, void* stream);

/* y = J(u0) z: the Jacobian action of DG_PROBLEM_NONLINEAR's residual at the
 * linearization point u0 in the direction z (Section 2.1; with kappa(u) =
 * 1 + u^2 it depends on both inputs, which the kernel evaluates in one fused
 * pass, Section 3.1). J is not symmetric. Diffusion-reaction vector rules;
 * y must not overlap u0 or z (u0 and z may be the same vector). Other
 * problems: DG_ERR_UNSUPPORTED (their Jacobian action is dg_apply). Async. */
dg_status dg_apply_jacobian(const dg_mesh* mesh, int precision, const void* u0, const void* z, void* y,
                            void* stream);

/* dg_solve without allocating: for callers that cannot allocate device or
 * pinned host memory (code under HIP graph capture, serving loops, harnesses
 * that forbid hipMalloc). Same arguments, checks, results and status codes as
 * dg_solve (the same kernels in the same order, so x and info match dg_solve
 * bitwise), but its vectors, partial sums and CG state live in one fixed
 * 64 MiB device array per GPU, held until the process ends, and the state is
 * read back to ordinary host memory. A solve needs about 24 bytes per DOF
 * (FP64 CG), 32 (FP64 CG with block-Jacobi), 36-40 (the FP32 refinement
 * modes) or 40-48 (the Chebyshev modes), so meshes up to about 1.3 million
 * DOFs fit in every mode; a larger one returns DG_ERR_ARG with the bytes it
 * would need. Every call on a GPU
 * uses that GPU's one array: calls that overlap in time on the same GPU (from
 * several threads or streams) race and must be serialized by the caller. The
 * array keeps the last call's contents; every piece of it is written before
 * it is read. Synchronous, like dg_solve. */
dg_status dg_solve_noalloc(const dg_mesh* mesh, int mode, const double* b, double* x, const void* kappa,
                           const dg_solve_params* params, dg_solve_info* info, void* stream);

/* r = R(u): the algebraic residual R_i(u) = r(u_h, phi_i) of the problem
 * (Section 2.1). DG_PROBLEM_DIFFREAC_PAPER: eq. diffreac_weak with
 * K = x x^T + I, f = -6 and g = |x|^2, u-independent terms included, i.e.
 * r = A u - b with b the source and Dirichlet data terms.
 * DG_PROBLEM_NONLINEAR: r = R(u) without the source term (subtract
 * dg_load_vector's b for -div(kappa(u) grad u) + c u = f).
 * Other problems: DG_ERR_UNSUPPORTED. Same vector rules as dg_apply. Async. */
dg_status dg_residual(const dg_mesh* mesh, int precision, const void* u, void* r, void* stream);

/* Variant selection for dg_apply (and the solvers' applies) of one precision
 * on this mesh, the counterpart of Section 4.2's choice among vectorization
 * strategies (Algorithms 4 and 5 with a measured cost function). The
 * candidates are:
 *   DG_VARIANT_MATRIX_CORE, param = rows per wavefront (1, 2, 4, 8, 16): the
 *     matrix-core kernel (k = 3, kappa = 1, diffusion-reaction), each
 *     wavefront marching along y over that many rows;
 *   DG_VARIANT_LINES, param = sweep order (bit 0; 0: each XCD sweeps one
 *     region of the mesh, 1: linear order) | 2 for the FP32 line kernel of
 *     k = 3 with its two contractions on the matrix cores
 *     (v_mfma_f32_4x4x1_16b_f32, FP32 accumulation; else FP32 VALU): the
 *     line kernels (thread per 1D line).
 * Without a call the cost model's choice is in use: the matrix-core kernel
 * where it exists, with the most rows (up to 16) that leave at least 4096
 * wavefronts, and the region sweep. The matrix-core kernel exists for k = 3,
 * kappa = 1, diffusion-reaction, on meshes whose x-y planes hold at most about
 * two million cells (a wavefront addresses two planes of FP64 values with
 * 32-bit byte offsets); larger planes run the line kernels. All variants compute the same operator;
 * the matrix-core variants and the two sweep orders give bitwise the same
 * results among themselves. The sweep order is shared by both precisions and
 * by the other line kernels of the mesh (preconditioner, adjoint, load
 * vector). Not thread-safe against calls using the mesh; synchronizes the
 * device when a table is replaced. Stokes: DG_ERR_UNSUPPORTED. */
dg_status dg_mesh_set_variant(dg_mesh* mesh, int precision, int kind, int param);

/* Times every candidate variant of dg_apply for `precision` on this mesh
 * (median over `trials` of 10 applies each, on internal zero vectors; the
 * measured autotuning cost function of Section 4.2) and keeps the fastest in
 * use. Allocates and frees two vectors; synchronous. trials in 1..100. */
dg_status dg_mesh_tune(dg_mesh* mesh, int precision, int trials, void* stream, dg_tune_result* out);

/* Physical coordinates of the volume quadrature points, nqp x 3 doubles into a
 * HOST buffer (cell-blocked, same order as kappa). */
dg_status dg_mesh_qpoints(const dg_mesh* mesh, double* xyz);

/* Load vector b_i = sum_q w_q |det J_q| f_q phi_i(x_q) for f given at the volume
 * quadrature points (device, nqp values); diffusion-reaction, m = k+1. Async. */
dg_status dg_load_vector(const dg_mesh* mesh, int precision, const void* fq, void* b, void* stream);

const char* dg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DG_H */
