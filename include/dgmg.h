/*
 * libdgmg -- matrix-free DG operator, block smoothers and hybrid multigrid
 * for high-order DG discretisations on one MI355X (gfx950).
 *
 * Method: Bastian, Mueller, Muething, Piatkowski, "Matrix-free multigrid
 * block-preconditioners for higher order Discontinuous Galerkin
 * discretisations" (arXiv:1805.11930).
 *
 * Problem (Sec. 2, eqns linearproblem / boundary_conditions):
 *     div(b u - K grad u) + c u = f  in a box,
 *     u = g on Dirichlet faces, (b u - K grad u).nu = j on Neumann faces,
 * discretised with the weighted symmetric interior penalty method plus
 * upwind flux (Sec. 2.1, eqn bilinear_form_split, right-hand side eqn rhs)
 * on a uniform Cartesian mesh of hexahedra with a tensor-product nodal
 * Lagrange basis of degree p whose nodes are the p+1 Gauss-Legendre
 * points (collocated with the tensor Gauss quadrature of p+1 points).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Cells: c = ix + nx*(iy + ny*iz).  DOF (jx,jy,jz) of cell c has global
 *    index c*(p+1)^3 + jx + (p+1)*(jy + (p+1)*jz).  Values are nodal.
 *  - Box faces are numbered 0..5 = -x, +x, -y, +y, -z, +z.
 *  - K is diagonal and constant per cell, c constant per cell, and the
 *    advection field affine: b(x) = b0 + B x (B row-major).
 *  - Vectors passed to dg_apply / dg_block_* / dg_mg_vcycle are DEVICE
 *    pointers owned by the caller, contiguous, of type double (DG_FP64) or
 *    float (DG_FP32), 16-byte aligned, and must stay alive until the work
 *    queued on `stream` has completed.  Input and output must not overlap.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *    dg_apply, dg_block_apply, dg_block_smooth and dg_mg_vcycle only
 *    enqueue work and return; calls that fill host results synchronise.
 *  - A problem handle may be used by one stream at a time.
 *  - Every call returns DG_OK (0) or a status below; no exception crosses
 *    the interface.  dg_last_error() returns a text for the last failure
 *    of the calling thread.
 */
#ifndef DGMG_H
#define DGMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes --------------------------------------------------- */
#define DG_OK 0
#define DG_ENOCONV 1     /* finished without reaching rtol; outputs valid   */
#define DG_EAGAIN 2      /* serving: solve still running                     */
#define DG_EINVAL (-1)   /* bad argument (null pointer, p out of range, ...) */
#define DG_ENOMEM (-2)   /* device allocation or admission failure           */
#define DG_EDEVICE (-3)  /* HIP runtime error                                */
#define DG_EBREAKDOWN (-4) /* NaN/Inf or CG breakdown (p^T A p <= 0)         */

#define DG_MAX_P 5       /* polynomial degrees 1..DG_MAX_P are compiled      */

enum { DG_FP64 = 0, DG_FP32 = 1 };
enum { DG_BC_DIRICHLET = 0, DG_BC_NEUMANN = 1 };
enum { DG_INNER_CG = 0, DG_INNER_GMRES = 1, DG_INNER_FDM = 2, DG_INNER_PMF = 3 };
enum { DG_KRYLOV_CG = 0, DG_KRYLOV_FCG = 1, DG_KRYLOV_FGMRES = 2 };
enum { DG_PRECOND_NONE = 0, DG_PRECOND_BLOCK = 1, DG_PRECOND_MG = 2 };
#define DG_PRECOND_BLOCK_JACOBI DG_PRECOND_BLOCK
/* Sweep of the block smoother (Sec. 2.2.1): block-Jacobi (alg
 * block_jacobi), forward or backward block-SOR (alg block_SOR) and
 * block-SSOR (a forward then a backward sweep).  The SOR sweeps visit the
 * cells colour by colour, colour = (ix + iy + iz) mod C (C = 2: red-black;
 * backward: the colours in reverse): cells of one colour share no face, so
 * each colour is swept in parallel, in place.  Larger C moves the order
 * towards the diagonal wavefront order, which is downwind for b with
 * positive components. */
enum { DG_SWEEP_JACOBI = 0, DG_SWEEP_SOR = 1, DG_SWEEP_SSOR = 2, DG_SWEEP_SOR_BACKWARD = 3 };
enum { DG_IPREC_DIAG = 0, DG_IPREC_TRIDIAG = 1 };
enum { DG_COARSE_P0 = 0, DG_COARSE_Q1 = 1, DG_COARSE_AUTO = 2 };
enum { DG_COARSE_SOLVER_GEOMETRIC = 0, DG_COARSE_SOLVER_AMG = 1 };
enum { DG_FIELD_NONE = 0, DG_FIELD_AXIS_QUADRATIC = 1, DG_FIELD_ROTATED_QUADRATIC = 2 };
enum { DG_BASIS_GL = 0, DG_BASIS_GLL = 1 };

typedef struct dg_problem dg_problem;          /* opaque, library-owned */
typedef struct dg_solve_state dg_solve_state;  /* opaque, library-owned */

/* Problem description (Sec. 2 problem statement; Sec. 2.1 discretisation).
 * All arrays are HOST memory and are copied by dg_problem_create. */
typedef struct {
  int nx, ny, nz;          /* cells per direction, >= 1                    */
  double lx, ly, lz;       /* box edge lengths, > 0; box = [0,lx]x[0,ly]x[0,lz] */
  int p;                   /* polynomial degree, 1..DG_MAX_P               */
  int bc[6];               /* DG_BC_DIRICHLET / DG_BC_NEUMANN per box face */
  double penalty_factor;   /* prefactor sigma of gamma_F (Sec. 2.1, penalty
                              definition, which uses alpha p (p+d-1)); <= 0
                              selects 1.25 p (p+2)                         */
  const double *K;         /* [ncell][3] diagonal of K per cell, or NULL    */
  double K_scalar;         /* K = K_scalar * I when K == NULL (must be > 0) */
  const double *c;         /* [ncell] reaction per cell, or NULL            */
  double c_scalar;         /* c when c == NULL                              */
  double b0[3];            /* b(x) = b0 + B x                               */
  double B[9];
  int field;               /* DG_FIELD_NONE (0, default): K and c as above.
                              Otherwise coefficient fields evaluated at the
                              quadrature points of the operator (Sec. 4.2,
                              second diffusion test):
                                K(x) = sum_m P_m(x_m) n_m n_m^T,
                                P_m(s) = kq[m] + kq[3+m] s + kq[6+m] s^2,
                                c(x) = cq[0] + cq[1] (x^2 + y^2 + z^2),
                              with n_m = e_m (DG_FIELD_AXIS_QUADRATIC:
                              K(x) = diag(P_1(x), P_2(y), P_3(z))) or n_m =
                              row m of nrot, an orthonormal basis
                              (DG_FIELD_ROTATED_QUADRATIC: a full tensor).
                              P_m must be > 0 on [0, L_m] and c >= 0 on the
                              box.  K, K_scalar, c, c_scalar are then
                              ignored.  The preconditioner (dg_block_*,
                              dg_mg_vcycle and the preconditioner of
                              dg_solve) works with the field's values at the
                              cell centres, as in the paper (for a full
                              tensor: its diagonal there); dg_apply,
                              dg_assemble_rhs and the outer Krylov method use
                              the field itself.                              */
  double kq[9];
  double cq[2];
  double nrot[9];          /* DG_FIELD_ROTATED_QUADRATIC: rows n_1, n_2, n_3 */
  int basis;               /* nodes of the 1-D Lagrange basis (Sec. 2.1,
                              basis paragraph):
                              DG_BASIS_GL (0, default): the p+1 Gauss-Legendre
                                points, collocated with the quadrature;
                              DG_BASIS_GLL: the p+1 Gauss-Lobatto points (end
                                points included), the paper's choice.
                              Both span Q_p per cell with the same (p+1)-point
                              Gauss quadrature, so the discrete solution as a
                              function is the same; vectors hold the values at
                              the basis nodes (dg_node_points).  With GLL the
                              operator is S^T A S, S = V (x) V (x) V with
                              V[q][j] = GLL polynomial j at Gauss point q
                              (Stage 1 of Sec. 3.1 with a value matrix), and
                              the block smoother solves S^T D_T S (its
                              tridiagonal inner preconditioner takes the
                              band of the whole block, which in this basis
                              also couples consecutive x-lines).  GLL does
                              not support the Q1 coarse space (AUTO selects
                              P0), the fast-diagonalisation and
                              stored-inverse block solves, or the serving
                              entry point dg_solve_start (DG_EINVAL).  The
                              problem holds 7 more DOF-sized vectors per
                              precision (scratch and block entries).       */
} dg_problem_desc;

/* Block smoother options (alg block_jacobi, alg block_SOR, Sec. 2.2.1;
 * inner solve Sec. 3.2). */
typedef struct {
  int n_sweeps;     /* number of smoothing steps (an SSOR step is a forward
                       and a backward sweep), >= 1                          */
  double omega;     /* damping / relaxation: W = omega^-1 D (Jacobi),
                       omega^-1 D + L (SOR)                                 */
  double eps;       /* inner stop: ||d_T - D_T x||_2 <= eps ||d_T||_2       */
  int max_inner;    /* cap on D_T applications per block (<= 0: (p+1)^3)   */
  int inner;        /* DG_INNER_CG (b = 0) or DG_INNER_GMRES, the paper's
                       iterative block solves; DG_INNER_FDM (b = 0 only):
                       exact block solve with stored per-cell factors (fast
                       diagonalisation of the Kronecker-sum block, built on
                       first use; eps, max_inner, restart are ignored);
                       DG_INNER_PMF (any b, p <= 4): the partially
                       matrix-free variant of Sec. 4.1 -- exact block solve
                       with the stored inverse of every block D_T
                       ((p+1)^6 numbers per cell, built on the device on
                       first use in FP64, FP32 its rounding; eps,
                       max_inner, restart, inner_precond are ignored)     */
  int restart;      /* inner GMRES restart length, 1..16 (<= 0: 12)        */
  int zero_guess;   /* 1: u_in is taken as zero and not read                */
  int sweep;        /* DG_SWEEP_* (default DG_SWEEP_JACOBI)                 */
  int inner_precond; /* preconditioner of the inner Krylov method (Sec. 3.2):
                       DG_IPREC_DIAG (default), the diagonal of D_T, or
                       DG_IPREC_TRIDIAG (inner GMRES only): the tridiagonal
                       part of D_T in the x-fastest DOF order, solved by the
                       Thomas algorithm -- for strongly convective blocks,
                       Sec. 4.3                                              */
  int colours;      /* SOR sweeps: number C of colours (ix + iy + iz) mod C
                       of the cell order, 2..64 (<= 0: 2, red-black)        */
} dg_smooth_opts;

/* Optional smoother statistics (filled after a synchronisation). */
typedef struct {
  long long blocks;       /* block solves performed                        */
  long long inner_total;  /* sum of inner iterations                       */
  int inner_max;          /* largest inner iteration count                 */
  double inner_avg;       /* inner_total / blocks                          */
} dg_smooth_stats;

/* Hybrid V-cycle options (alg hybrid_multigrid; coarse subspaces of
 * Sec. 2.2.2-2.2.3).  coarse_space:
 *   DG_COARSE_P0  piecewise constants, one unknown per cell, A_hat = P^T A P
 *                 by the direct formula of App. A.1; coarse solver: a
 *                 structured 2x2x2 aggregation V-cycle (7-point stencils);
 *   DG_COARSE_Q1  continuous trilinears, one unknown per mesh vertex,
 *                 A_hat = a_h on the vertex functions (App. A.2), equal to
 *                 P^T A P; coarse solver: a vertex-grid V-cycle with
 *                 trilinear Galerkin coarsening (27-point stencils), built
 *                 on first use;
 *   DG_COARSE_AUTO (default) Q1 when b = 0, P0 otherwise (the Q1 matrix
 *                 has no upwinding inside the domain, so it is a poor
 *                 coarse model of convection-dominated problems).
 * Both coarse solvers use damped Jacobi and a dense inverse of the
 * coarsest level (<= 128 unknowns), with a fixed number of cycles, so the
 * V-cycle is a fixed linear operator. */
typedef struct {
  int n_pre, n_post;        /* smoothing steps, 0..64                       */
  dg_smooth_opts smooth;    /* smoother (n_sweeps and zero_guess ignored);
                               with DG_SWEEP_SOR the presmoothing sweeps go
                               forward and the postsmoothing ones backward
                               (DG_SWEEP_SOR_BACKWARD: the reverse), so the
                               cycle is symmetric for a symmetric A        */
  int coarse_space;         /* DG_COARSE_P0, DG_COARSE_Q1 or DG_COARSE_AUTO */
  int coarse_cycles;        /* V-cycles of the coarse solver (0 or 1: one)  */
  int coarse_smooth;        /* Jacobi sweeps per level, 0..64; 0 (default):
                               6 when some cell's K_kk / h_k^2 differ by
                               more than a factor 4 between axes, else 4
                               with advection (b != 0) and 2 without     */
  double coarse_omega;      /* Jacobi damping on the coarse levels (<= 0: 2/3) */
  int graph;                /* 1: replay the coarse solve from a HIP graph
                               (captured on first use per option set, kernel
                               nodes only); 0 (default): launch its kernels
                               directly (measured as fast in steady state,
                               and without the capture cost per problem)  */
  int coarse_solver;        /* DG_COARSE_SOLVER_GEOMETRIC (default): the
                               structured cycles above;
                               DG_COARSE_SOLVER_AMG: smoothed-aggregation
                               AMG on the coarse-space matrix (the paper
                               solves the coarse problem by AMG, Sec. 2.2):
                               strength max(|a_ij|, |a_ji|) >= theta
                               sqrt(|a_ii a_jj|) (theta = 0.08, halved per
                               level), greedy aggregation, prolongation
                               smoothed once by damped Jacobi on the
                               filtered matrix, R = P^T, Galerkin coarse
                               matrices, CSR levels down to <= 1024 unknowns
                               (dense inverse).  Set up on the host on first
                               use; cycled on the device with the same
                               damped Jacobi (coarse_smooth, coarse_omega,
                               coarse_cycles) as the geometric solver.     */
  int fuse_small_levels;    /* 1 (default): the small levels of a Q1
                               vertex-grid hierarchy and its dense bottom
                               (at most 1024 unknowns on the first of them,
                               192 KB of coefficients in the working
                               precision) run as one single-workgroup
                               kernel per cycle with their vectors in LDS;
                               the same steps and arithmetic, bit for bit,
                               as one kernel per step (0), which at these
                               sizes is bound by launch latency            */
} dg_mg_opts;

/* Outer solve options (Sec. 4.2: CG to 1e-8; Sec. 4.3: flexible GMRES). */
typedef struct {
  int krylov;               /* DG_KRYLOV_CG / _FCG / _FGMRES                */
  int restart;              /* FGMRES restart (<= 0: 30)                    */
  double rtol;              /* stop when ||f - A u||_2 <= rtol ||f - A u0||_2 */
  int maxit;                /* iteration cap                                */
  int precond;              /* DG_PRECOND_*                                 */
  int precond_precision;    /* DG_FP64 or DG_FP32 (mixed precision)         */
  dg_mg_opts mg;            /* V-cycle options; DG_PRECOND_BLOCK applies
                               mg.smooth.n_sweeps smoother steps (kind
                               mg.smooth.sweep) from a zero guess           */
  const double *u_ref;      /* DEVICE [ndof] reference solution (an exact
                               solution, or the FP64-preconditioned answer
                               that a mixed-precision solve is compared
                               with), or NULL; the result's `error` is then
                               ||u - u_ref||_2 / ||u_ref||_2 in FP64.  Read
                               once at the end of the solve; must not
                               overlap f or u.                              */
  int inner_stats;          /* 1: statistics of the preconditioner: count
                               the inner iterations of every block solve
                               (result inner_avg, inner_max, inner_blocks;
                               one small reduction kernel per smoothing
                               step) and time its phases with HIP events
                               (result t_smoother ... t_prolong).  0
                               (default): neither.                         */
} dg_solve_opts;

typedef struct {
  int status;               /* DG_OK, DG_ENOCONV, DG_EBREAKDOWN             */
  int iters;                /* outer iterations                             */
  double rel_residual;      /* true FP64 ||f - A u||_2 / ||f - A u0||_2     */
  double t_setup, t_solve;  /* seconds                                      */
  double inner_avg;         /* mean inner iterations per block solve inside
                               the preconditioner (opts->inner_stats; else 0) */
  int inner_max;            /* largest inner iteration count (same)         */
  size_t footprint;         /* device bytes held by the problem + solve     */
  double t_apply;           /* seconds in FP64 operator-apply kernels (HIP
                               events on the solve's stream)                */
  int n_apply;              /* number of those applies                      */
  double t_precond;         /* seconds in the preconditioner (HIP events)   */
  int n_precond;            /* preconditioner applications                  */
  double error;             /* ||u - u_ref||_2 / ||u_ref||_2 (FP64), or -1
                               when opts->u_ref is NULL                     */
  long long inner_blocks;   /* block solves counted (opts->inner_stats)     */
  /* seconds in the phases of the preconditioner (opts->inner_stats; else
     0): block smoothing steps (with the P0 prolongation that is fused into
     the first postsmoothing step), residual + restriction to the coarse
     space, coarse solve, Q1 prolongation */
  double t_smoother, t_restrict, t_coarse, t_prolong;
} dg_solve_result;

/* ---- problem lifetime ---------------------------------------------- */
/* Validates the description (DG_EINVAL on nx,ny,nz < 1, lengths <= 0,
 * p outside 1..DG_MAX_P, bad bc, K not finite or <= 0, c not finite or
 * < 0, non-finite b), copies coefficients to the device and builds the
 * 1-D tables and the P0 coarse hierarchy.  *out is NULL on failure. */
int dg_problem_create(const dg_problem_desc *desc, dg_problem **out);
void dg_problem_destroy(dg_problem *prob);
const char *dg_last_error(void);

/* Number of DOFs (ncell (p+1)^3) and of boundary quadrature points. */
int64_t dg_ndof(const dg_problem *prob);
int64_t dg_boundary_npoints(const dg_problem *prob);

/* Physical coordinates, HOST output [ndof][3], of the DOF nodes: the
 * Gauss points (DG_BASIS_GL) or the Gauss-Lobatto points (DG_BASIS_GLL) of
 * each cell, in DOF order. */
int dg_node_points(const dg_problem *prob, double *xyz);
/* Physical coordinates, HOST output [ndof][3], of the volume quadrature
 * points (the (p+1)^3 Gauss points of each cell, in DOF order) at which
 * dg_assemble_rhs takes f.  Equal to dg_node_points for DG_BASIS_GL. */
int dg_quadrature_points(const dg_problem *prob, double *xyz);
/* Physical coordinates, HOST output [npts][3], of the boundary face
 * quadrature points: box faces 0..5 in order; on each box face, the faces
 * of the boundary cells with the first tangential cell index fastest
 * (tangential axes in increasing order), and on each cell face the
 * (p+1)^2 Gauss points, first tangential coordinate fastest. */
int dg_boundary_points(const dg_problem *prob, double *xyz);

/* Right-hand side l_h(psi_i) (eqn rhs).  f_qp: DEVICE [ndof] values of f
 * at the volume quadrature points (NULL = 0).  bnd_qp: DEVICE [npts]
 * values at the boundary points, read as g on Dirichlet faces and as j on
 * Neumann faces (NULL = 0).  rhs: DEVICE [ndof] double output. */
int dg_assemble_rhs(dg_problem *prob, const double *f_qp, const double *bnd_qp, double *rhs,
                    void *stream);

/* ---- hot path -------------------------------------------------------- */
/* v = A u, A_ij = a_h(psi_j, psi_i) (eqn linear_equation), matrix-free by
 * sum factorisation (Sec. 3.1): volume, interior-face and boundary-face
 * terms.  precision: DG_FP64 (double vectors) or DG_FP32 (float vectors). */
int dg_apply(dg_problem *prob, int precision, const void *u, void *v, void *stream);

/* y_T = D_T x_T for every cell T, D_T = A_{T,T} (eqn block_diag_apply). */
int dg_block_apply(dg_problem *prob, int precision, const void *x, void *y, void *stream);

/* diag(D_T) for every cell, DEVICE [ndof] output (Sec. 3.2, the diagonal
 * preconditioner of the inner solve). */
int dg_block_diag(dg_problem *prob, int precision, void *diag, void *stream);

/* x_T ~= D_T^-1 d_T for every cell by the inner Krylov method of
 * dg_block_smooth (eqn block_system, Sec. 2.2.1 / 3.2).  iters: DEVICE
 * [ncell] int output of inner iterations per block, or NULL. */
int dg_block_solve(dg_problem *prob, int precision, const void *d, void *x,
                   const dg_smooth_opts *opts, int *iters, void *stream);

/* n_sweeps smoothing steps from u^(0) = u_in (or 0 when opts->zero_guess),
 * result in u_out; stats (nullable) forces a synchronisation.
 *   DG_SWEEP_JACOBI (alg block_jacobi):
 *     u^(k) = u^(k-1) + omega D^-1_eps (f - A u^(k-1));  u_in != u_out.
 *   DG_SWEEP_SOR / _SOR_BACKWARD / _SSOR (alg block_SOR): per cell T, in
 *     the colour order (opts->colours), d_T = f_T - sum over the face neighbours S of
 *     A_{T,S} u_S (current values), D_T x = d_T solved to eps, then
 *     u_T = (1 - omega) u_T + omega x, in place in u_out (u_in may equal
 *     u_out; otherwise u_in is copied first). */
int dg_block_smooth(dg_problem *prob, int precision, const void *f, const void *u_in, void *u_out,
                    const dg_smooth_opts *opts, dg_smooth_stats *stats, void *stream);

/* dg_block_smooth without device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same smoothing steps, kernels and results
 * as dg_block_smooth, but its scratch -- the ping-pong vector of
 * block-Jacobi with n_sweeps > 1, and with stats the per-cell inner
 * iteration counts and their reduction -- lives in a fixed device array of
 * 128 MiB (134217728 bytes) that each GPU the library runs on holds until
 * the process ends.  Needs at most ndof * sizeof(element) + ncell * 4 +
 * 768 bytes (rounded up to 256-byte parts); a call that needs more fails
 * with DG_EINVAL, as does DG_INNER_FDM before its stored factors exist (a
 * dg_block_smooth call with DG_INNER_FDM builds them) and a problem created
 * on a device other than the current one.  The first call on a device
 * looks up that device's copy of the array.  Every call on one GPU shares
 * that GPU's array: calls that overlap on one GPU (different streams or
 * threads) race and must be serialised by the caller.  No part of the
 * array needs to start at zero: each call writes what it reads. */
int dg_block_smooth_noalloc(dg_problem *prob, int precision, const void *f, const void *u_in, void *u_out,
                            const dg_smooth_opts *opts, dg_smooth_stats *stats, void *stream);

/* z ~= A^-1 r by one hybrid V-cycle from a zero initial guess
 * (alg hybrid_multigrid): presmooth, residual, restriction R = P^T
 * (Sec. 2.2.2), coarse correction with A_hat = P^T A P in the P0 or Q1
 * subspace (App. A.1 / A.2; the Q1 hierarchy is built on the first call
 * that asks for it, a synchronous host setup), prolongation, postsmooth. */
int dg_mg_vcycle(dg_problem *prob, int precision, const void *r, void *z, const dg_mg_opts *opts,
                 void *stream);

/* Solve A u = f with an FP64 outer Krylov method preconditioned by the
 * V-cycle (or block-Jacobi) in precond_precision.  f, u: DEVICE double
 * [ndof]; u holds the initial guess on entry and the solution on return.
 * Synchronises; fills *res (nullable). */
int dg_solve(dg_problem *prob, const double *f, double *u, const dg_solve_opts *opts,
             dg_solve_result *res, void *stream);

/* Coarse-hierarchy introspection (tests, diagnostics).  Level `level` of
 * the DG_COARSE_P0 or DG_COARSE_Q1 hierarchy (built if needed; level 0 is
 * the coarse space itself, A_hat = P^T A P): dims (HOST int[5]) receives
 * (vx, vy, vz, ns, nlevels), the grid of unknowns (x fastest), the stencil
 * width (7: diag, -x, +x, -y, +y, -z, +z; 27: o = (dx+1) + 3 (dy+1) +
 * 9 (dz+1) for the coupling to the unknown at offset (dx, dy, dz)) and the
 * number of levels.  When out is not NULL it receives the FP64 stencil,
 * HOST [ns][vx*vy*vz].  Synchronous.  DG_EINVAL for a level out of range. */
int dg_coarse_stencil(dg_problem *prob, int coarse_space, int level, int *dims, double *out);
/* The aggregation-AMG hierarchy of the P0 or Q1 coarse space (built if
 * needed): level 0 is the coarse-space matrix A_hat itself, level l >= 1
 * the Galerkin product A_l = R_l A_(l-1) P_l.  which = 0: A_l; 1: P_l
 * (rows: unknowns of level l-1, columns: of level l); 2: R_l = P_l^T
 * (level >= 1 for 1 and 2).  dims (HOST int64[4]) receives (rows, cols,
 * nnz, nlevels); when row_ptr is not NULL, HOST arrays row_ptr [rows+1],
 * col [nnz] and val [nnz] receive the FP64 CSR matrix (sorted columns).
 * Synchronous.  DG_EINVAL for a level or matrix out of range. */
int dg_coarse_csr(dg_problem *prob, int coarse_space, int level, int which, int64_t *dims, int *row_ptr, int *col,
                  double *val);

/* ---- resident solves and continuous batching ---------------------- */
/* Start an outer CG / flexible-CG solve of A u = f (options as dg_solve;
 * FGMRES is not available here) that stays resident on the device: the
 * state owns its workspace and a HIP stream of default priority, computes
 * the initial residual and first preconditioned residual, and returns.
 * f and u (DEVICE double [ndof], caller-owned) must stay valid until the
 * state is destroyed; u holds the initial guess and receives the solution.
 * One state per problem handle at a time (a problem's V-cycle temporaries
 * are shared by its solves).  DG_ENOMEM when the workspace does not fit. */
int dg_solve_start(dg_problem *prob, const double *f, double *u, const dg_solve_opts *opts,
                   dg_solve_state **out);
/* One step of every unfinished state in active[0..n_active): take the
 * convergence decision of the outer iteration in flight (waiting only for
 * that state's residual norm, while its preconditioner still runs) and
 * enqueue the next iteration on the state's stream.  An iteration (apply,
 * update, precondition) is enqueued as a whole with its scalars in device
 * memory, so requests of different sizes and degrees overlap on the device
 * and the device does not idle between iterations.  A solve of k
 * iterations takes k + 1 steps (the last one only decides).  A request's
 * arithmetic is the same alone and in any batch.  `stream` is not used
 * (reserved). */
int dg_batch_step(dg_solve_state **active, int n_active, void *stream);
/* DG_EAGAIN while the solve runs; DG_OK once finished, with *res (nullable)
 * filled (its status is DG_OK, DG_ENOCONV or DG_EBREAKDOWN). */
int dg_solve_poll(dg_solve_state *state, dg_solve_result *res);
void dg_solve_state_destroy(dg_solve_state *state);

/* Device bytes the library would hold for this problem and solve. */
int dg_footprint(const dg_problem_desc *desc, const dg_solve_opts *opts, size_t *bytes);

/* ---- defaults ------------------------------------------------------- */
/* smoother: n_sweeps 1, omega 0.8, eps 1e-2 (the paper's choice),
 *   max_inner (p+1)^3, inner CG, restart 12;
 * V-cycle: n_pre = n_post = 1, coarse_space AUTO, coarse_cycles 1,
 *   coarse_smooth 0 (2 or 6 by anisotropy), coarse_omega 2/3, graph 0,
 *   coarse_solver GEOMETRIC, fuse_small_levels 1;
 * solve: FCG, restart 30, rtol 1e-8, maxit 500, MG preconditioner in FP32. */
void dg_default_smooth_opts(dg_smooth_opts *o);
void dg_default_mg_opts(dg_mg_opts *o);
void dg_default_solve_opts(dg_solve_opts *o);

#ifdef __cplusplus
}
#endif
#endif /* DGMG_H */
