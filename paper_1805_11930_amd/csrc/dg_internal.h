// Internal declarations of libdgmg (not part of the public interface).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dgmg.h"
#include "ctables.h"

namespace dgmg {

constexpr int kMaxN = DG_MAX_P + 1;

// Face kinds of a cell side.
enum FaceKind : int { FACE_INTERIOR = 0, FACE_DIRICHLET = 1, FACE_NEUMANN = 2 };

// 1-D tables of the Gauss-Legendre nodal basis on [0,1] (double, host).
// D[q][j] = l_j'(xi_q); S = D^T W D; end values / derivatives of l_j.
struct Tables1D {
  int n = 0;
  double xi[kMaxN], w[kMaxN];
  double D[kMaxN][kMaxN];
  double S[kMaxN][kMaxN];
  double e0[kMaxN], e1[kMaxN], d0[kMaxN], d1[kMaxN];
};
void build_tables(int n, Tables1D &t);
void gll_nodes(int n, double *xi);  // the n Gauss-Lobatto points on [0,1]

// Kernel-side copy of the tables in the compute precision, built at compile
// time from the constexpr tables (ctables.h); inside kernels every entry is
// a literal.  N is fixed at compile time; every loop over it unrolls.
template <typename T, int N>
struct DevTab {
  T S[N][N] = {};   // D^T diag(w) D
  T Dt[N][N] = {};  // Dt[i][q] = D[q][i]
  T w[N] = {}, xi[N] = {}, e0[N] = {}, e1[N] = {}, d0[N] = {}, d1[N] = {};
};

template <typename T, int N>
constexpr DevTab<T, N> make_ctab() {
  constexpr ct::Tab<N> t = ct::make_tab<N>();
  DevTab<T, N> d;
  for (int i = 0; i < N; ++i) {
    for (int j = 0; j < N; ++j) {
      d.S[i][j] = (T)t.S[i][j];
      d.Dt[i][j] = (T)t.D[j][i];
    }
    d.w[i] = (T)t.w[i];
    d.xi[i] = (T)t.xi[i];
    d.e0[i] = (T)t.e0[i];
    d.e1[i] = (T)t.e1[i];
    d.d0[i] = (T)t.d0[i];
    d.d1[i] = (T)t.d1[i];
  }
  return d;
}

// Kernel-side GLL value matrix V[q][j] = l_j^GLL(xi_q^GL) (ctables.h) in
// the compute precision, literals inside kernels.
template <int N, typename T>
struct GllDev {
  T V[N][N] = {};
};

template <int N, typename T>
constexpr GllDev<N, T> make_gll_dev() {
  constexpr ct::GllTab<N> g = ct::make_gll_tab<N>();
  GllDev<N, T> d;
  for (int q = 0; q < N; ++q)
    for (int j = 0; j < N; ++j) d.V[q][j] = (T)g.V[q][j];
  return d;
}

// Even-odd split of the 1-D tables.  The Gauss nodes are symmetric about
// the cell centre, so S is centro-symmetric (S[i][l] = S[N-1-i][N-1-l]) and
// e1[j] = e0[N-1-j], d1[j] = -d0[N-1-j].  With M = N / 2, the even part
// ue[l] = u[l] + u[N-1-l] (l < M; ue[M] = u[M] for odd N) and the odd part
// uo[l] = u[l] - u[N-1-l] of a line, (S u)[i] = ve[i] + vo[i] and
// (S u)[N-1-i] = ve[i] - vo[i] with ve = Se ue, vo = So uo (and the middle
// entry Sm . ue for odd N); the end values follow the same pattern.  Entries
// carry the factor 1/2 of the back transform.
template <typename T, int N>
struct EoTab {
  static constexpr int M = N / 2, O = N % 2, ME = M + O;
  T Se[M][ME] = {}, So[M][M] = {}, Sm[ME] = {};
  T ee[ME] = {}, eo[M] = {}, de[ME] = {}, dd[M] = {}, wh[ME] = {};
};

template <typename T, int N>
constexpr EoTab<T, N> make_eotab() {
  constexpr ct::Tab<N> t = ct::make_tab<N>();
  using E = EoTab<T, N>;
  constexpr int M = E::M;
  E e;
  for (int i = 0; i < M; ++i) {
    for (int l = 0; l < M; ++l) {
      e.Se[i][l] = (T)(0.5 * (t.S[i][l] + t.S[i][N - 1 - l]));
      e.So[i][l] = (T)(0.5 * (t.S[i][l] - t.S[i][N - 1 - l]));
    }
    if (E::O) e.Se[i][M] = (T)t.S[i][M];
    e.ee[i] = (T)(0.5 * (t.e0[i] + t.e0[N - 1 - i]));
    e.eo[i] = (T)(0.5 * (t.e0[i] - t.e0[N - 1 - i]));
    e.de[i] = (T)(0.5 * (t.d0[i] + t.d0[N - 1 - i]));
    e.dd[i] = (T)(0.5 * (t.d0[i] - t.d0[N - 1 - i]));
    e.wh[i] = (T)(0.5 * t.w[i]);
  }
  if (E::O) {
    for (int l = 0; l < M; ++l) e.Sm[l] = (T)t.S[M][l];
    e.Sm[M] = (T)t.S[M][M];
    e.ee[M] = (T)t.e0[M];
    e.de[M] = (T)t.d0[M];
    e.wh[M] = (T)t.w[M];
  }
  return e;
}

// Exact division of 0 <= n < 2^31 by a fixed divisor d >= 1 with one
// multiply and one shift (Granlund and Montgomery, "Division by invariant
// integers using multiplication", 1994): m = ceil(2^s / d) with
// s = 31 + ceil(log2 d) fits in 32 bits and q = (n m) >> s.
struct FastDiv {
  uint32_t m = 1;
  int s = 0;
};
inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  int l = 0;
  while ((1ull << l) < d) ++l;
  f.s = 31 + l;
  f.m = (uint32_t)(((1ull << f.s) + d - 1) / d);
  return f;
}
__host__ __device__ inline int fdiv(int n, FastDiv f) { return (int)(((uint64_t)(uint32_t)n * f.m) >> f.s); }

// Mesh, coefficients and discretisation constants passed to kernels.
struct Geo {
  int nx, ny, nz;
  int ncell;
  FastDiv fx, fxy;  // division by nx and by nx * ny
  double h[3];
  double ih[3];     // 1 / h
  double vol;
  double sigma;   // penalty prefactor
  int bc[6];      // FACE_DIRICHLET / FACE_NEUMANN per box face
  double b0[3];
  double B[9];
  int has_b;
  int has_c;
  const double *K;  // device [ncell][3]
  const double *c;  // device [ncell] (valid when has_c)
  // coefficient field of the outer operator: K(x) = sum_m P_m(x_m) n_m n_m^T
  // with P_m(s) = kq[m] + kq[3+m] s + kq[6+m] s^2 and n_m = row m of nrot
  // (the identity for DG_FIELD_AXIS_QUADRATIC), c(x) = cq[0] + cq[1] |x|^2;
  // K and c above then hold the (diagonal) values at the cell centres
  int field;
  double kq[9];
  double cq[2];
  double nrot[9];
};

// P_k(s) of the axis-quadratic coefficient field
__host__ __device__ inline double field_K(const Geo &g, int k, double s) {
  return g.kq[k] + s * (g.kq[3 + k] + s * g.kq[6 + k]);
}
__host__ __device__ inline double field_c(const Geo &g, double x, double y, double z) {
  return g.cq[0] + g.cq[1] * (x * x + y * y + z * z);
}
// the full tensor K(x) of the rotated field (symmetric)
__host__ __device__ inline void field_tensor(const Geo &g, const double (&x)[3], double (&K)[3][3]) {
  double P[3];
  for (int m = 0; m < 3; ++m) P[m] = field_K(g, m, x[m]);
  for (int k = 0; k < 3; ++k)
    for (int l = k; l < 3; ++l) {
      double s = 0.0;
      for (int m = 0; m < 3; ++m) s += P[m] * g.nrot[3 * m + k] * g.nrot[3 * m + l];
      K[k][l] = s;
      K[l][k] = s;
    }
}

// One level of a coarse hierarchy on a structured grid of vx * vy * vz
// unknowns: P0 (one unknown per cell, 7-point stencil, piecewise-constant
// 2x2x2 aggregation between levels) or Q1 (one unknown per mesh vertex,
// 27-point stencil, trilinear interpolation between levels).
struct CoarseLevel {
  int nx, ny, nz, n;
  int ns = 7;             // stencil entries per unknown (7 or 27)
  double *A64 = nullptr;  // device [ns][n]
  float *A32 = nullptr;
  // 27-point levels: inverse of the smoothing diagonal, 2 / sum_o |A[o][i]|
  // (half the l1 row norm; equal to the diagonal on the isotropic Q1
  // stencil, and it keeps damped Jacobi convergent on anisotropic cells)
  double *dinv64 = nullptr;
  float *dinv32 = nullptr;
  double *r64 = nullptr, *x64 = nullptr, *t64 = nullptr;  // device [n]
  float *r32 = nullptr, *x32 = nullptr, *t32 = nullptr;
  // level 0 only: accumulated solution and saved right-hand side of
  // repeated coarse cycles
  double *acc64 = nullptr, *rs64 = nullptr;
  float *acc32 = nullptr, *rs32 = nullptr;
  // levels of the aggregation AMG (ns == 0): A in CSR (values in A64 /
  // A32, nnz of them, sorted columns), and the transfers from the next
  // finer level of nf unknowns: P (nf x n) and R = P^T (n x nf), CSR
  int nnz = 0, nf = 0, pnnz = 0;  // entries of A and of P (= of R)
  int *rp = nullptr, *ci = nullptr;
  int *prp = nullptr, *pci = nullptr, *rrp = nullptr, *rci = nullptr;
  double *pv64 = nullptr, *rv64 = nullptr;
  float *pv32 = nullptr, *rv32 = nullptr;
  // level 0 of an AMG hierarchy is the structured level 0 of the
  // geometric hierarchy of the same coarse space (shared, not owned)
  bool borrowed = false;
};

// 7-point stencil order: diag, -x, +x, -y, +y, -z, +z.
// 27-point stencil order: o = (dx+1) + 3 (dy+1) + 9 (dz+1), diag at 13.
constexpr int kDiag27 = 13;

enum CoarseKind : int { COARSE_P0 = 0, COARSE_Q1 = 1 };

// DG_COARSE_* option -> hierarchy (AUTO: Q1 without advection, else P0;
// always P0 in the Gauss-Lobatto basis, which has no Q1 transfer)
inline int coarse_kind(int option, bool has_b, bool gll = false) {
  if (option == DG_COARSE_Q1) return COARSE_Q1;
  if (option == DG_COARSE_AUTO) return (has_b || gll) ? COARSE_P0 : COARSE_Q1;
  return COARSE_P0;
}

// A captured coarse solve (see coarse_solve_graph).
struct CoarseGraph {
  int kind, solver, prec, cycles, nu;
  double w;
  bool x_init, tail;
  hipGraphExec_t exec;
  void *result;  // device buffer that holds the coarse solution after a launch
};

enum CoarseSolver : int { SOLVER_GEOMETRIC = 0, SOLVER_AMG = 1 };

struct Hierarchy {
  int kind = COARSE_P0;
  int solver = SOLVER_GEOMETRIC;
  int built = 0;  // 0: not yet, 1: ready, < 0: failed with that status
  std::vector<CoarseLevel> levels;
  double *inv64 = nullptr;  // dense inverse of the coarsest matrix
  float *inv32 = nullptr;
  int bottom_n = 0;
};

}  // namespace dgmg

struct dg_problem {
  dg_problem_desc desc;
  int p = 0, n = 0, nloc = 0;
  int64_t ncell = 0, ndof = 0;
  dgmg::Geo geo;
  dgmg::Tables1D tab;
  double *dK = nullptr;
  double *dc = nullptr;
  int device = 0;
  // host copies of the coefficients (for building coarse spaces)
  std::vector<double> hK, hc;
  // largest ratio over cells of max_k / min_k of K_kk / h_k^2 (the
  // anisotropy that point smoothers on the coarse levels have to overcome)
  double aniso = 1.0;
  // coarse hierarchies: P0 and Q1 (built on first use)
  dgmg::Hierarchy p0h, q1h;
  // aggregation AMG coarse solvers on the same coarse spaces (on first use)
  dgmg::Hierarchy p0amg, q1amg;
  void *corner_buf[2] = {nullptr, nullptr};  // [ncell][8] Q1 corner sums per precision
  void *fdm[2] = {nullptr, nullptr};          // fast-diagonalisation factors per precision
  void *pmf[2] = {nullptr, nullptr};          // stored block inverses per precision (DG_INNER_PMF)
  int pmf_built = 0;                          // 0: not yet, 1: ready, < 0: failed with that status
  std::vector<dgmg::CoarseGraph> graphs;      // captured coarse solves
  hipStream_t capture_stream = nullptr;       // private stream used only for capturing
  // DG-sized temporaries for the V-cycle and smoother (allocated lazily)
  void *mg_tmp[2][4] = {{nullptr}};  // [precision][k]
  int *iters_buf = nullptr;          // [ncell]
  void *red_buf = nullptr;           // reduction scratch
  // inner-iteration counting inside a solve (dg_solve_opts.inner_stats):
  // while count_inner is set, every smoothing step writes its per-cell
  // counts to iters_buf and adds them to inner_acc (device: total, max,
  // blocks)
  int count_inner = 0;
  unsigned long long *inner_acc = nullptr;
  // per-phase timing of the preconditioner while count_inner is set:
  // event pairs recorded on the solve's stream around each phase of every
  // V-cycle (phase: 0 smoothing, 1 residual + restriction, 2 coarse solve,
  // 3 prolongation), read when the solve ends; spare events are reused
  struct PhaseMark {
    int phase;
    hipEvent_t a, b;
  };
  std::vector<PhaseMark> phase_marks;
  std::vector<hipEvent_t> phase_spare;
  // DG_BASIS_GLL: three DOF-sized scratch vectors per precision for the
  // basis changes, and the diagonal, band and band factors of the blocks
  // S^T D_T S ([4][ndof] per precision; see basis.hip)
  int basis = DG_BASIS_GL;
  void *gll_tmp[2][3] = {{nullptr}};
  void *gll_blk[2] = {nullptr, nullptr};
  // device memory of the problem (dmalloc): small buffers are carved from
  // shared chunks, large ones get a block of their own; every block is
  // freed by dg_problem_destroy (hipFree waits for the device, so the
  // handful of blocks keeps teardown short)
  std::vector<void *> blocks;
  char *chunk_cur = nullptr;
  size_t chunk_left = 0;
  size_t held_bytes = 0;
};

namespace dgmg {

void set_error(const std::string &msg);
int hip_fail(hipError_t e, const char *what);

#define DG_HIP(call)                                   \
  do {                                                 \
    hipError_t e__ = (call);                           \
    if (e__ != hipSuccess) return dgmg::hip_fail(e__, #call); \
  } while (0)

// kernel launchers (apply.hip / smooth.hip / vec.hip / coarse.hip)
// The operators of the problem's basis: for DG_BASIS_GLL the basis change
// S (basis.hip) around the Gauss-point kernels (the *_gl launchers, which
// always work in the Gauss-point basis).
// ev0 / ev1 (optional): recorded around the apply (by the kernel dispatch
// itself for the Gauss-point basis)
int launch_apply(const dg_problem *pr, int prec, const void *u, void *v, hipStream_t s, hipEvent_t ev0 = nullptr,
                 hipEvent_t ev1 = nullptr);
int launch_block_apply(const dg_problem *pr, int prec, const void *x, void *y, hipStream_t s);
// rh[c] = sum_{i in cell c} (r - A u)_i                  (P0 restriction)
// rh[8 c + q] = sum_{i in cell c} phi_q(xi_i) (r - A u)_i  (Q1 corner sums)
int launch_residual_restrict(const dg_problem *pr, int prec, const void *u, const void *r, void *rh, hipStream_t s,
                             int kind = COARSE_P0);
int launch_block_diag(const dg_problem *pr, int prec, void *diag, hipStream_t s);
int launch_rhs(const dg_problem *pr, const double *f_qp, const double *bnd, double *rhs, hipStream_t s);
// v = A u (FP64, Gauss-point basis, not the rotated-tensor field) with the
// per-block partials of u . v in part[apply_blocks(p, ncell)]
int launch_apply_dot_gl(const dg_problem *pr, const double *u, double *v, double *part, hipStream_t s,
                        hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
int64_t apply_blocks(int p, int64_t ncell);
int launch_apply_gl(const dg_problem *pr, int prec, const void *u, void *v, hipStream_t s, hipEvent_t ev0 = nullptr,
                    hipEvent_t ev1 = nullptr);
int launch_block_apply_gl(const dg_problem *pr, int prec, const void *x, void *y, hipStream_t s);
// the apply with the coefficients at the cell centres (the preconditioner's
// operator when K and c are fields)
int launch_apply_cc_gl(const dg_problem *pr, int prec, const void *u, void *v, hipStream_t s);
int launch_residual_restrict_gl(const dg_problem *pr, int prec, const void *u, const void *r, void *rh,
                                hipStream_t s, int kind = COARSE_P0);
int launch_block_diag_gl(const dg_problem *pr, int prec, void *diag, hipStream_t s);
int launch_rhs_gl(const dg_problem *pr, const double *f_qp, const double *bnd, double *rhs, hipStream_t s);
// outer operator of a full-tensor (rotated) coefficient field (apply_tensor.hip)
int launch_apply_tensor(const dg_problem *pr, int prec, const void *u, void *v, hipStream_t s);
// basis.hip: out = S (in + P zadd) (tr = false; zadd [ncell] or null) or
// S^T in (tr = true), cell by cell; d = f - y elementwise (d may alias f or
// y); the GLL scratch and block entries of a problem
int launch_basis(const dg_problem *pr, int prec, const void *in, void *out, bool tr, hipStream_t s,
                 const void *zadd = nullptr);
int launch_diff(int64_t n, int prec, const void *f, const void *y, void *d, hipStream_t s);
int gll_setup(dg_problem *pr);

// The last sweep of a preconditioner may also take the outer iteration's
// dots: per workgroup, the partial sums of z . b0 (and z . b1 when m = 2)
// in part[j * blocks + block].  FP32: z = (1 / (1 / sqrt(rr))) u_new in
// FP64 (the inverse of the factor r was scaled by) is written to z and the
// FP32 result is not; FP64: z is the sweep's own output (rr and z unused).
struct CastBackArgs {
  const double *rr = nullptr;
  double *z = nullptr;
  const double *b0 = nullptr, *b1 = nullptr;
  double *part = nullptr;
  int m = 0;
};
// workgroups of a Jacobi sweep of the Gauss-point smoother (the partials
// of CastBackArgs per dot)
int64_t smooth_blocks(int p, int64_t ncell);
// whether the sweep of this precision and inner solver (DG_INNER_*) has
// the epilogue (all but FP64 inner GMRES)
bool smooth_takes_dots(int prec, int inner);

struct SmoothArgs {
  double omega, eps;
  int max_inner, inner, restart;
  int zero_guess;   // u_in treated as 0
  int write_du;     // output is the correction only (block solve)
  int defect;       // compute d = f - A u (otherwise d = f)
  const void *zh = nullptr;  // optional P0 correction: u_in + P zh is smoothed
  int colour = -1;  // >= 0: one colour (ix + iy + iz) mod ncol, in place (uin == uout)
  int ncol = 2;     // number of colours of the SOR order
  int sor = 0;      // block-SOR update form (alg block_SOR)
  int sweep = 0;    // DG_SWEEP_* of the options (host-side dispatch)
  int tridiag = 0;  // inner preconditioner: tridiagonal part of D_T (Thomas)
  const CastBackArgs *cb = nullptr;  // Jacobi sweep, Gauss-point basis only
};
int launch_smooth(const dg_problem *pr, int prec, const void *f, const void *uin, void *uout,
                  const SmoothArgs &a, int *iters, hipStream_t s);
// the same for the Gauss-Lobatto basis (smooth_gll.hip; called by launch_smooth)
int launch_smooth_gll(const dg_problem *pr, int prec, const void *f, const void *uin, void *uout,
                      const SmoothArgs &a, int *iters, hipStream_t s);
// fast-diagonalisation factors of the cell blocks (b = 0), built on first use
int ensure_fdm(dg_problem *pr, int prec);
// stored inverses of the cell blocks D_T (any b, p <= 4), built on first use
int ensure_pmf(dg_problem *pr, int prec);
size_t pmf_bytes(const dg_problem *pr, int prec);

}  // namespace dgmg
