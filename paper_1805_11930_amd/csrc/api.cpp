// C-ABI entry points: argument checks and dispatch to the kernels, the
// hybrid V-cycle (alg hybrid_multigrid) and the outer Krylov solvers.
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "dg_internal.h"
#include "solve_common.h"
#include "vec.h"

namespace dgmg {
// fixed device scratch of the allocation-free entry points (noalloc.hip)
size_t scratch_capacity();
int scratch_device_ptr(int device, void **out);
int alloc_tmp(dg_problem *pr, int prec, int k, void **out);
int alloc_small(dg_problem *pr);
int ensure_hierarchy(dg_problem *pr, int kind);
int ensure_amg(dg_problem *pr, int kind);
int amg_level_csr(dg_problem *pr, int kind, int level, int which, int64_t *dims, int *rp, int *ci, double *v);

int validate_mg_opts(const dg_mg_opts *o) {
  if (o->n_pre < 0 || o->n_post < 0 || o->n_pre > 64 || o->n_post > 64) {
    set_error("n_pre and n_post must be in 0..64");
    return DG_EINVAL;
  }
  if (o->coarse_space != DG_COARSE_P0 && o->coarse_space != DG_COARSE_Q1 && o->coarse_space != DG_COARSE_AUTO) {
    set_error("coarse_space must be DG_COARSE_P0, DG_COARSE_Q1 or DG_COARSE_AUTO");
    return DG_EINVAL;
  }
  if (o->coarse_cycles < 0 || o->coarse_cycles > 64 || o->coarse_smooth < 0 || o->coarse_smooth > 64) {
    set_error("coarse_cycles and coarse_smooth must be in 0..64");
    return DG_EINVAL;
  }
  if (o->coarse_solver != DG_COARSE_SOLVER_GEOMETRIC && o->coarse_solver != DG_COARSE_SOLVER_AMG) {
    set_error("coarse_solver must be DG_COARSE_SOLVER_GEOMETRIC or DG_COARSE_SOLVER_AMG");
    return DG_EINVAL;
  }
  if (o->fuse_small_levels != 0 && o->fuse_small_levels != 1) {
    set_error("fuse_small_levels must be 0 or 1");
    return DG_EINVAL;
  }
  return DG_OK;
}
}  // namespace dgmg

using namespace dgmg;

namespace {

inline hipStream_t S(void *s) { return (hipStream_t)s; }

// Scratch of the block smoother given by the caller (instead of the problem's own):
// the fixed device array of dg_block_smooth_noalloc.
struct ScratchParts {
  void *alt = nullptr;                // Jacobi ping-pong vector (n_sweeps > 1)
  int *iters = nullptr;               // [ncell] inner iterations per cell (stats)
  unsigned long long *red = nullptr;  // [2] sum and max of iters (stats)
};

int check_vec(const void *p, const char *name) {
  if (!p) {
    set_error(std::string(name) + " is NULL");
    return DG_EINVAL;
  }
  if (((uintptr_t)p) % 16 != 0) {
    set_error(std::string(name) + " is not 16-byte aligned");
    return DG_EINVAL;
  }
  return DG_OK;
}

int check_prec(int prec) {
  if (prec != DG_FP64 && prec != DG_FP32) {
    set_error("precision must be DG_FP64 or DG_FP32");
    return DG_EINVAL;
  }
  return DG_OK;
}

int smooth_args(dg_problem *pr, const dg_smooth_opts *o, SmoothArgs &a) {
  if (!o) {
    set_error("smoother options are NULL");
    return DG_EINVAL;
  }
  if (!(o->eps >= 0) || !std::isfinite(o->omega) ||
      (o->inner != DG_INNER_CG && o->inner != DG_INNER_GMRES && o->inner != DG_INNER_FDM &&
       o->inner != DG_INNER_PMF) ||
      o->sweep < DG_SWEEP_JACOBI || o->sweep > DG_SWEEP_SOR_BACKWARD ||
      (o->inner_precond != DG_IPREC_DIAG && o->inner_precond != DG_IPREC_TRIDIAG) ||
      (o->inner_precond == DG_IPREC_TRIDIAG && o->inner != DG_INNER_GMRES) || o->colours > 64) {
    set_error(
        "invalid smoother options (eps >= 0, finite omega, inner CG, GMRES, FDM or PMF, sweep DG_SWEEP_*, "
        "inner_precond DG_IPREC_DIAG, or DG_IPREC_TRIDIAG with inner GMRES, colours <= 64)");
    return DG_EINVAL;
  }
  if (pr->basis == DG_BASIS_GLL && o->inner != DG_INNER_CG && o->inner != DG_INNER_GMRES) {
    set_error("the Gauss-Lobatto basis supports the inner CG and GMRES block solves");
    return DG_EINVAL;
  }
  if (o->inner == DG_INNER_FDM) {
    int rc = ensure_fdm(pr, DG_FP64);
    if (!rc) rc = ensure_fdm(pr, DG_FP32);
    if (rc) return rc;
  }
  if (o->inner == DG_INNER_PMF) {
    int rc = ensure_pmf(pr, DG_FP64);
    if (!rc) rc = ensure_pmf(pr, DG_FP32);
    if (rc) return rc;
  }
  a.omega = o->omega;
  a.eps = o->eps;
  a.max_inner = o->max_inner > 0 ? o->max_inner : (int)pr->nloc;
  a.inner = o->inner;
  a.restart = o->restart > 0 ? o->restart : 12;
  if (a.restart > 16) a.restart = 16;
  if (a.restart > pr->nloc) a.restart = (int)pr->nloc;
  a.zero_guess = o->zero_guess;
  a.write_du = 0;
  a.defect = 1;
  a.sweep = o->sweep;
  a.tridiag = o->inner_precond == DG_IPREC_TRIDIAG;
  a.ncol = o->colours >= 2 ? o->colours : 2;
  return DG_OK;
}

size_t esize(int prec) { return prec == DG_FP64 ? sizeof(double) : sizeof(float); }

// Per-cell iteration counts for a smoother launch: the caller's buffer, or
// the problem's own while a solve counts its inner iterations.
int *count_buf(dg_problem *pr, int *iters) { return iters ? iters : (pr->count_inner ? pr->iters_buf : nullptr); }

// Phase timing of the preconditioner inside a solve that collects
// statistics: phase_begin records the start event of a phase on s, and
// phase_end its end event; both are no-ops otherwise.
enum { PH_SMOOTH = 0, PH_RESTRICT = 1, PH_COARSE = 2, PH_PROLONG = 3 };

int phase_event(dg_problem *pr, hipEvent_t *e) {
  if (!pr->phase_spare.empty()) {
    *e = pr->phase_spare.back();
    pr->phase_spare.pop_back();
    return DG_OK;
  }
  DG_HIP(hipEventCreate(e));
  return DG_OK;
}

int phase_begin(dg_problem *pr, int phase, hipStream_t s) {
  if (!pr->count_inner) return DG_OK;
  dg_problem::PhaseMark m{phase, nullptr, nullptr};
  int rc = phase_event(pr, &m.a);
  if (!rc) rc = phase_event(pr, &m.b);
  if (rc) return rc;
  DG_HIP(hipEventRecord(m.a, s));
  pr->phase_marks.push_back(m);
  return DG_OK;
}

int phase_end(dg_problem *pr, hipStream_t s) {
  if (!pr->count_inner || pr->phase_marks.empty()) return DG_OK;
  DG_HIP(hipEventRecord(pr->phase_marks.back().b, s));
  return DG_OK;
}

// Adds the counts of one finished smoothing step (every cell solved once)
// to the solve's running totals, when the solve counts them.
int count_step(dg_problem *pr, int *iters, hipStream_t s) {
  if (iters || !pr->count_inner) return DG_OK;
  return iter_accum(pr->ncell, pr->iters_buf, pr->inner_acc, s);
}

// n block-Jacobi sweeps from `src` (NULL = zero) ending in `dst`, using
// `alt` as the other ping-pong buffer.  dst != alt; src may equal alt but
// not dst unless n == 0.
// cb: the last sweep also does the cast back of an FP32 preconditioner
// (its FP32 result is then not written, so it must be the sweep into dst)
int sweeps(dg_problem *pr, int prec, const void *f, const void *src, void *dst, void *alt, int n,
           const SmoothArgs &base, int *iters, hipStream_t s, const void *zh = nullptr,
           const CastBackArgs *cb = nullptr) {
  if (n <= 0) {
    if (src == nullptr)
      DG_HIP(hipMemsetAsync(dst, 0, (size_t)pr->ndof * esize(prec), s));
    else if (src != dst)
      DG_HIP(hipMemcpyAsync(dst, src, (size_t)pr->ndof * esize(prec), hipMemcpyDeviceToDevice, s));
    return DG_OK;
  }
  const void *cur = src;
  for (int k = 1; k <= n; ++k) {
    void *out = ((n - k) % 2 == 0) ? dst : alt;
    if (out == cur) out = (out == dst) ? alt : dst;  // never smooth in place
    SmoothArgs a = base;
    a.zero_guess = cur == nullptr ? 1 : 0;
    a.zh = (k == 1 && cur != nullptr) ? zh : nullptr;  // P0 correction enters the first sweep
    a.cb = k == n ? cb : nullptr;
    int rc = launch_smooth(pr, prec, f, cur ? cur : f, out, a, count_buf(pr, iters), s);
    if (!rc) rc = count_step(pr, iters, s);
    if (rc) return rc;
    cur = out;
  }
  if (cur != dst) {
    if (cb) {
      set_error("internal: the cast-back sweep must end in its output");
      return DG_EINVAL;
    }
    DG_HIP(hipMemcpyAsync(dst, cur, (size_t)pr->ndof * esize(prec), hipMemcpyDeviceToDevice, s));
  }
  return DG_OK;
}

// One block-SOR sweep (alg block_SOR) over the colour order, in place on
// u: colours 0, 1, ..., C-1 (backward: C-1, ..., 0).  zero: u is taken as
// 0 (the first colour skips the defect and clears the other colours).
int sor_pass(dg_problem *pr, int prec, const void *f, void *u, bool backward, bool zero, const SmoothArgs &base,
             int *iters, hipStream_t s) {
  const int C = base.ncol;
  for (int h = 0; h < C; ++h) {
    SmoothArgs a = base;
    a.colour = backward ? C - 1 - h : h;
    a.sor = 1;
    a.zh = nullptr;
    a.zero_guess = (zero && h == 0) ? 1 : 0;
    int rc = launch_smooth(pr, prec, f, u, u, a, count_buf(pr, iters), s);
    if (rc) return rc;
  }
  return count_step(pr, iters, s);  // each cell was solved once by its colour
}

// Direction of the k-th of the n_dir single-direction sweeps of n steps of
// the given SOR kind (SSOR: forward, backward, forward, ...).
bool sor_backward(int sweep, int k) {
  if (sweep == DG_SWEEP_SSOR) return k % 2 == 1;
  return sweep == DG_SWEEP_SOR_BACKWARD;
}
int sor_dirs(int sweep, int n) { return sweep == DG_SWEEP_SSOR ? 2 * n : n; }

// n block-SOR/SSOR steps in place on dst, starting from src (NULL = zero;
// src != dst is copied first) plus the optional P0 correction P zh.
int sor_sweeps(dg_problem *pr, int prec, const void *f, const void *src, void *dst, int n, int sweep,
               const SmoothArgs &base, hipStream_t s, const void *zh = nullptr) {
  const bool zero = src == nullptr;
  int rc;
  if (!zero && src != dst) DG_HIP(hipMemcpyAsync(dst, src, (size_t)pr->ndof * esize(prec), hipMemcpyDeviceToDevice, s));
  if (zh) {
    if (zero) {
      set_error("internal: a P0 correction needs a smoothed input");
      return DG_EINVAL;
    }
    rc = prec == DG_FP64 ? prolong_add_p0<double>(pr->ndof, pr->nloc, (const double *)zh, (double *)dst, s)
                         : prolong_add_p0<float>(pr->ndof, pr->nloc, (const float *)zh, (float *)dst, s);
    if (rc) return rc;
  }
  if (n <= 0) {
    if (zero) DG_HIP(hipMemsetAsync(dst, 0, (size_t)pr->ndof * esize(prec), s));
    return DG_OK;
  }
  const int nd = sor_dirs(sweep, n);
  for (int k = 0; k < nd; ++k)
    if ((rc = sor_pass(pr, prec, f, dst, sor_backward(sweep, k), zero && k == 0, base, nullptr, s))) return rc;
  return DG_OK;
}

// ---- coarse cycles (P0 aggregation or Q1 vertex-grid hierarchy) ---------
template <typename T>
struct LevelPtr;
template <>
struct LevelPtr<double> {
  static double *r(CoarseLevel &L) { return L.r64; }
  static double *x(CoarseLevel &L) { return L.x64; }
  static double *t(CoarseLevel &L) { return L.t64; }
  static double *acc(CoarseLevel &L) { return L.acc64; }
  static double *rs(CoarseLevel &L) { return L.rs64; }
  static const double *A(const CoarseLevel &L) { return L.A64; }
  static const double *dinv(const CoarseLevel &L) { return L.dinv64; }
  static const double *inv(const Hierarchy &H) { return H.inv64; }
  static const double *pv(const CoarseLevel &L) { return L.pv64; }
  static const double *rv(const CoarseLevel &L) { return L.rv64; }
};
template <>
struct LevelPtr<float> {
  static float *r(CoarseLevel &L) { return L.r32; }
  static float *x(CoarseLevel &L) { return L.x32; }
  static float *t(CoarseLevel &L) { return L.t32; }
  static float *acc(CoarseLevel &L) { return L.acc32; }
  static float *rs(CoarseLevel &L) { return L.rs32; }
  static const float *A(const CoarseLevel &L) { return L.A32; }
  static const float *dinv(const CoarseLevel &L) { return L.dinv32; }
  static const float *inv(const Hierarchy &H) { return H.inv32; }
  static const float *pv(const CoarseLevel &L) { return L.pv32; }
  static const float *rv(const CoarseLevel &L) { return L.rv32; }
};

template <typename T>
int level_jacobi(const CoarseLevel &L, T w, const T *r, const T *xi, T *xo, hipStream_t s) {
  const T *A = LevelPtr<T>::A(L);
  if (L.ns == 0) return csr_jacobi<T>(L.n, L.nnz, L.rp, L.ci, A, LevelPtr<T>::dinv(L), w, r, xi, xo, s);
  return L.ns == 27 ? jacobi27<T>(A, LevelPtr<T>::dinv(L), L.nx, L.ny, L.nz, w, r, xi, xo, s)
                    : coarse_jacobi<T>(A, L.nx, L.ny, L.nz, w, r, xi, xo, s);
}

// out = r - A_l x on a level of any kind
template <typename T>
int level_residual(const CoarseLevel &L, const T *r, const T *x, T *out, hipStream_t s) {
  const T *A = LevelPtr<T>::A(L);
  if (L.ns == 0) return csr_residual<T>(L.n, L.nnz, L.rp, L.ci, A, r, x, out, s);
  return L.ns == 27 ? residual27<T>(A, L.nx, L.ny, L.nz, r, x, out, s)
                    : residual7<T>(A, L.nx, L.ny, L.nz, r, x, out, s);
}

// Levels l .. end run as one single-workgroup kernel (k_coarse_tail) when
// they are all 27-point vertex-grid levels, level l has at most
// kTailMaxUnknowns unknowns, the dense bottom at most kTailBottomMax, all
// of them together at most kTailLds, at least one level lies above the
// bottom, and their coefficients (A and dinv above the bottom, the dense
// inverse) take at most kTailCoefBytes: the workgroup pulls them through
// one compute unit each cycle.
bool tail_from(const Hierarchy &H, size_t l, size_t elem) {
  const size_t nl = H.levels.size() - l;
  if (nl < 2 || nl > (size_t)kTailLevels || H.levels[l].n > kTailMaxUnknowns || H.bottom_n > kTailBottomMax)
    return false;
  int64_t total = 0, coef = (int64_t)H.bottom_n * H.bottom_n;
  for (size_t k = l; k < H.levels.size(); ++k) {
    if (H.levels[k].ns != 27) return false;
    total += H.levels[k].n;
    if (k + 1 < H.levels.size()) coef += 28 * (int64_t)H.levels[k].n;
  }
  return total <= kTailLds && coef * (int64_t)elem <= kTailCoefBytes;
}

template <typename T>
int run_tail(Hierarchy &H, size_t l, int nu, T w, hipStream_t s, T **result, bool x_init) {
  using LP = LevelPtr<T>;
  TailArgs<T> a;
  a.nl = (int)(H.levels.size() - l);
  for (int k = 0; k < a.nl; ++k) {
    CoarseLevel &L = H.levels[l + k];
    a.lv[k].A = LP::A(L);
    a.lv[k].dinv = LP::dinv(L);
    a.lv[k].r = LP::r(L);
    a.lv[k].x = LP::x(L);
    a.lv[k].t = LP::t(L);
    a.lv[k].vx = L.nx;
    a.lv[k].vy = L.ny;
    a.lv[k].vz = L.nz;
  }
  a.inv = LP::inv(H);
  a.bn = H.bottom_n;
  a.nu = nu;
  a.w = w;
  a.x_init = x_init ? 1 : 0;
  *result = LP::x(H.levels[l]);
  return coarse_tail<T>(a, s);
}

// x_l ~= A_l^-1 r_l: one V-cycle of the hierarchy from a zero guess; r_l is
// level l's r buffer, the result is left in one of level l's x / t buffers
// and returned in *result.  x_init: level l's x buffer already holds the
// first damped Jacobi sweep from zero, w D^-1 r_l (fused into the kernel
// that produced r_l).
template <typename T>
int coarse_cycle(Hierarchy &H, size_t l, int nu, T w, hipStream_t s, T **result, bool x_init, bool tail) {
  using LP = LevelPtr<T>;
  CoarseLevel &L = H.levels[l];
  if (tail && tail_from(H, l, sizeof(T))) return run_tail<T>(H, l, nu, w, s, result, x_init);
  if (l + 1 == H.levels.size()) {
    *result = LP::x(L);
    return dense_mv<T>(H.bottom_n, LP::inv(H), LP::r(L), LP::x(L), s);
  }
  int rc;
  T *x = LP::x(L), *t = LP::t(L);
  const T *A = LP::A(L), *r = LP::r(L);
  // presmooth from zero: x = w D^-1 r, then nu-1 more sweeps
  if (!x_init && (rc = level_jacobi<T>(L, w, r, nullptr, x, s))) return rc;
  for (int k = 1; k < nu; ++k) {
    if ((rc = level_jacobi<T>(L, w, r, x, t, s))) return rc;
    std::swap(x, t);
  }
  CoarseLevel &C = H.levels[l + 1];
  // the coarser level smooths: its first sweep is fused into the restriction
  const bool fuse = L.ns == 27 && C.ns == 27 && l + 2 < H.levels.size();
  if (C.ns == 0) {
    // aggregation AMG level below: r_C = R (r - A x)
    if ((rc = level_residual<T>(L, r, x, t, s))) return rc;
    if ((rc = csr_spmv<T>(C.n, C.pnnz, C.rrp, C.rci, LP::rv(C), t, LP::r(C), false, s))) return rc;
  } else if (L.ns == 27) {
    if ((rc = residual27<T>(A, L.nx, L.ny, L.nz, r, x, t, s))) return rc;
    if ((rc = restrict27<T>(L.nx, L.ny, L.nz, t, C.nx, C.ny, C.nz, LP::r(C), LP::dinv(C), w,
                            fuse ? LP::x(C) : nullptr, s)))
      return rc;
  } else if ((rc = coarse_restrict<T>(A, L.nx, L.ny, L.nz, r, x, C.nx, C.ny, C.nz, LP::r(C), s))) {
    return rc;
  }
  T *xc = nullptr;
  if ((rc = coarse_cycle<T>(H, l + 1, nu, w, s, &xc, fuse, tail))) return rc;
  if (C.ns == 0)
    rc = csr_spmv<T>(L.n, C.pnnz, C.prp, C.pci, LP::pv(C), xc, x, true, s);  // x += P x_C
  else if (L.ns == 27)
    rc = prolong27<T>(L.nx, L.ny, L.nz, C.nx, C.ny, C.nz, xc, x, s);
  else
    rc = coarse_prolong<T>(L.nx, L.ny, L.nz, C.nx, C.ny, xc, x, s);
  if (rc) return rc;
  for (int k = 0; k < nu; ++k) {
    if ((rc = level_jacobi<T>(L, w, r, x, t, s))) return rc;
    std::swap(x, t);
  }
  *result = x;
  return DG_OK;
}

// x_0 ~= A_0^-1 r_0 on level 0 of H by `cycles` V-cycles (a fixed number,
// so the result is a linear function of r_0): x += V(r_0 - A_0 x).
// x_init as for coarse_cycle (first cycle only).  Kernels only: the
// sequence can be captured into a HIP graph.
template <typename T>
int coarse_solve(Hierarchy &H, int cycles, int nu, T w, hipStream_t s, T **result, bool x_init, bool tail) {
  using LP = LevelPtr<T>;
  CoarseLevel &L = H.levels[0];
  if (cycles <= 1 || H.levels.size() == 1) return coarse_cycle<T>(H, 0, nu, w, s, result, x_init, tail);
  const int64_t n = L.n;
  T *acc = LP::acc(L), *rs = LP::rs(L);
  int rc;
  if ((rc = copy_vec<T>(n, LP::r(L), rs, s))) return rc;
  T *x = nullptr;
  if ((rc = coarse_cycle<T>(H, 0, nu, w, s, &x, x_init, tail))) return rc;
  if ((rc = copy_vec<T>(n, x, acc, s))) return rc;
  for (int c = 1; c < cycles; ++c) {
    if ((rc = level_residual<T>(L, rs, acc, LP::r(L), s))) return rc;
    if ((rc = coarse_cycle<T>(H, 0, nu, w, s, &x, false, tail))) return rc;
    if ((rc = add_to<T>(n, x, acc, s))) return rc;
  }
  // restore r_0 for callers that read it again
  if ((rc = copy_vec<T>(n, rs, LP::r(L), s))) return rc;
  *result = acc;
  return DG_OK;
}

// The coarse solve replayed from a HIP graph: captured once per hierarchy,
// precision and cycle parameters on a private stream of default priority,
// then launched on the caller's stream.  The graph holds kernel nodes only.
template <typename T>
int coarse_solve_graph(dg_problem *pr, Hierarchy &H, int prec, int cycles, int nu, T w, hipStream_t s, T **result,
                       bool x_init, bool tail) {
  CoarseGraph *hit = nullptr;
  for (auto &cg : pr->graphs)
    if (cg.kind == H.kind && cg.solver == H.solver && cg.prec == prec && cg.cycles == cycles && cg.nu == nu &&
        cg.w == (double)w && cg.x_init == x_init && cg.tail == tail) {
      hit = &cg;
      break;
    }
  if (!hit) {
    if (!pr->capture_stream) DG_HIP(hipStreamCreateWithFlags(&pr->capture_stream, hipStreamNonBlocking));
    DG_HIP(hipStreamBeginCapture(pr->capture_stream, hipStreamCaptureModeThreadLocal));
    T *res = nullptr;
    int rc = coarse_solve<T>(H, cycles, nu, w, pr->capture_stream, &res, x_init, tail);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(pr->capture_stream, &graph);
    if (rc) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e2 != hipSuccess) return hip_fail(e2, "hipGraphInstantiate");
    CoarseGraph cg;
    cg.kind = H.kind;
    cg.solver = H.solver;
    cg.prec = prec;
    cg.cycles = cycles;
    cg.nu = nu;
    cg.w = (double)w;
    cg.x_init = x_init;
    cg.tail = tail;
    cg.exec = exec;
    cg.result = res;
    pr->graphs.push_back(cg);
    hit = &pr->graphs.back();
  }
  DG_HIP(hipGraphLaunch(hit->exec, s));
  *result = (T *)hit->result;
  return DG_OK;
}

// cb (FP32 only, nullable): the last postsmoothing sweep also does the
// cast back (see CastBackArgs); *fused tells whether it did.
template <typename T>
int vcycle_t(dg_problem *pr, int prec, const T *r, T *z, const dg_mg_opts *o, hipStream_t s,
             const CastBackArgs *cb = nullptr, bool *fused = nullptr) {
  if (fused) *fused = false;
  SmoothArgs sa;
  int rc = smooth_args(pr, &o->smooth, sa);
  if (rc) return rc;
  const int kind = coarse_kind(o->coarse_space, pr->geo.has_b != 0, pr->basis == DG_BASIS_GLL);
  if (kind == COARSE_Q1 && pr->basis == DG_BASIS_GLL) {
    set_error("the Gauss-Lobatto basis supports the P0 coarse space only");
    return DG_EINVAL;
  }
  if ((rc = ensure_hierarchy(pr, kind))) return rc;
  const bool amg = o->coarse_solver == DG_COARSE_SOLVER_AMG;
  if (amg && (rc = ensure_amg(pr, kind))) return rc;
  Hierarchy &H = kind == COARSE_Q1 ? (amg ? pr->q1amg : pr->q1h) : (amg ? pr->p0amg : pr->p0h);
  void *t0;
  if ((rc = alloc_tmp(pr, prec, 0, &t0))) return rc;
  // presmoothing ends in X so that postsmoothing ends in z without a copy
  // (the SOR sweeps work in place: X = z)
  const int sw = sa.sweep;
  const bool sor = sw != DG_SWEEP_JACOBI;
  const int sw_post = sw == DG_SWEEP_SOR ? DG_SWEEP_SOR_BACKWARD : (sw == DG_SWEEP_SOR_BACKWARD ? DG_SWEEP_SOR : sw);
  void *X = (!sor && o->n_post % 2 == 1) ? t0 : (void *)z;
  void *Y = (X == t0) ? (void *)z : t0;
  if ((rc = phase_begin(pr, PH_SMOOTH, s))) return rc;
  if (sor)
    rc = sor_sweeps(pr, prec, r, nullptr, X, o->n_pre, sw, sa, s);
  else
    rc = sweeps(pr, prec, r, nullptr, X, Y, o->n_pre, sa, nullptr, s);
  if (rc || (rc = phase_end(pr, s)) || (rc = phase_begin(pr, PH_RESTRICT, s))) return rc;
  // residual and restriction R = P^T
  using LP = LevelPtr<T>;
  CoarseLevel &L0 = H.levels[0];
  // coarse Jacobi sweeps per level: as given, or 6 when K_kk / h_k^2
  // differ by more than 4 between axes, 4 with advection, else 2
  const int nu =
      o->coarse_smooth > 0 ? o->coarse_smooth : (pr->aniso > 4.0 ? 6 : (pr->geo.has_b ? 4 : 2));
  const T w = (T)(o->coarse_omega > 0 ? o->coarse_omega : 2.0 / 3.0);
  bool x_init = false;
  if (kind == COARSE_Q1) {
    T *cs = (T *)pr->corner_buf[prec];
    if ((rc = launch_residual_restrict(pr, prec, X, r, cs, s, COARSE_Q1))) return rc;
    x_init = H.levels.size() > 1;  // level 0 smooths: fuse its first sweep into the gather
    if ((rc = q1_gather<T>(pr->geo.nx, pr->geo.ny, pr->geo.nz, cs, LP::r(L0), LP::dinv(L0), w,
                           x_init ? LP::x(L0) : nullptr, s)))
      return rc;
  } else if ((rc = launch_residual_restrict(pr, prec, X, r, LP::r(L0), s, COARSE_P0))) {
    return rc;
  }
  const int cycles = o->coarse_cycles > 1 ? o->coarse_cycles : 1;
  T *xh = nullptr;
  if ((rc = phase_end(pr, s)) || (rc = phase_begin(pr, PH_COARSE, s))) return rc;
  const bool tail = o->fuse_small_levels != 0;
  if (o->graph)
    rc = coarse_solve_graph<T>(pr, H, prec, cycles, nu, w, s, &xh, x_init, tail);
  else
    rc = coarse_solve<T>(H, cycles, nu, w, s, &xh, x_init, tail);
  if (rc || (rc = phase_end(pr, s))) return rc;
  if (kind == COARSE_Q1) {
    // prolongation P (nodal interpolation of the trilinear correction)
    if ((rc = phase_begin(pr, PH_PROLONG, s))) return rc;
    if ((rc = q1_prolong_add<T>(pr->p, pr->geo.nx, pr->geo.ny, pr->geo.nz, xh, (T *)X, s))) return rc;
    if ((rc = phase_end(pr, s))) return rc;
    if (o->n_post == 0) return DG_OK;  // X == z here
    if ((rc = phase_begin(pr, PH_SMOOTH, s))) return rc;
    if (sor) {
      rc = sor_sweeps(pr, prec, r, z, z, o->n_post, sw_post, sa, s);
    } else {
      rc = sweeps(pr, prec, r, X, z, Y == z ? t0 : Y, o->n_post, sa, nullptr, s, nullptr, cb);
      if (!rc && cb && fused) *fused = true;
    }
    return rc ? rc : phase_end(pr, s);
  }
  if (o->n_post == 0) {
    if ((rc = phase_begin(pr, PH_PROLONG, s))) return rc;
    rc = prolong_add_p0<T>(pr->ndof, pr->nloc, xh, (T *)X, s);  // X == z here
    return rc ? rc : phase_end(pr, s);
  }
  // prolongation P (injection) fused into the first postsmoothing sweep
  if ((rc = phase_begin(pr, PH_SMOOTH, s))) return rc;
  if (sor) {
    rc = sor_sweeps(pr, prec, r, z, z, o->n_post, sw_post, sa, s, xh);
  } else {
    rc = sweeps(pr, prec, r, X, z, Y == z ? t0 : Y, o->n_post, sa, nullptr, s, xh, cb);
    if (!rc && cb && fused) *fused = true;
  }
  return rc ? rc : phase_end(pr, s);
}

int vcycle(dg_problem *pr, int prec, const void *r, void *z, const dg_mg_opts *o, hipStream_t s) {
  if (prec == DG_FP64) return vcycle_t<double>(pr, prec, (const double *)r, (double *)z, o, s);
  return vcycle_t<float>(pr, prec, (const float *)r, (float *)z, o, s);
}

// dg_block_smooth with its scratch (the Jacobi ping-pong vector, per-cell
// iteration counts, reduction results) either from the problem (sp ==
// NULL: allocated on first use) or from the caller's fixed buffers.
int block_smooth_impl(dg_problem *pr, int precision, const void *f, const void *u_in, void *u_out,
                      const dg_smooth_opts *opts, dg_smooth_stats *stats, hipStream_t s, const ScratchParts *sp) {
  if (!pr) {
    set_error("problem is NULL");
    return DG_EINVAL;
  }
  int rc;
  if ((rc = check_prec(precision)) || (rc = check_vec(f, "f")) || (rc = check_vec(u_out, "u_out"))) return rc;
  if (!opts) {
    set_error("smoother options are NULL");
    return DG_EINVAL;
  }
  if (!opts->zero_guess && (rc = check_vec(u_in, "u_in"))) return rc;
  if (opts->n_sweeps < 1) {
    set_error("n_sweeps must be >= 1");
    return DG_EINVAL;
  }
  SmoothArgs a;
  if ((rc = smooth_args(pr, opts, a))) return rc;
  if (a.sweep != DG_SWEEP_JACOBI) {
    if (f == u_out) {
      set_error("dg_block_smooth: u_out must differ from f");
      return DG_EINVAL;
    }
    const bool zero = opts->zero_guess != 0;
    if (!zero && u_in != u_out)
      DG_HIP(hipMemcpyAsync(u_out, u_in, (size_t)pr->ndof * esize(precision), hipMemcpyDeviceToDevice, s));
    int *iters = stats ? (sp ? sp->iters : pr->iters_buf) : nullptr;
    unsigned long long tot = 0;
    int mx = 0;
    const int nd = sor_dirs(a.sweep, opts->n_sweeps);
    for (int k = 0; k < nd; ++k) {
      if ((rc = sor_pass(pr, precision, f, u_out, sor_backward(a.sweep, k), zero && k == 0, a, iters, s))) return rc;
      if (stats) {
        unsigned long long *dev = sp ? sp->red : (unsigned long long *)pr->red_buf;
        if ((rc = iter_stats(pr->ncell, iters, dev, s))) return rc;
        unsigned long long h[2];
        DG_HIP(hipMemcpyAsync(h, dev, sizeof(h), hipMemcpyDeviceToHost, s));
        DG_HIP(hipStreamSynchronize(s));
        tot += h[0];
        mx = (int)h[1] > mx ? (int)h[1] : mx;
      }
    }
    if (stats) {
      stats->blocks = (long long)pr->ncell * nd;
      stats->inner_total = (long long)tot;
      stats->inner_max = mx;
      stats->inner_avg = stats->blocks ? (double)tot / stats->blocks : 0.0;
    }
    return DG_OK;
  }
  if (u_in == u_out || f == u_out) {
    set_error("dg_block_smooth: u_out must differ from u_in and f");
    return DG_EINVAL;
  }
  void *alt = nullptr;
  if (opts->n_sweeps > 1) {
    if (sp)
      alt = sp->alt;
    else if ((rc = alloc_tmp(pr, precision, 2, &alt)))
      return rc;
  }
  int *iters = stats ? (sp ? sp->iters : pr->iters_buf) : nullptr;
  unsigned long long tot = 0;
  int mx = 0;
  const void *cur = opts->zero_guess ? nullptr : u_in;
  for (int k = 1; k <= opts->n_sweeps; ++k) {
    void *out = ((opts->n_sweeps - k) % 2 == 0) ? u_out : alt;
    SmoothArgs ak = a;
    ak.zero_guess = cur == nullptr;
    if ((rc = launch_smooth(pr, precision, f, cur ? cur : f, out, ak, iters, s))) return rc;
    if (stats) {
      unsigned long long *dev = sp ? sp->red : (unsigned long long *)pr->red_buf;
      if ((rc = iter_stats(pr->ncell, iters, dev, s))) return rc;
      unsigned long long h[2];
      DG_HIP(hipMemcpyAsync(h, dev, sizeof(h), hipMemcpyDeviceToHost, s));
      DG_HIP(hipStreamSynchronize(s));
      tot += h[0];
      mx = (int)h[1] > mx ? (int)h[1] : mx;
    }
    cur = out;
  }
  if (stats) {
    stats->blocks = (long long)pr->ncell * opts->n_sweeps;
    stats->inner_total = (long long)tot;
    stats->inner_max = mx;
    stats->inner_avg = stats->blocks ? (double)tot / stats->blocks : 0.0;
  }
  return DG_OK;
}

}  // namespace

extern "C" {

void dg_default_smooth_opts(dg_smooth_opts *o) {
  if (!o) return;
  o->n_sweeps = 1;
  o->omega = 0.8;
  o->eps = 1e-2;
  o->max_inner = 0;
  o->inner = DG_INNER_CG;
  o->restart = 12;
  o->zero_guess = 0;
  o->sweep = DG_SWEEP_JACOBI;
  o->inner_precond = DG_IPREC_DIAG;
  o->colours = 2;
}

void dg_default_mg_opts(dg_mg_opts *o) {
  if (!o) return;
  o->n_pre = 1;
  o->n_post = 1;
  dg_default_smooth_opts(&o->smooth);
  o->coarse_space = DG_COARSE_AUTO;
  o->coarse_cycles = 1;
  o->coarse_smooth = 0;
  o->coarse_omega = 2.0 / 3.0;
  o->graph = 0;
  o->fuse_small_levels = 1;
  o->coarse_solver = DG_COARSE_SOLVER_GEOMETRIC;
}

void dg_default_solve_opts(dg_solve_opts *o) {
  if (!o) return;
  o->krylov = DG_KRYLOV_FCG;
  o->restart = 30;
  o->rtol = 1e-8;
  o->maxit = 500;
  o->precond = DG_PRECOND_MG;
  o->precond_precision = DG_FP32;
  dg_default_mg_opts(&o->mg);
  o->u_ref = nullptr;
  o->inner_stats = 0;
}

int dg_assemble_rhs(dg_problem *pr, const double *f_qp, const double *bnd_qp, double *rhs, void *stream) {
  if (!pr) {
    set_error("problem is NULL");
    return DG_EINVAL;
  }
  int rc = check_vec(rhs, "rhs");
  if (rc) return rc;
  return launch_rhs(pr, f_qp, bnd_qp, rhs, S(stream));
}

int dg_apply(dg_problem *pr, int precision, const void *u, void *v, void *stream) {
  if (!pr) {
    set_error("problem is NULL");
    return DG_EINVAL;
  }
  int rc;
  if ((rc = check_prec(precision)) || (rc = check_vec(u, "u")) || (rc = check_vec(v, "v"))) return rc;
  if (u == v) {
    set_error("dg_apply: u and v must differ");
    return DG_EINVAL;
  }
  return launch_apply(pr, precision, u, v, S(stream));
}

int dg_block_apply(dg_problem *pr, int precision, const void *x, void *y, void *stream) {
  if (!pr) {
    set_error("problem is NULL");
    return DG_EINVAL;
  }
  int rc;
  if ((rc = check_prec(precision)) || (rc = check_vec(x, "x")) || (rc = check_vec(y, "y"))) return rc;
  if (x == y) {
    set_error("dg_block_apply: x and y must differ");
    return DG_EINVAL;
  }
  return launch_block_apply(pr, precision, x, y, S(stream));
}

int dg_block_diag(dg_problem *pr, int precision, void *diag, void *stream) {
  if (!pr) {
    set_error("problem is NULL");
    return DG_EINVAL;
  }
  int rc;
  if ((rc = check_prec(precision)) || (rc = check_vec(diag, "diag"))) return rc;
  return launch_block_diag(pr, precision, diag, S(stream));
}

int dg_block_solve(dg_problem *pr, int precision, const void *d, void *x, const dg_smooth_opts *opts, int *iters,
                   void *stream) {
  if (!pr) {
    set_error("problem is NULL");
    return DG_EINVAL;
  }
  int rc;
  if ((rc = check_prec(precision)) || (rc = check_vec(d, "d")) || (rc = check_vec(x, "x"))) return rc;
  if (d == x) {
    set_error("dg_block_solve: d and x must differ");
    return DG_EINVAL;
  }
  SmoothArgs a;
  if ((rc = smooth_args(pr, opts, a))) return rc;
  a.zero_guess = 1;
  a.write_du = 1;
  a.defect = 0;
  return launch_smooth(pr, precision, d, d, x, a, iters, S(stream));
}

int dg_block_smooth(dg_problem *pr, int precision, const void *f, const void *u_in, void *u_out,
                    const dg_smooth_opts *opts, dg_smooth_stats *stats, void *stream) {
  return block_smooth_impl(pr, precision, f, u_in, u_out, opts, stats, S(stream), nullptr);
}

int dg_block_smooth_noalloc(dg_problem *pr, int precision, const void *f, const void *u_in, void *u_out,
                            const dg_smooth_opts *opts, dg_smooth_stats *stats, void *stream) {
  if (!pr) {
    set_error("problem is NULL");
    return DG_EINVAL;
  }
  int rc;
  if ((rc = check_prec(precision))) return rc;
  if (!opts) {
    set_error("smoother options are NULL");
    return DG_EINVAL;
  }
  if ((opts->inner == DG_INNER_FDM && !(pr->fdm[DG_FP64] && pr->fdm[DG_FP32])) ||
      (opts->inner == DG_INNER_PMF && !(pr->pmf[DG_FP64] && pr->pmf[DG_FP32]))) {
    set_error("dg_block_smooth_noalloc: the stored factors of DG_INNER_FDM / DG_INNER_PMF do not exist yet (a "
              "call of dg_block_smooth with that inner solve builds them)");
    return DG_EINVAL;
  }
  int dev = -1;
  DG_HIP(hipGetDevice(&dev));
  if (dev != pr->device) {
    set_error("dg_block_smooth_noalloc: the problem's device is not the current device");
    return DG_EINVAL;
  }
  // scratch layout: [ping-pong vector (Jacobi, n_sweeps > 1)][per-cell
  // iteration counts][two reduction results]; every part is written before
  // it is read within one call, so nothing has to start at zero
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  const bool jac_alt = opts->sweep == DG_SWEEP_JACOBI && opts->n_sweeps > 1;
  const size_t alt_bytes = jac_alt ? up((size_t)pr->ndof * esize(precision)) : 0;
  const size_t cnt_bytes = stats ? up((size_t)pr->ncell * sizeof(int)) : 0;
  const size_t red_bytes = stats ? 256 : 0;
  const size_t need = alt_bytes + cnt_bytes + red_bytes;
  const size_t cap = scratch_capacity();
  if (need > cap) {
    set_error("dg_block_smooth_noalloc: needs " + std::to_string(need) + " bytes of scratch, more than its fixed " +
              std::to_string(cap) + " bytes");
    return DG_EINVAL;
  }
  char *base = nullptr;
  if (need > 0 && (rc = scratch_device_ptr(dev, (void **)&base))) return rc;
  ScratchParts sp;
  sp.alt = jac_alt ? base : nullptr;
  sp.iters = stats ? (int *)(base + alt_bytes) : nullptr;
  sp.red = stats ? (unsigned long long *)(base + alt_bytes + cnt_bytes) : nullptr;
  return block_smooth_impl(pr, precision, f, u_in, u_out, opts, stats, S(stream), &sp);
}

int dg_mg_vcycle(dg_problem *pr, int precision, const void *r, void *z, const dg_mg_opts *opts, void *stream) {
  if (!pr || !opts) {
    set_error("problem or options are NULL");
    return DG_EINVAL;
  }
  int rc;
  if ((rc = check_prec(precision)) || (rc = check_vec(r, "r")) || (rc = check_vec(z, "z"))) return rc;
  if (r == z) {
    set_error("dg_mg_vcycle: r and z must differ");
    return DG_EINVAL;
  }
  if ((rc = validate_mg_opts(opts))) return rc;
  return vcycle(pr, precision, r, z, opts, S(stream));
}

int dg_coarse_csr(dg_problem *pr, int coarse_space, int level, int which, int64_t *dims, int *row_ptr, int *col,
                  double *val) {
  if (!pr || !dims) {
    set_error("dg_coarse_csr: problem or dims is NULL");
    return DG_EINVAL;
  }
  if (coarse_space != DG_COARSE_P0 && coarse_space != DG_COARSE_Q1) {
    set_error("coarse_space must be DG_COARSE_P0 or DG_COARSE_Q1");
    return DG_EINVAL;
  }
  if (row_ptr && (!col || !val)) {
    set_error("dg_coarse_csr: row_ptr given without col / val");
    return DG_EINVAL;
  }
  return amg_level_csr(pr, coarse_space == DG_COARSE_Q1 ? COARSE_Q1 : COARSE_P0, level, which, dims, row_ptr, col,
                       val);
}

int dg_coarse_stencil(dg_problem *pr, int coarse_space, int level, int *dims, double *out) {
  if (!pr || !dims) {
    set_error("dg_coarse_stencil: problem or dims is NULL");
    return DG_EINVAL;
  }
  if (coarse_space != DG_COARSE_P0 && coarse_space != DG_COARSE_Q1) {
    set_error("coarse_space must be DG_COARSE_P0 or DG_COARSE_Q1");
    return DG_EINVAL;
  }
  const int kind = coarse_space == DG_COARSE_Q1 ? COARSE_Q1 : COARSE_P0;
  int rc = ensure_hierarchy(pr, kind);
  if (rc) return rc;
  const Hierarchy &H = kind == COARSE_Q1 ? pr->q1h : pr->p0h;
  if (level < 0 || level >= (int)H.levels.size()) {
    set_error("dg_coarse_stencil: level out of range");
    return DG_EINVAL;
  }
  const CoarseLevel &L = H.levels[level];
  dims[0] = L.nx;
  dims[1] = L.ny;
  dims[2] = L.nz;
  dims[3] = L.ns;
  dims[4] = (int)H.levels.size();
  if (out) DG_HIP(hipMemcpy(out, L.A64, (size_t)L.ns * L.n * sizeof(double), hipMemcpyDeviceToHost));
  return DG_OK;
}

}  // extern "C"

// exported for solve.cpp
namespace dgmg {

int check_solve_vectors(const double *f, const double *u, const dg_solve_opts *o) {
  int rc;
  if ((rc = check_vec(f, "f")) || (rc = check_vec(u, "u"))) return rc;
  if (f == u) {
    set_error("solve: f and u must differ");
    return DG_EINVAL;
  }
  if (o->u_ref) {
    if ((rc = check_vec(o->u_ref, "u_ref"))) return rc;
    if (o->u_ref == f || o->u_ref == u) {
      set_error("solve: u_ref must differ from f and u");
      return DG_EINVAL;
    }
  }
  if (o->inner_stats != 0 && o->inner_stats != 1) {
    set_error("solve: inner_stats must be 0 or 1");
    return DG_EINVAL;
  }
  return DG_OK;
}

int inner_count_begin(dg_problem *pr, const dg_solve_opts *o, hipStream_t s) {
  pr->count_inner = 0;
  for (auto &m : pr->phase_marks) {
    pr->phase_spare.push_back(m.a);
    pr->phase_spare.push_back(m.b);
  }
  pr->phase_marks.clear();
  if (!o->inner_stats) return DG_OK;
  DG_HIP(hipMemsetAsync(pr->inner_acc, 0, 3 * sizeof(unsigned long long), s));
  pr->count_inner = 1;
  return DG_OK;
}

int inner_count_end(dg_problem *pr, const dg_solve_opts *o, dg_solve_result *res, hipStream_t s) {
  pr->count_inner = 0;
  if (!o->inner_stats) return DG_OK;
  unsigned long long h[3];
  DG_HIP(hipMemcpyAsync(h, pr->inner_acc, sizeof(h), hipMemcpyDeviceToHost, s));
  DG_HIP(hipStreamSynchronize(s));
  res->inner_blocks = (long long)h[2];
  res->inner_max = (int)h[1];
  res->inner_avg = h[2] ? (double)h[0] / (double)h[2] : 0.0;
  double t[4] = {0.0, 0.0, 0.0, 0.0};
  for (auto &m : pr->phase_marks) {
    float ms = 0.f;
    DG_HIP(hipEventElapsedTime(&ms, m.a, m.b));
    t[m.phase] += 1e-3 * ms;
    pr->phase_spare.push_back(m.a);
    pr->phase_spare.push_back(m.b);
  }
  pr->phase_marks.clear();
  res->t_smoother = t[PH_SMOOTH];
  res->t_restrict = t[PH_RESTRICT];
  res->t_coarse = t[PH_COARSE];
  res->t_prolong = t[PH_PROLONG];
  return DG_OK;
}

int solution_error(int64_t n, const double *u, const double *u_ref, double *tmp, double *part, double *dout,
                   hipStream_t s, double *err) {
  *err = -1.0;
  if (!u_ref) return DG_OK;
  int rc = sub(n, u, u_ref, tmp, s);
  if (rc) return rc;
  DotSet ds;
  ds.m = 2;
  ds.a[0] = tmp;
  ds.b[0] = tmp;
  ds.a[1] = u_ref;
  ds.b[1] = u_ref;
  if ((rc = dots(ds, n, part, dout, s))) return rc;
  double h[2];
  DG_HIP(hipMemcpyAsync(h, dout, sizeof(h), hipMemcpyDeviceToHost, s));
  DG_HIP(hipStreamSynchronize(s));
  *err = h[1] > 0 ? std::sqrt(h[0] / h[1]) : std::sqrt(h[0]);
  return DG_OK;
}

namespace {
// the preconditioner proper on rin -> zout in precision prec
// cb (Jacobi sweeps in the Gauss-point basis): the last sweep also takes
// the dots (and, FP32, the cast back); *fused tells whether it did.
int precond_run(dg_problem *pr, const dg_solve_opts *o, int prec, const void *rin, void *zout, hipStream_t s,
                const CastBackArgs *cb = nullptr, bool *fused = nullptr) {
  int rc;
  if (fused) *fused = false;
  if (pr->basis != DG_BASIS_GL || !smooth_takes_dots(prec, o->mg.smooth.inner)) cb = nullptr;
  if (o->precond == DG_PRECOND_MG) {
    if (prec == DG_FP32)
      rc = vcycle_t<float>(pr, prec, (const float *)rin, (float *)zout, &o->mg, s, cb, fused);
    else
      rc = vcycle_t<double>(pr, prec, (const double *)rin, (double *)zout, &o->mg, s, cb, fused);
    if (rc) return rc;
  } else {
    // block smoother steps from zero: mg.smooth.n_sweeps of mg.smooth.sweep
    SmoothArgs a;
    if ((rc = smooth_args(pr, &o->mg.smooth, a))) return rc;
    if ((rc = phase_begin(pr, PH_SMOOTH, s))) return rc;
    const int n = o->mg.smooth.n_sweeps > 1 ? o->mg.smooth.n_sweeps : 1;
    if (a.sweep != DG_SWEEP_JACOBI) {
      rc = sor_sweeps(pr, prec, rin, nullptr, zout, n, a.sweep, a, s);
    } else if (n == 1) {
      a.zero_guess = 1;
      a.cb = cb;
      rc = launch_smooth(pr, prec, rin, rin, zout, a, count_buf(pr, nullptr), s);
      if (!rc) rc = count_step(pr, nullptr, s);
      if (!rc && cb && fused) *fused = true;
    } else {
      void *alt;
      if ((rc = alloc_tmp(pr, prec, 2, &alt))) return rc;
      rc = sweeps(pr, prec, rin, nullptr, zout, alt, n, a, nullptr, s, nullptr, cb);
      if (!rc && cb && fused) *fused = true;
    }
    if (rc || (rc = phase_end(pr, s))) return rc;
  }
  return DG_OK;
}

// z = M(r); with an FP32 preconditioner r is scaled by 1 / ||r||_2 (host
// value rnorm) before the cast and z scaled back after it.
int precond_core(dg_problem *pr, const dg_solve_opts *o, const double *r, double *z, double rnorm, float *r32,
                 float *z32, hipStream_t s) {
  int rc;
  if (o->precond == DG_PRECOND_NONE) {
    DG_HIP(hipMemcpyAsync(z, r, (size_t)pr->ndof * sizeof(double), hipMemcpyDeviceToDevice, s));
    return DG_OK;
  }
  const bool mixed = o->precond_precision == DG_FP32;
  const double sc = (mixed && rnorm > 0) ? 1.0 / rnorm : 1.0;
  const void *rin = r;
  void *zout = z;
  if (mixed) {
    rc = cast_d2f(pr->ndof, sc, r, r32, s);
    if (rc) return rc;
    rin = r32;
    zout = z32;
  }
  if ((rc = precond_run(pr, o, mixed ? DG_FP32 : DG_FP64, rin, zout, s))) return rc;
  if (mixed) {
    rc = cast_f2d(pr->ndof, 1.0 / sc, z32, z, s);
    if (rc) return rc;
  }
  return DG_OK;
}
}  // namespace

int precond_apply(dg_problem *pr, const dg_solve_opts *o, const double *r, double *z, double rnorm, float *r32,
                  float *z32, hipStream_t s) {
  return precond_core(pr, o, r, z, rnorm, r32, z32, s);
}

int precond_apply_fp32_dots(dg_problem *pr, const dg_solve_opts *o, const float *r32, float *z32, double *z,
                            const double *rr_dev, int m, const double *b0, const double *b1, double *part,
                            double *out, hipStream_t s) {
  // the cast back and the dots in the last smoothing sweep where it is a
  // Gauss-point Jacobi sweep, else in a pass of their own
  CastBackArgs cb;
  cb.rr = rr_dev;
  cb.z = z;
  cb.b0 = b0;
  cb.b1 = b1;
  cb.part = part;
  cb.m = m;
  bool fused = false;
  int rc = precond_run(pr, o, DG_FP32, r32, z32, s, &cb, &fused);
  if (rc) return rc;
  if (fused) return dots_final(m, (int)smooth_blocks(pr->p, pr->ncell), part, out, s);
  return cast_back_dots(pr->ndof, rr_dev, z32, z, m, b0, b1, part, out, s);
}

int precond_apply_fp64_dots(dg_problem *pr, const dg_solve_opts *o, const double *r, double *z, int m,
                            const double *b0, const double *b1, double *part, double *out, hipStream_t s) {
  // the dots in the last smoothing sweep where it is a Gauss-point Jacobi
  // sweep, else in a pass of their own
  CastBackArgs cb;
  cb.b0 = b0;
  cb.b1 = b1;
  cb.part = part;
  cb.m = m;
  bool fused = false;
  int rc;
  if (o->precond == DG_PRECOND_NONE) {
    DG_HIP(hipMemcpyAsync(z, r, (size_t)pr->ndof * sizeof(double), hipMemcpyDeviceToDevice, s));
  } else if ((rc = precond_run(pr, o, DG_FP64, r, z, s, &cb, &fused))) {
    return rc;
  }
  if (fused) return dots_final(m, (int)smooth_blocks(pr->p, pr->ncell), part, out, s);
  DotSet ds;
  ds.m = m;
  ds.a[0] = z;
  ds.b[0] = b0;
  ds.a[1] = z;
  ds.b[1] = b1;
  return dots(ds, pr->ndof, part, out, s);
}
}  // namespace dgmg
