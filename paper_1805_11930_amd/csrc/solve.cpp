// Outer Krylov solvers of dg_solve: FP64 CG / flexible CG / flexible
// GMRES(m) around the hybrid-multigrid (or block-Jacobi) preconditioner,
// which may run in FP32 (iterative refinement: the outer residuals, inner
// products and the operator apply stay in FP64).
//
// Sec. 4.2 solves the diffusion problems with CG to ||r||/||r_0|| = 1e-8;
// Sec. 4.3 uses flexible GMRES for the convection-dominated problem.  A
// preconditioner with inexact inner block solves, or one applied in FP32,
// is not a fixed linear operator, so the flexible variants are the
// defaults: flexible CG uses the Polak-Ribiere form of beta, and FGMRES
// keeps the preconditioned vectors Z.  Before the FP32 cast the residual
// is scaled by 1/||r||_2 so that it is O(1) whatever the problem scale.
#include <chrono>
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "dg_internal.h"
#include "vec.h"

#include "solve_common.h"

using namespace dgmg;

namespace dgmg {
int solve_cg_batched(dg_problem *pr, const double *f, double *u, const dg_solve_opts *o, dg_solve_result *res,
                     hipStream_t s);

int validate_solve_opts(const dg_solve_opts *o) {
  if (o->krylov < DG_KRYLOV_CG || o->krylov > DG_KRYLOV_FGMRES || o->precond < DG_PRECOND_NONE ||
      o->precond > DG_PRECOND_MG || (o->precond_precision != DG_FP64 && o->precond_precision != DG_FP32) ||
      !(o->rtol > 0) || o->maxit < 1) {
    set_error("invalid solve options");
    return DG_EINVAL;
  }
  if (o->precond == DG_PRECOND_MG) return validate_mg_opts(&o->mg);
  if (o->precond == DG_PRECOND_BLOCK && (o->mg.smooth.n_sweeps > 64 || o->mg.smooth.sweep < DG_SWEEP_JACOBI ||
                                         o->mg.smooth.sweep > DG_SWEEP_SOR_BACKWARD)) {
    set_error("block preconditioner: n_sweeps <= 64 and sweep DG_SWEEP_*");
    return DG_EINVAL;
  }
  return DG_OK;
}
}  // namespace dgmg

namespace {

// Timed phases: a pair of events around each FP64 apply (recorded by its
// dispatch) and each preconditioner application.  They are read at the
// host synchronisations the solver makes anyway (one per Arnoldi step), so
// timing adds no wait of its own.
struct TimedPair {
  hipEvent_t a = nullptr, b = nullptr;
  int kind = 0;  // 0: apply, 1: preconditioner
};

struct Ctx {
  dg_problem *pr;
  const dg_solve_opts *o;
  hipStream_t s;
  double *part, *dout;
  // pinned host copy of dout (the per-step copies to the host wait on it:
  // from pageable memory each took about 80 us)
  double *hout = nullptr;
  float *r32 = nullptr, *z32 = nullptr;
  int64_t n;
  std::vector<TimedPair> spare, pending;
  int created = 0;
  double t_apply = 0.0, t_precond = 0.0;
  int n_apply = 0, n_precond = 0;
  ~Ctx() {
    for (auto *v : {&spare, &pending})
      for (auto &tp : *v) {
        (void)hipEventDestroy(tp.a);
        (void)hipEventDestroy(tp.b);
      }
    if (hout) (void)hipHostFree(hout);
  }
};

// Reads the pending phase times; `wait`: wait for them first (otherwise the
// caller has just synchronised the stream).
int harvest(Ctx &c, bool wait) {
  for (auto &tp : c.pending) {
    if (wait) DG_HIP(hipEventSynchronize(tp.b));
    float ms = 0.f;
    DG_HIP(hipEventElapsedTime(&ms, tp.a, tp.b));
    if (tp.kind == 0) {
      c.t_apply += 1e-3 * ms;
      ++c.n_apply;
    } else {
      c.t_precond += 1e-3 * ms;
      ++c.n_precond;
    }
    c.spare.push_back(tp);
  }
  c.pending.clear();
  return DG_OK;
}

int take_pair(Ctx &c, int kind, TimedPair *out) {
  if (c.spare.empty()) {
    if (c.created >= 8) {
      int rc = harvest(c, true);
      if (rc) return rc;
    } else {
      TimedPair tp;
      DG_HIP(hipEventCreate(&tp.a));
      hipError_t e = hipEventCreate(&tp.b);
      if (e != hipSuccess) {
        (void)hipEventDestroy(tp.a);
        return hip_fail(e, "hipEventCreate");
      }
      ++c.created;
      c.spare.push_back(tp);
    }
  }
  *out = c.spare.back();
  c.spare.pop_back();
  out->kind = kind;
  return DG_OK;
}

// FP64 operator apply timed by HIP events that its dispatch records.
int timed_apply(Ctx &c, const double *u, double *v) {
  TimedPair tp;
  int rc = take_pair(c, 0, &tp);
  if (rc) return rc;
  c.pending.push_back(tp);
  return launch_apply(c.pr, DG_FP64, u, v, c.s, tp.a, tp.b);
}

int timed_precond(Ctx &c, const double *r, double *z, double rnorm) {
  TimedPair tp;
  int rc = take_pair(c, 1, &tp);
  if (rc) return rc;
  c.pending.push_back(tp);
  DG_HIP(hipEventRecord(tp.a, c.s));
  if ((rc = precond_apply(c.pr, c.o, r, z, rnorm, c.r32, c.z32, c.s))) return rc;
  DG_HIP(hipEventRecord(tp.b, c.s));
  return DG_OK;
}

int host_dots(Ctx &c, const DotSet &ds, double *out) {
  int rc = dots(ds, c.n, c.part, c.dout, c.s);
  if (rc) return rc;
  DG_HIP(hipMemcpyAsync(c.hout, c.dout, ds.m * sizeof(double), hipMemcpyDeviceToHost, c.s));
  DG_HIP(hipStreamSynchronize(c.s));
  for (int j = 0; j < ds.m; ++j) out[j] = c.hout[j];
  return harvest(c, false);
}

int host_dot(Ctx &c, const double *a, const double *b, double *out) {
  DotSet ds;
  ds.m = 1;
  ds.a[0] = a;
  ds.b[0] = b;
  return host_dots(c, ds, out);
}

int residual(Ctx &c, const double *f, const double *u, double *r, double *tmp) {
  int rc = timed_apply(c, u, tmp);
  if (rc) return rc;
  return sub(c.n, f, tmp, r, c.s);
}

int solve_fgmres(Ctx &c, const double *f, double *u, dg_solve_result *res, DevBuf &wb, double r0) {
  const int m = c.o->restart > 0 ? (c.o->restart < kMaxBasis - 1 ? c.o->restart : kMaxBasis - 1) : 30;
  std::vector<double *> V(m + 1), Z(m);
  int rc;
  for (auto &v : V)
    if ((rc = wb.get(&v, c.n))) return rc;
  for (auto &z : Z)
    if ((rc = wb.get(&z, c.n))) return rc;
  double *r, *tmp;
  if ((rc = wb.get(&r, c.n)) || (rc = wb.get(&tmp, c.n))) return rc;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1);
  const double *h = c.hout;  // 2 kMaxBasis + 1 coefficients copied per step
  if ((rc = residual(c, f, u, r, tmp))) return rc;
  double beta = r0;
  int it = 0;
  res->status = DG_ENOCONV;
  bool done = false;
  while (!done && it < c.o->maxit) {
    if ((rc = axpby(c.n, 1.0 / beta, r, 0.0, V[0], c.s))) return rc;
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int k = 0;
    for (int j = 0; j < m; ++j) {
      if ((rc = timed_precond(c, V[j], Z[j], 1.0))) return rc;
      double *w = V[j + 1];
      if ((rc = timed_apply(c, Z[j], w))) return rc;
      // classical Gram-Schmidt applied twice, in three passes over the basis:
      // h1 = V^T w; w -= V h1 and h2 = V^T w; w -= V h2 and |w|^2.  The
      // coefficients stay on the device; one host copy per step.
      VecList vl;
      for (int i = 0; i <= j; ++i) vl.v[i] = V[i];
      double *h1 = c.dout, *h2 = c.dout + kMaxBasis, *nw = c.dout + 2 * kMaxBasis;
      if ((rc = gs_dot(vl, j + 1, w, c.n, c.part, h1, c.s))) return rc;
      if ((rc = gs_update_dot(vl, j + 1, h1, w, c.n, c.part, h2, c.s))) return rc;
      if ((rc = gs_update_norm(vl, j + 1, h2, w, c.n, c.part, nw, c.s))) return rc;
      DG_HIP(hipMemcpyAsync(c.hout, c.dout, (2 * kMaxBasis + 1) * sizeof(double), hipMemcpyDeviceToHost, c.s));
      DG_HIP(hipStreamSynchronize(c.s));
      if ((rc = harvest(c, false))) return rc;
      std::vector<double> hc(j + 1);
      for (int i = 0; i <= j; ++i) hc[i] = h[i] + h[kMaxBasis + i];
      const double hn2 = h[2 * kMaxBasis];
      const double hn = std::sqrt(hn2);
      for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hc[i];
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * H[(size_t)i * m + j] + sn[i] * H[(size_t)(i + 1) * m + j];
        H[(size_t)(i + 1) * m + j] = -sn[i] * H[(size_t)i * m + j] + cs[i] * H[(size_t)(i + 1) * m + j];
        H[(size_t)i * m + j] = t;
      }
      const double hj = H[(size_t)j * m + j];
      const double rr = std::hypot(hj, hn);
      cs[j] = hj / rr;
      sn[j] = hn / rr;
      H[(size_t)j * m + j] = rr;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      ++it;
      k = j + 1;
      if (!std::isfinite(g[j + 1])) {
        res->status = DG_EBREAKDOWN;
        set_error("non-finite residual estimate in FGMRES");
        done = true;
        break;
      }
      if (std::fabs(g[j + 1]) <= c.o->rtol * r0 || it >= c.o->maxit || hn == 0.0) {
        done = true;
        break;
      }
      if ((rc = axpby(c.n, 1.0 / hn, w, 0.0, w, c.s))) return rc;
    }
    // y = H^-1 g, u += Z y
    std::vector<double> y(k);
    for (int i = k - 1; i >= 0; --i) {
      double s = g[i];
      for (int l = i + 1; l < k; ++l) s -= H[(size_t)i * m + l] * y[l];
      y[i] = s / H[(size_t)i * m + i];
    }
    VecList zl;
    Coefs yc;
    for (int i = 0; i < k; ++i) {
      zl.v[i] = Z[i];
      yc.c[i] = y[i];
    }
    if ((rc = mcombine(zl, yc, k, c.n, u, c.s))) return rc;
    if ((rc = residual(c, f, u, r, tmp))) return rc;
    double rr;
    if ((rc = host_dot(c, r, r, &rr))) return rc;
    beta = std::sqrt(rr);
    if (beta <= c.o->rtol * r0) {
      res->status = DG_OK;
      done = true;
    } else if (done && res->status != DG_EBREAKDOWN) {
      done = it >= c.o->maxit;  // estimate converged but true residual not yet: restart
    }
  }
  res->iters = it;
  return DG_OK;
}

}  // namespace

extern "C" int dg_solve(dg_problem *pr, const double *f, double *u, const dg_solve_opts *o, dg_solve_result *res,
                        void *stream) {
  if (!pr || !f || !u || !o) {
    set_error("dg_solve: NULL argument");
    return DG_EINVAL;
  }
  int rc = validate_solve_opts(o);
  if (!rc) rc = check_solve_vectors(f, u, o);
  if (rc) return rc;
  dg_solve_result tmp;
  if (!res) res = &tmp;
  std::memset(res, 0, sizeof(*res));
  res->error = -1.0;
  hipStream_t s = (hipStream_t)stream;
  if (o->krylov != DG_KRYLOV_FGMRES) return solve_cg_batched(pr, f, u, o, res, s);
  const double t0 = now_s();
  DevBuf wb;
  Ctx c;
  c.pr = pr;
  c.o = o;
  c.s = s;
  c.n = pr->ndof;
  if ((rc = wb.get(&c.part, (size_t)kMaxBasis * kDotBlocks)) || (rc = wb.get(&c.dout, 2 * kMaxBasis + 1))) return rc;
  {
    const hipError_t e = hipHostMalloc((void **)&c.hout, (2 * kMaxBasis + 1) * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) {
      c.hout = nullptr;
      return hip_fail(e, "hipHostMalloc");
    }
  }
  if (o->precond_precision == DG_FP32 && o->precond != DG_PRECOND_NONE) {
    if ((rc = wb.get(&c.r32, c.n)) || (rc = wb.get(&c.z32, c.n))) return rc;
  }
  // preconditioner temporaries are allocated here so that the solve phase
  // measures no allocation
  void *dummy;
  if (o->precond == DG_PRECOND_MG && (rc = alloc_tmp(pr, o->precond_precision, 0, &dummy))) return rc;
  double *r, *t;
  if ((rc = wb.get(&r, c.n)) || (rc = wb.get(&t, c.n))) return rc;
  if ((rc = inner_count_begin(pr, o, s))) return rc;
  struct CountGuard {
    dg_problem *pr;
    ~CountGuard() { pr->count_inner = 0; }
  } count_guard{pr};
  DG_HIP(hipStreamSynchronize(s));
  const double t1 = now_s();
  if ((rc = residual(c, f, u, r, t))) return rc;
  double rr0;
  if ((rc = host_dot(c, r, r, &rr0))) return rc;
  const double r0 = std::sqrt(rr0);
  if (!std::isfinite(r0)) {
    set_error("initial residual is not finite");
    res->status = DG_EBREAKDOWN;
    return DG_EBREAKDOWN;
  }
  if (r0 == 0.0) {
    res->status = DG_OK;
  } else if ((rc = solve_fgmres(c, f, u, res, wb, r0))) {
    return rc;
  }
  // true FP64 residual
  if ((rc = residual(c, f, u, r, t))) return rc;
  double rr;
  if ((rc = host_dot(c, r, r, &rr))) return rc;
  const double t2 = now_s();
  if ((rc = inner_count_end(pr, o, res, s))) return rc;
  if ((rc = solution_error(c.n, u, o->u_ref, t, c.part, c.dout, s, &res->error))) return rc;
  res->rel_residual = r0 > 0 ? std::sqrt(rr) / r0 : 0.0;
  res->t_setup = t1 - t0;
  res->t_solve = t2 - t1;
  res->footprint = pr->held_bytes + wb.bytes;
  if ((rc = harvest(c, true))) return rc;
  res->t_apply = c.t_apply;
  res->n_apply = c.n_apply;
  res->t_precond = c.t_precond;
  res->n_precond = c.n_precond;
  if (res->status == DG_OK && !(res->rel_residual <= o->rtol * 1.0000001)) res->status = DG_ENOCONV;
  return res->status;
}

extern "C" int dg_footprint(const dg_problem_desc *d, const dg_solve_opts *o, size_t *bytes) {
  if (!d || !bytes) {
    set_error("dg_footprint: NULL argument");
    return DG_EINVAL;
  }
  if (d->p < 1 || d->p > DG_MAX_P || d->nx < 1 || d->ny < 1 || d->nz < 1) {
    set_error("dg_footprint: invalid description");
    return DG_EINVAL;
  }
  const int64_t ncell = (int64_t)d->nx * d->ny * d->nz;
  const int64_t nloc = (int64_t)(d->p + 1) * (d->p + 1) * (d->p + 1);
  const int64_t ndof = ncell * nloc;
  size_t b = 0;
  b += ncell * 4 * sizeof(double);       // K, c
  b += ncell * sizeof(int) + 8 * 1024 * sizeof(double) + 64;
  dg_solve_opts def;
  if (!o) {
    dg_default_solve_opts(&def);
    o = &def;
  }
  const size_t both = sizeof(double) + sizeof(float);
  bool has_b = false;
  for (int i = 0; i < 3; ++i) has_b = has_b || d->b0[i] != 0.0;
  for (int i = 0; i < 9; ++i) has_b = has_b || d->B[i] != 0.0;
  const bool q1 = o->precond == DG_PRECOND_MG &&
                  coarse_kind(o->mg.coarse_space, has_b, d->basis == DG_BASIS_GLL) == COARSE_Q1;
  if (o->precond == DG_PRECOND_MG && !q1) {
    // P0 hierarchy: levels ~8/7 of level 0, 7 stencil entries + 3 vectors
    // per unknown, 2 more vectors on level 0, dense bottom
    const int64_t nco = ncell + ncell / 7 + 1;
    b += (nco * (7 + 3) + 2 * ncell) * both;
    b += 128 * 128 * both;
  }
  if (q1) {
    // Q1 hierarchy: vertex levels (27-point stencils), corner sums
    const int64_t nv = (int64_t)(d->nx + 1) * (d->ny + 1) * (d->nz + 1);
    b += ((nv + nv / 7 + 1) * (27 + 3) + 2 * nv) * both;
    b += 8 * ncell * both + 128 * 128 * both;
  }
  if (d->basis == DG_BASIS_GLL) {
    // basis-change scratch (three vectors) and the stored block diagonal,
    // band and band factors (four vectors), both precisions
    b += 7 * ndof * both;
  }
  if (o->precond == DG_PRECOND_MG && o->mg.coarse_solver == DG_COARSE_SOLVER_AMG) {
    // AMG levels below the coarse space: P and R (about 10 entries per fine
    // unknown each) and the Galerkin matrices (about 2 more per fine unknown)
    const int64_t n0 = q1 ? (int64_t)(d->nx + 1) * (d->ny + 1) * (d->nz + 1) : ncell;
    b += n0 * (22 * (both + sizeof(int)) + 4 * both);
  }
  const size_t pe = o->precond_precision == DG_FP32 ? sizeof(float) : sizeof(double);
  if (o->precond == DG_PRECOND_MG) b += 2 * ndof * pe;
  if (o->precond == DG_PRECOND_BLOCK && o->mg.smooth.sweep == DG_SWEEP_JACOBI && o->mg.smooth.n_sweeps > 1)
    b += ndof * pe;
  if (o->precond != DG_PRECOND_NONE && o->mg.smooth.inner == DG_INNER_FDM)
    b += ncell * 3 * (int64_t)(d->p + 1) * (d->p + 2) * both;  // stored factors T_k, lambda_k
  if (o->precond != DG_PRECOND_NONE && o->mg.smooth.inner == DG_INNER_PMF)
    b += (size_t)ncell * nloc * nloc * both;  // stored block inverses, FP64 and FP32
  if (o->precond_precision == DG_FP32 && o->precond != DG_PRECOND_NONE) b += 2 * ndof * sizeof(float);
  int64_t nvec = 2;  // residual + temporary of dg_solve
  if (o->krylov == DG_KRYLOV_FGMRES) {
    const int m = o->restart > 0 ? (o->restart < kMaxBasis - 1 ? o->restart : kMaxBasis - 1) : 30;
    nvec += 2 * m + 1 + 2;
  } else {
    nvec += o->krylov == DG_KRYLOV_FCG ? 5 : 4;
  }
  b += nvec * ndof * sizeof(double);
  const int64_t npart = std::max<int64_t>(
      {(int64_t)kMaxBasis * kDotBlocks, apply_blocks(d->p, ncell), 2 * smooth_blocks(d->p, ncell)});
  b += (npart + kMaxBasis) * sizeof(double);
  *bytes = b;
  return DG_OK;
}
