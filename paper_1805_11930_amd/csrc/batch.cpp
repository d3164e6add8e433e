// Resident solve states and continuous batching of outer CG iterations.
//
// A solve state holds one request's outer FP64 (flexible) CG iteration
// (Sec. 4.2: CG to a relative residual; flexible beta because the FP32 /
// inexact V-cycle preconditioner is not a fixed linear operator) together
// with its workspace and its own HIP stream (default priority).  One
// iteration is split into three phases, each ending in a host scalar
// decision:
//   A: q = A p, (p, q)              -> alpha
//   B: u += alpha p, r -= alpha q, (r, r)  -> convergence test
//   C: z = M(r), (z, r), (z, r_old) -> beta, p = z + beta p
// dg_batch_step runs phase A for every active state, waits once for all,
// then B, then C, so a batch of requests pays three host round trips per
// iteration in total and their kernels overlap on the device (one stream
// per request).  Each request's arithmetic is exactly the same as alone:
// nothing is shared between requests except the device.
#include <cmath>
#include <cstring>
#include <vector>

#include "dg_internal.h"
#include "solve_common.h"
#include "vec.h"

using namespace dgmg;

struct dg_solve_state {
  dg_problem *pr = nullptr;
  dg_solve_opts o;
  const double *f = nullptr;
  double *u = nullptr;
  hipStream_t s = nullptr;
  bool own_stream = false;
  DevBuf wb;
  double *r = nullptr, *p = nullptr, *q = nullptr, *z = nullptr, *rold = nullptr;
  float *r32 = nullptr, *z32 = nullptr;
  double *part = nullptr, *dout = nullptr;
  double *hdots = nullptr;  // pinned host copy of the phase's inner products
  hipEvent_t ea0 = nullptr, ea1 = nullptr, ep0 = nullptr, ep1 = nullptr;
  bool flex = true;
  double r0 = 0, rnorm = 0, rz = 0, alpha = 0;
  int it = 0;
  bool done = false, finalized = false;
  double t_start = 0, t_iter0 = 0;
  double t_apply = 0, t_precond = 0;
  int n_apply = 0, n_precond = 0;
  dg_solve_result res;

  ~dg_solve_state() {
    for (hipEvent_t e : {ea0, ea1, ep0, ep1})
      if (e) (void)hipEventDestroy(e);
    if (hdots) (void)hipHostFree(hdots);
    if (own_stream && s) (void)hipStreamDestroy(s);
  }
};

namespace dgmg {

namespace {

int enqueue_dots(dg_solve_state *st, int m, const double *a0, const double *b0, const double *a1 = nullptr,
                 const double *b1 = nullptr) {
  DotSet ds;
  ds.m = m;
  ds.a[0] = a0;
  ds.b[0] = b0;
  ds.a[1] = a1;
  ds.b[1] = b1;
  int rc = dots(ds, st->pr->ndof, st->part, st->dout, st->s);
  if (rc) return rc;
  DG_HIP(hipMemcpyAsync(st->hdots, st->dout, m * sizeof(double), hipMemcpyDeviceToHost, st->s));
  return DG_OK;
}

float elapsed_ms(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) ms = 0.f;
  return ms;
}

void finish(dg_solve_state *st, int status) {
  st->done = true;
  st->res.status = status;
}

// ---- phases ------------------------------------------------------------
int enqueue_A(dg_solve_state *st) {
  DG_HIP(hipEventRecord(st->ea0, st->s));
  int rc = launch_apply(st->pr, DG_FP64, st->p, st->q, st->s);
  if (rc) return rc;
  DG_HIP(hipEventRecord(st->ea1, st->s));
  return enqueue_dots(st, 1, st->p, st->q);
}

void complete_A(dg_solve_state *st) {
  st->t_apply += 1e-3 * elapsed_ms(st->ea0, st->ea1);
  ++st->n_apply;
  const double pq = st->hdots[0];
  if (!(pq > 0) || !std::isfinite(pq) || !std::isfinite(st->rz)) {
    set_error("CG breakdown: p^T A p <= 0 or not finite");
    finish(st, DG_EBREAKDOWN);
    return;
  }
  st->alpha = st->rz / pq;
}

int enqueue_B(dg_solve_state *st) {
  int rc;
  if (st->flex) {
    // the new residual goes to the other buffer; the previous one is kept
    if ((rc = cg_update(st->pr->ndof, st->alpha, st->p, st->q, st->u, st->r, st->rold, st->s))) return rc;
    std::swap(st->r, st->rold);
  } else if ((rc = cg_update(st->pr->ndof, st->alpha, st->p, st->q, st->u, st->r, st->r, st->s))) {
    return rc;
  }
  return enqueue_dots(st, 1, st->r, st->r);
}

void complete_B(dg_solve_state *st) {
  ++st->it;
  st->rnorm = std::sqrt(st->hdots[0]);
  if (!std::isfinite(st->rnorm)) {
    set_error("non-finite residual");
    finish(st, DG_EBREAKDOWN);
  } else if (st->rnorm <= st->o.rtol * st->r0) {
    finish(st, DG_OK);
  } else if (st->it >= st->o.maxit) {
    finish(st, DG_ENOCONV);
  }
}

int enqueue_C(dg_solve_state *st) {
  DG_HIP(hipEventRecord(st->ep0, st->s));
  int rc = precond_apply(st->pr, &st->o, st->r, st->z, st->rnorm, st->r32, st->z32, st->s);
  if (rc) return rc;
  DG_HIP(hipEventRecord(st->ep1, st->s));
  if (st->flex) return enqueue_dots(st, 2, st->z, st->r, st->z, st->rold);
  return enqueue_dots(st, 1, st->z, st->r);
}

int complete_C(dg_solve_state *st) {
  st->t_precond += 1e-3 * elapsed_ms(st->ep0, st->ep1);
  ++st->n_precond;
  double beta;
  if (st->flex) {
    beta = (st->hdots[0] - st->hdots[1]) / st->rz;
  } else {
    beta = st->hdots[0] / st->rz;
  }
  st->rz = st->hdots[0];
  return axpby(st->pr->ndof, 1.0, st->z, beta, st->p, st->s);
}

// true FP64 residual of a finished state and its result record
int finalize(dg_solve_state *st) {
  int rc = launch_apply(st->pr, DG_FP64, st->u, st->q, st->s);
  if (rc) return rc;
  if ((rc = sub(st->pr->ndof, st->f, st->q, st->z, st->s))) return rc;
  if ((rc = enqueue_dots(st, 1, st->z, st->z))) return rc;
  DG_HIP(hipStreamSynchronize(st->s));
  const double t_end = now_s();
  dg_solve_result &R = st->res;
  R.iters = st->it;
  R.rel_residual = st->r0 > 0 ? std::sqrt(st->hdots[0]) / st->r0 : 0.0;
  R.t_setup = st->t_iter0 - st->t_start;
  R.t_solve = t_end - st->t_iter0;
  R.footprint = st->pr->held_bytes + st->wb.bytes;
  R.t_apply = st->t_apply;
  R.n_apply = st->n_apply;
  R.t_precond = st->t_precond;
  R.n_precond = st->n_precond;
  if (R.status == DG_OK && !(R.rel_residual <= st->o.rtol * 1.0000001)) R.status = DG_ENOCONV;
  st->finalized = true;
  return DG_OK;
}

int start(dg_problem *pr, const double *f, double *u, const dg_solve_opts *o, hipStream_t s, bool own_stream,
          dg_solve_state **out) {
  *out = nullptr;
  if (!pr || !f || !u || !o) {
    set_error("solve start: NULL argument");
    return DG_EINVAL;
  }
  int rc = validate_solve_opts(o);
  if (rc) return rc;
  if (o->krylov == DG_KRYLOV_FGMRES) {
    set_error("resident solve states support CG and flexible CG");
    return DG_EINVAL;
  }
  dg_solve_state *st = new dg_solve_state();
  st->t_start = now_s();
  st->pr = pr;
  st->o = *o;
  st->f = f;
  st->u = u;
  st->flex = o->krylov == DG_KRYLOV_FCG;
  std::memset(&st->res, 0, sizeof(st->res));
  st->res.status = DG_EAGAIN;
  const int64_t n = pr->ndof;
  auto fail = [&](int code) {
    delete st;
    return code;
  };
  hipError_t e = hipSuccess;
  if (own_stream) {
    e = hipStreamCreateWithFlags(&st->s, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(hip_fail(e, "hipStreamCreateWithFlags"));
    st->own_stream = true;
  } else {
    st->s = s;
  }
  for (hipEvent_t *ev : {&st->ea0, &st->ea1, &st->ep0, &st->ep1}) {
    e = hipEventCreate(ev);
    if (e != hipSuccess) return fail(hip_fail(e, "hipEventCreate"));
  }
  e = hipHostMalloc((void **)&st->hdots, 4 * sizeof(double), hipHostMallocDefault);
  if (e != hipSuccess) return fail(hip_fail(e, "hipHostMalloc"));
  if ((rc = st->wb.get(&st->r, n)) || (rc = st->wb.get(&st->p, n)) || (rc = st->wb.get(&st->q, n)) ||
      (rc = st->wb.get(&st->z, n)) || (rc = st->wb.get(&st->part, (size_t)kMaxDots * kDotBlocks)) ||
      (rc = st->wb.get(&st->dout, kMaxDots)))
    return fail(rc);
  if (st->flex && (rc = st->wb.get(&st->rold, n))) return fail(rc);
  if (o->precond_precision == DG_FP32 && o->precond != DG_PRECOND_NONE) {
    if ((rc = st->wb.get(&st->r32, n)) || (rc = st->wb.get(&st->z32, n))) return fail(rc);
  }
  void *dummy;
  if (o->precond == DG_PRECOND_MG && (rc = alloc_tmp(pr, o->precond_precision, 0, &dummy))) return fail(rc);
  // r = f - A u, r0 = ||r||
  if ((rc = launch_apply(pr, DG_FP64, u, st->q, st->s)) || (rc = sub(n, f, st->q, st->r, st->s)) ||
      (rc = enqueue_dots(st, 1, st->r, st->r)))
    return fail(rc);
  e = hipStreamSynchronize(st->s);
  if (e != hipSuccess) return fail(hip_fail(e, "hipStreamSynchronize"));
  st->t_iter0 = now_s();
  st->r0 = std::sqrt(st->hdots[0]);
  st->rnorm = st->r0;
  if (!std::isfinite(st->r0)) {
    set_error("initial residual is not finite");
    return fail(DG_EBREAKDOWN);
  }
  if (st->r0 == 0.0) {
    finish(st, DG_OK);
  } else {
    // z = M(r), rho = (r, z), p = z
    if ((rc = precond_apply(pr, o, st->r, st->z, st->rnorm, st->r32, st->z32, st->s)) ||
        (rc = enqueue_dots(st, 1, st->r, st->z)))
      return fail(rc);
    e = hipStreamSynchronize(st->s);
    if (e != hipSuccess) return fail(hip_fail(e, "hipStreamSynchronize"));
    st->rz = st->hdots[0];
    e = hipMemcpyAsync(st->p, st->z, n * sizeof(double), hipMemcpyDeviceToDevice, st->s);
    if (e != hipSuccess) return fail(hip_fail(e, "hipMemcpyAsync"));
  }
  *out = st;
  return DG_OK;
}

int wait_all(dg_solve_state **sts, const std::vector<int> &idx) {
  for (int i : idx) DG_HIP(hipStreamSynchronize(sts[i]->s));
  return DG_OK;
}

int batch_step(dg_solve_state **sts, int n) {
  int rc;
  std::vector<int> act;
  for (int i = 0; i < n; ++i)
    if (!sts[i]->done) act.push_back(i);
  // phase A
  for (int i : act)
    if ((rc = enqueue_A(sts[i]))) return rc;
  if ((rc = wait_all(sts, act))) return rc;
  std::vector<int> act2;
  for (int i : act) {
    complete_A(sts[i]);
    if (!sts[i]->done) act2.push_back(i);
  }
  // phase B
  for (int i : act2)
    if ((rc = enqueue_B(sts[i]))) return rc;
  if ((rc = wait_all(sts, act2))) return rc;
  std::vector<int> act3;
  for (int i : act2) {
    complete_B(sts[i]);
    if (!sts[i]->done) act3.push_back(i);
  }
  // phase C
  for (int i : act3)
    if ((rc = enqueue_C(sts[i]))) return rc;
  if ((rc = wait_all(sts, act3))) return rc;
  for (int i : act3)
    if ((rc = complete_C(sts[i]))) return rc;
  // results of the requests that finished in this step
  for (int i : act)
    if (sts[i]->done && !sts[i]->finalized && (rc = finalize(sts[i]))) return rc;
  return DG_OK;
}

}  // namespace

int solve_cg_batched(dg_problem *pr, const double *f, double *u, const dg_solve_opts *o, dg_solve_result *res,
                     hipStream_t s) {
  dg_solve_state *st = nullptr;
  int rc = start(pr, f, u, o, s, false, &st);
  if (rc) return rc;
  while (!st->done && !rc) rc = batch_step(&st, 1);
  if (!rc && !st->finalized) rc = finalize(st);
  if (!rc) {
    *res = st->res;
    rc = res->status;
  }
  delete st;
  return rc;
}

}  // namespace dgmg

extern "C" {

int dg_solve_start(dg_problem *prob, const double *f, double *u, const dg_solve_opts *opts, dg_solve_state **out) {
  if (!out) {
    set_error("dg_solve_start: out is NULL");
    return DG_EINVAL;
  }
  return dgmg::start(prob, f, u, opts, nullptr, true, out);
}

int dg_batch_step(dg_solve_state **active, int n_active, void *stream) {
  (void)stream;  // every state runs on its own stream; the call returns after all of them
  if (n_active < 0 || (n_active > 0 && !active)) {
    set_error("dg_batch_step: bad state list");
    return DG_EINVAL;
  }
  for (int i = 0; i < n_active; ++i)
    if (!active[i]) {
      set_error("dg_batch_step: NULL state");
      return DG_EINVAL;
    }
  return dgmg::batch_step(active, n_active);
}

int dg_solve_poll(dg_solve_state *st, dg_solve_result *res) {
  if (!st) {
    set_error("dg_solve_poll: NULL state");
    return DG_EINVAL;
  }
  if (!st->done) return DG_EAGAIN;
  if (!st->finalized) {
    int rc = dgmg::finalize(st);
    if (rc) return rc;
  }
  if (res) *res = st->res;
  return DG_OK;
}

void dg_solve_state_destroy(dg_solve_state *st) { delete st; }

}  // extern "C"
