// Resident solve states and continuous batching of outer CG iterations.
//
// A solve state holds one request's outer FP64 (flexible) CG iteration
// (Sec. 4.2: CG to a relative residual; flexible beta because the FP32 /
// inexact V-cycle preconditioner is not a fixed linear operator) together
// with its workspace and its own HIP stream (default priority).  One
// iteration is enqueued as a whole, its scalars kept in device memory:
//   q = A p, pq = (p, q); u += alpha p, r -= alpha q with alpha = rz / pq;
//   rr = (r, r) -> copied to pinned host memory, event;
//   z = M(r) (FP32: scaled by 1 / sqrt(rr) on the device);
//   (z, r), (z, r_old); p = z + beta p, rz = (z, r).
// The host then only waits for the event after rr: it takes the
// convergence decision while the device runs the preconditioner, and the
// next iteration is enqueued behind it, so the device does not idle between
// iterations.  When the decision is "converged", the preconditioner and
// beta update of that iteration still run but touch only z, p and the
// scalars: u is the same as with a blocking test after every phase.
// dg_batch_step takes the pending decision of every active state and
// enqueues its next iteration; their kernels overlap on the device (one
// stream per request).  Each request's arithmetic is exactly the same as
// alone: nothing is shared between requests except the device.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "dg_internal.h"
#include "solve_common.h"
#include "vec.h"

using namespace dgmg;

namespace {

// Pinned host slots (8 doubles) and per-device streams reused by the solve
// states of the process: pinned allocation and stream creation cost more
// than the whole solve of a small request.  Held until the process ends.
struct StatePool {
  std::mutex m;
  std::vector<double *> slots;
  std::map<int, std::vector<hipStream_t>> streams;
};
StatePool &state_pool() {
  static StatePool *p = new StatePool();  // never destroyed: states may outlive static destruction order
  return *p;
}

constexpr int kSlotDoubles = 8, kSlotsPerBlock = 64;

int take_slot(double **out) {
  StatePool &P = state_pool();
  std::lock_guard<std::mutex> g(P.m);
  if (P.slots.empty()) {
    double *blk = nullptr;
    hipError_t e = hipHostMalloc((void **)&blk, sizeof(double) * kSlotDoubles * kSlotsPerBlock, hipHostMallocDefault);
    if (e != hipSuccess) return hip_fail(e, "hipHostMalloc");
    for (int k = kSlotsPerBlock - 1; k >= 0; --k) P.slots.push_back(blk + k * kSlotDoubles);
  }
  *out = P.slots.back();
  P.slots.pop_back();
  return DG_OK;
}

void give_slot(double *p) {
  StatePool &P = state_pool();
  std::lock_guard<std::mutex> g(P.m);
  P.slots.push_back(p);
}

int take_stream(hipStream_t *out) {
  int dev = 0;
  DG_HIP(hipGetDevice(&dev));
  StatePool &P = state_pool();
  {
    std::lock_guard<std::mutex> g(P.m);
    auto &v = P.streams[dev];
    if (!v.empty()) {
      *out = v.back();
      v.pop_back();
      return DG_OK;
    }
  }
  DG_HIP(hipStreamCreateWithFlags(out, hipStreamNonBlocking));
  return DG_OK;
}

// s was taken on the current device and has no work in flight
void give_stream(hipStream_t s) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipStreamDestroy(s);
    return;
  }
  StatePool &P = state_pool();
  std::lock_guard<std::mutex> g(P.m);
  P.streams[dev].push_back(s);
}

}  // namespace

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
  // device scalars: [0] pq, [1] rr of the FP32 scaling in use, [2] (z, r),
  // [3] (z, r_old), [4..5] rz by iteration parity, [6] rr, [7] breakdown flag
  double *dsc = nullptr;
  double *hdots = nullptr;  // pinned host: [0] setup dots, [1 + 2 par] rr and [2 + 2 par] flag by parity
  hipEvent_t ea0[2] = {nullptr, nullptr}, ea1[2] = {nullptr, nullptr};
  hipEvent_t ep0[2] = {nullptr, nullptr}, ep1[2] = {nullptr, nullptr}, err[2] = {nullptr, nullptr};
  int pending = -1;       // parity of the enqueued iteration whose decision is open
  int prec_unread = -1;   // parity of the last preconditioner not yet timed
  bool flex = true;
  double r0 = 0, rnorm = 0;
  int it = 0;
  bool done = false, finalized = false;
  bool counting = false;  // this state counts its preconditioner's inner iterations
  double t_start = 0, t_iter0 = 0;
  double t_apply = 0, t_precond = 0;
  int n_apply = 0, n_precond = 0;
  dg_solve_result res;

  ~dg_solve_state() {
    if (pr && counting) pr->count_inner = 0;
    // nothing of this solve may still run when its slot and stream are reused
    if (s) (void)hipStreamSynchronize(s);
    for (int k = 0; k < 2; ++k)
      for (hipEvent_t e : {ea0[k], ea1[k], ep0[k], ep1[k], err[k]})
        if (e) (void)hipEventDestroy(e);
    if (hdots) give_slot(hdots);
    if (own_stream && s) give_stream(s);
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

// ---- one outer iteration ---------------------------------------------------
// The apply computes (p, A p) itself (Gauss-point basis, not the
// rotated-tensor field)
bool fused_pq(const dg_problem *pr) {
  return pr->basis == DG_BASIS_GL && pr->geo.field != DG_FIELD_ROTATED_QUADRATIC;
}

int enqueue_iter(dg_solve_state *st) {
  const int par = st->it & 1;
  const int64_t n = st->pr->ndof;
  double *rz_cur = st->dsc + 4 + par, *rz_next = st->dsc + 4 + (par ^ 1);
  int rc;
  // q = A p, pq (fused into the apply where it has the fused form)
  // the events are recorded by the apply's dispatch (its own start and end)
  DotSet ds;
  if (fused_pq(st->pr)) {
    if ((rc = launch_apply_dot_gl(st->pr, st->p, st->q, st->part, st->s, st->ea0[par], st->ea1[par])) ||
        (rc = dots_final(1, (int)apply_blocks(st->pr->p, st->pr->ncell), st->part, st->dsc + 0, st->s)))
      return rc;
  } else {
    if ((rc = launch_apply(st->pr, DG_FP64, st->p, st->q, st->s, st->ea0[par], st->ea1[par]))) return rc;
    ds.m = 1;
    ds.a[0] = st->p;
    ds.b[0] = st->q;
    if ((rc = dots(ds, n, st->part, st->dsc + 0, st->s))) return rc;
  }
  // u += alpha p, r -= alpha q (flexible: the new residual goes to the other
  // buffer) and rr = (r, r) in the same pass
  double *r_out = st->flex ? st->rold : st->r;
  // with the FP32 preconditioner the same pass writes r in FP32, scaled by
  // the previous residual norm (its rr kept in dsc[1] for the cast back)
  const bool f32 = st->o.precond_precision == DG_FP32 && st->o.precond != DG_PRECOND_NONE;
  // (u += alpha p is left to the beta update, which reads p anyway)
  if ((rc = cg_update_rr(n, rz_cur, st->dsc + 0, st->p, st->q, nullptr, st->r, r_out, st->dsc + 7, st->part,
                         st->dsc + 6, st->s, f32 ? st->r32 : nullptr, st->dsc + 6, st->dsc + 1)))
    return rc;
  if (st->flex) std::swap(st->r, st->rold);
  // rr and the breakdown flag are adjacent: one copy to the host
  DG_HIP(hipMemcpyAsync(st->hdots + 1 + 2 * par, st->dsc + 6, 2 * sizeof(double), hipMemcpyDeviceToHost, st->s));
  DG_HIP(hipEventRecord(st->err[par], st->s));
  // z = M(r), beta, p
  DG_HIP(hipEventRecord(st->ep0[par], st->s));
  if (f32) {
    // z = M(r) and (z, r), (z, r_old) with the cast back
    if ((rc = precond_apply_fp32_dots(st->pr, &st->o, st->r32, st->z32, st->z, st->dsc + 1, st->flex ? 2 : 1, st->r,
                                      st->rold, st->part, st->dsc + 2, st->s)))
      return rc;
    DG_HIP(hipEventRecord(st->ep1[par], st->s));
  } else {
    // z = M(r) and (z, r), (z, r_old)
    if ((rc = precond_apply_fp64_dots(st->pr, &st->o, st->r, st->z, st->flex ? 2 : 1, st->r, st->rold, st->part,
                                      st->dsc + 2, st->s)))
      return rc;
    DG_HIP(hipEventRecord(st->ep1[par], st->s));
  }
  // p = z + beta p, and u += alpha p of the old p
  if ((rc = beta_update(n, st->dsc + 2, st->dsc + 3, rz_cur, rz_next, st->flex, st->z, st->p, st->s, st->u,
                        st->dsc + 0)))
    return rc;
  st->pending = par;
  return DG_OK;
}

void take_prec_time(dg_solve_state *st) {
  if (st->prec_unread < 0) return;
  st->t_precond += 1e-3 * elapsed_ms(st->ep0[st->prec_unread], st->ep1[st->prec_unread]);
  ++st->n_precond;
  st->prec_unread = -1;
}

// Waits for the residual norm of the pending iteration and decides.
int check_iter(dg_solve_state *st) {
  const int par = st->pending;
  st->pending = -1;
  DG_HIP(hipEventSynchronize(st->err[par]));
  st->t_apply += 1e-3 * elapsed_ms(st->ea0[par], st->ea1[par]);
  ++st->n_apply;
  take_prec_time(st);  // the previous iteration's preconditioner has finished
  st->prec_unread = par;
  if (st->hdots[2 + 2 * par] != 0.0) {
    set_error("CG breakdown: p^T A p <= 0 or not finite");
    finish(st, DG_EBREAKDOWN);
    return DG_OK;
  }
  ++st->it;
  st->rnorm = std::sqrt(st->hdots[1 + 2 * par]);
  if (!std::isfinite(st->rnorm)) {
    set_error("non-finite residual");
    finish(st, DG_EBREAKDOWN);
  } else if (st->rnorm <= st->o.rtol * st->r0) {
    finish(st, DG_OK);
  } else if (st->it >= st->o.maxit) {
    finish(st, DG_ENOCONV);
  }
  return DG_OK;
}

// true FP64 residual of a finished state and its result record
int finalize(dg_solve_state *st) {
  int rc = launch_apply(st->pr, DG_FP64, st->u, st->q, st->s);
  if (rc) return rc;
  if ((rc = sub(st->pr->ndof, st->f, st->q, st->z, st->s))) return rc;
  if ((rc = enqueue_dots(st, 1, st->z, st->z))) return rc;
  DG_HIP(hipStreamSynchronize(st->s));
  take_prec_time(st);
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
  if (st->counting) {
    st->counting = false;
    if ((rc = inner_count_end(st->pr, &st->o, &R, st->s))) return rc;
  }
  if ((rc = solution_error(st->pr->ndof, st->u, st->o.u_ref, st->q, st->part, st->dout, st->s, &R.error)))
    return rc;
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
  if (!rc) rc = check_solve_vectors(f, u, o);
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
  st->res.error = -1.0;
  const int64_t n = pr->ndof;
  auto fail = [&](int code) {
    delete st;
    return code;
  };
  hipError_t e = hipSuccess;
  if (own_stream) {
    if ((rc = take_stream(&st->s))) return fail(rc);
    st->own_stream = true;
  } else {
    st->s = s;
  }
  for (int k = 0; k < 2; ++k)
    for (hipEvent_t *ev : {&st->ea0[k], &st->ea1[k], &st->ep0[k], &st->ep1[k], &st->err[k]}) {
      e = hipEventCreate(ev);
      if (e != hipSuccess) return fail(hip_fail(e, "hipEventCreate"));
    }
  if ((rc = take_slot(&st->hdots))) return fail(rc);
  // partial sums: the dots' fixed grid, one per block of the fused apply,
  // or two per workgroup of the smoothing sweep with the cast back
  const size_t npart = std::max<size_t>({(size_t)kMaxDots * kDotBlocks, (size_t)apply_blocks(pr->p, pr->ncell),
                                          2 * (size_t)smooth_blocks(pr->p, pr->ncell)});
  {
    // one block for the whole workspace
    const bool f32 = o->precond_precision == DG_FP32 && o->precond != DG_PRECOND_NONE;
    const size_t vec = DevBuf::round(n * sizeof(double));
    const size_t total = (st->flex ? 5 : 4) * vec + DevBuf::round(npart * sizeof(double)) +
                         DevBuf::round(kMaxDots * sizeof(double)) + DevBuf::round(8 * sizeof(double)) +
                         (f32 ? 2 * DevBuf::round(n * sizeof(float)) : 0);
    if ((rc = st->wb.reserve(total))) return fail(rc);
  }
  if ((rc = st->wb.get(&st->r, n)) || (rc = st->wb.get(&st->p, n)) || (rc = st->wb.get(&st->q, n)) ||
      (rc = st->wb.get(&st->z, n)) || (rc = st->wb.get(&st->part, npart)) ||
      (rc = st->wb.get(&st->dout, kMaxDots)) || (rc = st->wb.get(&st->dsc, 8)))
    return fail(rc);
  if (st->flex && (rc = st->wb.get(&st->rold, n))) return fail(rc);
  if (o->precond_precision == DG_FP32 && o->precond != DG_PRECOND_NONE) {
    if ((rc = st->wb.get(&st->r32, n)) || (rc = st->wb.get(&st->z32, n))) return fail(rc);
  }
  void *dummy;
  if (o->precond == DG_PRECOND_MG && (rc = alloc_tmp(pr, o->precond_precision, 0, &dummy))) return fail(rc);
  if ((rc = inner_count_begin(pr, o, st->s))) return fail(rc);
  st->counting = o->inner_stats != 0;
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
    // device scalars cleared (breakdown flag), z = M(r), rho = (r, z) into
    // the device scalar of iteration 0, p = z
    e = hipMemsetAsync(st->dsc, 0, 8 * sizeof(double), st->s);
    if (e != hipSuccess) return fail(hip_fail(e, "hipMemsetAsync"));
    // rr of the initial residual: the FP32 scaling of the first iteration
    e = hipMemcpyAsync(st->dsc + 6, st->dout, sizeof(double), hipMemcpyDeviceToDevice, st->s);
    if (e != hipSuccess) return fail(hip_fail(e, "hipMemcpyAsync"));
    DotSet ds;
    ds.m = 1;
    ds.a[0] = st->r;
    ds.b[0] = st->z;
    if ((rc = precond_apply(pr, o, st->r, st->z, st->rnorm, st->r32, st->z32, st->s)) ||
        (rc = dots(ds, n, st->part, st->dsc + 4, st->s)))
      return fail(rc);
    e = hipMemcpyAsync(st->p, st->z, n * sizeof(double), hipMemcpyDeviceToDevice, st->s);
    if (e != hipSuccess) return fail(hip_fail(e, "hipMemcpyAsync"));
  }
  *out = st;
  return DG_OK;
}


// One step of every active state: the pending decision (waiting for that
// state's residual norm only), then the next iteration is enqueued.
int batch_step(dg_solve_state **sts, int n) {
  int rc;
  std::vector<int> act;
  for (int i = 0; i < n; ++i)
    if (!sts[i]->done) act.push_back(i);
  for (int i : act) {
    dg_solve_state *st = sts[i];
    if (st->pending >= 0 && (rc = check_iter(st))) return rc;
    if (!st->done && (rc = enqueue_iter(st))) return rc;
  }
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
  if (prob && prob->basis == DG_BASIS_GLL) {
    // the basis changes use scratch owned by the problem, which the
    // concurrent streams of several solves would share
    set_error("dg_solve_start: the Gauss-Lobatto basis is not supported by the serving entry points");
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
