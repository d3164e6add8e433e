"""Continuous-batching solve server over the libdgmg resident-solve calls.

Requests (a problem description and a right-hand side) arrive over time.
The loop admits waiting requests, first come first served, as long as the
device bytes they need (dg_footprint plus their f and u vectors) fit in
the HBM budget and a slot is free; it then advances every active solve by
one dg_batch_step call (the decision of its iteration in flight, then the
next iteration enqueued; the kernels of all solves overlap on the device,
each on its own stream), retires finished solves (freeing their memory)
and admits again.  A request whose footprint exceeds the
whole budget is rejected (DG_ENOMEM).  All numerical work runs in the HIP
library; this module only schedules.

Admission (problem creation, the upload of f, dg_solve_start with its
coarse-space set-up and first preconditioner application) costs the host
a few milliseconds per request, longer than a batch step, so it runs on a
worker thread (the library calls release the interpreter lock) while the
loop keeps stepping the active solves; an admitted request joins the
batch at the next step after its preparation finished.

Freeing device memory (hipFree) waits for the whole device, so a retired
request keeps its memory until the loop is idle (no active solve) or until
an admission needs the bytes; only then are the retired states and
problems destroyed, together.
"""
from __future__ import annotations

import concurrent.futures as cf
import ctypes
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as L
from .problem import Problem


@dataclass
class Request:
    rid: int
    arrival: float            # seconds after the start of the run
    spec: L.ProblemSpec
    rhs: np.ndarray           # DG load vector (FP64)
    # filled by the server
    admitted: float = float("nan")
    finished: float = float("nan")
    status: int = L.DG_EAGAIN
    iters: int = 0
    rel_residual: float = float("nan")
    solution: np.ndarray | None = field(default=None, repr=False)

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class _Active:
    def __init__(self, req: Request, prob: Problem, f: torch.Tensor, u: torch.Tensor, state: ctypes.c_void_p,
                 nbytes: int):
        self.req, self.prob, self.f, self.u, self.state, self.nbytes = req, prob, f, u, state, nbytes


class SolveServer:
    def __init__(self, opts: L.SolveOpts, hbm_budget: int | None = None, max_active: int = 32,
                 keep_solutions: bool = False, prepare_ahead: int = 2):
        self.lib = L.load()
        self.opts = opts
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info()
            hbm_budget = int(0.8 * free)
        self.budget = int(hbm_budget)
        self.max_active = max_active
        self.keep = keep_solutions
        # admissions in preparation on the worker thread at a time; 0: admit
        # on the loop's own thread (every request that fits joins the next
        # step together, as for a fixed batch)
        self.prepare_ahead = max(0, int(prepare_ahead))

    def footprint(self, req: Request) -> int:
        ndof = int(np.prod(req.spec.cells)) * (req.spec.p + 1) ** 3
        return L.footprint(req.spec, self.opts) + 2 * 8 * ndof

    def _admit(self, req: Request, t0: float, need: int) -> _Active:
        """Runs on the admission thread."""
        prob = Problem(req.spec)
        f = torch.from_numpy(np.ascontiguousarray(req.rhs, dtype=np.float64)).cuda()
        u = torch.zeros_like(f)
        # f and u are ready once this thread's torch stream has run; the
        # solve runs on its own stream, so only that stream is waited for
        torch.cuda.current_stream().synchronize()
        st = ctypes.c_void_p()
        L._check(self.lib.dg_solve_start(prob.h, f.data_ptr(), u.data_ptr(), ctypes.byref(self.opts), ctypes.byref(st)))
        req.admitted = time.perf_counter() - t0
        return _Active(req, prob, f, u, st, need)

    def _retire(self, a: _Active, now: float):
        res = L.SolveResult()
        L._check(self.lib.dg_solve_poll(a.state, ctypes.byref(res)))
        a.req.finished = now
        a.req.status = res.status
        a.req.iters = res.iters
        a.req.rel_residual = res.rel_residual
        if self.keep:
            a.req.solution = a.u.cpu().numpy()
        self._dead.append(a)

    def _flush(self) -> int:
        """Destroys the retired states and problems; returns their bytes."""
        freed = 0
        for a in self._dead:
            self.lib.dg_solve_state_destroy(a.state)
            a.prob.close()
            freed += a.nbytes
        self._dead = []
        return freed

    def run(self, requests: list[Request], log=None) -> dict:
        pending = sorted(requests, key=lambda r: r.arrival)
        queue: list[Request] = []
        active: list[_Active] = []
        preparing: list[cf.Future] = []
        self._dead = []
        used = 0  # bytes of the active, preparing and retired-but-not-freed requests
        steps = 0
        peak_active = 0
        t0 = time.perf_counter()
        with cf.ThreadPoolExecutor(max_workers=1, thread_name_prefix="dg-admit") as pool:
            while pending or queue or active or preparing:
                now = time.perf_counter() - t0
                while pending and pending[0].arrival <= now:
                    queue.append(pending.pop(0))
                # admission by HBM footprint, first come first served
                depth = self.prepare_ahead if self.prepare_ahead > 0 else self.max_active
                while queue and len(active) + len(preparing) < self.max_active and len(preparing) < depth:
                    req = queue[0]
                    need = self.footprint(req)
                    if need > self.budget:
                        queue.pop(0)
                        req.status = L.DG_ENOMEM
                        req.finished = now
                        continue
                    if used + need > self.budget and self._dead:
                        used -= self._flush()
                    if used + need > self.budget:
                        break
                    queue.pop(0)
                    if self.prepare_ahead > 0:
                        preparing.append(pool.submit(self._admit, req, t0, need))
                    else:
                        active.append(self._admit(req, t0, need))
                    used += need
                # prepared requests join the batch
                if not active and preparing:
                    cf.wait(preparing, return_when=cf.FIRST_COMPLETED)
                still = []
                for fut in preparing:
                    if fut.done():
                        active.append(fut.result())
                    else:
                        still.append(fut)
                preparing = still
                if not active:
                    used -= self._flush()  # idle: nothing waits on the frees
                    if pending and not queue:
                        time.sleep(max(0.0, pending[0].arrival - (time.perf_counter() - t0)))
                    continue
                peak_active = max(peak_active, len(active))
                arr = (ctypes.c_void_p * len(active))(*[a.state.value for a in active])
                L._check(self.lib.dg_batch_step(arr, len(active), None))
                steps += 1
                now = time.perf_counter() - t0
                still = []
                for a in active:
                    if self.lib.dg_solve_poll(a.state, None) == L.DG_EAGAIN:
                        still.append(a)
                    else:
                        self._retire(a, now)
                active = still
        makespan = time.perf_counter() - t0
        used -= self._flush()
        done = [r for r in requests if r.status in (L.DG_OK, L.DG_ENOCONV)]
        lat = np.array([r.latency for r in done])
        return {
            "requests": len(requests),
            "completed": len(done),
            "converged": sum(r.status == L.DG_OK for r in requests),
            "rejected": sum(r.status == L.DG_ENOMEM for r in requests),
            "makespan_s": makespan,
            "solves_per_s": len(done) / makespan if makespan > 0 else 0.0,
            "p50_latency_s": float(np.percentile(lat, 50)) if len(lat) else None,
            "p99_latency_s": float(np.percentile(lat, 99)) if len(lat) else None,
            "batch_steps": steps,
            "peak_active": peak_active,
        }


def make_requests(mix, rate: float | None, seed: int = 55) -> list[Request]:
    """Requests for a list of (N, p, seed) from inputs.w5_requests; arrivals
    form a Poisson process of the given rate (None: all at time 0)."""
    from . import inputs

    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i, (N, p, s) in enumerate(mix):
        if rate:
            t += rng.exponential(1.0 / rate)
        w, rhs = inputs.w5_problem(N, p, s)
        spec = L.ProblemSpec(cells=w.cells, lengths=w.lengths, p=w.p, bc=w.bc, sigma=w.sigma, K=w.K, c=w.c)
        out.append(Request(i, t if rate else 0.0, spec, rhs))
    return out
