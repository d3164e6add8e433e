"""Benchmark of the DG hot path on one MI355X.

A step is one pass of the whole hot path over the workload: one FP64
flexible-CG solve to a relative residual of 1e-8, preconditioned by one
FP32 hybrid-multigrid V-cycle per iteration (block-Jacobi smoother with
inner PCG at eps = 1e-2, Q1 coarse space with a vertex-grid coarse
cycle), i.e. operator applies, fused smoother sweeps, transfers, coarse
cycle and outer vector work.  The convection workload (w4) takes
FGMRES(30), inner GMRES(8) with the Thomas preconditioner and the P0
coarse space.

value  = DG operator-apply throughput (GDOF/s) of the FP64 applies that
         run inside the timed solves, each timed by the start and end
         events that its dispatch records (dg_solve_result.t_apply /
         n_apply).
ms_per_step = mean wall time of one solve (time-to-solve, mixed).
Also reported: FP64-preconditioned time-to-solve, FP32 apply throughput,
smoother and V-cycle timings, the roofline of the apply kernel, and the
CPU oracle (explicitly assembled BSR matrix, scipy matvec) on a bounded
sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload w2]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DG apply GDOF/s + time-to-solve @1e-8 rel residual, FP64 vs mixed; p99 latency"
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3  # published MI355X FP32 vector peak (packed FMA)
APPLY_SOURCES = ["paper_1805_11930_amd/csrc/apply.hip", "paper_1805_11930_amd/csrc/line_ops.h"]
COUNTERS = os.path.join(ROOT, "profiles", "apply_fp64_poisson32_p4_counters.md")


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def apply_source_hash() -> str:
    h = hashlib.sha256()
    for p in APPLY_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def bytes_per_dof(p: int, elem: int) -> float:
    """Algorithmic HBM bytes per DOF of one apply: read u, write v, and the
    per-cell diagonal K (3 values, stored in FP64)."""
    n3 = (p + 1) ** 3
    return 2 * elem + 24.0 / n3


def make_workload(name: str):
    from paper_1805_11930_amd import inputs

    return {"w1": inputs.w1, "w2": inputs.w2, "w3": inputs.w3, "w4": inputs.w4}[name]()


def cpu_baseline(w, seconds: float = 12.0) -> dict:
    """Oracle apply (explicit BSR matrix, scipy matvec) on a bounded sample
    of the workload: the same p, coefficients and boundary types on an
    8x8x8-cell sub-box."""
    import numpy as np

    from oracle import dg

    sub = (8, 8, 8)
    nc = 512
    K = w.K if np.ndim(w.K) == 0 else np.asarray(w.K)[:nc]
    lengths = tuple(L * s / N for L, s, N in zip(w.lengths, sub, w.cells))
    pr = dg.Problem(cells=sub, lengths=lengths, p=w.p, bc=w.bc, sigma=w.sigma, K=K, c=w.c, b0=w.b0, B=w.B)
    t0 = time.perf_counter()
    A = dg.assemble(pr)
    t_asm = time.perf_counter() - t0
    u = np.random.default_rng(1).normal(size=pr.ndof)
    v = A @ u
    reps = 0
    t0 = time.perf_counter()
    while True:
        v = A @ u
        reps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return {
        "value": pr.ndof * reps / el / 1e9,
        "unit": "GDOF/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"apply v=Au with the oracle's assembled BSR matrix (scipy matvec, single thread), "
                  f"p={w.p}, 8x8x8 cells = {pr.ndof} DOF, {reps} applies in {el:.1f} s "
                  f"(assembly {t_asm:.1f} s not timed)",
    }


def serving_leg(n_requests: int) -> dict:
    """Serving mix W5: closed-loop FP64 throughput sets the arrival rate
    (0.7 x solves/s); the same Poisson arrival trace (seed 55) is then
    served with the FP64 and with the mixed-precision preconditioner."""
    from paper_1805_11930_amd import DG_FP32, DG_FP64, DG_KRYLOV_FCG, DG_PRECOND_MG, inputs, solve_opts
    from paper_1805_11930_amd.serve import SolveServer, make_requests

    mix = inputs.w5_requests(n_requests)

    def opts(prec):
        return solve_opts(krylov=DG_KRYLOV_FCG, precond=DG_PRECOND_MG, precond_precision=prec, rtol=1e-8, maxit=500)

    closed = SolveServer(opts(DG_FP64)).run(make_requests(mix, None))
    rate = 0.7 * closed["solves_per_s"]
    log(f"[bench] serving closed-loop FP64: {closed['solves_per_s']:.1f} solves/s -> arrival rate {rate:.1f}/s")
    out = {"requests": n_requests, "arrival_rate_per_s": round(rate, 2),
           "closed_loop_fp64_solves_per_s": round(closed["solves_per_s"], 2)}
    for name, prec in (("fp64", DG_FP64), ("mixed", DG_FP32)):
        st = SolveServer(opts(prec)).run(make_requests(mix, rate))
        log(f"[bench] serving {name}: p50 {st['p50_latency_s'] * 1e3:.1f} ms, p99 {st['p99_latency_s'] * 1e3:.1f} ms, "
            f"{st['solves_per_s']:.1f} solves/s, converged {st['converged']}/{st['requests']}")
        out[name] = {k: (round(v, 5) if isinstance(v, float) else v) for k, v in st.items()}
    return out


def pe2000_leg(p: int = 3) -> dict:
    """Convection-dominated problem of Sec. 4.3 on the paper's isotropic grid
    for degree p: FGMRES(30) to 1e-8 preconditioned by two block-SSOR
    steps in the 12-colour diagonal cell order (ix + iy + iz mod 12), whose
    block solves are GMRES to eps = 1e-2 with the
    tridiagonal (Thomas) preconditioner, FP32 and FP64 preconditioner.
    Reported as time per unknown, the paper's unit for this test."""
    import torch

    from paper_1805_11930_amd import (DG_FP32, DG_FP64, DG_INNER_GMRES, DG_IPREC_TRIDIAG, DG_KRYLOV_FGMRES,
                                      DG_PRECOND_BLOCK, DG_SWEEP_SSOR, Problem, ProblemSpec, inputs, solve_opts)

    out = {"preconditioner": "2 x block-SSOR in the 12-colour diagonal order, inner GMRES(8) eps=1e-2 with the "
                             "Thomas preconditioner",
           "krylov": "FGMRES(30), rtol 1e-8"}
    for tag, b in (("b100", (1.0, 0.0, 0.0)), ("b1_05_03", (1.0, 0.5, 0.3))):
        w = inputs.pe2000(b=b, p=p)
        P = Problem(ProblemSpec(cells=w.cells, lengths=w.lengths, p=w.p, bc=w.bc, sigma=w.sigma, K=w.K, c=w.c,
                                b0=w.b0, B=w.B))
        f = P.rhs_from_functions(f=w.f)
        u = torch.zeros_like(f)
        row = {"workload": w.name, "ndof": P.ndof}
        for name, prec in (("mixed", DG_FP32), ("fp64", DG_FP64)):
            o = solve_opts(krylov=DG_KRYLOV_FGMRES, restart=30, precond=DG_PRECOND_BLOCK, precond_precision=prec,
                           rtol=1e-8, maxit=300,
                           smooth=dict(n_sweeps=2, sweep=DG_SWEEP_SSOR, omega=1.0, eps=1e-2, inner=DG_INNER_GMRES,
                                       restart=8, inner_precond=DG_IPREC_TRIDIAG, colours=12))
            best = None
            for _ in range(3):
                u.zero_()
                _, r = P.solve(f, u, o)
                best = r if best is None or r.t_solve < best.t_solve else best
            row[name] = {"time_to_solve_s": round(best.t_solve, 4), "iterations": best.iters,
                         "rel_residual": best.rel_residual,
                         "us_per_dof": round(best.t_solve / P.ndof * 1e6, 5)}
            if name == "mixed":
                # the FP64 applies inside the solve (dispatch-recorded events)
                row["apply_fp64_gdofs"] = round(P.ndof * best.n_apply / max(best.t_apply, 1e-30) / 1e9, 2)
            log(f"[bench] Pe=2000 {tag} {name}: {best.t_solve * 1e3:.1f} ms, {best.iters} it, "
                f"rel_res {best.rel_residual:.2e}")
        out[tag] = row
        P.close()
    return out


def diffusion_leg(p: int = 3) -> dict:
    """The two diffusion tests of Sec. 4.2 on the paper's isotropic grid for
    degree p ([0,1]^2 x [0,2]): Poisson and the inhomogeneous problem with
    K(x), c(x) at the quadrature points of the outer operator (axis-aligned
    directions n_m = e_m, and a rotated basis: a full tensor) and their
    cell-centre values in the FP32 / FP64 V-cycle; FCG to 1e-8, inner PCG
    eps = 1e-2.  Time per unknown, the paper's unit for these tests."""
    import torch

    from paper_1805_11930_amd import (DG_FP32, DG_FP64, DG_KRYLOV_FCG, DG_PRECOND_MG, Problem, ProblemSpec, inputs,
                                      solve_opts)

    out = {"krylov": "flexible CG, rtol 1e-8", "preconditioner": "V-cycle, block-Jacobi, inner PCG eps=1e-2, Q1"}
    cases = (("poisson", inputs.poisson_gauss(p)), ("inhomogeneous", inputs.inhomogeneous(p)),
             ("inhomogeneous_rotated", inputs.inhomogeneous(p, nrot=inputs.rotation(0.4, -0.7, 1.1))))
    for tag, w in cases:
        P = Problem(ProblemSpec(cells=w.cells, lengths=w.lengths, p=w.p, bc=w.bc, sigma=w.sigma, K=w.K, c=w.c,
                                b0=w.b0, B=w.B, kfield=w.kfield, cfield=w.cfield, nrot=w.nrot))
        f = P.rhs_from_functions(f=w.f, g=w.g, j=w.j)
        u = torch.zeros_like(f)
        row = {"workload": w.name, "ndof": P.ndof}
        for name, prec in (("mixed", DG_FP32), ("fp64", DG_FP64)):
            o = solve_opts(krylov=DG_KRYLOV_FCG, precond=DG_PRECOND_MG, precond_precision=prec, rtol=1e-8,
                           maxit=500)
            best = None
            for _ in range(3):
                u.zero_()
                _, r = P.solve(f, u, o)
                best = r if best is None or r.t_solve < best.t_solve else best
            row[name] = {"time_to_solve_s": round(best.t_solve, 4), "iterations": best.iters,
                         "rel_residual": best.rel_residual,
                         "us_per_dof": round(best.t_solve / P.ndof * 1e6, 5)}
            if name == "mixed":
                # the FP64 applies inside the solve (dispatch-recorded events)
                row["apply_fp64_gdofs"] = round(P.ndof * best.n_apply / max(best.t_apply, 1e-30) / 1e9, 2)
            log(f"[bench] {tag} p={p} {name}: {best.t_solve * 1e3:.1f} ms, {best.iters} it, "
                f"rel_res {best.rel_residual:.2e}")
        out[tag] = row
        P.close()
    return out


def event_time(fn, reps: int) -> float:
    """Mean seconds per call of fn() on torch's current stream (HIP events)."""
    import torch

    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    e.synchronize()
    return s.elapsed_time(e) * 1e-3 / reps


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="w2", choices=["w1", "w2", "w3", "w4"])
    ap.add_argument("--coarse", default="auto", choices=["auto", "p0", "q1"],
                    help="coarse space of the V-cycle (auto: the workload's own; Q1 for the diffusion boxes, P0 "
                         "for the convection box and the layered SPE10-like field)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=256, help="serving leg size (0 = skip)")
    ap.add_argument("--pe2000", type=int, default=1, help="run the Pe=2000 convection leg (0 = skip)")
    ap.add_argument("--diffusion", type=int, default=1,
                    help="run the Poisson / inhomogeneous diffusion leg on the paper's p=3 grid (0 = skip)")
    ap.add_argument("--apply-only", type=int, default=0,
                    help="profiling aid: run this many FP64 applies and exit")
    ap.add_argument("--smooth-only", type=int, default=0,
                    help="profiling aid: run this many FP32 block-Jacobi sweeps (the workload's block "
                         "solver: inner PCG, or inner GMRES with the Thomas preconditioner when b != 0) and exit")
    ap.add_argument("--copy-only", type=int, default=0,
                    help="counter calibration: run this many 256 MiB device-to-device copies and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(the hot path runs on one MI355X, see the sharding notes).", file=sys.stderr)
        return 2
    import numpy as np
    import torch

    from paper_1805_11930_amd import (DG_COARSE_P0, DG_COARSE_Q1, DG_FP32, DG_FP64, DG_INNER_CG, DG_INNER_FDM,
                                      DG_INNER_GMRES, DG_IPREC_DIAG, DG_IPREC_TRIDIAG, DG_KRYLOV_FCG,
                                      DG_KRYLOV_FGMRES, DG_PRECOND_MG, Problem, ProblemSpec, mg_opts, smooth_opts,
                                      solve_opts)

    torch.cuda.set_device(0)
    if args.copy_only:
        src = torch.ones(64 * 2**20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(args.copy_only):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] ran {args.copy_only} copies of {src.numel() * 4} bytes")
        return 0
    w = make_workload(args.workload)
    log(f"[bench] workload {w.name}: cells={w.cells} p={w.p} ndof={w.ndof}")
    P = Problem(ProblemSpec(cells=w.cells, lengths=w.lengths, p=w.p, bc=w.bc, sigma=w.sigma, K=w.K, c=w.c,
                            b0=w.b0, B=w.B))
    u_rand = torch.from_numpy(np.random.default_rng(3).normal(size=P.ndof)).cuda()
    if args.apply_only:
        v = torch.empty_like(u_rand)
        for _ in range(args.apply_only):
            P.apply(u_rand, v)
        torch.cuda.synchronize()
        log(f"[bench] ran {args.apply_only} FP64 applies")
        return 0
    conv = bool(w.b0 != (0.0, 0.0, 0.0) or np.any(np.asarray(w.B) != 0))
    if args.smooth_only:
        f32 = (u_rand / u_rand.norm()).float()
        u32 = torch.zeros_like(f32)
        o32 = torch.empty_like(f32)
        # the workload's own block solver (as in its V-cycle)
        sm = (smooth_opts(eps=1e-2, inner=DG_INNER_GMRES, restart=8, inner_precond=DG_IPREC_TRIDIAG) if conv
              else smooth_opts(eps=1e-2, inner=DG_INNER_CG))
        for _ in range(args.smooth_only):
            P.block_smooth(f32, u32, sm, out=o32)
        torch.cuda.synchronize()
        log(f"[bench] ran {args.smooth_only} FP32 smoother sweeps")
        return 0
    f = P.rhs_from_functions(f=w.f, g=w.g, j=w.j)
    inner = DG_INNER_GMRES if conv else DG_INNER_CG
    krylov = DG_KRYLOV_FGMRES if conv else DG_KRYLOV_FCG
    # convection-dominated blocks: the tridiagonal (Thomas) inner preconditioner (Sec. 3.2)
    iprec = DG_IPREC_TRIDIAG if conv else DG_IPREC_DIAG

    coarse_name = w.coarse if args.coarse == "auto" else args.coarse
    if coarse_name == "auto":
        coarse_name = "p0" if conv else "q1"
    coarse = DG_COARSE_Q1 if coarse_name == "q1" else DG_COARSE_P0

    def opts(prec):
        return solve_opts(krylov=krylov, restart=30, precond=DG_PRECOND_MG, precond_precision=prec, rtol=1e-8,
                          maxit=1000, smooth=dict(eps=1e-2, inner=inner, restart=8 if conv else 12, inner_precond=iprec),
                          mg=dict(coarse_space=coarse))

    o_mixed, o_fp64 = opts(DG_FP32), opts(DG_FP64)
    u = torch.zeros_like(f)

    def step(o):
        u.zero_()
        _, res = P.solve(f, u, o)
        return res

    for i in range(args.warmup):
        res = step(o_mixed)
        log(f"[bench] warmup {i}: iters={res.iters} rel_res={res.rel_residual:.2e} t={res.t_solve:.3f}s")
    torch.cuda.synchronize()
    t_apply = 0.0
    n_apply = 0
    iters = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        res = step(o_mixed)
        t_apply += res.t_apply
        n_apply += res.n_apply
        iters.append(res.iters)
        if res.status != 0:
            log(f"[bench] step {i} did not converge: status={res.status} rel_res={res.rel_residual:.2e}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    log(f"[bench] timed {args.steps} mixed solves: {ms_per_step:.1f} ms/step, iters={iters}")
    apply_s = t_apply / max(n_apply, 1)
    gdofs = P.ndof / apply_s / 1e9
    bpd = bytes_per_dof(w.p, 8)
    achieved = bpd * P.ndof / apply_s / 1e9
    # ---- other rows of the hot path (outside the timed region) ----------
    res64 = step(o_fp64)
    log(f"[bench] FP64-preconditioned solve: iters={res64.iters} t={res64.t_solve:.3f}s")
    res_m = step(o_mixed)
    u32 = u_rand.float()
    v32 = torch.empty_like(u32)
    v64 = torch.empty_like(u_rand)
    t_a64 = event_time(lambda: P.apply(u_rand, v64), 20)
    t_a32 = event_time(lambda: P.apply(u32, v32), 20)
    # the same FP64 apply cycling through 8 input/output pairs (16 vectors,
    # more than the 256 MB MALL holds at this size): every pass reads u from
    # HBM instead of the MALL
    pairs = [(u_rand * (1.0 + 0.01 * k), torch.empty_like(u_rand)) for k in range(8)]
    cyc = [0]

    def apply_cycled():
        uu, vv = pairs[cyc[0] % len(pairs)]
        cyc[0] += 1
        P.apply(uu, vv)

    for _ in range(8):
        apply_cycled()
    t_cold = event_time(apply_cycled, 24)
    del pairs
    f32 = f.float() / f.norm()
    sm = smooth_opts(eps=1e-2, inner=inner, restart=12)
    out32 = torch.empty_like(f32)
    t_sm = event_time(lambda: P.block_smooth(f32, u32, sm, out=out32), 5)
    _, st = P.block_smooth(f32, u32, sm, out=out32, stats=True)
    # algorithmic flops of the sweep: per cell the defect (three line
    # operators of N^2 lines with N x N contractions and the face terms:
    # 6 N^4 + 20 N^3) and per inner PCG iteration one D_T product (6 N^4)
    # plus the dot products and updates (13 N^3)
    nn = w.p + 1
    sm_flops = P.ncell * (6 * nn**4 + 20 * nn**3) + st.inner_total * (6 * nn**4 + 13 * nn**3)
    sm_tflops = sm_flops / t_sm / 1e12
    mo = mg_opts(smooth=dict(eps=1e-2, inner=inner, restart=12), coarse_space=coarse)
    t_vc = event_time(lambda: P.mg_vcycle(f32, mo, out=out32), 5)
    # stored-factor exact block solve (b = 0 only): same V-cycle and solves
    fdm = None
    if not conv:
        def opts_fdm(prec):
            return solve_opts(krylov=krylov, restart=30, precond=DG_PRECOND_MG, precond_precision=prec, rtol=1e-8,
                              maxit=1000, smooth=dict(inner=DG_INNER_FDM), mg=dict(coarse_space=coarse))
        smf = smooth_opts(inner=DG_INNER_FDM)
        P.block_smooth(f32, u32, smf, out=out32)
        t_smf = event_time(lambda: P.block_smooth(f32, u32, smf, out=out32), 5)
        fdm_res = {}
        for name, prec in (("mixed", DG_FP32), ("fp64", DG_FP64)):
            step(opts_fdm(prec))
            best = None
            for _ in range(3):
                r_ = step(opts_fdm(prec))
                best = r_ if best is None or r_.t_solve < best.t_solve else best
            fdm_res[name] = best
        fdm = {
            "inner": "exact block solve by fast diagonalisation (stored per-cell factors)",
            "smoother_sweep_fp32_ms": round(t_smf * 1e3, 3),
            "time_to_solve_s": {k: round(v.t_solve, 4) for k, v in fdm_res.items()},
            "iterations": {k: v.iters for k, v in fdm_res.items()},
            "rel_residual": {k: v.rel_residual for k, v in fdm_res.items()},
        }
        log(f"[bench] FDM smoother: sweep {t_smf * 1e3:.3f} ms, mixed solve {fdm_res['mixed'].t_solve * 1e3:.1f} ms "
            f"({fdm_res['mixed'].iters} it), FP64 {fdm_res['fp64'].t_solve * 1e3:.1f} ms")
    traffic = None
    if os.path.exists(COUNTERS):
        with open(COUNTERS) as fh:
            cnt = {}
            for ln in fh:
                if ln.startswith("counters-json:"):
                    cnt = json.loads(ln.split(":", 1)[1])
        if cnt.get("source_hash") == apply_source_hash() and cnt.get("workload") == w.name:
            traffic = cnt.get("hbm_bytes_per_launch")
    line = {
        "metric": METRIC,
        "value": round(gdofs, 3),
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": w.name,
            "cells": list(w.cells),
            "p": w.p,
            "ndof": P.ndof,
            "step": "one FP64 flexible Krylov solve to 1e-8 preconditioned by an FP32 hybrid-multigrid V-cycle",
            "coarse_space": coarse_name,
            "block_solver": ("inner GMRES(8), Thomas-preconditioned" if conv else "inner PCG, diagonal") + ", eps 1e-2",
            "value_from": "mean duration of the FP64 operator-apply kernel inside the timed solves (HIP events)",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": "k_apply<P=4,double>",
            "bytes_per_dof": round(bpd, 3),
        },
        "time_to_solve_s": {"mixed": round(ms_per_step / 1e3, 4), "fp64": round(res64.t_solve, 4)},
        "iterations": {"mixed": iters, "fp64": res64.iters},
        "rel_residual": {"mixed": res_m.rel_residual, "fp64": res64.rel_residual},
        "rows": {
            "apply_fp64_gdofs": round(P.ndof / t_a64 / 1e9, 2),
            "apply_fp32_gdofs": round(P.ndof / t_a32 / 1e9, 2),
            "apply_fp64_mall_cold": {"pairs": 8, "gdofs": round(P.ndof / t_cold / 1e9, 2),
                                     "algorithmic_gbs": round(bpd * P.ndof / t_cold / 1e9, 1)},
            "smoother_sweep_fp32_ms": round(t_sm * 1e3, 3),
            "smoother_roofline": {"bound": "alu", "kernel": f"k_smooth<P={w.p},PCG,float>",
                                  "achieved": round(sm_tflops, 2), "peak": FP32_VECTOR_PEAK_TFLOPS,
                                  "unit": "TFLOP/s", "frac": round(sm_tflops / FP32_VECTOR_PEAK_TFLOPS, 4),
                                  "flops_per_launch": int(sm_flops)},
            "smoother_inner_avg": round(st.inner_avg, 3),
            "smoother_inner_max": st.inner_max,
            "vcycle_fp32_ms": round(t_vc * 1e3, 3),
            "precond_ms_per_iter_mixed": round(res_m.t_precond * 1e3 / max(res_m.n_precond, 1), 3),
            "apply_launches_timed": n_apply,
        },
        "fdm_smoother": fdm,
    }
    if args.diffusion:
        line["diffusion_sec42"] = diffusion_leg()
    if args.pe2000:
        line["convection_pe2000"] = pe2000_leg()
    if args.serve_requests > 0:
        line["serving"] = serving_leg(args.serve_requests)
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline ...")
        line["cpu_baseline"] = cpu_baseline(w)
    P.close()
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
