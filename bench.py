"""Benchmark of the DG hot path on one MI355X.

A step is one pass of the whole hot path over the main workload (default:
Poisson, 32^3 cells, p = 4): one FP64 flexible-CG solve to a relative
residual of 1e-8, preconditioned by one FP32 hybrid-multigrid V-cycle per
iteration (block-Jacobi smoother with inner PCG at eps = 1e-2, Q1 coarse
space with a vertex-grid coarse cycle), i.e. operator applies, fused
smoother sweeps, transfers, coarse cycle and outer vector work.

value  = DG operator-apply throughput (GDOF/s) of the FP64 applies that
         run inside the timed solves, each timed by the start and end
         events that its dispatch records (dg_solve_result.t_apply /
         n_apply).
ms_per_step = mean wall time of one mixed-precision solve (setup included).

Every other single-GPU configuration runs as its own leg with the same
report (`workloads`): the 8^3 p = 2 Poisson problem (CG + one block-Jacobi
sweep to 1e-10), the SPE10-like 60x220x85 p = 2 box and the 48^3 p = 3
convection box (FGMRES(30), inner GMRES(8) with the Thomas preconditioner,
P0 coarse space).  Per leg: FP64-preconditioned and mixed time-to-solve
(both from dg_solve_result.t_solve, setup reported separately),
iterations, true FP64 residuals, FP64 errors (against the exact solution
where it is known, and mixed against the FP64-preconditioned answer), the
inner iterations counted inside the solve, the in-solve FP64 apply rate
with its HBM roofline, FP32 apply, smoother sweep and V-cycle times.
Then the Sec. 4.2 diffusion tests, the Sec. 4.3 Pe = 2000 problem, the
serving mix, and the CPU oracle (explicitly assembled BSR matrix, scipy
matvec on 1 and on all host threads; its CG solve of the 8^3 problem).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload w2] [--legs w1,w3,w4]
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


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _host_threads() -> int:
    """Threads the CPU baseline may use: the cores this process may run on,
    at most 16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(w, seconds: float = 4.0) -> dict:
    """The oracle on the host cores, on bounded samples of the workloads.

    Apply: the oracle's explicitly assembled BSR matrix (scipy matvec) of the
    workload's p, coefficients and boundary types on an 8x8x8-cell sub-box,
    on one thread and on all host threads (row blocks of the same matrix,
    one per thread; scipy releases the GIL in the matvec).  Solve: the
    oracle's flexible CG with one block-Jacobi sweep (inner PCG, eps = 1e-2)
    to 1e-10 on the 8^3, p = 2 Poisson problem, the same solve as the
    workload's first configuration."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    import scipy.sparse as sp

    from oracle import dg, solvers
    from paper_1805_11930_amd import inputs

    sub = (8, 8, 8)
    nc = 512
    K = w.K if np.ndim(w.K) == 0 else np.asarray(w.K)[:nc]
    lengths = tuple(L * s / N for L, s, N in zip(w.lengths, sub, w.cells))
    pr = dg.Problem(cells=sub, lengths=lengths, p=w.p, bc=w.bc, sigma=w.sigma, K=K, c=w.c, b0=w.b0, B=w.B)
    t0 = time.perf_counter()
    A = dg.assemble(pr)
    t_asm = time.perf_counter() - t0
    u = np.random.default_rng(1).normal(size=pr.ndof)

    def rate(fn):
        fn()
        reps = 0
        t0 = time.perf_counter()
        while True:
            fn()
            reps += 1
            el = time.perf_counter() - t0
            if el >= seconds:
                return pr.ndof * reps / el / 1e9, reps, el

    g1, reps1, el1 = rate(lambda: A @ u)
    nt = _host_threads()
    nb = pr.nloc
    Acsr = A.tocsr()
    parts = [sp.bsr_matrix(Acsr[r[0] * nb:(r[-1] + 1) * nb], blocksize=(nb, nb))
             for r in np.array_split(np.arange(pr.ncell), nt)]
    with ThreadPoolExecutor(nt) as ex:
        gN, repsN, elN = rate(lambda: np.concatenate(list(ex.map(lambda B: B @ u, parts))))
    # time-to-solve of the 8^3, p = 2 Poisson problem
    w1 = inputs.w1()
    p1 = dg.Problem(cells=w1.cells, lengths=w1.lengths, p=w1.p, bc=w1.bc, sigma=w1.sigma, K=w1.K, c=w1.c)
    A1 = dg.assemble(p1)
    D1 = dg.block_diagonal(A1, p1.ncell)
    f1 = dg.assemble_rhs(p1, f=w1.f)
    M = lambda r: solvers.block_jacobi(A1, D1, r, np.zeros_like(r), omega=1.0, nsweeps=1, inner="cg",  # noqa: E731
                                       eps=1e-2)
    t0 = time.perf_counter()
    _, it1, hist = solvers.cg(A1, f1, precond=M, rtol=1e-10, flexible=True)
    t_solve = time.perf_counter() - t0
    return {
        "value": round(gN, 6),
        "unit": "GDOF/s",
        "cores": nt,
        "kind": "oracle",
        "sample": f"apply v=Au with the oracle's assembled BSR matrix (scipy matvec, row blocks on {nt} threads), "
                  f"p={w.p}, 8x8x8 cells = {pr.ndof} DOF, {repsN} applies in {elN:.1f} s "
                  f"(assembly {t_asm:.1f} s not timed)",
        "one_core_gdofs": round(g1, 6),
        "one_core_sample": f"same matrix on 1 thread, {reps1} applies in {el1:.1f} s",
        "nproc": os.cpu_count(),
        "cpu_model": _cpu_model(),
        "solve_poisson_8cube_p2": {"time_to_solve_s": round(t_solve, 3), "iterations": it1,
                                   "rel_residual": hist[-1], "threads": 1,
                                   "method": "flexible CG, one block-Jacobi sweep (inner PCG eps 1e-2), rtol 1e-10"},
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

    from paper_1805_11930_amd import (DG_FP32, DG_FP64, DG_INNER_GMRES, DG_INNER_PMF, DG_IPREC_TRIDIAG,
                                      DG_KRYLOV_FGMRES, DG_PRECOND_BLOCK, DG_SWEEP_SSOR, Problem, ProblemSpec, inputs,
                                      solve_opts)

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
            # partially matrix-free: the same SSOR steps with exact block
            # solves by the stored inverses (the paper's PMF variant)
            op = solve_opts(krylov=DG_KRYLOV_FGMRES, restart=30, precond=DG_PRECOND_BLOCK, precond_precision=prec,
                            rtol=1e-8, maxit=300,
                            smooth=dict(n_sweeps=2, sweep=DG_SWEEP_SSOR, omega=1.0, inner=DG_INNER_PMF, colours=12))
            bp = None
            for _ in range(3):
                u.zero_()
                _, r = P.solve(f, u, op)
                bp = r if bp is None or r.t_solve < bp.t_solve else bp
            row[name + "_pmf"] = {"time_to_solve_s": round(bp.t_solve, 4), "iterations": bp.iters,
                                  "rel_residual": bp.rel_residual,
                                  "us_per_dof": round(bp.t_solve / P.ndof * 1e6, 5)}
            log(f"[bench] Pe=2000 {tag} {name} PMF: {bp.t_solve * 1e3:.1f} ms, {bp.iters} it")
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
        if tag != "inhomogeneous_rotated":
            out[tag + "_eps_sweep"] = eps_sweep(w)
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


def basis_leg(p: int = 3) -> dict:
    """Inner block-solver iterations in the two nodal bases (Sec. 2.1: the
    paper's Gauss-Lobatto basis; the library's default Gauss-Legendre
    basis).  The paper reports, at eps = 1e-2, fewer than four inner
    iterations on average and at most 15 (Poisson) / 25 (varying
    coefficients) in Sec. 4.2, and around four for b = (1, 0, 0) at
    Pe = 2000 with the Thomas preconditioner in Sec. 4.3.  Diffusion: FCG
    to 1e-8, V-cycle (block-Jacobi, inner PCG, P0 coarse space in both
    bases: the GLL basis has no Q1 transfer), FP64 preconditioner as in the
    paper's counts.  Convection: the pe2000 leg's FGMRES / block-SSOR
    setup."""
    import dataclasses

    import torch

    from paper_1805_11930_amd import (DG_COARSE_P0, DG_FP64, DG_INNER_GMRES, DG_IPREC_TRIDIAG, DG_KRYLOV_FCG,
                                      DG_KRYLOV_FGMRES, DG_PRECOND_BLOCK, DG_PRECOND_MG, DG_SWEEP_SSOR, Problem,
                                      ProblemSpec, inputs, solve_opts)

    diff = dict(krylov=DG_KRYLOV_FCG, precond=DG_PRECOND_MG, precond_precision=DG_FP64, rtol=1e-8, maxit=500,
                smooth=dict(eps=1e-2), coarse_space=DG_COARSE_P0)
    conv = dict(krylov=DG_KRYLOV_FGMRES, restart=30, precond=DG_PRECOND_BLOCK, precond_precision=DG_FP64, rtol=1e-8,
                maxit=300, smooth=dict(n_sweeps=2, sweep=DG_SWEEP_SSOR, omega=1.0, eps=1e-2, inner=DG_INNER_GMRES,
                                       restart=8, inner_precond=DG_IPREC_TRIDIAG, colours=12))
    cases = (("poisson", inputs.poisson_gauss(p), diff), ("inhomogeneous", inputs.inhomogeneous(p), diff),
             ("pe2000_b100", inputs.pe2000(b=(1.0, 0.0, 0.0), p=p), conv),
             ("pe2000_b1_05_03", inputs.pe2000(b=(1.0, 0.5, 0.3), p=p), conv))
    out = {"eps": 1e-2, "paper": "inner avg < 4, max 15 (Poisson) / 25 (varying coefficients); about 4 for "
                                 "b=(1,0,0) at Pe=2000 with the Thomas preconditioner"}
    for tag, w, kw in cases:
        row = {"workload": w.name}
        for bname in ("gl", "gll"):
            spec = ProblemSpec(cells=w.cells, lengths=w.lengths, p=w.p, bc=w.bc, sigma=w.sigma, K=w.K, c=w.c,
                               b0=w.b0, B=w.B, kfield=w.kfield, cfield=w.cfield, nrot=w.nrot)
            P = Problem(dataclasses.replace(spec, basis=bname))
            f = P.rhs_from_functions(f=w.f, g=w.g, j=w.j)
            u = torch.zeros_like(f)
            kwo = dict(kw)
            cs = kwo.pop("coarse_space", None)
            o = solve_opts(**kwo)
            if cs is not None:
                o.mg.coarse_space = cs
            P.solve(f, u, o)  # warm-up (builds the hierarchy)
            u.zero_()
            _, r = P.solve(f, u, o)
            o.inner_stats = 1
            u.zero_()
            _, rs = P.solve(f, u, o)
            row[bname] = {"iterations": r.iters, "time_to_solve_s": round(r.t_solve, 4),
                          "us_per_dof": round(r.t_solve / P.ndof * 1e6, 5), "inner_avg": round(rs.inner_avg, 3),
                          "inner_max": rs.inner_max, "rel_residual": r.rel_residual}
            log(f"[bench] basis {bname} {w.name}: {r.iters} it, {r.t_solve * 1e3:.1f} ms, inner avg "
                f"{rs.inner_avg:.2f} max {rs.inner_max}")
            P.close()
        out[tag] = row
    return out


def eps_sweep(w) -> dict:
    """Outer iterations and inner iterations against the inner tolerance eps
    of the block solves (Sec. 4.2, the MF(eps) variants), and the exact
    block solve by stored inverses (PMF), FP64 preconditioner as in the
    paper: flexible CG to 1e-8, V-cycle with the Q1 coarse space."""
    import torch

    from paper_1805_11930_amd import (DG_FP64, DG_INNER_PMF, DG_KRYLOV_FCG, DG_PRECOND_MG, Problem, ProblemSpec,
                                      solve_opts)

    P = Problem(ProblemSpec(cells=w.cells, lengths=w.lengths, p=w.p, bc=w.bc, sigma=w.sigma, K=w.K, c=w.c,
                            b0=w.b0, B=w.B, kfield=w.kfield, cfield=w.cfield, nrot=w.nrot))
    f = P.rhs_from_functions(f=w.f, g=w.g, j=w.j)
    u = torch.zeros_like(f)
    rows = {}
    for eps in (1e-12, 1e-8, 1e-4, 1e-2, "pmf"):
        sm = dict(inner=DG_INNER_PMF) if eps == "pmf" else dict(eps=eps)
        o = solve_opts(krylov=DG_KRYLOV_FCG, precond=DG_PRECOND_MG, precond_precision=DG_FP64, rtol=1e-8,
                       maxit=500, smooth=sm)
        u.zero_()
        P.solve(f, u, o)
        u.zero_()
        _, r = P.solve(f, u, o)
        o.inner_stats = 1
        u.zero_()
        _, rs = P.solve(f, u, o)
        key = "pmf" if eps == "pmf" else f"{eps:.0e}"
        rows[key] = {"iterations": r.iters, "time_to_solve_s": round(r.t_solve, 4),
                     "us_per_dof": round(r.t_solve / P.ndof * 1e6, 5), "inner_avg": round(rs.inner_avg, 3),
                     "inner_max": rs.inner_max}
        log(f"[bench] {w.name} eps={key}: {r.iters} it, {r.t_solve * 1e3:.1f} ms, inner avg {rs.inner_avg:.2f} "
            f"max {rs.inner_max}")
    P.close()
    return rows


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


def is_convective(w) -> bool:
    import numpy as np

    return bool(tuple(w.b0) != (0.0, 0.0, 0.0) or np.any(np.asarray(w.B) != 0))


# workloads whose coarse problem is solved by the aggregation AMG (two
# cycles, two Jacobi sweeps per level): the SPE10-like field and the
# convection box; the isotropic Poisson boxes keep the geometric cycle
AMG_WORKLOADS = ("spe10-like", "convection-48")


def leg_settings(w, coarse_opt: str = "auto", coarse_solver: str = "auto"):
    """Solver settings of a workload: (solve-option builder, smoother dict,
    coarse-space name, description).  The 8^3 Poisson problem takes one
    block-Jacobi sweep as the preconditioner of CG to 1e-10 (its stated
    solve); the others the hybrid V-cycle to 1e-8: FCG and block-Jacobi with
    inner PCG for diffusion, FGMRES(30) and inner GMRES(8) with the Thomas
    preconditioner for convection (Sec. 3.2, 4.3); the coarse problem by the
    geometric cycle or the aggregation AMG (AMG_WORKLOADS)."""
    from paper_1805_11930_amd import (DG_COARSE_P0, DG_COARSE_Q1, DG_INNER_CG, DG_INNER_GMRES, DG_IPREC_DIAG,
                                      DG_IPREC_TRIDIAG, DG_KRYLOV_FCG, DG_KRYLOV_FGMRES, DG_PRECOND_BLOCK,
                                      DG_PRECOND_MG, solve_opts)

    conv = is_convective(w)
    sm = (dict(eps=1e-2, inner=DG_INNER_GMRES, restart=8, inner_precond=DG_IPREC_TRIDIAG) if conv
          else dict(eps=1e-2, inner=DG_INNER_CG, inner_precond=DG_IPREC_DIAG))
    coarse_name = w.coarse if coarse_opt == "auto" else coarse_opt
    if coarse_name == "auto":
        coarse_name = "p0" if conv else "q1"
    coarse = DG_COARSE_Q1 if coarse_name == "q1" else DG_COARSE_P0
    krylov = DG_KRYLOV_FGMRES if conv else DG_KRYLOV_FCG
    if w.name.startswith("poisson-8^3"):
        def opts(prec, **kw):
            return solve_opts(krylov=DG_KRYLOV_FCG, precond=DG_PRECOND_BLOCK, precond_precision=prec, rtol=1e-10,
                              maxit=1000, smooth=dict(sm, n_sweeps=1), **kw)
        desc = "flexible CG to 1e-10, one block-Jacobi sweep (inner PCG eps 1e-2) as preconditioner"
        return opts, sm, "none", desc

    amg = coarse_solver == "amg" or (coarse_solver == "auto" and w.name.startswith(AMG_WORKLOADS))
    mg = dict(coarse_space=coarse)
    if amg:
        mg.update(coarse_solver=1, coarse_cycles=2, coarse_smooth=2)

    def opts(prec, **kw):
        return solve_opts(krylov=krylov, restart=30, precond=DG_PRECOND_MG, precond_precision=prec, rtol=1e-8,
                          maxit=1000, smooth=sm, mg=mg, **kw)
    desc = (("FGMRES(30)" if conv else "flexible CG") + " to 1e-8, hybrid V-cycle (block-Jacobi, " +
            ("inner GMRES(8) with the Thomas preconditioner" if conv else "inner PCG") +
            f" eps 1e-2, {coarse_name.upper()} coarse space, " +
            ("aggregation AMG coarse solver, 2 cycles)" if amg else "geometric coarse cycle)"))
    return opts, sm, coarse_name, desc


def apply_kernel_name(w) -> str:
    return f"k_apply<{w.p}, double, true, 0, false, {'true' if is_convective(w) else 'false'}>"


def pmf_rows(P, w, f, opts, steps: int) -> dict:
    """The partially matrix-free variant (Sec. 4.1): the same solves with
    the block solves done by the stored inverses of the blocks D_T (built
    on the device on first use; the build is timed as setup)."""
    import torch

    from paper_1805_11930_amd import DG_FP32, DG_FP64, DG_INNER_PMF, smooth_opts

    f32 = f.float() / f.norm()
    u32 = torch.zeros_like(f32)
    out32 = torch.empty_like(f32)
    smp = smooth_opts(inner=DG_INNER_PMF)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P.block_smooth(f32, u32, smp, out=out32)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    t_sm = event_time(lambda: P.block_smooth(f32, u32, smp, out=out32), 5)
    nn = (w.p + 1) ** 3
    mat_bytes = P.ncell * nn * nn * 4
    u = torch.zeros_like(f)
    res = {}
    for name, prec in (("fp64", DG_FP64), ("mixed", DG_FP32)):
        o = opts(prec)
        o.mg.smooth.inner = DG_INNER_PMF
        o.mg.smooth.inner_precond = 0  # an exact block solve has no inner preconditioner
        rs = []
        for _ in range(steps + 1):
            u.zero_()
            _, r = P.solve(f, u, o)
            rs.append(r)
        res[name] = rs[1:]
    import numpy as np

    row = {
        "inner": "stored inverse of every block D_T (partially matrix-free)",
        "build_s": round(t_build, 4),
        "stored_bytes_fp64_fp32": int(P.ncell * nn * nn * 12),
        "smoother_sweep_fp32_ms": round(t_sm * 1e3, 4),
        "smoother_sweep_roofline": {"bound": "hbm", "kernel": f"k_smooth<{w.p}, 3, float, ...> (stored inverse)",
                                    "achieved": round(mat_bytes / t_sm / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                    "frac": round(mat_bytes / t_sm / 1e9 / HBM_PEAK_GBS, 4),
                                    "bytes_per_launch": int(mat_bytes)},
        "time_to_solve_s": {k: round(float(np.median([r.t_solve for r in v])), 5) for k, v in res.items()},
        "iterations": {k: v[-1].iters for k, v in res.items()},
        "rel_residual": {k: v[-1].rel_residual for k, v in res.items()},
    }
    log(f"[bench] {w.name} PMF: build {t_build * 1e3:.1f} ms, sweep {t_sm * 1e3:.3f} ms, FP64-prec "
        f"{row['time_to_solve_s']['fp64'] * 1e3:.1f} ms ({row['iterations']['fp64']} it), mixed "
        f"{row['time_to_solve_s']['mixed'] * 1e3:.1f} ms ({row['iterations']['mixed']} it)")
    return row


def solve_leg(w, steps: int, warmup: int, coarse_opt: str = "auto", smoother_rows: bool = True,
              pmf: bool = True) -> dict:
    """One workload: FP64-preconditioned and mixed-precision solves (each
    time-to-solve from dg_solve_result.t_solve, setup separately), the FP64
    applies inside the mixed solves (dispatch-recorded events), per-result
    FP64 errors (against the exact solution when known, and mixed against
    the FP64-preconditioned answer), the inner iterations counted inside the
    solve, and the smoother sweep and V-cycle of the same settings."""
    import numpy as np
    import torch

    from paper_1805_11930_amd import DG_FP32, DG_FP64, Problem, ProblemSpec, mg_opts, smooth_opts

    opts, smd, coarse_name, desc = leg_settings(w, coarse_opt)
    t0 = time.perf_counter()
    P = Problem(ProblemSpec(cells=w.cells, lengths=w.lengths, p=w.p, bc=w.bc, sigma=w.sigma, K=w.K, c=w.c,
                            b0=w.b0, B=w.B))
    f = P.rhs_from_functions(f=w.f, g=w.g, j=w.j)
    exact = None
    if w.exact is not None:
        exact = torch.from_numpy(np.ascontiguousarray(w.exact(P.node_points()), dtype=np.float64)).cuda()
    torch.cuda.synchronize()
    t_problem = time.perf_counter() - t0
    u = torch.zeros_like(f)

    def run(o):
        u.zero_()
        _, r = P.solve(f, u, o)
        return r

    out = {"workload": w.name, "cells": list(w.cells), "p": w.p, "ndof": P.ndof, "solver": desc,
           "problem_setup_s": round(t_problem, 3)}
    res = {}
    for name, prec in (("fp64", DG_FP64), ("mixed", DG_FP32)):
        o = opts(prec)
        for _ in range(warmup):
            run(o)
        torch.cuda.synchronize()
        rs = []
        t0 = time.perf_counter()
        for _ in range(steps):
            rs.append(run(o))
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps
        res[name] = (rs, wall)
        if name == "fp64":
            u64 = u.clone()
    ts = {k: [r.t_solve for r in v[0]] for k, v in res.items()}
    out["time_to_solve_s"] = {k: round(float(np.median(v)), 5) for k, v in ts.items()}
    out["time_to_solve_min_s"] = {k: round(min(v), 5) for k, v in ts.items()}
    out["wall_per_solve_s"] = {k: round(v[1], 5) for k, v in res.items()}
    out["solve_setup_s"] = {k: round(float(np.median([r.t_setup for r in v[0]])), 5) for k, v in res.items()}
    out["iterations"] = {k: v[0][-1].iters for k, v in res.items()}
    out["rel_residual"] = {k: v[0][-1].rel_residual for k, v in res.items()}
    out["status"] = {k: v[0][-1].status for k, v in res.items()}
    mixed = res["mixed"][0]
    t_apply = sum(r.t_apply for r in mixed)
    n_apply = sum(r.n_apply for r in mixed)
    apply_s = t_apply / max(n_apply, 1)
    bpd = bytes_per_dof(w.p, 8)
    out["apply_fp64_gdofs_in_solve"] = round(P.ndof / apply_s / 1e9, 3)
    out["apply_launches_timed"] = n_apply
    achieved = bpd * P.ndof / apply_s / 1e9
    out["roofline"] = {"bound": "hbm", "kernel": apply_kernel_name(w), "achieved": round(achieved, 1),
                       "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                       "bytes_per_dof": round(bpd, 3), "launch_us": round(apply_s * 1e6, 2)}
    # per-result errors and in-solve inner counts (untimed runs)
    err = {}
    inner = {}
    phases = {}
    for name, prec in (("fp64", DG_FP64), ("mixed", DG_FP32)):
        ref = exact if exact is not None else (u64 if name == "mixed" else None)
        r = run(opts(prec, inner_stats=1, u_ref=ref.data_ptr() if ref is not None else None))
        inner[name] = {"avg": round(r.inner_avg, 3), "max": r.inner_max, "blocks": r.inner_blocks}
        # where the time of the solve goes (event-timed phases of that run)
        phases[name] = {"solve_s": round(r.t_solve, 5), "apply_outer_s": round(r.t_apply, 5),
                        "precond_s": round(r.t_precond, 5), "smoother_s": round(r.t_smoother, 5),
                        "residual_restrict_s": round(r.t_restrict, 5), "coarse_s": round(r.t_coarse, 5),
                        "prolong_s": round(r.t_prolong, 5),
                        "rest_s": round(max(r.t_solve - r.t_apply - r.t_precond, 0.0), 5)}
        if exact is not None:
            err[f"{name}_vs_exact"] = r.error
        elif name == "mixed":
            err["mixed_vs_fp64"] = r.error
    if exact is not None:
        r = run(opts(DG_FP32, u_ref=u64.data_ptr()))
        err["mixed_vs_fp64"] = r.error
    out["error"] = err
    out["inner_in_solve"] = inner
    out["phases"] = phases
    # standalone applies and the preconditioner pieces of the same settings
    u_rand = torch.from_numpy(np.random.default_rng(3).normal(size=P.ndof)).cuda()
    v64 = torch.empty_like(u_rand)
    u32 = u_rand.float()
    v32 = torch.empty_like(u32)
    out["apply_fp64_gdofs"] = round(P.ndof / event_time(lambda: P.apply(u_rand, v64), 20) / 1e9, 2)
    out["apply_fp32_gdofs"] = round(P.ndof / event_time(lambda: P.apply(u32, v32), 20) / 1e9, 2)
    if smoother_rows:
        f32 = f.float() / f.norm()
        sm = smooth_opts(**smd)
        out32 = torch.empty_like(f32)
        t_sm = event_time(lambda: P.block_smooth(f32, u32, sm, out=out32), 5)
        _, st = P.block_smooth(f32, u32, sm, out=out32, stats=True)
        out["smoother_sweep_fp32_ms"] = round(t_sm * 1e3, 4)
        out["smoother_inner_avg"] = round(st.inner_avg, 3)
        out["smoother_inner_max"] = st.inner_max
        if smd["inner"] == 0:
            # algorithmic flops of the inner-PCG sweep: per cell the defect
            # (three line operators on N^2 lines, N x N contractions, and the
            # face terms: 6 N^4 + 20 N^3) and per inner iteration one D_T
            # product (6 N^4) plus the dot products and updates (13 N^3)
            nn = w.p + 1
            fl = P.ncell * (6 * nn**4 + 20 * nn**3) + st.inner_total * (6 * nn**4 + 13 * nn**3)
            out["smoother_roofline"] = {"bound": "alu", "kernel": f"k_smooth<{w.p}, 0, float, false, false, 16>",
                                        "achieved": round(fl / t_sm / 1e12, 2), "peak": FP32_VECTOR_PEAK_TFLOPS,
                                        "unit": "TFLOP/s", "frac": round(fl / t_sm / 1e12 / FP32_VECTOR_PEAK_TFLOPS, 4),
                                        "flops_per_launch": int(fl)}
        else:
            out["smoother_kernel"] = f"k_smooth<{w.p}, 1, float, true, true, 8> (inner GMRES(8), Thomas)"
        if coarse_name != "none":
            from paper_1805_11930_amd import DG_COARSE_P0, DG_COARSE_Q1

            o1 = opts(1)
            mo = mg_opts(smooth=smd, coarse_space=DG_COARSE_Q1 if coarse_name == "q1" else DG_COARSE_P0,
                         coarse_solver=o1.mg.coarse_solver, coarse_cycles=o1.mg.coarse_cycles,
                         coarse_smooth=o1.mg.coarse_smooth)
            out["vcycle_fp32_ms"] = round(event_time(lambda: P.mg_vcycle(f32, mo, out=out32), 5) * 1e3, 4)
    if pmf and w.p <= 4:
        out["pmf"] = pmf_rows(P, w, f, opts, steps)
    log(f"[bench] {w.name}: FP64-prec {out['time_to_solve_s']['fp64'] * 1e3:.1f} ms ({out['iterations']['fp64']} it), "
        f"mixed {out['time_to_solve_s']['mixed'] * 1e3:.1f} ms ({out['iterations']['mixed']} it), apply "
        f"{out['apply_fp64_gdofs_in_solve']} GDOF/s (frac {out['roofline']['frac']}), errors {err}, inner {inner}")
    P.close()
    return out


def fdm_leg(w, steps: int = 3) -> dict:
    """Stored-factor (fast diagonalisation) exact block solve in the same
    V-cycle and solves (b = 0)."""
    import torch

    from paper_1805_11930_amd import DG_FP32, DG_FP64, DG_INNER_FDM, Problem, ProblemSpec, smooth_opts, solve_opts

    opts, _, coarse_name, _ = leg_settings(w)
    P = Problem(ProblemSpec(cells=w.cells, lengths=w.lengths, p=w.p, bc=w.bc, sigma=w.sigma, K=w.K, c=w.c,
                            b0=w.b0, B=w.B))
    f = P.rhs_from_functions(f=w.f, g=w.g, j=w.j)
    u = torch.zeros_like(f)
    f32 = f.float() / f.norm()
    u32 = torch.zeros_like(f32)
    out32 = torch.empty_like(f32)
    smf = smooth_opts(inner=DG_INNER_FDM)
    P.block_smooth(f32, u32, smf, out=out32)
    t_smf = event_time(lambda: P.block_smooth(f32, u32, smf, out=out32), 5)
    res = {}
    for name, prec in (("mixed", DG_FP32), ("fp64", DG_FP64)):
        o = opts(prec)
        o.mg.smooth.inner = DG_INNER_FDM
        best = None
        for _ in range(steps + 1):
            u.zero_()
            _, r = P.solve(f, u, o)
            best = r if best is None or r.t_solve < best.t_solve else best
        res[name] = best
    P.close()
    log(f"[bench] FDM smoother: sweep {t_smf * 1e3:.3f} ms, mixed solve {res['mixed'].t_solve * 1e3:.1f} ms "
        f"({res['mixed'].iters} it), FP64 {res['fp64'].t_solve * 1e3:.1f} ms")
    return {
        "inner": "exact block solve by fast diagonalisation (stored per-cell factors)",
        "smoother_sweep_fp32_ms": round(t_smf * 1e3, 3),
        "time_to_solve_s": {k: round(v.t_solve, 4) for k, v in res.items()},
        "iterations": {k: v.iters for k, v in res.items()},
        "rel_residual": {k: v.rel_residual for k, v in res.items()},
    }


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="w2", choices=["w1", "w2", "w3", "w4"])
    ap.add_argument("--coarse", default="auto", choices=["auto", "p0", "q1"],
                    help="coarse space of the V-cycle (auto: the workload's own; Q1 for the diffusion boxes, P0 "
                         "for the convection box)")
    ap.add_argument("--legs", default="w1,w3,w4",
                    help="other single-GPU configurations to run as their own legs (comma list of w1..w4, "
                         "or 'none')")
    ap.add_argument("--leg-steps", type=int, default=3, help="timed solves per precision in each extra leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=256, help="serving leg size (0 = skip)")
    ap.add_argument("--pe2000", type=int, default=1, help="run the Pe=2000 convection leg (0 = skip)")
    ap.add_argument("--basis", type=int, default=1,
                    help="run the Gauss-Lobatto vs Gauss-Legendre inner-iteration leg on the p=3 grids (0 = skip)")
    ap.add_argument("--diffusion", type=int, default=1,
                    help="run the Poisson / inhomogeneous diffusion leg on the paper's p=3 grid (0 = skip)")
    ap.add_argument("--fdm", type=int, default=1, help="run the stored-factor smoother leg on the main workload")
    ap.add_argument("--pmf", type=int, default=1,
                    help="time the partially matrix-free variant (stored block inverses) in every leg")
    ap.add_argument("--smooth-inner", default="own", choices=["own", "pmf"],
                    help="--smooth-only: the workload's own block solver, or the stored block inverses")
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

    from paper_1805_11930_amd import Problem, ProblemSpec, smooth_opts

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
    if args.apply_only or args.smooth_only:
        P = Problem(ProblemSpec(cells=w.cells, lengths=w.lengths, p=w.p, bc=w.bc, sigma=w.sigma, K=w.K, c=w.c,
                                b0=w.b0, B=w.B))
        u_rand = torch.from_numpy(np.random.default_rng(3).normal(size=P.ndof)).cuda()
        if args.apply_only:
            v = torch.empty_like(u_rand)
            for _ in range(args.apply_only):
                P.apply(u_rand, v)
            torch.cuda.synchronize()
            log(f"[bench] ran {args.apply_only} FP64 applies")
        else:
            f32 = (u_rand / u_rand.norm()).float()
            u32 = torch.zeros_like(f32)
            o32 = torch.empty_like(f32)
            _, smd, _, _ = leg_settings(w, args.coarse)  # the workload's own block solver
            if args.smooth_inner == "pmf":
                smd = dict(inner=3)  # DG_INNER_PMF
            sm = smooth_opts(**smd)
            for _ in range(args.smooth_only):
                P.block_smooth(f32, u32, sm, out=o32)
            torch.cuda.synchronize()
            log(f"[bench] ran {args.smooth_only} FP32 smoother sweeps")
        P.close()
        return 0
    # ---- the timed steps: mixed-precision solves of the main workload -----
    opts, smd, coarse_name, desc = leg_settings(w, args.coarse)
    P = Problem(ProblemSpec(cells=w.cells, lengths=w.lengths, p=w.p, bc=w.bc, sigma=w.sigma, K=w.K, c=w.c,
                            b0=w.b0, B=w.B))
    f = P.rhs_from_functions(f=w.f, g=w.g, j=w.j)
    u = torch.zeros_like(f)
    o_mixed = opts(1)
    for i in range(args.warmup):
        u.zero_()
        _, res = P.solve(f, u, o_mixed)
        log(f"[bench] warmup {i}: iters={res.iters} rel_res={res.rel_residual:.2e} t={res.t_solve:.3f}s")
    torch.cuda.synchronize()
    t_apply = 0.0
    n_apply = 0
    iters = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        u.zero_()
        _, res = P.solve(f, u, o_mixed)
        t_apply += res.t_apply
        n_apply += res.n_apply
        iters.append(res.iters)
        if res.status != 0:
            log(f"[bench] step {i} did not converge: status={res.status} rel_res={res.rel_residual:.2e}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    log(f"[bench] timed {args.steps} mixed solves: {ms_per_step:.1f} ms/step, iters={iters}")
    P.close()
    apply_s = t_apply / max(n_apply, 1)
    gdofs = w.ndof / apply_s / 1e9
    bpd = bytes_per_dof(w.p, 8)
    achieved = bpd * w.ndof / apply_s / 1e9
    # ---- the rest of the hot path, outside the timed region ---------------
    main_leg = solve_leg(w, max(args.steps, 3), 1, args.coarse, pmf=bool(args.pmf))
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
            "ndof": w.ndof,
            "step": "one FP64 Krylov solve preconditioned in FP32: " + desc,
            "coarse_space": coarse_name,
            "value_from": "mean duration of the FP64 operator-apply kernel inside the timed solves (HIP events "
                          "recorded by its dispatch)",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": apply_kernel_name(w),
            "bytes_per_dof": round(bpd, 3),
            "launch_us": round(apply_s * 1e6, 2),
        },
        "time_to_solve_s": main_leg["time_to_solve_s"],
        "iterations": {"mixed_timed": iters, **main_leg["iterations"]},
        "rel_residual": main_leg["rel_residual"],
        "error": main_leg["error"],
        "inner_in_solve": main_leg["inner_in_solve"],
        "main": main_leg,
    }
    if args.fdm and not is_convective(w):
        line["fdm_smoother"] = fdm_leg(w)
    legs = [] if args.legs in ("", "none", "0") else [x for x in args.legs.split(",") if x and x != args.workload]
    line["workloads"] = {}
    for name in legs:
        wl = make_workload(name)
        log(f"[bench] leg {name}: {wl.name}, {wl.ndof} DOF")
        line["workloads"][name] = solve_leg(wl, args.leg_steps, 1, pmf=bool(args.pmf))
    if args.diffusion:
        line["diffusion_sec42"] = diffusion_leg()
    if args.pe2000:
        line["convection_pe2000"] = pe2000_leg()
    if args.basis:
        line["inner_iterations_by_basis"] = basis_leg()
    if args.serve_requests > 0:
        line["serving"] = serving_leg(args.serve_requests)
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline ...")
        line["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
