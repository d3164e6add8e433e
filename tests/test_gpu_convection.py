"""GPU parity of the tridiagonal (Thomas) inner preconditioner and of the
convection-dominated solve of Sec. 4.3 against the oracle, through the
C ABI.

  * block solves with inner GMRES preconditioned by the tridiagonal part of
    D_T: at eps = 1e-2 the GPU replays the oracle's steps (equal per-cell
    iteration counts, iterates <= 1e-9), at a tiny eps it reaches the dense
    block solve; Pe = 2000 blocks with b = (1,0,0) and (1, 0.5, 0.3) at
    p = 2-4, and random affine-b cases at p = 1-3;
  * block-SSOR sweeps with the Thomas-preconditioned inner GMRES match the
    oracle's alg block_SOR sweeps;
  * the Pe = 2000 problem (small grid) solved by FGMRES preconditioned with
    two block-SSOR steps reaches 1e-8 in FP64 and mixed precision and the
    sparse direct solution; its exact solution lies in the DG space, so the
    discrete solution reproduces it.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import dg, solvers
from paper_1805_11930_amd import inputs
from tests.helpers import oracle_problem, rel, spec

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")


def _lib(w):
    from paper_1805_11930_amd import Problem

    return Problem(spec(w))


CASES = [("pe-x", 2), ("pe-x", 3), ("pe-x", 4), ("pe-xyz", 2), ("pe-xyz", 3), ("pe-xyz", 4),
         ("rand", 1), ("rand", 2), ("rand", 3)]


def _case(kind, p):
    if kind == "rand":
        return inputs.random_case(p, cells=(5, 3, 4), seed=30 + p, with_b=True)
    b = (1.0, 0.0, 0.0) if kind == "pe-x" else (1.0, 0.5, 0.3)
    return inputs.pe2000(b=b, p=p, cells=(3, 4, 5))


@pytest.mark.parametrize("kind,p", CASES)
def test_thomas_block_gmres_replay(kind, p):
    from paper_1805_11930_amd import DG_INNER_GMRES, DG_IPREC_TRIDIAG, smooth_opts

    print(f"Thomas block GMRES {kind} p={p}", flush=True)
    w = _case(kind, p)
    opr = oracle_problem(w)
    A = dg.assemble(opr)
    Db = dg.block_diagonal(A, opr.ncell)
    d = inputs.random_vector(opr.ndof, 51)
    D = d.reshape(opr.ncell, -1)
    restart = min(12, opr.nloc)
    ref, its = [], []
    for T in range(opr.ncell):
        x, it = solvers.block_gmres(Db[T], D[T], 1e-2, opr.nloc, restart, "tridiag")
        ref.append(x)
        its.append(it)
    P = _lib(w)
    o = smooth_opts(eps=1e-2, inner=DG_INNER_GMRES, restart=12, inner_precond=DG_IPREC_TRIDIAG)
    x, it_gpu = P.block_solve(torch.from_numpy(d).cuda(), o, iters=True)
    assert list(it_gpu.cpu().numpy()) == its
    xg = x.cpu().numpy().reshape(opr.ncell, -1)
    for T in range(opr.ncell):
        assert rel(xg[T], ref[T]) <= 1e-9
    xt = P.block_solve(torch.from_numpy(d).cuda(),
                       smooth_opts(eps=1e-13, inner=DG_INNER_GMRES, restart=12, inner_precond=DG_IPREC_TRIDIAG,
                                   max_inner=20 * opr.nloc))
    dense = np.concatenate([np.linalg.solve(Db[T], D[T]) for T in range(opr.ncell)])
    assert rel(xt.cpu().numpy(), dense) <= 1e-9
    # FP32: every block meets the tolerance (within FP32 rounding)
    x32 = P.block_solve(torch.from_numpy(d).float().cuda(), o).cpu().numpy().astype(np.float64)
    x32 = x32.reshape(opr.ncell, -1)
    for T in range(opr.ncell):
        assert np.linalg.norm(D[T] - Db[T] @ x32[T]) <= 1.05e-2 * np.linalg.norm(D[T])
    P.close()


@pytest.mark.parametrize("kind,p", [("pe-xyz", 3), ("rand", 2)])
def test_ssor_with_thomas_vs_oracle(kind, p):
    from paper_1805_11930_amd import DG_INNER_GMRES, DG_IPREC_TRIDIAG, DG_SWEEP_SSOR, smooth_opts

    print(f"SSOR + Thomas {kind} p={p}", flush=True)
    w = _case(kind, p)
    opr = oracle_problem(w)
    A = dg.assemble(opr)
    Db = dg.block_diagonal(A, opr.ncell)
    f = inputs.random_vector(opr.ndof, 52)
    ref = solvers.block_ssor(A, Db, f, np.zeros_like(f), solvers.multicolour_order(opr), omega=1.0, nsweeps=2,
                             inner="gmres", eps=1e-2, restart=12, precond="tridiag")
    P = _lib(w)
    o = smooth_opts(n_sweeps=2, omega=1.0, eps=1e-2, inner=DG_INNER_GMRES, restart=12,
                    inner_precond=DG_IPREC_TRIDIAG, sweep=DG_SWEEP_SSOR)
    got = P.block_smooth(torch.from_numpy(f).cuda(), None, o)
    assert rel(got.cpu().numpy(), ref) <= 1e-9
    P.close()


@pytest.mark.parametrize("b", [(1.0, 0.0, 0.0), (1.0, 0.5, 0.3)])
def test_pe2000_solve_block_ssor_fgmres(b):
    from paper_1805_11930_amd import (DG_FP32, DG_FP64, DG_INNER_GMRES, DG_IPREC_TRIDIAG, DG_KRYLOV_FGMRES,
                                      DG_PRECOND_BLOCK, DG_SWEEP_SSOR, solve_opts)

    w = inputs.pe2000(b=b, p=2, cells=(6, 6, 12))
    print(f"Pe=2000 solve b={b} 6x6x12 p=2", flush=True)
    opr = oracle_problem(w)
    A = dg.assemble(opr)
    rhs = dg.assemble_rhs(opr, f=w.f)
    ref = spla.spsolve(A.tocsc(), rhs)
    ue = dg.interpolate(opr, w.exact)
    assert rel(ref, ue) <= 1e-9  # the exact solution is in the DG space
    P = _lib(w)
    f = P.rhs_from_functions(f=w.f)
    its = {}
    for prec in (DG_FP64, DG_FP32):
        o = solve_opts(krylov=DG_KRYLOV_FGMRES, restart=30, precond=DG_PRECOND_BLOCK, precond_precision=prec,
                       rtol=1e-8, maxit=200,
                       smooth=dict(n_sweeps=2, sweep=DG_SWEEP_SSOR, omega=1.0, eps=1e-2, inner=DG_INNER_GMRES,
                                   restart=12, inner_precond=DG_IPREC_TRIDIAG))
        u, res = P.solve(f, opts=o)
        print(f"  prec={prec} iters={res.iters} rel_res={res.rel_residual:.3e} inner_avg={res.inner_avg:.2f}",
              flush=True)
        assert res.status == 0 and res.rel_residual <= 1e-8
        assert rel(u.cpu().numpy(), ref) <= 1e-6
        its[prec] = res.iters
    assert its[DG_FP64] <= 40
    P.close()


def test_tridiag_rejected_with_cg():
    from paper_1805_11930_amd import DG_INNER_CG, DG_IPREC_TRIDIAG, DgError, smooth_opts

    w = inputs.random_case(1, cells=(2, 2, 2), seed=3)
    P = _lib(w)
    d = torch.from_numpy(inputs.random_vector(w.ndof, 53)).cuda()
    with pytest.raises(DgError):
        P.block_solve(d, smooth_opts(inner=DG_INNER_CG, inner_precond=DG_IPREC_TRIDIAG))
    P.close()
