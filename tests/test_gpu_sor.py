"""GPU parity of the red-black block-SOR / block-SSOR smoother (alg
block_SOR, Sec. 2.2.1) against the oracle, through the C ABI.

  * forward, backward and symmetric sweeps from a given u and from zero in
    the red-black and in 3-, 4- and 5-colour diagonal orders, p = 1-4, with and without advection, on grids with odd and even cell
    counts per axis (the colour slots of a row and its partner cell), inner
    PCG / GMRES at the paper's eps = 1e-2 (the GPU replays the oracle's
    inner steps) and the exact stored-factor solve: FP64 <= 1e-9;
  * in place (u_in == u_out) equals out of place;
  * with one colour per diagonal plane the order is downwind, and one SOR
    sweep solves a pure-advection problem (red-black does not);
  * FP32 sweeps <= 1e-3 of the FP64 oracle;
  * the V-cycle with SOR / SSOR smoothing and the exact P0 coarse solve
    matches the oracle's cycle (forward pre-, backward postsmoothing);
  * two block-SSOR steps precondition FGMRES on a convection problem (the
    paper's preconditioner for convection-dominated flow, Sec. 4.3) and the
    solve reaches the sparse direct solution.
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


def _setup(p, with_b, cells, seed=0):
    w = inputs.random_case(p, cells=cells, seed=seed, with_b=with_b)
    opr = oracle_problem(w)
    A = dg.assemble(opr)
    Db = dg.block_diagonal(A, opr.ncell)
    return w, opr, A, Db


def _oracle_sweeps(A, Db, opr, f, u0, kind, n, colours=2, **kw):
    order = solvers.multicolour_order(opr, colours)
    if kind == "ssor":
        return solvers.block_ssor(A, Db, f, u0, order, nsweeps=n, **kw)
    return solvers.block_sor(A, Db, f, u0, order[::-1] if kind == "back" else order, nsweeps=n, **kw)


KINDS = {"sor": 1, "ssor": 2, "back": 3}


@pytest.mark.parametrize("p,with_b,cells,kind,C", [
    (1, False, (5, 4, 3), "sor", 2),
    (2, False, (6, 3, 4), "ssor", 2),
    (2, True, (5, 4, 3), "back", 2),
    (3, True, (4, 5, 3), "ssor", 2),
    (4, False, (3, 3, 5), "sor", 2),
    (3, False, (1, 3, 4), "ssor", 2),
    (2, True, (7, 4, 3), "ssor", 3),
    (1, False, (5, 6, 2), "sor", 5),
    (3, True, (9, 2, 3), "back", 4),
])
def test_sor_sweeps_vs_oracle(p, with_b, cells, kind, C):
    from paper_1805_11930_amd import DG_INNER_CG, DG_INNER_GMRES, smooth_opts

    print(f"block-SOR {kind} p={p} b={with_b} cells={cells} colours={C}", flush=True)
    w, opr, A, Db = _setup(p, with_b, cells, seed=21)
    f = inputs.random_vector(opr.ndof, 41)
    u0 = inputs.random_vector(opr.ndof, 42)
    inner = "gmres" if with_b else "cg"
    kw = dict(omega=1.1, inner=inner, eps=1e-2, restart=12, colours=C)
    P = _lib(w)
    o = smooth_opts(n_sweeps=2, omega=1.1, eps=1e-2, inner=DG_INNER_GMRES if with_b else DG_INNER_CG, restart=12,
                    sweep=KINDS[kind], colours=C)
    ref = _oracle_sweeps(A, Db, opr, f, u0, kind, 2, **kw)
    got, st = P.block_smooth(torch.from_numpy(f).cuda(), torch.from_numpy(u0).cuda(), o, stats=True)
    assert rel(got.cpu().numpy(), ref) <= 1e-9
    ndir = 4 if kind == "ssor" else 2
    assert st.blocks == ndir * opr.ncell and 1 <= st.inner_max <= opr.nloc
    # from zero
    ref0 = _oracle_sweeps(A, Db, opr, f, np.zeros_like(f), kind, 1, **kw)
    o.n_sweeps = 1
    got0 = P.block_smooth(torch.from_numpy(f).cuda(), None, o, out=torch.full_like(torch.from_numpy(f).cuda(), 7.0))
    assert rel(got0.cpu().numpy(), ref0) <= 1e-9
    # in place
    u = torch.from_numpy(u0).cuda()
    o.n_sweeps = 2
    P.block_smooth(torch.from_numpy(f).cuda(), u, o, out=u)
    assert rel(u.cpu().numpy(), ref) <= 1e-9
    # FP32
    got32 = P.block_smooth(torch.from_numpy(f).float().cuda(), torch.from_numpy(u0).float().cuda(), o)
    assert rel(got32.cpu().numpy().astype(np.float64), ref) <= 1e-3
    P.close()


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_ssor_exact_blocks(p):
    from paper_1805_11930_amd import DG_INNER_FDM, smooth_opts

    print(f"block-SSOR exact blocks p={p}", flush=True)
    w, opr, A, Db = _setup(p, False, (5, 3, 4), seed=22)
    f = inputs.random_vector(opr.ndof, 43)
    u0 = inputs.random_vector(opr.ndof, 44)
    ref = _oracle_sweeps(A, Db, opr, f, u0, "ssor", 2, omega=1.3, inner="exact")
    P = _lib(w)
    o = smooth_opts(n_sweeps=2, omega=1.3, inner=DG_INNER_FDM, sweep=KINDS["ssor"])
    got = P.block_smooth(torch.from_numpy(f).cuda(), torch.from_numpy(u0).cuda(), o)
    assert rel(got.cpu().numpy(), ref) <= 1e-11
    P.close()


@pytest.mark.parametrize("p,with_b,kind", [(2, False, "sor"), (3, False, "ssor"), (2, True, "ssor")])
def test_vcycle_sor_smoothing(p, with_b, kind):
    from paper_1805_11930_amd import DG_COARSE_P0, DG_INNER_CG, DG_INNER_GMRES, mg_opts

    print(f"V-cycle {kind} p={p} b={with_b}", flush=True)
    w, opr, A, Db = _setup(p, with_b, (5, 4, 3), seed=23)
    r = inputs.random_vector(opr.ndof, 45)
    inner = "gmres" if with_b else "cg"
    cs = solvers.exact_coarse(solvers.p0_direct(opr))
    ref = solvers.vcycle(A, Db, opr, r, cs, n_pre=1, n_post=1, omega=1.0, inner=inner, eps=1e-2, restart=12,
                         smoother=kind)
    P = _lib(w)
    o = mg_opts(smooth=dict(omega=1.0, eps=1e-2, inner=DG_INNER_GMRES if with_b else DG_INNER_CG, restart=12,
                            sweep=KINDS[kind]),
                n_pre=1, n_post=1, coarse_space=DG_COARSE_P0)
    z = P.mg_vcycle(torch.from_numpy(r).cuda(), o)
    assert rel(z.cpu().numpy(), ref) <= 1e-9
    P.close()


def test_block_ssor_preconditioned_fgmres_convection():
    from paper_1805_11930_amd import (DG_FP32, DG_FP64, DG_INNER_GMRES, DG_KRYLOV_FGMRES, DG_PRECOND_BLOCK,
                                      solve_opts)

    w = inputs.w4(cells=(8, 8, 8), p=2)
    print("FGMRES + 2 block-SSOR, convection 8^3 p=2", flush=True)
    opr = oracle_problem(w)
    A = dg.assemble(opr)
    rhs = dg.assemble_rhs(opr, f=w.f)
    ref = spla.spsolve(A.tocsc(), rhs)
    P = _lib(w)
    f = P.rhs_from_functions(f=w.f)
    its = {}
    for prec in (DG_FP64, DG_FP32):
        o = solve_opts(krylov=DG_KRYLOV_FGMRES, restart=30, precond=DG_PRECOND_BLOCK, precond_precision=prec,
                       rtol=1e-8, maxit=300,
                       smooth=dict(n_sweeps=2, sweep=KINDS["ssor"], omega=1.0, eps=1e-2, inner=DG_INNER_GMRES,
                                   restart=12))
        u, res = P.solve(f, opts=o)
        print(f"  prec={prec} iters={res.iters} rel_res={res.rel_residual:.3e}", flush=True)
        assert res.status == 0 and res.rel_residual <= 1e-8
        assert rel(u.cpu().numpy(), ref) <= 1e-6
        its[prec] = res.iters
    assert abs(its[DG_FP32] - its[DG_FP64]) <= 2
    P.close()


def test_sor_options_rejected():
    from paper_1805_11930_amd import DgError, smooth_opts

    w, opr, A, Db = _setup(1, False, (2, 2, 2))
    P = _lib(w)
    f = torch.from_numpy(inputs.random_vector(opr.ndof, 46)).cuda()
    with pytest.raises(DgError):
        P.block_smooth(f, f, smooth_opts(sweep=7))
    with pytest.raises(DgError):
        P.block_smooth(f, None, smooth_opts(sweep=1), out=f)  # u_out == f
    with pytest.raises(DgError):
        P.block_smooth(f, None, smooth_opts(sweep=1, colours=65))
    P.close()


def test_wavefront_colours_solve_pure_advection_in_one_sweep():
    # as many colours as diagonal planes (3 + 3 + 2 - 2 = 6): the colour
    # order is the downwind wavefront order for b > 0, and one SOR sweep
    # with (nearly) exact block solves solves the upwind system (Sec. 4.3)
    from paper_1805_11930_amd import DG_INNER_GMRES, DG_SWEEP_SOR, smooth_opts

    w = inputs.pe2000(b=(1.0, 0.5, 0.3), p=2, cells=(3, 3, 2))
    w.K = 1e-13
    opr = oracle_problem(w)
    A = dg.assemble(opr)
    f = inputs.random_vector(opr.ndof, 47)
    u0 = inputs.random_vector(opr.ndof, 48)
    ue = spla.spsolve(A.tocsc(), f)
    P = _lib(w)
    o = smooth_opts(n_sweeps=1, omega=1.0, eps=1e-14, inner=DG_INNER_GMRES, restart=16, max_inner=400,
                    sweep=DG_SWEEP_SOR, colours=6)
    got = P.block_smooth(torch.from_numpy(f).cuda(), torch.from_numpy(u0).cuda(), o).cpu().numpy()
    assert rel(got, ue) <= 1e-9
    o.colours = 2
    rb = P.block_smooth(torch.from_numpy(f).cuda(), torch.from_numpy(u0).cuda(), o).cpu().numpy()
    assert rel(rb, ue) > 1e-3
    P.close()
