"""GPU parity of the Gauss-Lobatto basis (the paper's basis, Sec. 2.1)
against the oracle assembled directly in that basis, through the C ABI.

The library runs the GLL operators as S -> Gauss-point kernels -> S^T
(S = V (x) V (x) V per cell) and the block solves with S inside the inner
iteration; the oracle assembles A', D_T' and l' from the GLL tables.

  * node points are the GLL points; quadrature points the Gauss points;
  * apply, block apply and block diagonal: FP64 <= 1e-12, FP32 <= 1e-5,
    p = 1-5, with and without advection, mixed boundaries;
  * right-hand side: <= 1e-13;
  * inner PCG / GMRES (diagonal and tridiagonal M) at eps = 1e-2 replay the
    oracle's steps on D_T' (equal per-cell counts, iterates <= 1e-9);
  * block-Jacobi and block-SOR / SSOR sweeps and the P0 V-cycle with the
    exact coarse solve match the oracle's algorithms on A' to 1e-9;
  * coefficient fields (axis-aligned and rotated K(x), c(x)): apply and
    right-hand side with the field, V-cycle with the cell-centre problem;
  * a solve in the GLL basis reaches the sparse direct solution, and S u'
    equals the Gauss-basis solution of the same problem.
"""
import dataclasses

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import basis, dg, solvers
from paper_1805_11930_amd import inputs
from tests.helpers import oracle_problem, rel, spec

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")


def _lib(w, b="gll"):
    from paper_1805_11930_amd import Problem

    return Problem(dataclasses.replace(spec(w), basis=b))


def _setup(p, with_b, cells=(5, 3, 4), seed=0):
    w = inputs.random_case(p, cells=cells, seed=seed, with_b=with_b)
    opr = oracle_problem(w, basis="gll")
    A = dg.assemble(opr)
    Db = dg.block_diagonal(A, opr.ncell)
    return w, opr, A, Db


def _t(x, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype).cuda()


@pytest.mark.parametrize("p,with_b", [(1, True), (2, False), (3, True), (4, False), (4, True), (5, False)])
def test_apply_block_apply_diag(p, with_b):
    print(f"GLL apply p={p} b={with_b}", flush=True)
    w, opr, A, Db = _setup(p, with_b, cells=(4, 3, 3), seed=p)
    P = _lib(w)
    assert np.allclose(P.node_points(), dg.node_points(opr), atol=1e-14)
    xl = basis.gauss_legendre(p + 1)[0]
    assert np.allclose(P.quadrature_points()[: p + 1, 0] / opr.h[0], xl, atol=1e-14)
    u = inputs.random_vector(opr.ndof, 11)
    ref = A @ u
    assert rel(P.apply(_t(u)).cpu().numpy(), ref) <= 1e-12
    assert rel(P.apply(_t(u, torch.float32)).cpu().numpy().astype(np.float64), ref) <= 1e-5
    U = u.reshape(opr.ncell, -1)
    bref = np.concatenate([Db[T] @ U[T] for T in range(opr.ncell)])
    assert rel(P.block_apply(_t(u)).cpu().numpy(), bref) <= 1e-12
    assert rel(P.block_apply(_t(u, torch.float32)).cpu().numpy().astype(np.float64), bref) <= 1e-5
    dref = np.concatenate([np.diag(Db[T]) for T in range(opr.ncell)])
    assert rel(P.block_diag().cpu().numpy(), dref) <= 1e-12
    assert rel(P.block_diag(torch.float32).cpu().numpy().astype(np.float64), dref) <= 1e-6
    P.close()


@pytest.mark.parametrize("p", [2, 3])
def test_rhs(p):
    print(f"GLL rhs p={p}", flush=True)
    w = inputs.random_case(p, cells=(4, 3, 3), seed=3, with_b=True)
    opr = oracle_problem(w, basis="gll")

    def f(x):
        return np.sin(2 * x[:, 0]) + x[:, 1] * x[:, 2]

    def g(x):
        return np.cos(x[:, 0] + x[:, 1]) - x[:, 2]

    def j(x):
        return 0.3 + x[:, 0] * x[:, 1]

    ref = dg.assemble_rhs(opr, f=f, g=g, j=j)
    P = _lib(w)
    got = P.rhs_from_functions(f=f, g=g, j=j)
    assert rel(got.cpu().numpy(), ref) <= 1e-13
    P.close()


@pytest.mark.parametrize("p,with_b", [(1, False), (2, True), (3, False), (4, True)])
def test_block_pcg_replay(p, with_b):
    from paper_1805_11930_amd import DG_INNER_CG, smooth_opts

    print(f"GLL block PCG replay p={p} b={with_b}", flush=True)
    w, opr, A, Db = _setup(p, with_b, seed=4)
    d = inputs.random_vector(opr.ndof, 32)
    D = d.reshape(opr.ncell, -1)
    ref, its = [], []
    for T in range(opr.ncell):
        x, it = solvers.block_pcg(Db[T], D[T], 1e-2, opr.nloc)
        ref.append(x)
        its.append(it)
    P = _lib(w)
    x, it_gpu = P.block_solve(_t(d), smooth_opts(eps=1e-2, inner=DG_INNER_CG), iters=True)
    assert list(it_gpu.cpu().numpy()) == its
    xg = x.cpu().numpy().reshape(opr.ncell, -1)
    for T in range(opr.ncell):
        assert rel(xg[T], ref[T]) <= 1e-9
    # tight: the dense block solve
    xt = P.block_solve(_t(d), smooth_opts(eps=1e-14, max_inner=10 * opr.nloc, inner=DG_INNER_CG))
    dense = np.concatenate([np.linalg.solve(Db[T], D[T]) for T in range(opr.ncell)])
    assert rel(xt.cpu().numpy(), dense) <= 1e-10
    # FP32 meets the tolerance on every block
    x32, it32 = P.block_solve(_t(d, torch.float32), smooth_opts(eps=1e-2, inner=DG_INNER_CG), iters=True)
    x32 = x32.cpu().numpy().astype(np.float64).reshape(opr.ncell, -1)
    for T in range(opr.ncell):
        assert np.linalg.norm(D[T] - Db[T] @ x32[T]) <= 1.01e-2 * np.linalg.norm(D[T])
    assert np.abs(it32.cpu().numpy() - np.array(its)).max() <= 1
    P.close()


@pytest.mark.parametrize("p,tri,restart", [(2, False, 12), (3, True, 12), (4, True, 12), (3, True, 8), (2, False, 8)])
def test_block_gmres_replay(p, tri, restart):
    from paper_1805_11930_amd import DG_INNER_GMRES, DG_IPREC_DIAG, DG_IPREC_TRIDIAG, smooth_opts

    print(f"GLL block GMRES replay p={p} tridiag={tri} restart={restart}", flush=True)
    w, opr, A, Db = _setup(p, True, seed=5)
    d = inputs.random_vector(opr.ndof, 33)
    D = d.reshape(opr.ncell, -1)
    prec = "tridiag" if tri else "diag"
    ref, its = [], []
    for T in range(opr.ncell):
        x, it = solvers.block_gmres(Db[T], D[T], 1e-2, opr.nloc, min(restart, opr.nloc), precond=prec)
        ref.append(x)
        its.append(it)
    P = _lib(w)
    o = smooth_opts(eps=1e-2, inner=DG_INNER_GMRES, restart=restart,
                    inner_precond=DG_IPREC_TRIDIAG if tri else DG_IPREC_DIAG)
    x, it_gpu = P.block_solve(_t(d), o, iters=True)
    assert list(it_gpu.cpu().numpy()) == its
    xg = x.cpu().numpy().reshape(opr.ncell, -1)
    for T in range(opr.ncell):
        assert rel(xg[T], ref[T]) <= 1e-9
    P.close()


@pytest.mark.parametrize("p,with_b,kind", [(2, False, "jacobi"), (3, True, "jacobi"), (2, True, "ssor"),
                                           (3, False, "sor"), (4, False, "back")])
def test_sweeps(p, with_b, kind):
    from paper_1805_11930_amd import DG_INNER_CG, DG_INNER_GMRES, smooth_opts

    print(f"GLL sweeps {kind} p={p} b={with_b}", flush=True)
    w, opr, A, Db = _setup(p, with_b, cells=(5, 4, 3), seed=6)
    f = inputs.random_vector(opr.ndof, 34)
    u0 = inputs.random_vector(opr.ndof, 35)
    inner = "gmres" if with_b else "cg"
    kw = dict(omega=0.9, inner=inner, eps=1e-2, restart=12)
    sweep = {"jacobi": 0, "sor": 1, "ssor": 2, "back": 3}[kind]

    def oracle(u, n):
        if kind == "jacobi":
            return solvers.block_jacobi(A, Db, f, u, nsweeps=n, **kw)
        order = solvers.multicolour_order(opr, 2)
        if kind == "ssor":
            return solvers.block_ssor(A, Db, f, u, order, nsweeps=n, **kw)
        return solvers.block_sor(A, Db, f, u, order[::-1] if kind == "back" else order, nsweeps=n, **kw)

    P = _lib(w)
    o = smooth_opts(n_sweeps=2, omega=0.9, eps=1e-2, inner=DG_INNER_GMRES if with_b else DG_INNER_CG, restart=12,
                    sweep=sweep)
    got = P.block_smooth(_t(f), _t(u0), o)
    assert rel(got.cpu().numpy(), oracle(u0, 2)) <= 1e-9
    o.n_sweeps = 1
    got0 = P.block_smooth(_t(f), None, o)
    assert rel(got0.cpu().numpy(), oracle(np.zeros_like(f), 1)) <= 1e-9
    P.close()


@pytest.mark.parametrize("p,with_b,npre,npost", [(2, False, 1, 1), (3, True, 2, 1), (4, False, 1, 2)])
def test_vcycle_exact_coarse(p, with_b, npre, npost):
    from paper_1805_11930_amd import DG_COARSE_AUTO, DG_INNER_CG, DG_INNER_GMRES, mg_opts

    print(f"GLL V-cycle p={p} b={with_b}", flush=True)
    w, opr, A, Db = _setup(p, with_b, cells=(5, 4, 3), seed=7)
    r = inputs.random_vector(opr.ndof, 36)
    inner = "gmres" if with_b else "cg"
    cs = solvers.exact_coarse(solvers.p0_galerkin(A, opr))
    ref = solvers.vcycle(A, Db, opr, r, cs, n_pre=npre, n_post=npost, omega=0.9, inner=inner, eps=1e-2, restart=12)
    P = _lib(w)
    # AUTO selects P0 in the GLL basis
    o = mg_opts(smooth=dict(omega=0.9, eps=1e-2, inner=DG_INNER_GMRES if with_b else DG_INNER_CG, restart=12),
                n_pre=npre, n_post=npost, coarse_space=DG_COARSE_AUTO)
    z = P.mg_vcycle(_t(r), o)
    assert rel(z.cpu().numpy(), ref) <= 1e-9
    z32 = P.mg_vcycle(_t(r, torch.float32), o)
    assert rel(z32.cpu().numpy().astype(np.float64), ref) <= 1e-3
    P.close()


@pytest.mark.parametrize("p,rotated", [(2, False), (3, True)])
def test_field_apply_rhs_and_vcycle(p, rotated):
    """Coefficient fields (Sec. 4.2): the outer operator with K(x), c(x) at
    the quadrature points, the preconditioner with their cell-centre values,
    in the GLL basis."""
    from paper_1805_11930_amd import DG_COARSE_P0, DG_INNER_CG, mg_opts

    print(f"GLL field p={p} rotated={rotated}", flush=True)
    nrot = inputs.rotation(0.4, -0.7, 1.1) if rotated else None
    w = inputs.inhomogeneous(p=p, cells=(4, 3, 5), kfield=((1.0, 0.5, 2.0), (0.4, -0.2, 0.3), (3.0, 1.0, 0.5)),
                             nrot=nrot)
    w.cfield = (0.3, 0.7)
    opr = oracle_problem(w, basis="gll")
    A = dg.assemble(opr)
    P = _lib(w)
    u = inputs.random_vector(opr.ndof, 12)
    assert rel(P.apply(_t(u)).cpu().numpy(), A @ u) <= 1e-12
    ref = dg.assemble_rhs(opr, f=w.f, g=w.g, j=w.j)
    assert rel(P.rhs_from_functions(f=w.f, g=w.g, j=w.j).cpu().numpy(), ref) <= 1e-12
    # the V-cycle works with the cell-centre problem
    cc = dg.cell_centre_problem(opr)
    Acc = dg.assemble(cc)
    Dcc = dg.block_diagonal(Acc, cc.ncell)
    r = inputs.random_vector(opr.ndof, 38)
    cs = solvers.exact_coarse(solvers.p0_galerkin(Acc, cc))
    zref = solvers.vcycle(Acc, Dcc, cc, r, cs, n_pre=1, n_post=1, omega=0.9, inner="cg", eps=1e-2)
    z = P.mg_vcycle(_t(r), mg_opts(smooth=dict(omega=0.9, eps=1e-2, inner=DG_INNER_CG), coarse_space=DG_COARSE_P0))
    assert rel(z.cpu().numpy(), zref) <= 1e-9
    P.close()


def test_unsupported_options_fail():
    from paper_1805_11930_amd import DG_COARSE_Q1, DG_INNER_FDM, DG_INNER_PMF, DgError, mg_opts, smooth_opts

    w, opr, A, Db = _setup(2, False, cells=(3, 3, 3), seed=8)
    P = _lib(w)
    r = _t(inputs.random_vector(opr.ndof, 37))
    for inner in (DG_INNER_FDM, DG_INNER_PMF):
        with pytest.raises(DgError):
            P.block_solve(r, smooth_opts(inner=inner))
    with pytest.raises(DgError):
        P.mg_vcycle(r, mg_opts(coarse_space=DG_COARSE_Q1))
    P.close()


@pytest.mark.parametrize("p", [2, 3])
def test_solve_matches_gauss_basis(p):
    from paper_1805_11930_amd import DG_FP32, DG_KRYLOV_FCG, DG_PRECOND_MG, solve_opts

    print(f"GLL solve p={p}", flush=True)
    w = inputs.w1(cells=(6, 6, 6))
    w = dataclasses.replace(w, p=p, sigma=None)
    opr = oracle_problem(w, basis="gll")
    A = dg.assemble(opr)
    rhs = dg.assemble_rhs(opr, f=w.f)
    ref = spla.spsolve(A.tocsc(), rhs)
    o = solve_opts(krylov=DG_KRYLOV_FCG, precond=DG_PRECOND_MG, precond_precision=DG_FP32, rtol=1e-10, maxit=200,
                   smooth=dict(eps=1e-2))
    P = _lib(w)
    f = P.rhs_from_functions(f=w.f)
    assert rel(f.cpu().numpy(), rhs) <= 1e-13
    u, res = P.solve(f, opts=o)
    assert res.status == 0 and res.rel_residual <= 1e-10
    assert rel(u.cpu().numpy(), ref) <= 1e-8
    # the same function as the Gauss-basis solution: S u' = u
    G = _lib(w, "gl")
    ug, resg = G.solve(G.rhs_from_functions(f=w.f), opts=o)
    n = p + 1
    V = basis.lagrange_values(basis.gauss_lobatto(n)[0], basis.gauss_legendre(n)[0])
    ST = np.kron(V, np.kron(V, V))
    Su = (u.cpu().numpy().reshape(-1, n**3) @ ST.T).ravel()
    assert rel(Su, ug.cpu().numpy()) <= 1e-8
    print(f"  outer iterations GLL {res.iters}, GL {resg.iters}", flush=True)
    P.close()
    G.close()
