"""Pins of the oracle's smoothers, coarse space, V-cycle and outer solvers,
and of the memory model (CPU only).

  * inner PCG / GMRES with a tiny eps reproduce the dense block solve
    (brute force), PCG on a diagonal block needs exactly one iteration,
    restarted GMRES still converges;
  * one exact block-Jacobi sweep on a one-cell mesh solves A u = f (A = D),
    and the exact solution is a fixed point of the sweep (alg block_jacobi);
  * the hybrid V-cycle (alg hybrid_multigrid) with exact block solves,
    n_pre = n_post and an exact coarse solve is a symmetric positive
    definite operator for b = 0;
  * outer CG / flexible CG / flexible GMRES converge to the sparse direct
    solution within the tolerance;
  * block-SOR / block-SSOR sweeps (alg block_SOR) equal the matrix
    splitting iterations u + W^-1 (f - A u) with the paper's W for SOR and
    SSOR, computed globally from dense D, L, U for the same cell order;
    red-black results do not depend on the order inside a colour; with
    (almost) no diffusion and cells ordered along b one SOR sweep solves the
    upwind system (Sec. 4.3), a red-black one does not; SSOR from zero and
    the SOR/SSOR V-cycles are symmetric for b = 0; tight inner solves
    reproduce the exact sweeps;
  * the Thomas algorithm solves tridiagonal systems (dense solve); the
    tridiagonal part of a DG cell block splits into one system per x-line,
    and GMRES preconditioned with it converges in one step on that part;
    at Pe = 2000 and eps = 1e-2 the tridiagonally preconditioned block
    GMRES needs about four iterations for b = (1,0,0) at p = 2-4 and more
    for b = (1, 0.5, 0.3), fewer than with the diagonal (Sec. 4.3);
  * the memory model reproduces every printed entry of the paper's four
    memory tables (tests/golden/*.csv, Sec. 4.4).
"""
import csv
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import dg, memory_model as mm, solvers

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def read_golden(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return list(csv.DictReader(line for line in fh if not line.startswith("#")))


def small(p=2, with_b=False, seed=0, cells=(3, 3, 2), **kw):
    rng = np.random.default_rng(seed)
    nc = int(np.prod(cells))
    extra = {}
    if with_b:
        extra = dict(b0=(0.6, -0.4, 0.3), B=((0.0, 1.0, 0.0), (-1.0, 0.0, 0.0), (0.0, 0.0, 0.0)))
    extra.update(kw)
    return dg.Problem(cells=cells, p=p, K=np.exp(rng.normal(size=(nc, 3))), **extra)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_block_pcg_tight_equals_dense(p):
    pr = small(p)
    A = dg.assemble(pr)
    Db = dg.block_diagonal(A, pr.ncell)
    rng = np.random.default_rng(1)
    for T in range(pr.ncell):
        d = rng.normal(size=pr.nloc)
        x, it = solvers.block_pcg(Db[T], d, 1e-14, 10 * pr.nloc)
        xe, _ = solvers.block_solve_exact(Db[T], d)
        assert np.linalg.norm(x - xe) <= 1e-11 * np.linalg.norm(xe)
        assert 1 <= it <= 10 * pr.nloc


def test_block_pcg_diagonal_one_iteration():
    D = np.diag(np.arange(1.0, 9.0))
    d = np.linspace(-1, 2, 8)
    x, it = solvers.block_pcg(D, d, 1e-12, 8)
    assert it == 1
    np.testing.assert_allclose(x, d / np.diag(D), rtol=1e-15)
    x0, it0 = solvers.block_pcg(D, np.zeros(8), 1e-2, 8)
    assert it0 == 0 and not x0.any()


@pytest.mark.parametrize("restart", [4, 30])
def test_block_gmres_tight_equals_dense(restart):
    pr = small(2, with_b=True)
    A = dg.assemble(pr)
    Db = dg.block_diagonal(A, pr.ncell)
    assert np.abs(Db[0] - Db[0].T).max() > 1e-3  # really nonsymmetric
    rng = np.random.default_rng(2)
    for T in range(pr.ncell):
        d = rng.normal(size=pr.nloc)
        x, it = solvers.block_gmres(Db[T], d, 1e-13, 20 * pr.nloc, restart)
        xe, _ = solvers.block_solve_exact(Db[T], d)
        assert np.linalg.norm(x - xe) <= 1e-10 * np.linalg.norm(xe)


def test_block_gmres_loose_tolerance_is_met():
    pr = small(3, with_b=True)
    A = dg.assemble(pr)
    Db = dg.block_diagonal(A, pr.ncell)
    rng = np.random.default_rng(3)
    for T in range(pr.ncell):
        d = rng.normal(size=pr.nloc)
        x, it = solvers.block_gmres(Db[T], d, 1e-2, pr.nloc, 30)
        assert np.linalg.norm(d - Db[T] @ x) <= 1e-2 * np.linalg.norm(d) * (1 + 1e-10)


def test_block_jacobi_single_cell_exact():
    pr = small(2, cells=(1, 1, 1))
    A = dg.assemble(pr)
    Db = dg.block_diagonal(A, pr.ncell)
    f = np.random.default_rng(4).normal(size=pr.ndof)
    u = solvers.block_jacobi(A, Db, f, np.zeros(pr.ndof), omega=1.0, nsweeps=1, inner="exact")
    np.testing.assert_allclose(A @ u, f, rtol=0, atol=1e-12 * np.abs(f).max())


def test_block_jacobi_fixed_point_and_damping():
    pr = small(2)
    A = dg.assemble(pr)
    Db = dg.block_diagonal(A, pr.ncell)
    rng = np.random.default_rng(5)
    ue = rng.normal(size=pr.ndof)
    f = A @ ue
    u = solvers.block_jacobi(A, Db, f, ue, omega=0.7, nsweeps=2, inner="exact")
    np.testing.assert_allclose(u, ue, rtol=1e-12, atol=1e-12)
    # one damped sweep from zero: u = omega D^-1 f, cell by cell
    u1 = solvers.block_jacobi(A, Db, f, np.zeros(pr.ndof), omega=0.7, nsweeps=1, inner="exact")
    F = f.reshape(pr.ncell, -1)
    expect = np.concatenate([0.7 * np.linalg.solve(Db[T], F[T]) for T in range(pr.ncell)])
    np.testing.assert_allclose(u1, expect, rtol=1e-12, atol=1e-13)


def test_vcycle_symmetric_positive_definite():
    pr = small(2, cells=(3, 2, 2))
    A = dg.assemble(pr)
    Db = dg.block_diagonal(A, pr.ncell)
    Ah = solvers.p0_direct(pr)
    cs = solvers.exact_coarse(Ah)
    rng = np.random.default_rng(6)
    r1, r2 = rng.normal(size=(2, pr.ndof))
    kw = dict(n_pre=1, n_post=1, omega=0.8, inner="exact")
    z1 = solvers.vcycle(A, Db, pr, r1, cs, **kw)
    z2 = solvers.vcycle(A, Db, pr, r2, cs, **kw)
    assert r2 @ z1 == pytest.approx(r1 @ z2, rel=1e-11)
    assert r1 @ z1 > 0 and r2 @ z2 > 0
    # linearity
    z12 = solvers.vcycle(A, Db, pr, r1 + 2 * r2, cs, **kw)
    np.testing.assert_allclose(z12, z1 + 2 * z2, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("flexible", [False, True])
def test_outer_cg_with_vcycle(flexible):
    pr = small(2, cells=(4, 3, 3))
    A = dg.assemble(pr)
    Db = dg.block_diagonal(A, pr.ncell)
    cs = solvers.exact_coarse(solvers.p0_direct(pr))
    f = np.random.default_rng(7).normal(size=pr.ndof)
    ue = spla.spsolve(A.tocsc(), f)
    it_stats = []

    def M(r):
        return solvers.vcycle(A, Db, pr, r, cs, inner="cg", eps=1e-2, stats=it_stats)

    x, it, hist = solvers.cg(A, f, precond=M, rtol=1e-10, maxit=200, flexible=flexible)
    assert hist[-1] <= 1e-10
    assert np.linalg.norm(f - A @ x) <= 1e-10 * np.linalg.norm(f) * (1 + 1e-6)
    assert np.linalg.norm(x - ue) <= 1e-7 * np.linalg.norm(ue)
    assert it < 60
    assert max(it_stats) <= pr.nloc


def test_outer_fgmres_with_vcycle_convection():
    pr = small(2, with_b=True, cells=(4, 3, 3))
    A = dg.assemble(pr)
    Db = dg.block_diagonal(A, pr.ncell)
    cs = solvers.exact_coarse(solvers.p0_direct(pr))
    f = np.random.default_rng(8).normal(size=pr.ndof)
    ue = spla.spsolve(A.tocsc(), f)

    def M(r):
        return solvers.vcycle(A, Db, pr, r, cs, inner="gmres", eps=1e-2)

    for restart in (5, 30):
        x, it, hist = solvers.fgmres(A, f, precond=M, rtol=1e-10, maxit=300, restart=restart)
        assert np.linalg.norm(f - A @ x) <= 1.01e-10 * np.linalg.norm(f)
        assert np.linalg.norm(x - ue) <= 1e-7 * np.linalg.norm(ue)


def test_unpreconditioned_cg_matches_dense():
    pr = small(1, cells=(2, 2, 2))
    A = dg.assemble(pr)
    f = np.random.default_rng(9).normal(size=pr.ndof)
    x, it, hist = solvers.cg(A, f, rtol=1e-12, maxit=2000)
    np.testing.assert_allclose(x, np.linalg.solve(A.toarray(), f), rtol=1e-8, atol=1e-10)


# ---------------------------------------------------------------------------
# memory model vs the paper's printed tables
# ---------------------------------------------------------------------------
def _grids():
    return {int(r["p"]): (int(r["nx"]) * int(r["ny"]) * int(r["nz"]), r) for r in read_golden("problem_sizes.csv")}


def test_problem_size_table():
    for p, (nc, r) in _grids().items():
        assert round(mm.matrix_doubles(p, nc) * 8 / 2**30, 1) == float(r["matrix_gib"])
        assert round(mm.vector_doubles(p, nc) / 1e6, 1) == float(r["dofs_1e6"])
        assert mm.matrix_doubles(p, nc) // mm.vector_doubles(p, nc) == int(r["ratio"])
        assert (p + 1) ** 3 == int(r["dofs_per_cell"])


@pytest.mark.parametrize(
    "fname,fun,unit",
    [
        ("memory_diffusion.csv", mm.diffusion_doubles, 1e9),
        ("memory_convection_restart100.csv", lambda p, nc: mm.convection_doubles(p, nc, 100, 100), 2**30),
        ("memory_convection_restart15_12.csv", lambda p, nc: mm.convection_doubles(p, nc, 15, 12), 2**30),
    ],
)
def test_memory_tables(fname, fun, unit):
    grids = _grids()
    for r in read_golden(fname):
        p = int(r["p"])
        t = fun(p, grids[p][0])
        mx, pmf, mf = (t[k] * 8 / unit for k in ("MX", "PMF", "MF"))
        assert round(mx, 1) == float(r["mx_gb"])
        assert round(pmf, 1) == float(r["pmf_gb"])
        assert round(mx / pmf, 1) == float(r["pmf_ratio"])
        assert round(mf, 3) == float(r["mf_gb"])
        assert round(mx / mf, 1) == float(r["mf_ratio"])


# ---------------------------------------------------------------------------
# Q1 subspace (App. A.2)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("with_b", [False, True])
def test_q1_galerkin_equals_direct(with_b):
    """P^T A P on the conforming Q1 subspace equals the direct evaluation of
    a_h on the trilinear functions: volume terms plus Dirichlet-face terms
    only, the interior jump terms vanishing (App. A.2)."""
    kw = {}
    if with_b:
        kw = dict(b0=(0.3, -0.7, 0.2), B=((0.5, 1.0, 0.0), (-1.0, -0.2, 0.5), (0.3, 0.0, -0.3)))
    pr = small(2, cells=(3, 2, 2), seed=9, bc=("D", "N", "D", "D", "N", "D"), c=0.7, **kw)
    A = dg.assemble(pr)
    G = solvers.q1_galerkin(A, pr)
    D = solvers.q1_direct(pr)
    assert np.abs(G - D).max() <= 1e-12 * np.abs(G).max()


def test_q1_prolongation_reproduces_trilinear():
    """P applied to the vertex values of a global trilinear function gives
    its nodal interpolant (Q1 is a subspace of V_h^p)."""
    pr = small(3, cells=(3, 2, 4))
    nx, ny, nz = pr.cells
    h = pr.h
    coef = np.random.default_rng(3).normal(size=8)

    def f(x):
        X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
        return (coef[0] + coef[1] * X + coef[2] * Y + coef[3] * Z + coef[4] * X * Y + coef[5] * Y * Z
                + coef[6] * X * Z + coef[7] * X * Y * Z)

    V = np.array([[vx * h[0], vy * h[1], vz * h[2]] for vz in range(nz + 1) for vy in range(ny + 1)
                  for vx in range(nx + 1)])
    P = solvers.q1_prolongation(pr)
    np.testing.assert_allclose(P @ f(V), dg.interpolate(pr, f), rtol=1e-13, atol=1e-13)


def test_vcycle_q1_symmetric():
    pr = small(2, cells=(3, 2, 2))
    A = dg.assemble(pr)
    Db = dg.block_diagonal(A, pr.ncell)
    P = solvers.q1_prolongation(pr)
    cs = solvers.exact_coarse(solvers.q1_direct(pr))
    rng = np.random.default_rng(6)
    r1, r2 = rng.normal(size=(2, pr.ndof))
    kw = dict(n_pre=1, n_post=1, omega=0.7, inner="exact", P=P)
    z1 = solvers.vcycle(A, Db, pr, r1, cs, **kw)
    z2 = solvers.vcycle(A, Db, pr, r2, cs, **kw)
    assert r2 @ z1 == pytest.approx(r1 @ z2, rel=1e-11)
    assert r1 @ z1 > 0


# ---------------------------------------------------------------------------
# block-SOR / block-SSOR (alg block_SOR, Sec. 2.2.1)
# ---------------------------------------------------------------------------
def _splitting(A, pr, order):
    """Dense D, L, U of A for the cell order: L holds the blocks A_{rho,sigma}
    with sigma visited before rho, U those visited after."""
    Ad = A.toarray()
    nb = pr.nloc
    pos = np.empty(pr.ncell, dtype=int)
    pos[np.asarray(order)] = np.arange(pr.ncell)
    cell = np.arange(pr.ndof) // nb
    before = pos[cell][None, :] < pos[cell][:, None]
    same = cell[None, :] == cell[:, None]
    return Ad * same, Ad * before, Ad * ~(before | same)


@pytest.mark.parametrize("with_b", [False, True])
@pytest.mark.parametrize("omega", [1.0, 1.3])
@pytest.mark.parametrize("ordering", ["lex", "rb"])
def test_block_sor_is_the_splitting_iteration(with_b, omega, ordering):
    # one sweep is u + W^-1 (f - A u) with W = omega^-1 D + L (Sec. 2.2.1)
    pr = small(2, with_b=with_b, cells=(3, 2, 2))
    A = dg.assemble(pr)
    Db = dg.block_diagonal(A, pr.ncell)
    order = solvers.lexicographic_order(pr) if ordering == "lex" else solvers.multicolour_order(pr)
    rng = np.random.default_rng(11)
    f, u0 = rng.normal(size=(2, pr.ndof))
    D, L, _ = _splitting(A, pr, order)
    W = D / omega + L
    expect = u0 + np.linalg.solve(W, f - A @ u0)
    got = solvers.block_sor(A, Db, f, u0, order, omega=omega, nsweeps=1)
    np.testing.assert_allclose(got, expect, rtol=0, atol=1e-11 * np.abs(expect).max())


@pytest.mark.parametrize("with_b", [False, True])
def test_block_ssor_is_the_splitting_iteration(with_b):
    # W = (omega (2 - omega))^-1 (D + omega L) D^-1 (D + omega U) (Sec. 2.2.1)
    omega = 1.2
    pr = small(1, with_b=with_b, cells=(3, 3, 2))
    A = dg.assemble(pr)
    Db = dg.block_diagonal(A, pr.ncell)
    order = solvers.multicolour_order(pr)
    rng = np.random.default_rng(12)
    f, u0 = rng.normal(size=(2, pr.ndof))
    D, L, U = _splitting(A, pr, order)
    W = (D + omega * L) @ np.linalg.solve(D, D + omega * U) / (omega * (2.0 - omega))
    expect = u0 + np.linalg.solve(W, f - A @ u0)
    got = solvers.block_ssor(A, Db, f, u0, order, omega=omega, nsweeps=1)
    np.testing.assert_allclose(got, expect, rtol=0, atol=1e-11 * np.abs(expect).max())


@pytest.mark.parametrize("C", [2, 3, 5])
def test_multicolour_order_is_independent_within_a_colour(C):
    pr = small(2, with_b=True, cells=(4, 3, 3))
    A = dg.assemble(pr)
    Db = dg.block_diagonal(A, pr.ncell)
    order = solvers.multicolour_order(pr, C)
    ijk = np.array([pr.cell_ijk(c) for c in order])
    colour = ijk.sum(axis=1) % C
    assert np.all(colour[:-1] <= colour[1:])  # one colour after the other
    assert sorted(order) == list(range(pr.ncell))
    # no two cells of one colour share a face
    for c in range(pr.ncell):
        for d in range(pr.ncell):
            if np.abs(np.subtract(pr.cell_ijk(c), pr.cell_ijk(d))).sum() == 1:
                assert sum(pr.cell_ijk(c)) % C != sum(pr.cell_ijk(d)) % C
    rng = np.random.default_rng(13)
    f, u0 = rng.normal(size=(2, pr.ndof))
    shuffled = np.concatenate([rng.permutation(order[colour == q]) for q in range(C)])
    a = solvers.block_ssor(A, Db, f, u0, order, omega=1.1)
    b = solvers.block_ssor(A, Db, f, u0, shuffled, omega=1.1)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-12 * np.abs(a).max())


def test_block_sor_pure_advection_downwind_one_sweep_is_exact():
    # Pe -> infinity: with the cells ordered along b, one sweep with
    # omega = 1 solves the upwind system exactly (Sec. 4.3); K = 1e-13
    # leaves couplings against the flow of relative size ~1e-13
    pr = dg.Problem(cells=(3, 3, 2), p=2, K=1e-13, b0=(1.0, 0.5, 0.3))
    A = dg.assemble(pr)
    Db = dg.block_diagonal(A, pr.ncell)
    rng = np.random.default_rng(14)
    f, u0 = rng.normal(size=(2, pr.ndof))
    ue = spla.spsolve(A.tocsc(), f)
    u = solvers.block_sor(A, Db, f, u0, solvers.lexicographic_order(pr), omega=1.0)
    np.testing.assert_allclose(u, ue, rtol=0, atol=1e-9 * np.abs(ue).max())
    # red-black is not a downwind order: one sweep is not exact
    u_rb = solvers.block_sor(A, Db, f, u0, solvers.multicolour_order(pr), omega=1.0)
    assert np.abs(u_rb - ue).max() > 1e-3 * np.abs(ue).max()
    # as many colours as diagonal planes (3 + 3 + 2 - 2 = 6): the colour
    # order is the wavefront order, downwind for b > 0, and one sweep is
    # exact again
    u_hp = solvers.block_sor(A, Db, f, u0, solvers.multicolour_order(pr, 6), omega=1.0)
    np.testing.assert_allclose(u_hp, ue, rtol=0, atol=1e-9 * np.abs(ue).max())


def test_block_ssor_from_zero_is_symmetric_positive_definite():
    pr = small(2, cells=(3, 2, 2))
    A = dg.assemble(pr)
    Db = dg.block_diagonal(A, pr.ncell)
    order = solvers.multicolour_order(pr)
    rng = np.random.default_rng(15)
    r1, r2 = rng.normal(size=(2, pr.ndof))
    z = lambda r: solvers.block_ssor(A, Db, r, np.zeros(pr.ndof), order, omega=1.3)
    z1, z2 = z(r1), z(r2)
    assert r2 @ z1 == pytest.approx(r1 @ z2, rel=1e-11)
    assert r1 @ z1 > 0 and r2 @ z2 > 0


@pytest.mark.parametrize("smoother", ["sor", "ssor"])
def test_vcycle_sor_smoothers_symmetric(smoother):
    pr = small(2, cells=(3, 2, 2))
    A = dg.assemble(pr)
    Db = dg.block_diagonal(A, pr.ncell)
    cs = solvers.exact_coarse(solvers.p0_direct(pr))
    rng = np.random.default_rng(16)
    r1, r2 = rng.normal(size=(2, pr.ndof))
    kw = dict(n_pre=1, n_post=1, omega=1.0, inner="exact", smoother=smoother)
    z1 = solvers.vcycle(A, Db, pr, r1, cs, **kw)
    z2 = solvers.vcycle(A, Db, pr, r2, cs, **kw)
    assert r2 @ z1 == pytest.approx(r1 @ z2, rel=1e-11)
    assert r1 @ z1 > 0


@pytest.mark.parametrize("inner,with_b", [("cg", False), ("gmres", True)])
def test_block_sor_tight_inner_equals_exact(inner, with_b):
    pr = small(2, with_b=with_b, cells=(3, 2, 2))
    A = dg.assemble(pr)
    Db = dg.block_diagonal(A, pr.ncell)
    order = solvers.multicolour_order(pr)
    rng = np.random.default_rng(17)
    f, u0 = rng.normal(size=(2, pr.ndof))
    a = solvers.block_ssor(A, Db, f, u0, order, omega=0.9, inner="exact")
    b = solvers.block_ssor(A, Db, f, u0, order, omega=0.9, inner=inner, eps=1e-14, max_inner=200, restart=27)
    np.testing.assert_allclose(b, a, rtol=0, atol=1e-10 * np.abs(a).max())


# ---------------------------------------------------------------------------
# tridiagonal (Thomas) inner preconditioner (Sec. 3.2, Sec. 4.3)
# ---------------------------------------------------------------------------
def test_thomas_solves_tridiagonal_systems():
    rng = np.random.default_rng(18)
    n = 11
    sub, sup = rng.normal(size=(2, n))
    sub[0] = sup[-1] = 0.0
    diag = 4.0 + rng.random(n)
    T = np.diag(diag) + np.diag(sub[1:], -1) + np.diag(sup[:-1], 1)
    v = rng.normal(size=n)
    np.testing.assert_allclose(solvers.thomas(sub, diag, sup, v), np.linalg.solve(T, v), rtol=1e-13, atol=1e-14)


def _pe2000_blocks(b, p, cells=(4, 4, 8)):
    from paper_1805_11930_amd import inputs

    w = inputs.pe2000(b=b, p=p, cells=cells)
    pr = dg.Problem(cells=w.cells, lengths=w.lengths, p=p, K=w.K, b0=w.b0)
    A = dg.assemble(pr)
    return pr, dg.block_diagonal(A, pr.ncell)


def test_tridiagonal_part_splits_into_x_lines():
    # with the x-fastest DOF order the entries between the last node of one
    # x-line and the first of the next vanish: the Thomas solve is one
    # independent tridiagonal solve per x-line
    pr, Db = _pe2000_blocks((1.0, 0.5, 0.3), 3)
    N = pr.n
    for T in (0, 17, pr.ncell - 1):
        ends = np.arange(N - 1, pr.nloc - 1, N)
        assert np.all(Db[T][ends, ends + 1] == 0.0) and np.all(Db[T][ends + 1, ends] == 0.0)
    # M = tridiagonal part of D: GMRES on M itself needs one iteration
    D = Db[5]
    M = np.diag(np.diag(D)) + np.diag(np.diag(D, -1), -1) + np.diag(np.diag(D, 1), 1)
    d = np.random.default_rng(19).normal(size=pr.nloc)
    x, it = solvers.block_gmres(M, d, 1e-12, 10, 10, "tridiag")
    assert it == 1
    np.testing.assert_allclose(M @ x, d, rtol=0, atol=1e-11 * np.abs(d).max())


def _mean_inner(Db, precond, step=5):
    rng = np.random.default_rng(20)
    its = [solvers.block_gmres(Db[T], rng.normal(size=Db.shape[1]), 1e-2, 200, 64, precond)[1]
           for T in range(0, Db.shape[0], step)]
    return float(np.mean(its))


def test_tridiagonal_preconditioner_iterations_as_reported():
    # Sec. 4.3: at Pe = 2000 and eps = 1e-2 the tridiagonally preconditioned
    # block GMRES needs about four iterations for b = (1,0,0), without a
    # strong dependence on p, and more for b = (1, 0.5, 0.3); the diagonal
    # preconditioner is worse
    for p in (2, 3, 4):
        _, Dx = _pe2000_blocks((1.0, 0.0, 0.0), p)
        _, Dxyz = _pe2000_blocks((1.0, 0.5, 0.3), p)
        tx, txyz = _mean_inner(Dx, "tridiag"), _mean_inner(Dxyz, "tridiag")
        assert 2.5 <= tx <= 5.5
        assert txyz > tx
        assert _mean_inner(Dx, "diag") > tx
