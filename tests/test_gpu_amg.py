"""The aggregation-AMG coarse solver (dg_mg_opts.coarse_solver =
DG_COARSE_SOLVER_AMG) through the C ABI:

  * its hierarchy is a Galerkin hierarchy: R_l = P_l^T exactly and
    A_l = R_l A_(l-1) P_l (checked with scipy on the downloaded CSR
    matrices), level 0 being the coarse-space matrix A_hat = P^T A P of the
    oracle (P0 and Q1, with and without advection);
  * the device V-cycle of the coarse solve equals a CPU replay of the same
    cycle (damped Jacobi, residual, restriction, dense bottom,
    prolongation) on those matrices: the DG V-cycle without smoothing is
    z = P_DG M_AMG(P_DG^T r), compared with the oracle's P_DG;
  * repeated AMG cycles converge to the exact coarse solution, and outer
    solves with the AMG coarse solver reach the tolerance.
"""
import numpy as np
import pytest
import scipy.sparse as sp
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


def _csr(P, space, level, which):
    rp, ci, v, shape, nlev = P.coarse_csr(space, level, which)
    return sp.csr_matrix((v, ci, rp), shape=shape), nlev


def _hierarchy(P, space):
    A0, nlev = _csr(P, space, 0, 0)
    levels = [(A0, None, None)]
    for l in range(1, nlev):
        Al, _ = _csr(P, space, l, 0)
        Pl, _ = _csr(P, space, l, 1)
        Rl, _ = _csr(P, space, l, 2)
        levels.append((Al, Pl, Rl))
    return levels


# coarse spaces of a few thousand unknowns: several AMG levels above the
# dense bottom (at most 1024 unknowns)
CASES = [
    ("q1", False, (16, 14, 15)),
    ("p0", False, (18, 16, 15)),
    ("p0", True, (18, 16, 15)),
]


def _case(space, with_b, cells):
    from paper_1805_11930_amd import DG_COARSE_P0, DG_COARSE_Q1, Problem

    w = inputs.random_case(1, cells=cells, seed=51, with_b=with_b, bc=("D",) * 6 if space == "q1" else
                           ("D", "N", "D", "D", "N", "D"))
    return w, Problem(spec(w)), DG_COARSE_Q1 if space == "q1" else DG_COARSE_P0


_ORACLE = {}


def _oracle(w, key):
    """The oracle problem and its assembled A (assembled once per case)."""
    if key not in _ORACLE:
        opr = oracle_problem(w)
        _ORACLE[key] = (opr, dg.assemble(opr))
    return _ORACLE[key]


def _ahat(opr, A, space):
    Pdg = solvers.q1_prolongation(opr) if space == "q1" else solvers.p0_prolongation(opr)
    return Pdg, sp.csr_matrix(Pdg.T @ (A.tocsr() @ Pdg))


@pytest.mark.parametrize("space,with_b,cells", CASES)
def test_amg_is_a_galerkin_hierarchy(space, with_b, cells):
    print(f"AMG hierarchy {space} b={with_b} cells={cells}", flush=True)
    w, P, cs = _case(space, with_b, cells)
    opr, A = _oracle(w, (space, with_b, cells))
    _, Ahat = _ahat(opr, A, space)
    levels = _hierarchy(P, cs)
    P.close()
    assert len(levels) >= 2
    A0 = levels[0][0]
    assert abs(A0 - Ahat).max() <= 1e-12 * abs(Ahat).max()
    for l in range(1, len(levels)):
        Al, Pl, Rl = levels[l]
        Af = levels[l - 1][0]
        assert Pl.shape == (Af.shape[0], Al.shape[0]) and Al.shape[0] < Af.shape[0]
        assert (Rl != Pl.T.tocsr()).nnz == 0
        G = Rl @ Af @ Pl
        assert abs(Al - G).max() <= 1e-12 * abs(G).max()
    assert levels[-1][0].shape[0] <= 1024


def _dinv(A, structured_p0):
    if structured_p0:
        return 1.0 / A.diagonal()
    return 2.0 / np.asarray(abs(A).sum(axis=1)).ravel()


def _cycle(levels, l, r, nu, w, p0_level0):
    A = levels[l][0]
    if l == len(levels) - 1:
        return np.linalg.solve(A.toarray(), r)
    d = _dinv(A, p0_level0 and l == 0)
    x = w * d * r
    for _ in range(nu - 1):
        x = x + w * d * (r - A @ x)
    Pn, Rn = levels[l + 1][1], levels[l + 1][2]
    xc = _cycle(levels, l + 1, Rn @ (r - A @ x), nu, w, p0_level0)
    x = x + Pn @ xc
    for _ in range(nu):
        x = x + w * d * (r - A @ x)
    return x


@pytest.mark.parametrize("space,with_b,cells", CASES)
def test_amg_cycle_equals_cpu_replay(space, with_b, cells):
    from paper_1805_11930_amd import DG_COARSE_SOLVER_AMG, mg_opts

    w, P, cs = _case(space, with_b, cells)
    opr, _ = _oracle(w, (space, with_b, cells))
    Pdg = solvers.q1_prolongation(opr) if space == "q1" else solvers.p0_prolongation(opr)
    levels = _hierarchy(P, cs)
    assert len(levels) >= 2
    r = inputs.random_vector(opr.ndof, 71)
    nu, om = 3, 2.0 / 3.0
    for cycles in (1, 3):
        o = mg_opts(n_pre=0, n_post=0, coarse_space=cs, coarse_solver=DG_COARSE_SOLVER_AMG, coarse_smooth=nu,
                    coarse_omega=om, coarse_cycles=cycles)
        z = P.mg_vcycle(torch.from_numpy(r).cuda(), o).cpu().numpy()
        rc = Pdg.T @ r
        acc = _cycle(levels, 0, rc, nu, om, space == "p0")
        for _ in range(cycles - 1):
            acc = acc + _cycle(levels, 0, rc - levels[0][0] @ acc, nu, om, space == "p0")
        ref = Pdg @ acc
        assert rel(z, ref) <= 1e-10, (cycles, rel(z, ref))
        z32 = P.mg_vcycle(torch.from_numpy(r).float().cuda(), o).cpu().numpy()
        assert rel(z32, ref) <= 1e-4
    P.close()


@pytest.mark.parametrize("space,with_b,cells", CASES)
def test_amg_cycles_converge_to_exact_coarse_solve(space, with_b, cells):
    from paper_1805_11930_amd import DG_COARSE_SOLVER_AMG, mg_opts

    w, P, cs = _case(space, with_b, cells)
    opr, A = _oracle(w, (space, with_b, cells))
    Pdg, Ahat = _ahat(opr, A, space)
    Ahat = Ahat.tocsc()
    r = inputs.random_vector(opr.ndof, 72)
    ref = Pdg @ spla.spsolve(Ahat, Pdg.T @ r)
    o = mg_opts(n_pre=0, n_post=0, coarse_space=cs, coarse_solver=DG_COARSE_SOLVER_AMG, coarse_cycles=40)
    z = P.mg_vcycle(torch.from_numpy(r).cuda(), o).cpu().numpy()
    assert rel(z, ref) <= 1e-8
    P.close()


@pytest.mark.parametrize("with_b", [False, True])
def test_solves_with_amg_coarse_solver(with_b):
    from paper_1805_11930_amd import DG_COARSE_SOLVER_AMG, DG_KRYLOV_FCG, DG_KRYLOV_FGMRES, solve_opts

    w = inputs.random_case(3, cells=(8, 6, 7), seed=52, with_b=with_b)
    opr = oracle_problem(w)
    A = dg.assemble(opr).tocsc()
    P = __import__("paper_1805_11930_amd").Problem(spec(w))
    f = inputs.random_vector(P.ndof, 73)
    for prec in (0, 1):
        o = solve_opts(krylov=DG_KRYLOV_FGMRES if with_b else DG_KRYLOV_FCG, precond_precision=prec, rtol=1e-10,
                       maxit=300, mg=dict(coarse_solver=DG_COARSE_SOLVER_AMG))
        u, res = P.solve(torch.from_numpy(f).cuda(), opts=o)
        assert res.status == 0 and res.rel_residual <= 1e-10
        assert rel(u.cpu().numpy(), spla.spsolve(A, f)) <= 1e-7
    P.close()
