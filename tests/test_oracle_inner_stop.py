"""Pins of the inner block solves' stopping rule (CPU only).

Sec. 2.2.1 solves each block system D_T du_T = d_T (eqn block_system) only
until the 2-norm of the block residual d_T - D_T du_T has dropped by the
factor eps, starting from zero.  The oracle's block PCG (b = 0) and block
GMRES (b != 0, diagonal or tridiagonal preconditioner, with restarts) must
therefore return the FIRST iterate that meets the rule:

  * the returned iterate x_k satisfies ||d - D x_k||_2 <= eps ||d||_2, with
    the residual recomputed here from D, d and x_k (not taken from the
    solver's own recursion);
  * the same solver stopped one D-application earlier (max_inner = k - 1)
    returns an iterate that does not.

Both conditions together fix the iteration count, so a solver that stops on
another norm (for instance the preconditioned one, sqrt(r^T M^-1 r)), or one
iteration late or early, fails one of them.  The last tests plant exactly
those mistakes in copies of the oracle's PCG and check that the pins catch
them.  The blocks are the DG cell blocks of small random-coefficient meshes
at p = 2, 3, 4 and eps = 1e-2, the paper's inner tolerance (Sec. 4.2).
"""
import numpy as np
import pytest

from oracle import dg, solvers

EPS = 1e-2


def blocks(p, with_b, seed=0, cells=(2, 2, 2)):
    rng = np.random.default_rng(seed)
    nc = int(np.prod(cells))
    kw = {}
    if with_b:
        kw = dict(b0=(0.6, -0.4, 0.3), B=((0.0, 1.0, 0.0), (-1.0, 0.0, 0.0), (0.0, 0.0, 0.0)))
    pr = dg.Problem(cells=cells, p=p, K=np.exp(rng.normal(size=(nc, 3))), **kw)
    A = dg.assemble(pr)
    return dg.block_diagonal(A, pr.ncell), pr


def true_ratio(D, d, x):
    return np.linalg.norm(d - D @ x) / np.linalg.norm(d)


def check_first_iterate(solve, D, d):
    """solve(D, d, max_inner) -> (x, it).  Returns the iteration count."""
    x, k = solve(D, d, 10 * D.shape[0])
    assert k >= 1
    assert true_ratio(D, d, x) <= EPS * (1.0 + 1e-9), (k, true_ratio(D, d, x))
    xm, km = solve(D, d, k - 1)
    assert km == k - 1
    # one application earlier the rule is not met yet (k - 1 = 0: x = 0)
    assert true_ratio(D, d, xm) > EPS, (k, true_ratio(D, d, xm))
    return k


def rhs(rng, n, kind):
    if kind == "random":
        return rng.normal(size=n)
    # a smooth defect (what a smoother sees after the first sweeps)
    return np.cos(np.linspace(0.0, 3.0, n)) + 0.1 * rng.normal(size=n)


@pytest.mark.parametrize("p", [2, 3, 4])
@pytest.mark.parametrize("kind", ["random", "smooth"])
def test_block_pcg_stops_at_first_iterate_meeting_eps(p, kind):
    Db, pr = blocks(p, with_b=False, seed=p)
    rng = np.random.default_rng(10 + p)
    counts = []
    for T in range(pr.ncell):
        d = rhs(rng, pr.nloc, kind)
        counts.append(check_first_iterate(
            lambda D, v, mi: solvers.block_pcg(D, v, EPS, mi), Db[T], d))
    assert max(counts) >= 2  # the rule is exercised beyond the first step


@pytest.mark.parametrize("p", [2, 3, 4])
@pytest.mark.parametrize("precond", ["diag", "tridiag"])
@pytest.mark.parametrize("restart", [4, 30])
def test_block_gmres_stops_at_first_iterate_meeting_eps(p, precond, restart):
    Db, pr = blocks(p, with_b=True, seed=20 + p)
    assert np.abs(Db[0] - Db[0].T).max() > 1e-3  # nonsymmetric blocks
    rng = np.random.default_rng(30 + p)
    counts = []
    for T in range(pr.ncell):
        d = rng.normal(size=pr.nloc)
        counts.append(check_first_iterate(
            lambda D, v, mi: solvers.block_gmres(D, v, EPS, mi, restart, precond), Db[T], d))
    assert max(counts) >= 2
    if restart == 4:
        assert max(counts) > 4  # at least one block goes through a restart


def test_block_gmres_on_spd_block_meets_rule():
    """b = 0 blocks through GMRES (the smoother's GMRES path also takes them)."""
    Db, pr = blocks(3, with_b=False, seed=7)
    rng = np.random.default_rng(8)
    for T in range(pr.ncell):
        check_first_iterate(
            lambda D, v, mi: solvers.block_gmres(D, v, EPS, mi, 12, "diag"), Db[T], rng.normal(size=pr.nloc))


# ---------------------------------------------------------------------------
# planted mistakes: copies of the PCG with a wrong stopping rule must fail
# ---------------------------------------------------------------------------
def pcg_variant(D, d, eps, max_inner, rule):
    """The oracle's PCG with a deliberately altered stopping rule."""
    x = np.zeros_like(d)
    r = d.copy()
    dn = np.linalg.norm(d)
    diag = np.diag(D).copy()
    z = r / diag
    p = z.copy()
    rho = r @ z
    rho0 = rho
    it = 0
    late = False
    while it < max_inner:
        q = D @ p
        it += 1
        alpha = rho / (p @ q)
        x = x + alpha * p
        r = r - alpha * q
        z = r / diag
        rho_new = r @ z
        if rule == "preconditioned" and np.sqrt(rho_new) <= eps * np.sqrt(rho0):
            break
        if rule == "one_late":
            if late:
                break
            late = np.linalg.norm(r) <= eps * dn
        p = z + (rho_new / rho) * p
        rho = rho_new
    return x, it


@pytest.mark.parametrize("rule", ["preconditioned", "one_late"])
def test_pins_reject_wrong_stopping_rules(rule):
    caught = 0
    for p in (2, 3, 4):
        Db, pr = blocks(p, with_b=False, seed=p)
        rng = np.random.default_rng(10 + p)
        for T in range(pr.ncell):
            d = rng.normal(size=pr.nloc)
            try:
                check_first_iterate(lambda D, v, mi: pcg_variant(D, v, EPS, mi, rule), Db[T], d)
            except AssertionError:
                caught += 1
    assert caught > 0
