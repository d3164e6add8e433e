"""Pins of the oracle's Gauss-Lobatto basis (Sec. 2.1, basis paragraph).

Both nodal bases span Q_p on every cell and use the same (p+1)-point Gauss
quadrature, so with V[q, j] = GLL polynomial j at Gauss point q and
S = blockdiag(V (x) V (x) V) (the Gauss-point values of a GLL-coefficient
function, x fastest):
  * the GLL operator is S^T A_GL S, its blocks S_T^T D_T S_T and its
    right-hand side S^T l_GL;
  * a GLL solution u' and the GL solution u of the same problem satisfy
    S u' = u.
The oracle assembles each basis directly from its own 1-D tables (values
and derivatives of the GLL polynomials at the Gauss points), so these
identities check the GLL tables, the assembly loops and the right-hand side
against the Gauss-Legendre code path (itself pinned elsewhere) through a
fact of linear algebra, not by re-running the same formula.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import basis, dg


def _S(prob):
    n = prob.p + 1
    V = basis.lagrange_values(basis.gauss_lobatto(n)[0], basis.gauss_legendre(n)[0])
    ST = np.kron(V, np.kron(V, V))  # index (z, y, x), x fastest on both sides
    return sp.block_diag([ST] * prob.ncell, format="csr"), V


def _pair(p, **kw):
    common = dict(cells=(3, 2, 2), lengths=(1.0, 0.7, 1.3), p=p, bc=("D", "N", "D", "D", "N", "D"), **kw)
    return dg.Problem(basis="gl", **common), dg.Problem(basis="gll", **common)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_value_matrix_interpolates(p):
    # V reproduces polynomials of degree p: the Gauss-point values of the
    # GLL interpolant of x^k equal x^k at the Gauss points
    n = p + 1
    xl = basis.gauss_lobatto(n)[0]
    xg = basis.gauss_legendre(n)[0]
    V = basis.lagrange_values(xl, xg)
    for k in range(n):
        assert np.allclose(V @ xl**k, xg**k, atol=1e-13)
    assert np.allclose(V.sum(axis=1), 1.0, atol=1e-14)


@pytest.mark.parametrize("p,with_b", [(1, True), (2, False), (3, True), (4, False)])
def test_gll_operator_is_change_of_basis(p, with_b):
    rng = np.random.default_rng(p)
    kw = dict(K=rng.uniform(0.5, 2.0, (12, 3)), c=rng.uniform(0.0, 1.0, 12))
    if with_b:
        kw.update(b0=(0.7, -0.4, 0.3), B=((0.1, 0.0, 0.2), (0.0, -0.3, 0.0), (0.05, 0.0, 0.1)))
    gl, gll = _pair(p, **kw)
    S, _ = _S(gl)
    A = dg.assemble(gl).toarray()
    Ap = dg.assemble(gll).toarray()
    assert np.abs(Ap - S.T @ A @ S).max() <= 1e-11 * np.abs(A).max()
    # the blocks transform cell by cell
    D = dg.block_diagonal(dg.assemble(gl), gl.ncell)
    Dp = dg.block_diagonal(dg.assemble(gll), gl.ncell)
    ST = S[: gl.nloc, : gl.nloc].toarray()
    for T in range(gl.ncell):
        assert np.abs(Dp[T] - ST.T @ D[T] @ ST).max() <= 1e-11 * np.abs(D[T]).max()


@pytest.mark.parametrize("p", [1, 3])
def test_gll_rhs_and_solution(p):
    def f(x):
        return np.sin(2 * x[:, 0]) + x[:, 1] * x[:, 2]

    def g(x):
        return np.cos(x[:, 0] + x[:, 1]) - x[:, 2]

    def j(x):
        return 0.3 + x[:, 0] * x[:, 1]

    gl, gll = _pair(p, b0=(0.5, 0.2, -0.1))
    S, _ = _S(gl)
    l = dg.assemble_rhs(gl, f=f, g=g, j=j)
    lp = dg.assemble_rhs(gll, f=f, g=g, j=j)
    assert np.abs(lp - S.T @ l).max() <= 1e-12 * np.abs(l).max()
    u = spla.spsolve(dg.assemble(gl).tocsc(), l)
    up = spla.spsolve(dg.assemble(gll).tocsc(), lp)
    assert np.abs(S @ up - u).max() <= 1e-10 * np.abs(u).max()
    # GLL coefficients are the values at the GLL nodes
    pts = dg.node_points(gll)
    xl = basis.gauss_lobatto(p + 1)[0]
    assert np.allclose(pts[1, 0] / gll.h[0], xl[1])
