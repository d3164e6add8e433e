"""Pins of the oracle's 1-D tables against closed forms (CPU only).

The tensor-product nodal basis and tensor quadrature are described in
Sec. 2.1 (basis paragraph) and Sec. 3.1 (Stage 1: 1-D matrices of shape
function values at quadrature points).  Closed forms of the Gauss-Legendre
and Gauss-Lobatto rules are textbook values on [-1, 1].
"""
import numpy as np
import pytest

from oracle import basis

S = np.sqrt

GL_CLOSED = {
    2: ([-1 / S(3), 1 / S(3)], [1.0, 1.0]),
    3: ([-S(3 / 5), 0.0, S(3 / 5)], [5 / 9, 8 / 9, 5 / 9]),
    4: (
        [-S(3 / 7 + 2 / 7 * S(6 / 5)), -S(3 / 7 - 2 / 7 * S(6 / 5)), S(3 / 7 - 2 / 7 * S(6 / 5)), S(3 / 7 + 2 / 7 * S(6 / 5))],
        [(18 - S(30)) / 36, (18 + S(30)) / 36, (18 + S(30)) / 36, (18 - S(30)) / 36],
    ),
    5: (
        [-S(5 + 2 * S(10 / 7)) / 3, -S(5 - 2 * S(10 / 7)) / 3, 0.0, S(5 - 2 * S(10 / 7)) / 3, S(5 + 2 * S(10 / 7)) / 3],
        [(322 - 13 * S(70)) / 900, (322 + 13 * S(70)) / 900, 128 / 225, (322 + 13 * S(70)) / 900, (322 - 13 * S(70)) / 900],
    ),
}

GLL_CLOSED = {
    2: ([-1.0, 1.0], [1.0, 1.0]),
    3: ([-1.0, 0.0, 1.0], [1 / 3, 4 / 3, 1 / 3]),
    4: ([-1.0, -1 / S(5), 1 / S(5), 1.0], [1 / 6, 5 / 6, 5 / 6, 1 / 6]),
    5: ([-1.0, -S(3 / 7), 0.0, S(3 / 7), 1.0], [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10]),
}


@pytest.mark.parametrize("n", sorted(GL_CLOSED))
def test_gauss_legendre_closed_form(n):
    x, w = basis.gauss_legendre(n)
    xe, we = GL_CLOSED[n]
    np.testing.assert_allclose(2 * x - 1, xe, rtol=0, atol=1e-15)
    np.testing.assert_allclose(2 * w, we, rtol=0, atol=1e-15)


@pytest.mark.parametrize("n", sorted(GLL_CLOSED))
def test_gauss_lobatto_closed_form(n):
    x, w = basis.gauss_lobatto(n)
    xe, we = GLL_CLOSED[n]
    np.testing.assert_allclose(2 * x - 1, xe, rtol=0, atol=1e-15)
    np.testing.assert_allclose(2 * w, we, rtol=0, atol=1e-15)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_gauss_exactness(n):
    x, w = basis.gauss_legendre(n)
    assert abs(w.sum() - 1.0) < 1e-15
    for k in range(2 * n):
        assert abs(np.sum(w * x**k) - 1.0 / (k + 1)) < 2e-15
    # degree 2n is not integrated exactly
    assert abs(np.sum(w * x ** (2 * n)) - 1.0 / (2 * n + 1)) > 1e-8


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_lobatto_exactness(n):
    x, w = basis.gauss_lobatto(n)
    for k in range(2 * n - 2):
        assert abs(np.sum(w * x**k) - 1.0 / (k + 1)) < 2e-15


@pytest.mark.parametrize("kind", ["gl", "gll"])
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_lagrange_tables(kind, p):
    nodes = basis.basis_nodes(p, kind)
    L = basis.lagrange_values(nodes, nodes)
    np.testing.assert_allclose(L, np.eye(p + 1), atol=1e-14)
    xs = np.linspace(0, 1, 7)
    Lx = basis.lagrange_values(nodes, xs)
    Dx = basis.lagrange_derivatives(nodes, xs)
    for k in range(p + 1):
        # interpolation reproduces xi^k and its derivative k xi^(k-1)
        np.testing.assert_allclose(Lx @ nodes**k, xs**k, atol=1e-13)
        dk = k * xs ** (k - 1) if k > 0 else np.zeros_like(xs)
        np.testing.assert_allclose(Dx @ nodes**k, dk, atol=1e-12)
