"""1-D quadrature rules and Lagrange tables on the reference interval [0, 1].

Oracle (test infrastructure only; see the package docstring).

The DG space uses a tensor-product nodal Lagrange basis on each hexahedral
cell (Sec. 2.1, the basis paragraph; Sec. 3.1, the Stage 1 paragraph, where
the 1-D matrices A^(k) hold shape-function values at quadrature points).
The paper's own basis is nodal at the Gauss-Lobatto points; this build's
default places the nodes at the Gauss-Legendre points instead (both span
Q_p, so the discrete function space is identical).  Both are provided here.

Gauss-Legendre nodes and weights come from numpy's Golub-Welsch routine
(``numpy.polynomial.legendre.leggauss``) used as a library primitive; the
Gauss-Lobatto rule is the textbook one: the end points plus the roots of
P'_{n-1}, weights 2 / (n (n-1) P_{n-1}(x)^2) on [-1, 1].
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg


def gauss_legendre(n: int):
    """n-point Gauss-Legendre rule on [0, 1]: (nodes, weights), sum(w) = 1."""
    if n < 1:
        raise ValueError("n >= 1 required")
    x, w = npleg.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def gauss_lobatto(n: int):
    """n-point Gauss-Lobatto rule on [0, 1] (n >= 2): (nodes, weights)."""
    if n < 2:
        raise ValueError("Gauss-Lobatto needs n >= 2")
    # Legendre polynomial P_{n-1} in the Legendre series basis.
    c = np.zeros(n)
    c[-1] = 1.0
    interior = npleg.legroots(npleg.legder(c)) if n > 2 else np.zeros(0)
    x = np.concatenate(([-1.0], np.sort(interior.real), [1.0]))
    w = 2.0 / (n * (n - 1) * npleg.legval(x, c) ** 2)
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange_values(nodes, x):
    """L[a, j] = l_j(x_a) for the Lagrange polynomials on ``nodes``.

    Direct product formula l_j(x) = prod_{m != j} (x - x_m) / (x_j - x_m).
    """
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = nodes.size
    L = np.ones((x.size, n))
    for j in range(n):
        for m in range(n):
            if m != j:
                L[:, j] *= (x - nodes[m]) / (nodes[j] - nodes[m])
    return L


def lagrange_derivatives(nodes, x):
    """Dl[a, j] = l_j'(x_a): product rule on the product formula."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = nodes.size
    Dl = np.zeros((x.size, n))
    for j in range(n):
        denom = 1.0
        for m in range(n):
            if m != j:
                denom *= nodes[j] - nodes[m]
        for r in range(n):  # factor that is differentiated
            if r == j:
                continue
            term = np.ones(x.size)
            for m in range(n):
                if m != j and m != r:
                    term *= x - nodes[m]
            Dl[:, j] += term
        Dl[:, j] /= denom
    return Dl


def basis_nodes(p: int, basis: str = "gl"):
    """Nodes of the 1-D nodal basis of degree p: 'gl' (default) or 'gll'."""
    if basis == "gl":
        return gauss_legendre(p + 1)[0]
    if basis == "gll":
        return gauss_lobatto(p + 1)[0]
    raise ValueError(f"unknown basis {basis!r}")
