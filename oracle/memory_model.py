"""Memory estimates of the matrix-explicit (MX), partially matrix-free (PMF)
and fully matrix-free (MF) solvers.

Oracle (test infrastructure only; see the package docstring).

Sec. 4.4: a DG vector holds M_vector = N_cell (p+1)^d doubles, the DG
matrix M_matrix = 7 N_cell (p+1)^(2d) and its block diagonal
M_blockdiag = N_cell (p+1)^(2d).  The totals are eqn memory_diffusion
(CG + hybrid multigrid with a Q1 coarse level) and eqn memory_convection
(flexible GMRES + block-SSOR, inner GMRES + tridiagonal preconditioner).
All counts are in doubles (8 bytes).
"""
from __future__ import annotations

D = 3  # spatial dimension used throughout the paper's tables


def vector_doubles(p: int, ncell: int, d: int = D) -> int:
    return ncell * (p + 1) ** d


def matrix_doubles(p: int, ncell: int, d: int = D) -> int:
    return 7 * ncell * (p + 1) ** (2 * d)


def blockdiag_doubles(p: int, ncell: int, d: int = D) -> int:
    return ncell * (p + 1) ** (2 * d)


def diffusion_doubles(p: int, ncell: int, d: int = D) -> dict:
    """eqn memory_diffusion: totals for MX, PMF, MF (doubles)."""
    nl = (p + 1) ** d
    return {
        "MX": (7 * nl * nl + 6 * nl + 30) * ncell,
        "PMF": (nl * nl + 7 * nl + 30) * ncell,
        "MF": (8 * nl + 30) * ncell,
    }


def convection_doubles(p: int, ncell: int, n_outer: int, n_block: int, d: int = D) -> dict:
    """eqn memory_convection: totals for MX, PMF, MF (doubles)."""
    nl = (p + 1) ** d
    return {
        "MX": (7 * nl * nl + (2 * n_outer + 4) * nl) * ncell,
        "PMF": (nl * nl + (2 * n_outer + 4) * nl) * ncell,
        "MF": (2 * n_outer + 7) * nl * ncell + (n_block + 1) * nl,
    }
