"""Shared test helpers: build the oracle problem and the library problem from
one seeded workload (paper_1805_11930_amd.inputs)."""
from __future__ import annotations

import numpy as np

from oracle import dg


def oracle_problem(w, **kw) -> dg.Problem:
    if getattr(w, "kfield", None) is not None:
        from paper_1805_11930_amd import inputs

        Kf, cf = inputs.field_functions(w.kfield, w.cfield, getattr(w, "nrot", None))
        kw = dict(kw, Kfield=Kf, cfield=cf)
    return dg.Problem(cells=w.cells, lengths=w.lengths, p=w.p, bc=w.bc, sigma=w.sigma, K=w.K, c=w.c, b0=w.b0, B=w.B,
                      **kw)


def spec(w):
    from paper_1805_11930_amd import ProblemSpec

    return ProblemSpec(cells=w.cells, lengths=w.lengths, p=w.p, bc=w.bc, sigma=w.sigma, K=w.K, c=w.c, b0=w.b0, B=w.B,
                       kfield=getattr(w, "kfield", None), cfield=getattr(w, "cfield", (0.0, 0.0)),
                       nrot=getattr(w, "nrot", None))


def rel(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def oracle_rows(pr: dg.Problem, cells, u: np.ndarray) -> dict:
    """(A u)_T for a few cells T, from the oracle's local matrices only
    (usable at sizes where assembling A is out of reach)."""
    tab = dg.Tables(pr)
    Phi, G = dg.volume_tab(pr, tab)
    nl = pr.nloc
    U = u.reshape(pr.ncell, nl)
    out = {}
    for c in cells:
        v = dg.volume_matrix(pr, tab, c, Phi, G) @ U[c]
        for bf, k, side in dg.boundary_faces(pr, c):
            if pr.bc[bf] == "D":
                v += dg.dirichlet_face_matrix(pr, tab, c, k, side) @ U[c]
        ijk = pr.cell_ijk(c)
        for k in range(3):
            for dlt in (-1, 1):
                nb = list(ijk)
                nb[k] += dlt
                if not 0 <= nb[k] < pr.cells[k]:
                    continue
                cn = pr.cell_id(*nb)
                lo, hi = (cn, c) if dlt < 0 else (c, cn)
                blocks = dg.interior_face_blocks(pr, tab, k, lo, hi)
                v += blocks[(c, c)] @ U[c] + blocks[(c, cn)] @ U[cn]
        out[c] = v
    return out
