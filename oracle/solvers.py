"""Block smoothers, P0 coarse space, hybrid V-cycle and outer Krylov methods.

Oracle (test infrastructure only; see the package docstring).

Each routine takes the paper's steps in the paper's order:
  * block-Jacobi: alg block_jacobi (Sec. 2.2.1) with W = omega^-1 D;
  * block-SOR: alg block_SOR in a given cell order, in place (Sec. 2.2.1):
    the local defect leaves out the cell's own block and the new value is
    (1 - omega) u + omega du; the backward sweep reverses the order and
    block-SSOR is a forward then a backward sweep; the red-black (two
    colour) cell order is the one whose colours can be swept in parallel;
  * the block systems D_T du_T = d_T (eqn block_system) are solved either
    exactly (dense LU) or inexactly with a Krylov method stopped when the
    2-norm of the block residual has dropped by the factor eps (Sec. 2.2.1),
    preconditioned by the diagonal of D_T or, for strongly convective
    blocks, by its tridiagonal part solved with the Thomas algorithm
    (Sec. 3.2, Sec. 4.3);
  * intergrid operators: P0 injection, P|_T = (1, ..., 1)^T, R = P^T
    (Sec. 2.2.2);
  * coarse matrix A_hat = P^T A P (eqn galerkin_product) and its direct
    evaluation a_h(psi_hat_j, psi_hat_i) on P0 indicator functions
    (App. A.1, eqn p0_galerkin1);
  * hybrid V-cycle: alg hybrid_multigrid;
  * outer CG / flexible CG / flexible GMRES with right preconditioning,
    stopped on ||r_k||_2 <= rtol ||r_0||_2 (Sec. 4.2, Sec. 4.3).
Where the paper leaves the step order open (inner PCG, GMRES details) the
textbook algorithms are written out: Hestenes-Stiefel PCG, and Saad's
restarted GMRES with modified Gram-Schmidt and Givens rotations.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import dg as _dg


# ---------------------------------------------------------------------------
# inner block solves
# ---------------------------------------------------------------------------
def block_solve_exact(D: np.ndarray, d: np.ndarray):
    """du = D^-1 d by dense LU.  Returns (du, 0)."""
    return sla.lu_solve(sla.lu_factor(D), d), 0


def block_pcg(D: np.ndarray, d: np.ndarray, eps: float, max_inner: int):
    """Diagonally preconditioned CG on D x = d from x = 0.

    Stops when ||d - D x||_2 <= eps ||d||_2 (the recursive residual) or
    after max_inner applications of D.  Returns (x, iterations).
    """
    x = np.zeros_like(d)
    r = d.copy()
    dnorm = np.linalg.norm(d)
    if dnorm == 0.0:
        return x, 0
    diag = np.diag(D).copy()
    z = r / diag
    p = z.copy()
    rho = r @ z
    it = 0
    while it < max_inner:
        q = D @ p
        it += 1
        alpha = rho / (p @ q)
        x = x + alpha * p
        r = r - alpha * q
        if np.linalg.norm(r) <= eps * dnorm:
            break
        z = r / diag
        rho_new = r @ z
        beta = rho_new / rho
        p = z + beta * p
        rho = rho_new
    return x, it


def thomas(sub: np.ndarray, diag: np.ndarray, sup: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Solve the tridiagonal system  sub_i x_{i-1} + diag_i x_i + sup_i x_{i+1}
    = v_i  by the Thomas algorithm (Gaussian elimination without pivoting:
    a forward sweep that removes the sub-diagonal, then back substitution)."""
    n = v.size
    cp = np.zeros(n)
    y = np.zeros(n)
    for i in range(n):
        m = diag[i] - (sub[i] * cp[i - 1] if i > 0 else 0.0)
        cp[i] = sup[i] / m if i < n - 1 else 0.0
        y[i] = (v[i] - (sub[i] * y[i - 1] if i > 0 else 0.0)) / m
    x = np.zeros(n)
    for i in range(n - 1, -1, -1):
        x[i] = y[i] - (cp[i] * x[i + 1] if i < n - 1 else 0.0)
    return x


def block_preconditioner(D: np.ndarray, kind: str):
    """v -> M^-1 v for the inner Krylov method (Sec. 3.2): 'diag' divides by
    the diagonal of D_T; 'tridiag' solves with the tridiagonal part of D_T
    (cell DOFs in their x-fastest order) by the Thomas algorithm."""
    if kind == "diag":
        minv = 1.0 / np.diag(D)
        return lambda v: minv * v
    if kind == "tridiag":
        n = D.shape[0]
        diag = np.diag(D).copy()
        sub = np.concatenate([[0.0], np.diag(D, -1)])
        sup = np.concatenate([np.diag(D, 1), [0.0]])
        return lambda v: thomas(sub, diag, sup, v)
    raise ValueError(kind)


def block_gmres(D: np.ndarray, d: np.ndarray, eps: float, max_inner: int, restart: int, precond: str = "diag"):
    """Right-preconditioned restarted GMRES on D x = d from x = 0 with
    M = diag(D) or the tridiagonal part of D (block_preconditioner).

    Modified Gram-Schmidt Arnoldi, Givens rotations; stops when the
    Arnoldi residual estimate |g_{j+1}| <= eps ||d||_2 or after max_inner
    applications of D.  Returns (x, iterations).
    """
    n = d.size
    x = np.zeros_like(d)
    dnorm = np.linalg.norm(d)
    if dnorm == 0.0:
        return x, 0
    minv = block_preconditioner(D, precond)
    target = eps * dnorm
    it = 0
    r = d.copy()
    beta = dnorm
    while True:
        m = restart
        V = np.zeros((m + 1, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        V[0] = r / beta
        g[0] = beta
        done = False
        k = 0
        for j in range(m):
            w = D @ minv(V[j])
            it += 1
            for i in range(j + 1):
                H[i, j] = w @ V[i]
                w = w - H[i, j] * V[i]
            hnext = np.linalg.norm(w)
            H[j + 1, j] = hnext
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            rr = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / rr
            sn[j] = H[j + 1, j] / rr
            H[j, j] = rr
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            if abs(g[j + 1]) <= target or it >= max_inner:
                done = True
                break
            V[j + 1] = w / hnext
        y = sla.solve_triangular(H[:k, :k], g[:k], lower=False)
        x = x + minv(V[:k].T @ y)
        if done or it >= max_inner:
            return x, it
        r = d - D @ x
        beta = np.linalg.norm(r)
        if beta <= target:
            return x, it


# ---------------------------------------------------------------------------
# block-Jacobi smoother (alg block_jacobi)
# ---------------------------------------------------------------------------
def block_jacobi(A, Dblocks, f, u0, omega=1.0, nsweeps=1, inner="exact", eps=1e-2,
                 max_inner=None, restart=30, stats=None, precond="diag"):
    """n_sweeps block-Jacobi steps u <- u + omega D^-1_eps (f - A u)."""
    ncell, nb, _ = Dblocks.shape
    if max_inner is None:
        max_inner = nb
    u = np.array(u0, dtype=np.float64, copy=True)
    for _ in range(nsweeps):
        d = (f - A @ u).reshape(ncell, nb)
        du = np.zeros_like(d)
        for T in range(ncell):
            if inner == "exact":
                du[T], it = block_solve_exact(Dblocks[T], d[T])
            elif inner == "cg":
                du[T], it = block_pcg(Dblocks[T], d[T], eps, max_inner)
            elif inner == "gmres":
                du[T], it = block_gmres(Dblocks[T], d[T], eps, max_inner, min(restart, nb), precond)
            else:
                raise ValueError(inner)
            if stats is not None:
                stats.append(it)
        u = u + omega * du.ravel()
    return u


def _inner_solve(D, d, inner, eps, max_inner, restart, precond="diag"):
    if inner == "exact":
        return block_solve_exact(D, d)
    if inner == "cg":
        return block_pcg(D, d, eps, max_inner)
    if inner == "gmres":
        return block_gmres(D, d, eps, max_inner, min(restart, d.size), precond)
    raise ValueError(inner)


# ---------------------------------------------------------------------------
# block-SOR / block-SSOR smoothers (alg block_SOR, Sec. 2.2.1)
# ---------------------------------------------------------------------------
def lexicographic_order(prob: _dg.Problem) -> np.ndarray:
    """Cells in index order (x fastest)."""
    return np.arange(prob.ncell)


def multicolour_order(prob: _dg.Problem, colours: int = 2) -> np.ndarray:
    """Cells ordered by colour (ix + iy + iz) mod C, C = colours >= 2, each
    colour in index order; C = 2 is the red-black order.  Face neighbours
    differ by one in exactly one index, so no two cells of one colour share
    a face.  When C is at least the number of diagonal planes
    ix + iy + iz = const, the colour is the plane index and the order is a
    hyperplane (wavefront) order."""
    ijk = np.array([prob.cell_ijk(c) for c in range(prob.ncell)]).reshape(-1, 3)
    colour = ijk.sum(axis=1) % colours
    cells = np.arange(prob.ncell)
    return np.concatenate([cells[colour == q] for q in range(colours)])


def block_sor(A, Dblocks, f, u0, order, omega=1.0, nsweeps=1, inner="exact", eps=1e-2,
              max_inner=None, restart=30, stats=None, precond="diag"):
    """n_sweeps forward block-SOR steps over the cells in ``order``.

    Alg block_SOR: cell T_rho, taken in the given order, forms its local
    defect from f_rho minus the couplings to every other cell (the cells
    visited before it already carry step-k values, the others step k-1
    values, so updating u in place is exactly the algorithm), solves
    D_rho du = d_rho (exactly or to the relative tolerance eps) and sets
    u_rho = (1 - omega) u_rho + omega du.  The backward sweep is the same
    with the order reversed.
    """
    ncell, nb, _ = Dblocks.shape
    if max_inner is None:
        max_inner = nb
    Ab = sp.bsr_matrix(A, blocksize=(nb, nb))
    Ab.sort_indices()
    u = np.array(u0, dtype=np.float64, copy=True).reshape(ncell, nb)
    fb = np.asarray(f, dtype=np.float64).reshape(ncell, nb)
    for _ in range(nsweeps):
        for rho in order:
            d = fb[rho].copy()
            for k in range(Ab.indptr[rho], Ab.indptr[rho + 1]):
                sigma = Ab.indices[k]
                if sigma != rho:
                    d -= Ab.data[k] @ u[sigma]
            du, it = _inner_solve(Dblocks[rho], d, inner, eps, max_inner, restart, precond)
            if stats is not None:
                stats.append(it)
            u[rho] = (1.0 - omega) * u[rho] + omega * du
    return u.ravel()


def block_ssor(A, Dblocks, f, u0, order, omega=1.0, nsweeps=1, **kw):
    """n_sweeps block-SSOR steps: each is a forward block-SOR sweep over
    ``order`` followed by a backward sweep over the reversed order
    (Sec. 2.2.1)."""
    u = np.array(u0, dtype=np.float64, copy=True)
    rev = np.asarray(order)[::-1]
    for _ in range(nsweeps):
        u = block_sor(A, Dblocks, f, u, order, omega=omega, nsweeps=1, **kw)
        u = block_sor(A, Dblocks, f, u, rev, omega=omega, nsweeps=1, **kw)
    return u


# ---------------------------------------------------------------------------
# P0 subspace (Sec. 2.2.2, 2.2.3, App. A.1)
# ---------------------------------------------------------------------------
def p0_prolongation(prob: _dg.Problem) -> sp.csr_matrix:
    """P with P|_T = (1, ..., 1)^T: (ndof, ncell)."""
    return sp.kron(sp.identity(prob.ncell, format="csr"), np.ones((prob.nloc, 1)), format="csr")


def p0_galerkin(A, prob: _dg.Problem) -> np.ndarray:
    """A_hat = P^T A P (eqn galerkin_product), dense (ncell, ncell)."""
    P = p0_prolongation(prob)
    return np.asarray((P.T @ (A.tocsr() @ P)).todense())


def p0_direct(prob: _dg.Problem) -> np.ndarray:
    """A_hat_{T,T'} = a_h(1_T', 1_T) evaluated directly on P0 indicators.

    Gradients of P0 functions vanish, so only c |T| on the diagonal, the
    upwind terms and the penalty terms remain (eqn p0_galerkin1); the
    face integrals use the same face quadrature as A.
    """
    if prob.Kfield is not None or prob.cfield is not None:
        raise ValueError("coarse matrices are built from the cell-centre problem (dg.cell_centre_problem)")
    tab = _dg.Tables(prob)
    h = prob.h
    nc = prob.ncell
    Ah = np.zeros((nc, nc))
    vol = np.prod(h)
    for c in range(nc):
        Ah[c, c] += prob.creact(c) * vol
        for bf, k, side in _dg.boundary_faces(prob, c):
            if prob.bc[bf] != "D":
                continue
            WF = _dg.face_weights(prob, tab, k)
            _, _, xi = _dg.face_tab(prob, tab, k, side)
            nu_k = 1.0 if side == 1 else -1.0
            gam = _dg.penalty_boundary(prob, k, prob.Kdiag(c)[k])
            val = gam * WF.sum()
            if prob.has_b:
                bnu = nu_k * prob.bfield(prob.origin(c) + xi * h)[:, k]
                val += np.sum(WF * bnu * (bnu >= 0.0))
            Ah[c, c] += val
    for c in range(nc):
        ijk = prob.cell_ijk(c)
        for k in range(3):
            if ijk[k] + 1 >= prob.cells[k]:
                continue
            nb = list(ijk)
            nb[k] += 1
            cu = prob.cell_id(*nb)
            WF = _dg.face_weights(prob, tab, k)
            _, _, xi = _dg.face_tab(prob, tab, k, 1)
            dm, dp = prob.Kdiag(c)[k], prob.Kdiag(cu)[k]
            gam = _dg.penalty_interior(prob, k, dm, dp)
            if prob.has_b:
                bnu = prob.bfield(prob.origin(c) + xi * h)[:, k]
            else:
                bnu = np.zeros(WF.shape)
            chim = (bnu >= 0.0).astype(np.float64)
            # (s, t) in {-, +} with sign [[1_s]] = +1 / -1
            for s, cs_, ss in (("-", c, 1.0), ("+", cu, -1.0)):
                for t, ct, st in (("-", c, 1.0), ("+", cu, -1.0)):
                    chit = chim if t == "-" else 1.0 - chim
                    Ah[cs_, ct] += ss * np.sum(WF * bnu * chit) + gam * ss * st * WF.sum()
    return Ah


# ---------------------------------------------------------------------------
# conforming Q1 subspace (Sec. 2.2.2, 2.2.3, App. A.2)
# ---------------------------------------------------------------------------
def q1_vertex_id(prob: _dg.Problem, vx, vy, vz) -> int:
    nx, ny, _ = prob.cells
    return vx + (nx + 1) * (vy + (ny + 1) * vz)


def q1_nvert(prob: _dg.Problem) -> int:
    nx, ny, nz = prob.cells
    return (nx + 1) * (ny + 1) * (nz + 1)


def q1_prolongation(prob: _dg.Problem) -> sp.csr_matrix:
    """P with (P|_T)_ij = psi_hat_j(zeta_i): the trilinear vertex functions
    evaluated at the DG nodes (the nodal interpolation of Sec. 2.2.2)."""
    tab = _dg.Tables(prob)
    xi = tab.nodes
    n = prob.n
    rows, cols, vals = [], [], []
    for c in range(prob.ncell):
        ix, iy, iz = prob.cell_ijk(c)
        for kz in range(n):
            for ky in range(n):
                for kx in range(n):
                    row = c * prob.nloc + kx + n * (ky + n * kz)
                    for dz in (0, 1):
                        for dy in (0, 1):
                            for dx in (0, 1):
                                wgt = ((xi[kx] if dx else 1 - xi[kx]) * (xi[ky] if dy else 1 - xi[ky])
                                       * (xi[kz] if dz else 1 - xi[kz]))
                                rows.append(row)
                                cols.append(q1_vertex_id(prob, ix + dx, iy + dy, iz + dz))
                                vals.append(wgt)
    return sp.csr_matrix((vals, (rows, cols)), shape=(prob.ndof, q1_nvert(prob)))


def q1_galerkin(A, prob: _dg.Problem) -> np.ndarray:
    """A_hat = P^T A P for the Q1 subspace, dense (nvert, nvert)."""
    P = q1_prolongation(prob)
    return np.asarray((P.T @ (A.tocsr() @ P)).todense())


def q1_direct(prob: _dg.Problem) -> np.ndarray:
    """A_hat_ij = a_h(psi_hat_j, psi_hat_i) evaluated directly on the
    trilinear vertex functions (App. A.2): continuous functions have no
    jumps, so only the volume terms and the Dirichlet-face terms of a_h
    remain; same quadrature as A."""
    if prob.Kfield is not None or prob.cfield is not None:
        raise ValueError("coarse matrices are built from the cell-centre problem (dg.cell_centre_problem)")
    tab = _dg.Tables(prob)
    h = prob.h
    xq, wq = tab.xq, tab.wq
    # 1-D linear hats and derivatives at the quadrature points
    L1 = np.stack([1 - xq, xq], axis=1)  # (m, 2)
    D1 = np.stack([-np.ones_like(xq), np.ones_like(xq)], axis=1)
    Phi = _dg.tensor_tab(L1, L1, L1)  # (Q, 8), corner index dx + 2dy + 4dz
    G = [_dg.tensor_tab(D1 / h[0], L1, L1), _dg.tensor_tab(L1, D1 / h[1], L1), _dg.tensor_tab(L1, L1, D1 / h[2])]
    W = _dg.tensor_weights(wq, wq, wq) * np.prod(h)
    xi_vol = _dg.tensor_points(xq, xq, xq)
    nv = q1_nvert(prob)
    Ah = np.zeros((nv, nv))
    ends = [np.array([[1.0, 0.0]]), np.array([[0.0, 1.0]])]
    dends = [np.array([[-1.0, 1.0]]), np.array([[-1.0, 1.0]])]
    for c in range(prob.ncell):
        ix, iy, iz = prob.cell_ijk(c)
        verts = [q1_vertex_id(prob, ix + (q & 1), iy + ((q >> 1) & 1), iz + (q >> 2)) for q in range(8)]
        K = prob.Kdiag(c)
        E = np.zeros((8, 8))
        for k in range(3):
            E += K[k] * (G[k].T * W) @ G[k]
        if prob.has_b:
            bq = prob.bfield(prob.origin(c) + xi_vol * h)
            for k in range(3):
                E -= (G[k].T * (W * bq[:, k])) @ Phi
        E += prob.creact(c) * (Phi.T * W) @ Phi
        for bf, k, side in _dg.boundary_faces(prob, c):
            if prob.bc[bf] != "D":
                continue
            vals = [L1, L1, L1]
            ders = [L1, L1, L1]
            vals[k] = ends[side]
            ders[k] = dends[side] / h[k]
            Tr = _dg.tensor_tab(*vals)
            Dk = _dg.tensor_tab(*ders)
            pts = [xq, xq, xq]
            pts[k] = np.array([float(side)])
            xi = _dg.tensor_points(*pts)
            WF = _dg.face_weights(prob, tab, k)
            nu_k = 1.0 if side == 1 else -1.0
            d = K[k]
            gam = _dg.penalty_boundary(prob, k, d)
            Dn = nu_k * Dk
            E += -d * (Tr.T * WF) @ Dn - d * (Dn.T * WF) @ Tr + gam * (Tr.T * WF) @ Tr
            if prob.has_b:
                bnu = nu_k * prob.bfield(prob.origin(c) + xi * h)[:, k]
                E += (Tr.T * (WF * bnu * (bnu >= 0.0))) @ Tr
        for a_, va in enumerate(verts):
            for b_, vb in enumerate(verts):
                Ah[va, vb] += E[a_, b_]
    return Ah


# ---------------------------------------------------------------------------
# hybrid V-cycle (alg hybrid_multigrid)
# ---------------------------------------------------------------------------
def vcycle(A, Dblocks, prob: _dg.Problem, r, coarse_solve, n_pre=1, n_post=1, omega=1.0,
           inner="exact", eps=1e-2, max_inner=None, restart=30, stats=None, P=None,
           smoother="jacobi", order=None, precond="diag"):
    """z ~= A^-1 r: presmooth from zero, residual, restrict, coarse solve,
    prolongate-add, postsmooth.  P: prolongation (default: P0).

    smoother: 'jacobi', 'ssor', or 'sor' (forward sweeps before the coarse
    correction, backward sweeps after it, so that the cycle is symmetric
    for a symmetric A); order: the cell order of the SOR sweeps (default
    red-black)."""
    if P is None:
        P = p0_prolongation(prob)
    if order is None:
        order = multicolour_order(prob)
    order = np.asarray(order)
    kw = dict(omega=omega, inner=inner, eps=eps, max_inner=max_inner, restart=restart, stats=stats,
              precond=precond)

    def smooth(u, n, post):
        if smoother == "jacobi":
            return block_jacobi(A, Dblocks, r, u, nsweeps=n, **kw)
        if smoother == "ssor":
            return block_ssor(A, Dblocks, r, u, order, nsweeps=n, **kw)
        if smoother == "sor":
            return block_sor(A, Dblocks, r, u, order[::-1] if post else order, nsweeps=n, **kw)
        raise ValueError(smoother)

    z = smooth(np.zeros_like(r), n_pre, False)
    res = r - A @ z
    rh = P.T @ res
    zh = coarse_solve(rh)
    z = z + P @ zh
    z = smooth(z, n_post, True)
    return z


def exact_coarse(Ahat: np.ndarray):
    lu = sla.lu_factor(Ahat)
    return lambda rh: sla.lu_solve(lu, rh)


# ---------------------------------------------------------------------------
# outer Krylov methods
# ---------------------------------------------------------------------------
def cg(A, f, x0=None, precond=None, rtol=1e-8, maxit=1000, flexible=False):
    """Preconditioned CG (flexible: Polak-Ribiere beta).

    Returns (x, iterations, history of ||r_k|| / ||r_0||)."""
    x = np.zeros_like(f) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    M = (lambda r: r.copy()) if precond is None else precond
    r = f - A @ x
    r0 = np.linalg.norm(r)
    hist = [1.0]
    if r0 == 0.0:
        return x, 0, hist
    z = M(r)
    p = z.copy()
    rho = r @ z
    it = 0
    while it < maxit:
        q = A @ p
        alpha = rho / (p @ q)
        x = x + alpha * p
        r_old = r
        r = r - alpha * q
        it += 1
        hist.append(np.linalg.norm(r) / r0)
        if hist[-1] <= rtol:
            break
        z = M(r)
        if flexible:
            rho_new = r @ z
            beta = (z @ (r - r_old)) / rho
        else:
            rho_new = r @ z
            beta = rho_new / rho
        p = z + beta * p
        rho = rho_new
    return x, it, hist


def fgmres(A, f, x0=None, precond=None, rtol=1e-8, maxit=1000, restart=30):
    """Flexible GMRES(restart), right preconditioning, MGS, Givens.

    Returns (x, iterations, history of the estimated ||r_k|| / ||r_0||)."""
    x = np.zeros_like(f) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    M = (lambda r: r.copy()) if precond is None else precond
    r = f - A @ x
    r0 = np.linalg.norm(r)
    hist = [1.0]
    if r0 == 0.0:
        return x, 0, hist
    it = 0
    beta = r0
    while it < maxit:
        m = restart
        V = np.zeros((m + 1, f.size))
        Z = np.zeros((m, f.size))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        V[0] = r / beta
        g[0] = beta
        k = 0
        done = False
        for j in range(m):
            Z[j] = M(V[j])
            w = A @ Z[j]
            for i in range(j + 1):
                H[i, j] = w @ V[i]
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            rr = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / rr
            sn[j] = H[j + 1, j] / rr
            hnext = H[j + 1, j]
            H[j, j] = rr
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            k = j + 1
            hist.append(abs(g[j + 1]) / r0)
            if hist[-1] <= rtol or it >= maxit:
                done = True
                break
            V[j + 1] = w / hnext
        y = sla.solve_triangular(H[:k, :k], g[:k], lower=False)
        x = x + Z[:k].T @ y
        if done:
            break
        r = f - A @ x
        beta = np.linalg.norm(r)
        if beta / r0 <= rtol:
            break
    return x, it, hist
