"""Explicit assembly of the WSIPG + upwind DG matrix and right-hand side.

Oracle (test infrastructure only; see the package docstring).

Problem (Sec. 2, eqns linearproblem / boundary_conditions):
    div(b u - K grad u) + c u = f   in a box, u = g on Gamma_D,
    (b u - K grad u) . nu = j on Gamma_N.

The matrix is A_ij = a_h(psi_j, psi_i) (eqn linear_equation) with the
bilinear form split into volume, interior-face and boundary-face parts
(eqn bilinear_form_split), the Ern-Stephansen-Zunino weights omega^+-, the
penalty gamma_F with the harmonic average of delta = nu^T K nu, and the
upwind flux Phi (all in Sec. 2.1).  The right-hand side is l_h (eqn rhs).

Everything here is the plain definition: every local matrix is a sum over
quadrature points of products of basis values / gradients (numpy matrix
products perform the sums), and the local matrices are scattered into a
block-sparse global matrix whose block (T, T') is A_{T,T'} (eqn block_ls).
No sum factorisation is used.

Conventions (shared with the public interface of the library, which is
documented separately):
  * uniform Cartesian box mesh of nx*ny*nz cells, cell index
    c = ix + nx*(iy + ny*iz) (x fastest);
  * in each cell the nodal DOF (jx, jy, jz) has local index
    jx + n*(jy + n*jz), n = p + 1;
  * box faces are numbered 0..5 = -x, +x, -y, +y, -z, +z; each has a
    boundary type 'D' (Dirichlet) or 'N' (Neumann);
  * K is diagonal and constant per cell, or a field K(x) given as a
    callable and evaluated at the quadrature points, either diagonal
    (returning (npts, 3)) or a full symmetric tensor (returning
    (npts, 3, 3)); c likewise; the advection field is affine,
    b(x) = b0 + B x.  With a K field the face quantities
    delta = nu^T K nu, the weights omega and the penalty gamma_F are taken
    pointwise at each face quadrature point, each side's delta from its
    own evaluation of the field (the same value for a continuous field,
    so omega = 1/2 there), and the normal fluxes nu . K grad use the full
    gradient (normal and tangential derivatives) at the face points.
Readings of the paper where it is silent:
  * interior face normal nu points from T- (lower cell index along the
    axis) into T+; ``flip=True`` reverses every interior face (the form is
    invariant under this, which the tests check);
  * upwind tie b_nu = 0 takes u- (the flux is zero either way);
  * on boundary faces the plain K is used (omega- = 1);
  * quadrature is tensor Gauss-Legendre with m = p + 1 points per
    direction on cells and faces (exact for every integrand of this
    problem class).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from . import basis as _basis

AXES = (0, 1, 2)


@dataclass
class Problem:
    """A DG problem on a uniform box mesh (all arrays float64, host)."""

    cells: tuple  # (nx, ny, nz)
    lengths: tuple = (1.0, 1.0, 1.0)
    p: int = 1
    basis: str = "gl"
    bc: tuple = ("D", "D", "D", "D", "D", "D")
    sigma: float | None = None  # penalty prefactor; None -> alpha p (p+d-1), alpha = 1.25
    K: np.ndarray | float = 1.0  # (ncell, 3) diagonal of K per cell, or a scalar
    b0: tuple = (0.0, 0.0, 0.0)
    B: tuple = ((0.0, 0.0, 0.0), (0.0, 0.0, 0.0), (0.0, 0.0, 0.0))
    c: np.ndarray | float = 0.0  # (ncell,) or a scalar
    nq: int | None = None  # quadrature points per direction (default p + 1)
    flip: bool = False  # orientation of interior faces (test of invariance)
    Kfield: object = None  # callable x (npts, 3) -> diagonal of K (npts, 3); overrides K
    cfield: object = None  # callable x (npts, 3) -> c (npts,); overrides c
    _Kc: np.ndarray = field(init=False, repr=False, default=None)
    _cc: np.ndarray = field(init=False, repr=False, default=None)

    def __post_init__(self):
        nc = self.ncell
        K = np.asarray(self.K, dtype=np.float64)
        self._Kc = np.broadcast_to(K if K.ndim == 2 else np.full((nc, 3), float(K)), (nc, 3)).copy()
        c = np.asarray(self.c, dtype=np.float64)
        self._cc = np.broadcast_to(c, (nc,)).copy() if c.ndim else np.full(nc, float(c))
        if len(self.bc) != 6 or any(t not in ("D", "N") for t in self.bc):
            raise ValueError("bc must hold six entries 'D' or 'N'")

    # -- mesh -------------------------------------------------------------
    @property
    def n(self) -> int:
        return self.p + 1

    @property
    def nloc(self) -> int:
        return self.n ** 3

    @property
    def ncell(self) -> int:
        nx, ny, nz = self.cells
        return nx * ny * nz

    @property
    def ndof(self) -> int:
        return self.ncell * self.nloc

    @property
    def h(self) -> np.ndarray:
        return np.array([L / N for L, N in zip(self.lengths, self.cells)], dtype=np.float64)

    @property
    def sigma_p(self) -> float:
        if self.sigma is not None:
            return float(self.sigma)
        return 1.25 * self.p * (self.p + 3 - 1)

    def cell_id(self, ix, iy, iz) -> int:
        nx, ny, _ = self.cells
        return ix + nx * (iy + ny * iz)

    def cell_ijk(self, c):
        nx, ny, _ = self.cells
        return c % nx, (c // nx) % ny, c // (nx * ny)

    def origin(self, c) -> np.ndarray:
        return np.array(self.cell_ijk(c), dtype=np.float64) * self.h

    def Kdiag(self, c) -> np.ndarray:
        return self._Kc[c]

    def creact(self, c) -> float:
        return float(self._cc[c])

    def K_at(self, c, x) -> np.ndarray:
        """K of cell c at physical points x (npts, 3) -> (npts, 3, 3)."""
        if self.Kfield is not None:
            K = np.asarray(self.Kfield(x), dtype=np.float64)
            if K.ndim == 2:
                K = K[:, :, None] * np.eye(3)[None, :, :]
            return K.reshape(len(x), 3, 3)
        return np.broadcast_to(np.diag(self._Kc[c]), (len(x), 3, 3))

    def c_at(self, c, x) -> np.ndarray:
        """c of cell c at physical points x -> (npts,)."""
        if self.cfield is not None:
            return np.asarray(self.cfield(x), dtype=np.float64).reshape(len(x))
        return np.full(len(x), float(self._cc[c]))

    def bfield(self, x: np.ndarray) -> np.ndarray:
        """b at points x[..., 3] -> [..., 3]."""
        return np.asarray(self.b0, dtype=np.float64) + x @ np.asarray(self.B, dtype=np.float64).T

    @property
    def has_b(self) -> bool:
        return bool(np.any(np.asarray(self.b0) != 0) or np.any(np.asarray(self.B) != 0))


def cell_centre_problem(prob: Problem) -> Problem:
    """The same problem with K and c frozen at the cell centres (constant per
    cell): the operator the preconditioner works with when K and c are
    fields (Sec. 4.2: K and c only at cell centres in the preconditioner)."""
    from dataclasses import replace

    if prob.Kfield is None and prob.cfield is None:
        return prob
    centres = np.array([prob.origin(c) + 0.5 * prob.h for c in range(prob.ncell)])
    if prob.Kfield is not None:
        Kc = np.asarray(prob.Kfield(centres), dtype=np.float64)
        K = Kc if Kc.ndim == 2 else np.diagonal(Kc, axis1=1, axis2=2)  # a full tensor keeps its diagonal
    else:
        K = prob._Kc
    cc = prob.cfield(centres) if prob.cfield is not None else prob._cc
    return replace(prob, K=np.asarray(K, dtype=np.float64).reshape(prob.ncell, 3),
                   c=np.asarray(cc, dtype=np.float64).reshape(prob.ncell), Kfield=None, cfield=None)


# ---------------------------------------------------------------------------
# tabulation of basis functions
# ---------------------------------------------------------------------------
class Tables:
    """1-D tables of the nodal basis on [0, 1] and the quadrature rule."""

    def __init__(self, prob: Problem):
        p = prob.p
        self.n = p + 1
        self.m = prob.nq if prob.nq is not None else p + 1
        self.nodes = _basis.basis_nodes(p, prob.basis)
        self.xq, self.wq = _basis.gauss_legendre(self.m)
        self.L = _basis.lagrange_values(self.nodes, self.xq)  # (m, n)
        self.Dl = _basis.lagrange_derivatives(self.nodes, self.xq)  # (m, n)
        self.end_val = [_basis.lagrange_values(self.nodes, [s])[0] for s in (0.0, 1.0)]
        self.end_der = [_basis.lagrange_derivatives(self.nodes, [s])[0] for s in (0.0, 1.0)]


def tensor_tab(Ex, Ey, Ez) -> np.ndarray:
    """M[q, j] = Ex[qx, jx] Ey[qy, jy] Ez[qz, jz], q and j both x-fastest."""
    M = np.einsum("ai,bj,ck->cbakji", Ex, Ey, Ez)
    return M.reshape(Ex.shape[0] * Ey.shape[0] * Ez.shape[0], -1)


def tensor_points(px, py, pz) -> np.ndarray:
    """Tensor grid of points, x fastest: returns (npts, 3)."""
    Z, Y, X = np.meshgrid(pz, py, px, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def tensor_weights(wx, wy, wz) -> np.ndarray:
    return np.einsum("a,b,c->cba", wx, wy, wz).ravel()


def volume_tab(prob: Problem, tab: Tables):
    """Values and physical gradients of all basis functions at the volume
    quadrature points of a cell: Phi (Q, n^3), G[k] (Q, n^3)."""
    h = prob.h
    L, Dl = tab.L, tab.Dl
    Phi = tensor_tab(L, L, L)
    G = [tensor_tab(Dl / h[0], L, L), tensor_tab(L, Dl / h[1], L), tensor_tab(L, L, Dl / h[2])]
    return Phi, G


def face_tab(prob: Problem, tab: Tables, k: int, side: int):
    """Traces on the cell face xi_k = side (0 or 1).

    Returns (Tr, Dk, xi) with Tr[q, j] = phi_j at the face points,
    Dk[q, j] = d/dx_k phi_j (physical) there and xi (Q, 3) the reference
    coordinates of the face points.  Face points: tensor Gauss rule in the
    two tangential directions, x fastest among them.
    """
    h = prob.h
    ev = tab.end_val[side][None, :]
    ed = tab.end_der[side][None, :] / h[k]
    vals = [tab.L, tab.L, tab.L]
    ders = [tab.L, tab.L, tab.L]
    vals[k] = ev
    ders[k] = ed
    Tr = tensor_tab(*vals)
    Dk = tensor_tab(*ders)
    pts = [tab.xq, tab.xq, tab.xq]
    pts[k] = np.array([float(side)])
    xi = tensor_points(*pts)
    return Tr, Dk, xi


def face_grad_tab(prob: Problem, tab: Tables, k: int, side: int):
    """Physical gradients of all basis functions at the points of the face
    xi_k = side: list over l of (Q, n^3) tables of d/dx_l phi_j."""
    h = prob.h
    out = []
    for l in AXES:
        f = [tab.L, tab.L, tab.L]
        f[k] = tab.end_val[side][None, :]
        if l == k:
            f[k] = tab.end_der[side][None, :] / h[k]
        else:
            f[l] = tab.Dl / h[l]
        out.append(tensor_tab(*f))
    return out


def face_flux_tab(prob: Problem, tab: Tables, c: int, k: int, side: int, x: np.ndarray, nu_k: float):
    """(Q, n^3) table of nu . K(x) grad phi_j at the face points x of cell c
    on its face xi_k = side, nu = nu_k e_k: nu_k sum_l K_kl(x) d_l phi_j."""
    Gf = face_grad_tab(prob, tab, k, side)
    Kx = prob.K_at(c, x)
    return nu_k * sum(Kx[:, k, l][:, None] * Gf[l] for l in AXES)


def face_weights(prob: Problem, tab: Tables, k: int) -> np.ndarray:
    """Physical face quadrature weights W^F_q = w_a w_b |F| for axis k."""
    h = prob.h
    ws = [tab.wq, tab.wq, tab.wq]
    ws[k] = np.array([1.0])
    area = np.prod([h[a] for a in AXES if a != k])
    return tensor_weights(*ws) * area


# ---------------------------------------------------------------------------
# local matrices (rows = test function i, columns = trial function j)
# ---------------------------------------------------------------------------
def volume_matrix(prob: Problem, tab: Tables, c: int, Phi, G) -> np.ndarray:
    """(A^v_{T,T})_{ij} = a^v(psi_j, psi_i) on cell T = c:
    sum_q W_q [ (K(x_q) grad phi_j - b phi_j) . grad phi_i + c(x_q) phi_j phi_i ]."""
    h = prob.h
    W = tensor_weights(tab.wq, tab.wq, tab.wq) * np.prod(h)
    xq = prob.origin(c) + tensor_points(tab.xq, tab.xq, tab.xq) * h
    Kq = prob.K_at(c, xq)
    V = np.zeros((Phi.shape[1], Phi.shape[1]))
    for k in AXES:
        for l in AXES:
            if np.any(Kq[:, k, l] != 0.0):
                V += (G[k].T * (W * Kq[:, k, l])) @ G[l]
    if prob.has_b:
        bq = prob.bfield(xq)
        for k in AXES:
            V -= (G[k].T * (W * bq[:, k])) @ Phi
    cq = prob.c_at(c, xq)
    if np.any(cq != 0.0):
        V += (Phi.T * (W * cq)) @ Phi
    return V


def penalty_interior(prob: Problem, k: int, dm, dp):
    """gamma_F = sigma_p <delta-, delta+> |F| / min(|T-|, |T+|) (uniform mesh:
    |F| / |T| = 1 / h_k), <a, b> = 2ab / (a + b); delta scalars or arrays
    over the face points."""
    h = prob.h
    area = np.prod([h[a] for a in AXES if a != k])
    vol = np.prod(h)
    return prob.sigma_p * (2.0 * dm * dp / (dm + dp)) * area / vol


def penalty_boundary(prob: Problem, k: int, d):
    """gamma_F = sigma_p delta |F| / |T| on a Dirichlet face."""
    h = prob.h
    area = np.prod([h[a] for a in AXES if a != k])
    return prob.sigma_p * d * area / np.prod(h)


def interior_face_blocks(prob: Problem, tab: Tables, k: int, cl: int, cu: int):
    """The four blocks a^if(psi_j in T^t, psi_i in T^s) of the interior face
    between the lower cell cl and the upper cell cu along axis k.

    Returns {(row_cell, col_cell): block}.  The face orientation is
    nu = +e_k from T- = cl to T+ = cu, or the reverse when prob.flip.
    """
    h = prob.h
    # side of the face in each cell's reference coordinates
    Tr_l, Dk_l, xi_l = face_tab(prob, tab, k, 1)
    Tr_u, Dk_u, _ = face_tab(prob, tab, k, 0)
    WF = face_weights(prob, tab, k)
    x = prob.origin(cl) + xi_l * h  # physical face points
    if not prob.flip:
        cells = {"-": cl, "+": cu}
        Tr = {"-": Tr_l, "+": Tr_u}
        Dk = {"-": Dk_l, "+": Dk_u}
        nu_k = 1.0
    else:
        cells = {"-": cu, "+": cl}
        Tr = {"-": Tr_u, "+": Tr_l}
        Dk = {"-": Dk_u, "+": Dk_l}
        nu_k = -1.0
    delta = {s: prob.K_at(cells[s], x)[:, k, k] for s in "-+"}  # nu^T K nu at the face points
    side_of = {"-": 1, "+": 0} if not prob.flip else {"-": 0, "+": 1}
    flux = {s: face_flux_tab(prob, tab, cells[s], k, side_of[s], x, nu_k) for s in "-+"}  # nu . K grad phi
    omega = {"-": delta["+"] / (delta["-"] + delta["+"]), "+": delta["-"] / (delta["-"] + delta["+"])}
    gam = penalty_interior(prob, k, delta["-"], delta["+"])
    sgn = {"-": 1.0, "+": -1.0}  # [[v]] = v- - v+
    if prob.has_b:
        bnu = nu_k * prob.bfield(x)[:, k]
    else:
        bnu = np.zeros(WF.shape)
    chi = {"-": (bnu >= 0.0).astype(np.float64)}
    chi["+"] = 1.0 - chi["-"]
    blocks = {}
    for s in "-+":  # test side
        for t in "-+":  # trial side
            F = sgn[s] * (Tr[s].T * (WF * bnu * chi[t])) @ Tr[t]
            F -= sgn[s] * (Tr[s].T * (WF * omega[t])) @ flux[t]
            F -= sgn[t] * (flux[s].T * (WF * omega[s])) @ Tr[t]
            F += sgn[s] * sgn[t] * (Tr[s].T * (WF * gam)) @ Tr[t]
            blocks[(cells[s], cells[t])] = F
    return blocks


def dirichlet_face_matrix(prob: Problem, tab: Tables, c: int, k: int, side: int) -> np.ndarray:
    """a^bf(psi_j, psi_i) on the Dirichlet face xi_k = side of cell c
    (outward normal nu = -e_k for side 0, +e_k for side 1)."""
    h = prob.h
    Tr, Dk, xi = face_tab(prob, tab, k, side)
    WF = face_weights(prob, tab, k)
    nu_k = 1.0 if side == 1 else -1.0
    x = prob.origin(c) + xi * h
    d = prob.K_at(c, x)[:, k, k]
    gam = penalty_boundary(prob, k, d)
    flux = face_flux_tab(prob, tab, c, k, side, x, nu_k)
    Bm = -(Tr.T * WF) @ flux - (flux.T * WF) @ Tr + (Tr.T * (WF * gam)) @ Tr
    if prob.has_b:
        bnu = nu_k * prob.bfield(prob.origin(c) + xi * h)[:, k]
        chi = (bnu >= 0.0).astype(np.float64)
        Bm += (Tr.T * (WF * bnu * chi)) @ Tr
    return Bm


def boundary_faces(prob: Problem, c: int):
    """Yield (box_face, axis, side) for each face of cell c on the box boundary."""
    ijk = prob.cell_ijk(c)
    for k in AXES:
        if ijk[k] == 0:
            yield 2 * k, k, 0
        if ijk[k] == prob.cells[k] - 1:
            yield 2 * k + 1, k, 1


# ---------------------------------------------------------------------------
# global assembly
# ---------------------------------------------------------------------------
def local_blocks(prob: Problem) -> dict:
    """All blocks A_{T,T'} as a dict {(T, T'): dense (n^3, n^3)}."""
    tab = Tables(prob)
    Phi, G = volume_tab(prob, tab)
    blocks: dict = {}

    def add(key, M):
        if key in blocks:
            blocks[key] = blocks[key] + M
        else:
            blocks[key] = M.copy()

    for c in range(prob.ncell):
        add((c, c), volume_matrix(prob, tab, c, Phi, G))
        for bf, k, side in boundary_faces(prob, c):
            if prob.bc[bf] == "D":
                add((c, c), dirichlet_face_matrix(prob, tab, c, k, side))
    nx, ny, nz = prob.cells
    for c in range(prob.ncell):
        ijk = prob.cell_ijk(c)
        for k in AXES:
            if ijk[k] + 1 < prob.cells[k]:
                nb = list(ijk)
                nb[k] += 1
                cu = prob.cell_id(*nb)
                for key, M in interior_face_blocks(prob, tab, k, c, cu).items():
                    add(key, M)
    return blocks


def assemble(prob: Problem) -> sp.bsr_matrix:
    """The DG matrix A (eqn linear_equation) as a BSR matrix, block n^3."""
    blocks = local_blocks(prob)
    nb = prob.nloc
    keys = sorted(blocks)
    rows = np.array([k[0] for k in keys])
    cols = np.array([k[1] for k in keys])
    data = np.stack([blocks[k] for k in keys])
    indptr = np.zeros(prob.ncell + 1, dtype=np.int64)
    np.add.at(indptr, rows + 1, 1)
    indptr = np.cumsum(indptr)
    return sp.bsr_matrix((data, cols, indptr), shape=(prob.ndof, prob.ndof), blocksize=(nb, nb))


def block_diagonal(A: sp.bsr_matrix, ncell: int) -> np.ndarray:
    """D_T = A_{T,T} for every cell, shape (ncell, n^3, n^3)."""
    A = A.tobsr()
    out = np.zeros((ncell,) + A.blocksize)
    for r in range(ncell):
        for idx in range(A.indptr[r], A.indptr[r + 1]):
            if A.indices[idx] == r:
                out[r] = A.data[idx]
    return out


# ---------------------------------------------------------------------------
# right-hand side (eqn rhs) and grid functions
# ---------------------------------------------------------------------------
def assemble_rhs(prob: Problem, f=None, g=None, j=None) -> np.ndarray:
    """l_h(psi_i).  f, g, j are callables of an (npts, 3) array of physical
    points (None means zero).  g is used on Dirichlet faces, j on Neumann
    faces."""
    tab = Tables(prob)
    h = prob.h
    Phi, _ = volume_tab(prob, tab)
    W = tensor_weights(tab.wq, tab.wq, tab.wq) * np.prod(h)
    xi_vol = tensor_points(tab.xq, tab.xq, tab.xq)
    rhs = np.zeros((prob.ncell, prob.nloc))
    for c in range(prob.ncell):
        x0 = prob.origin(c)
        if f is not None:
            rhs[c] += Phi.T @ (W * f(x0 + xi_vol * h))
        for bf, k, side in boundary_faces(prob, c):
            Tr, Dk, xi = face_tab(prob, tab, k, side)
            WF = face_weights(prob, tab, k)
            x = x0 + xi * h
            nu_k = 1.0 if side == 1 else -1.0
            if prob.bc[bf] == "N":
                if j is not None:
                    rhs[c] -= Tr.T @ (WF * j(x))
                continue
            if g is None:
                continue
            gv = g(x)
            d = prob.K_at(c, x)[:, k, k]
            gam = penalty_boundary(prob, k, d)
            flux = face_flux_tab(prob, tab, c, k, side, x, nu_k)
            bnu = nu_k * prob.bfield(x)[:, k] if prob.has_b else np.zeros(WF.shape)
            inflow = (bnu < 0.0).astype(np.float64)  # Phi(0, g, b_nu) = b_nu g when b_nu < 0
            rhs[c] -= Tr.T @ (WF * inflow * bnu * gv)
            rhs[c] -= flux.T @ (WF * gv)
            rhs[c] += Tr.T @ (WF * gam * gv)
    return rhs.ravel()


def node_points(prob: Problem) -> np.ndarray:
    """Physical coordinates of all DOF nodes in global DOF order, (ndof, 3)."""
    tab = Tables(prob)
    xi = tensor_points(tab.nodes, tab.nodes, tab.nodes)
    return np.concatenate([prob.origin(c) + xi * prob.h for c in range(prob.ncell)])


def interpolate(prob: Problem, fun) -> np.ndarray:
    """Nodal interpolant of a callable: the DOF vector u_i = fun(zeta_i)."""
    return fun(node_points(prob))


def l2_error(prob: Problem, u: np.ndarray, exact, extra: int = 2) -> float:
    """||u_h - exact||_{L2} with a tensor Gauss rule of p + 1 + extra points."""
    m = prob.p + 1 + extra
    tab = Tables(prob)
    xq, wq = _basis.gauss_legendre(m)
    L = _basis.lagrange_values(tab.nodes, xq)
    Phi = tensor_tab(L, L, L)
    xi = tensor_points(xq, xq, xq)
    W = tensor_weights(wq, wq, wq) * np.prod(prob.h)
    U = u.reshape(prob.ncell, prob.nloc)
    err2 = 0.0
    for c in range(prob.ncell):
        diff = Phi @ U[c] - exact(prob.origin(c) + xi * prob.h)
        err2 += float(np.sum(W * diff * diff))
    return float(np.sqrt(err2))
