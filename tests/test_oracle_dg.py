"""Pins of the oracle's DG matrix and right-hand side (CPU only).

What is pinned and by what (Sec. 2.1: eqns bilinear_form_split and rhs,
the weights omega^+-, the penalty gamma_F and the upwind flux Phi):
  * symmetry and positive definiteness of A for b = 0 (WSIPG is symmetric);
  * Galerkin consistency: for any global polynomial u in Q_p, constant K,
    affine divergence-free b and constant c, l_h - A u_I = 0 exactly
    (volume, consistency terms, weights summing to one, upwind flux,
    Dirichlet and Neumann data);
  * hand-computed closed forms of a_h on simple functions that isolate
    the penalty gamma_F (P0 indicators) and the weights omega^+- (a ramp
    across a face with a jump in K);
  * (A 1)_T = 0 on cells without Dirichlet faces for any K and any
    divergence-free b (conservation);
  * the upwind energy identity u^T (A - A_{b=0}) u = 1/2 sum_F |b_nu| [[u]]^2
    + boundary terms;
  * invariance under flipping every interior face normal;
  * convergence O(h^(p+1)) in L2 for a smooth manufactured solution
    (observed rate in [p + 0.7, p + 1.3] on the finest pair of meshes);
  * the P0 Galerkin product P^T A P equals the direct evaluation of a_h on
    P0 indicators (App. A.1);
  * coefficient fields (Sec. 4.2): a constant field gives the cell-constant
    matrix and right-hand side; with K(x) = diag(P_1(x), P_2(y), P_3(z)),
    P_k quadratic, every integrand is exact, so Q_p solutions are
    reproduced (this fails if K is frozen anywhere); symmetric positive
    definite; L2 rates p+1 for a smooth solution; the cell-centre problem
    of the preconditioner holds the field's centre values;
  * full-tensor fields K(x) = sum_m P_m(x_m) n_m n_m^T: with n = I they give
    the diagonal field's matrix; with a rotated basis and linear P_m every
    integrand (cross derivatives included) is exact, so Q_p solutions are
    reproduced -- this fails if the cross-derivative volume terms or the
    tangential derivatives in the face fluxes are dropped; SPD; L2 rate
    p + 1 for a smooth solution with quadratic P_m.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import dg, solvers


def rand_problem(p, cells=(3, 2, 2), seed=0, **kw):
    rng = np.random.default_rng(seed)
    nc = int(np.prod(cells))
    args = dict(cells=cells, lengths=(1.0, 0.7, 1.3), p=p, K=np.exp(rng.normal(size=(nc, 3))),
                c=np.abs(rng.normal(size=nc)))
    args.update(kw)
    return dg.Problem(**args)


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("sigma", [None, 12.0])
def test_symmetric_positive_definite(p, sigma):
    pr = rand_problem(p, sigma=sigma, bc=("D", "N", "D", "D", "N", "D"))
    A = dg.assemble(pr).toarray()
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    np.linalg.cholesky(A)  # raises if not SPD


def test_default_penalty_factor():
    for p in range(1, 6):
        assert dg.Problem(cells=(1, 1, 1), p=p).sigma_p == pytest.approx(1.25 * p * (p + 2))


def _poly_case(p, rng):
    """A random polynomial of degree <= p in each variable (u in Q_p)."""
    C = rng.normal(size=(p + 1, p + 1, p + 1))

    def u(x):
        out = np.zeros(len(x))
        for a in range(p + 1):
            for b in range(p + 1):
                for c in range(p + 1):
                    out += C[a, b, c] * x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** c
        return out

    def grad(x):
        g = np.zeros((len(x), 3))
        for a in range(p + 1):
            for b in range(p + 1):
                for c in range(p + 1):
                    m = C[a, b, c]
                    if a:
                        g[:, 0] += m * a * x[:, 0] ** (a - 1) * x[:, 1] ** b * x[:, 2] ** c
                    if b:
                        g[:, 1] += m * b * x[:, 0] ** a * x[:, 1] ** (b - 1) * x[:, 2] ** c
                    if c:
                        g[:, 2] += m * c * x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** (c - 1)
        return g

    def hess_diag(x):
        hd = np.zeros((len(x), 3))
        for a in range(p + 1):
            for b in range(p + 1):
                for c in range(p + 1):
                    m = C[a, b, c]
                    if a > 1:
                        hd[:, 0] += m * a * (a - 1) * x[:, 0] ** (a - 2) * x[:, 1] ** b * x[:, 2] ** c
                    if b > 1:
                        hd[:, 1] += m * b * (b - 1) * x[:, 0] ** a * x[:, 1] ** (b - 2) * x[:, 2] ** c
                    if c > 1:
                        hd[:, 2] += m * c * (c - 1) * x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** (c - 2)
        return hd

    return u, grad, hess_diag


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("with_b", [False, True])
def test_polynomial_reproduction(p, with_b):
    rng = np.random.default_rng(10 + p)
    K = np.array([1.3, 0.7, 2.0])
    cvals = 0.4
    # divergence-free affine field: trace(B) = 0
    b0 = (0.2, -0.1, 0.3) if with_b else (0.0, 0.0, 0.0)
    B = ((0.1, 1.0, 0.0), (-1.0, 0.2, 0.5), (0.3, 0.0, -0.3)) if with_b else ((0,) * 3,) * 3
    bc = ("D", "N", "D", "D", "N", "D")
    pr = dg.Problem(cells=(3, 2, 2), lengths=(1.0, 0.7, 1.3), p=p, K=np.tile(K, (12, 1)), b0=b0, B=B,
                    c=cvals, bc=bc)
    u, grad, hd = _poly_case(p, rng)

    def f(x):  # div(b u - K grad u) + c u with div b = 0
        return -(hd(x) @ K) + np.sum(pr.bfield(x) * grad(x), axis=1) + cvals * u(x)

    def j(x):  # (b u - K grad u) . nu on the Neumann faces +x and -z
        flux = pr.bfield(x) * u(x)[:, None] - grad(x) * K
        out = np.full(len(x), np.nan)
        on_px = np.isclose(x[:, 0], 1.0)
        on_mz = np.isclose(x[:, 2], 0.0)
        out[on_px] = flux[on_px, 0]
        out[on_mz] = -flux[on_mz, 2]
        assert not np.isnan(out).any()
        return out

    A = dg.assemble(pr)
    rhs = dg.assemble_rhs(pr, f=f, g=u, j=j)
    uI = dg.interpolate(pr, u)
    assert np.abs(rhs - A @ uI).max() <= 1e-13 * np.abs(rhs).max()


def test_penalty_closed_form_p0():
    """a_h(1_T, 1_T) and a_h(1_T', 1_T) for b = 0, c = 0 on two cells along x.

    h = (0.5, 1, 1), K- = diag(1, 2, 4), K+ = diag(3, 1, 1), sigma = 2,
    all faces Dirichlet.  Interior face (|F| = 1, |T| = 0.5):
    gamma = 2 * <1, 3> * 1 / 0.5 = 2 * 1.5 * 2 = 6, contribution 6 * |F| = 6.
    Dirichlet faces of T-: -x: gamma = 2*1*1/0.5 = 4, |F| = 1 -> 4;
    +-y: gamma = 2*2*0.5/0.5 = 4, |F| = 0.5 -> 2 each; +-z: 2*4*0.5/0.5 = 8,
    |F| = 0.5 -> 4 each.  Total for T-: 6 + 4 + 2*2 + 2*4 = 22.
    T+: interior 6; +x: 2*3*1/0.5 = 12 -> 12; +-y: 2*1*.5/.5 = 2 -> 1 each;
    +-z: 2 -> 1 each.  Total 6 + 12 + 4 = 22.  Off-diagonal: -6.
    """
    K = np.array([[1.0, 2.0, 4.0], [3.0, 1.0, 1.0]])
    for p in (1, 2, 3):
        pr = dg.Problem(cells=(2, 1, 1), lengths=(1.0, 1.0, 1.0), p=p, K=K, sigma=2.0)
        A = dg.assemble(pr)
        P = solvers.p0_prolongation(pr)
        Ah = np.asarray((P.T @ (A @ P.toarray())))
        np.testing.assert_allclose(Ah, [[22.0, -6.0], [-6.0, 22.0]], rtol=1e-13)


def test_weights_closed_form():
    """Ramp u = (x - x_F) on T-, zero on T+; v = 1 on T+ (p = 1, b = 0).

    Only the consistency term survives: a_h(u, v) = -({K grad u}_omega . nu)
    [[v]] |F| = omega- K- |F| = K- K+ / (K- + K+) |F|.  With K-_xx = 2,
    K+_xx = 6, |F| = 0.7 * 1.3: 2*6/8 * 0.91 = 1.365.  (Swapped weights
    would give K-^2/(K- + K+) |F| = 0.455.)
    """
    K = np.array([[2.0, 1.0, 1.0], [6.0, 5.0, 0.3]])
    pr = dg.Problem(cells=(2, 1, 1), lengths=(1.0, 0.7, 1.3), p=1, K=K, sigma=3.0)
    A = dg.assemble(pr)
    X = dg.node_points(pr)
    nl = pr.nloc
    u = np.zeros(pr.ndof)
    u[:nl] = X[:nl, 0] - 0.5
    v = np.zeros(pr.ndof)
    v[nl:] = 1.0
    assert v @ (A @ u) == pytest.approx(2 * 6 / 8 * 0.7 * 1.3, rel=1e-13)
    assert u @ (A @ v) == pytest.approx(2 * 6 / 8 * 0.7 * 1.3, rel=1e-13)


@pytest.mark.parametrize("p", [1, 2])
def test_conservation_rows(p):
    """(A 1)_T = 0 for cells without Dirichlet faces (c = 0, div b = 0)."""
    rng = np.random.default_rng(3)
    cells = (4, 3, 3)
    nc = 36
    pr = dg.Problem(cells=cells, p=p, K=np.exp(2 * rng.normal(size=(nc, 3))), b0=(0.3, -0.2, 0.1),
                    B=((0.5, 0.2, 0.0), (0.1, -0.2, 1.0), (0.0, 0.4, -0.3)), c=0.0)
    A = dg.assemble(pr)
    r = (A @ np.ones(pr.ndof)).reshape(nc, -1)
    scale = np.abs(A.data).max()
    for c in range(nc):
        ijk = pr.cell_ijk(c)
        if all(0 < ijk[k] < cells[k] - 1 for k in range(3)):
            assert np.abs(r[c]).max() <= 1e-13 * scale


@pytest.mark.parametrize("p", [1, 2])
def test_upwind_energy_identity(p):
    rng = np.random.default_rng(4)
    bc = ("D", "N", "D", "N", "D", "D")
    b0 = (0.3, -0.7, 0.2)
    B = ((0.5, 1.0, 0.0), (-1.0, -0.2, 0.5), (0.3, 0.0, -0.3))
    kw = dict(cells=(3, 3, 2), lengths=(1.0, 1.0, 1.0), p=p, K=np.exp(rng.normal(size=(18, 3))), c=0.2, bc=bc)
    pb = dg.Problem(b0=b0, B=B, **kw)
    p0 = dg.Problem(**kw)
    Ab, A0 = dg.assemble(pb), dg.assemble(p0)
    u = rng.normal(size=pb.ndof)
    lhs = u @ ((Ab - A0) @ u)
    # right side: 1/2 sum_int |b_nu| [[u]]^2 + 1/2 sum_D |b_nu| u^2 - 1/2 sum_N b_nu u^2
    tab = dg.Tables(pb)
    U = u.reshape(pb.ncell, -1)
    rhs = 0.0
    for c in range(pb.ncell):
        ijk = pb.cell_ijk(c)
        for k in range(3):
            WF = dg.face_weights(pb, tab, k)
            if ijk[k] + 1 < pb.cells[k]:
                nb = list(ijk)
                nb[k] += 1
                cu = pb.cell_id(*nb)
                Tl, _, xi = dg.face_tab(pb, tab, k, 1)
                Tu, _, _ = dg.face_tab(pb, tab, k, 0)
                bnu = pb.bfield(pb.origin(c) + xi * pb.h)[:, k]
                jump = Tl @ U[c] - Tu @ U[cu]
                rhs += 0.5 * np.sum(WF * np.abs(bnu) * jump**2)
        for bf, k, side in dg.boundary_faces(pb, c):
            Tr, _, xi = dg.face_tab(pb, tab, k, side)
            WF = dg.face_weights(pb, tab, k)
            bnu = (1.0 if side else -1.0) * pb.bfield(pb.origin(c) + xi * pb.h)[:, k]
            tr = Tr @ U[c]
            if bc[bf] == "D":
                rhs += 0.5 * np.sum(WF * np.abs(bnu) * tr**2)
            else:
                rhs -= 0.5 * np.sum(WF * bnu * tr**2)
    assert lhs == pytest.approx(rhs, rel=1e-12)


@pytest.mark.parametrize("p", [1, 2])
def test_orientation_invariance(p):
    kw = dict(b0=(0.3, -0.7, 0.2), B=((0.5, 1.0, 0.0), (-1.0, -0.2, 0.5), (0.3, 0.0, -0.3)))
    a = rand_problem(p, seed=5, **kw)
    b = rand_problem(p, seed=5, flip=True, **kw)
    Aa, Ab = dg.assemble(a).toarray(), dg.assemble(b).toarray()
    assert np.abs(Aa - Ab).max() <= 1e-14 * np.abs(Aa).max()


@pytest.mark.parametrize("with_b", [False, True])
def test_p0_galerkin_equals_direct(with_b):
    kw = {}
    if with_b:
        kw = dict(b0=(0.3, -0.7, 0.2), B=((0.5, 1.0, 0.0), (-1.0, -0.2, 0.5), (0.3, 0.0, -0.3)))
    pr = rand_problem(2, cells=(3, 3, 2), seed=6, bc=("D", "N", "D", "D", "N", "D"), **kw)
    A = dg.assemble(pr)
    G = solvers.p0_galerkin(A, pr)
    Dd = solvers.p0_direct(pr)
    assert np.abs(G - Dd).max() <= 1e-13 * np.abs(G).max()


@pytest.mark.parametrize("p,Ns", [(1, (4, 8)), (2, (2, 4, 8)), (3, (2, 4))])
def test_l2_convergence(p, Ns):
    """Manufactured u = sin(pi x) sin(pi y) sin(pi z), K = I, Dirichlet 0."""
    pi = np.pi

    def uex(x):
        return np.sin(pi * x[:, 0]) * np.sin(pi * x[:, 1]) * np.sin(pi * x[:, 2])

    errs = []
    for N in Ns:
        pr = dg.Problem(cells=(N, N, N), p=p, sigma=2 * p * (p + 1))
        A = dg.assemble(pr).tocsc()
        rhs = dg.assemble_rhs(pr, f=lambda x: 3 * pi**2 * uex(x))
        u = spla.spsolve(A, rhs)
        errs.append(dg.l2_error(pr, u, uex))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] >= p + 0.7, (errs, rates)
    assert rates[-1] <= p + 1.3, (errs, rates)


# ---------------------------------------------------------------------------
# coefficient fields K(x), c(x) at the quadrature points (Sec. 4.2)
# ---------------------------------------------------------------------------
def _axis_field(q0, q1, q2):
    """K(x) = diag(P_1(x), P_2(y), P_3(z)), P_k(s) = q0_k + q1_k s + q2_k s^2,
    and its derivative dP_k/dx_k."""
    q0, q1, q2 = (np.asarray(v, dtype=np.float64) for v in (q0, q1, q2))
    return (lambda x: q0 + q1 * x + q2 * x ** 2), (lambda x: q1 + 2.0 * q2 * x)


FIELD = ((1.0, 0.5, 2.0), (0.3, -0.2, 0.1), (3.0, 1.0, 0.5))


def test_constant_field_equals_cell_constant_coefficients():
    K0 = np.array([1.3, 0.7, 2.0])
    bc = ("D", "N", "D", "D", "N", "D")
    a = dg.Problem(cells=(3, 2, 2), lengths=(1.0, 0.7, 1.3), p=2, K=np.tile(K0, (12, 1)), c=0.4, bc=bc,
                   b0=(0.2, -0.1, 0.3))
    b = dg.Problem(cells=(3, 2, 2), lengths=(1.0, 0.7, 1.3), p=2, bc=bc, b0=(0.2, -0.1, 0.3),
                   Kfield=lambda x: np.tile(K0, (len(x), 1)), cfield=lambda x: np.full(len(x), 0.4))
    Aa, Ab = dg.assemble(a).toarray(), dg.assemble(b).toarray()
    assert np.abs(Aa - Ab).max() <= 1e-14 * np.abs(Aa).max()
    g = lambda x: np.sin(x[:, 0]) + x[:, 1] * x[:, 2]
    ra, rb = dg.assemble_rhs(a, f=g, g=g, j=g), dg.assemble_rhs(b, f=g, g=g, j=g)
    assert np.abs(ra - rb).max() <= 1e-14 * np.abs(ra).max()


@pytest.mark.parametrize("p", [1, 2, 3])
def test_field_polynomial_reproduction(p):
    # every integrand is a polynomial of degree <= 2p per direction for a
    # quadratic P_k(x_k) and u in Q_p, so the p+1-point Gauss rule is exact
    # and the consistent form reproduces u
    rng = np.random.default_rng(40 + p)
    K, dK = _axis_field(*FIELD)
    c0 = 0.4
    bc = ("D", "N", "D", "D", "N", "D")
    pr = dg.Problem(cells=(3, 2, 2), lengths=(1.0, 0.7, 1.3), p=p, bc=bc, Kfield=K,
                    cfield=lambda x: np.full(len(x), c0))
    u, grad, hd = _poly_case(p, rng)

    def f(x):  # -div(K grad u) + c u, K_kk depending on x_k only
        return -np.sum(dK(x) * grad(x) + K(x) * hd(x), axis=1) + c0 * u(x)

    def j(x):  # -K grad u . nu on the Neumann faces +x and -z
        flux = -K(x) * grad(x)
        out = np.full(len(x), np.nan)
        on_px = np.isclose(x[:, 0], 1.0)
        on_mz = np.isclose(x[:, 2], 0.0)
        out[on_px] = flux[on_px, 0]
        out[on_mz] = -flux[on_mz, 2]
        assert not np.isnan(out).any()
        return out

    A = dg.assemble(pr)
    rhs = dg.assemble_rhs(pr, f=f, g=u, j=j)
    uI = dg.interpolate(pr, u)
    assert np.abs(rhs - A @ uI).max() <= 1e-12 * np.abs(rhs).max()


def test_field_operator_symmetric_positive_definite():
    K, _ = _axis_field(*FIELD)
    pr = dg.Problem(cells=(3, 2, 2), p=2, Kfield=K, cfield=lambda x: 1e-8 * np.sum(x ** 2, axis=1))
    A = dg.assemble(pr).toarray()
    assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()
    assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0


@pytest.mark.parametrize("p,Ns", [(1, (4, 8)), (2, (2, 4))])
def test_field_l2_convergence(p, Ns):
    pi = np.pi
    K, dK = _axis_field(*FIELD)

    def uex(x):
        return np.sin(pi * x[:, 0]) * np.sin(pi * x[:, 1]) * np.sin(pi * x[:, 2])

    def grad(x):
        s = np.sin(pi * x)
        cs = np.cos(pi * x)
        return pi * np.stack([cs[:, 0] * s[:, 1] * s[:, 2], s[:, 0] * cs[:, 1] * s[:, 2],
                              s[:, 0] * s[:, 1] * cs[:, 2]], axis=1)

    def f(x):
        return -np.sum(dK(x) * grad(x), axis=1) + pi ** 2 * np.sum(K(x), axis=1) * uex(x)

    errs = []
    for N in Ns:
        pr = dg.Problem(cells=(N, N, N), p=p, Kfield=K)
        u = spla.spsolve(dg.assemble(pr).tocsc(), dg.assemble_rhs(pr, f=f))
        errs.append(dg.l2_error(pr, u, uex))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert p + 0.6 <= rates[-1] <= p + 1.4, (errs, rates)


def test_cell_centre_problem():
    K, _ = _axis_field(*FIELD)
    pr = dg.Problem(cells=(3, 2, 2), lengths=(1.0, 0.7, 1.3), p=1, Kfield=K,
                    cfield=lambda x: 2.0 + np.sum(x ** 2, axis=1))
    pc = dg.cell_centre_problem(pr)
    for c in (0, 5, 11):
        xc = pr.origin(c) + 0.5 * pr.h
        assert np.allclose(pc.Kdiag(c), K(xc[None, :])[0], rtol=1e-15)
        assert pc.creact(c) == pytest.approx(2.0 + xc @ xc, rel=1e-15)
    with pytest.raises(ValueError):
        solvers.p0_direct(pr)
    assert solvers.p0_direct(pc).shape == (12, 12)


def _rotated_field(q0, q1, q2, n):
    """K(x) = sum_m P_m(x_m) n_m n_m^T (rows of n orthonormal) as a full
    tensor, and the divergence of K grad u for a polynomial u."""
    q0, q1, q2 = (np.asarray(v, dtype=np.float64) for v in (q0, q1, q2))
    n = np.asarray(n, dtype=np.float64)

    def K(x):
        P = q0 + q1 * x + q2 * x ** 2  # (npts, 3): P_m(x_m)
        return np.einsum("qm,mk,ml->qkl", P, n, n)

    def dK(x):  # d/dx_j K_kl = P_j'(x_j) n_jk n_jl
        dP = q1 + 2.0 * q2 * x
        return np.einsum("qj,jk,jl->qjkl", dP, n, n)

    return K, dK


def _rotation(a, b, c):
    ca, sa, cb, sb, cc, sc = np.cos(a), np.sin(a), np.cos(b), np.sin(b), np.cos(c), np.sin(c)
    Rz = np.array([[ca, -sa, 0], [sa, ca, 0], [0, 0, 1]])
    Ry = np.array([[cb, 0, sb], [0, 1, 0], [-sb, 0, cb]])
    Rx = np.array([[1, 0, 0], [0, cc, -sc], [0, sc, cc]])
    return Rz @ Ry @ Rx


def test_full_tensor_field_with_axis_directions_equals_diagonal_field():
    Kd, _ = _axis_field(*FIELD)
    Kf, _ = _rotated_field(*FIELD, np.eye(3))
    bc = ("D", "N", "D", "D", "N", "D")
    a = dg.Problem(cells=(3, 2, 2), lengths=(1.0, 0.7, 1.3), p=2, bc=bc, Kfield=Kd)
    b = dg.Problem(cells=(3, 2, 2), lengths=(1.0, 0.7, 1.3), p=2, bc=bc, Kfield=Kf)
    Aa, Ab = dg.assemble(a).toarray(), dg.assemble(b).toarray()
    assert np.abs(Aa - Ab).max() <= 1e-14 * np.abs(Aa).max()


@pytest.mark.parametrize("p", [1, 2, 3])
def test_rotated_field_polynomial_reproduction(p):
    # K_kl depends on one coordinate x_m, linearly here (q2 = 0); the
    # integrands K_kl d_l u d_k v have degree <= 2p + 1 in every direction,
    # so the p+1-point rule is exact and Q_p solutions are reproduced.  This
    # pins the cross-derivative volume terms and the tangential derivatives
    # in the face fluxes (dropping either breaks it).
    rng = np.random.default_rng(50 + p)
    n = _rotation(0.4, -0.7, 1.1)
    K, dK = _rotated_field((1.0, 0.5, 2.0), (0.3, -0.2, 0.1), (0.0, 0.0, 0.0), n)
    bc = ("D", "N", "D", "D", "N", "D")
    pr = dg.Problem(cells=(3, 2, 2), lengths=(1.0, 0.7, 1.3), p=p, bc=bc, Kfield=K)
    u, grad, hd = _poly_case(p, rng)

    def hess(x):  # full Hessian of the polynomial by central differences of the exact gradient
        e = 1e-6
        Hm = np.zeros((len(x), 3, 3))
        for j in range(3):
            dx = np.zeros(3)
            dx[j] = e
            Hm[:, :, j] = (grad(x + dx) - grad(x - dx)) / (2 * e)
        return Hm

    def f(x):  # -div(K grad u) = -sum_kl (d_k K_kl d_l u + K_kl d_kl u)
        g = grad(x)
        div = np.einsum("qkkl,ql->q", dK(x), g) + np.einsum("qkl,qkl->q", K(x), hess(x))
        return -div

    def j(x):
        flux = -np.einsum("qkl,ql->qk", K(x), grad(x))
        out = np.full(len(x), np.nan)
        on_px = np.isclose(x[:, 0], 1.0)
        on_mz = np.isclose(x[:, 2], 0.0)
        out[on_px] = flux[on_px, 0]
        out[on_mz] = -flux[on_mz, 2]
        assert not np.isnan(out).any()
        return out

    A = dg.assemble(pr)
    rhs = dg.assemble_rhs(pr, f=f, g=u, j=j)
    uI = dg.interpolate(pr, u)
    # central differences of the exact gradient of a cubic are exact up to
    # ~1e-10 relative rounding
    assert np.abs(rhs - A @ uI).max() <= 1e-8 * np.abs(rhs).max()


def test_rotated_field_spd_and_convergence():
    n = _rotation(0.4, -0.7, 1.1)
    K, dK = _rotated_field(*FIELD, n)
    pr = dg.Problem(cells=(3, 2, 2), p=2, Kfield=K)
    A = dg.assemble(pr).toarray()
    assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()
    assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0
    pi = np.pi

    def uex(x):
        return np.sin(pi * x[:, 0]) * np.sin(pi * x[:, 1]) * np.sin(pi * x[:, 2])

    def grad(x):
        s, cs = np.sin(pi * x), np.cos(pi * x)
        return pi * np.stack([cs[:, 0] * s[:, 1] * s[:, 2], s[:, 0] * cs[:, 1] * s[:, 2],
                              s[:, 0] * s[:, 1] * cs[:, 2]], axis=1)

    def hess(x):
        s, cs = np.sin(pi * x), np.cos(pi * x)
        H = np.empty((len(x), 3, 3))
        for a in range(3):
            for b in range(3):
                t = np.ones(len(x))
                for m in range(3):
                    if m == a and m == b:
                        t = t * -s[:, m]
                    elif m == a or m == b:
                        t = t * cs[:, m]
                    else:
                        t = t * s[:, m]
                H[:, a, b] = pi ** 2 * t
        return H

    def f(x):
        return -(np.einsum("qkkl,ql->q", dK(x), grad(x)) + np.einsum("qkl,qkl->q", K(x), hess(x)))

    errs = []
    for N in (2, 4):
        pr = dg.Problem(cells=(N, N, N), p=2, Kfield=K)
        u = spla.spsolve(dg.assemble(pr).tocsc(), dg.assemble_rhs(pr, f=f))
        errs.append(dg.l2_error(pr, u, uex))
    rate = np.log2(errs[0] / errs[1])
    assert 2.6 <= rate <= 3.4, (errs, rate)
