"""GPU parity of the conforming Q1 coarse space (Sec. 2.2.2-2.2.3, App. A.2)
against the CPU oracle, through the C ABI.

  * level 0 of the Q1 hierarchy equals the oracle's Galerkin product
    P^T A P on the trilinear vertex functions, entry by entry (FP64,
    <= 1e-12 relative to the largest entry), with reaction, advection and
    mixed Dirichlet / Neumann faces;
  * every coarser vertex level is the Galerkin product of the level above
    with trilinear interpolation (interpolation matrices built here from
    their definition: every second vertex and the last one kept);
  * the V-cycle with the Q1 coarse space matches the oracle's
    alg hybrid_multigrid with P = nodal interpolation of the trilinears
    and an exact coarse solve (meshes of at most 128 vertices, where the
    library inverts level 0 densely) to 1e-9 in FP64;
  * on deeper hierarchies, many coarse cycles converge to that exact
    coarse solve, and with exact block solves the whole V-cycle is a
    symmetric positive definite operator for b = 0;
  * outer CG with the Q1 V-cycle needs fewer iterations than with P0.
"""
import numpy as np
import pytest

from oracle import dg, solvers
from paper_1805_11930_amd import inputs
from tests.helpers import oracle_problem, rel, spec

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")


def _lib(w):
    from paper_1805_11930_amd import Problem

    return Problem(spec(w))


def stencil_to_dense(dims, S):
    vx, vy, vz = dims
    n = vx * vy * vz
    M = np.zeros((n, n))
    for i in range(n):
        ix, iy, iz = i % vx, (i // vx) % vy, i // (vx * vy)
        for o in range(S.shape[0]):
            jx, jy, jz = ix + o % 3 - 1, iy + (o // 3) % 3 - 1, iz + o // 9 - 1
            if 0 <= jx < vx and 0 <= jy < vy and 0 <= jz < vz:
                M[i, jx + vx * (jy + vy * jz)] += S[o, i]
            else:
                assert S[o, i] == 0.0
    return M


def interp_1d(vf):
    """Linear interpolation from the coarse vertex line: coarse J sits on
    fine min(2J, vf-1)."""
    vc = vf // 2 + 1 if vf > 2 else vf
    P = np.zeros((vf, vc))
    pos = [min(2 * J, vf - 1) for J in range(vc)]
    for i in range(vf):
        if i in pos:
            P[i, pos.index(i)] = 1.0
        else:
            J = max(j for j in range(vc) if pos[j] < i)
            t = (i - pos[J]) / (pos[J + 1] - pos[J])
            P[i, J], P[i, J + 1] = 1 - t, t
    return P


@pytest.mark.parametrize("p,with_b", [(1, False), (2, True), (3, False), (4, True)])
def test_q1_level0_equals_galerkin(p, with_b):
    from paper_1805_11930_amd import DG_COARSE_Q1

    print(f"Q1 level 0 p={p} b={with_b}", flush=True)
    w = inputs.random_case(p, cells=(4, 3, 3), seed=11, with_b=with_b)
    opr = oracle_problem(w)
    ref = solvers.q1_galerkin(dg.assemble(opr), opr)
    P = _lib(w)
    dims, S, _ = P.coarse_stencil(DG_COARSE_Q1, 0)
    assert dims == (5, 4, 4)
    got = stencil_to_dense(dims, S)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    P.close()


def test_q1_coarser_levels_are_galerkin():
    from paper_1805_11930_amd import DG_COARSE_Q1

    w = inputs.random_case(1, cells=(12, 9, 7), seed=12, with_b=True)
    P = _lib(w)
    dims, S, nlev = P.coarse_stencil(DG_COARSE_Q1, 0)
    assert nlev >= 3
    A = stencil_to_dense(dims, S)
    for lev in range(1, nlev):
        cdims, cS, _ = P.coarse_stencil(DG_COARSE_Q1, lev)
        Pi = np.kron(interp_1d(dims[2]), np.kron(interp_1d(dims[1]), interp_1d(dims[0])))
        assert Pi.shape[1] == np.prod(cdims)
        ref = Pi.T @ A @ Pi
        got = stencil_to_dense(cdims, cS)
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
        dims, A = cdims, got
    assert np.prod(dims) <= 128
    P.close()


@pytest.mark.parametrize("p,with_b,npre,npost", [(1, False, 1, 1), (2, False, 1, 1), (3, False, 2, 1),
                                                  (2, True, 1, 2), (4, False, 0, 1), (3, True, 1, 0)])
def test_vcycle_q1_exact_coarse(p, with_b, npre, npost):
    from paper_1805_11930_amd import DG_COARSE_Q1, DG_INNER_CG, DG_INNER_GMRES, mg_opts

    print(f"Q1 V-cycle p={p} b={with_b} pre={npre} post={npost}", flush=True)
    w = inputs.random_case(p, cells=(5, 4, 3), seed=7, with_b=with_b)
    opr = oracle_problem(w)
    A = dg.assemble(opr)
    Db = dg.block_diagonal(A, opr.ncell)
    r = inputs.random_vector(opr.ndof, 36)
    inner = "gmres" if with_b else "cg"
    Pq = solvers.q1_prolongation(opr)
    cs = solvers.exact_coarse(solvers.q1_galerkin(A, opr))
    ref = solvers.vcycle(A, Db, opr, r, cs, n_pre=npre, n_post=npost, omega=0.9, inner=inner, eps=1e-2, restart=12,
                         P=Pq)
    P = _lib(w)
    o = mg_opts(smooth=dict(omega=0.9, eps=1e-2, inner=DG_INNER_GMRES if with_b else DG_INNER_CG, restart=12),
                n_pre=npre, n_post=npost, coarse_space=DG_COARSE_Q1)
    z = P.mg_vcycle(torch.from_numpy(r).cuda(), o)
    assert rel(z.cpu().numpy(), ref) <= 1e-9
    z32 = P.mg_vcycle(torch.from_numpy(r).float().cuda(), o)
    assert rel(z32.cpu().numpy(), ref) <= 1e-3  # FP32 smoother iterations may differ by one near eps
    P.close()


@pytest.mark.parametrize("with_b", [False, True])
def test_q1_many_coarse_cycles_reach_exact_coarse_solve(with_b):
    from paper_1805_11930_amd import DG_COARSE_Q1, DG_INNER_CG, DG_INNER_GMRES, mg_opts

    w = inputs.random_case(2, cells=(8, 6, 5), seed=13, with_b=with_b)
    opr = oracle_problem(w)
    A = dg.assemble(opr)
    Db = dg.block_diagonal(A, opr.ncell)
    r = inputs.random_vector(opr.ndof, 37)
    inner = "gmres" if with_b else "cg"
    cs = solvers.exact_coarse(solvers.q1_galerkin(A, opr))
    ref = solvers.vcycle(A, Db, opr, r, cs, n_pre=1, n_post=1, omega=0.8, inner=inner, eps=1e-2, restart=12,
                         P=solvers.q1_prolongation(opr))
    P = _lib(w)
    assert P.coarse_stencil(DG_COARSE_Q1, 0)[2] >= 2
    base = dict(smooth=dict(omega=0.8, eps=1e-2, inner=DG_INNER_GMRES if with_b else DG_INNER_CG, restart=12),
                coarse_space=DG_COARSE_Q1)
    z1 = P.mg_vcycle(torch.from_numpy(r).cuda(), mg_opts(coarse_cycles=1, **base)).cpu().numpy()
    z40 = P.mg_vcycle(torch.from_numpy(r).cuda(), mg_opts(coarse_cycles=40, **base)).cpu().numpy()
    assert rel(z40, ref) <= 1e-8
    assert rel(z1, ref) > 1e-6  # one cycle is an approximate coarse solve
    P.close()


def test_q1_vcycle_symmetric_with_exact_blocks():
    from paper_1805_11930_amd import DG_COARSE_Q1, DG_INNER_CG, mg_opts

    w = inputs.random_case(2, cells=(8, 6, 5), seed=14, with_b=False)
    P = _lib(w)
    n = P.ndof
    o = mg_opts(smooth=dict(omega=0.8, eps=1e-14, max_inner=4 * 27, inner=DG_INNER_CG), n_pre=2, n_post=2,
                coarse_space=DG_COARSE_Q1, coarse_cycles=2)
    r1 = torch.from_numpy(inputs.random_vector(n, 38)).cuda()
    r2 = torch.from_numpy(inputs.random_vector(n, 39)).cuda()
    z1, z2 = P.mg_vcycle(r1, o), P.mg_vcycle(r2, o)
    a, b = float(r2 @ z1), float(r1 @ z2)
    assert abs(a - b) <= 1e-9 * abs(a)
    assert float(r1 @ z1) > 0 and float(r2 @ z2) > 0
    z12 = P.mg_vcycle(r1 + 2 * r2, o)
    assert rel(z12.cpu().numpy(), (z1 + 2 * z2).cpu().numpy()) <= 1e-10
    P.close()


def test_q1_outer_cg_fewer_iterations_than_p0():
    from paper_1805_11930_amd import DG_COARSE_P0, DG_COARSE_Q1, DG_KRYLOV_FCG, solve_opts

    w = inputs.w1(cells=(8, 8, 8))
    P = _lib(w)
    f = torch.from_numpy(inputs.random_vector(P.ndof, 40)).cuda()
    its = {}
    for cs in (DG_COARSE_P0, DG_COARSE_Q1):
        o = solve_opts(mg=dict(coarse_space=cs), krylov=DG_KRYLOV_FCG, rtol=1e-8)
        u, res = P.solve(f, opts=o)
        assert res.status == 0 and res.rel_residual <= 1e-8
        its[cs] = res.iters
    print("iterations P0 / Q1:", its[DG_COARSE_P0], its[DG_COARSE_Q1], flush=True)
    assert its[DG_COARSE_Q1] < its[DG_COARSE_P0]
    P.close()


def test_q1_rejects_bad_options():
    from paper_1805_11930_amd import mg_opts
    from paper_1805_11930_amd._lib import DgError

    w = inputs.random_case(1, cells=(2, 2, 2), seed=1)
    P = _lib(w)
    r = torch.ones(P.ndof, dtype=torch.float64, device="cuda")
    with pytest.raises(DgError):
        P.mg_vcycle(r, mg_opts(coarse_space=7))
    with pytest.raises(DgError):
        P.mg_vcycle(r, mg_opts(coarse_cycles=-1))
    with pytest.raises(DgError):
        P.coarse_stencil(1, 99)
    P.close()


@pytest.mark.parametrize("space", ["p0", "q1"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("cycles", [1, 3])
def test_coarse_graph_replays_equal_eager(space, prec, cycles):
    """The coarse solve replayed from its captured HIP graph gives the same
    bits as the eager launches, on every replay, with other eager work and
    synchronisations in between (the graph holds kernel nodes only)."""
    from paper_1805_11930_amd import DG_COARSE_P0, DG_COARSE_Q1, mg_opts

    w = inputs.random_case(2, cells=(9, 7, 6), seed=21)
    P = _lib(w)
    dt = torch.float64 if prec == "f64" else torch.float32
    cs = DG_COARSE_Q1 if space == "q1" else DG_COARSE_P0
    assert P.coarse_stencil(cs, 0)[2] >= 2  # a real multilevel coarse cycle
    base = dict(coarse_space=cs, coarse_cycles=cycles)
    rs = [torch.from_numpy(inputs.random_vector(P.ndof, 50 + k)).to(dt).cuda() for k in range(3)]
    eager = [P.mg_vcycle(r, mg_opts(graph=0, **base)).clone() for r in rs]
    junk = torch.empty_like(rs[0])
    for rep in range(3):
        for k, r in enumerate(rs):
            z = P.mg_vcycle(r, mg_opts(graph=1, **base))
            torch.cuda.synchronize()
            assert torch.equal(z, eager[k]), (rep, k)
            P.apply(rs[(k + 1) % 3], junk)  # eager work between replays
            P.mg_vcycle(rs[(k + 2) % 3], mg_opts(graph=0, **base), out=junk)
    P.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("cycles,nu", [(1, 1), (3, 2)])
@pytest.mark.parametrize("cells", [(9, 7, 6), (9, 9, 9), (16, 14, 12)])
def test_fused_small_levels_equal_kernel_per_step(prec, cycles, nu, cells):
    """The single-workgroup cycle of the small vertex levels gives the same
    bits as one kernel per step, whether it takes the whole hierarchy
    (560 vertices on level 0 and the dense bottom; in FP32 also 1000, 216
    and the bottom) or starts below level 0 (3315 vertices; 1000 in FP64,
    whose coefficients exceed what the cycle takes), in eager launches and
    in the replayed coarse graph."""
    from paper_1805_11930_amd import DG_COARSE_Q1, mg_opts

    print(f"fused small levels {prec} cycles={cycles} nu={nu} cells={cells}", flush=True)
    w = inputs.random_case(1, cells=cells, seed=23)
    P = _lib(w)
    _, _, nlev = P.coarse_stencil(DG_COARSE_Q1, 0)
    assert nlev >= 2
    dt = torch.float64 if prec == "f64" else torch.float32
    base = dict(coarse_space=DG_COARSE_Q1, coarse_cycles=cycles, coarse_smooth=nu)
    rs = [torch.from_numpy(inputs.random_vector(P.ndof, 60 + k)).to(dt).cuda() for k in range(2)]
    for r in rs:
        ref = P.mg_vcycle(r, mg_opts(fuse_small_levels=0, **base)).clone()
        for graph in (0, 1, 1):
            z = P.mg_vcycle(r, mg_opts(fuse_small_levels=1, graph=graph, **base))
            torch.cuda.synchronize()
            assert torch.equal(z, ref), graph
    P.close()


def test_fused_small_levels_solve_identical():
    """Outer FCG with the Q1 V-cycle: the same iterations and solution bits
    with and without the single-workgroup small-level cycle."""
    from paper_1805_11930_amd import DG_COARSE_Q1, DG_KRYLOV_FCG, DG_PRECOND_MG, solve_opts

    w = inputs.random_case(2, cells=(12, 10, 8), seed=24)
    P = _lib(w)
    f = torch.from_numpy(inputs.random_vector(P.ndof, 70)).cuda()
    out = []
    for fuse in (0, 1):
        o = solve_opts(krylov=DG_KRYLOV_FCG, precond=DG_PRECOND_MG, precond_precision=1, rtol=1e-8, maxit=200,
                       mg=dict(coarse_space=DG_COARSE_Q1, fuse_small_levels=fuse))
        u, res = P.solve(f, opts=o)
        assert res.status == 0
        out.append((u, res.iters))
    assert out[0][1] == out[1][1]
    assert torch.equal(out[0][0], out[1][0])
    P.close()
