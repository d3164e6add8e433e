"""GPU parity of the exact block solve with stored fast-diagonalisation
factors (inner = DG_INNER_FDM, b = 0) against the CPU oracle's dense block
solve (brute force), through the C ABI:

  * x_T = D_T^-1 d_T cell by cell equals numpy's dense solve of the
    oracle's assembled diagonal block, FP64 <= 1e-11, FP32 <= 1e-4, for
    p = 1..4 with reaction, mixed Dirichlet / Neumann faces and
    heterogeneous K;
  * block-Jacobi sweeps and the hybrid V-cycle with the FDM inner solve
    equal the oracle's alg block_jacobi / alg hybrid_multigrid with exact
    block solves;
  * an outer solve with the FDM smoother reaches the tolerance, and the
    FDM option is refused when b != 0.
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


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_fdm_block_solve_equals_dense(p):
    from paper_1805_11930_amd import DG_INNER_FDM, smooth_opts

    print(f"FDM block solve p={p}", flush=True)
    w = inputs.random_case(p, cells=(4, 3, 3), seed=31)
    opr = oracle_problem(w)
    A = dg.assemble(opr)
    Db = dg.block_diagonal(A, opr.ncell)
    d = inputs.random_vector(opr.ndof, 60)
    D = d.reshape(opr.ncell, -1)
    ref = np.concatenate([solvers.block_solve_exact(Db[T], D[T])[0] for T in range(opr.ncell)])
    P = _lib(w)
    o = smooth_opts(inner=DG_INNER_FDM)
    x, it = P.block_solve(torch.from_numpy(d).cuda(), o, iters=True)
    assert rel(x.cpu().numpy(), ref) <= 1e-11
    assert int(it.min()) == 1 and int(it.max()) == 1
    x32 = P.block_solve(torch.from_numpy(d).float().cuda(), o)
    assert rel(x32.cpu().numpy(), ref) <= 1e-4
    P.close()


@pytest.mark.parametrize("p", [2, 4])
def test_fdm_block_jacobi_equals_exact_sweeps(p):
    from paper_1805_11930_amd import DG_INNER_FDM, smooth_opts

    w = inputs.random_case(p, cells=(5, 4, 3), seed=32)
    opr = oracle_problem(w)
    A = dg.assemble(opr)
    Db = dg.block_diagonal(A, opr.ncell)
    f = inputs.random_vector(opr.ndof, 61)
    u0 = inputs.random_vector(opr.ndof, 62)
    ref = solvers.block_jacobi(A, Db, f, u0, omega=0.8, nsweeps=3, inner="exact")
    P = _lib(w)
    got = P.block_smooth(torch.from_numpy(f).cuda(), torch.from_numpy(u0).cuda(),
                         smooth_opts(n_sweeps=3, omega=0.8, inner=DG_INNER_FDM))
    assert rel(got.cpu().numpy(), ref) <= 1e-10
    P.close()


@pytest.mark.parametrize("space", ["p0", "q1"])
def test_fdm_vcycle_equals_oracle(space):
    from paper_1805_11930_amd import DG_COARSE_P0, DG_COARSE_Q1, DG_INNER_FDM, mg_opts

    w = inputs.random_case(3, cells=(5, 4, 3), seed=33)
    opr = oracle_problem(w)
    A = dg.assemble(opr)
    Db = dg.block_diagonal(A, opr.ncell)
    r = inputs.random_vector(opr.ndof, 63)
    if space == "q1":
        Pm, Ah = solvers.q1_prolongation(opr), solvers.q1_galerkin(A, opr)
    else:
        Pm, Ah = solvers.p0_prolongation(opr), solvers.p0_direct(opr)
    ref = solvers.vcycle(A, Db, opr, r, solvers.exact_coarse(Ah), n_pre=1, n_post=1, omega=0.9, inner="exact",
                         P=Pm)
    P = _lib(w)
    o = mg_opts(smooth=dict(omega=0.9, inner=DG_INNER_FDM), coarse_space=DG_COARSE_Q1 if space == "q1" else DG_COARSE_P0)
    z = P.mg_vcycle(torch.from_numpy(r).cuda(), o)
    assert rel(z.cpu().numpy(), ref) <= 1e-10
    z32 = P.mg_vcycle(torch.from_numpy(r).float().cuda(), o)
    assert rel(z32.cpu().numpy(), ref) <= 1e-4
    P.close()


def test_fdm_outer_solve_and_refusal():
    from paper_1805_11930_amd import DG_INNER_FDM, DgError, smooth_opts, solve_opts

    w = inputs.w1(cells=(8, 8, 8))
    P = _lib(w)
    f = torch.from_numpy(inputs.random_vector(P.ndof, 64)).cuda()
    u, res = P.solve(f, opts=solve_opts(rtol=1e-10, smooth=dict(inner=DG_INNER_FDM)))
    assert res.status == 0 and res.rel_residual <= 1e-10
    P.close()
    wb = inputs.random_case(2, cells=(3, 3, 3), seed=34, with_b=True)
    Pb = _lib(wb)
    with pytest.raises(DgError):
        Pb.block_solve(torch.ones(Pb.ndof, dtype=torch.float64, device="cuda"), smooth_opts(inner=DG_INNER_FDM))
    Pb.close()
