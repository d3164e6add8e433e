"""Outer-iteration work fused into other kernels, through the C ABI, on a
mesh large enough that the per-workgroup partial sums of the last
smoothing sweep (73,728 of them per dot at p = 2, 48 x 48 x 32 cells) are
added in two stages:

  * flexible CG with the V-cycle in FP32 (cast back and dots in the last
    sweep) and in FP64 (dots in the last sweep) reaches the requested
    relative residual, which the library recomputes from scratch in FP64;
  * the two solutions agree to the tolerance, and with the error against
    the exact solution of the Poisson problem each reports the same
    discretisation error;
  * the same holds with the block-SOR sweep, which keeps the separate
    passes, as a reference for the iteration counts.
"""
import numpy as np
import pytest

from paper_1805_11930_amd import inputs
from tests.helpers import spec

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")


@pytest.fixture(scope="module")
def problem():
    from paper_1805_11930_amd import Problem

    w = inputs.w1(cells=(48, 48, 32))
    P = Problem(spec(w))
    f = P.rhs_from_functions(f=w.f)
    exact = torch.from_numpy(np.ascontiguousarray(w.exact(P.node_points()))).cuda()
    yield P, f, exact
    P.close()


def _solve(P, f, exact, prec, sweep):
    from paper_1805_11930_amd import DG_KRYLOV_FCG, DG_PRECOND_MG, solve_opts

    o = solve_opts(krylov=DG_KRYLOV_FCG, precond=DG_PRECOND_MG, precond_precision=prec, rtol=1e-8, maxit=300,
                   smooth=dict(sweep=sweep), u_ref=exact.data_ptr())
    u, res = P.solve(f, opts=o)
    torch.cuda.synchronize()
    return u, res


@pytest.mark.parametrize("sweep", [0, 2])  # block Jacobi (fused epilogue), block SSOR (separate passes)
def test_fused_outer_dots_converge(problem, sweep):
    P, f, exact = problem
    print(f"fused outer dots: {P.ndof} DOF, sweep {sweep}", flush=True)
    out = {}
    for prec in (0, 1):
        u, res = _solve(P, f, exact, prec, sweep)
        assert res.status == 0, (prec, res.status)
        assert res.rel_residual <= 1e-8
        assert np.isfinite(res.error) and res.error < 1e-3
        out[prec] = (u, res)
    (u0, r0), (u1, r1) = out[0], out[1]
    assert abs(r0.iters - r1.iters) <= 2
    d = (torch.linalg.vector_norm(u0 - u1) / torch.linalg.vector_norm(u0)).item()
    assert d <= 1e-6
    assert abs(r0.error - r1.error) <= 1e-3 * r0.error
