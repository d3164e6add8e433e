"""What dg_solve reports about each result, through the C ABI: the FP64
error against a reference solution (u_ref), the inner iterations counted
inside the preconditioner (inner_stats), and the argument checks of the
solve entry points (16-byte alignment, f != u, u_ref distinct)."""
import ctypes

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


def _w1_small():
    from paper_1805_11930_amd import Problem

    w = inputs.w1(cells=(4, 4, 4))
    P = Problem(spec(w))
    f = P.rhs_from_functions(f=w.f)
    exact = torch.from_numpy(np.ascontiguousarray(w.exact(P.node_points()))).cuda()
    return w, P, f, exact


@pytest.mark.parametrize("krylov", [1, 2])  # flexible CG (resident), FGMRES
@pytest.mark.parametrize("prec", [0, 1])
def test_error_against_reference(krylov, prec):
    from paper_1805_11930_amd import solve_opts

    print(f"solve error krylov={krylov} prec={prec}", flush=True)
    w, P, f, exact = _w1_small()
    u, res = P.solve(f, opts=solve_opts(krylov=krylov, precond_precision=prec, rtol=1e-10))
    assert res.error == -1.0  # no reference given
    u2, res2 = P.solve(f, opts=solve_opts(krylov=krylov, precond_precision=prec, rtol=1e-10,
                                          u_ref=exact.data_ptr()))
    un, en = u2.cpu().numpy(), exact.cpu().numpy()
    want = np.linalg.norm(un - en) / np.linalg.norm(en)
    assert abs(res2.error - want) <= 1e-10 * want
    # discretisation error of the p = 2 solution on 4^3 cells: small, not zero
    assert 1e-6 < res2.error < 1e-2
    # the same solve against its own FP64-preconditioned answer
    u3, res3 = P.solve(f, opts=solve_opts(krylov=krylov, precond_precision=prec, rtol=1e-10, u_ref=u2.data_ptr()))
    assert res3.error <= 1e-8
    P.close()


@pytest.mark.parametrize("krylov", [1, 2])
def test_inner_counts_in_solve(krylov):
    from paper_1805_11930_amd import DG_PRECOND_BLOCK, DG_PRECOND_MG, solve_opts

    w, P, f, _ = _w1_small()
    # one block-Jacobi sweep per preconditioner application
    _, res = P.solve(f, opts=solve_opts(krylov=krylov, precond=DG_PRECOND_BLOCK, precond_precision=0, rtol=1e-10,
                                        inner_stats=1, smooth=dict(n_sweeps=1, eps=1e-2)))
    assert res.status == 0
    napps = res.iters + 1 if krylov == 1 else res.n_precond  # CG also preconditions r_0 (and its last r)
    assert res.inner_blocks == P.ncell * napps
    assert 1.0 <= res.inner_avg <= res.inner_max <= P.nloc
    _, res0 = P.solve(f, opts=solve_opts(krylov=krylov, precond=DG_PRECOND_BLOCK, precond_precision=0, rtol=1e-10,
                                         smooth=dict(n_sweeps=1, eps=1e-2)))
    assert res0.inner_blocks == 0 and res0.inner_avg == 0.0
    assert res0.iters == res.iters  # counting does not change the iteration
    # V-cycle: one pre- and one post-smoothing sweep per application
    _, res = P.solve(f, opts=solve_opts(krylov=krylov, precond=DG_PRECOND_MG, precond_precision=1, rtol=1e-10,
                                        inner_stats=1))
    napps = res.iters + 1 if krylov == 1 else res.n_precond
    assert res.inner_blocks == 2 * P.ncell * napps
    assert 1.0 <= res.inner_avg <= res.inner_max
    P.close()


def test_solve_argument_checks():
    from paper_1805_11930_amd import _lib as L, solve_opts

    w, P, f, exact = _w1_small()
    u = torch.zeros_like(f)
    big = torch.zeros(P.ndof + 2, dtype=torch.float64, device="cuda")
    o = solve_opts()
    res = L.SolveResult()
    s = torch.cuda.current_stream().cuda_stream
    lib = P.lib
    assert lib.dg_solve(P.h, f.data_ptr(), f.data_ptr(), ctypes.byref(o), ctypes.byref(res), s) == L.DG_EINVAL
    assert lib.dg_solve(P.h, f.data_ptr(), big.data_ptr() + 8, ctypes.byref(o), ctypes.byref(res), s) == L.DG_EINVAL
    assert b"aligned" in lib.dg_last_error()
    assert lib.dg_solve(P.h, big.data_ptr() + 8, u.data_ptr(), ctypes.byref(o), ctypes.byref(res), s) == L.DG_EINVAL
    o.u_ref = u.data_ptr()
    assert lib.dg_solve(P.h, f.data_ptr(), u.data_ptr(), ctypes.byref(o), ctypes.byref(res), s) == L.DG_EINVAL
    o.u_ref = None
    st = ctypes.c_void_p()
    assert lib.dg_solve_start(P.h, f.data_ptr(), f.data_ptr(), ctypes.byref(o), ctypes.byref(st)) == L.DG_EINVAL
    assert lib.dg_solve_start(P.h, f.data_ptr(), big.data_ptr() + 8, ctypes.byref(o), ctypes.byref(st)) == L.DG_EINVAL
    assert not st.value
    # a valid call still works afterwards
    assert lib.dg_solve(P.h, f.data_ptr(), u.data_ptr(), ctypes.byref(o), ctypes.byref(res), s) == L.DG_OK
    P.close()


@pytest.mark.parametrize("krylov", [1, 2])
def test_phase_times_in_solve(krylov):
    from paper_1805_11930_amd import DG_COARSE_P0, DG_COARSE_Q1, solve_opts

    w, P, f, _ = _w1_small()
    for cs in (DG_COARSE_Q1, DG_COARSE_P0):
        _, res = P.solve(f, opts=solve_opts(krylov=krylov, rtol=1e-10, inner_stats=1, mg=dict(coarse_space=cs)))
        phases = (res.t_smoother, res.t_restrict, res.t_coarse, res.t_prolong)
        assert all(t >= 0.0 for t in phases)
        assert res.t_smoother > 0.0 and res.t_restrict > 0.0 and res.t_coarse > 0.0
        if cs == DG_COARSE_Q1:
            assert res.t_prolong > 0.0
        # the phases lie inside the timed preconditioner applications (the
        # first application of CG, on r_0, is not among those)
        assert sum(phases) <= res.t_solve
        _, res0 = P.solve(f, opts=solve_opts(krylov=krylov, rtol=1e-10, mg=dict(coarse_space=cs)))
        assert (res0.t_smoother, res0.t_restrict, res0.t_coarse, res0.t_prolong) == (0.0, 0.0, 0.0, 0.0)
    P.close()
