"""dg_block_smooth_noalloc (fixed device scratch, no allocation) gives the
same smoothing steps as dg_block_smooth, through the C ABI: block-Jacobi
with several sweeps (ping-pong vector in the scratch) and block-SOR, with
per-cell iteration statistics (counts in the scratch), FP64 and FP32, on two
calls in a row, the second on a smaller problem; and it refuses inputs
that need more than its fixed scratch."""
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


def _smooth(P, entry, f, u_in, opts):
    from paper_1805_11930_amd import _lib as L

    out = torch.empty_like(f)
    st = L.SmoothStats()
    prec = L.DG_FP64 if f.dtype == torch.float64 else L.DG_FP32
    fn = getattr(P.lib, entry)
    L._check(fn(P.h, prec, f.data_ptr(), u_in.data_ptr(), out.data_ptr(), ctypes.byref(opts), ctypes.byref(st),
                torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return out.cpu().numpy(), (st.blocks, st.inner_total, st.inner_max)


CASES = [
    # (degree, cells, advection, options)
    (3, (6, 5, 4), True, dict(n_sweeps=3, inner=1, restart=8, inner_precond=1)),
    (2, (3, 3, 2), True, dict(n_sweeps=2, inner=1, restart=8, inner_precond=1)),
]


@pytest.mark.parametrize("dtype", ["float64", "float32"])
@pytest.mark.parametrize("sweep", [0, 2])  # block-Jacobi, block-SSOR
def test_noalloc_equals_block_smooth_twice(dtype, sweep):
    from paper_1805_11930_amd import Problem, smooth_opts

    dt = getattr(torch, dtype)
    tol = 1e-12 if dtype == "float64" else 1e-5
    for k, (p, cells, with_b, kw) in enumerate(CASES):  # the second call has the smaller input
        print(f"noalloc {dtype} sweep={sweep} call {k}: p={p} cells={cells}", flush=True)
        w = inputs.random_case(p, cells=cells, seed=7 + k, with_b=with_b)
        P = Problem(spec(w))
        f = torch.from_numpy(inputs.random_vector(P.ndof, 70 + k)).to(dtype=dt, device="cuda")
        u0 = torch.from_numpy(inputs.random_vector(P.ndof, 80 + k)).to(dtype=dt, device="cuda")
        o = smooth_opts(eps=1e-2, sweep=sweep, **kw)
        ref, st_ref = _smooth(P, "dg_block_smooth", f, u0, o)
        got, st_got = _smooth(P, "dg_block_smooth_noalloc", f, u0, o)
        err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        assert err <= tol, (k, err)
        assert st_got == st_ref, (k, st_got, st_ref)
        assert st_ref[0] == P.ncell * kw["n_sweeps"] * (2 if sweep == 2 else 1)
        P.close()


def test_noalloc_pcg_sweeps_then_smaller():
    from paper_1805_11930_amd import Problem, smooth_opts

    for k, (p, cells) in enumerate([(4, (5, 4, 3)), (1, (2, 2, 3))]):
        print(f"noalloc PCG call {k}: p={p} cells={cells}", flush=True)
        w = inputs.random_case(p, cells=cells, seed=3 + k)
        P = Problem(spec(w))
        f = torch.from_numpy(inputs.random_vector(P.ndof, 90 + k)).cuda()
        u0 = torch.from_numpy(inputs.random_vector(P.ndof, 95 + k)).cuda()
        o = smooth_opts(eps=1e-2, n_sweeps=4, inner=0)
        ref, st_ref = _smooth(P, "dg_block_smooth", f, u0, o)
        got, st_got = _smooth(P, "dg_block_smooth_noalloc", f, u0, o)
        assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
        assert st_got == st_ref
        P.close()


def test_noalloc_refuses_what_does_not_fit():
    from paper_1805_11930_amd import DG_INNER_FDM, Problem, ProblemSpec, _lib as L, smooth_opts

    DG_EINVAL = L.DG_EINVAL

    # 64^3 cells at p = 3: an FP64 vector alone is the whole 128 MiB
    P = Problem(ProblemSpec(cells=(64, 64, 64), p=3))
    f = torch.zeros(P.ndof, dtype=torch.float64, device="cuda")
    u0 = torch.zeros_like(f)
    out = torch.empty_like(f)
    st = L.SmoothStats()
    o = smooth_opts(n_sweeps=2)
    rc = P.lib.dg_block_smooth_noalloc(P.h, L.DG_FP64, f.data_ptr(), u0.data_ptr(), out.data_ptr(), ctypes.byref(o),
                                       ctypes.byref(st), torch.cuda.current_stream().cuda_stream)
    assert rc == DG_EINVAL
    assert b"scratch" in P.lib.dg_last_error()
    P.close()
    # the stored factors of the exact block solve are not built by this call
    w = inputs.random_case(2, cells=(2, 2, 2), seed=1)
    P = Problem(spec(w))
    f = torch.ones(P.ndof, dtype=torch.float64, device="cuda")
    out = torch.empty_like(f)
    o = smooth_opts(inner=DG_INNER_FDM, zero_guess=1)
    rc = P.lib.dg_block_smooth_noalloc(P.h, L.DG_FP64, f.data_ptr(), None, out.data_ptr(), ctypes.byref(o), None,
                                       torch.cuda.current_stream().cuda_stream)
    assert rc == DG_EINVAL
    P.close()
