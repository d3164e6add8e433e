"""The C-ABI library loads and exports every function include/dgmg.h
declares; host-side argument validation and the footprint estimate run
without a GPU (no compute calls are made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dgmg.h")
LIB = os.path.join(ROOT, "paper_1805_11930_amd", "libdgmg.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dg_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libdgmg.so is not built (python -m paper_1805_11930_amd.build)")
    from paper_1805_11930_amd import _lib

    return _lib.load(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 19
    for n in names:
        assert hasattr(lib, n), n
    # and the binding registers exactly what the header declares
    from paper_1805_11930_amd import _lib

    assert set(_lib.EXPORTS) == set(names)


def _desc(**kw):
    from paper_1805_11930_amd import ProblemSpec

    args = dict(cells=(2, 2, 2), p=2)
    args.update(kw)
    return ProblemSpec(**args)


@pytest.mark.parametrize(
    "kw",
    [
        dict(cells=(0, 2, 2)),
        dict(p=0),
        dict(p=9),
        dict(K=-1.0),
        dict(K=float("nan")),
        dict(c=-0.5),
        dict(lengths=(1.0, 0.0, 1.0)),
        dict(b0=(float("inf"), 0.0, 0.0)),
        dict(bc=(0, 1, 2, 0, 0, 0)),
    ],
)
def test_invalid_descriptions_rejected(lib, kw):
    from paper_1805_11930_amd import _lib

    spec = _desc(**kw)
    d = spec.desc()
    h = ctypes.c_void_p()
    rc = lib.dg_problem_create(ctypes.byref(d), ctypes.byref(h))
    assert rc == _lib.DG_EINVAL
    assert not h.value
    assert lib.dg_last_error()


def test_null_arguments(lib):
    from paper_1805_11930_amd import _lib

    assert lib.dg_problem_create(None, None) == _lib.DG_EINVAL
    assert lib.dg_apply(None, 0, None, None, None) == _lib.DG_EINVAL
    assert lib.dg_solve(None, None, None, None, None, None) == _lib.DG_EINVAL
    assert lib.dg_ndof(None) == -1


def test_defaults_and_footprint(lib):
    from paper_1805_11930_amd import _lib

    o = _lib.solve_opts()
    assert o.rtol == 1e-8 and o.krylov == _lib.DG_KRYLOV_FCG and o.precond == _lib.DG_PRECOND_MG
    assert o.mg.n_pre == 1 and o.mg.n_post == 1 and o.mg.smooth.eps == 1e-2
    # footprint grows with the problem and with FGMRES's basis
    small = _lib.footprint(_desc(cells=(8, 8, 8), p=2))
    big = _lib.footprint(_desc(cells=(32, 32, 32), p=4))
    assert 0 < small < big
    fg = _lib.footprint(_desc(cells=(32, 32, 32), p=4), _lib.solve_opts(krylov=_lib.DG_KRYLOV_FGMRES))
    assert fg > big
    ndof = 32**3 * 125
    assert big >= 6 * 8 * ndof  # FCG's FP64 vectors at least
