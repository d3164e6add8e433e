"""ctypes binding of libdgmg (include/dgmg.h): argument marshalling only.

Every numerical step runs in the HIP library; this module converts torch
tensors to device pointers and HIP streams, mirrors the C structs, and
turns status codes into exceptions.  There is no fallback: if the shared
library is missing or cannot be loaded, loading raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdgmg.so")

DG_OK, DG_ENOCONV, DG_EAGAIN = 0, 1, 2
DG_EINVAL, DG_ENOMEM, DG_EDEVICE, DG_EBREAKDOWN = -1, -2, -3, -4
DG_MAX_P = 5
DG_FP64, DG_FP32 = 0, 1
DG_BC_DIRICHLET, DG_BC_NEUMANN = 0, 1
DG_INNER_CG, DG_INNER_GMRES, DG_INNER_FDM, DG_INNER_PMF = 0, 1, 2, 3
DG_KRYLOV_CG, DG_KRYLOV_FCG, DG_KRYLOV_FGMRES = 0, 1, 2
DG_PRECOND_NONE, DG_PRECOND_BLOCK, DG_PRECOND_MG = 0, 1, 2
DG_PRECOND_BLOCK_JACOBI = DG_PRECOND_BLOCK
DG_SWEEP_JACOBI, DG_SWEEP_SOR, DG_SWEEP_SSOR, DG_SWEEP_SOR_BACKWARD = 0, 1, 2, 3
DG_IPREC_DIAG, DG_IPREC_TRIDIAG = 0, 1
DG_COARSE_P0, DG_COARSE_Q1, DG_COARSE_AUTO = 0, 1, 2
DG_COARSE_SOLVER_GEOMETRIC, DG_COARSE_SOLVER_AMG = 0, 1
DG_FIELD_NONE, DG_FIELD_AXIS_QUADRATIC, DG_FIELD_ROTATED_QUADRATIC = 0, 1, 2
DG_BASIS_GL, DG_BASIS_GLL = 0, 1

EXPORTS = (
    "dg_problem_create", "dg_problem_destroy", "dg_last_error", "dg_ndof", "dg_boundary_npoints",
    "dg_node_points", "dg_boundary_points", "dg_assemble_rhs", "dg_apply", "dg_block_apply",
    "dg_block_diag", "dg_block_solve", "dg_block_smooth", "dg_mg_vcycle", "dg_solve", "dg_footprint",
    "dg_coarse_stencil", "dg_default_smooth_opts", "dg_default_mg_opts", "dg_default_solve_opts",
    "dg_solve_start", "dg_batch_step", "dg_solve_poll", "dg_solve_state_destroy", "dg_block_smooth_noalloc",
    "dg_coarse_csr", "dg_quadrature_points",
)


class DgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libdgmg status {code}: {msg}")
        self.code = code


class ProblemDesc(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lz", ctypes.c_double),
        ("p", ctypes.c_int), ("bc", ctypes.c_int * 6), ("penalty_factor", ctypes.c_double),
        ("K", ctypes.POINTER(ctypes.c_double)), ("K_scalar", ctypes.c_double),
        ("c", ctypes.POINTER(ctypes.c_double)), ("c_scalar", ctypes.c_double),
        ("b0", ctypes.c_double * 3), ("B", ctypes.c_double * 9),
        ("field", ctypes.c_int), ("kq", ctypes.c_double * 9), ("cq", ctypes.c_double * 2),
        ("nrot", ctypes.c_double * 9), ("basis", ctypes.c_int),
    ]


class SmoothOpts(ctypes.Structure):
    _fields_ = [
        ("n_sweeps", ctypes.c_int), ("omega", ctypes.c_double), ("eps", ctypes.c_double),
        ("max_inner", ctypes.c_int), ("inner", ctypes.c_int), ("restart", ctypes.c_int),
        ("zero_guess", ctypes.c_int), ("sweep", ctypes.c_int), ("inner_precond", ctypes.c_int),
        ("colours", ctypes.c_int),
    ]


class SmoothStats(ctypes.Structure):
    _fields_ = [("blocks", ctypes.c_longlong), ("inner_total", ctypes.c_longlong), ("inner_max", ctypes.c_int),
                ("inner_avg", ctypes.c_double)]


class MgOpts(ctypes.Structure):
    _fields_ = [
        ("n_pre", ctypes.c_int), ("n_post", ctypes.c_int), ("smooth", SmoothOpts),
        ("coarse_space", ctypes.c_int), ("coarse_cycles", ctypes.c_int), ("coarse_smooth", ctypes.c_int),
        ("coarse_omega", ctypes.c_double), ("graph", ctypes.c_int), ("coarse_solver", ctypes.c_int),
        ("fuse_small_levels", ctypes.c_int),
    ]


class SolveOpts(ctypes.Structure):
    _fields_ = [
        ("krylov", ctypes.c_int), ("restart", ctypes.c_int), ("rtol", ctypes.c_double), ("maxit", ctypes.c_int),
        ("precond", ctypes.c_int), ("precond_precision", ctypes.c_int), ("mg", MgOpts),
        ("u_ref", ctypes.c_void_p), ("inner_stats", ctypes.c_int),
    ]


class SolveResult(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int), ("iters", ctypes.c_int), ("rel_residual", ctypes.c_double),
        ("t_setup", ctypes.c_double), ("t_solve", ctypes.c_double), ("inner_avg", ctypes.c_double),
        ("inner_max", ctypes.c_int), ("footprint", ctypes.c_size_t), ("t_apply", ctypes.c_double),
        ("n_apply", ctypes.c_int), ("t_precond", ctypes.c_double), ("n_precond", ctypes.c_int),
        ("error", ctypes.c_double), ("inner_blocks", ctypes.c_longlong),
        ("t_smoother", ctypes.c_double), ("t_restrict", ctypes.c_double), ("t_coarse", ctypes.c_double),
        ("t_prolong", ctypes.c_double),
    ]


_LIB = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libdgmg.so (raises OSError / RuntimeError when absent)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1805_11930_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i64, dp = ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
    lib.dg_problem_create.argtypes = [ctypes.POINTER(ProblemDesc), ctypes.POINTER(vp)]
    lib.dg_problem_destroy.argtypes = [vp]
    lib.dg_problem_destroy.restype = None
    lib.dg_last_error.restype = ctypes.c_char_p
    lib.dg_ndof.argtypes = [vp]
    lib.dg_ndof.restype = i64
    lib.dg_boundary_npoints.argtypes = [vp]
    lib.dg_boundary_npoints.restype = i64
    lib.dg_node_points.argtypes = [vp, dp]
    lib.dg_quadrature_points.argtypes = [vp, dp]
    lib.dg_boundary_points.argtypes = [vp, dp]
    lib.dg_assemble_rhs.argtypes = [vp, vp, vp, vp, vp]
    lib.dg_apply.argtypes = [vp, ctypes.c_int, vp, vp, vp]
    lib.dg_block_apply.argtypes = [vp, ctypes.c_int, vp, vp, vp]
    lib.dg_block_diag.argtypes = [vp, ctypes.c_int, vp, vp]
    lib.dg_block_solve.argtypes = [vp, ctypes.c_int, vp, vp, ctypes.POINTER(SmoothOpts), vp, vp]
    lib.dg_block_smooth.argtypes = [vp, ctypes.c_int, vp, vp, vp, ctypes.POINTER(SmoothOpts),
                                    ctypes.POINTER(SmoothStats), vp]
    lib.dg_block_smooth_noalloc.argtypes = lib.dg_block_smooth.argtypes
    lib.dg_mg_vcycle.argtypes = [vp, ctypes.c_int, vp, vp, ctypes.POINTER(MgOpts), vp]
    lib.dg_solve.argtypes = [vp, vp, vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveResult), vp]
    lib.dg_footprint.argtypes = [ctypes.POINTER(ProblemDesc), ctypes.POINTER(SolveOpts), ctypes.POINTER(ctypes.c_size_t)]
    lib.dg_coarse_stencil.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int), vp]
    lib.dg_coarse_csr.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int64), vp,
                                  vp, vp]
    lib.dg_default_smooth_opts.argtypes = [ctypes.POINTER(SmoothOpts)]
    lib.dg_default_smooth_opts.restype = None
    lib.dg_default_mg_opts.argtypes = [ctypes.POINTER(MgOpts)]
    lib.dg_default_mg_opts.restype = None
    lib.dg_default_solve_opts.argtypes = [ctypes.POINTER(SolveOpts)]
    lib.dg_default_solve_opts.restype = None
    lib.dg_solve_start.argtypes = [vp, vp, vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(vp)]
    lib.dg_batch_step.argtypes = [ctypes.POINTER(vp), ctypes.c_int, vp]
    lib.dg_solve_poll.argtypes = [vp, ctypes.POINTER(SolveResult)]
    lib.dg_solve_state_destroy.argtypes = [vp]
    lib.dg_solve_state_destroy.restype = None
    _LIB = lib
    return lib


def _check(rc: int, allow=(DG_OK,)) -> int:
    if rc not in allow:
        msg = load().dg_last_error()
        raise DgError(rc, msg.decode() if msg else "")
    return rc


def smooth_opts(**kw) -> SmoothOpts:
    o = SmoothOpts()
    load().dg_default_smooth_opts(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def mg_opts(smooth: dict | None = None, **kw) -> MgOpts:
    o = MgOpts()
    load().dg_default_mg_opts(ctypes.byref(o))
    for k, v in (smooth or {}).items():
        setattr(o.smooth, k, v)
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def solve_opts(mg: dict | None = None, smooth: dict | None = None, **kw) -> SolveOpts:
    o = SolveOpts()
    load().dg_default_solve_opts(ctypes.byref(o))
    for k, v in (mg or {}).items():
        setattr(o.mg, k, v)
    for k, v in (smooth or {}).items():
        setattr(o.mg.smooth, k, v)
    for k, v in kw.items():
        setattr(o, k, v)
    return o


_BC = {"D": DG_BC_DIRICHLET, "N": DG_BC_NEUMANN}


@dataclass
class ProblemSpec:
    """Host-side description mirroring dg_problem_desc."""

    cells: tuple
    lengths: tuple = (1.0, 1.0, 1.0)
    p: int = 1
    bc: tuple = ("D",) * 6
    sigma: float | None = None
    K: np.ndarray | float = 1.0
    c: np.ndarray | float = 0.0
    b0: tuple = (0.0, 0.0, 0.0)
    B: tuple = ((0.0,) * 3,) * 3
    # coefficient field (DG_FIELD_AXIS_QUADRATIC): kq = (q0[3], q1[3], q2[3]),
    # K_kk(x) = q0_k + q1_k x_k + q2_k x_k^2; cq = (c0, c2), c(x) = c0 + c2 |x|^2;
    # K and c are then ignored
    kfield: tuple | None = None
    cfield: tuple = (0.0, 0.0)
    nrot: tuple | None = None  # rows n_m of an orthonormal basis: K(x) = sum_m P_m(x_m) n_m n_m^T
    basis: str = "gl"  # nodes of the 1-D basis: "gl" (Gauss-Legendre) or "gll" (Gauss-Lobatto)
    _keep: list = field(default_factory=list, repr=False)

    def desc(self) -> ProblemDesc:
        d = ProblemDesc()
        d.nx, d.ny, d.nz = (int(v) for v in self.cells)
        d.lx, d.ly, d.lz = (float(v) for v in self.lengths)
        d.p = int(self.p)
        for i, t in enumerate(self.bc):
            d.bc[i] = _BC[t] if isinstance(t, str) else int(t)
        d.penalty_factor = float(self.sigma) if self.sigma is not None else 0.0
        ncell = d.nx * d.ny * d.nz
        self._keep = []
        K = np.asarray(self.K, dtype=np.float64)
        if K.ndim == 0:
            d.K = None
            d.K_scalar = float(K)
        else:
            K = np.ascontiguousarray(np.broadcast_to(K, (ncell, 3)), dtype=np.float64)
            self._keep.append(K)
            d.K = K.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            d.K_scalar = 0.0
        c = np.asarray(self.c, dtype=np.float64)
        if c.ndim == 0:
            d.c = None
            d.c_scalar = float(c)
        else:
            c = np.ascontiguousarray(np.broadcast_to(c, (ncell,)), dtype=np.float64)
            self._keep.append(c)
            d.c = c.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            d.c_scalar = 0.0
        for i in range(3):
            d.b0[i] = float(self.b0[i])
        Bm = np.asarray(self.B, dtype=np.float64).reshape(9)
        for i in range(9):
            d.B[i] = float(Bm[i])
        d.field = DG_FIELD_NONE
        if self.kfield is not None:
            d.field = DG_FIELD_AXIS_QUADRATIC if self.nrot is None else DG_FIELD_ROTATED_QUADRATIC
            kq = np.asarray(self.kfield, dtype=np.float64).reshape(9)
            for i in range(9):
                d.kq[i] = float(kq[i])
            d.cq[0], d.cq[1] = (float(v) for v in self.cfield)
            nr = np.eye(3) if self.nrot is None else np.asarray(self.nrot, dtype=np.float64)
            for i in range(9):
                d.nrot[i] = float(nr.reshape(9)[i])
        d.basis = {"gl": DG_BASIS_GL, "gll": DG_BASIS_GLL}[self.basis] if isinstance(self.basis, str) else int(
            self.basis)
        return d


def footprint(spec: ProblemSpec, opts: SolveOpts | None = None) -> int:
    out = ctypes.c_size_t(0)
    d = spec.desc()
    _check(load().dg_footprint(ctypes.byref(d), ctypes.byref(opts) if opts is not None else None, ctypes.byref(out)))
    return int(out.value)
