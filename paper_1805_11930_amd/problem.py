"""Torch-facing wrapper of a libdgmg problem handle.

Tensors are device tensors on the current HIP device (torch's "cuda"
device under ROCm); the library enqueues work on torch's current stream.
Only argument marshalling happens here.
"""
from __future__ import annotations

import ctypes
import sys

import numpy as np
import torch

from . import _lib as L


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t: torch.Tensor | None, dtype=None, n: int | None = None, name: str = "tensor") -> int | None:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} must have {n} elements, got {t.numel()}")
    return t.data_ptr()


def _prec(dtype) -> int:
    if dtype == torch.float64:
        return L.DG_FP64
    if dtype == torch.float32:
        return L.DG_FP32
    raise ValueError("vectors must be float64 or float32")


class Problem:
    """A DG problem resident on the GPU (dg_problem_create / _destroy)."""

    def __init__(self, spec: L.ProblemSpec):
        self.lib = L.load()
        if not torch.cuda.is_available():
            raise RuntimeError("libdgmg needs a HIP device; none is visible")
        self.spec = spec
        d = spec.desc()
        h = ctypes.c_void_p()
        L._check(self.lib.dg_problem_create(ctypes.byref(d), ctypes.byref(h)))
        self.h = h
        self.ndof = int(self.lib.dg_ndof(h))
        self.p = spec.p
        self.nloc = (spec.p + 1) ** 3
        self.ncell = self.ndof // self.nloc

    def close(self):
        if getattr(self, "h", None):
            self.lib.dg_problem_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # not while the interpreter shuts down (module globals may already
        # be gone; the process is ending and the device memory goes with it)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    # -- geometry -------------------------------------------------------
    def node_points(self) -> np.ndarray:
        out = np.zeros((self.ndof, 3))
        L._check(self.lib.dg_node_points(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def quadrature_points(self) -> np.ndarray:
        out = np.zeros((self.ndof, 3))
        L._check(self.lib.dg_quadrature_points(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    def boundary_points(self) -> np.ndarray:
        n = int(self.lib.dg_boundary_npoints(self.h))
        out = np.zeros((n, 3))
        L._check(self.lib.dg_boundary_points(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return out

    # -- right-hand side ------------------------------------------------
    def assemble_rhs(self, f_qp: torch.Tensor | None, bnd_qp: torch.Tensor | None, out: torch.Tensor | None = None):
        if out is None:
            out = torch.empty(self.ndof, dtype=torch.float64, device="cuda")
        nb = int(self.lib.dg_boundary_npoints(self.h))
        L._check(self.lib.dg_assemble_rhs(
            self.h, _ptr(f_qp, torch.float64, self.ndof, "f_qp"), _ptr(bnd_qp, torch.float64, nb, "bnd_qp"),
            _ptr(out, torch.float64, self.ndof, "rhs"), _stream()))
        return out

    def rhs_from_functions(self, f=None, g=None, j=None, bc=None) -> torch.Tensor:
        """l_h from host callables of (npts, 3) point arrays (g on Dirichlet
        faces, j on Neumann faces)."""
        fq = None
        if f is not None:
            fq = torch.from_numpy(np.ascontiguousarray(f(self.quadrature_points()), dtype=np.float64)).cuda()
        bq = None
        if g is not None or j is not None:
            pts = self.boundary_points()
            vals = np.zeros(len(pts))
            bc = bc or self.spec.bc
            n2 = (self.p + 1) ** 2
            nx, ny, nz = self.spec.cells
            nn = (nx, ny, nz)
            off = 0
            for face in range(6):
                k = face // 2
                t1, t2 = [a for a in range(3) if a != k]
                cnt = nn[t1] * nn[t2] * n2
                sl = slice(off, off + cnt)
                fun = g if bc[face] in ("D", L.DG_BC_DIRICHLET) else j
                if fun is not None:
                    vals[sl] = fun(pts[sl])
                off += cnt
            bq = torch.from_numpy(vals).cuda()
        return self.assemble_rhs(fq, bq)

    # -- hot path ---------------------------------------------------------
    def apply(self, u: torch.Tensor, v: torch.Tensor | None = None) -> torch.Tensor:
        if v is None:
            v = torch.empty_like(u)
        prec = _prec(u.dtype)
        L._check(self.lib.dg_apply(self.h, prec, _ptr(u, u.dtype, self.ndof, "u"), _ptr(v, u.dtype, self.ndof, "v"),
                                   _stream()))
        return v

    def block_apply(self, x: torch.Tensor, y: torch.Tensor | None = None) -> torch.Tensor:
        if y is None:
            y = torch.empty_like(x)
        L._check(self.lib.dg_block_apply(self.h, _prec(x.dtype), _ptr(x, x.dtype, self.ndof, "x"),
                                         _ptr(y, x.dtype, self.ndof, "y"), _stream()))
        return y

    def block_diag(self, dtype=torch.float64) -> torch.Tensor:
        out = torch.empty(self.ndof, dtype=dtype, device="cuda")
        L._check(self.lib.dg_block_diag(self.h, _prec(dtype), _ptr(out), _stream()))
        return out

    def block_solve(self, d: torch.Tensor, opts: L.SmoothOpts | None = None, iters: bool = False):
        opts = opts or L.smooth_opts()
        x = torch.empty_like(d)
        it = torch.zeros(self.ncell, dtype=torch.int32, device="cuda") if iters else None
        L._check(self.lib.dg_block_solve(self.h, _prec(d.dtype), _ptr(d, d.dtype, self.ndof, "d"),
                                         _ptr(x, d.dtype, self.ndof, "x"), ctypes.byref(opts), _ptr(it), _stream()))
        return (x, it) if iters else x

    def block_smooth(self, f: torch.Tensor, u_in: torch.Tensor | None, opts: L.SmoothOpts | None = None,
                     out: torch.Tensor | None = None, stats: bool = False):
        opts = opts or L.smooth_opts()
        if u_in is None and not opts.zero_guess:
            opts = L.SmoothOpts.from_buffer_copy(opts)  # leave the caller's options unchanged
            opts.zero_guess = 1
        if out is None:
            out = torch.empty_like(f)
        st = L.SmoothStats() if stats else None
        L._check(self.lib.dg_block_smooth(
            self.h, _prec(f.dtype), _ptr(f, f.dtype, self.ndof, "f"),
            _ptr(u_in, f.dtype, self.ndof, "u_in") if u_in is not None else None,
            _ptr(out, f.dtype, self.ndof, "u_out"), ctypes.byref(opts), ctypes.byref(st) if st else None,
            _stream()))
        return (out, st) if stats else out

    def coarse_stencil(self, coarse_space: int, level: int = 0):
        """(dims (vx, vy, vz), stencil [ns, vx*vy*vz] float64 numpy, nlevels)
        of one level of the P0 or Q1 coarse hierarchy."""
        dims = (ctypes.c_int * 5)()
        L._check(self.lib.dg_coarse_stencil(self.h, coarse_space, level, dims, None))
        vx, vy, vz, ns, nlev = list(dims)
        out = np.empty((ns, vx * vy * vz), dtype=np.float64)
        L._check(self.lib.dg_coarse_stencil(self.h, coarse_space, level, dims, out.ctypes.data))
        return (vx, vy, vz), out, nlev

    def coarse_csr(self, coarse_space: int, level: int, which: int = 0):
        """(row_ptr, col, val, shape, nlevels) of a level of the aggregation-AMG
        hierarchy (which = 0: A_l, 1: P_l, 2: R_l), as numpy arrays."""
        dims = (ctypes.c_int64 * 4)()
        L._check(self.lib.dg_coarse_csr(self.h, coarse_space, level, which, dims, None, None, None))
        rows, cols, nnz, nlev = (int(v) for v in dims)
        rp = np.empty(rows + 1, dtype=np.int32)
        ci = np.empty(max(nnz, 1), dtype=np.int32)
        v = np.empty(max(nnz, 1), dtype=np.float64)
        L._check(self.lib.dg_coarse_csr(self.h, coarse_space, level, which, dims, rp.ctypes.data, ci.ctypes.data,
                                        v.ctypes.data))
        return rp, ci[:nnz], v[:nnz], (rows, cols), nlev

    def mg_vcycle(self, r: torch.Tensor, opts: L.MgOpts | None = None, out: torch.Tensor | None = None):
        opts = opts or L.mg_opts()
        if out is None:
            out = torch.empty_like(r)
        L._check(self.lib.dg_mg_vcycle(self.h, _prec(r.dtype), _ptr(r, r.dtype, self.ndof, "r"),
                                       _ptr(out, r.dtype, self.ndof, "z"), ctypes.byref(opts), _stream()))
        return out

    def solve(self, f: torch.Tensor, u: torch.Tensor | None = None, opts: L.SolveOpts | None = None,
              check: bool = True):
        opts = opts or L.solve_opts()
        if u is None:
            u = torch.zeros_like(f)
        res = L.SolveResult()
        rc = self.lib.dg_solve(self.h, _ptr(f, torch.float64, self.ndof, "f"), _ptr(u, torch.float64, self.ndof, "u"),
                               ctypes.byref(opts), ctypes.byref(res), _stream())
        if check:
            L._check(rc, allow=(L.DG_OK, L.DG_ENOCONV))
        return u, res
