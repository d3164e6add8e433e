"""libdgmg: matrix-free DG operator, block smoothers and hybrid multigrid on
MI355X (gfx950), after Bastian, Mueller, Muething, Piatkowski,
"Matrix-free multigrid block-preconditioners for higher order
Discontinuous Galerkin discretisations" (arXiv:1805.11930).

The numerical work is in the HIP shared library ``libdgmg.so`` (C ABI in
``include/dgmg.h``); this package only marshals arguments.  Importing the
package does not load the library; constructing a Problem does, and fails
loudly if it is missing.
"""
from ._lib import (  # noqa: F401
    DG_BASIS_GL, DG_BASIS_GLL, DG_BC_DIRICHLET, DG_BC_NEUMANN, DG_COARSE_AUTO, DG_COARSE_P0, DG_COARSE_Q1,
    DG_COARSE_SOLVER_AMG, DG_COARSE_SOLVER_GEOMETRIC, DG_FIELD_AXIS_QUADRATIC,
    DG_FIELD_NONE, DG_FIELD_ROTATED_QUADRATIC, DG_FP32, DG_FP64, DG_INNER_CG, DG_INNER_FDM, DG_INNER_GMRES, DG_INNER_PMF,
    DG_IPREC_DIAG, DG_IPREC_TRIDIAG, DG_KRYLOV_CG, DG_KRYLOV_FCG, DG_KRYLOV_FGMRES, DG_PRECOND_BLOCK,
    DG_PRECOND_BLOCK_JACOBI, DG_PRECOND_MG, DG_PRECOND_NONE, DG_SWEEP_JACOBI, DG_SWEEP_SOR, DG_SWEEP_SOR_BACKWARD,
    DG_SWEEP_SSOR, DgError, ProblemSpec, footprint, load, mg_opts, smooth_opts, solve_opts,
)


def Problem(spec):  # noqa: N802 - factory keeps torch out of the package import
    from .problem import Problem as _P

    return _P(spec)
