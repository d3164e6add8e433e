"""FP64 CPU oracle for the DG operator, block smoother, V-cycle and solves.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check of the
package entry point and the CPU-baseline leg of the benchmark may import
this package.  The product path (the HIP library and its Python binding)
never calls into it, and it shares no code with the product path: tables,
quadrature rules, assembly and solvers are all written here independently
from the paper's definitions.

Everything is plain and slow on purpose: the DG matrix is assembled
explicitly from element and face matrices evaluated by quadrature loops
(numpy matrix products serve as the summation step), and the iterative
methods take the paper's steps in the paper's order.

Modules
-------
basis         Gauss-Legendre / Gauss-Lobatto rules and 1-D Lagrange tables.
dg            mesh, coefficients, assembly of A (bilinear form, Sec. 2.1,
              eqn bilinear_form_split) and of the right-hand side (eqn rhs).
solvers       block-Jacobi smoother (alg block_jacobi), inner PCG / GMRES,
              P0 transfers and coarse matrix (Sec. 2.2.2-2.2.3, App. A.1),
              hybrid V-cycle (alg hybrid_multigrid), outer CG / FCG / FGMRES.
memory_model  memory estimates of Sec. 4.4 (eqns memory_diffusion,
              memory_convection).
"""
