// Setup of the conforming Q1 coarse space (Sec. 2.2.2-2.2.3, App. A.2) on
// the device.
//
// The coarse space is the continuous trilinear functions on the DG mesh,
// one unknown per mesh vertex.  Level 0 holds A_hat_ij = a_h(psi_j, psi_i)
// on the trilinear vertex functions as a 27-point stencil, assembled by
// one thread per vertex from the rows of the cells' element matrices
// (q1_element.h: equal to the Galerkin product P^T A P of the DG matrix).
// Coarser levels keep every second vertex along each axis and the last
// one; their matrices are Galerkin products with trilinear interpolation,
// formed by one thread per coarse vertex, until at most bottom_max
// unknowns remain; that level's matrix is copied to the host and inverted
// densely.
#include <cmath>
#include <vector>

#include "dg_internal.h"
#include "vec.h"

namespace dgmg {

int dmalloc(dg_problem *pr, void **p, size_t bytes);
int alloc_level(dg_problem *pr, CoarseLevel &L, bool first);
int upload_bottom(dg_problem *pr, Hierarchy &H, const std::vector<double> &A);

int build_q1(dg_problem *pr, int bottom_max) {
  Hierarchy &H = pr->q1h;
  H.kind = COARSE_Q1;
  int vx = pr->geo.nx + 1, vy = pr->geo.ny + 1, vz = pr->geo.nz + 1;
  int rc;
  while (true) {
    CoarseLevel L;
    L.nx = vx;
    L.ny = vy;
    L.nz = vz;
    L.n = vx * vy * vz;
    L.ns = 27;
    rc = alloc_level(pr, L, H.levels.empty());
    H.levels.push_back(L);
    if (rc) return rc;
    CoarseLevel &C = H.levels.back();
    if (H.levels.size() == 1) {
      if ((rc = q1_assemble(pr, C.A64, 0))) return rc;
    } else {
      const CoarseLevel &F = H.levels[H.levels.size() - 2];
      if ((rc = galerkin27(F.A64, F.nx, F.ny, F.nz, C.A64, C.nx, C.ny, C.nz, 0))) return rc;
    }
    if ((rc = level_finish(C.A64, C.n, C.A32, C.dinv64, C.dinv32, 0))) return rc;
    if (C.n <= bottom_max) break;
    // coarser vertex grid: every second vertex and the last one per axis
    vx = vx > 2 ? vx / 2 + 1 : vx;
    vy = vy > 2 ? vy / 2 + 1 : vy;
    vz = vz > 2 ? vz / 2 + 1 : vz;
  }
  const CoarseLevel &B = H.levels.back();
  std::vector<double> A((size_t)27 * B.n);
  DG_HIP(hipMemcpy(A.data(), B.A64, A.size() * sizeof(double), hipMemcpyDeviceToHost));  // waits for the builds
  if ((rc = upload_bottom(pr, H, A))) return rc;
  for (int prec = 0; prec < 2; ++prec) {
    const size_t es = prec == DG_FP64 ? sizeof(double) : sizeof(float);
    if (!pr->corner_buf[prec] && (rc = dmalloc(pr, &pr->corner_buf[prec], 8 * (size_t)pr->ncell * es))) return rc;
  }
  // the kernels ran on the null stream; later work runs on other streams
  DG_HIP(hipStreamSynchronize(0));
  return DG_OK;
}

}  // namespace dgmg
