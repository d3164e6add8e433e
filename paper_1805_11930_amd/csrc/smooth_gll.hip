// Block smoother steps in the Gauss-Lobatto basis (Sec. 2.1 basis; alg
// block_jacobi and alg block_SOR of Sec. 2.2.1).
//
// The defect of the GLL system is d' = f' - S^T A S u' (block-SOR form:
// f' - S^T (A - D) S u', the cell's own block left out), formed here with
// the Gauss-point kernels around the basis change; the sweep kernel
// (smooth_kernel.h with GLL = true) then solves S^T D_T S x = d' per cell
// with S inside its inner CG / GMRES and updates u' as in the Gauss-point
// basis.  The preconditioner operator is the one with the coefficients at
// the cell centres, as in the fused Gauss-point sweep.
#include "smooth_kernel.h"

namespace dgmg {

template <int P, typename T>
static int launch_smooth_gll_t(const dg_problem *pr, const void *d, const void *uin, void *uout, const SmoothArgs &a,
                               int *iters, hipStream_t s) {
  constexpr int N = P + 1;
  using Sh = SmoothShape<N>;
  SmoothKArgs ka;
  ka.colour = a.colour;
  ka.ncol = a.ncol;
  ka.hx = (pr->geo.nx + a.ncol - 1) / a.ncol;
  ka.rows = pr->geo.ny * pr->geo.nz;
  ka.sor = a.sor;
  const int64_t slots = a.colour >= 0 ? (int64_t)ka.hx * ka.rows : pr->ncell;
  const int G = (int)((slots + Sh::CPW - 1) / Sh::CPW);
  ka.omega = a.omega;
  ka.eps = a.eps;
  ka.max_inner = a.max_inner;
  ka.restart = a.restart;
  ka.zero_guess = a.zero_guess;
  ka.write_du = a.write_du;
  ka.defect = 0;  // d is the defect
  const bool hb = pr->geo.has_b != 0;
  const T *blk = (const T *)pr->gll_blk[sizeof(T) == 8 ? DG_FP64 : DG_FP32];
#define DG_GLL_LAUNCH_RM(INNER, HB, TRI, RM)                                                                \
  hipLaunchKernelGGL((k_smooth<P, INNER, T, HB, TRI, RM, true>), dim3(G), dim3(kSmoothThreads), 0, s, pr->geo, \
                     (const T *)d, (const T *)uin, (T *)uout, ka, iters, (const T *)a.zh, blk)
  // inner GMRES: the restart-8 build (smaller Krylov basis in LDS and
  // registers, more waves per SIMD) when the restart length allows
#define DG_GLL_LAUNCH_GMRES(HB, TRI)                           \
  do {                                                         \
    if (a.restart <= 8)                                        \
      DG_GLL_LAUNCH_RM(DG_INNER_GMRES, HB, TRI, 8);            \
    else                                                       \
      DG_GLL_LAUNCH_RM(DG_INNER_GMRES, HB, TRI, kGmresMax);    \
  } while (0)
  if (a.inner == DG_INNER_CG) {
    if (hb)
      DG_GLL_LAUNCH_RM(DG_INNER_CG, true, false, kGmresMax);
    else
      DG_GLL_LAUNCH_RM(DG_INNER_CG, false, false, kGmresMax);
  } else if (a.tridiag) {
    if (hb)
      DG_GLL_LAUNCH_GMRES(true, true);
    else
      DG_GLL_LAUNCH_GMRES(false, true);
  } else {
    if (hb)
      DG_GLL_LAUNCH_GMRES(true, false);
    else
      DG_GLL_LAUNCH_GMRES(false, false);
  }
#undef DG_GLL_LAUNCH_GMRES
#undef DG_GLL_LAUNCH_RM
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int launch_smooth_gll(const dg_problem *pr, int prec, const void *f, const void *uin, void *uout, const SmoothArgs &a,
                      int *iters, hipStream_t s) {
  if (a.inner != DG_INNER_CG && a.inner != DG_INNER_GMRES) {
    set_error("the Gauss-Lobatto basis supports the inner CG and GMRES block solves");
    return DG_EINVAL;
  }
  if (a.cb) {
    set_error("internal: no cast-back epilogue in the Gauss-Lobatto sweep");
    return DG_EINVAL;
  }
  if (a.inner == DG_INNER_CG && a.tridiag) {
    set_error("the tridiagonal inner preconditioner needs inner GMRES");
    return DG_EINVAL;
  }
  if (a.inner == DG_INNER_GMRES && (a.restart < 1 || a.restart > kGmresMax)) {
    set_error("inner GMRES restart must be in 1..16");
    return DG_EINVAL;
  }
  if (a.zh && (a.zero_guess || !a.defect)) {
    set_error("a P0 correction needs a smoothed input");
    return DG_EINVAL;
  }
  if ((a.colour >= 0) != (uin == uout) || (a.colour >= 0 && (a.zh || a.write_du || !a.defect)) ||
      a.ncol < 2 || a.colour >= a.ncol) {
    set_error("internal: a colour sweep runs in place, without a P0 correction");
    return DG_EINVAL;
  }
  // d' = f - S^T (A [- D]) S (u + P zh); from a zero guess d' = f
  const void *d = f;
  if (a.defect && !a.zero_guess) {
    void *w = pr->gll_tmp[prec][0], *y = pr->gll_tmp[prec][1], *z = pr->gll_tmp[prec][2];
    int rc;
    if ((rc = launch_basis(pr, prec, uin, w, false, s, a.zh)) || (rc = launch_apply_cc_gl(pr, prec, w, y, s)))
      return rc;
    if (a.sor && ((rc = launch_block_apply_gl(pr, prec, w, z, s)) || (rc = launch_diff(pr->ndof, prec, y, z, y, s))))
      return rc;
    if ((rc = launch_basis(pr, prec, y, w, true, s)) || (rc = launch_diff(pr->ndof, prec, f, w, w, s))) return rc;
    d = w;
  }
  const bool dp = prec == DG_FP64;
  switch (pr->p) {
    case 1: return dp ? launch_smooth_gll_t<1, double>(pr, d, uin, uout, a, iters, s)
                      : launch_smooth_gll_t<1, float>(pr, d, uin, uout, a, iters, s);
    case 2: return dp ? launch_smooth_gll_t<2, double>(pr, d, uin, uout, a, iters, s)
                      : launch_smooth_gll_t<2, float>(pr, d, uin, uout, a, iters, s);
    case 3: return dp ? launch_smooth_gll_t<3, double>(pr, d, uin, uout, a, iters, s)
                      : launch_smooth_gll_t<3, float>(pr, d, uin, uout, a, iters, s);
    case 4: return dp ? launch_smooth_gll_t<4, double>(pr, d, uin, uout, a, iters, s)
                      : launch_smooth_gll_t<4, float>(pr, d, uin, uout, a, iters, s);
    case 5: return dp ? launch_smooth_gll_t<5, double>(pr, d, uin, uout, a, iters, s)
                      : launch_smooth_gll_t<5, float>(pr, d, uin, uout, a, iters, s);
  }
  set_error("unsupported degree");
  return DG_EINVAL;
}

}  // namespace dgmg
