// Launchers of the block smoother kernel (smooth_kernel.h) for the
// Gauss-point basis.
#include "smooth_kernel.h"

namespace dgmg {

template <int P, typename T>
static int launch_smooth_t(const dg_problem *pr, const void *f, const void *uin, void *uout, const SmoothArgs &a,
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
  ka.defect = a.defect;
  if (a.cb) {
    if (!smooth_takes_dots(sizeof(T) == 8 ? DG_FP64 : DG_FP32, a.inner) || a.colour >= 0 || a.write_du || !a.cb->b0 || !a.cb->part || a.cb->m < 1 || a.cb->m > 2 ||
        (a.cb->m == 2 && !a.cb->b1) || (sizeof(T) == 4 && (!a.cb->rr || !a.cb->z))) {
      set_error("internal: the dots epilogue needs a Jacobi sweep and its buffers");
      return DG_EINVAL;
    }
    ka.cb = *a.cb;
  }
  const bool hb = pr->geo.has_b != 0;
#define DG_SMOOTH_LAUNCH_RM(INNER, HB, TRI, RM)                                                                 \
  hipLaunchKernelGGL((k_smooth<P, INNER, T, HB, TRI, RM>), dim3(G), dim3(kSmoothThreads), 0, s, pr->geo,        \
                     (const T *)f, (const T *)uin, (T *)uout, ka, iters, (const T *)a.zh, (const T *)factors)
  // inner GMRES takes the smallest build that holds its restart length
#define DG_SMOOTH_LAUNCH(INNER, HB, TRI) DG_SMOOTH_LAUNCH_RM(INNER, HB, TRI, kGmresMax)
#define DG_SMOOTH_LAUNCH_GMRES(HB, TRI)                    \
  do {                                                     \
    if (a.restart <= 8)                                    \
      DG_SMOOTH_LAUNCH_RM(DG_INNER_GMRES, HB, TRI, 8);     \
    else if (a.restart <= 12)                              \
      DG_SMOOTH_LAUNCH_RM(DG_INNER_GMRES, HB, TRI, 12);    \
    else                                                   \
      DG_SMOOTH_LAUNCH_RM(DG_INNER_GMRES, HB, TRI, kGmresMax); \
  } while (0)
  // stored per-cell factors of the exact block solves (FDM, PMF)
  const int pi = sizeof(T) == 8 ? DG_FP64 : DG_FP32;
  const void *factors = a.inner == DG_INNER_PMF ? pr->pmf[pi] : pr->fdm[pi];
  if (a.inner == DG_INNER_FDM) {
    if (hb || !factors) {
      set_error("the fast-diagonalisation block solve needs b = 0 and its factors");
      return DG_EINVAL;
    }
    DG_SMOOTH_LAUNCH(DG_INNER_FDM, false, false);
  } else if (a.inner == DG_INNER_PMF) {
    if (!factors || a.tridiag) {
      set_error("the stored-inverse block solve needs its factors (and no inner preconditioner)");
      return DG_EINVAL;
    }
    if (hb)
      DG_SMOOTH_LAUNCH(DG_INNER_PMF, true, false);
    else
      DG_SMOOTH_LAUNCH(DG_INNER_PMF, false, false);
  } else if (a.inner == DG_INNER_CG) {
    if (a.tridiag) {
      set_error("the tridiagonal inner preconditioner needs inner GMRES");
      return DG_EINVAL;
    }
    if (hb)
      DG_SMOOTH_LAUNCH(DG_INNER_CG, true, false);
    else
      DG_SMOOTH_LAUNCH(DG_INNER_CG, false, false);
  } else if (a.tridiag) {
    if (hb)
      DG_SMOOTH_LAUNCH_GMRES(true, true);
    else
      DG_SMOOTH_LAUNCH_GMRES(false, true);
  } else {
    if (hb)
      DG_SMOOTH_LAUNCH_GMRES(true, false);
    else
      DG_SMOOTH_LAUNCH_GMRES(false, false);
  }
#undef DG_SMOOTH_LAUNCH
#undef DG_SMOOTH_LAUNCH_RM
#undef DG_SMOOTH_LAUNCH_GMRES
  DG_HIP(hipGetLastError());
  return DG_OK;
}

bool smooth_takes_dots(int prec, int inner) { return prec == DG_FP32 || inner != DG_INNER_GMRES; }

int64_t smooth_blocks(int p, int64_t ncell) {
  int cpw = 1;
  switch (p) {
    case 1: cpw = SmoothShape<2>::CPW; break;
    case 2: cpw = SmoothShape<3>::CPW; break;
    case 3: cpw = SmoothShape<4>::CPW; break;
    case 4: cpw = SmoothShape<5>::CPW; break;
    case 5: cpw = SmoothShape<6>::CPW; break;
  }
  return (ncell + cpw - 1) / cpw;
}

int launch_smooth(const dg_problem *pr, int prec, const void *f, const void *uin, void *uout, const SmoothArgs &a,
                  int *iters, hipStream_t s) {
  if (pr->basis == DG_BASIS_GLL) return launch_smooth_gll(pr, prec, f, uin, uout, a, iters, s);
  if (a.zh && (a.zero_guess || !a.defect)) {
    set_error("a P0 correction needs a smoothed input");
    return DG_EINVAL;
  }
  if ((a.colour >= 0) != (uin == uout) || (a.colour >= 0 && (a.zh || a.write_du || !a.defect)) ||
      a.ncol < 2 || a.colour >= a.ncol) {
    set_error("internal: a colour sweep runs in place, without a P0 correction");
    return DG_EINVAL;
  }
  if (a.inner == DG_INNER_GMRES && (a.restart < 1 || a.restart > kGmresMax)) {
    set_error("inner GMRES restart must be in 1..16");
    return DG_EINVAL;
  }
  const bool d = prec == DG_FP64;
  switch (pr->p) {
    case 1: return d ? launch_smooth_t<1, double>(pr, f, uin, uout, a, iters, s)
                     : launch_smooth_t<1, float>(pr, f, uin, uout, a, iters, s);
    case 2: return d ? launch_smooth_t<2, double>(pr, f, uin, uout, a, iters, s)
                     : launch_smooth_t<2, float>(pr, f, uin, uout, a, iters, s);
    case 3: return d ? launch_smooth_t<3, double>(pr, f, uin, uout, a, iters, s)
                     : launch_smooth_t<3, float>(pr, f, uin, uout, a, iters, s);
    case 4: return d ? launch_smooth_t<4, double>(pr, f, uin, uout, a, iters, s)
                     : launch_smooth_t<4, float>(pr, f, uin, uout, a, iters, s);
    case 5: return d ? launch_smooth_t<5, double>(pr, f, uin, uout, a, iters, s)
                     : launch_smooth_t<5, float>(pr, f, uin, uout, a, iters, s);
  }
  set_error("unsupported degree");
  return DG_EINVAL;
}

}  // namespace dgmg
