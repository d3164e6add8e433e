// Stored factors for the exact inversion of the cell blocks D_T when b = 0
// (fast diagonalisation; the stored-factor, partially matrix-free variant of
// the block smoother).
//
// With b = 0 and a cell-constant diagonal K the block of a Cartesian cell is
// a Kronecker sum (x fastest):
//   D_T = Wz (x) Wy (x) Mx + Wz (x) My (x) Wx + Mz (x) Wy (x) Wx,
// M_k the cell's 1-D matrix along axis k (volume term, own-side face terms
// of both faces, and on axis 0 the reaction; see line_matrix_entry) and
// W = diag(w) the Gauss weights.  M_k is symmetric and W positive, so the
// pencil (M_k, W) has a W-orthonormal eigenbasis: with
//   W^(-1/2) M_k W^(-1/2) = Q_k diag(lambda_k) Q_k^T,   T_k = W^(-1/2) Q_k,
// T_k^T M_k T_k = diag(lambda_k) and T_k^T W T_k = I, so
//   D_T^(-1) = (Tz (x) Ty (x) Tx) diag(1 / (lx_i + ly_j + lz_l)) (Tz (x) Ty (x) Tx)^T,
// six 1-D contractions and a diagonal scaling per application.
//
// Factors per cell and axis: T_k (row-major, N x N) then lambda_k (N);
// layout [ncell][3][N*N + N].  Built once per problem and precision on the
// device, in double, by the cyclic Jacobi eigenvalue method (plane
// rotations that annihilate one off-diagonal pair at a time, repeated over
// all pairs until the off-diagonal part is negligible).
#include <cmath>

#include "line_ops.h"
#include "vec.h"

namespace dgmg {

namespace {

template <int N>
__device__ inline void jacobi_eigen(double (&A)[N][N], double (&V)[N][N]) {
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j < N; ++j) V[i][j] = i == j ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0.0, dia = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      dia += A[i][i] * A[i][i];
#pragma unroll
      for (int j = i + 1; j < N; ++j) off += A[i][j] * A[i][j];
    }
    if (!(off > 1e-34 * dia)) break;
#pragma unroll
    for (int p = 0; p < N - 1; ++p) {
#pragma unroll
      for (int q = p + 1; q < N; ++q) {
        const double apq = A[p][q];
        if (apq == 0.0) continue;
        // tangent t of the angle that annihilates A[p][q]: the smaller root
        // of t^2 + 2 tau t - 1 = 0, tau = (A[q][q] - A[p][p]) / (2 A[p][q])
        const double tau = (A[q][q] - A[p][p]) / (2.0 * apq);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(tau * tau + 1.0));
        const double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
        // A <- J^T A J, V <- V J with J = identity except J[p][p] = J[q][q] = cs,
        // J[p][q] = sn, J[q][p] = -sn
#pragma unroll
        for (int r = 0; r < N; ++r) {
          const double arp = A[r][p], arq = A[r][q];
          A[r][p] = cs * arp - sn * arq;
          A[r][q] = sn * arp + cs * arq;
        }
#pragma unroll
        for (int r = 0; r < N; ++r) {
          const double apr = A[p][r], aqr = A[q][r];
          A[p][r] = cs * apr - sn * aqr;
          A[q][r] = sn * apr + cs * aqr;
        }
#pragma unroll
        for (int r = 0; r < N; ++r) {
          const double vrp = V[r][p], vrq = V[r][q];
          V[r][p] = cs * vrp - sn * vrq;
          V[r][q] = sn * vrp + cs * vrq;
        }
      }
    }
  }
}

// One thread per (cell, axis).
template <int P>
__global__ __launch_bounds__(128) void k_fdm_build(Geo g, double *__restrict__ out) {
  constexpr int N = P + 1;
  constexpr int NF = N * N + N;
  constexpr DevTab<double, N> tb = make_ctab<double, N>();
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= 3 * (int64_t)g.ncell) return;
  const int c = (int)(gid / 3);
  const int k = (int)(gid - 3 * (int64_t)c);
  int ijk[3];
  cell_coords(g, c, ijk);
  const AxisCoef<double> f = make_axis_coef<double>(g, c, k, ijk);
  const double cre = (k == 0 && g.has_c) ? g.c[c] : 0.0;
  double isw[N];
#pragma unroll
  for (int i = 0; i < N; ++i) isw[i] = 1.0 / sqrt(tb.w[i]);
  double A[N][N], V[N][N];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int l = 0; l < N; ++l) A[i][l] = isw[i] * line_matrix_entry<double, N>(tb, f, g.vol, cre, i, l) * isw[l];
  // exact symmetry (the entries of the two triangles are formed from the
  // same products in a different order)
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int l = i + 1; l < N; ++l) A[i][l] = A[l][i] = 0.5 * (A[i][l] + A[l][i]);
  jacobi_eigen<N>(A, V);
  double *o = out + gid * NF;
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int j = 0; j < N; ++j) o[i * N + j] = isw[i] * V[i][j];
    o[N * N + i] = A[i][i];
  }
}

template <int P>
int launch_build(const dg_problem *pr, double *out, hipStream_t s) {
  const int64_t n = 3 * (int64_t)pr->ncell;
  hipLaunchKernelGGL((k_fdm_build<P>), dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s, pr->geo, out);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

}  // namespace

int dmalloc(dg_problem *pr, void **p, size_t bytes);

// Factors in the requested precision (built on first use, synchronously).
int ensure_fdm(dg_problem *pr, int prec) {
  if (pr->fdm[prec]) return DG_OK;
  if (pr->geo.has_b) {
    set_error("the fast-diagonalisation block solve needs b = 0");
    return DG_EINVAL;
  }
  const int N = pr->n;
  const size_t count = (size_t)pr->ncell * 3 * (N * N + N);
  int rc;
  double *f64 = (double *)pr->fdm[DG_FP64];
  if (!f64) {
    if ((rc = dmalloc(pr, (void **)&f64, count * sizeof(double)))) return rc;
    pr->fdm[DG_FP64] = f64;
    switch (pr->p) {
      case 1: rc = launch_build<1>(pr, f64, 0); break;
      case 2: rc = launch_build<2>(pr, f64, 0); break;
      case 3: rc = launch_build<3>(pr, f64, 0); break;
      case 4: rc = launch_build<4>(pr, f64, 0); break;
      case 5: rc = launch_build<5>(pr, f64, 0); break;
      default: set_error("unsupported degree"); return DG_EINVAL;
    }
    if (rc) return rc;
  }
  if (prec == DG_FP32) {
    float *f32 = nullptr;
    if ((rc = dmalloc(pr, (void **)&f32, count * sizeof(float)))) return rc;
    pr->fdm[DG_FP32] = f32;
    if ((rc = cast_d2f((int64_t)count, 1.0, f64, f32, 0))) return rc;
  }
  // built on the null stream; the smoothers run on other (possibly
  // non-blocking) streams, so wait here
  DG_HIP(hipStreamSynchronize(0));
  return DG_OK;
}

}  // namespace dgmg
