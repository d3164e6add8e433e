// The paper's Gauss-Lobatto basis (Sec. 2.1) on top of the Gauss-Legendre
// kernels.
//
// Both bases span Q_p on every cell.  With S = V (x) V (x) V (ctables.h:
// V[q][j] = value of the j-th GLL Lagrange polynomial at the q-th Gauss
// point), the Gauss-point values of a function with GLL coefficients u' are
// u = S u', the GLL basis functions are psi'_a = sum_i S_ia psi_i, and so
//   A' = S^T A S,  l' = S^T l,  D_T' = S^T D_T S  (per cell),
// with the same quadrature on both sides (p+1 Gauss points per direction).
// The GLL operator is therefore Stage 1 of Sec. 3.1 with the value matrix
// V (S u'), the Gauss-point operator, and Stage 3 with V^T -- here as three
// passes: k_basis (S), the collocated apply, k_basis (S^T).
//
// The block smoother takes S inside its inner iteration (smooth_kernel.h,
// smooth_gll.hip).
//
// Kernels:
//   k_basis<P, T, TR>: out = S in (TR = false) or S^T in (TR = true), cell
//     by cell; one thread per DOF, the three 1-D contractions through LDS;
//   k_gll_blk<P, T>: the diagonal and the first sub- and super-diagonal of
//     S^T D_T S from the 1-D line operators of D_T (with advection they
//     depend on the line), for the inner preconditioners;
//   k_gll_factor<P, T>: the Thomas factors of that band, per cell;
//   k_diff<T>: d = f - y.
#include <hip/hip_runtime.h>

#include "dg_internal.h"
#include "line_ops.h"

namespace dgmg {

int dmalloc(dg_problem *pr, void **p, size_t bytes);

namespace {

constexpr int kBasisThreads = 256;

// out = S (in + P zadd) or S^T in; cells are independent, CPB cells per
// workgroup, one thread per DOF (x fastest within a cell).  S P = P (the
// rows of V sum to one), so a cell constant zadd[c] is added to the output.
template <int P, typename T, bool TR>
__global__ __launch_bounds__(kBasisThreads) void k_basis(int64_t ncell, const T *in, T *out,
                                                          const T *__restrict__ zadd) {
  constexpr int N = P + 1, N2 = N * N, N3 = N2 * N;
  constexpr int CPB = kBasisThreads / N3;
  constexpr GllDev<N, T> gd = make_gll_dev<N, T>();
  __shared__ T a[CPB * N3], b[CPB * N3];
  const int tid = threadIdx.x;
  const int cl = tid / N3;
  const int j = tid - cl * N3;
  const int64_t c = (int64_t)blockIdx.x * CPB + cl;
  const bool on = cl < CPB && c < ncell;
  const int i0 = j % N, i1 = (j / N) % N, i2 = j / N2;
  T *A = a + cl * N3, *B = b + cl * N3;
  if (on) A[j] = in[c * N3 + j];
  __syncthreads();
  // axis 0: B[i0, i1, i2] = sum_l M[i0][l] A[l, i1, i2], M = V or V^T
  if (on) {
    T s = T(0);
#pragma unroll
    for (int l = 0; l < N; ++l) s += (TR ? gd.V[l][i0] : gd.V[i0][l]) * A[l + N * i1 + N2 * i2];
    B[j] = s;
  }
  __syncthreads();
  if (on) {
    T s = T(0);
#pragma unroll
    for (int l = 0; l < N; ++l) s += (TR ? gd.V[l][i1] : gd.V[i1][l]) * B[i0 + N * l + N2 * i2];
    A[j] = s;
  }
  __syncthreads();
  if (on) {
    T s = T(0);
#pragma unroll
    for (int l = 0; l < N; ++l) s += (TR ? gd.V[l][i2] : gd.V[i2][l]) * A[i0 + N * i1 + N2 * l];
    if (zadd) s += zadd[c];
    out[c * N3 + j] = s;
  }
}

// Entry (I, J) of the GLL block S^T D_T S of cell c for DOFs I and J of the
// cell (index triples): D_T is a sum over the three axes of line operators
// L (the lines along axis k through the Gauss points (a, b) of the two
// other axes), so the entry is the sum over k and the lines of
//   V[a][I_t1] V[a][J_t1] V[b][I_t2] V[b][J_t2] (V^T L V)[I_k][J_k].
template <int N>
__device__ inline double gll_block_entry(const Geo &g, int c, const int (&ijk)[3], const DevTab<double, N> &tb,
                                         const GllDev<N, double> &gd, const int (&I)[3], const int (&J)[3]) {
  const bool hasb = g.has_b != 0;
  const double cre = g.has_c ? g.c[c] : 0.0;
  double s = 0.0;
  for (int k = 0; k < 3; ++k) {
    const int t1 = (k == 0) ? 1 : 0, t2 = (k == 2) ? 1 : 2;
    const AxisCoef<double> f = make_axis_coef<double>(g, c, k, ijk);
    for (int a = 0; a < N; ++a)
      for (int b = 0; b < N; ++b) {
        const double wt = gd.V[a][I[t1]] * gd.V[a][J[t1]] * gd.V[b][I[t2]] * gd.V[b][J[t2]];
        const LineConv<double> lc =
            hasb ? make_line_conv<double, N>(g, tb, k, ijk, a, b) : LineConv<double>{0.0, 0.0, 0.0, 0.0};
        double m = 0.0;
        for (int i = 0; i < N; ++i)
          for (int l = 0; l < N; ++l)
            m += gd.V[i][I[k]] *
                 line_entry<double, N>(tb, f, tb.w[a] * tb.w[b], g.vol, k == 0 ? cre : 0.0, hasb, lc, i, l) *
                 gd.V[l][J[k]];
        s += wt * m;
      }
  }
  return s;
}

// Entries of the GLL blocks for the inner preconditioners, planar:
// out[0..ndof) = D'_(k,k), out[ndof..2 ndof) = D'_(k,k-1) (0 at k = 0),
// out[2 ndof..3 ndof) = D'_(k,k+1) (0 at the last k), with k the DOF index
// within the cell (x fastest): the diagonal and the first sub- and
// super-diagonal of the whole block.  In the GLL basis the band also
// couples the last DOF of an x-line to the first of the next.
template <int P, typename T>
__global__ __launch_bounds__(256) void k_gll_blk(Geo g, T *__restrict__ out) {
  constexpr int N = P + 1, N2 = N * N, N3 = N * N * N;
  constexpr DevTab<double, N> tb = make_ctab<double, N>();
  constexpr GllDev<N, double> gd = make_gll_dev<N, double>();
  const int64_t ndof = (int64_t)g.ncell * N3;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= ndof) return;
  const int c = (int)(gid / N3);
  const int j = (int)(gid - (int64_t)c * N3);
  auto idx = [](int k, int(&I)[3]) {
    I[0] = k % N;
    I[1] = (k / N) % N;
    I[2] = k / N2;
  };
  int I[3], Jm[3], Jp[3];
  idx(j, I);
  idx(j > 0 ? j - 1 : 0, Jm);
  idx(j < N3 - 1 ? j + 1 : 0, Jp);
  int ijk[3];
  cell_coords(g, c, ijk);
  out[gid] = (T)gll_block_entry<N>(g, c, ijk, tb, gd, I, I);
  out[ndof + gid] = j > 0 ? (T)gll_block_entry<N>(g, c, ijk, tb, gd, I, Jm) : T(0);
  out[2 * ndof + gid] = j < N3 - 1 ? (T)gll_block_entry<N>(g, c, ijk, tb, gd, I, Jp) : T(0);
}

// Thomas factors of each block's band (one thread per cell, in place):
// pivots m_k = D_kk - sub_k c_(k-1), c_k = sup_k / m_k; plane 2 becomes
// c_k and plane 3 receives 1 / m_k.
template <int P, typename T>
__global__ __launch_bounds__(64) void k_gll_factor(int ncell, T *__restrict__ out) {
  constexpr int N3 = (P + 1) * (P + 1) * (P + 1);
  const int c = blockIdx.x * 64 + threadIdx.x;
  if (c >= ncell) return;
  const size_t ndof = (size_t)ncell * N3, base = (size_t)c * N3;
  T cprev = T(0);
  for (int k = 0; k < N3; ++k) {
    const size_t q = base + k;
    const T m = out[q] - out[ndof + q] * cprev;
    const T inv = T(1) / m;
    cprev = out[2 * ndof + q] * inv;
    out[2 * ndof + q] = cprev;
    out[3 * ndof + q] = inv;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_diff(int64_t n, const T *__restrict__ f, const T *__restrict__ y,
                                              T *__restrict__ d) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) d[i] = f[i] - y[i];
}

template <int P, typename T>
int basis_t(const dg_problem *pr, const void *in, void *out, bool tr, hipStream_t s, const void *zadd) {
  constexpr int N3 = (P + 1) * (P + 1) * (P + 1);
  constexpr int CPB = kBasisThreads / N3;
  const dim3 grid((unsigned)((pr->ncell + CPB - 1) / CPB));
  if (tr)
    hipLaunchKernelGGL((k_basis<P, T, true>), grid, dim3(kBasisThreads), 0, s, (int64_t)pr->ncell, (const T *)in,
                       (T *)out, (const T *)nullptr);
  else
    hipLaunchKernelGGL((k_basis<P, T, false>), grid, dim3(kBasisThreads), 0, s, (int64_t)pr->ncell, (const T *)in,
                       (T *)out, (const T *)zadd);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

template <int P, typename T>
int gll_blk_t(const dg_problem *pr, void *out, hipStream_t s) {
  const int64_t n = pr->ndof;
  hipLaunchKernelGGL((k_gll_blk<P, T>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pr->geo, (T *)out);
  DG_HIP(hipGetLastError());
  hipLaunchKernelGGL((k_gll_factor<P, T>), dim3((unsigned)((pr->ncell + 63) / 64)), dim3(64), 0, s, (int)pr->ncell,
                     (T *)out);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

}  // namespace

// out = S (in + P zadd) (tr = false) or S^T in (tr = true), cell by cell;
// in and out may be the same vector (each cell is read whole before it is
// written, by the same workgroup).
int launch_basis(const dg_problem *pr, int prec, const void *in, void *out, bool tr, hipStream_t s,
                 const void *zadd) {
  const bool d = prec == DG_FP64;
  switch (pr->p) {
    case 1: return d ? basis_t<1, double>(pr, in, out, tr, s, zadd) : basis_t<1, float>(pr, in, out, tr, s, zadd);
    case 2: return d ? basis_t<2, double>(pr, in, out, tr, s, zadd) : basis_t<2, float>(pr, in, out, tr, s, zadd);
    case 3: return d ? basis_t<3, double>(pr, in, out, tr, s, zadd) : basis_t<3, float>(pr, in, out, tr, s, zadd);
    case 4: return d ? basis_t<4, double>(pr, in, out, tr, s, zadd) : basis_t<4, float>(pr, in, out, tr, s, zadd);
    case 5: return d ? basis_t<5, double>(pr, in, out, tr, s, zadd) : basis_t<5, float>(pr, in, out, tr, s, zadd);
  }
  set_error("unsupported degree");
  return DG_EINVAL;
}

// block entries and band factors of the GLL blocks into out (DEVICE
// [4][ndof], precision prec; see k_gll_blk and k_gll_factor)
static int launch_gll_blk(const dg_problem *pr, int prec, void *out, hipStream_t s) {
  const bool d = prec == DG_FP64;
  switch (pr->p) {
    case 1: return d ? gll_blk_t<1, double>(pr, out, s) : gll_blk_t<1, float>(pr, out, s);
    case 2: return d ? gll_blk_t<2, double>(pr, out, s) : gll_blk_t<2, float>(pr, out, s);
    case 3: return d ? gll_blk_t<3, double>(pr, out, s) : gll_blk_t<3, float>(pr, out, s);
    case 4: return d ? gll_blk_t<4, double>(pr, out, s) : gll_blk_t<4, float>(pr, out, s);
    case 5: return d ? gll_blk_t<5, double>(pr, out, s) : gll_blk_t<5, float>(pr, out, s);
  }
  set_error("unsupported degree");
  return DG_EINVAL;
}

int launch_diff(int64_t n, int prec, const void *f, const void *y, void *d, hipStream_t s) {
  const dim3 grid((unsigned)((n + 255) / 256));
  if (prec == DG_FP64)
    hipLaunchKernelGGL((k_diff<double>), grid, dim3(256), 0, s, n, (const double *)f, (const double *)y,
                       (double *)d);
  else
    hipLaunchKernelGGL((k_diff<float>), grid, dim3(256), 0, s, n, (const float *)f, (const float *)y, (float *)d);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

// The GLL scratch vectors (three per precision) and the block entries and
// band factors of the GLL blocks (both precisions), allocated and computed
// at problem creation.
int gll_setup(dg_problem *pr) {
  int rc;
  for (int prec = 0; prec < 2; ++prec) {
    const size_t es = prec == DG_FP64 ? sizeof(double) : sizeof(float);
    for (int k = 0; k < 3; ++k)
      if ((rc = dmalloc(pr, &pr->gll_tmp[prec][k], (size_t)pr->ndof * es))) return rc;
    if ((rc = dmalloc(pr, &pr->gll_blk[prec], 4 * (size_t)pr->ndof * es))) return rc;
    if ((rc = launch_gll_blk(pr, prec, pr->gll_blk[prec], 0))) return rc;
  }
  DG_HIP(hipStreamSynchronize(0));
  return DG_OK;
}

// ---- operators of the problem's basis -------------------------------------

static bool gll(const dg_problem *pr) { return pr->basis == DG_BASIS_GLL; }

// v = S^T A S u
int launch_apply(const dg_problem *pr, int prec, const void *u, void *v, hipStream_t s, hipEvent_t ev0,
                 hipEvent_t ev1) {
  if (!gll(pr)) return launch_apply_gl(pr, prec, u, v, s, ev0, ev1);
  void *w = pr->gll_tmp[prec][0], *y = pr->gll_tmp[prec][1];
  int rc;
  if (ev0) DG_HIP(hipEventRecord(ev0, s));
  if ((rc = launch_basis(pr, prec, u, w, false, s)) || (rc = launch_apply_gl(pr, prec, w, y, s)) ||
      (rc = launch_basis(pr, prec, y, v, true, s)))
    return rc;
  if (ev1) DG_HIP(hipEventRecord(ev1, s));
  return DG_OK;
}

// y_T = S^T D_T S x_T
int launch_block_apply(const dg_problem *pr, int prec, const void *x, void *y, hipStream_t s) {
  if (!gll(pr)) return launch_block_apply_gl(pr, prec, x, y, s);
  void *w = pr->gll_tmp[prec][0], *t = pr->gll_tmp[prec][1];
  int rc;
  if ((rc = launch_basis(pr, prec, x, w, false, s)) || (rc = launch_block_apply_gl(pr, prec, w, t, s)) ||
      (rc = launch_basis(pr, prec, t, y, true, s)))
    return rc;
  return DG_OK;
}

int launch_block_diag(const dg_problem *pr, int prec, void *diag, hipStream_t s) {
  if (!gll(pr)) return launch_block_diag_gl(pr, prec, diag, s);
  const size_t es = prec == DG_FP64 ? sizeof(double) : sizeof(float);
  DG_HIP(hipMemcpyAsync(diag, pr->gll_blk[prec], (size_t)pr->ndof * es, hipMemcpyDeviceToDevice, s));
  return DG_OK;
}

// l' = S^T l: the GLL basis functions are psi'_a = sum_i S_ia psi_i
int launch_rhs(const dg_problem *pr, const double *fq, const double *bq, double *rhs, hipStream_t s) {
  if (!gll(pr)) return launch_rhs_gl(pr, fq, bq, rhs, s);
  void *t = pr->gll_tmp[DG_FP64][0];
  int rc;
  if ((rc = launch_rhs_gl(pr, fq, bq, (double *)t, s)) || (rc = launch_basis(pr, DG_FP64, t, rhs, true, s)))
    return rc;
  return DG_OK;
}

// P0 restriction of r - A' u: the P0 basis function of a cell is the sum of
// the cell's basis functions in either basis (S 1 = 1), so
// sum_(i in T) (A' u)_i = sum_(i in T) (A S u)_i and the fused Gauss-point
// kernel takes S u with the unchanged r.  The Q1 corner sums would need the
// Q1 functions in the GLL nodes; not supported.
int launch_residual_restrict(const dg_problem *pr, int prec, const void *u, const void *r, void *rh, hipStream_t s,
                             int kind) {
  if (!gll(pr)) return launch_residual_restrict_gl(pr, prec, u, r, rh, s, kind);
  if (kind != COARSE_P0) {
    set_error("the Gauss-Lobatto basis supports the P0 coarse space only");
    return DG_EINVAL;
  }
  void *w = pr->gll_tmp[prec][0];
  int rc;
  if ((rc = launch_basis(pr, prec, u, w, false, s)) ||
      (rc = launch_residual_restrict_gl(pr, prec, w, r, rh, s, COARSE_P0)))
    return rc;
  return DG_OK;
}

}  // namespace dgmg
