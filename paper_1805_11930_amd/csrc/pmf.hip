// Stored block factors for the partially matrix-free smoother (Sec. 4.1,
// solver variant PMF): the operator stays matrix-free, and the block
// solves of the smoother use a factorisation of every diagonal block D_T
// computed once and kept in memory, (p+1)^(2d) numbers per cell.
//
// The stored factor here is the inverse D_T^-1 itself, so that a block
// solve is one dense product per cell: the (p+1)^3 lanes of a cell read
// one contiguous column of D_T^-1 per step, a coalesced stream at the HBM
// bound, where forward and backward substitution with L and U would be a
// chain of (p+1)^3 dependent steps.  It takes the same memory as the
// paper's packed LU factors.
//
// Build (one workgroup per cell, FP64): D_T is assembled in LDS entry by
// entry from the 1-D line operators without neighbour couplings
// (line_entry: volume, own-side face and boundary terms, advection and
// reaction), D_T[(i0,i1,i2),(j0,j1,j2)] = sum over the axes k of the line
// operator along k when the other two indices agree, and inverted in
// place by Gauss-Jordan elimination with partial (row) pivoting.  The
// result is stored transposed, column J of D_T^-1 contiguous:
// out[(c n3 + J) n3 + I] = (D_T^-1)[I][J], in FP64 or rounded to FP32.
#include <hip/hip_runtime.h>

#include "dg_internal.h"
#include "line_ops.h"

namespace dgmg {

int dmalloc(dg_problem *pr, void **p, size_t bytes);

namespace {

constexpr int kPmfThreads = 256;

template <int P, typename TO>
__global__ __launch_bounds__(kPmfThreads) void k_pmf_build(Geo g, TO *__restrict__ out, int *__restrict__ fail) {
  constexpr int N = P + 1;
  constexpr int M = N * N * N;
  constexpr DevTab<double, N> tb = make_ctab<double, N>();
  __shared__ double A[M * M];
  __shared__ double fcol[M];
  __shared__ int piv[M];
  __shared__ int prow;
  const int c = blockIdx.x;
  const int tid = threadIdx.x;
  int ijk[3];
  cell_coords(g, c, ijk);
  AxisCoef<double> f[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) f[k] = make_axis_coef<double>(g, c, k, ijk);
  const double vol = g.vol;
  const double cre = g.has_c ? g.c[c] : 0.0;
  const bool hasb = g.has_b != 0;
  const LineConv<double> zero = {0.0, 0.0, 0.0, 0.0};
  // ---- D_T, entry by entry ----------------------------------------------
  for (int e = tid; e < M * M; e += kPmfThreads) {
    const int I = e / M, J = e - I * M;
    const int i0 = I % N, i1 = (I / N) % N, i2 = I / (N * N);
    const int j0 = J % N, j1 = (J / N) % N, j2 = J / (N * N);
    double v = 0.0;
    if (i1 == j1 && i2 == j2) {  // x-line through (y, z) = (i1, i2)
      const LineConv<double> lc = hasb ? make_line_conv<double, N>(g, tb, 0, ijk, i1, i2) : zero;
      v += line_entry<double, N>(tb, f[0], tb.w[i1] * tb.w[i2], vol, cre, hasb, lc, i0, j0);
    }
    if (i0 == j0 && i2 == j2) {  // y-line through (x, z) = (i0, i2)
      const LineConv<double> lc = hasb ? make_line_conv<double, N>(g, tb, 1, ijk, i0, i2) : zero;
      v += line_entry<double, N>(tb, f[1], tb.w[i0] * tb.w[i2], vol, 0.0, hasb, lc, i1, j1);
    }
    if (i0 == j0 && i1 == j1) {  // z-line through (x, y) = (i0, i1)
      const LineConv<double> lc = hasb ? make_line_conv<double, N>(g, tb, 2, ijk, i0, i1) : zero;
      v += line_entry<double, N>(tb, f[2], tb.w[i0] * tb.w[i1], vol, 0.0, hasb, lc, i2, j2);
    }
    A[e] = v;
  }
  __syncthreads();
  // ---- in-place Gauss-Jordan inversion with partial pivoting ---------------
  for (int k = 0; k < M; ++k) {
    if (tid == 0) {
      int r = k;
      double best = fabs(A[k * M + k]);
      for (int i = k + 1; i < M; ++i) {
        const double v = fabs(A[i * M + k]);
        if (v > best) {
          best = v;
          r = i;
        }
      }
      prow = r;
      piv[k] = r;
      if (!(best > 0.0)) atomicExch(fail, 1);  // singular block: reported to the host
    }
    __syncthreads();
    const int r = prow;
    if (r != k) {
      for (int j = tid; j < M; j += kPmfThreads) {
        const double t = A[k * M + j];
        A[k * M + j] = A[r * M + j];
        A[r * M + j] = t;
      }
      __syncthreads();
    }
    const double pv = A[k * M + k];
    const double d = pv != 0.0 ? 1.0 / pv : 0.0;
    __syncthreads();
    // pivot row scaled; its diagonal becomes 1 / pivot
    for (int j = tid; j < M; j += kPmfThreads) A[k * M + j] = (j == k ? 1.0 : A[k * M + j]) * d;
    // the column multipliers, read before the elimination changes them
    for (int i = tid; i < M; i += kPmfThreads) fcol[i] = i == k ? 0.0 : A[i * M + k];
    __syncthreads();
    for (int e = tid; e < M * M; e += kPmfThreads) {
      const int i = e / M, j = e - i * M;
      if (i == k) continue;
      A[e] = (j == k ? 0.0 : A[e]) - fcol[i] * A[k * M + j];
    }
    __syncthreads();
  }
  // undo the row interchanges as column interchanges, last first
  for (int k = M - 1; k >= 0; --k) {
    const int r = piv[k];
    if (r != k) {
      for (int i = tid; i < M; i += kPmfThreads) {
        const double t = A[i * M + k];
        A[i * M + k] = A[i * M + r];
        A[i * M + r] = t;
      }
    }
    __syncthreads();
  }
  // ---- store transposed: column J of the inverse contiguous ----------------
  TO *o = out + (size_t)c * M * M;
  for (int e = tid; e < M * M; e += kPmfThreads) {
    const int J = e / M, I = e - J * M;
    o[e] = (TO)A[I * M + J];
  }
}

template <int P, typename TO>
int launch_pmf_build(const dg_problem *pr, TO *out, int *fail, hipStream_t s) {
  hipLaunchKernelGGL((k_pmf_build<P, TO>), dim3((unsigned)pr->ncell), dim3(kPmfThreads), 0, s, pr->geo, out, fail);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

template <typename TO>
int build_for(const dg_problem *pr, TO *out, int *fail, hipStream_t s) {
  switch (pr->p) {
    case 1: return launch_pmf_build<1, TO>(pr, out, fail, s);
    case 2: return launch_pmf_build<2, TO>(pr, out, fail, s);
    case 3: return launch_pmf_build<3, TO>(pr, out, fail, s);
    case 4: return launch_pmf_build<4, TO>(pr, out, fail, s);
  }
  set_error("the stored block inverses (DG_INNER_PMF) are built for p <= 4");
  return DG_EINVAL;
}

}  // namespace

size_t pmf_bytes(const dg_problem *pr, int prec) {
  const size_t m = (size_t)pr->nloc;
  return (size_t)pr->ncell * m * m * (prec == DG_FP64 ? sizeof(double) : sizeof(float));
}

int cast_d2f(int64_t n, double sc, const double *x, float *y, hipStream_t s);

// Stored inverses in the requested precision, built on first use,
// synchronously, on the null stream: the FP64 inverse always (FP32 is its
// rounding, so both precisions invert the same FP64 block).
int ensure_pmf(dg_problem *pr, int prec) {
  if (pr->pmf_built < 0) {
    set_error("the stored block inverses could not be built for this problem (a singular block or a failed launch)");
    return pr->pmf_built;
  }
  if (pr->pmf[prec]) return DG_OK;
  if (pr->p > 4) {
    set_error("the stored block inverses (DG_INNER_PMF) are built for p <= 4");
    return DG_EINVAL;
  }
  int rc;
  if (!pr->pmf[DG_FP64]) {
    void *buf = nullptr;
    if ((rc = dmalloc(pr, &buf, pmf_bytes(pr, DG_FP64)))) return rc;
    pr->pmf[DG_FP64] = buf;  // owned by the problem from here on
    pr->pmf_built = DG_EDEVICE;  // until the build has finished
    int *fail = (int *)pr->red_buf;  // reduction scratch, free outside a launch
    DG_HIP(hipMemsetAsync(fail, 0, sizeof(int), 0));
    if ((rc = build_for<double>(pr, (double *)buf, fail, 0))) return pr->pmf_built = rc;
    int hfail = 0;
    DG_HIP(hipMemcpy(&hfail, fail, sizeof(int), hipMemcpyDeviceToHost));
    if (hfail) {
      set_error("a diagonal block D_T is singular: no stored inverse");
      return pr->pmf_built = DG_EINVAL;
    }
    pr->pmf_built = 1;
  }
  if (prec == DG_FP32) {
    void *buf = nullptr;
    if ((rc = dmalloc(pr, &buf, pmf_bytes(pr, DG_FP32)))) return rc;
    const int64_t count = (int64_t)(pmf_bytes(pr, DG_FP32) / sizeof(float));
    if ((rc = cast_d2f(count, 1.0, (const double *)pr->pmf[DG_FP64], (float *)buf, 0)))
      return rc;  // buf stays with the problem's memory until it is destroyed
    pr->pmf[DG_FP32] = buf;
  }
  DG_HIP(hipStreamSynchronize(0));
  return DG_OK;
}

}  // namespace dgmg
