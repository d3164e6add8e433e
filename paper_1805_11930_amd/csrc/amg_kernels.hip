// Kernels of the aggregation-AMG levels (CSR matrices set up in amg.cpp):
// damped Jacobi with the stored smoothing diagonal, residual, and the
// transfers R (restriction) and P (prolongation, added to the finer
// iterate) as CSR products.  A group of LPR lanes (a power of two chosen
// from the mean row length) takes one row: the lanes read consecutive
// entries of the row, so the loads of a wavefront coalesce, and the partial
// sums meet in a butterfly inside the group.
#include <hip/hip_runtime.h>

#include "dg_internal.h"
#include "vec.h"

namespace dgmg {

namespace {

constexpr int kCsrThreads = 256;

// sum over row i of v[k] * x[ci[k]] by the LPR lanes of the row's group.
// Four entries per lane and step: their column indices and values, then
// the four gathers of x, are in flight together; the products are added
// in entry order (as one entry per step would).
template <int LPR, typename T>
__device__ inline T row_dot(int i, int j, const int *__restrict__ rp, const int *__restrict__ ci,
                            const T *__restrict__ v, const T *__restrict__ x) {
  constexpr int U = 4;
  T s = T(0);
  const int e = rp[i + 1];
  for (int k0 = rp[i] + j; k0 < e; k0 += U * LPR) {
    int c[U];
    T a[U], xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + u * LPR;
      const int kc = k < e ? k : k0;  // in the row; not added below
      c[u] = ci[kc];
      a[u] = v[kc];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) xv[u] = x[c[u]];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (k0 + u * LPR < e) s += a[u] * xv[u];
  }
#pragma unroll
  for (int m = LPR / 2; m >= 1; m >>= 1) s += __shfl_xor(s, m, LPR);
  return s;
}

// mode 0: xo = xi + w dinv (r - A xi) (xi == NULL: xo = w dinv r);
// mode 1: xo = r - A xi (residual); mode 2: xo (+)= A xi (add: `add`)
template <int LPR, typename T>
__global__ __launch_bounds__(kCsrThreads) void k_csr(int mode, int n, const int *__restrict__ rp,
                                                     const int *__restrict__ ci, const T *__restrict__ v,
                                                     const T *__restrict__ dinv, T w, const T *__restrict__ r,
                                                     const T *__restrict__ xi, T *__restrict__ xo, int add) {
  const int g = blockIdx.x * (kCsrThreads / LPR) + (int)threadIdx.x / LPR;
  const int j = (int)threadIdx.x % LPR;
  const bool ok = g < n;
  const int i = ok ? g : n - 1;  // the whole group takes part in the butterfly
  T s = T(0);
  if (xi) s = row_dot<LPR, T>(i, j, rp, ci, v, xi);
  if (!ok || j != 0) return;
  if (mode == 0)
    xo[i] = xi ? xi[i] + w * dinv[i] * (r[i] - s) : w * dinv[i] * r[i];
  else if (mode == 1)
    xo[i] = r[i] - s;
  else
    xo[i] = add ? xo[i] + s : s;
}

template <typename T>
int launch_csr(int mode, int n, int nnz, const int *rp, const int *ci, const T *v, const T *dinv, T w, const T *r,
               const T *xi, T *xo, int add, hipStream_t s) {
  const int mean = n > 0 ? nnz / n : 0;
#define DG_CSR(LPR)                                                                                          \
  hipLaunchKernelGGL((k_csr<LPR, T>), dim3((unsigned)((n + kCsrThreads / LPR - 1) / (kCsrThreads / LPR))),    \
                     dim3(kCsrThreads), 0, s, mode, n, rp, ci, v, dinv, w, r, xi, xo, add)
  if (mean >= 24)
    DG_CSR(16);
  else if (mean >= 8)
    DG_CSR(8);
  else if (mean >= 3)
    DG_CSR(4);
  else
    DG_CSR(1);
#undef DG_CSR
  DG_HIP(hipGetLastError());
  return DG_OK;
}

}  // namespace

template <typename T>
int csr_jacobi(int n, int nnz, const int *rp, const int *ci, const T *v, const T *dinv, T w, const T *r, const T *xi,
               T *xo, hipStream_t s) {
  return launch_csr<T>(0, n, nnz, rp, ci, v, dinv, w, r, xi, xo, 0, s);
}

template <typename T>
int csr_residual(int n, int nnz, const int *rp, const int *ci, const T *v, const T *r, const T *x, T *out,
                 hipStream_t s) {
  return launch_csr<T>(1, n, nnz, rp, ci, v, nullptr, T(0), r, x, out, 0, s);
}

template <typename T>
int csr_spmv(int n, int nnz, const int *rp, const int *ci, const T *v, const T *x, T *y, bool add, hipStream_t s) {
  return launch_csr<T>(2, n, nnz, rp, ci, v, nullptr, T(0), nullptr, x, y, add ? 1 : 0, s);
}

#define DG_INST(T)                                                                                              \
  template int csr_jacobi<T>(int, int, const int *, const int *, const T *, const T *, T, const T *, const T *, \
                             T *, hipStream_t);                                                                 \
  template int csr_residual<T>(int, int, const int *, const int *, const T *, const T *, const T *, T *,         \
                               hipStream_t);                                                                    \
  template int csr_spmv<T>(int, int, const int *, const int *, const T *, const T *, T *, bool, hipStream_t);
DG_INST(double)
DG_INST(float)
#undef DG_INST

}  // namespace dgmg
