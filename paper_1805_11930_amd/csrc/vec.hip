// Vector kernels of the outer Krylov methods, the mixed-precision casts,
// the P0 intergrid transfers (Sec. 2.2.2: P|_T = (1,...,1)^T, R = P^T) and
// the levels of the simple P0 aggregation cycle used as coarse solver.
//
// Reductions are deterministic: a fixed grid of partial sums followed by a
// final sum of each result in one block, in a fixed order, so repeated
// calls on the same data give the same bits.
#include <hip/hip_runtime.h>

#include <utility>

#include "dg_internal.h"
#include "vec.h"

namespace dgmg {

constexpr int kRedThreads = 256;

// ---- deterministic dot products ------------------------------------------
// out[j] = sum_i a_j[i] * b_j[i] for M <= kMaxDots pairs in one pass.  Each
// thread loads U grid-stride elements before it adds them, in the order
// i, i + stride, ... (the order of the fused partial sums below).
template <int M>
__global__ __launch_bounds__(kRedThreads) void k_dots_partial(DotSet ds, int64_t n, double *__restrict__ part) {
  constexpr int U = 4;
  __shared__ double sh[M][kRedThreads / 64];
  double acc[M];
#pragma unroll
  for (int j = 0; j < M; ++j) acc[j] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kRedThreads;
  for (int64_t i0 = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i0 < n; i0 += U * stride) {
    double av[U][M], bv[U][M];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + u * stride;
      const int64_t ic = i < n ? i : i0;  // in bounds; not added below
#pragma unroll
      for (int j = 0; j < M; ++j) {
        av[u][j] = ds.a[j][ic];
        bv[u][j] = ds.b[j][ic];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (i0 + u * stride < n) {
#pragma unroll
        for (int j = 0; j < M; ++j) acc[j] += av[u][j] * bv[u][j];
      }
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < M; ++j) {
    double v = acc[j];
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    if (lane == 0) sh[j][wv] = v;
  }
  __syncthreads();
  if (threadIdx.x < M) {
    const int j = threadIdx.x;
    double s = 0.0;
    for (int w = 0; w < kRedThreads / 64; ++w) s += sh[j][w];
    part[(size_t)j * gridDim.x + blockIdx.x] = s;
  }
}

__global__ __launch_bounds__(kRedThreads) void k_dots_final(int m, int nblk, const double *__restrict__ part,
                                                             double *__restrict__ out) {
  __shared__ double sh[kRedThreads / 64];
  // one block per sum when launched with m blocks (same order either way)
  for (int j = blockIdx.x; j < m; j += gridDim.x) {
    double v = 0.0;
    for (int i = threadIdx.x; i < nblk; i += kRedThreads) v += part[(size_t)j * nblk + i];
    for (int mm = 32; mm >= 1; mm >>= 1) v += __shfl_xor(v, mm, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int w = 0; w < kRedThreads / 64; ++w) s += sh[w];
      out[j] = s;
    }
    __syncthreads();
  }
}

int dots(const DotSet &ds, int64_t n, double *part, double *out_dev, hipStream_t s) {
  switch (ds.m) {
    case 1: hipLaunchKernelGGL(k_dots_partial<1>, dim3(kDotBlocks), dim3(kRedThreads), 0, s, ds, n, part); break;
    case 2: hipLaunchKernelGGL(k_dots_partial<2>, dim3(kDotBlocks), dim3(kRedThreads), 0, s, ds, n, part); break;
    case 3: hipLaunchKernelGGL(k_dots_partial<3>, dim3(kDotBlocks), dim3(kRedThreads), 0, s, ds, n, part); break;
    case 4: hipLaunchKernelGGL(k_dots_partial<4>, dim3(kDotBlocks), dim3(kRedThreads), 0, s, ds, n, part); break;
    default: set_error("dots: 1..4 pairs"); return DG_EINVAL;
  }
  hipLaunchKernelGGL(k_dots_final, dim3(ds.m), dim3(kRedThreads), 0, s, ds.m, kDotBlocks, part, out_dev);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

// Sum j of many partials (one block of 1024 threads per sum): thread t
// adds part[j * nblk + t + 1024 k] over k in four interleaved
// accumulators (k mod 4, their loads in flight together), combined in
// order, then the wavefront and block sums in a fixed order.
constexpr int kFinThreads = 1024;
__global__ __launch_bounds__(kFinThreads) void k_sum_partials(int nblk, const double *__restrict__ part,
                                                              double *__restrict__ out) {
  __shared__ double sh[kFinThreads / 64];
  const double *pj = part + (size_t)blockIdx.x * nblk;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i0 = threadIdx.x; i0 < nblk; i0 += 4 * kFinThreads) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + u * kFinThreads;
      v[u] = i < nblk ? pj[i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] += v[u];
  }
  double t = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  for (int m = 32; m >= 1; m >>= 1) t += __shfl_xor(t, m, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < kFinThreads / 64; ++w) r += sh[w];
    out[blockIdx.x] = r;
  }
}

// Many partials: chunk c of sum j (kFinChunk entries, blockIdx = (c, j))
// is added as in k_sum_partials and its sum stored over the chunk's first
// entry (read only by this block, before the barrier); k_sum_chunks then
// adds the chunk sums of each sum in order.
constexpr int kFinChunk = 4 * kFinThreads;
__global__ __launch_bounds__(kFinThreads) void k_sum_chunk(int nblk, double *__restrict__ part) {
  __shared__ double sh[kFinThreads / 64];
  double *pc = part + (size_t)blockIdx.y * nblk + (size_t)blockIdx.x * kFinChunk;
  const int len = min(kFinChunk, nblk - (int)blockIdx.x * kFinChunk);
  double v[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int i = threadIdx.x + u * kFinThreads;
    v[u] = i < len ? pc[i] : 0.0;
  }
  double t = (v[0] + v[1]) + (v[2] + v[3]);
  for (int m = 32; m >= 1; m >>= 1) t += __shfl_xor(t, m, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < kFinThreads / 64; ++w) r += sh[w];
    pc[0] = r;
  }
}
__global__ __launch_bounds__(kRedThreads) void k_sum_chunks(int nblk, int nchunk, const double *__restrict__ part,
                                                            double *__restrict__ out) {
  __shared__ double sh[kRedThreads / 64];
  const double *pj = part + (size_t)blockIdx.x * nblk;
  double v = 0.0;
  for (int c = threadIdx.x; c < nchunk; c += kRedThreads) v += pj[(size_t)c * kFinChunk];
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int w = 0; w < kRedThreads / 64; ++w) r += sh[w];
    out[blockIdx.x] = r;
  }
}

// out[j] = the sum of part[j * nblk .. (j + 1) * nblk), j < m (part is
// overwritten above 4 * kFinChunk entries per sum)
int dots_final(int m, int nblk, double *part, double *out, hipStream_t s) {
  if (nblk > 4 * kFinChunk) {
    const int nchunk = (nblk + kFinChunk - 1) / kFinChunk;
    hipLaunchKernelGGL(k_sum_chunk, dim3(nchunk, m), dim3(kFinThreads), 0, s, nblk, part);
    hipLaunchKernelGGL(k_sum_chunks, dim3(m), dim3(kRedThreads), 0, s, nblk, nchunk, part, out);
    DG_HIP(hipGetLastError());
    return DG_OK;
  }
  hipLaunchKernelGGL(k_sum_partials, dim3(m), dim3(kFinThreads), 0, s, nblk, part, out);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

// ---- BLAS-1 -----------------------------------------------------------------
// y = a*x + b*y
__global__ void k_axpby(int64_t n, double a, const double *__restrict__ x, double b, double *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i] + b * y[i];
}
// z = x - y
__global__ void k_sub(int64_t n, const double *__restrict__ x, const double *__restrict__ y, double *__restrict__ z) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[i] = x[i] - y[i];
}
template <typename S, typename D>
__global__ void k_cast_scale(int64_t n, double s, const S *__restrict__ x, D *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (D)(s * (double)x[i]);
}

// Outer-iteration kernels with their scalars in device memory, so that an
// iteration is enqueued without waiting for the host.
// cg_alpha: a = rz / pq, or 0 on a breakdown (pq <= 0 or a not finite).
__device__ inline double cg_alpha(double rz, double pq, bool *bad) {
  double a = rz / pq;
  *bad = !(pq > 0.0) || !isfinite(a);
  return *bad ? 0.0 : a;
}
// x += a p (x == nullptr: left to k_beta_update, which reads p anyway) ;
// r_out = r_in - a q with a = cg_alpha (a breakdown leaves x and r
// unchanged and sets *flag = 1), and the partial
// sums of r_out . r_out (grid-stride over the fixed grid of k_dots_partial,
// same order; k_dots_final adds them)
__global__ __launch_bounds__(kRedThreads) void k_cg_update_rr(int64_t n, const double *__restrict__ rz,
                                                              const double *__restrict__ pq,
                                                              const double *__restrict__ p,
                                                              const double *__restrict__ q, double *__restrict__ x,
                                                              const double *r_in, double *r_out,
                                                              double *__restrict__ flag, double *__restrict__ part,
                                                              float *__restrict__ r32,
                                                              const double *__restrict__ rr_old,
                                                              double *__restrict__ rr_keep) {
  __shared__ double sh[kRedThreads / 64];
  bool bad;
  const double a = cg_alpha(*rz, *pq, &bad);
  // FP32 copy scaled by 1 / ||r|| of the previous iteration (the current
  // norm is what this pass computes); the factor's rr is kept for the cast
  // back of the preconditioned vector
  double sc = 1.0;
  if (r32) {
    const double r2 = *rr_old;
    sc = r2 > 0.0 ? 1.0 / sqrt(r2) : 1.0;
  }
  double acc = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kRedThreads;
  for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += stride) {
    if (x) x[i] += a * p[i];
    const double ro = r_in[i] - a * q[i];
    r_out[i] = ro;
    acc += ro * ro;
    if (r32) r32[i] = (float)(sc * ro);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (bad) *flag = 1.0;
    if (r32) *rr_keep = *rr_old;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
  if (lane == 0) sh[wv] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kRedThreads / 64; ++w) s += sh[w];
    part[blockIdx.x] = s;
  }
}

// z = (1 / (1 / sqrt(rr))) z32 (the inverse of the rounded factor
// 1 / sqrt(rr) that k_cg_update_rr scaled r32 by; 1 when rr is not
// positive) fused with the partial sums of z . b_j, j < m <= 2
// (the order of k_dots_partial; k_dots_final adds them)
__global__ __launch_bounds__(kRedThreads) void k_cast_back_dots(int64_t n, const double *__restrict__ rr,
                                                                const float *__restrict__ z32,
                                                                double *__restrict__ z, int m,
                                                                const double *__restrict__ b0,
                                                                const double *__restrict__ b1,
                                                                double *__restrict__ part) {
  __shared__ double sh[2][kRedThreads / 64];
  const double r2 = *rr;
  double sc = r2 > 0.0 ? 1.0 / sqrt(r2) : 1.0;
  sc = 1.0 / sc;
  double acc0 = 0.0, acc1 = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kRedThreads;
  for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += stride) {
    const double zi = (double)(sc * (double)z32[i]);
    z[i] = zi;
    acc0 += zi * b0[i];
    if (m > 1) acc1 += zi * b1[i];
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int k = 32; k >= 1; k >>= 1) {
    acc0 += __shfl_xor(acc0, k, 64);
    acc1 += __shfl_xor(acc1, k, 64);
  }
  if (lane == 0) {
    sh[0][wv] = acc0;
    sh[1][wv] = acc1;
  }
  __syncthreads();
  if (threadIdx.x < m) {
    const int j = threadIdx.x;
    double t = 0.0;
    for (int w = 0; w < kRedThreads / 64; ++w) t += sh[j][w];
    part[(size_t)j * gridDim.x + blockIdx.x] = t;
  }
}

// p = z + beta p with beta = (zr - zro) / rz_old (flexible CG) or
// zr / rz_old; thread 0 stores rz_new = zr (rz_new is not rz_old).  With
// x: first x += a p of the old p, a = cg_alpha(rz_old, pq) (the update
// k_cg_update_rr left out).
__global__ void k_beta_update(int64_t n, const double *__restrict__ zr, const double *__restrict__ zro,
                              const double *__restrict__ rz_old, double *__restrict__ rz_new, int flex,
                              const double *__restrict__ z, double *__restrict__ p, double *__restrict__ x,
                              const double *__restrict__ pq) {
  const double b = flex ? (*zr - *zro) / *rz_old : *zr / *rz_old;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double po = p[i];
    if (x) {
      bool bad;
      x[i] += cg_alpha(*rz_old, *pq, &bad) * po;
    }
    p[i] = 1.0 * z[i] + b * po;
  }
  if (i == 0) *rz_new = *zr;
}
static inline dim3 grid1(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

int axpby(int64_t n, double a, const double *x, double b, double *y, hipStream_t s) {
  hipLaunchKernelGGL(k_axpby, grid1(n), dim3(256), 0, s, n, a, x, b, y);
  DG_HIP(hipGetLastError());
  return DG_OK;
}
int sub(int64_t n, const double *x, const double *y, double *z, hipStream_t s) {
  hipLaunchKernelGGL(k_sub, grid1(n), dim3(256), 0, s, n, x, y, z);
  DG_HIP(hipGetLastError());
  return DG_OK;
}
int cg_update_rr(int64_t n, const double *rz, const double *pq, const double *p, const double *q, double *x,
                 const double *r_in, double *r_out, double *flag, double *part, double *rr, hipStream_t s,
                 float *r32, const double *rr_old, double *rr_keep) {
  hipLaunchKernelGGL(k_cg_update_rr, dim3(kDotBlocks), dim3(kRedThreads), 0, s, n, rz, pq, p, q, x, r_in, r_out, flag,
                     part, r32, rr_old, rr_keep);
  hipLaunchKernelGGL(k_dots_final, dim3(1), dim3(kRedThreads), 0, s, 1, kDotBlocks, part, rr);
  DG_HIP(hipGetLastError());
  return DG_OK;
}
int beta_update(int64_t n, const double *zr, const double *zro, const double *rz_old, double *rz_new, bool flex,
                const double *z, double *p, hipStream_t s, double *x, const double *pq) {
  if ((x == nullptr) != (pq == nullptr)) {
    set_error("internal: beta_update takes x and pq together");
    return DG_EINVAL;
  }
  hipLaunchKernelGGL(k_beta_update, grid1(n), dim3(256), 0, s, n, zr, zro, rz_old, rz_new, flex ? 1 : 0, z, p, x,
                     pq);
  DG_HIP(hipGetLastError());
  return DG_OK;
}
int cast_back_dots(int64_t n, const double *rr, const float *z32, double *z, int m, const double *b0,
                   const double *b1, double *part, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_cast_back_dots, dim3(kDotBlocks), dim3(kRedThreads), 0, s, n, rr, z32, z, m, b0, b1, part);
  hipLaunchKernelGGL(k_dots_final, dim3(m), dim3(kRedThreads), 0, s, m, kDotBlocks, part, out);
  DG_HIP(hipGetLastError());
  return DG_OK;
}
int cast_d2f(int64_t n, double sc, const double *x, float *y, hipStream_t s) {
  hipLaunchKernelGGL((k_cast_scale<double, float>), grid1(n), dim3(256), 0, s, n, sc, x, y);
  DG_HIP(hipGetLastError());
  return DG_OK;
}
int cast_f2d(int64_t n, double sc, const float *x, double *y, hipStream_t s) {
  hipLaunchKernelGGL((k_cast_scale<float, double>), grid1(n), dim3(256), 0, s, n, sc, x, y);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

// ---- P0 transfers ---------------------------------------------------------
// rh[c] = sum_{i in T_c} (r[i] - ar[i])  (restriction of the residual; ar may be null)
template <typename T>
__global__ void k_restrict(int64_t ncell, int nloc, const T *__restrict__ r, const T *__restrict__ ar,
                           T *__restrict__ rh) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncell) return;
  T s = T(0);
  const T *rc = r + c * nloc;
  if (ar) {
    const T *ac = ar + c * nloc;
    for (int i = 0; i < nloc; ++i) s += rc[i] - ac[i];
  } else {
    for (int i = 0; i < nloc; ++i) s += rc[i];
  }
  rh[c] = s;
}
// u[i] += zh[cell(i)]
template <typename T>
__global__ void k_prolong_add(int64_t n, int nloc, const T *__restrict__ zh, T *__restrict__ u) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) u[i] += zh[i / nloc];
}

template <typename T>
int restrict_p0(int64_t ncell, int nloc, const T *r, const T *ar, T *rh, hipStream_t s) {
  hipLaunchKernelGGL((k_restrict<T>), grid1(ncell), dim3(256), 0, s, ncell, nloc, r, ar, rh);
  DG_HIP(hipGetLastError());
  return DG_OK;
}
template <typename T>
int prolong_add_p0(int64_t n, int nloc, const T *zh, T *u, hipStream_t s) {
  hipLaunchKernelGGL((k_prolong_add<T>), grid1(n), dim3(256), 0, s, n, nloc, zh, u);
  DG_HIP(hipGetLastError());
  return DG_OK;
}
template int restrict_p0<double>(int64_t, int, const double *, const double *, double *, hipStream_t);
template int restrict_p0<float>(int64_t, int, const float *, const float *, float *, hipStream_t);
template int prolong_add_p0<double>(int64_t, int, const double *, double *, hipStream_t);
template int prolong_add_p0<float>(int64_t, int, const float *, float *, hipStream_t);

// ---- P0 aggregation levels (7-point stencils) ------------------------------
// A[0][i] = diagonal, A[1..6][i] = couplings to -x,+x,-y,+y,-z,+z.
// All 14 loads are issued before the first product (a neighbour outside
// the grid reads the point itself and its term is not added), the terms
// added in the order of the couplings.
template <typename T>
__device__ inline T stencil_apply(const T *__restrict__ A, int64_t n, const T *__restrict__ x, int i, int ix, int iy,
                                  int iz, int nx, int ny, int nz) {
  const bool in[6] = {ix > 0, ix < nx - 1, iy > 0, iy < ny - 1, iz > 0, iz < nz - 1};
  const int off[6] = {-1, 1, -nx, nx, -nx * ny, nx * ny};
  T a[7], v[7];
  a[0] = A[i];
  v[0] = x[i];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    a[k + 1] = A[(k + 1) * n + i];
    v[k + 1] = x[in[k] ? i + off[k] : i];
  }
  T s = a[0] * v[0];
#pragma unroll
  for (int k = 0; k < 6; ++k)
    if (in[k]) s += a[k + 1] * v[k + 1];
  return s;
}

// one damped Jacobi sweep xo = xi + w D^-1 (r - A xi); xi == null means xi = 0
template <typename T>
__global__ void k_jacobi(const T *__restrict__ A, int nx, int ny, int nz, T w, const T *__restrict__ r,
                         const T *__restrict__ xi, T *__restrict__ xo) {
  const int n = nx * ny * nz;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (!xi) {
    xo[i] = w * r[i] / A[i];
    return;
  }
  const int ix = i % nx, iy = (i / nx) % ny, iz = i / (nx * ny);
  const T ax = stencil_apply(A, n, xi, i, ix, iy, iz, nx, ny, nz);
  xo[i] = xi[i] + w * (r[i] - ax) / A[i];
}

// rc[agg] = sum over the aggregate of (r - A x)
template <typename T>
__global__ void k_coarse_restrict(const T *__restrict__ A, int nx, int ny, int nz, const T *__restrict__ r,
                                  const T *__restrict__ x, int cnx, int cny, int cnz, T *__restrict__ rc) {
  const int nc = cnx * cny * cnz;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nc) return;
  const int jx = j % cnx, jy = (j / cnx) % cny, jz = j / (cnx * cny);
  const int n = nx * ny * nz;
  // the eight children, unrolled with clamped coordinates so that their
  // loads can be in flight together; a child outside the grid is not added
  T s = T(0);
#pragma unroll
  for (int dz = 0; dz < 2; ++dz)
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
      for (int dx = 0; dx < 2; ++dx) {
        const int ix = 2 * jx + dx, iy = 2 * jy + dy, iz = 2 * jz + dz;
        const bool inside = ix < nx && iy < ny && iz < nz;
        const int cx = inside ? ix : 2 * jx, cy = inside ? iy : 2 * jy, cz = inside ? iz : 2 * jz;
        const int i = cx + nx * (cy + ny * cz);
        const T t = r[i] - stencil_apply(A, n, x, i, cx, cy, cz, nx, ny, nz);
        if (inside) s += t;
      }
  rc[j] = s;
}

// x += xc[agg(i)]
template <typename T>
__global__ void k_coarse_prolong(int nx, int ny, int nz, int cnx, int cny, const T *__restrict__ xc,
                                 T *__restrict__ x) {
  const int n = nx * ny * nz;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int ix = i % nx, iy = (i / nx) % ny, iz = i / (nx * ny);
  x[i] += xc[(ix >> 1) + cnx * ((iy >> 1) + cny * (iz >> 1))];
}

// x = Ainv r, dense (n <= 512): one wavefront per row, coalesced row reads
template <typename T>
__global__ __launch_bounds__(256) void k_dense_mv(int n, const T *__restrict__ Ainv, const T *__restrict__ r,
                                                  T *__restrict__ x) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;  // uniform per wavefront
  T s = T(0);
  for (int j = lane; j < n; j += 64) s += Ainv[(size_t)row * n + j] * r[j];
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m, 64);
  if (lane == 0) x[row] = s;
}

template <typename T>
int coarse_jacobi(const T *A, int nx, int ny, int nz, T w, const T *r, const T *xi, T *xo, hipStream_t s) {
  const int n = nx * ny * nz;
  hipLaunchKernelGGL((k_jacobi<T>), dim3((n + 255) / 256), dim3(256), 0, s, A, nx, ny, nz, w, r, xi, xo);
  DG_HIP(hipGetLastError());
  return DG_OK;
}
template <typename T>
int coarse_restrict(const T *A, int nx, int ny, int nz, const T *r, const T *x, int cnx, int cny, int cnz, T *rc,
                    hipStream_t s) {
  const int nc = cnx * cny * cnz;
  hipLaunchKernelGGL((k_coarse_restrict<T>), dim3((nc + 255) / 256), dim3(256), 0, s, A, nx, ny, nz, r, x, cnx,
                     cny, cnz, rc);
  DG_HIP(hipGetLastError());
  return DG_OK;
}
template <typename T>
int coarse_prolong(int nx, int ny, int nz, int cnx, int cny, const T *xc, T *x, hipStream_t s) {
  const int n = nx * ny * nz;
  hipLaunchKernelGGL((k_coarse_prolong<T>), dim3((n + 255) / 256), dim3(256), 0, s, nx, ny, nz, cnx, cny, xc, x);
  DG_HIP(hipGetLastError());
  return DG_OK;
}
template <typename T>
int dense_mv(int n, const T *Ainv, const T *r, T *x, hipStream_t s) {
  hipLaunchKernelGGL((k_dense_mv<T>), dim3((n + 3) / 4), dim3(256), 0, s, n, Ainv, r, x);
  DG_HIP(hipGetLastError());
  return DG_OK;
}
#define DG_INST(T)                                                                                          \
  template int coarse_jacobi<T>(const T *, int, int, int, T, const T *, const T *, T *, hipStream_t);       \
  template int coarse_restrict<T>(const T *, int, int, int, const T *, const T *, int, int, int, T *,       \
                                  hipStream_t);                                                             \
  template int coarse_prolong<T>(int, int, int, int, int, const T *, T *, hipStream_t);                     \
  template int dense_mv<T>(int, const T *, const T *, T *, hipStream_t);
DG_INST(double)
DG_INST(float)
#undef DG_INST


// ---- Gram-Schmidt passes of the Arnoldi step in FGMRES --------------------
// The basis size M is a compile-time constant so that the M loads of one
// element are all in flight before the first is used.  MODE 0: part = V_i . w;
// MODE 1: w -= sum_i h_i V_i, then part = V_i . w of the new w (first update
// and second projection of classical Gram-Schmidt applied twice, one pass);
// MODE 2: w -= sum_i h_i V_i, then part = w . w.  h is in device memory.
template <int M, int MODE>
__global__ __launch_bounds__(kRedThreads) void k_gs(VecList vl, const double *__restrict__ h, double *__restrict__ w,
                                                    int64_t n, double *__restrict__ part) {
  constexpr int NA = MODE == 2 ? 1 : M;
  __shared__ double sh[NA][kRedThreads / 64];
  double acc[NA];
#pragma unroll
  for (int j = 0; j < NA; ++j) acc[j] = 0.0;
  double hc[M];
#pragma unroll
  for (int j = 0; j < M; ++j) hc[j] = MODE == 0 ? 0.0 : h[j];
  const int64_t stride = (int64_t)gridDim.x * kRedThreads;
  for (int64_t i = (int64_t)blockIdx.x * kRedThreads + threadIdx.x; i < n; i += stride) {
    double v[M];
#pragma unroll
    for (int j = 0; j < M; ++j) v[j] = vl.v[j][i];
    double wi = w[i];
    // all M + 1 loads before the first product (at large M the scheduler
    // would otherwise trade them for registers and issue one at a time)
    __builtin_amdgcn_sched_barrier(0);
    if (MODE != 0) {
#pragma unroll
      for (int j = 0; j < M; ++j) wi -= hc[j] * v[j];
      w[i] = wi;
    }
    if (MODE == 2) {
      acc[0] += wi * wi;
    } else {
#pragma unroll
      for (int j = 0; j < M; ++j) acc[j] += v[j] * wi;
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < NA; ++j) {
    double t = acc[j];
    for (int mm = 32; mm >= 1; mm >>= 1) t += __shfl_xor(t, mm, 64);
    if (lane == 0) sh[j][wv] = t;
  }
  __syncthreads();
  if ((int)threadIdx.x < NA) {
    const int j = threadIdx.x;
    double t = 0.0;
    for (int q = 0; q < kRedThreads / 64; ++q) t += sh[j][q];
    part[(size_t)j * gridDim.x + blockIdx.x] = t;
  }
}

using GsKernel = void (*)(VecList, const double *, double *, int64_t, double *);
template <int MODE, int... I>
static GsKernel gs_pick(int m, std::integer_sequence<int, I...>) {
  static const GsKernel tab[] = {&k_gs<I + 1, MODE>...};
  return tab[m - 1];
}
template <int MODE>
static int gs_pass(const VecList &vl, int m, const double *h_dev, double *w, int64_t n, double *part, double *out_dev,
                   hipStream_t s) {
  if (m < 1 || m > kMaxBasis) {
    set_error("Gram-Schmidt pass: basis size out of range");
    return DG_EINVAL;
  }
  const GsKernel k = gs_pick<MODE>(m, std::make_integer_sequence<int, kMaxBasis>{});
  hipLaunchKernelGGL(k, dim3(kDotBlocks), dim3(kRedThreads), 0, s, vl, h_dev, w, n, part);
  const int na = MODE == 2 ? 1 : m;
  hipLaunchKernelGGL(k_dots_final, dim3(na), dim3(kRedThreads), 0, s, na, kDotBlocks, part, out_dev);
  DG_HIP(hipGetLastError());
  return DG_OK;
}
int gs_dot(const VecList &vl, int m, const double *w, int64_t n, double *part, double *out_dev, hipStream_t s) {
  return gs_pass<0>(vl, m, nullptr, const_cast<double *>(w), n, part, out_dev, s);
}
int gs_update_dot(const VecList &vl, int m, const double *h_dev, double *w, int64_t n, double *part,
                  double *out_dev, hipStream_t s) {
  return gs_pass<1>(vl, m, h_dev, w, n, part, out_dev, s);
}
int gs_update_norm(const VecList &vl, int m, const double *h_dev, double *w, int64_t n, double *part,
                   double *out_dev, hipStream_t s) {
  return gs_pass<2>(vl, m, h_dev, w, n, part, out_dev, s);
}

// x += sum_i y_i Z_i
__global__ void k_mcombine(VecList vl, Coefs y, int m, int64_t n, double *__restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = x[i];
  for (int j = 0; j < m; ++j) s += y.c[j] * vl.v[j][i];
  x[i] = s;
}

int mcombine(const VecList &vl, const Coefs &y, int m, int64_t n, double *x, hipStream_t s) {
  hipLaunchKernelGGL(k_mcombine, grid1(n), dim3(256), 0, s, vl, y, m, n, x);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

// ---- smoother statistics: sum and max of the per-cell iteration counts ----
__global__ void k_iter_stats(int64_t n, const int *__restrict__ it, unsigned long long *__restrict__ out) {
  // single block, deterministic
  __shared__ unsigned long long ssum[256];
  __shared__ int smax[256];
  unsigned long long s = 0;
  int m = 0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    s += (unsigned long long)it[i];
    m = it[i] > m ? it[i] : m;
  }
  ssum[threadIdx.x] = s;
  smax[threadIdx.x] = m;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      ssum[threadIdx.x] += ssum[threadIdx.x + w];
      smax[threadIdx.x] = smax[threadIdx.x] > smax[threadIdx.x + w] ? smax[threadIdx.x] : smax[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = ssum[0];
    out[1] = (unsigned long long)smax[0];
  }
}

int iter_stats(int64_t n, const int *it, unsigned long long *out_dev, hipStream_t s) {
  hipLaunchKernelGGL(k_iter_stats, dim3(1), dim3(256), 0, s, n, it, out_dev);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

// acc[0] += sum it, acc[1] = max(acc[1], max it), acc[2] += n: the counts of
// one smoothing step added to a solve's running totals (integer atomics, so
// the totals do not depend on the order of the blocks)
__global__ __launch_bounds__(256) void k_iter_accum(int64_t n, const int *__restrict__ it,
                                                    unsigned long long *__restrict__ acc) {
  __shared__ unsigned long long ssum[4];
  __shared__ unsigned long long smax[4];
  unsigned long long s = 0, m = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const unsigned long long v = (unsigned long long)it[i];
    s += v;
    m = v > m ? v : m;
  }
  for (int k = 32; k >= 1; k >>= 1) {
    s += __shfl_xor(s, k, 64);
    const unsigned long long o = __shfl_xor(m, k, 64);
    m = o > m ? o : m;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    ssum[wv] = s;
    smax[wv] = m;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long ts = 0, tm = 0;
    for (int w = 0; w < 4; ++w) {
      ts += ssum[w];
      tm = smax[w] > tm ? smax[w] : tm;
    }
    atomicAdd(&acc[0], ts);
    atomicMax(&acc[1], tm);
    if (blockIdx.x == 0) atomicAdd(&acc[2], (unsigned long long)n);
  }
}

int iter_accum(int64_t n, const int *it, unsigned long long *acc_dev, hipStream_t s) {
  const int64_t nb = (n + 255) / 256;
  const int g = (int)(nb < 512 ? (nb > 0 ? nb : 1) : 512);
  hipLaunchKernelGGL(k_iter_accum, dim3(g), dim3(256), 0, s, n, it, acc_dev);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

}  // namespace dgmg
