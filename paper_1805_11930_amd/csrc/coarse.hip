// Kernels of the conforming Q1 coarse space (Sec. 2.2.2-2.2.3, App. A.2):
// the transfers between the DG space and the vertex grid, and the levels of
// the vertex-grid multigrid cycle used as the coarse solver.
//
// Vertex grid of a level: vx * vy * vz unknowns, x fastest.  Level 0 has
// one unknown per mesh vertex, (nx+1)(ny+1)(nz+1).  Its matrix is the
// 27-point stencil A[o][i], o = (dx+1) + 3 (dy+1) + 9 (dz+1) for the
// coupling of vertex i to vertex i + (dx, dy, dz).
//
// Coarsening between vertex levels keeps every second vertex along each
// axis and always the last one: coarse vertex J sits on fine vertex
// min(2J, vf-1), so vc = vf/2 + 1.  Interpolation is linear along each
// axis (the nodal interpolation of a coarser trilinear function), and the
// coarse matrix is the Galerkin product P^T A P (built on the host).
#include "dg_internal.h"
#include "vec.h"

namespace dgmg {

namespace {

inline dim3 grid_for(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

// 1-D interpolation weights of fine vertex i: coarse J0 (and J0+1 when
// two == true) with weights 1 (or 1/2, 1/2).
struct W1 {
  int j0;
  bool two;
};
__device__ inline W1 interp1(int i, int vf, int vc) {
  if (i == vf - 1) return {vc - 1, false};
  if ((i & 1) == 0) return {i >> 1, false};
  return {i >> 1, true};
}

// (A x)_i for the 27-point stencil.  Couplings to unknowns outside the grid
// are exact zeros in every level's stencil (the level-0 matrix only couples
// vertices of a common cell, and Galerkin products keep that), so the
// neighbour index is clamped into the grid instead of branching: all 54
// loads are independent and issue at once.
template <typename T>
__device__ inline T stencil27(const T *__restrict__ A, int64_t n, const T *__restrict__ x, int64_t i, int ix, int iy,
                              int iz, int vx, int vy, int vz) {
  const int ox[3] = {ix > 0 ? -1 : 0, 0, ix < vx - 1 ? 1 : 0};
  const int64_t oy[3] = {iy > 0 ? -(int64_t)vx : 0, 0, iy < vy - 1 ? (int64_t)vx : 0};
  const int64_t oz[3] = {iz > 0 ? -(int64_t)vx * vy : 0, 0, iz < vz - 1 ? (int64_t)vx * vy : 0};
  T s = T(0);
#pragma unroll
  for (int dz = 0; dz < 3; ++dz)
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
      for (int dx = 0; dx < 3; ++dx) {
        const int o = dx + 3 * dy + 9 * dz;
        s += A[o * n + i] * x[i + ox[dx] + oy[dy] + oz[dz]];
      }
  return s;
}

// xo = xi + w Dinv (r - A xi); xi == null means xi = 0.  Dinv is the
// inverse of half the l1 row norm (see CoarseLevel).
template <typename T>
__global__ void k_jacobi27(const T *__restrict__ A, const T *__restrict__ dinv, int vx, int vy, int vz, T w,
                           const T *__restrict__ r, const T *__restrict__ xi, T *__restrict__ xo) {
  const int64_t n = (int64_t)vx * vy * vz;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const T wd = w * dinv[i];
  if (!xi) {
    xo[i] = wd * r[i];
    return;
  }
  const int ix = (int)(i % vx), iy = (int)((i / vx) % vy), iz = (int)(i / ((int64_t)vx * vy));
  xo[i] = xi[i] + wd * (r[i] - stencil27(A, n, xi, i, ix, iy, iz, vx, vy, vz));
}

// out = r - A x
template <typename T>
__global__ void k_residual27(const T *__restrict__ A, int vx, int vy, int vz, const T *__restrict__ r,
                             const T *__restrict__ x, T *__restrict__ out) {
  const int64_t n = (int64_t)vx * vy * vz;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int ix = (int)(i % vx), iy = (int)((i / vx) % vy), iz = (int)(i / ((int64_t)vx * vy));
  out[i] = r[i] - stencil27(A, n, x, i, ix, iy, iz, vx, vy, vz);
}

// rc = P^T t: coarse J gathers the fine vertices within one fine step of
// its own fine position, with their interpolation weights towards J.
// When xz is not null, also xz = w dinv rc: the first damped Jacobi sweep
// from zero on the coarse level.
template <typename T>
__global__ void k_restrict27(int vx, int vy, int vz, const T *__restrict__ t, int cx, int cy, int cz,
                             T *__restrict__ rc, const T *__restrict__ dinv, T w, T *__restrict__ xz) {
  const int64_t nc = (int64_t)cx * cy * cz;
  const int64_t J = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (J >= nc) return;
  const int jj[3] = {(int)(J % cx), (int)((J / cx) % cy), (int)(J / ((int64_t)cx * cy))};
  const int vf[3] = {vx, vy, vz}, vcs[3] = {cx, cy, cz};
  // per axis: up to three fine indices and their weights towards jj
  int fi[3][3];
  T fw[3][3];
  int cnt[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    cnt[k] = 0;
    const int f = min(2 * jj[k], vf[k] - 1);
#pragma unroll
    for (int d = -1; d <= 1; ++d) {
      const int i = f + d;
      if (i < 0 || i >= vf[k]) continue;
      const W1 w = interp1(i, vf[k], vcs[k]);
      T wt = T(0);
      if (w.j0 == jj[k]) wt = w.two ? T(0.5) : T(1);
      else if (w.two && w.j0 + 1 == jj[k]) wt = T(0.5);
      if (wt != T(0)) {
        fi[k][cnt[k]] = i;
        fw[k][cnt[k]] = wt;
        ++cnt[k];
      }
    }
  }
  T s = T(0);
  for (int c = 0; c < cnt[2]; ++c)
    for (int b = 0; b < cnt[1]; ++b)
      for (int a = 0; a < cnt[0]; ++a)
        s += fw[0][a] * fw[1][b] * fw[2][c] * t[fi[0][a] + (int64_t)vx * (fi[1][b] + (int64_t)vy * fi[2][c])];
  rc[J] = s;
  if (xz) xz[J] = w * dinv[J] * s;
}

// x += P xc (trilinear interpolation from the coarser vertex level)
template <typename T>
__global__ void k_prolong27(int vx, int vy, int vz, int cx, int cy, int cz, const T *__restrict__ xc,
                            T *__restrict__ x) {
  const int64_t n = (int64_t)vx * vy * vz;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int ii[3] = {(int)(i % vx), (int)((i / vx) % vy), (int)(i / ((int64_t)vx * vy))};
  const int vf[3] = {vx, vy, vz}, vcs[3] = {cx, cy, cz};
  int j[3][2];
  T w[3][2];
  int cnt[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const W1 q = interp1(ii[k], vf[k], vcs[k]);
    j[k][0] = q.j0;
    j[k][1] = q.j0 + 1;
    w[k][0] = q.two ? T(0.5) : T(1);
    w[k][1] = T(0.5);
    cnt[k] = q.two ? 2 : 1;
  }
  T s = T(0);
  for (int c = 0; c < cnt[2]; ++c)
    for (int b = 0; b < cnt[1]; ++b)
      for (int a = 0; a < cnt[0]; ++a)
        s += w[0][a] * w[1][b] * w[2][c] * xc[j[0][a] + (int64_t)cx * (j[1][b] + (int64_t)cy * j[2][c])];
  x[i] += s;
}

// r_hat[v] = sum over the (up to eight) cells around vertex v of that
// cell's corner sum for the corner at v: the restriction R = P^T of the
// Q1 prolongation, second half (the first half, the per-cell corner sums,
// is fused into the residual kernel).
template <typename T>
__global__ void k_q1_gather(int nx, int ny, int nz, const T *__restrict__ cs, T *__restrict__ rv,
                            const T *__restrict__ dinv, T w, T *__restrict__ xz) {
  const int vx = nx + 1, vy = ny + 1;
  const int64_t n = (int64_t)vx * vy * (nz + 1);
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int ix = (int)(v % vx), iy = (int)((v / vx) % vy), iz = (int)(v / ((int64_t)vx * vy));
  T s = T(0);
#pragma unroll
  for (int sz = 0; sz < 2; ++sz) {
    const int cz = iz - 1 + sz;
    if (cz < 0 || cz >= nz) continue;
#pragma unroll
    for (int sy = 0; sy < 2; ++sy) {
      const int cyy = iy - 1 + sy;
      if (cyy < 0 || cyy >= ny) continue;
#pragma unroll
      for (int sx = 0; sx < 2; ++sx) {
        const int cxx = ix - 1 + sx;
        if (cxx < 0 || cxx >= nx) continue;
        const int64_t c = cxx + (int64_t)nx * (cyy + (int64_t)ny * cz);
        // the vertex is corner (1-sx, 1-sy, 1-sz) of that cell
        s += cs[8 * c + (1 - sx) + 2 * (1 - sy) + 4 * (1 - sz)];
      }
    }
  }
  rv[v] = s;
  if (xz) xz[v] = w * dinv[v] * s;
}

// u += P x_hat: every DG node receives the trilinear interpolant of the
// vertex values of its cell, evaluated at the node (Sec. 2.2.2).
template <int N, typename T>
__global__ void k_q1_prolong_add(int nx, int ny, int nz, const T *__restrict__ xv, T *__restrict__ u) {
  constexpr int N3 = N * N * N;
  constexpr DevTab<T, N> tb = make_ctab<T, N>();
  const int64_t ndof = (int64_t)nx * ny * nz * N3;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ndof) return;
  const int64_t c = g / N3;
  const int j = (int)(g - c * N3);
  const int kx = j % N, ky = (j / N) % N, kz = j / (N * N);
  const int ix = (int)(c % nx), iy = (int)((c / nx) % ny), iz = (int)(c / ((int64_t)nx * ny));
  const int vx = nx + 1, vy = ny + 1;
  const T x1 = tb.xi[kx], y1 = tb.xi[ky], z1 = tb.xi[kz];
  const T lx[2] = {T(1) - x1, x1}, ly[2] = {T(1) - y1, y1}, lz[2] = {T(1) - z1, z1};
  const int64_t v0 = ix + (int64_t)vx * (iy + (int64_t)vy * iz);
  T s = T(0);
#pragma unroll
  for (int dz = 0; dz < 2; ++dz)
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
      for (int dx = 0; dx < 2; ++dx)
        s += lx[dx] * ly[dy] * lz[dz] * xv[v0 + dx + (int64_t)vx * (dy + (int64_t)vy * dz)];
  u[g] += s;
}

// out = r - A x for the 7-point (P0) levels
template <typename T>
__global__ void k_residual7(const T *__restrict__ A, int nx, int ny, int nz, const T *__restrict__ r,
                            const T *__restrict__ x, T *__restrict__ out) {
  const int64_t n = (int64_t)nx * ny * nz;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int ix = (int)(i % nx), iy = (int)((i / nx) % ny), iz = (int)(i / ((int64_t)nx * ny));
  T s = A[i] * x[i];
  if (ix > 0) s += A[n + i] * x[i - 1];
  if (ix < nx - 1) s += A[2 * n + i] * x[i + 1];
  if (iy > 0) s += A[3 * n + i] * x[i - nx];
  if (iy < ny - 1) s += A[4 * n + i] * x[i + nx];
  if (iz > 0) s += A[5 * n + i] * x[i - (int64_t)nx * ny];
  if (iz < nz - 1) s += A[6 * n + i] * x[i + (int64_t)nx * ny];
  out[i] = r[i] - s;
}

template <typename T>
__global__ void k_add(int64_t n, const T *__restrict__ x, T *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += x[i];
}

template <typename T>
__global__ void k_copy(int64_t n, const T *__restrict__ x, T *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i];
}

}  // namespace

template <typename T>
int jacobi27(const T *A, const T *dinv, int vx, int vy, int vz, T w, const T *r, const T *xi, T *xo, hipStream_t s) {
  hipLaunchKernelGGL((k_jacobi27<T>), grid_for((int64_t)vx * vy * vz), dim3(256), 0, s, A, dinv, vx, vy, vz, w, r, xi,
                     xo);
  DG_HIP(hipGetLastError());
  return DG_OK;
}
template <typename T>
int residual27(const T *A, int vx, int vy, int vz, const T *r, const T *x, T *out, hipStream_t s) {
  hipLaunchKernelGGL((k_residual27<T>), grid_for((int64_t)vx * vy * vz), dim3(256), 0, s, A, vx, vy, vz, r, x, out);
  DG_HIP(hipGetLastError());
  return DG_OK;
}
template <typename T>
int restrict27(int vx, int vy, int vz, const T *t, int cx, int cy, int cz, T *rc, const T *dinv, T w, T *xz,
               hipStream_t s) {
  hipLaunchKernelGGL((k_restrict27<T>), grid_for((int64_t)cx * cy * cz), dim3(256), 0, s, vx, vy, vz, t, cx, cy, cz,
                     rc, dinv, w, xz);
  DG_HIP(hipGetLastError());
  return DG_OK;
}
template <typename T>
int prolong27(int vx, int vy, int vz, int cx, int cy, int cz, const T *xc, T *x, hipStream_t s) {
  hipLaunchKernelGGL((k_prolong27<T>), grid_for((int64_t)vx * vy * vz), dim3(256), 0, s, vx, vy, vz, cx, cy, cz, xc,
                     x);
  DG_HIP(hipGetLastError());
  return DG_OK;
}
template <typename T>
int q1_gather(int nx, int ny, int nz, const T *cs, T *rv, const T *dinv, T w, T *xz, hipStream_t s) {
  hipLaunchKernelGGL((k_q1_gather<T>), grid_for((int64_t)(nx + 1) * (ny + 1) * (nz + 1)), dim3(256), 0, s, nx, ny,
                     nz, cs, rv, dinv, w, xz);
  DG_HIP(hipGetLastError());
  return DG_OK;
}
template <typename T>
int q1_prolong_add(int p, int nx, int ny, int nz, const T *xv, T *u, hipStream_t s) {
  const int n = p + 1;
  const dim3 g = grid_for((int64_t)nx * ny * nz * n * n * n);
  switch (p) {
    case 1: hipLaunchKernelGGL((k_q1_prolong_add<2, T>), g, dim3(256), 0, s, nx, ny, nz, xv, u); break;
    case 2: hipLaunchKernelGGL((k_q1_prolong_add<3, T>), g, dim3(256), 0, s, nx, ny, nz, xv, u); break;
    case 3: hipLaunchKernelGGL((k_q1_prolong_add<4, T>), g, dim3(256), 0, s, nx, ny, nz, xv, u); break;
    case 4: hipLaunchKernelGGL((k_q1_prolong_add<5, T>), g, dim3(256), 0, s, nx, ny, nz, xv, u); break;
    default: set_error("q1_prolong_add: unsupported degree"); return DG_EINVAL;
  }
  DG_HIP(hipGetLastError());
  return DG_OK;
}
template <typename T>
int residual7(const T *A, int nx, int ny, int nz, const T *r, const T *x, T *out, hipStream_t s) {
  hipLaunchKernelGGL((k_residual7<T>), grid_for((int64_t)nx * ny * nz), dim3(256), 0, s, A, nx, ny, nz, r, x, out);
  DG_HIP(hipGetLastError());
  return DG_OK;
}
template <typename T>
int add_to(int64_t n, const T *x, T *y, hipStream_t s) {
  hipLaunchKernelGGL((k_add<T>), grid_for(n), dim3(256), 0, s, n, x, y);
  DG_HIP(hipGetLastError());
  return DG_OK;
}
template <typename T>
int copy_vec(int64_t n, const T *x, T *y, hipStream_t s) {
  hipLaunchKernelGGL((k_copy<T>), grid_for(n), dim3(256), 0, s, n, x, y);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

#define DG_INST(T)                                                                                        \
  template int jacobi27<T>(const T *, const T *, int, int, int, T, const T *, const T *, T *, hipStream_t); \
  template int residual27<T>(const T *, int, int, int, const T *, const T *, T *, hipStream_t);           \
  template int restrict27<T>(int, int, int, const T *, int, int, int, T *, const T *, T, T *, hipStream_t); \
  template int prolong27<T>(int, int, int, int, int, int, const T *, T *, hipStream_t);                   \
  template int q1_gather<T>(int, int, int, const T *, T *, const T *, T, T *, hipStream_t);                \
  template int q1_prolong_add<T>(int, int, int, int, const T *, T *, hipStream_t);                        \
  template int residual7<T>(const T *, int, int, int, const T *, const T *, T *, hipStream_t);            \
  template int add_to<T>(int64_t, const T *, T *, hipStream_t);                                           \
  template int copy_vec<T>(int64_t, const T *, T *, hipStream_t);
DG_INST(double)
DG_INST(float)
#undef DG_INST

}  // namespace dgmg
