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
#include "q1_element.h"
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

// (ix, iy, iz) of index i on an nx-by-ny-by-* grid, x fastest; 32-bit
// divisions below 2^31 (every realistic level), 64-bit above.
__device__ inline void grid_coords(int64_t i, int nx, int ny, int &ix, int &iy, int &iz) {
  if (i < 0x7fffffff) {
    const unsigned u = (unsigned)i, a = (unsigned)nx, b = (unsigned)ny;
    const unsigned q = u / a;
    ix = (int)(u - q * a);
    iy = (int)(q % b);
    iz = (int)(q / b);
  } else {
    ix = (int)(i % nx);
    iy = (int)((i / nx) % ny);
    iz = (int)(i / ((int64_t)nx * ny));
  }
}

// (A x)_i for the 27-point stencil.  Couplings to unknowns outside the grid
// are exact zeros in every level's stencil (the level-0 matrix only couples
// vertices of a common cell, and Galerkin products keep that), so the
// neighbour index is clamped into the grid instead of branching: all 54
// loads are independent and issue at once.
// The index type I is int in the single-workgroup cycle (x in LDS, every
// index of the level below 2^31), int64_t in the one-kernel-per-step form.
template <typename T, typename I>
__device__ inline T stencil27(const T *__restrict__ A, int64_t n, const T *__restrict__ x, I i, int ix, int iy,
                              int iz, int vx, int vy, int vz) {
  const int ox[3] = {ix > 0 ? -1 : 0, 0, ix < vx - 1 ? 1 : 0};
  const int64_t oy[3] = {iy > 0 ? -(int64_t)vx : 0, 0, iy < vy - 1 ? (int64_t)vx : 0};
  const int64_t oz[3] = {iz > 0 ? -(int64_t)vx * vy : 0, 0, iz < vz - 1 ? (int64_t)vx * vy : 0};
  T s = T(0);
  if constexpr (sizeof(I) == 4) {
    // x in LDS: the 27 coefficients are all requested before the first
    // product (in the large single-workgroup kernel the scheduler would
    // otherwise issue them one at a time to save registers); the products
    // are summed in the same order as below
    T a[27];
#pragma unroll
    for (int o = 0; o < 27; ++o) {
      const T *Ao = A + o * n;
      a[o] = Ao[i];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int dz = 0; dz < 3; ++dz)
#pragma unroll
      for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) s += a[dx + 3 * dy + 9 * dz] * x[i + ox[dx] + oy[dy] + oz[dz]];
  } else {
#pragma unroll
    for (int dz = 0; dz < 3; ++dz)
#pragma unroll
      for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) {
          const int o = dx + 3 * dy + 9 * dz;
          s += A[o * n + i] * x[i + ox[dx] + oy[dy] + oz[dz]];
        }
  }
  return s;
}

// Per-unknown bodies of the 27-point level operations, shared by the
// one-thread-per-unknown kernels below and the single-workgroup cycle of
// the small levels (k_coarse_tail), so that both give the same bits.

// xo_i = xi_i + w Dinv_i (r_i - (A xi)_i); xi == null means xi = 0.  Dinv is
// the inverse of half the l1 row norm (see CoarseLevel).
template <typename T, typename I>
__device__ inline void jacobi27_at(const T *__restrict__ A, const T *__restrict__ dinv, int vx, int vy, int vz, T w,
                                   const T *__restrict__ r, const T *xi, T *xo, I i) {
  const int64_t n = (int64_t)vx * vy * vz;
  const T wd = w * dinv[i];
  if (!xi) {
    xo[i] = wd * r[i];
    return;
  }
  int ix, iy, iz;
  grid_coords(i, vx, vy, ix, iy, iz);
  xo[i] = xi[i] + wd * (r[i] - stencil27(A, n, xi, i, ix, iy, iz, vx, vy, vz));
}

// out_i = r_i - (A x)_i
template <typename T, typename I>
__device__ inline void residual27_at(const T *__restrict__ A, int vx, int vy, int vz, const T *__restrict__ r,
                                     const T *x, T *out, I i) {
  const int64_t n = (int64_t)vx * vy * vz;
  int ix, iy, iz;
  grid_coords(i, vx, vy, ix, iy, iz);
  out[i] = r[i] - stencil27(A, n, x, i, ix, iy, iz, vx, vy, vz);
}

// rc_J = (P^T t)_J: coarse J gathers the fine vertices within one fine step
// of its own fine position, with their interpolation weights towards J.
// When xz is not null, also xz_J = w dinv_J rc_J: the first damped Jacobi
// sweep from zero on the coarse level.  Branch-free: per axis the three
// candidates f - 1, f, f + 1 (clamped into the grid, weight 0 where the
// vertex is outside or does not interpolate from J), all 27 loads issued
// at once; the nonzero terms are added in the same order as a loop over
// the contributing vertices only, and a zero-weight term leaves the sum
// unchanged.
template <typename T>
__device__ inline void restrict27_at(int vx, int vy, int vz, const T *t, int cx, int cy, int cz, T *rc,
                                     const T *__restrict__ dinv, T w, T *xz, int64_t J) {
  int jj[3];
  grid_coords(J, cx, cy, jj[0], jj[1], jj[2]);
  const int vf[3] = {vx, vy, vz}, vcs[3] = {cx, cy, cz};
  int fi[3][3];
  T fw[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int f = min(2 * jj[k], vf[k] - 1);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int i = f + d - 1;
      const bool in = i >= 0 && i < vf[k];
      const int ic = in ? i : f;
      const W1 w1 = interp1(ic, vf[k], vcs[k]);
      T wt = T(0);
      if (w1.j0 == jj[k]) wt = w1.two ? T(0.5) : T(1);
      else if (w1.two && w1.j0 + 1 == jj[k]) wt = T(0.5);
      fi[k][d] = ic;
      fw[k][d] = in ? wt : T(0);
    }
  }
  T tv[27];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int a = 0; a < 3; ++a) tv[a + 3 * b + 9 * c] = t[fi[0][a] + (int64_t)vx * (fi[1][b] + (int64_t)vy * fi[2][c])];
  T s = T(0);
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int a = 0; a < 3; ++a) s += fw[0][a] * fw[1][b] * fw[2][c] * tv[a + 3 * b + 9 * c];
  rc[J] = s;
  if (xz) xz[J] = w * dinv[J] * s;
}

// x_i += (P xc)_i (trilinear interpolation from the coarser vertex level).
// Branch-free: per axis the coarse vertices j0 and j0 + 1 (clamped into the
// grid, weight 0 when the fine vertex sits on j0), all eight loads issued
// at once, the terms added in the same order as a loop over the
// contributing vertices only (a zero-weight term leaves the sum unchanged).
template <typename T>
__device__ inline void prolong27_at(int vx, int vy, int vz, int cx, int cy, int cz, const T *xc, T *x, int64_t i) {
  int ii[3];
  grid_coords(i, vx, vy, ii[0], ii[1], ii[2]);
  const int vf[3] = {vx, vy, vz}, vcs[3] = {cx, cy, cz};
  int j[3][2];
  T w[3][2];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const W1 q = interp1(ii[k], vf[k], vcs[k]);
    j[k][0] = q.j0;
    j[k][1] = min(q.j0 + 1, vcs[k] - 1);
    w[k][0] = q.two ? T(0.5) : T(1);
    w[k][1] = q.two ? T(0.5) : T(0);
  }
  T v[8];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) v[a + 2 * b + 4 * c] = xc[j[0][a] + (int64_t)cx * (j[1][b] + (int64_t)cy * j[2][c])];
  T s = T(0);
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) s += w[0][a] * w[1][b] * w[2][c] * v[a + 2 * b + 4 * c];
  x[i] += s;
}

template <typename T>
__global__ void k_jacobi27(const T *__restrict__ A, const T *__restrict__ dinv, int vx, int vy, int vz, T w,
                           const T *__restrict__ r, const T *__restrict__ xi, T *__restrict__ xo) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (int64_t)vx * vy * vz) jacobi27_at<T>(A, dinv, vx, vy, vz, w, r, xi, xo, i);
}

template <typename T>
__global__ void k_residual27(const T *__restrict__ A, int vx, int vy, int vz, const T *__restrict__ r,
                             const T *__restrict__ x, T *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (int64_t)vx * vy * vz) residual27_at<T>(A, vx, vy, vz, r, x, out, i);
}

template <typename T>
__global__ void k_restrict27(int vx, int vy, int vz, const T *__restrict__ t, int cx, int cy, int cz,
                             T *__restrict__ rc, const T *__restrict__ dinv, T w, T *__restrict__ xz) {
  const int64_t J = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (J < (int64_t)cx * cy * cz) restrict27_at<T>(vx, vy, vz, t, cx, cy, cz, rc, dinv, w, xz, J);
}

template <typename T>
__global__ void k_prolong27(int vx, int vy, int vz, int cx, int cy, int cz, const T *__restrict__ xc,
                            T *__restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (int64_t)vx * vy * vz) prolong27_at<T>(vx, vy, vz, cx, cy, cz, xc, x, i);
}

// One V-cycle of the small 27-point levels l_0 .. (from a zero guess, the
// same steps and per-unknown arithmetic as the kernel-per-step cycle in
// api.cpp: nu damped Jacobi sweeps before and after, residual, restriction
// with the coarser level's first sweep fused, the dense inverse at the
// bottom, prolongation) in one workgroup, with a barrier between steps:
// at these sizes the kernel-per-step cycle is bound by launch latency.
// The levels' vectors r, x, t live in LDS (level k at offset off[k] of each
// of the three arrays); memory holds only the coefficients, r of level l_0
// (read) and the result (written to level l_0's x buffer).
template <typename T>
__global__ __launch_bounds__(kTailThreads) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_coarse_tail(TailArgs<T> a) {
  __shared__ T sr[kTailLds], sx[kTailLds], st[kTailLds];
  const int tid = threadIdx.x;
  const int *off = a.off;
  {
    // one word of every 128-byte line of the levels' coefficients (A and
    // dinv above the bottom, the dense inverse at it), all in flight
    // together: the steps below then find them in this XCD's L2 instead of
    // waiting for memory one step at a time.  Thread tid takes lines tid +
    // kTailThreads j, j < kTailPrefetch, of the regions laid end to end.
    constexpr int kLine = 128 / (int)sizeof(T);
    const T *pf[kTailPrefetch];
#pragma unroll
    for (int j = 0; j < kTailPrefetch; ++j) pf[j] = a.inv;
    int start = 0;
    for (int q = 0; q < 2 * a.nl - 1; ++q) {
      const int k = q >> 1;
      const int n = off[k + 1] - off[k];
      const T *base = k + 1 == a.nl ? a.inv : (q & 1) ? a.lv[k].dinv : a.lv[k].A;
      const int cnt = k + 1 == a.nl ? a.bn * a.bn : (q & 1) ? n : 27 * n;
      const int lines = (cnt + kLine - 1) / kLine;
#pragma unroll
      for (int j = 0; j < kTailPrefetch; ++j) {
        const int g = tid + kTailThreads * j - start;
        if (g >= 0 && g < lines) pf[j] = base + (size_t)g * kLine;
      }
      start += lines;
    }
    T v[kTailPrefetch];
#pragma unroll
    for (int j = 0; j < kTailPrefetch; ++j) v[j] = *pf[j];
    const TailLevel<T> &L0 = a.lv[0];
    const int n = off[1];
    if (tid < n) {
      sr[tid] = L0.r[tid];
      if (a.x_init) sx[tid] = L0.x[tid];
    }
#pragma unroll
    for (int j = 0; j < kTailPrefetch; ++j) asm volatile("" ::"v"(v[j]));
    __syncthreads();
  }
  // bit l set: level l's current iterate is in t, else in x
  unsigned in_t = 0;
  bool fused = a.x_init != 0;  // the level's x holds its first sweep
  for (int l = 0; l + 1 < a.nl; ++l) {
    const TailLevel<T> &L = a.lv[l];
    const int n = off[l + 1] - off[l];
    const T *r = sr + off[l];
    T *x = sx + off[l], *t = st + off[l];
    if (!fused) {
      if (tid < n)
        jacobi27_at<T>(L.A, L.dinv, L.vx, L.vy, L.vz, a.w, r, nullptr, x, tid);
      __syncthreads();
    }
    for (int k = 1; k < a.nu; ++k) {
      if (tid < n) jacobi27_at<T>(L.A, L.dinv, L.vx, L.vy, L.vz, a.w, r, x, t, tid);
      __syncthreads();
      T *sw = x;
      x = t;
      t = sw;
    }
    if (tid < n) residual27_at<T>(L.A, L.vx, L.vy, L.vz, r, x, t, tid);
    __syncthreads();
    const TailLevel<T> &C = a.lv[l + 1];
    fused = l + 2 < a.nl;  // the coarser level smooths (it is not the bottom)
    const int nc = off[l + 2] - off[l + 1];
    if (tid < nc)
      restrict27_at<T>(L.vx, L.vy, L.vz, t, C.vx, C.vy, C.vz, sr + off[l + 1], C.dinv, a.w,
                       fused ? sx + off[l + 1] : nullptr, tid);
    __syncthreads();
    if (x != sx + off[l]) in_t |= 1u << l;
  }
  {
    // bottom: x = inv r.  Row wv + 16 k on wavefront wv: the lane-strided
    // sums and shuffle reduction of k_dense_mv, row by row in the same
    // order, with the rows of one wavefront interleaved so that their loads
    // are in flight together.
    constexpr int W = kTailThreads / 64, R = kTailBottomMax / W;
    const T *br = sr + off[a.nl - 1];
    T *bx = sx + off[a.nl - 1];
    const int lane = tid & 63, wv = tid >> 6;
    T s[R];
#pragma unroll
    for (int k = 0; k < R; ++k) s[k] = T(0);
    for (int j = lane; j < a.bn; j += 64) {
      const T rj = br[j];
      T m[R];
#pragma unroll
      for (int k = 0; k < R; ++k) {
        const int row = min(wv + W * k, a.bn - 1);
        m[k] = a.inv[row * a.bn + j];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int k = 0; k < R; ++k)
        if (wv + W * k < a.bn) s[k] += m[k] * rj;
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
#pragma unroll
      for (int m = 32; m >= 1; m >>= 1) s[k] += __shfl_xor(s[k], m, 64);
      const int row = wv + W * k;
      if (lane == 0 && row < a.bn) bx[row] = s[k];
    }
    __syncthreads();
  }
  for (int l = a.nl - 2; l >= 0; --l) {
    const TailLevel<T> &L = a.lv[l];
    const TailLevel<T> &C = a.lv[l + 1];
    const int n = off[l + 1] - off[l];
    const bool lt = (in_t >> l) & 1u;
    const T *r = sr + off[l];
    T *x = (lt ? st : sx) + off[l], *t = (lt ? sx : st) + off[l];
    const T *xc = ((in_t >> (l + 1)) & 1u ? st : sx) + off[l + 1];
    if (tid < n) prolong27_at<T>(L.vx, L.vy, L.vz, C.vx, C.vy, C.vz, xc, x, tid);
    __syncthreads();
    for (int k = 0; k < a.nu; ++k) {
      if (tid < n) jacobi27_at<T>(L.A, L.dinv, L.vx, L.vy, L.vz, a.w, r, x, t, tid);
      __syncthreads();
      T *sw = x;
      x = t;
      t = sw;
    }
    in_t = (in_t & ~(1u << l)) | ((x != sx + off[l] ? 1u : 0u) << l);
  }
  const T *res = ((in_t & 1u) ? st : sx);
  if (tid < off[1]) a.lv[0].x[tid] = res[tid];
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
  int ix, iy, iz;
  grid_coords(v, vx, vy, ix, iy, iz);
  // the (up to) eight cells around v, loaded at once (a cell outside the
  // grid is replaced by a clamped one and its value by 0, which leaves the
  // sum unchanged); the vertex is corner (1-sx, 1-sy, 1-sz) of cell s
  T val[8];
  bool in[8];
#pragma unroll
  for (int sz = 0; sz < 2; ++sz)
#pragma unroll
    for (int sy = 0; sy < 2; ++sy)
#pragma unroll
      for (int sx = 0; sx < 2; ++sx) {
        const int cz = iz - 1 + sz, cyy = iy - 1 + sy, cxx = ix - 1 + sx;
        const int q = sx + 2 * sy + 4 * sz;
        in[q] = cz >= 0 && cz < nz && cyy >= 0 && cyy < ny && cxx >= 0 && cxx < nx;
        const int64_t c = min(max(cxx, 0), nx - 1) + (int64_t)nx * (min(max(cyy, 0), ny - 1) +
                                                                    (int64_t)ny * min(max(cz, 0), nz - 1));
        val[q] = cs[8 * c + (1 - sx) + 2 * (1 - sy) + 4 * (1 - sz)];
      }
  T s = T(0);
#pragma unroll
  for (int q = 0; q < 8; ++q) s += in[q] ? val[q] : T(0);
  rv[v] = s;
  if (xz) xz[v] = w * dinv[v] * s;
}

// u += P x_hat: every DG node receives the trilinear interpolant of the
// vertex values of its cell, evaluated at the node (Sec. 2.2.2).  One
// thread per x-line of a cell: the eight vertex values are read once for
// the line's N nodes.
template <int N, typename T>
__global__ void k_q1_prolong_add(int nx, int ny, int nz, const T *__restrict__ xv, T *__restrict__ u) {
  constexpr int N2 = N * N, N3 = N * N * N;
  constexpr DevTab<T, N> tb = make_ctab<T, N>();
  const int64_t nlines = (int64_t)nx * ny * nz * N2;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nlines) return;
  const int64_t c = g / N2;
  const int j = (int)(g - c * N2);
  const int ky = j % N, kz = j / N;
  int ix, iy, iz;
  grid_coords(c, nx, ny, ix, iy, iz);
  const int vx = nx + 1, vy = ny + 1;
  const T y1 = tb.xi[ky], z1 = tb.xi[kz];
  const T ly[2] = {T(1) - y1, y1}, lz[2] = {T(1) - z1, z1};
  const int64_t v0 = ix + (int64_t)vx * (iy + (int64_t)vy * iz);
  T xc[2][2][2];
#pragma unroll
  for (int dz = 0; dz < 2; ++dz)
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
      for (int dx = 0; dx < 2; ++dx) xc[dz][dy][dx] = xv[v0 + dx + (int64_t)vx * (dy + (int64_t)vy * dz)];
  T *ul = u + c * N3 + (int64_t)N * ky + (int64_t)N2 * kz;
#pragma unroll
  for (int kx = 0; kx < N; ++kx) {
    const T x1 = tb.xi[kx];
    const T lx[2] = {T(1) - x1, x1};
    T s = T(0);
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
      for (int dy = 0; dy < 2; ++dy)
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) s += lx[dx] * ly[dy] * lz[dz] * xc[dz][dy][dx];
    ul[kx] += s;
  }
}

// out = r - A x for the 7-point (P0) levels
template <typename T>
__global__ void k_residual7(const T *__restrict__ A, int nx, int ny, int nz, const T *__restrict__ r,
                            const T *__restrict__ x, T *__restrict__ out) {
  const int64_t n = (int64_t)nx * ny * nz;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int ix, iy, iz;
  grid_coords(i, nx, ny, ix, iy, iz);
  // all 14 loads issued before the first product (a neighbour outside the
  // grid reads the point itself and its term is not added)
  const bool in[6] = {ix > 0, ix < nx - 1, iy > 0, iy < ny - 1, iz > 0, iz < nz - 1};
  const int64_t off[6] = {-1, 1, -(int64_t)nx, (int64_t)nx, -(int64_t)nx * ny, (int64_t)nx * ny};
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

// ---- setup of the Q1 hierarchy on the device ----------------------------
// Level 0: vertex v gathers, from each of its (up to eight) cells, the row
// of that cell's trilinear element matrix for the corner at v.
template <int P>
__global__ __launch_bounds__(128) void k_q1_assemble(Geo g, double *__restrict__ A) {
  constexpr int N = P + 1;
  constexpr DevTab<double, N> tb = make_ctab<double, N>();
  const int vx = g.nx + 1, vy = g.ny + 1;
  const int64_t n = (int64_t)vx * vy * (g.nz + 1);
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  int ix, iy, iz;
  grid_coords(v, vx, vy, ix, iy, iz);
  double acc[27];
  for (int o = 0; o < 27; ++o) acc[o] = 0.0;
  for (int sz = 0; sz < 2; ++sz) {
    const int cz = iz - 1 + sz;
    if (cz < 0 || cz >= g.nz) continue;
    for (int sy = 0; sy < 2; ++sy) {
      const int cy = iy - 1 + sy;
      if (cy < 0 || cy >= g.ny) continue;
      for (int sx = 0; sx < 2; ++sx) {
        const int cx = ix - 1 + sx;
        if (cx < 0 || cx >= g.nx) continue;
        const int c = cx + g.nx * (cy + g.ny * cz);
        const int ijk[3] = {cx, cy, cz};
        const int da[3] = {1 - sx, 1 - sy, 1 - sz};  // corner of the cell at v
        double row[8];
        q1_element_row<N>(g, tb, c, ijk, da[0] + 2 * da[1] + 4 * da[2], row);
        for (int b = 0; b < 8; ++b) {
          const int o = ((b & 1) - da[0] + 1) + 3 * (((b >> 1) & 1) - da[1] + 1) + 9 * ((b >> 2) - da[2] + 1);
          acc[o] += row[b];
        }
      }
    }
  }
  for (int o = 0; o < 27; ++o) A[o * n + v] = acc[o];
}

// Ac = P^T A P: coarse vertex I gathers the fine vertices i with P_iI != 0,
// their 27 couplings A_ij, and the interpolation weights of j towards the
// coarse vertices J around I.
__global__ __launch_bounds__(128) void k_galerkin27(const double *__restrict__ A, int vx, int vy, int vz,
                                                    double *__restrict__ Ac, int cx, int cy, int cz) {
  const int64_t n = (int64_t)vx * vy * vz, nc = (int64_t)cx * cy * cz;
  const int64_t I = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= nc) return;
  int II[3];
  grid_coords(I, cx, cy, II[0], II[1], II[2]);
  const int vf[3] = {vx, vy, vz}, vc[3] = {cx, cy, cz};
  double acc[27];
  for (int o = 0; o < 27; ++o) acc[o] = 0.0;
  for (int dz = -1; dz <= 1; ++dz) {
    const int iz = min(2 * II[2], vz - 1) + dz;
    if (iz < 0 || iz >= vz) continue;
    for (int dy = -1; dy <= 1; ++dy) {
      const int iy = min(2 * II[1], vy - 1) + dy;
      if (iy < 0 || iy >= vy) continue;
      for (int dx = -1; dx <= 1; ++dx) {
        const int ix = min(2 * II[0], vx - 1) + dx;
        if (ix < 0 || ix >= vx) continue;
        const int ii[3] = {ix, iy, iz};
        // weight of fine i towards coarse I
        double wi = 1.0;
        for (int k = 0; k < 3; ++k) {
          const W1 q = interp1(ii[k], vf[k], vc[k]);
          double wk = 0.0;
          if (q.j0 == II[k]) wk = q.two ? 0.5 : 1.0;
          else if (q.two && q.j0 + 1 == II[k]) wk = 0.5;
          wi *= wk;
        }
        if (wi == 0.0) continue;
        const int64_t i = ix + (int64_t)vx * (iy + (int64_t)vy * iz);
        for (int o = 0; o < 27; ++o) {
          const int jj[3] = {ix + o % 3 - 1, iy + (o / 3) % 3 - 1, iz + o / 9 - 1};
          if (jj[0] < 0 || jj[1] < 0 || jj[2] < 0 || jj[0] >= vx || jj[1] >= vy || jj[2] >= vz) continue;
          const double a = A[o * n + i];
          if (a == 0.0) continue;
          W1 q[3];
          for (int k = 0; k < 3; ++k) q[k] = interp1(jj[k], vf[k], vc[k]);
          for (int t2 = 0; t2 < (q[2].two ? 2 : 1); ++t2)
            for (int t1 = 0; t1 < (q[1].two ? 2 : 1); ++t1)
              for (int t0 = 0; t0 < (q[0].two ? 2 : 1); ++t0) {
                const int J[3] = {q[0].j0 + t0, q[1].j0 + t1, q[2].j0 + t2};
                const double wj = (q[0].two ? 0.5 : 1.0) * (q[1].two ? 0.5 : 1.0) * (q[2].two ? 0.5 : 1.0);
                const int oc = (J[0] - II[0] + 1) + 3 * (J[1] - II[1] + 1) + 9 * (J[2] - II[2] + 1);
                if (oc >= 0 && oc < 27) acc[oc] += wi * a * wj;  // always true: |J - I| <= 1 per axis
              }
        }
      }
    }
  }
  for (int o = 0; o < 27; ++o) Ac[o * nc + I] = acc[o];
}

// FP32 copy of a level's stencil and the l1 smoothing diagonal 2 / sum |A|.
__global__ __launch_bounds__(256) void k_level_finish(const double *__restrict__ A, int64_t n, float *__restrict__ A32,
                                                      double *__restrict__ d64, float *__restrict__ d32) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int o = 0; o < 27; ++o) {
    const double a = A[o * n + i];
    A32[o * n + i] = (float)a;
    s += fabs(a);
  }
  const double d = s > 0.0 ? 2.0 / s : 0.0;
  d64[i] = d;
  d32[i] = (float)d;
}

}  // namespace

int q1_assemble(const dg_problem *pr, double *A, hipStream_t s) {
  const int64_t n = (int64_t)(pr->geo.nx + 1) * (pr->geo.ny + 1) * (pr->geo.nz + 1);
  const dim3 g((unsigned)((n + 127) / 128)), b(128);
  switch (pr->p) {
    case 1: hipLaunchKernelGGL((k_q1_assemble<1>), g, b, 0, s, pr->geo, A); break;
    case 2: hipLaunchKernelGGL((k_q1_assemble<2>), g, b, 0, s, pr->geo, A); break;
    case 3: hipLaunchKernelGGL((k_q1_assemble<3>), g, b, 0, s, pr->geo, A); break;
    case 4: hipLaunchKernelGGL((k_q1_assemble<4>), g, b, 0, s, pr->geo, A); break;
    case 5: hipLaunchKernelGGL((k_q1_assemble<5>), g, b, 0, s, pr->geo, A); break;
    default: set_error("unsupported degree"); return DG_EINVAL;
  }
  DG_HIP(hipGetLastError());
  return DG_OK;
}
int galerkin27(const double *A, int vx, int vy, int vz, double *Ac, int cx, int cy, int cz, hipStream_t s) {
  const int64_t nc = (int64_t)cx * cy * cz;
  hipLaunchKernelGGL(k_galerkin27, dim3((unsigned)((nc + 127) / 128)), dim3(128), 0, s, A, vx, vy, vz, Ac, cx, cy,
                     cz);
  DG_HIP(hipGetLastError());
  return DG_OK;
}
int level_finish(const double *A, int64_t n, float *A32, double *d64, float *d32, hipStream_t s) {
  hipLaunchKernelGGL(k_level_finish, grid_for(n), dim3(256), 0, s, A, n, A32, d64, d32);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

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
int coarse_tail(const TailArgs<T> &args, hipStream_t s) {
  TailArgs<T> a = args;
  int64_t total = 0;
  a.off[0] = 0;
  for (int k = 0; k < a.nl && k < kTailLevels; ++k) {
    total += (int64_t)a.lv[k].vx * a.lv[k].vy * a.lv[k].vz;
    a.off[k + 1] = (int)std::min<int64_t>(total, kTailLds);
  }
  if (a.nl < 2 || a.nl > kTailLevels || a.bn < 1 || a.bn > kTailBottomMax ||
      (int64_t)a.lv[0].vx * a.lv[0].vy * a.lv[0].vz > kTailMaxUnknowns || total > kTailLds ||
      (int64_t)a.lv[a.nl - 1].vx * a.lv[a.nl - 1].vy * a.lv[a.nl - 1].vz != a.bn) {
    set_error("internal: coarse tail sizes");
    return DG_EINVAL;
  }
  hipLaunchKernelGGL((k_coarse_tail<T>), dim3(1), dim3(kTailThreads), 0, s, a);
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
  const dim3 g = grid_for((int64_t)nx * ny * nz * n * n);
  switch (p) {
    case 1: hipLaunchKernelGGL((k_q1_prolong_add<2, T>), g, dim3(256), 0, s, nx, ny, nz, xv, u); break;
    case 2: hipLaunchKernelGGL((k_q1_prolong_add<3, T>), g, dim3(256), 0, s, nx, ny, nz, xv, u); break;
    case 3: hipLaunchKernelGGL((k_q1_prolong_add<4, T>), g, dim3(256), 0, s, nx, ny, nz, xv, u); break;
    case 4: hipLaunchKernelGGL((k_q1_prolong_add<5, T>), g, dim3(256), 0, s, nx, ny, nz, xv, u); break;
    case 5: hipLaunchKernelGGL((k_q1_prolong_add<6, T>), g, dim3(256), 0, s, nx, ny, nz, xv, u); break;
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
  template int coarse_tail<T>(const TailArgs<T> &, hipStream_t);                                         \
  template int q1_gather<T>(int, int, int, const T *, T *, const T *, T, T *, hipStream_t);                \
  template int q1_prolong_add<T>(int, int, int, int, const T *, T *, hipStream_t);                        \
  template int residual7<T>(const T *, int, int, int, const T *, const T *, T *, hipStream_t);            \
  template int add_to<T>(int64_t, const T *, T *, hipStream_t);                                           \
  template int copy_vec<T>(int64_t, const T *, T *, hipStream_t);
DG_INST(double)
DG_INST(float)
#undef DG_INST

}  // namespace dgmg
