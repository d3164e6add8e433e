// Matrix-free DG operator apply v = A u (Sec. 3.1) and its block diagonal
// D_T (eqn block_diag_apply), on gfx950.
//
// Mapping.  A workgroup of 256 lanes takes CPB = floor(256 / (p+1)^2)
// consecutive cells (p=1: 64, p=2: 28, p=3: 16, p=4: 10).  The cells of a
// workgroup are one contiguous range of the cell-major DOF vector, so the
// staging load into LDS and the final store are fully coalesced.  Lane
// (cell, a, b) owns the line index (a, b) of its cell and processes, one
// after the other, the x-line (y=a, z=b), the y-line (x=a, z=b) and the
// z-line (x=a, y=b) through it: each line is a (p+1)-vector read from LDS,
// the 1-D operator is applied in registers, and the contributions of the
// three directions are summed in an LDS accumulator.  The workgroup also
// stages one cell on either side of its range, so every x-neighbour line is
// in LDS; the y- and z-neighbour lines are read from global memory (L2 /
// MALL hits): the y lines at the start, together with the staging loads,
// and reduced to their face traces at once; the z lines after the x lines,
// so that their latency hides behind the y-line work.  For b = 0 the line
// operator runs in its even-odd form (line_apply_eo).
//
// XCD-aware order: consecutive workgroup ids are spread round-robin over
// the eight XCDs, so the logical block index is remapped to give every XCD
// one contiguous slab of cells; the y and z neighbours a slab reads are then
// mostly in that XCD's own L2.
#include <type_traits>

#include <hip/hip_ext.h>

#include "line_ops.h"

namespace dgmg {

constexpr int kApplyThreads = 256;

template <int N>
struct ApplyShape {
  static constexpr int N2 = N * N;
  static constexpr int N3 = N * N * N;
  static constexpr int CPB = kApplyThreads / N2;
};

__device__ inline int xcd_block(int b, int G) {
  const int q = G >> 3, r = G & 7;
  const int x = b & 7, k = b >> 3;
  return x * q + (x < r ? x : r) + k;
}

// position in the cell of node i on the line (a, b) along axis k
template <int N>
__device__ __host__ inline int line_pos(int k, int i, int a, int b) {
  return k == 0 ? i + N * a + N * N * b : (k == 1 ? a + N * i + N * N * b : a + N * b + N * N * i);
}

// Shared prologue of both apply kernels: every global load of a workgroup
// is issued before the first one is waited for (the 16-byte loads of its
// cells plus one cell on either side, the y / z neighbour lines of each
// lane, the coefficient data), so that each workgroup pays one memory
// round trip.
template <int N, typename T, bool NB>
struct Stage {
  using S = ApplyShape<N>;
  static constexpr int N2 = S::N2, N3 = S::N3, CPB = S::CPB;
  static constexpr int H = NB ? 1 : 0;  // x-halo cells on each side
  static constexpr int V = 16 / sizeof(T);
  static constexpr int STAGE = (CPB + 2 * H) * N3 + 2 * V;
  static constexpr int NVEC = (STAGE / V + kApplyThreads - 1) / kApplyThreads;
  static constexpr int LDS = NVEC * kApplyThreads * V;
  using VT = typename std::conditional<sizeof(T) == 8, double2, float4>::type;
};

// Load the staged range [c0 - H, c0 + CPB + H) into registers, from an
// element offset rounded down to a 16-byte boundary (elements outside
// [0, ndof) read as zero).  Returns the LDS offset of cell c0 - H.
template <int N, typename T, bool NB>
__device__ inline int stage_load(const Geo &g, const T *__restrict__ u, int c0, int tid,
                                 typename Stage<N, T, NB>::VT (&pre)[Stage<N, T, NB>::NVEC]) {
  using St = Stage<N, T, NB>;
  using VT = typename St::VT;
  constexpr int V = St::V, N3 = St::N3;
  const int64_t ndof = (int64_t)g.ncell * N3;
  const int64_t e_first = (int64_t)(c0 - St::H) * N3;
  const int64_t eb = e_first >= 0 ? (e_first / V) * V : -(((-e_first) + V - 1) / V) * V;
  // every vector load is issued from an in-range, aligned address (all in
  // flight together); the few vectors that reach outside [0, ndof) are
  // then rebuilt element by element
  const int64_t elast = (ndof / V) * V - V;  // last aligned full vector
#pragma unroll
  for (int j = 0; j < St::NVEC; ++j) {
    const int64_t e = eb + (int64_t)(j * kApplyThreads + tid) * V;
    const int64_t ec = e < 0 ? 0 : (e > elast ? elast : e);
    pre[j] = *reinterpret_cast<const VT *>(u + ec);
  }
#pragma unroll
  for (int j = 0; j < St::NVEC; ++j) {
    const int64_t e = eb + (int64_t)(j * kApplyThreads + tid) * V;
    if (e < 0 || e + V > ndof) {
      T t[V];
#pragma unroll
      for (int q = 0; q < V; ++q) t[q] = (e + q >= 0 && e + q < ndof) ? u[e + q] : T(0);
      pre[j] = *reinterpret_cast<const VT *>(t);
    }
  }
  return (int)(e_first - eb);
}

// The y and z neighbour lines of line index (a, b) of cell c (the cell
// itself where there is no neighbour; those traces are discarded).
template <int N, typename T>
__device__ inline void neighbour_lines(const Geo &g, const T *__restrict__ u, int c, const int (&ijk)[3], int a,
                                       int b, T (&yl)[N], T (&yr)[N], T (&zl)[N], T (&zr)[N]) {
  constexpr int N3 = N * N * N;
  const int sy = g.nx, sz = g.nx * g.ny;
  const T *pyl = u + (size_t)(ijk[1] > 0 ? c - sy : c) * N3;
  const T *pyr = u + (size_t)(ijk[1] < g.ny - 1 ? c + sy : c) * N3;
  const T *pzl = u + (size_t)(ijk[2] > 0 ? c - sz : c) * N3;
  const T *pzr = u + (size_t)(ijk[2] < g.nz - 1 ? c + sz : c) * N3;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    yl[i] = pyl[line_pos<N>(1, i, a, b)];
    yr[i] = pyr[line_pos<N>(1, i, a, b)];
    zl[i] = pzl[line_pos<N>(2, i, a, b)];
    zr[i] = pzr[line_pos<N>(2, i, a, b)];
  }
}

template <int N, typename T>
__device__ inline void neighbour_lines_y(const Geo &g, const T *__restrict__ u, int c, const int (&ijk)[3], int a,
                                         int b, T (&yl)[N], T (&yr)[N]) {
  constexpr int N3 = N * N * N;
  const int sy = g.nx;
  const T *pyl = u + (size_t)(ijk[1] > 0 ? c - sy : c) * N3;
  const T *pyr = u + (size_t)(ijk[1] < g.ny - 1 ? c + sy : c) * N3;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    yl[i] = pyl[line_pos<N>(1, i, a, b)];
    yr[i] = pyr[line_pos<N>(1, i, a, b)];
  }
}
template <int N, typename T>
__device__ inline void neighbour_lines_z(const Geo &g, const T *__restrict__ u, int c, const int (&ijk)[3], int a,
                                         int b, T (&zl)[N], T (&zr)[N]) {
  constexpr int N3 = N * N * N;
  const int sz = g.nx * g.ny;
  const T *pzl = u + (size_t)(ijk[2] > 0 ? c - sz : c) * N3;
  const T *pzr = u + (size_t)(ijk[2] < g.nz - 1 ? c + sz : c) * N3;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    zl[i] = pzl[line_pos<N>(2, i, a, b)];
    zr[i] = pzr[line_pos<N>(2, i, a, b)];
  }
}

// Value / derivative traces at the shared faces: (e1 . left, d1 . left,
// e0 . right, d0 . right).
template <int N, typename T>
__device__ inline void face_traces(const DevTab<T, N> &tb, const T (&lo)[N], const T (&hi)[N], T (&t)[4]) {
  t[0] = t[1] = t[2] = t[3] = T(0);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    t[0] += tb.e1[i] * lo[i];
    t[1] += tb.d1[i] * lo[i];
    t[2] += tb.e0[i] * hi[i];
    t[3] += tb.d0[i] * hi[i];
  }
}

// Residual epilogue (RES = 1: P0 sums, RES = 2: Q1 corner sums) of the
// x-line (y = xi_a, z = xi_b) of cell c held by lane (cl, ln): qx = (A u)
// at its N DOFs.  Every lane of the workgroup must call this.
template <int N, typename T, int RES>
__device__ inline void residual_epilogue(const DevTab<T, N> &tb, bool active, int c, int cl, int ln, int a, int b,
                                         const T (&qx)[N], const T *__restrict__ r, T *__restrict__ rh) {
  constexpr int N2 = N * N, N3 = N * N * N, CPB = ApplyShape<N>::CPB;
  if constexpr (RES == 2) {
    // lane (a, b)'s share of corner q is (sum_i L_qx(xi_i) r_i)
    // L_qy(xi_a) L_qz(xi_b) with L_0 = 1 - xi, L_1 = xi; the shares of the
    // cell's lanes are summed in LDS
    __shared__ T part[CPB * 8 * N2];
    if (active) {
      const T *rb = r + (size_t)c * N3 + N * a + N2 * b;
      T s0 = T(0), s1 = T(0);
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const T ri = rb[i] - qx[i];
        s0 += (T(1) - tb.xi[i]) * ri;
        s1 += tb.xi[i] * ri;
      }
      const T ly[2] = {T(1) - tb.xi[a], tb.xi[a]};
      const T lz[2] = {T(1) - tb.xi[b], tb.xi[b]};
#pragma unroll
      for (int q = 0; q < 8; ++q) part[(cl * 8 + q) * N2 + ln] = ((q & 1) ? s1 : s0) * ly[(q >> 1) & 1] * lz[q >> 2];
    }
    __syncthreads();
    // a cell has N2 lanes (4 for p = 1): each reduces corners ln, ln + N2, ...
    if (active) {
      for (int q = ln; q < 8; q += N2) {
        T sum = T(0);
        for (int l = 0; l < N2; ++l) sum += part[(cl * 8 + q) * N2 + l];
        rh[8 * (size_t)c + q] = sum;
      }
    }
  } else {
    __shared__ T part[CPB * N2];
    if (active) {
      const T *rb = r + (size_t)c * N3 + N * a + N2 * b;
      T sum = T(0);
#pragma unroll
      for (int i = 0; i < N; ++i) sum += rb[i] - qx[i];
      part[cl * N2 + ln] = sum;
    }
    __syncthreads();
    if (active && ln == 0) {
      T sum = T(0);
      for (int l = 0; l < N2; ++l) sum += part[cl * N2 + l];
      rh[c] = sum;
    }
  }
}

// NB: with neighbour couplings (A) or without (D_T).
// RES = 0: write v = A u.
// RES = 3 (T = double): write v = A u and rh[block] = the block's partial
//   sum of u . v (per lane along its x-line, then over the wavefronts in
//   order): the outer iteration's (p, A p) without a second pass over p
//   and A p; dots_final adds the partials.
// RES = 1: write rh[c] = sum over the DOFs of cell c of (r - A u): the
//   residual followed by the P0 restriction R = P^T (Sec. 2.2.2), fused so
//   that A u never goes to memory.
// RES = 2: write rh[8c + q] = sum_i phi_q(x_i) (r - A u)_i for the eight
//   trilinear corner functions phi_q of cell c, q = qx + 2 qy + 4 qz: the
//   per-cell half of the Q1 restriction R = P^T (Sec. 2.2.2, the nodal
//   interpolation of the vertex functions); the vertex gather follows in a
//   separate kernel.
//
// Generic kernel (any affine b): lane (cell, a, b) applies the 1-D line
// operator along x, y and z to its three lines through (a, b); the
// contributions meet in LDS.
//
// HB = false: a build for b = 0 only (no advection code, fewer registers).
//
// FLD: the outer operator of a problem with a coefficient field: K_kk and
// c are evaluated at the nodes (= quadrature points) of each line instead
// of taken per cell (the preconditioner's kernels use the cell-centre
// values).
template <int P, typename T, bool NB, int RES = 0, bool FLD = false, bool HB = true>
__global__ __launch_bounds__(kApplyThreads) void k_apply(Geo g, const T *__restrict__ u, T *__restrict__ v,
                                                         const T *__restrict__ r = nullptr,
                                                         T *__restrict__ rh = nullptr) {
  constexpr int N = P + 1;
  using St = Stage<N, T, NB>;
  constexpr int N2 = St::N2, N3 = St::N3, CPB = St::CPB, H = St::H;
  using VT = typename St::VT;
  constexpr DevTab<T, N> tb = make_ctab<T, N>();
  __shared__ __align__(16) T us[St::LDS];
  __shared__ T qs[CPB * N3];  // y, then y + z contributions
  __shared__ AxisCoef<T> fcs[CPB][3];
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int c0 = blk * CPB;
  const int ncb = min(CPB, g.ncell - c0);
  const int tid = threadIdx.x;
  const int cl = tid / N2;
  const int ln = tid - cl * N2;
  const int a = ln % N, b = ln / N;
  const bool active = cl < ncb;
  const int c = c0 + cl;
  int ijk[3] = {0, 0, 0};
  if (active) cell_coords(g, c, ijk);
  const int nn[3] = {g.nx, g.ny, g.nz};
  const int stride[3] = {1, g.nx, g.nx * g.ny};

  VT pre[St::NVEC];
  const int shift = stage_load<N, T, NB>(g, u, c0, tid, pre);
  T yl[N], yr[N], zl[N], zr[N];
  if (NB && active) neighbour_lines_y<N, T>(g, u, c, ijk, a, b, yl, yr);
  // face coefficients: lane ln < 3 of each cell handles axis ln (neighbour
  // indices clamped to the cell itself, so that no load waits for another)
  double kd = 0.0, km = 0.0, kp = 0.0;
  const bool coef_lane = active && ln < 3;
  if (coef_lane && !FLD) {
    const int k = ln;
    const int ik = k == 0 ? ijk[0] : (k == 1 ? ijk[1] : ijk[2]);
    const int nk = k == 0 ? nn[0] : (k == 1 ? nn[1] : nn[2]);
    const int sk = k == 0 ? 1 : (k == 1 ? stride[1] : stride[2]);
    kd = g.K[3 * (size_t)c + k];
    km = g.K[3 * (size_t)(ik > 0 ? c - sk : c) + k];
    kp = g.K[3 * (size_t)(ik < nk - 1 ? c + sk : c) + k];
  }
  const T cre = (active && g.has_c && !FLD) ? (T)g.c[c] : T(0);
  const T stan = tb.w[a] * tb.w[b];

  T tr[2][4] = {{T(0), T(0), T(0), T(0)}, {T(0), T(0), T(0), T(0)}};
  if (NB) face_traces<N, T>(tb, yl, yr, tr[0]);
#pragma unroll
  for (int j = 0; j < St::NVEC; ++j) reinterpret_cast<VT *>(us)[j * kApplyThreads + tid] = pre[j];
  if (coef_lane) {
    // field: a compile-time axis per branch; cell-constant coefficients: one
    // path for the three axes (about a third of the instructions)
    if constexpr (FLD) {
      if (ln == 0)
        fcs[cl][0] = axis_coef_field<T>(g, 0, ijk);
      else if (ln == 1)
        fcs[cl][1] = axis_coef_field<T>(g, 1, ijk);
      else
        fcs[cl][2] = axis_coef_field<T>(g, 2, ijk);
    } else {
      fcs[cl][ln] = axis_coef_lane<T>(g, ln, ijk, kd, km, kp);
    }
  }
  __syncthreads();

  const bool hasb = HB && g.has_b != 0;
  const T vol = (T)g.vol;
  const T *own = us + shift + (cl + H) * N3;
  // The directions one after the other; their contributions meet in qs
  // (a DOF lies on exactly one line per direction, so the writes of one
  // direction do not collide), a barrier between directions.  Nothing but
  // the current line is held in registers: with HB = false the FP64 kernels
  // run at five (p = 4, 5) to seven (p = 1) waves per SIMD.  The z neighbour
  // lines are loaded after the x lines, behind the y-line work.
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (k == 1 && NB && active) neighbour_lines_z<N, T>(g, u, c, ijk, a, b, zl, zr);
    if (active) {
      T ul[N], out[N];
#pragma unroll
      for (int i = 0; i < N; ++i) ul[i] = own[line_pos<N>(k, i, a, b)];
      T t[4] = {T(0), T(0), T(0), T(0)};
      if (NB) {
        if (k == 0) {
          T lo[N], hi[N];
#pragma unroll
          for (int i = 0; i < N; ++i) {
            lo[i] = own[line_pos<N>(0, i, a, b) - N3];
            hi[i] = own[line_pos<N>(0, i, a, b) + N3];
          }
          face_traces<N, T>(tb, lo, hi, t);
        } else if (k == 1) {
#pragma unroll
          for (int q = 0; q < 4; ++q) t[q] = tr[0][q];
        } else {
          face_traces<N, T>(tb, zl, zr, t);
        }
        if (ijk[k] == 0) t[0] = t[1] = T(0);
        if (ijk[k] == nn[k] - 1) t[2] = t[3] = T(0);
      }
      LineConv<T> lc = {T(0), T(0), T(0), T(0)};
      if (hasb) lc = make_line_conv<T, N>(g, tb, k, ijk, a, b);
      if (FLD || hasb)
        line_apply<T, N>(tb, fcs[cl][k], stan, vol, k == 0 ? cre : T(0), hasb, lc, ul, t[0], t[1], t[2], t[3], out);
      else if (k == 0 && g.has_c)
        line_apply_eo<T, N, true>(fcs[cl][k], stan, vol, cre, ul, t[0], t[1], t[2], t[3], out);
      else
        line_apply_eo<T, N, false>(fcs[cl][k], stan, vol, T(0), ul, t[0], t[1], t[2], t[3], out);
      if constexpr (FLD) {
        // K_kk at the line's nodes; c at the nodes of the x-line
        T pk[N];
#pragma unroll
        for (int q = 0; q < N; ++q) pk[q] = (T)field_K(g, k, (ijk[k] + (double)tb.xi[q]) * g.h[k]);
        line_volume_field<T, N>(tb, stan, vol, (T)g.ih[k], pk, ul, out);
        if (k == 0 && g.has_c) {
          const double y = (ijk[1] + (double)tb.xi[a]) * g.h[1], z = (ijk[2] + (double)tb.xi[b]) * g.h[2];
#pragma unroll
          for (int i = 0; i < N; ++i)
            out[i] += (T)field_c(g, (ijk[0] + (double)tb.xi[i]) * g.h[0], y, z) * vol * stan * tb.w[i] * ul[i];
        }
      }
#pragma unroll
      for (int i = 0; i < N; ++i) {
        T *q = qs + cl * N3 + line_pos<N>(k, i, a, b);
        if (k == 0)
          *q = out[i];
        else
          *q += out[i];
      }
    }
    __syncthreads();
  }
  T qx[N];
  if (active) {
#pragma unroll
    for (int i = 0; i < N; ++i) qx[i] = qs[cl * N3 + line_pos<N>(0, i, a, b)];
  }
  if constexpr (RES == 0) {
    if (active) {
      T *vb = v + (size_t)c * N3 + N * a + N2 * b;
#pragma unroll
      for (int i = 0; i < N; ++i) vb[i] = qx[i];
    }
  } else if constexpr (RES == 3) {
    static_assert(sizeof(T) == 8, "the fused dot is an FP64 reduction");
    __shared__ double red[kApplyThreads / 64];
    double d = 0.0;
    if (active) {
      T *vb = v + (size_t)c * N3 + N * a + N2 * b;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        vb[i] = qx[i];
        d += own[line_pos<N>(0, i, a, b)] * qx[i];
      }
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) d += __shfl_xor(d, m, 64);
    if ((tid & 63) == 0) red[tid >> 6] = d;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < kApplyThreads / 64; ++w) t += red[w];
      rh[blk] = t;
    }
  } else {
    residual_epilogue<N, T, RES>(tb, active, c, cl, ln, a, b, qx, r, rh);
  }
}

// diag(D_T): one lane per DOF.
template <int P, typename T>
__global__ __launch_bounds__(256) void k_block_diag(Geo g, T *__restrict__ diag) {
  constexpr int N = P + 1, N2 = N * N, N3 = N * N * N;
  constexpr DevTab<T, N> tb = make_ctab<T, N>();
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)g.ncell * N3) return;
  const int c = (int)(gid / N3);
  const int j = (int)(gid - (int64_t)c * N3);
  const int q[3] = {j % N, (j / N) % N, j / N2};
  const int ijk[3] = {c % g.nx, (c / g.nx) % g.ny, c / (g.nx * g.ny)};
  const bool hasb = g.has_b != 0;
  T s = T(0);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int t1 = (k == 0) ? 1 : 0, t2 = (k == 2) ? 1 : 2;
    const AxisCoef<T> f = make_axis_coef<T>(g, c, k, ijk);
    LineConv<T> lc = {T(0), T(0), T(0), T(0)};
    if (hasb) lc = make_line_conv<T, N>(g, tb, k, ijk, q[t1], q[t2]);
    const T cre = (k == 0 && g.has_c) ? (T)g.c[c] : T(0);
    s += line_diag<T, N>(tb, f, tb.w[q[t1]] * tb.w[q[t2]], (T)g.vol, cre, hasb, lc, q[k]);
  }
  diag[gid] = s;
}

// Right-hand side l_h(psi_i) (eqn rhs), one lane per DOF.  With the
// collocated basis, (f, psi_i)_T = W_i f(x_i); boundary faces add the
// Neumann flux -(j, psi_i)_F and on Dirichlet faces
// -(Phi(0,g,b_nu), psi_i)_F - (nu.K grad psi_i, g)_F + gamma_F (g, psi_i)_F.
template <int P>
__global__ __launch_bounds__(256) void k_rhs(Geo g, const double *__restrict__ fq, const double *__restrict__ bq,
                                             double *__restrict__ rhs) {
  constexpr int N = P + 1, N2 = N * N, N3 = N * N * N;
  constexpr DevTab<double, N> tb = make_ctab<double, N>();
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (int64_t)g.ncell * N3) return;
  const int c = (int)(gid / N3);
  const int j = (int)(gid - (int64_t)c * N3);
  const int q[3] = {j % N, (j / N) % N, j / N2};
  const int ijk[3] = {c % g.nx, (c / g.nx) % g.ny, c / (g.nx * g.ny)};
  const int nn[3] = {g.nx, g.ny, g.nz};
  double val = 0.0;
  if (fq) val = tb.w[q[0]] * tb.w[q[1]] * tb.w[q[2]] * g.vol * fq[gid];
  if (bq) {
    int64_t off = 0;
    for (int f = 0; f < 6; ++f) {
      const int k = f >> 1, side = f & 1;
      const int t1 = (k == 0) ? 1 : 0, t2 = (k == 2) ? 1 : 2;
      const int64_t nface = (int64_t)nn[t1] * nn[t2];
      const bool on = side ? (ijk[k] == nn[k] - 1) : (ijk[k] == 0);
      if (on) {
        const int64_t cf = ijk[t1] + (int64_t)nn[t1] * ijk[t2];
        const double bv = bq[off + cf * N2 + q[t1] + N * q[t2]];
        const double WF = tb.w[q[t1]] * tb.w[q[t2]] * g.vol / g.h[k];
        const double ev = side ? tb.e1[q[k]] : tb.e0[q[k]];
        const double dv = (side ? tb.d1[q[k]] : tb.d0[q[k]]) / g.h[k];
        if (g.bc[f] == FACE_NEUMANN) {
          val -= WF * bv * ev;
        } else {
          const double nu = side ? 1.0 : -1.0;
          double d = g.field ? field_K(g, k, (ijk[k] + side) * g.h[k]) : g.K[3 * c + k];
          if (g.field == DG_FIELD_ROTATED_QUADRATIC) {
            // full tensor: K_kk here, and the tangential part of
            // nu . K grad psi_i paired with g over the face points that
            // share one tangential index with this DOF
            double x[3];
            x[k] = (ijk[k] + side) * g.h[k];
            x[t1] = (ijk[t1] + (double)tb.xi[q[t1]]) * g.h[t1];
            x[t2] = (ijk[t2] + (double)tb.xi[q[t2]]) * g.h[t2];
            double Kx[3][3];
            field_tensor(g, x, Kx);
            d = Kx[k][k];
            double tang = 0.0;
            for (int jj = 0; jj < N; ++jj) {
              // face point (jj, q[t2]): derivative along t1 of psi_i
              x[t1] = (ijk[t1] + (double)tb.xi[jj]) * g.h[t1];
              x[t2] = (ijk[t2] + (double)tb.xi[q[t2]]) * g.h[t2];
              field_tensor(g, x, Kx);
              const double g1 = bq[off + cf * N2 + jj + N * q[t2]];
              tang += tb.w[jj] * tb.w[q[t2]] * g1 * Kx[k][t1] * g.ih[t1] * tb.Dt[q[t1]][jj];
              // face point (q[t1], jj): derivative along t2
              x[t1] = (ijk[t1] + (double)tb.xi[q[t1]]) * g.h[t1];
              x[t2] = (ijk[t2] + (double)tb.xi[jj]) * g.h[t2];
              field_tensor(g, x, Kx);
              const double g2 = bq[off + cf * N2 + q[t1] + N * jj];
              tang += tb.w[q[t1]] * tb.w[jj] * g2 * Kx[k][t2] * g.ih[t2] * tb.Dt[q[t2]][jj];
            }
            val -= g.vol / g.h[k] * nu * ev * tang;
          }
          const double gam = g.sigma * d / g.h[k];
          double bnu = 0.0;
          if (g.has_b) {
            double x[3];
            for (int a = 0; a < 3; ++a) x[a] = (ijk[a] + (double)tb.xi[q[a]]) * g.h[a];
            x[k] = (ijk[k] + side) * g.h[k];
            double bk = g.b0[k];
            for (int a = 0; a < 3; ++a) bk += g.B[3 * k + a] * x[a];
            bnu = nu * bk;
          }
          const double inflow = bnu < 0.0 ? bnu : 0.0;
          val -= WF * (inflow * bv * ev + bv * nu * d * dv - gam * bv * ev);
        }
      }
      off += nface * N2;
    }
  }
  rhs[gid] = val;
}

// ev0 / ev1 (may be null): events recorded by the dispatch itself at the
// start and end of the apply kernel (hipExtLaunchKernelGGL), so that their
// difference is the kernel's own duration
template <int P, typename T>
static int launch_apply_t(const dg_problem *pr, const void *u, void *v, hipStream_t s, bool nb, hipEvent_t ev0,
                          hipEvent_t ev1) {
  constexpr int N = P + 1;
  const int G = (int)((pr->ncell + ApplyShape<N>::CPB - 1) / ApplyShape<N>::CPB);
  const dim3 grid(G), block(kApplyThreads);
  if (nb && pr->geo.field == DG_FIELD_ROTATED_QUADRATIC) {
    if (ev0) DG_HIP(hipEventRecord(ev0, s));
    const int rc = launch_apply_tensor(pr, sizeof(T) == 8 ? DG_FP64 : DG_FP32, u, v, s);
    if (ev1) DG_HIP(hipEventRecord(ev1, s));
    return rc;
  }
  if (nb && pr->geo.field)
    hipExtLaunchKernelGGL((k_apply<P, T, true, 0, true>), grid, block, 0, s, ev0, ev1, 0, pr->geo, (const T *)u,
                          (T *)v, (const T *)nullptr, (T *)nullptr);
  else if (nb && pr->geo.has_b)
    hipExtLaunchKernelGGL((k_apply<P, T, true>), grid, block, 0, s, ev0, ev1, 0, pr->geo, (const T *)u, (T *)v,
                          (const T *)nullptr, (T *)nullptr);
  else if (nb)
    hipExtLaunchKernelGGL((k_apply<P, T, true, 0, false, false>), grid, block, 0, s, ev0, ev1, 0, pr->geo,
                          (const T *)u, (T *)v, (const T *)nullptr, (T *)nullptr);
  else
    hipExtLaunchKernelGGL((k_apply<P, T, false>), grid, block, 0, s, ev0, ev1, 0, pr->geo, (const T *)u, (T *)v,
                          (const T *)nullptr, (T *)nullptr);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

template <typename T>
static int dispatch_apply(const dg_problem *pr, const void *u, void *v, hipStream_t s, bool nb, hipEvent_t ev0 = nullptr,
                          hipEvent_t ev1 = nullptr) {
  switch (pr->p) {
    case 1: return launch_apply_t<1, T>(pr, u, v, s, nb, ev0, ev1);
    case 2: return launch_apply_t<2, T>(pr, u, v, s, nb, ev0, ev1);
    case 3: return launch_apply_t<3, T>(pr, u, v, s, nb, ev0, ev1);
    case 4: return launch_apply_t<4, T>(pr, u, v, s, nb, ev0, ev1);
    case 5: return launch_apply_t<5, T>(pr, u, v, s, nb, ev0, ev1);
  }
  set_error("unsupported degree");
  return DG_EINVAL;
}

template <int P, typename T>
static int launch_res_t(const dg_problem *pr, const void *u, const void *r, void *rh, hipStream_t s, int kind) {
  constexpr int N = P + 1;
  const int G = (int)((pr->ncell + ApplyShape<N>::CPB - 1) / ApplyShape<N>::CPB);
  const bool hb = pr->geo.has_b != 0;
  if (kind == COARSE_Q1 && hb)
    hipLaunchKernelGGL((k_apply<P, T, true, 2>), dim3(G), dim3(kApplyThreads), 0, s, pr->geo, (const T *)u,
                       (T *)nullptr, (const T *)r, (T *)rh);
  else if (kind == COARSE_Q1)
    hipLaunchKernelGGL((k_apply<P, T, true, 2, false, false>), dim3(G), dim3(kApplyThreads), 0, s, pr->geo,
                       (const T *)u, (T *)nullptr, (const T *)r, (T *)rh);
  else if (hb)
    hipLaunchKernelGGL((k_apply<P, T, true, 1>), dim3(G), dim3(kApplyThreads), 0, s, pr->geo, (const T *)u,
                       (T *)nullptr, (const T *)r, (T *)rh);
  else
    hipLaunchKernelGGL((k_apply<P, T, true, 1, false, false>), dim3(G), dim3(kApplyThreads), 0, s, pr->geo,
                       (const T *)u, (T *)nullptr, (const T *)r, (T *)rh);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int launch_residual_restrict_gl(const dg_problem *pr, int prec, const void *u, const void *r, void *rh,
                                hipStream_t s, int kind) {
  const bool d = prec == DG_FP64;
  switch (pr->p) {
    case 1: return d ? launch_res_t<1, double>(pr, u, r, rh, s, kind) : launch_res_t<1, float>(pr, u, r, rh, s, kind);
    case 2: return d ? launch_res_t<2, double>(pr, u, r, rh, s, kind) : launch_res_t<2, float>(pr, u, r, rh, s, kind);
    case 3: return d ? launch_res_t<3, double>(pr, u, r, rh, s, kind) : launch_res_t<3, float>(pr, u, r, rh, s, kind);
    case 4: return d ? launch_res_t<4, double>(pr, u, r, rh, s, kind) : launch_res_t<4, float>(pr, u, r, rh, s, kind);
    case 5: return d ? launch_res_t<5, double>(pr, u, r, rh, s, kind) : launch_res_t<5, float>(pr, u, r, rh, s, kind);
  }
  set_error("unsupported degree");
  return DG_EINVAL;
}

// v = A u in FP64 with the partials of u . v (RES = 3); part holds
// apply_blocks(pr) entries.  Not for the rotated-tensor field (its own
// kernel): DG_EINVAL.
template <int P>
static int launch_apply_dot_t(const dg_problem *pr, const double *u, double *v, double *part, hipStream_t s,
                              hipEvent_t ev0, hipEvent_t ev1) {
  constexpr int N = P + 1;
  const int G = (int)((pr->ncell + ApplyShape<N>::CPB - 1) / ApplyShape<N>::CPB);
  const dim3 grid(G), block(kApplyThreads);
  if (pr->geo.field == DG_FIELD_ROTATED_QUADRATIC) {
    set_error("internal: no fused dot for the rotated-tensor apply");
    return DG_EINVAL;
  }
  if (pr->geo.field)
    hipExtLaunchKernelGGL((k_apply<P, double, true, 3, true>), grid, block, 0, s, ev0, ev1, 0, pr->geo, u, v,
                          (const double *)nullptr, part);
  else if (pr->geo.has_b)
    hipExtLaunchKernelGGL((k_apply<P, double, true, 3>), grid, block, 0, s, ev0, ev1, 0, pr->geo, u, v,
                          (const double *)nullptr, part);
  else
    hipExtLaunchKernelGGL((k_apply<P, double, true, 3, false, false>), grid, block, 0, s, ev0, ev1, 0, pr->geo, u,
                          v, (const double *)nullptr, part);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int launch_apply_dot_gl(const dg_problem *pr, const double *u, double *v, double *part, hipStream_t s, hipEvent_t ev0,
                        hipEvent_t ev1) {
  switch (pr->p) {
    case 1: return launch_apply_dot_t<1>(pr, u, v, part, s, ev0, ev1);
    case 2: return launch_apply_dot_t<2>(pr, u, v, part, s, ev0, ev1);
    case 3: return launch_apply_dot_t<3>(pr, u, v, part, s, ev0, ev1);
    case 4: return launch_apply_dot_t<4>(pr, u, v, part, s, ev0, ev1);
    case 5: return launch_apply_dot_t<5>(pr, u, v, part, s, ev0, ev1);
  }
  set_error("unsupported degree");
  return DG_EINVAL;
}

int64_t apply_blocks(int p, int64_t ncell) {
  const int n2 = (p + 1) * (p + 1);
  const int64_t cpb = kApplyThreads / n2;
  return (ncell + cpb - 1) / cpb;
}

int launch_apply_gl(const dg_problem *pr, int prec, const void *u, void *v, hipStream_t s, hipEvent_t ev0,
                    hipEvent_t ev1) {
  return prec == DG_FP64 ? dispatch_apply<double>(pr, u, v, s, true, ev0, ev1)
                         : dispatch_apply<float>(pr, u, v, s, true, ev0, ev1);
}

// v = A u with the coefficients at the cell centres: the operator of the
// preconditioner when K and c are fields (equal to launch_apply_gl
// otherwise)
template <int P, typename T>
static int launch_apply_cc_t(const dg_problem *pr, const void *u, void *v, hipStream_t s) {
  constexpr int N = P + 1;
  const dim3 grid((unsigned)((pr->ncell + ApplyShape<N>::CPB - 1) / ApplyShape<N>::CPB)), block(kApplyThreads);
  if (pr->geo.has_b)
    hipLaunchKernelGGL((k_apply<P, T, true>), grid, block, 0, s, pr->geo, (const T *)u, (T *)v, (const T *)nullptr,
                       (T *)nullptr);
  else
    hipLaunchKernelGGL((k_apply<P, T, true, 0, false, false>), grid, block, 0, s, pr->geo, (const T *)u, (T *)v,
                       (const T *)nullptr, (T *)nullptr);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int launch_apply_cc_gl(const dg_problem *pr, int prec, const void *u, void *v, hipStream_t s) {
  const bool d = prec == DG_FP64;
  switch (pr->p) {
    case 1: return d ? launch_apply_cc_t<1, double>(pr, u, v, s) : launch_apply_cc_t<1, float>(pr, u, v, s);
    case 2: return d ? launch_apply_cc_t<2, double>(pr, u, v, s) : launch_apply_cc_t<2, float>(pr, u, v, s);
    case 3: return d ? launch_apply_cc_t<3, double>(pr, u, v, s) : launch_apply_cc_t<3, float>(pr, u, v, s);
    case 4: return d ? launch_apply_cc_t<4, double>(pr, u, v, s) : launch_apply_cc_t<4, float>(pr, u, v, s);
    case 5: return d ? launch_apply_cc_t<5, double>(pr, u, v, s) : launch_apply_cc_t<5, float>(pr, u, v, s);
  }
  set_error("unsupported degree");
  return DG_EINVAL;
}

int launch_block_apply_gl(const dg_problem *pr, int prec, const void *x, void *y, hipStream_t s) {
  return prec == DG_FP64 ? dispatch_apply<double>(pr, x, y, s, false) : dispatch_apply<float>(pr, x, y, s, false);
}

template <int P, typename T>
static int launch_diag_t(const dg_problem *pr, void *diag, hipStream_t s) {
  constexpr int N = P + 1;
  const int64_t tot = pr->ndof;
  const int G = (int)((tot + 255) / 256);
  hipLaunchKernelGGL((k_block_diag<P, T>), dim3(G), dim3(256), 0, s, pr->geo, (T *)diag);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int launch_block_diag_gl(const dg_problem *pr, int prec, void *diag, hipStream_t s) {
  switch (pr->p) {
    case 1: return prec == DG_FP64 ? launch_diag_t<1, double>(pr, diag, s) : launch_diag_t<1, float>(pr, diag, s);
    case 2: return prec == DG_FP64 ? launch_diag_t<2, double>(pr, diag, s) : launch_diag_t<2, float>(pr, diag, s);
    case 3: return prec == DG_FP64 ? launch_diag_t<3, double>(pr, diag, s) : launch_diag_t<3, float>(pr, diag, s);
    case 4: return prec == DG_FP64 ? launch_diag_t<4, double>(pr, diag, s) : launch_diag_t<4, float>(pr, diag, s);
    case 5: return prec == DG_FP64 ? launch_diag_t<5, double>(pr, diag, s) : launch_diag_t<5, float>(pr, diag, s);
  }
  set_error("unsupported degree");
  return DG_EINVAL;
}

template <int P>
static int launch_rhs_t(const dg_problem *pr, const double *fq, const double *bq, double *rhs, hipStream_t s) {
  constexpr int N = P + 1;
  const int G = (int)((pr->ndof + 255) / 256);
  hipLaunchKernelGGL((k_rhs<P>), dim3(G), dim3(256), 0, s, pr->geo, fq, bq, rhs);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

int launch_rhs_gl(const dg_problem *pr, const double *fq, const double *bq, double *rhs, hipStream_t s) {
  switch (pr->p) {
    case 1: return launch_rhs_t<1>(pr, fq, bq, rhs, s);
    case 2: return launch_rhs_t<2>(pr, fq, bq, rhs, s);
    case 3: return launch_rhs_t<3>(pr, fq, bq, rhs, s);
    case 4: return launch_rhs_t<4>(pr, fq, bq, rhs, s);
    case 5: return launch_rhs_t<5>(pr, fq, bq, rhs, s);
  }
  set_error("unsupported degree");
  return DG_EINVAL;
}

}  // namespace dgmg
