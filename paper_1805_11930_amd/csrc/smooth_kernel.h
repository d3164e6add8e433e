// Fused matrix-free block-Jacobi sweep (alg block_jacobi, Sec. 2.2.1) with
// inexact iterative block inversion (Sec. 2.2.1, eqn block_system; the
// diagonal preconditioner of Sec. 3.2).
//
// One sweep  u_out = u_in + omega * D^-1_eps (f - A u_in)  runs as a single
// kernel:  defect (the same line operators as the apply, neighbours read
// from global memory), then a Krylov solve of D_T du_T = d_T in every cell,
// then the damped update.
//
// Mapping.  A workgroup is ONE wavefront of 64 lanes.  Each cell gets L
// lanes, L = the power of two >= (p+1)^2 (p=1: 4, p=2,3: 16, p=4: 32), so
// 64/L cells share a wavefront and the per-cell dot products are butterfly
// shuffles inside aligned lane groups (bitwise identical in every lane of
// the cell).  Lane (a, b) keeps the x-line (y=a, z=b) of every Krylov
// vector in registers.  D_T p is applied as in the apply: x-direction in
// registers, y- and z-directions through an LDS transpose, two barriers per
// application (a barrier of a one-wave workgroup is cheap).  Cells of a
// wavefront iterate until all of them have converged; a converged cell is
// masked, so the lock-step waste is bounded by the worst of 2-16 cells
// rather than of a whole grid.
//
// Inner methods (readings of the paper, which does not spell them out):
//   CG:    Hestenes-Stiefel PCG, x0 = 0, M = diag(D_T), stop when the
//          recursive residual satisfies ||r||_2 <= eps ||d_T||_2 or after
//          max_inner applications of D_T;
//   GMRES: right-preconditioned restarted GMRES(restart), classical
//          Gram-Schmidt applied twice (the projections of a pass are
//          independent cell sums), Givens rotations, stop when the Arnoldi residual
//          estimate <= eps ||d_T||_2 or after max_inner applications.
// and, for b = 0, the exact solve with stored factors (fdm.hip):
//   FDM:   x = (Tz (x) Ty (x) Tx) diag(1/(lx+ly+lz)) (Tz (x) Ty (x) Tx)^T d,
//          the six contractions through the same LDS transposes;
// and, for any b, the partially matrix-free exact solve (pmf.hip):
//   PMF:   x = D_T^-1 d with the stored inverse of the block, one dense
//          product per cell streamed from memory.
#pragma once

#include "line_ops.h"

namespace dgmg {

constexpr int kSmoothThreads = 64;
constexpr int kGmresMax = 16;  // largest inner GMRES restart length

template <int N>
struct SmoothShape {
  static constexpr int N2 = N * N;
  static constexpr int N3 = N * N * N;
  static constexpr int L = N2 <= 4 ? 4 : (N2 <= 16 ? 16 : (N2 <= 32 ? 32 : 64));
  static constexpr int CPW = kSmoothThreads / L;
};

template <int N>
__device__ inline int lpos(int k, int i, int a, int b) {
  return k == 0 ? i + N * a + N * N * b : (k == 1 ? a + N * i + N * N * b : a + N * b + N * N * i);
}

// Lane permutation of a 32-bit register within rows of 16 lanes (DPP).
// Every lane of the permutations used here has a source lane, so the
// bound-control bit changes nothing; with it set (and old = 0) the compiler
// folds the permutation into the add that consumes it (v_add_f32_dpp).
template <int CTRL>
__device__ inline float dpp_perm(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ inline double dpp_perm(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffff), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Value of lane i xor 16 within each group of 32 lanes (ds_swizzle in
// bit mode: and-mask 0x1f, or-mask 0, xor-mask 0x10; no LDS memory access).
__device__ inline float swz_xor16(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, v), 0x401F));
}
__device__ inline double swz_xor16(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_ds_swizzle((int)(b & 0xffffffff), 0x401F);
  const int hi = __builtin_amdgcn_ds_swizzle((int)(b >> 32), 0x401F);
  return __builtin_bit_cast(double, (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Sum over the L lanes (L = 4, 16, 32 or 64, aligned) of a cell; every lane
// of the cell receives the same bits.  Each step adds the value of a
// partner lane whose group is disjoint and of equal size: within quads
// (partner lane xor 1, then xor 2), then the mirrored half-row (lane 7 - i
// of each 8) and row (lane 15 - i of each 16) by DPP, then lane xor 16 and
// lane xor 32.  Both
// partners of a step add the same two numbers, and addition commutes, so
// the bits agree across the cell.
template <int L, typename T>
__device__ inline T cell_sum(T v) {
  static_assert(L == 4 || L == 16 || L == 32 || L == 64, "cell lane groups are 4, 16, 32 or 64 lanes");
  v += dpp_perm<0xB1>(v);  // quad_perm [1, 0, 3, 2]
  v += dpp_perm<0x4E>(v);  // quad_perm [2, 3, 0, 1]
  if constexpr (L >= 16) {
    v += dpp_perm<0x141>(v);  // row_half_mirror
    v += dpp_perm<0x140>(v);  // row_mirror
  }
  if constexpr (L >= 32) v += swz_xor16(v);
  if constexpr (L == 64) v += __shfl_xor(v, 32, 64);
  return v;
}

// a / b for the scalars of the inner iteration: FP32 by the hardware
// reciprocal (about 1 ulp; the FP32 inner solve stops at eps >= 1e-7)
// when b is a normal number, by IEEE division when b is zero or subnormal
// (whose reciprocal overflows; blocks with tiny right-hand sides reach such
// values), FP64 correctly rounded
__device__ inline float inner_div(float a, float b) {
  float r = a * __builtin_amdgcn_rcpf(b);
  if (!(fabsf(b) >= 1.17549435e-38f)) r = a / b;
  return r;
}
__device__ inline double inner_div(double a, double b) { return a / b; }

struct SmoothKArgs {
  double omega, eps;
  int max_inner, restart;
  int zero_guess, write_du, defect;
  // colour >= 0: only the cells with (ix + iy + iz) mod ncol == colour;
  // slot j of the grid -> row j / hx (hx = ceil(nx / ncol)) and block
  // t = j % hx of ncol consecutive cells of that row, whose cell
  // ix = ncol t + ((colour - iy - iz) mod ncol) has the colour;
  // rows = ny * nz.
  int colour, ncol, hx, rows;
  // block-SOR form (alg block_SOR): the defect leaves out the cell's own
  // block and the new value is (1 - omega) u + omega x
  int sor;
  CastBackArgs cb;  // cb.part != nullptr: the dots (and, T = float, cast-back) epilogue
};

// Per-lane data of the three lines (x: y=a,z=b; y: x=a,z=b; z: x=a,y=b)
// through the lane's line index; all three share the tangential weight
// product w_a w_b.
template <int P, typename T>
struct CellLines {
  AxisCoef<T> f[3];
  LineConv<T> lc[3];
  T stan, vol, cre;
};

// M u with one of the cell's per-axis matrices held in LDS (b = 0)
template <typename T, int N>
__device__ inline void mat_line(const T *M, const T (&u)[N], T (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T acc = T(0);
#pragma unroll
    for (int l = 0; l < N; ++l) acc += M[i * N + l] * u[l];
    v[i] = acc;
  }
}

// q = D_T p on the lane's x-line.  All lanes of the wavefront must call it.
// MS (b = 0): Ms holds the cell's three axis matrices with their rows
// divided by the node weights, Mt_k = W^-1 M_k: D_T is the Kronecker sum
// Mx (x) Wy (x) Wz + Wx (x) My (x) Wz + Wx (x) Wy (x) Mz, so
// D_T p = (Wx (x) Wy (x) Wz) (sum over k of Mt_k along axis k) p, and the
// weights w3[i] = w_i w_a w_b of the lane's DOFs are applied once at the
// end.  Otherwise the generic line operators (the stan weight inside).
template <int P, typename T, bool MS>
__device__ inline void dt_apply(const CellLines<P, T> &cl, const DevTab<T, P + 1> &tb, bool on, bool hasb,
                                const T *Ms, const T (&w3)[P + 1], const T (&p)[P + 1], T (&q)[P + 1], T *Ps,
                                T *Qy, T *Qz, int a, int b) {
  constexpr int N = P + 1;
  constexpr int N2 = N * N;
  T qx[N];
  if (on) {
    if constexpr (MS)
      mat_line<T, N>(Ms, p, qx);
    else
      line_apply<T, N>(tb, cl.f[0], cl.stan, cl.vol, cl.cre, hasb, cl.lc[0], p, T(0), T(0), T(0), T(0), qx);
#pragma unroll
    for (int i = 0; i < N; ++i) Ps[lpos<N>(0, i, a, b)] = p[i];
  }
  __syncthreads();
  if (on) {
    T yl[N], yo[N];
#pragma unroll
    for (int i = 0; i < N; ++i) yl[i] = Ps[lpos<N>(1, i, a, b)];
    if constexpr (MS)
      mat_line<T, N>(Ms + N2, yl, yo);
    else
      line_apply<T, N>(tb, cl.f[1], cl.stan, cl.vol, T(0), hasb, cl.lc[1], yl, T(0), T(0), T(0), T(0), yo);
#pragma unroll
    for (int i = 0; i < N; ++i) Qy[lpos<N>(1, i, a, b)] = yo[i];
#pragma unroll
    for (int i = 0; i < N; ++i) yl[i] = Ps[lpos<N>(2, i, a, b)];
    if constexpr (MS)
      mat_line<T, N>(Ms + 2 * N2, yl, yo);
    else
      line_apply<T, N>(tb, cl.f[2], cl.stan, cl.vol, T(0), hasb, cl.lc[2], yl, T(0), T(0), T(0), T(0), yo);
#pragma unroll
    for (int i = 0; i < N; ++i) Qz[lpos<N>(2, i, a, b)] = yo[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const T sum = qx[i] + Qy[lpos<N>(0, i, a, b)] + Qz[lpos<N>(0, i, a, b)];
    q[i] = on ? (MS ? w3[i] * sum : sum) : T(0);
  }
}

// q = D_T p with the lane's three line operators held as N x N matrices in
// registers, Mr[k][i * N + l] (axis k; the x-line, y-line and z-line of the
// lane).  All lanes of the wavefront must call it.
template <int P, typename T>
__device__ inline void dt_apply_reg(const T (&Mr)[3][(P + 1) * (P + 1)], bool on, const T (&p)[P + 1],
                                    T (&q)[P + 1], T *Ps, T *Qy, T *Qz, int a, int b) {
  constexpr int N = P + 1;
  T qx[N];
  if (on) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      T acc = T(0);
#pragma unroll
      for (int l = 0; l < N; ++l) acc += Mr[0][i * N + l] * p[l];
      qx[i] = acc;
    }
#pragma unroll
    for (int i = 0; i < N; ++i) Ps[lpos<N>(0, i, a, b)] = p[i];
  }
  __syncthreads();
  if (on) {
#pragma unroll
    for (int k = 1; k < 3; ++k) {
      T yl[N];
#pragma unroll
      for (int i = 0; i < N; ++i) yl[i] = Ps[lpos<N>(k, i, a, b)];
      T *Q = k == 1 ? Qy : Qz;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        T acc = T(0);
#pragma unroll
        for (int l = 0; l < N; ++l) acc += Mr[k][i * N + l] * yl[l];
        Q[lpos<N>(k, i, a, b)] = acc;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < N; ++i) q[i] = on ? qx[i] + Qy[lpos<N>(0, i, a, b)] + Qz[lpos<N>(0, i, a, b)] : T(0);
}

// HASB: advection present (compile-time, so the b = 0 kernels carry no
// advection code and keep only the per-cell matrices live in the loop).
// Contraction of the lane's line with a matrix stored row-major in LDS:
// v_i = sum_l M[i][l] u_l (TR = false) or sum_l M[l][i] u_l (TR = true).
template <typename T, int N, bool TR>
__device__ inline void contract(const T *M, const T (&u)[N], T (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T acc = T(0);
#pragma unroll
    for (int l = 0; l < N; ++l) acc += (TR ? M[l * N + i] : M[i * N + l]) * u[l];
    v[i] = acc;
  }
}

// Inner preconditioner M^-1 v on the lane's x-line: the diagonal of D_T
// (TRI = false: dinv = 1 / diag), or the tridiagonal part of D_T solved by
// the Thomas algorithm (TRI = true: dinv = 1 / pivot, tc = eliminated
// super-diagonal, tl = sub-diagonal).  With the x-fastest DOF order the
// tridiagonal part of D_T has no entries between two x-lines, so it is one
// tridiagonal system per x-line, held in the registers of its lane.
template <typename T, int N, bool TRI>
__device__ inline void prec_apply(const T (&dinv)[N], const T (&tc)[N], const T (&tl)[N], const T (&v)[N],
                                  T (&out)[N]) {
  if constexpr (!TRI) {
#pragma unroll
    for (int i = 0; i < N; ++i) out[i] = v[i] * dinv[i];
  } else {
    T y[N];
    y[0] = v[0] * dinv[0];
#pragma unroll
    for (int i = 1; i < N; ++i) y[i] = (v[i] - tl[i] * y[i - 1]) * dinv[i];
    out[N - 1] = y[N - 1];
#pragma unroll
    for (int i = N - 2; i >= 0; --i) out[i] = y[i] - tc[i] * out[i + 1];
  }
}

// Basis change on the cell held as x-lines by its lanes (Gauss-Lobatto
// basis, S = V (x) V (x) V): v = S u (TR = false) or S^T u (TR = true).
// x-direction in registers, then the y- and z-lines through Ps in place
// (lane (a, b) owns the y-line x=a, z=b and the z-line x=a, y=b, so no
// two lanes touch the same entries within a phase).  All lanes of the
// wavefront must call it.
template <typename T, int N, bool TR>
__device__ inline void gll_change(bool on, const T (&u)[N], T (&v)[N], T *Ps, int a, int b) {
  constexpr GllDev<N, T> gd = make_gll_dev<N, T>();
  auto line = [&](const T(&in)[N], T(&out)[N]) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      T acc = T(0);
#pragma unroll
      for (int l = 0; l < N; ++l) acc += (TR ? gd.V[l][i] : gd.V[i][l]) * in[l];
      out[i] = acc;
    }
  };
  T t[N];
  line(u, t);
  if (on) {
#pragma unroll
    for (int i = 0; i < N; ++i) Ps[lpos<N>(0, i, a, b)] = t[i];
  }
  __syncthreads();
#pragma unroll
  for (int k = 1; k < 3; ++k) {
    if (on) {
      T y[N];
#pragma unroll
      for (int i = 0; i < N; ++i) y[i] = Ps[lpos<N>(k, i, a, b)];
      line(y, t);
#pragma unroll
      for (int i = 0; i < N; ++i) Ps[lpos<N>(k, i, a, b)] = t[i];
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] = on ? Ps[lpos<N>(0, i, a, b)] : T(0);
}

// M^-1 v for M = the tridiagonal part of the whole cell block in its
// x-fastest DOF order (Gauss-Lobatto basis: unlike the Gauss-point basis,
// the block couples the last DOF of an x-line to the first of the next, so
// the band is one chain over the cell's (p+1)^3 DOFs).  Tf holds the cell's
// Thomas factors in LDS: [0, N3) 1/m_k, [N3, 2 N3) sub_k, [2 N3, 3 N3) c_k.
// The substitutions y_k = (v_k - sub_k y_(k-1)) / m_k and
// x_k = y_k - c_k x_(k+1) run along each lane's x-line as affine functions
// of the value carried in from the neighbouring line (A + B * carry); one
// lane then chains the (p+1)^2 line maps through LDS (Ab, carry), and every
// lane finishes its line from its carry: (p+1)^2 + 2 (p+1) dependent steps
// per substitution instead of (p+1)^3.  All lanes of the wavefront must call
// it.
template <typename T, int N>
__device__ inline void tri_cell(bool on, bool lead, const T (&v)[N], T (&out)[N], T *Ab, T *carry, const T *Tf,
                                int a, int b) {
  constexpr int N2 = N * N, N3 = N2 * N;
  const int ln = a + N * b;
  // forward: y_last = A + B * y_in on the lane's line
  T A = T(0), B = T(1);
  if (on) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const int k = i + N * ln;
      const T m = Tf[k], sb = Tf[N3 + k];
      A = (v[i] - sb * A) * m;
      B = -sb * m * B;
    }
    Ab[2 * ln] = A;
    Ab[2 * ln + 1] = B;
  }
  __syncthreads();
  if (lead) {
    T y = T(0);
    for (int l = 0; l < N2; ++l) {
      carry[l] = y;
      y = Ab[2 * l] + Ab[2 * l + 1] * y;
    }
  }
  __syncthreads();
  T y[N];
  {
    T prev = on ? carry[ln] : T(0);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const int k = i + N * ln;
      y[i] = on ? (v[i] - Tf[N3 + k] * prev) * Tf[k] : T(0);
      prev = y[i];
    }
  }
  __syncthreads();  // the carries are read before they are rewritten
  // backward: x_first = A + B * x_in on the lane's line
  A = T(0);
  B = T(1);
  if (on) {
#pragma unroll
    for (int i = N - 1; i >= 0; --i) {
      const T c = Tf[2 * N3 + i + N * ln];
      A = y[i] - c * A;
      B = -c * B;
    }
    Ab[2 * ln] = A;
    Ab[2 * ln + 1] = B;
  }
  __syncthreads();
  if (lead) {
    T x = T(0);
    for (int l = N2 - 1; l >= 0; --l) {
      carry[l] = x;
      x = Ab[2 * l] + Ab[2 * l + 1] * x;
    }
  }
  __syncthreads();
  {
    T next = on ? carry[ln] : T(0);
#pragma unroll
    for (int i = N - 1; i >= 0; --i) {
      out[i] = on ? y[i] - Tf[2 * N3 + i + N * ln] * next : T(0);
      next = out[i];
    }
  }
}

// uin and uout may be the same vector for a colour sweep: the cells written
// are exactly the cells of that colour, each by its own lanes after they
// read it, and the neighbours read all have the other colour.
// RM: bound of the inner GMRES restart length, sizing the Krylov basis in
// LDS and the rotation state in registers (8, 12 or kGmresMax; at p = 3 in
// FP32 the 8 build fits three wavefronts per SIMD, the 12 build two).
// GLL: Gauss-Lobatto basis.  The inner method (CG or GMRES) solves
// S^T D_T S x = d with S applied around D_T in every iteration, the inner
// preconditioner comes from stored entries of S^T D_T S (fdm = [4][ndof]:
// the diagonal, and the factored tridiagonal band of the whole block, see
// basis.hip), and the defect is formed outside the kernel (sa.defect = 0,
// f = the defect).
//
// The FP64 inner-CG sweep for b = 0 at p = 4 is held to 128 registers (four
// waves per SIMD instead of three, 14 registers spilled): on 32^3 cells the
// FP64-preconditioned solve went 16.3 -> 16.0 ms.
template <int P, int INNER, typename T, bool HASB, bool TRI, int RM = kGmresMax, bool GLL = false>
__global__ __launch_bounds__(kSmoothThreads) __attribute__((amdgpu_waves_per_eu(
    sizeof(T) == 8 && INNER == DG_INNER_CG && !HASB && P == 4 ? 4 : 1))) void k_smooth(Geo g, const T *__restrict__ f,
                                                                                       const T *uin, T *uout,
                                                           SmoothKArgs sa, int *__restrict__ iters,
                                                           const T *__restrict__ zh, const T *__restrict__ fdm) {
  constexpr int N = P + 1;
  using S = SmoothShape<N>;
  constexpr int L = S::L;
  constexpr DevTab<T, N> tb = make_ctab<T, N>();
  __shared__ T Ps_all[S::CPW * S::N3];
  __shared__ T Qy_all[S::CPW * S::N3];
  __shared__ T Qz_all[S::CPW * S::N3];
  __shared__ T Ms_all[S::CPW * 3 * S::N2];  // per-cell axis matrices (b = 0), or the FDM factors T_k
  __shared__ T Lm_all[INNER == DG_INNER_FDM ? S::CPW * 3 * N : 1];  // FDM eigenvalues
  // GMRES storage: Krylov basis (lane-private x-lines) and the rotated
  // Hessenberg columns of each cell.
  __shared__ T Vs_all[INNER == DG_INNER_GMRES ? S::CPW * (RM + 1) * S::N3 : 1];
  __shared__ T Hs_all[INNER == DG_INNER_GMRES ? S::CPW * RM * RM : 1];
  // Gauss-Lobatto basis with the tridiagonal inner preconditioner: the
  // cell's Thomas factors (see tri_cell)
  constexpr bool TRIC = GLL && TRI;
  __shared__ T Tf_all[TRIC ? S::CPW * 3 * S::N3 : 1];

  const int tid = threadIdx.x;
  const int cw = tid / L;
  const int lane = tid - cw * L;
  const int slot = blockIdx.x * S::CPW + cw;
  int c = slot;
  bool valid = slot < g.ncell;
  if (sa.colour >= 0) {
    const int C = sa.ncol;
    const int r = slot / sa.hx;
    const int t = slot - r * sa.hx;
    const int iy = r % g.ny, iz = r / g.ny;
    int s0 = (sa.colour - iy - iz) % C;
    if (s0 < 0) s0 += C;
    const int ix = C * t + s0;
    valid = r < sa.rows && ix < g.nx;
    c = valid ? ix + g.nx * r : 0;
    // from a zero guess the slot also clears the other cells of its block
    // (the blocks cover the row), so that the later colours start from zero
    if (sa.zero_guess && r < sa.rows && lane < S::N2) {
      for (int s1 = 0; s1 < C; ++s1) {
        const int px = C * t + s1;
        if (s1 == s0 || px >= g.nx) continue;
        T *dst = uout + ((size_t)px + (size_t)g.nx * r) * S::N3;
#pragma unroll
        for (int i = 0; i < N; ++i) dst[lpos<N>(0, i, lane % N, lane / N)] = T(0);
      }
    }
  }
  const bool on = (lane < S::N2) && valid;
  const int a = on ? lane % N : 0;
  const int b = on ? lane / N : 0;
  T *Ps = Ps_all + cw * S::N3;
  T *Qy = Qy_all + cw * S::N3;
  T *Qz = Qz_all + cw * S::N3;
  constexpr bool hasb = HASB;

  int ijk[3] = {0, 0, 0};
  CellLines<P, T> cl;
  cl.stan = tb.w[a] * tb.w[b];
  cl.vol = (T)g.vol;
  cl.cre = T(0);
  if (on) {
    ijk[0] = c % g.nx;
    ijk[1] = (c / g.nx) % g.ny;
    ijk[2] = c / (g.nx * g.ny);
    cl.cre = g.has_c ? (T)g.c[c] : T(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      cl.f[k] = make_axis_coef<T>(g, c, k, ijk);
      cl.lc[k] = hasb ? make_line_conv<T, N>(g, tb, k, ijk, a, b) : LineConv<T>{T(0), T(0), T(0), T(0)};
    }
  }
  const size_t base = (size_t)c * S::N3;
  // for b = 0 each axis of D_T is one n x n matrix per cell: lane (a, b)
  // builds entry (a, b) of the three matrices once
  T *Ms = HASB ? nullptr : Ms_all + cw * 3 * S::N2;
  T *Lm = Lm_all + (INNER == DG_INNER_FDM ? cw * 3 * N : 0);
  if (INNER == DG_INNER_FDM) {
    // the cell's stored factors [3][N*N + N] -> T_k into Ms, lambda_k into Lm
    constexpr int NF = S::N2 + N;
    if (valid) {
      const T *src = fdm + (size_t)c * 3 * NF;
      for (int e = lane; e < 3 * NF; e += L) {
        const int k = e / NF, j = e - k * NF;
        const T val = src[e];
        if (j < S::N2)
          Ms_all[cw * 3 * S::N2 + k * S::N2 + j] = val;
        else
          Lm[k * N + (j - S::N2)] = val;
      }
    }
  } else if (INNER != DG_INNER_PMF && Ms && on) {
    // row a of each axis matrix divided by w_a (see dt_apply)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      Ms[k * S::N2 + a * N + b] =
          line_matrix_entry<T, N>(tb, cl.f[k], cl.vol, k == 0 ? cl.cre : T(0), a, b) / tb.w[a];
  }
  // weights w_i w_a w_b of the lane's DOFs (the b = 0 form of dt_apply)
  T w3[N];
#pragma unroll
  for (int i = 0; i < N; ++i) w3[i] = cl.stan * tb.w[i];
  __syncthreads();

  // ---- defect d = f - A u -------------------------------------------------
  T ul[N], d[N];
  // the smoothed iterate is u_in + P zh when a P0 correction is given
  // (prolongation fused into the sweep; P|_T = (1,...,1)^T)
  const T zc = (on && zh) ? zh[c] : T(0);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    ul[i] = (on && !sa.zero_guess) ? uin[base + lpos<N>(0, i, a, b)] + zc : T(0);
    d[i] = on ? f[base + lpos<N>(0, i, a, b)] : T(0);
  }
  if (sa.defect && !sa.zero_guess) {
    const int nn[3] = {g.nx, g.ny, g.nz};
    const int stride[3] = {1, g.nx, g.nx * g.ny};
    T ax[N], own[N];
#pragma unroll
    for (int i = 0; i < N; ++i) own[i] = sa.sor ? T(0) : ul[i];
    if (on) {
#pragma unroll
      for (int i = 0; i < N; ++i) Ps[lpos<N>(0, i, a, b)] = own[i];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (on) {
        T line[N], out[N];
#pragma unroll
        for (int i = 0; i < N; ++i) line[i] = k == 0 ? own[i] : Ps[lpos<N>(k, i, a, b)];
        T tLu = T(0), tLd = T(0), tRu = T(0), tRd = T(0);
        if (ijk[k] > 0) {
          const int cn = c - stride[k];
          const T *src = uin + (size_t)cn * S::N3;
          const T zn = zh ? zh[cn] : T(0);
#pragma unroll
          for (int i = 0; i < N; ++i) {
            const T x = src[lpos<N>(k, i, a, b)] + zn;
            tLu += tb.e1[i] * x;
            tLd += tb.d1[i] * x;
          }
        }
        if (ijk[k] < nn[k] - 1) {
          const int cn = c + stride[k];
          const T *src = uin + (size_t)cn * S::N3;
          const T zn = zh ? zh[cn] : T(0);
#pragma unroll
          for (int i = 0; i < N; ++i) {
            const T x = src[lpos<N>(k, i, a, b)] + zn;
            tRu += tb.e0[i] * x;
            tRd += tb.d0[i] * x;
          }
        }
        if constexpr (HASB)
          line_apply<T, N>(tb, cl.f[k], cl.stan, cl.vol, k == 0 ? cl.cre : T(0), hasb, cl.lc[k], line, tLu, tLd, tRu,
                           tRd, out);
        else if (k == 0 && g.has_c)
          line_apply_eo<T, N, true>(cl.f[k], cl.stan, cl.vol, cl.cre, line, tLu, tLd, tRu, tRd, out);
        else
          line_apply_eo<T, N, false>(cl.f[k], cl.stan, cl.vol, T(0), line, tLu, tLd, tRu, tRd, out);
        if (k == 0) {
#pragma unroll
          for (int i = 0; i < N; ++i) ax[i] = out[i];
        } else {
          T *Q = k == 1 ? Qy : Qz;
#pragma unroll
          for (int i = 0; i < N; ++i) Q[lpos<N>(k, i, a, b)] = out[i];
        }
      }
    }
    __syncthreads();
    if (on) {
#pragma unroll
      for (int i = 0; i < N; ++i) d[i] -= ax[i] + Qy[lpos<N>(0, i, a, b)] + Qz[lpos<N>(0, i, a, b)];
    }
    __syncthreads();
  }

  // ---- inner preconditioner: M = diag(D_T) or its tridiagonal part ---------
  T dinv[N], tc[N], tl[N];
  const size_t ndof = (size_t)g.ncell * S::N3;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T dd = T(1);
    if (INNER == DG_INNER_FDM || INNER == DG_INNER_PMF) {
      // not used
    } else if (GLL) {
      if (on) dd = fdm[base + lpos<N>(0, i, a, b)];
    } else if (on && Ms) {
      // DOF (i, a, b): x-line (a, b), y-line (x=i, z=b), z-line (x=i, y=a)
      dd = w3[i] * (Ms[i * N + i] + Ms[S::N2 + a * N + a] + Ms[2 * S::N2 + b * N + b]);
    } else if (on) {
      // DOF (i, a, b) lies on the x-line (a, b), the y-line (x=i, z=b) and
      // the z-line (x=i, y=a)
      const LineConv<T> zero = {T(0), T(0), T(0), T(0)};
      const LineConv<T> ly = hasb ? make_line_conv<T, N>(g, tb, 1, ijk, i, b) : zero;
      const LineConv<T> lz = hasb ? make_line_conv<T, N>(g, tb, 2, ijk, i, a) : zero;
      dd = line_diag<T, N>(tb, cl.f[0], cl.stan, cl.vol, cl.cre, hasb, cl.lc[0], i) +
           line_diag<T, N>(tb, cl.f[1], tb.w[i] * tb.w[b], cl.vol, T(0), hasb, ly, a) +
           line_diag<T, N>(tb, cl.f[2], tb.w[i] * tb.w[a], cl.vol, T(0), hasb, lz, b);
    }
    dinv[i] = TRI ? dd : T(1) / dd;  // TRI: the diagonal, factored below
  }
  T *Tf = Tf_all + (TRIC ? cw * 3 * S::N3 : 0);
  const bool lead = valid && lane == 0;
  if constexpr (TRIC) {
    // planes 3, 1, 2 of the stored entries: 1/m_k, sub_k, c_k
    if (on) {
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const int q = lpos<N>(0, i, a, b);
        Tf[q] = fdm[3 * ndof + base + q];
        Tf[S::N3 + q] = fdm[ndof + base + q];
        Tf[2 * S::N3 + q] = fdm[2 * ndof + base + q];
      }
    }
#pragma unroll
    for (int i = 0; i < N; ++i) tc[i] = tl[i] = T(0);
  } else if constexpr (TRI) {
    // Thomas factorisation of the x-line's tridiagonal: pivots
    // m_i = diag_i - sub_i c_(i-1), c_i = sup_i / m_i
    T cprev = T(0);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const T sub = (on && i > 0) ? line_entry<T, N>(tb, cl.f[0], cl.stan, cl.vol, cl.cre, hasb, cl.lc[0], i, i - 1)
                                  : T(0);
      const T sup = (on && i < N - 1)
                        ? line_entry<T, N>(tb, cl.f[0], cl.stan, cl.vol, cl.cre, hasb, cl.lc[0], i, i + 1)
                        : T(0);
      const T m = dinv[i] - sub * cprev;
      dinv[i] = T(1) / m;
      tc[i] = sup * dinv[i];
      tl[i] = sub;
      cprev = tc[i];
    }
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) tc[i] = tl[i] = T(0);
  }

  // With advection the operator of a line depends on its position.  Where
  // registers allow, the lane's three line operators of D_T (zero
  // neighbour traces) are built once as N x N matrices: column l is the
  // operator applied to the unit vector e_l.
  constexpr bool REGM = HASB && INNER != DG_INNER_FDM && INNER != DG_INNER_PMF && (sizeof(T) == 4 ? N <= 5 : N <= 4);
  T Mr[3][S::N2];
  if constexpr (REGM) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
#pragma unroll
      for (int l = 0; l < N; ++l) {
        T e[N], col[N];
#pragma unroll
        for (int i = 0; i < N; ++i) e[i] = i == l ? T(1) : T(0);
        line_apply<T, N>(tb, cl.f[k], cl.stan, cl.vol, k == 0 ? cl.cre : T(0), true, cl.lc[k], e, T(0), T(0), T(0),
                         T(0), col);
#pragma unroll
        for (int i = 0; i < N; ++i) Mr[k][i * N + l] = on ? col[i] : T(0);
      }
    }
  }
  auto dtap0 = [&](const T(&pin)[N], T(&qout)[N]) {
    if constexpr (REGM)
      dt_apply_reg<P, T>(Mr, on, pin, qout, Ps, Qy, Qz, a, b);
    else
      dt_apply<P, T, !HASB>(cl, tb, on, hasb, Ms, w3, pin, qout, Ps, Qy, Qz, a, b);
  };
  auto dtap = [&](const T(&pin)[N], T(&qout)[N]) {
    if constexpr (GLL) {
      T sp[N], dq[N];
      gll_change<T, N, false>(on, pin, sp, Ps, a, b);
      dtap0(sp, dq);
      gll_change<T, N, true>(on, dq, qout, Ps, a, b);
    } else {
      dtap0(pin, qout);
    }
  };

  // ---- inner solve D_T x = d ------------------------------------------------
  T x[N];
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] = T(0);
  int it = 0;
  T dn2 = T(0);
#pragma unroll
  for (int i = 0; i < N; ++i) dn2 += d[i] * d[i];
  dn2 = cell_sum<L>(dn2);
  const T epsT = (T)sa.eps;

  if (INNER == DG_INNER_FDM) {
    // x = (Tz Ty Tx) Lambda^-1 (Tz Ty Tx)^T d by six 1-D contractions; the
    // eigen-index of axis k replaces the node index after its forward step
    const T *Tx = Ms_all + cw * 3 * S::N2, *Ty = Tx + S::N2, *Tz = Tx + 2 * S::N2;
    T u1[N], u2[N];
    if (on) {
      contract<T, N, true>(Tx, d, u1);
#pragma unroll
      for (int i = 0; i < N; ++i) Ps[lpos<N>(0, i, a, b)] = u1[i];
    }
    __syncthreads();
    if (on) {
#pragma unroll
      for (int i = 0; i < N; ++i) u1[i] = Ps[lpos<N>(1, i, a, b)];
      contract<T, N, true>(Ty, u1, u2);
#pragma unroll
      for (int i = 0; i < N; ++i) Qy[lpos<N>(1, i, a, b)] = u2[i];
    }
    __syncthreads();
    if (on) {
#pragma unroll
      for (int i = 0; i < N; ++i) u1[i] = Qy[lpos<N>(2, i, a, b)];
      contract<T, N, true>(Tz, u1, u2);
      // z-line (x = a, y = b): eigen-indices (a, b, i)
      const T lxy = Lm[a] + Lm[N + b];
#pragma unroll
      for (int i = 0; i < N; ++i) u2[i] /= lxy + Lm[2 * N + i];
      contract<T, N, false>(Tz, u2, u1);
#pragma unroll
      for (int i = 0; i < N; ++i) Qz[lpos<N>(2, i, a, b)] = u1[i];
    }
    __syncthreads();
    if (on) {
#pragma unroll
      for (int i = 0; i < N; ++i) u1[i] = Qz[lpos<N>(1, i, a, b)];
      contract<T, N, false>(Ty, u1, u2);
#pragma unroll
      for (int i = 0; i < N; ++i) Ps[lpos<N>(1, i, a, b)] = u2[i];
    }
    __syncthreads();
    if (on) {
#pragma unroll
      for (int i = 0; i < N; ++i) u1[i] = Ps[lpos<N>(0, i, a, b)];
      contract<T, N, false>(Tx, u1, x);
    }
    it = dn2 > T(0) ? 1 : 0;
  } else if (INNER == DG_INNER_PMF) {
    // x = D_T^-1 d with the stored inverse (pmf.hip), column by column: the
    // cell's defect goes to LDS, and step J adds d_J times column J of the
    // inverse, which the cell's lanes read as one contiguous run of (p+1)^3
    // values (each lane the N entries of its x-line)
    if (on) {
#pragma unroll
      for (int i = 0; i < N; ++i) Ps[lpos<N>(0, i, a, b)] = d[i];
    }
    __syncthreads();
    if (on) {
      const T *col = fdm + (size_t)c * S::N3 * S::N3 + lpos<N>(0, 0, a, b);
#pragma unroll 4
      for (int J = 0; J < S::N3; ++J) {
        const T dj = Ps[J];
#pragma unroll
        for (int i = 0; i < N; ++i) x[i] += col[(size_t)J * S::N3 + i] * dj;
      }
    }
    it = dn2 > T(0) ? 1 : 0;
  } else if (INNER == DG_INNER_CG) {
    T r[N], z[N], p[N], q[N];
    T rho = T(0);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      r[i] = d[i];
      z[i] = r[i] * dinv[i];
      p[i] = z[i];
      rho += r[i] * z[i];
    }
    rho = cell_sum<L>(rho);
    const T tgt2 = epsT * epsT * dn2;
    bool conv = !(dn2 > T(0));
#pragma unroll 1
    while (true) {
      const bool act = !conv && it < sa.max_inner;
      if (__ballot(act) == 0) break;
      dtap(p, q);
      T pq = T(0);
#pragma unroll
      for (int i = 0; i < N; ++i) pq += p[i] * q[i];
      pq = cell_sum<L>(pq);
      bool act2 = act;
      if (act && !(pq > T(0))) {  // breakdown: keep the iterate
        conv = true;
        act2 = false;
      }
      if (act2) {
        const T alpha = inner_div(rho, pq);
#pragma unroll
        for (int i = 0; i < N; ++i) {
          x[i] += alpha * p[i];
          r[i] -= alpha * q[i];
        }
        ++it;
      }
      T rr = T(0);
#pragma unroll
      for (int i = 0; i < N; ++i) rr += r[i] * r[i];
      rr = cell_sum<L>(rr);
      if (act2 && rr <= tgt2) conv = true;
      T rz = T(0);
#pragma unroll
      for (int i = 0; i < N; ++i) {
        z[i] = r[i] * dinv[i];
        rz += r[i] * z[i];
      }
      rz = cell_sum<L>(rz);
      if (act2 && !conv) {
        const T beta = inner_div(rz, rho);
#pragma unroll
        for (int i = 0; i < N; ++i) p[i] = z[i] + beta * p[i];
        rho = rz;
      }
    }
  } else {
    // restarted right-preconditioned GMRES
    const int R = sa.restart;
    T *Vs = Vs_all + cw * (RM + 1) * S::N3;
    T *Hs = Hs_all + cw * RM * RM;
    const int my = lane * N;  // private slot of this lane's x-line in Vs
    const T dnorm = sqrt(dn2);
    const T target = epsT * dnorm;
    bool done = !(dn2 > T(0));
    T r[N];
#pragma unroll
    for (int i = 0; i < N; ++i) r[i] = d[i];
    T beta = dnorm;
#pragma unroll 1
    while (__ballot(!done) != 0) {
      T cs[RM], sn[RM], gv[RM + 1];
#pragma unroll
      for (int j = 0; j < RM; ++j) {
        cs[j] = T(0);
        sn[j] = T(0);
        gv[j + 1] = T(0);
      }
      gv[0] = beta;
      const T ib = done ? T(0) : inner_div(T(1), beta);
      if (on) {
#pragma unroll
        for (int i = 0; i < N; ++i) Vs[my + i] = r[i] * ib;
      }
      int kk = 0;           // columns of this cycle for this cell
      bool cyc = !done;     // cell still in this cycle
      bool conv = false;
#pragma unroll 1
      for (int j = 0; j < R; ++j) {
        if (__ballot(cyc) == 0) break;
        T vj[N], w[N];
        if constexpr (TRI) {
          T vv[N];
#pragma unroll
          for (int i = 0; i < N; ++i) vv[i] = on ? Vs[j * S::N3 + my + i] : T(0);
          if constexpr (TRIC)
            tri_cell<T, N>(on, lead, vv, vj, Qy, Qz, Tf, a, b);
          else
            prec_apply<T, N, TRI>(dinv, tc, tl, vv, vj);
        } else {
#pragma unroll
          for (int i = 0; i < N; ++i) vj[i] = on ? Vs[j * S::N3 + my + i] * dinv[i] : T(0);
        }
        dtap(vj, w);
        if (cyc) ++it;
        // classical Gram-Schmidt applied twice (equal to modified
        // Gram-Schmidt in exact arithmetic, as stable in practice): the
        // projections of one pass are independent cell sums, reduced four at
        // a time so that their lane exchanges overlap
        T hcol[RM + 1];
#pragma unroll
        for (int i = 0; i <= RM; ++i) hcol[i] = T(0);
#pragma unroll
        for (int pass = 0; pass < 2; ++pass) {
          T hp[RM];
#pragma unroll
          for (int g0 = 0; g0 < RM; g0 += 4) {
            T s4[4] = {T(0), T(0), T(0), T(0)};
            if (g0 <= j) {
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const int i = g0 + q;
                if (i < RM && on && i <= j) {
#pragma unroll
                  for (int l = 0; l < N; ++l) s4[q] += w[l] * Vs[i * S::N3 + my + l];
                }
              }
#pragma unroll
              for (int q = 0; q < 4; ++q) s4[q] = cell_sum<L>(s4[q]);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
              if (g0 + q < RM) hp[g0 + q] = s4[q];
          }
#pragma unroll
          for (int i = 0; i < RM; ++i) {
            if (i <= j) {
              if (on) {
#pragma unroll
                for (int l = 0; l < N; ++l) w[l] -= hp[i] * Vs[i * S::N3 + my + l];
              }
              hcol[i] += hp[i];
            }
          }
        }
        T hn = T(0);
#pragma unroll
        for (int l = 0; l < N; ++l) hn += w[l] * w[l];
        hn = sqrt(cell_sum<L>(hn));
        // earlier rotations, then the new one
#pragma unroll
        for (int i = 0; i < RM; ++i) {
          if (i < j) {
            const T t0 = cs[i] * hcol[i] + sn[i] * hcol[i + 1];
            hcol[i + 1] = -sn[i] * hcol[i] + cs[i] * hcol[i + 1];
            hcol[i] = t0;
          }
        }
        T hj = T(0), gj = T(0);
#pragma unroll
        for (int i = 0; i < RM; ++i)
          if (i == j) {
            hj = hcol[i];
            gj = gv[i];
          }
        const T rr = sqrt(hj * hj + hn * hn);
        const T cj = inner_div(hj, rr), sj = inner_div(hn, rr);
        const T gnext = -sj * gj;
#pragma unroll
        for (int i = 0; i < RM; ++i)
          if (i == j) {
            cs[i] = cj;
            sn[i] = sj;
            hcol[i] = rr;
            gv[i] = cj * gj;
            gv[i + 1] = gnext;
          }
        if (cyc && lane == 0) {
#pragma unroll
          for (int i = 0; i < RM; ++i)
            if (i <= j) Hs[i * RM + j] = hcol[i];
        }
        if (cyc) {
          kk = j + 1;
          if (fabs(gnext) <= target || it >= sa.max_inner || !(rr > T(0))) {
            conv = fabs(gnext) <= target || !(rr > T(0));
            cyc = false;
          } else if (on) {
            const T ih = inner_div(T(1), hn);
#pragma unroll
            for (int l = 0; l < N; ++l) Vs[(j + 1) * S::N3 + my + l] = w[l] * ih;
          }
        }
      }
      __syncthreads();  // Hs written by lane 0 of each cell
      // back substitution H y = g and x += M^-1 V y (cells with kk > 0)
      T y[RM];
#pragma unroll
      for (int i = RM - 1; i >= 0; --i) {
        T s = T(0);
        if (i < kk) {
          s = gv[i];
#pragma unroll
          for (int l = 0; l < RM; ++l)
            if (l > i && l < kk) s -= Hs[i * RM + l] * y[l];
          s /= Hs[i * RM + i];
        }
        y[i] = s;
      }
      if constexpr (TRIC) {
        // x += M^-1 (V y), the whole-block band solved by all lanes together
        T vy[N], mv[N];
#pragma unroll
        for (int l = 0; l < N; ++l) vy[l] = T(0);
        if (on) {
#pragma unroll
          for (int i = 0; i < RM; ++i) {
            if (i < kk) {
#pragma unroll
              for (int l = 0; l < N; ++l) vy[l] += y[i] * Vs[i * S::N3 + my + l];
            }
          }
        }
        tri_cell<T, N>(on, lead, vy, mv, Qy, Qz, Tf, a, b);
        if (on) {
#pragma unroll
          for (int l = 0; l < N; ++l) x[l] += mv[l];
        }
      } else if (on) {
        if constexpr (TRI) {
          // x += M^-1 (V y)
          T vy[N], mv[N];
#pragma unroll
          for (int l = 0; l < N; ++l) vy[l] = T(0);
#pragma unroll
          for (int i = 0; i < RM; ++i) {
            if (i < kk) {
#pragma unroll
              for (int l = 0; l < N; ++l) vy[l] += y[i] * Vs[i * S::N3 + my + l];
            }
          }
          prec_apply<T, N, TRI>(dinv, tc, tl, vy, mv);
#pragma unroll
          for (int l = 0; l < N; ++l) x[l] += mv[l];
        } else {
#pragma unroll
          for (int i = 0; i < RM; ++i) {
            if (i < kk) {
#pragma unroll
              for (int l = 0; l < N; ++l) x[l] += dinv[l] * y[i] * Vs[i * S::N3 + my + l];
            }
          }
        }
      }
      __syncthreads();
      const bool was_active = !done;
      if (was_active && (conv || it >= sa.max_inner)) done = true;
      // restart: r = d - D_T x (all lanes take part in the transposes)
      if (__ballot(!done) != 0) {
        T dx[N];
        dtap(x, dx);
        T rn = T(0);
#pragma unroll
        for (int i = 0; i < N; ++i) {
          r[i] = d[i] - dx[i];
          rn += r[i] * r[i];
        }
        rn = sqrt(cell_sum<L>(rn));
        if (!done) {
          beta = rn;
          if (beta <= target) done = true;
        }
      }
    }
  }

  // ---- update ---------------------------------------------------------------
  // With sa.cb.part the outer iteration's dots (and, FP32, the cast back)
  // follow the update: the CastBackArgs epilogue, not built into the FP64
  // inner-GMRES sweeps, whose registers are already the tightest (see
  // smooth_takes_dots).
  constexpr bool kEpi = sizeof(T) == 4 || INNER != DG_INNER_GMRES;
  const bool epi = kEpi && sa.cb.part != nullptr;
  const bool cast_back = sizeof(T) == 4 && epi;
  double acc0 = 0.0, acc1 = 0.0;
  if (on) {
    const T om = (T)sa.omega;
    const T keep = sa.sor ? T(1) - om : T(1);
    double sc = 1.0;
    if (cast_back) {
      const double r2 = *sa.cb.rr;
      sc = r2 > 0.0 ? 1.0 / sqrt(r2) : 1.0;
      sc = 1.0 / sc;
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const T val = sa.write_du ? x[i] : keep * ul[i] + om * x[i];
      const size_t idx = base + lpos<N>(0, i, a, b);
      if (cast_back) {
        const double zi = sc * (double)val;
        sa.cb.z[idx] = zi;
        acc0 += zi * sa.cb.b0[idx];
        if (sa.cb.m > 1) acc1 += zi * sa.cb.b1[idx];
      } else {
        uout[idx] = val;
        if (epi) {
          acc0 += (double)val * sa.cb.b0[idx];
          if (sa.cb.m > 1) acc1 += (double)val * sa.cb.b1[idx];
        }
      }
    }
    if (iters && lane == 0) iters[c] = it;
  }
  if (epi) {
    // the workgroup is one wavefront: its partials by shuffles
    static_assert(kSmoothThreads == 64, "one wavefront per workgroup");
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
      acc0 += __shfl_xor(acc0, m, 64);
      acc1 += __shfl_xor(acc1, m, 64);
    }
    if (tid == 0) {
      sa.cb.part[blockIdx.x] = acc0;
      if (sa.cb.m > 1) sa.cb.part[(size_t)gridDim.x + blockIdx.x] = acc1;
    }
  }
}

}  // namespace dgmg
