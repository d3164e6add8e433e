// Outer operator v = A u for a full-tensor coefficient field
// K(x) = sum_m P_m(x_m) n_m n_m^T (Sec. 4.2, second diffusion test, with a
// rotated orthonormal basis n_m), K and c evaluated at the quadrature
// points (= nodes) of every cell and face.
//
// With off-diagonal K the volume term couples derivatives in different
// directions and the face fluxes nu . K grad u need the tangential
// derivatives of the traces, so the operator is no longer a sum of 1-D line
// operators.  It is applied by sum factorisation in the paper's three
// stages (Sec. 3.1), each stage on lines through LDS:
//   volume: g_l = d_l u at every node (one contraction per direction),
//           F_k = W sum_l K_kl g_l pointwise,
//           v += sum_k D_k^T F_k (one transposed contraction per direction);
//   faces normal to e_k, per face point (a, b) of the lane's k-line:
//           traces u-, u+ and normal derivatives along the line; tangential
//           derivatives of the traces from the neighbouring lines of the
//           face (LDS); consistency, symmetry and penalty terms with
//           omega = 1/2 and gamma_F = sigma K_kk / h_k (the field is
//           continuous, so delta- = delta+ = K_kk(x)); the tangential part
//           of nu . K grad v is a transposed tangential derivative of the
//           coefficient field, again through LDS.
// Advection and reaction act along lines as in the other operators
// (line_apply with the diffusion coefficients set to zero).
//
// Mapping: 256-lane workgroups of CPB = floor(256 / (p+1)^2) consecutive
// cells; lane (cell, a, b) owns line (a, b) in each of the three
// directions, as in k_apply.  This kernel serves the less common rotated
// field; it trades occupancy (about 40 KB of LDS per workgroup at p = 4)
// for simple, barrier-separated phases.
#include "line_ops.h"

namespace dgmg {

namespace {

constexpr int kTThreads = 256;

template <int N>
__device__ inline int tpos(int k, int i, int a, int b) {
  return k == 0 ? i + N * a + N * N * b : (k == 1 ? a + N * i + N * N * b : a + N * b + N * N * i);
}

template <int P, typename T>
__global__ __launch_bounds__(kTThreads) void k_apply_tensor(Geo g, const T *__restrict__ u, T *__restrict__ v) {
  constexpr int N = P + 1, N2 = N * N, N3 = N2 * N, CPB = kTThreads / N2;
  constexpr DevTab<T, N> tb = make_ctab<T, N>();
  __shared__ T us[(CPB + 2) * N3];  // the cells and one x-neighbour on either side
  constexpr int GS = 3 * N3 >= N3 + 8 * N2 ? 3 * CPB * N3 : CPB * (N3 + 8 * N2);
  __shared__ T Gs[GS];  // gradient, then flux; later the y/z sums and the face fields
  T *qs = Gs;           // y / z contributions (after the volume stages)
  T *FT = Gs + CPB * N3;      // four face trace fields
  T *FC = FT + 4 * CPB * N2;  // four face coefficient fields

  const int c0 = blockIdx.x * CPB;
  const int tid = threadIdx.x;
  const int cl = tid / N2;
  const int ln = tid - cl * N2;
  const int a = ln % N, b = ln / N;
  const int ncb = min(CPB, g.ncell - c0);
  const bool active = cl < ncb;
  const int c = c0 + cl;
  int ijk[3] = {0, 0, 0};
  if (active) cell_coords(g, c, ijk);
  const int nn[3] = {g.nx, g.ny, g.nz};

  // ---- loads --------------------------------------------------------------
  const int64_t ndof = (int64_t)g.ncell * N3;
  const int64_t e_first = (int64_t)(c0 - 1) * N3;
  for (int e = tid; e < (CPB + 2) * N3; e += kTThreads) {
    const int64_t ge = e_first + e;
    us[e] = (ge >= 0 && ge < ndof) ? u[ge] : T(0);
  }
  T yl[N], yr[N], zl[N], zr[N];
  {
    const int sy = g.nx, sz = g.nx * g.ny;
    const int cc = active ? c : 0;
    const T *pyl = u + (size_t)(active && ijk[1] > 0 ? cc - sy : cc) * N3;
    const T *pyr = u + (size_t)(active && ijk[1] < g.ny - 1 ? cc + sy : cc) * N3;
    const T *pzl = u + (size_t)(active && ijk[2] > 0 ? cc - sz : cc) * N3;
    const T *pzr = u + (size_t)(active && ijk[2] < g.nz - 1 ? cc + sz : cc) * N3;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      yl[i] = pyl[tpos<N>(1, i, a, b)];
      yr[i] = pyr[tpos<N>(1, i, a, b)];
      zl[i] = pzl[tpos<N>(2, i, a, b)];
      zr[i] = pzr[tpos<N>(2, i, a, b)];
    }
  }
  __syncthreads();

  const T *own = us + (cl + 1) * N3;
  const T vol = (T)g.vol;
  const T stan = tb.w[a] * tb.w[b];
  const bool hasb = g.has_b != 0;
  T out[3][N];
  // neighbour traces per direction: (e1 . lower line, d1 . lower line,
  // e0 . upper line, d0 . upper line), zero where there is no neighbour
  T tr[3][4];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T lo[N], hi[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      if (k == 0) {
        lo[i] = active ? own[tpos<N>(0, i, a, b) - N3] : T(0);
        hi[i] = active ? own[tpos<N>(0, i, a, b) + N3] : T(0);
      } else {
        lo[i] = k == 1 ? yl[i] : zl[i];
        hi[i] = k == 1 ? yr[i] : zr[i];
      }
    }
    T t0 = T(0), t1 = T(0), t2 = T(0), t3 = T(0);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      t0 += tb.e1[i] * lo[i];
      t1 += tb.d1[i] * lo[i];
      t2 += tb.e0[i] * hi[i];
      t3 += tb.d0[i] * hi[i];
    }
    if (ijk[k] == 0) t0 = t1 = T(0);
    if (ijk[k] == nn[k] - 1) t2 = t3 = T(0);
    tr[k][0] = t0;
    tr[k][1] = t1;
    tr[k][2] = t2;
    tr[k][3] = t3;
  }

  // ---- advection and reaction along lines, volume stage 1 -----------------
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T ul[N];
#pragma unroll
    for (int i = 0; i < N; ++i) ul[i] = active ? own[tpos<N>(k, i, a, b)] : T(0);
#pragma unroll
    for (int i = 0; i < N; ++i) out[k][i] = T(0);
    if (hasb && active) {
      AxisCoef<T> f;  // face presence only: no diffusion terms
      f.d = f.kL = f.gL = f.kR = f.gR = T(0);
      f.ih = (T)g.ih[k];
      f.fl = ((ijk[k] > 0 || g.bc[2 * k] == FACE_DIRICHLET) ? 1 : 0) |
             ((ijk[k] < nn[k] - 1 || g.bc[2 * k + 1] == FACE_DIRICHLET) ? 2 : 0);
      const LineConv<T> lc = make_line_conv<T, N>(g, tb, k, ijk, a, b);
      line_apply<T, N>(tb, f, stan, vol, T(0), true, lc, ul, tr[k][0], tr[k][1], tr[k][2], tr[k][3], out[k]);
    }
    if (k == 0 && g.has_c && active) {
      const double y = (ijk[1] + (double)tb.xi[a]) * g.h[1], z = (ijk[2] + (double)tb.xi[b]) * g.h[2];
#pragma unroll
      for (int i = 0; i < N; ++i)
        out[0][i] += (T)field_c(g, (ijk[0] + (double)tb.xi[i]) * g.h[0], y, z) * vol * stan * tb.w[i] * ul[i];
    }
    // gradient component k at the line's nodes
    if (active) {
      const T ih = (T)g.ih[k];
#pragma unroll
      for (int q = 0; q < N; ++q) {
        T s = T(0);
#pragma unroll
        for (int j = 0; j < N; ++j) s += tb.Dt[j][q] * ul[j];
        Gs[k * CPB * N3 + cl * N3 + tpos<N>(k, q, a, b)] = ih * s;
      }
    }
  }
  __syncthreads();

  // ---- volume stage 2: F = W K(x) g at the nodes of the lane's x-line ------
  if (active) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const int p0 = cl * N3 + tpos<N>(0, i, a, b);
      const double x[3] = {(ijk[0] + (double)tb.xi[i]) * g.h[0], (ijk[1] + (double)tb.xi[a]) * g.h[1],
                           (ijk[2] + (double)tb.xi[b]) * g.h[2]};
      double K[3][3];
      field_tensor(g, x, K);
      const T gv[3] = {Gs[p0], Gs[CPB * N3 + p0], Gs[2 * CPB * N3 + p0]};
      const T W = vol * stan * tb.w[i];
#pragma unroll
      for (int k = 0; k < 3; ++k)
        Gs[k * CPB * N3 + p0] = W * ((T)K[k][0] * gv[0] + (T)K[k][1] * gv[1] + (T)K[k][2] * gv[2]);
    }
  }
  __syncthreads();

  // ---- volume stage 3: v += D_k^T F_k along each direction ------------------
  if (active) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      T F[N];
#pragma unroll
      for (int q = 0; q < N; ++q) F[q] = Gs[k * CPB * N3 + cl * N3 + tpos<N>(k, q, a, b)];
      const T ih = (T)g.ih[k];
#pragma unroll
      for (int i = 0; i < N; ++i) {
        T s = T(0);
#pragma unroll
        for (int q = 0; q < N; ++q) s += tb.Dt[i][q] * F[q];
        out[k][i] += ih * s;
      }
    }
  }
  __syncthreads();  // Gs is reused for the face fields

  // ---- faces normal to e_k ---------------------------------------------------
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int t1 = (k == 0) ? 1 : 0, t2 = (k == 2) ? 1 : 2;
    const T ih = (T)g.ih[k];
    T ul[N];
#pragma unroll
    for (int i = 0; i < N; ++i) ul[i] = active ? own[tpos<N>(k, i, a, b)] : T(0);
    T uoL = T(0), uoR = T(0), doL = T(0), doR = T(0);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      uoL += tb.e0[i] * ul[i];
      uoR += tb.e1[i] * ul[i];
      doL += tb.d0[i] * ul[i];
      doR += tb.d1[i] * ul[i];
    }
    doL *= ih;
    doR *= ih;
    const T unL = tr[k][0], dnL = ih * tr[k][1], unR = tr[k][2], dnR = ih * tr[k][3];
    const int fp = cl * N2 + a + N * b;  // face point (a, b) of the cell
    if (active) {
      FT[fp] = uoL;
      FT[CPB * N2 + fp] = unL;
      FT[2 * CPB * N2 + fp] = uoR;
      FT[3 * CPB * N2 + fp] = unR;
    }
    __syncthreads();
    T cf[4] = {T(0), T(0), T(0), T(0)};  // tangential coefficient fields (L t1, L t2, R t1, R t2)
    if (active) {
      // tangential derivatives of the four trace fields at (a, b)
      T dt[4][2];
      const T ih1 = (T)g.ih[t1], ih2 = (T)g.ih[t2];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const T *Fm = FT + m * CPB * N2 + cl * N2;
        T s1 = T(0), s2 = T(0);
#pragma unroll
        for (int j = 0; j < N; ++j) {
          s1 += tb.Dt[j][a] * Fm[j + N * b];
          s2 += tb.Dt[j][b] * Fm[a + N * j];
        }
        dt[m][0] = ih1 * s1;
        dt[m][1] = ih2 * s2;
      }
      const T WF = stan * vol * ih;
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        const bool interior = side ? (ijk[k] < nn[k] - 1) : (ijk[k] > 0);
        const bool dirichlet = !interior && g.bc[2 * k + side] == FACE_DIRICHLET;
        if (!interior && !dirichlet) continue;
        double x[3];
        x[k] = (ijk[k] + side) * g.h[k];
        x[t1] = (ijk[t1] + (double)tb.xi[a]) * g.h[t1];
        x[t2] = (ijk[t2] + (double)tb.xi[b]) * g.h[t2];
        double Kd[3][3];
        field_tensor(g, x, Kd);
        const T Kkk = (T)Kd[k][k], Kk1 = (T)Kd[k][t1], Kk2 = (T)Kd[k][t2];
        const T gam = (T)g.sigma * Kkk * ih;
        // own trace / gradient and neighbour trace / gradient on this face
        const T uo = side ? uoR : uoL, dno = side ? doR : doL;
        const T d1o = dt[side ? 2 : 0][0], d2o = dt[side ? 2 : 0][1];
        const T flux_o = Kkk * dno + Kk1 * d1o + Kk2 * d2o;  // e_k . K grad u (own)
        T se, sd;  // coefficients of e_own[i] and of ih d_own[i] on the own line
        T ct1, ct2;
        if (interior) {
          const T un = side ? unR : unL, dnn = side ? dnR : dnL;
          const T d1n = dt[side ? 3 : 1][0], d2n = dt[side ? 3 : 1][1];
          const T flux_n = Kkk * dnn + Kk1 * d1n + Kk2 * d2n;
          // lower (-) / upper (+) cells of the face: own is - on the upper face
          const T jump = side ? (uo - un) : (un - uo);
          const T sg = side ? T(1) : T(-1);  // [[psi_i]] = sg * trace of psi_i
          const T avg = T(0.5) * (flux_o + flux_n);
          se = WF * sg * (gam * jump - avg);
          sd = -WF * T(0.5) * Kkk * jump;
          ct1 = -WF * T(0.5) * Kk1 * jump;
          ct2 = -WF * T(0.5) * Kk2 * jump;
        } else {
          // Dirichlet: outward normal nu_k = -1 (lower face) or +1 (upper)
          const T nu = side ? T(1) : T(-1);
          se = WF * (gam * uo - nu * flux_o);
          sd = -WF * nu * Kkk * uo;
          ct1 = -WF * nu * Kk1 * uo;
          ct2 = -WF * nu * Kk2 * uo;
        }
#pragma unroll
        for (int i = 0; i < N; ++i)
          out[k][i] += side ? (se * tb.e1[i] + sd * ih * tb.d1[i]) : (se * tb.e0[i] + sd * ih * tb.d0[i]);
        cf[2 * side] = ct1;
        cf[2 * side + 1] = ct2;
      }
      FC[fp] = cf[0];
      FC[CPB * N2 + fp] = cf[1];
      FC[2 * CPB * N2 + fp] = cf[2];
      FC[3 * CPB * N2 + fp] = cf[3];
    }
    __syncthreads();
    if (active) {
      // transposed tangential derivatives of the coefficient fields, lifted
      // onto the line by the traces of the own basis
      const T ih1 = (T)g.ih[t1], ih2 = (T)g.ih[t2];
      T s[2];
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        const T *F1 = FC + (2 * side) * CPB * N2 + cl * N2;
        const T *F2 = FC + (2 * side + 1) * CPB * N2 + cl * N2;
        T s1 = T(0), s2 = T(0);
#pragma unroll
        for (int j = 0; j < N; ++j) {
          s1 += tb.Dt[a][j] * F1[j + N * b];
          s2 += tb.Dt[b][j] * F2[a + N * j];
        }
        s[side] = ih1 * s1 + ih2 * s2;
      }
#pragma unroll
      for (int i = 0; i < N; ++i) out[k][i] += s[0] * tb.e0[i] + s[1] * tb.e1[i];
    }
    __syncthreads();
  }

  // ---- sum the three directions and store -----------------------------------
  if (active) {
#pragma unroll
    for (int i = 0; i < N; ++i) qs[cl * N3 + tpos<N>(1, i, a, b)] = out[1][i];
  }
  __syncthreads();
  if (active) {
#pragma unroll
    for (int i = 0; i < N; ++i) qs[cl * N3 + tpos<N>(2, i, a, b)] += out[2][i];
  }
  __syncthreads();
  if (active) {
    T *vb = v + (size_t)c * N3 + N * a + N2 * b;
#pragma unroll
    for (int i = 0; i < N; ++i) vb[i] = out[0][i] + qs[cl * N3 + tpos<N>(0, i, a, b)];
  }
}

template <int P, typename T>
int launch_t(const dg_problem *pr, const void *u, void *v, hipStream_t s) {
  constexpr int N = P + 1, CPB = kTThreads / (N * N);
  const int G = (int)((pr->ncell + CPB - 1) / CPB);
  hipLaunchKernelGGL((k_apply_tensor<P, T>), dim3(G), dim3(kTThreads), 0, s, pr->geo, (const T *)u, (T *)v);
  DG_HIP(hipGetLastError());
  return DG_OK;
}

}  // namespace

int launch_apply_tensor(const dg_problem *pr, int prec, const void *u, void *v, hipStream_t s) {
  const bool d = prec == DG_FP64;
  switch (pr->p) {
    case 1: return d ? launch_t<1, double>(pr, u, v, s) : launch_t<1, float>(pr, u, v, s);
    case 2: return d ? launch_t<2, double>(pr, u, v, s) : launch_t<2, float>(pr, u, v, s);
    case 3: return d ? launch_t<3, double>(pr, u, v, s) : launch_t<3, float>(pr, u, v, s);
    case 4: return d ? launch_t<4, double>(pr, u, v, s) : launch_t<4, float>(pr, u, v, s);
    case 5: return d ? launch_t<5, double>(pr, u, v, s) : launch_t<5, float>(pr, u, v, s);
  }
  set_error("unsupported degree");
  return DG_EINVAL;
}

}  // namespace dgmg
