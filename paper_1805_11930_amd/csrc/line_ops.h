// One-dimensional line operators from which the DG operator is built.
//
// On a Cartesian cell with diagonal, cell-constant K and the nodal
// Gauss-Legendre basis collocated with the Gauss quadrature, every term of
// the bilinear form (Sec. 2.1, eqn bilinear_form_split) acts along one
// coordinate direction at a time:
//   * volume diffusion  (K grad u, grad v)_T = sum_k K_kk/h_k^2 |T| (D^T W D)
//     along direction k, times the tangential weights w_a w_b;
//   * volume advection -(b u, grad v)_T involves only d/dx_k of the test
//     function along direction k, with b_k evaluated at the line's points;
//   * the reaction (c u, v)_T is diagonal;
//   * the faces normal to e_k couple only the line through the face point
//     (traces and normal derivatives of the nodal basis at xi_k = 0, 1).
// So A u on a cell is the sum over the three directions of a 1-D DG
// operator applied to each line of (p+1) nodes, plus couplings to the same
// line in the two neighbours along that direction.  This is the sum
// factorisation of Sec. 3.1 (Stages 1-3) specialised to this setting: the
// value interpolation is the identity, and Stage 1 / Stage 3 collapse into
// one (p+1)x(p+1) contraction per line and direction.
//
// Face terms (interior face, normal nu = +e_k from T- to T+):
//   Phi(u-,u+,b_nu)[[v]] - {K du/dnu}_omega [[v]] - {K dv/dnu}_omega [[u]]
//   + gamma_F [[u]][[v]],
// omega- = d+/(d- + d+), omega+ = d-/(d- + d+), d = K_kk, so both weighted
// fluxes carry the same coefficient kappa = d- d+ / (d- + d+); gamma_F =
// sigma <d-,d+> |F| / min|T| = 2 sigma kappa / h_k on a uniform mesh.
// A Dirichlet face (omega = 1, gamma_F = sigma d / h_k) is the same
// expression with kappa = d and a neighbour whose traces are zero; a
// Neumann face contributes nothing to A.
#pragma once

#include "dg_internal.h"

namespace dgmg {

// Face coefficients of one cell along one axis.
template <typename T>
struct AxisCoef {
  T d;        // K_kk of the cell
  T kL, gL;   // kappa and gamma_F of the face at xi_k = 0
  T kR, gR;   // ... and at xi_k = 1
  T ih;       // 1 / h_k
  int fl;     // bit 0: face at xi_k = 0 has terms; bit 1: face at xi_k = 1;
              // bit 2 / bit 3: that face is interior (a neighbour exists)
};

// Advection along one line: b_k(x) = beta + Bkk * x_k on the line.
template <typename T>
struct LineConv {
  T beta, Bkk, xk0, hk;
};

// Face coefficients along axis k from delta = K_kk on both sides of the
// lower face (own side dLo, neighbour dLn) and of the upper face (dRo,
// dRn); the neighbour values are not read where there is no neighbour.
// d is the cell's K_kk for the volume term.
template <typename T>
__host__ __device__ inline AxisCoef<T> axis_coef_faces(const Geo &g, int k, const int (&ijk)[3], double d,
                                                       double dLo, double dLn, double dRo, double dRn) {
  AxisCoef<T> f;
  const int nn[3] = {g.nx, g.ny, g.nz};
  const double ih = g.ih[k];
  double kL = 0.0, gL = 0.0, kR = 0.0, gR = 0.0;
  int fl = 0;
  if (ijk[k] > 0) {
    kL = dLo * dLn / (dLo + dLn);
    gL = 2.0 * g.sigma * kL * ih;
    fl |= 1 | 4;
  } else if (g.bc[2 * k] == FACE_DIRICHLET) {
    kL = dLo;
    gL = g.sigma * dLo * ih;
    fl |= 1;
  }
  if (ijk[k] < nn[k] - 1) {
    kR = dRo * dRn / (dRo + dRn);
    gR = 2.0 * g.sigma * kR * ih;
    fl |= 2 | 8;
  } else if (g.bc[2 * k + 1] == FACE_DIRICHLET) {
    kR = dRo;
    gR = g.sigma * dRo * ih;
    fl |= 2;
  }
  f.d = (T)d;
  f.kL = (T)kL;
  f.gL = (T)gL;
  f.kR = (T)kR;
  f.gR = (T)gR;
  f.ih = (T)ih;
  f.fl = fl;
  return f;
}

// Face coefficients from K_kk of the cell (d) and of its neighbours below
// and above along k (dm, dp; not read where there is no neighbour).
template <typename T>
__host__ __device__ inline AxisCoef<T> axis_coef_from(const Geo &g, int k, const int (&ijk)[3], double d, double dm,
                                                      double dp) {
  return axis_coef_faces<T>(g, k, ijk, d, d, dm, d, dp);
}

// axis_coef_from with the axis k a per-lane value: the per-axis mesh data
// are selected instead of branched on, so lanes of different axes take one
// path (same arithmetic, same results).
template <typename T>
__host__ __device__ inline AxisCoef<T> axis_coef_lane(const Geo &g, int k, const int (&ijk)[3], double d, double dm,
                                                      double dp) {
  const int ik = k == 0 ? ijk[0] : (k == 1 ? ijk[1] : ijk[2]);
  const int nk = k == 0 ? g.nx : (k == 1 ? g.ny : g.nz);
  const double ih = k == 0 ? g.ih[0] : (k == 1 ? g.ih[1] : g.ih[2]);
  const bool dirL = (k == 0 ? g.bc[0] : (k == 1 ? g.bc[2] : g.bc[4])) == FACE_DIRICHLET;
  const bool dirR = (k == 0 ? g.bc[1] : (k == 1 ? g.bc[3] : g.bc[5])) == FACE_DIRICHLET;
  const bool inL = ik > 0, inR = ik < nk - 1;
  const double hL = d * dm / (d + dm), hR = d * dp / (d + dp);
  const double kL = inL ? hL : (dirL ? d : 0.0);
  const double gL = inL ? 2.0 * g.sigma * hL * ih : (dirL ? g.sigma * d * ih : 0.0);
  const double kR = inR ? hR : (dirR ? d : 0.0);
  const double gR = inR ? 2.0 * g.sigma * hR * ih : (dirR ? g.sigma * d * ih : 0.0);
  AxisCoef<T> f;
  f.d = (T)d;
  f.kL = (T)kL;
  f.gL = (T)gL;
  f.kR = (T)kR;
  f.gR = (T)gR;
  f.ih = (T)ih;
  f.fl = (inL ? 5 : (dirL ? 1 : 0)) | (inR ? 10 : (dirR ? 2 : 0));
  return f;
}

// Face coefficients of the coefficient field along axis k: K_kk = P_k(x_k)
// is constant on a face normal to e_k and the same from both sides; the
// volume part (d = 0 here) is added by line_volume_field.
template <typename T>
__host__ __device__ inline AxisCoef<T> axis_coef_field(const Geo &g, int k, const int (&ijk)[3]) {
  const double pl = field_K(g, k, ijk[k] * g.h[k]);
  const double pr = field_K(g, k, (ijk[k] + 1) * g.h[k]);
  return axis_coef_faces<T>(g, k, ijk, 0.0, pl, pl, pr, pr);
}

// Volume diffusion along one line with K_kk varying along it (sum
// factorisation in three steps: derivative at the quadrature points,
// scaling by w_q K_kk(x_q), transposed derivative):
//   v_i += stan vol / h^2 sum_q D[q][i] w_q pk[q] sum_l D[q][l] u_l,
// pk[q] = K_kk at the q-th node of the line.
template <typename T, int N>
__host__ __device__ inline void line_volume_field(const DevTab<T, N> &tb, T stan, T vol, T ih, const T (&pk)[N],
                                                  const T (&u)[N], T (&v)[N]) {
  T gq[N];
#pragma unroll
  for (int q = 0; q < N; ++q) {
    T acc = T(0);
#pragma unroll
    for (int l = 0; l < N; ++l) acc += tb.Dt[l][q] * u[l];
    gq[q] = acc * tb.w[q] * pk[q];
  }
  const T alpha = stan * vol * ih * ih;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T acc = T(0);
#pragma unroll
    for (int q = 0; q < N; ++q) acc += tb.Dt[i][q] * gq[q];
    v[i] += alpha * acc;
  }
}

template <typename T>
__host__ __device__ inline AxisCoef<T> make_axis_coef(const Geo &g, int cell, int k, const int (&ijk)[3]) {
  const int nn[3] = {g.nx, g.ny, g.nz};
  const int stride[3] = {1, g.nx, g.nx * g.ny};
  const double d = g.K[3 * cell + k];
  const double dm = ijk[k] > 0 ? g.K[3 * (cell - stride[k]) + k] : d;
  const double dp = ijk[k] < nn[k] - 1 ? g.K[3 * (cell + stride[k]) + k] : d;
  return axis_coef_from<T>(g, k, ijk, d, dm, dp);
}

// Cell coordinates (ix, iy, iz) of cell c.
__host__ __device__ inline void cell_coords(const Geo &g, int c, int (&ijk)[3]) {
  const int iz = fdiv(c, g.fxy);
  const int rem = c - iz * (g.nx * g.ny);
  const int iy = fdiv(rem, g.fx);
  ijk[0] = rem - iy * g.nx;
  ijk[1] = iy;
  ijk[2] = iz;
}

// Advection data of the line along axis k through cell ijk with tangential
// node indices (ta, tb_) on the two other axes (in increasing axis order).
template <typename T, int N>
__host__ __device__ inline LineConv<T> make_line_conv(const Geo &g, const DevTab<T, N> &tb, int k, const int (&ijk)[3],
                                                      int ta, int tb_) {
  const int t1 = (k == 0) ? 1 : 0;
  const int t2 = (k == 2) ? 1 : 2;
  const double x1 = (ijk[t1] + (double)tb.xi[ta]) * g.h[t1];
  const double x2 = (ijk[t2] + (double)tb.xi[tb_]) * g.h[t2];
  LineConv<T> lc;
  lc.beta = (T)(g.b0[k] + g.B[3 * k + t1] * x1 + g.B[3 * k + t2] * x2);
  lc.Bkk = (T)g.B[3 * k + k];
  lc.xk0 = (T)(ijk[k] * g.h[k]);
  lc.hk = (T)g.h[k];
  return lc;
}

// v = (1-D operator along the line) u, scaled by the tangential weight
// product stan.  Neighbour traces: tLu = e1.uL, tLd = d1.uL (left neighbour
// at its face xi_k = 1), tRu = e0.uR, tRd = d0.uR (right neighbour).  For
// the block diagonal D_T, and on Dirichlet faces, they are zero.  cre is
// the reaction coefficient (added on one axis only).
template <typename T, int N>
__host__ __device__ inline void line_apply(const DevTab<T, N> &tb, const AxisCoef<T> &f, T stan, T vol, T cre,
                                           bool hasb, const LineConv<T> &lc, const T (&u)[N], T tLu, T tLd, T tRu,
                                           T tRd, T (&v)[N]) {
  const T ih = f.ih;
  const T alpha = stan * vol * f.d * ih * ih;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T acc = T(0);
#pragma unroll
    for (int l = 0; l < N; ++l) acc += tb.S[i][l] * u[l];
    v[i] = alpha * acc;
  }
  if (cre != T(0)) {
    const T rc = cre * vol * stan;
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += rc * tb.w[i] * u[i];
  }
  if (hasb) {
    const T coef = -stan * vol * ih;
    T bu[N];
#pragma unroll
    for (int q = 0; q < N; ++q) bu[q] = tb.w[q] * (lc.beta + lc.Bkk * (lc.xk0 + tb.xi[q] * lc.hk)) * u[q];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      T acc = T(0);
#pragma unroll
      for (int q = 0; q < N; ++q) acc += tb.Dt[i][q] * bu[q];
      v[i] += coef * acc;
    }
  }
  const T WF = stan * vol * ih;
  if (f.fl & 2) {
    T uM = T(0), gM = T(0);
#pragma unroll
    for (int l = 0; l < N; ++l) {
      uM += tb.e1[l] * u[l];
      gM += tb.d1[l] * u[l];
    }
    const T jump = uM - tRu;
    T s = -f.kR * (gM + tRd) * ih + f.gR * jump;
    if (hasb) {
      const T bnu = lc.beta + lc.Bkk * (lc.xk0 + lc.hk);
      s += bnu >= T(0) ? bnu * uM : bnu * tRu;
    }
    s *= WF;
    const T t = -WF * f.kR * jump * ih;
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += s * tb.e1[i] + t * tb.d1[i];
  }
  if (f.fl & 1) {
    T uP = T(0), gP = T(0);
#pragma unroll
    for (int l = 0; l < N; ++l) {
      uP += tb.e0[l] * u[l];
      gP += tb.d0[l] * u[l];
    }
    const T jump = tLu - uP;
    T s = -f.kL * (tLd + gP) * ih + f.gL * jump;
    if (hasb) {
      const T bk = lc.beta + lc.Bkk * lc.xk0;
      s += bk >= T(0) ? bk * tLu : bk * uP;
    }
    s *= -WF;
    const T t = -WF * f.kL * jump * ih;
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += s * tb.e0[i] + t * tb.d0[i];
  }
}

// line_apply for b = 0 in the even-odd form (EoTab): the same operator with
// about half the multiply-adds and table values.  REACT: add the reaction
// term cre (w_i u_i) (only the x line of a cell carries it).
template <typename T, int N, bool REACT>
__host__ __device__ inline void line_apply_eo(const AxisCoef<T> &f, T stan, T vol, T cre, const T (&u)[N], T tLu,
                                              T tLd, T tRu, T tRd, T (&v)[N]) {
  constexpr EoTab<T, N> et = make_eotab<T, N>();
  constexpr int M = N / 2, O = N % 2, ME = M + O;
  T ue[ME], uo[M];
#pragma unroll
  for (int l = 0; l < M; ++l) {
    ue[l] = u[l] + u[N - 1 - l];
    uo[l] = u[l] - u[N - 1 - l];
  }
  if constexpr (O) ue[M] = u[M];
  // own traces: e0.u = Pe + Po, e1.u = Pe - Po, d0.u = Qe + Qo, d1.u = Qo - Qe
  T Pe = T(0), Po = T(0), Qe = T(0), Qo = T(0);
#pragma unroll
  for (int l = 0; l < ME; ++l) {
    Pe += et.ee[l] * ue[l];
    Qe += et.de[l] * ue[l];
  }
#pragma unroll
  for (int l = 0; l < M; ++l) {
    Po += et.eo[l] * uo[l];
    Qo += et.dd[l] * uo[l];
  }
  const T uP = Pe + Po, uM = Pe - Po, gP = Qe + Qo, gM = Qo - Qe;
  const T ih = f.ih;
  const T WF = stan * vol * ih;
  const T alpha = WF * f.d * ih;
  // face terms as v += s0 e0 + t0 d0 (face xi = 0) + s1 e1 + t1 d1 (xi = 1)
  const T jR = uM - tRu;
  const T sR = WF * (f.gR * jR - f.kR * (gM + tRd) * ih);
  const T tR = -WF * f.kR * jR * ih;
  const T jL = tLu - uP;
  const T sL = -WF * (f.gL * jL - f.kL * (tLd + gP) * ih);
  const T tL = -WF * f.kL * jL * ih;
  const T s1 = (f.fl & 2) ? sR : T(0), t1 = (f.fl & 2) ? tR : T(0);
  const T s0 = (f.fl & 1) ? sL : T(0), t0 = (f.fl & 1) ? tL : T(0);
  const T se = s0 + s1, so = s0 - s1, te = t0 - t1, to = t0 + t1;
  T ve[ME], vo[M];
#pragma unroll
  for (int i = 0; i < M; ++i) {
    T ae = T(0), ao = T(0);
#pragma unroll
    for (int l = 0; l < ME; ++l) ae += et.Se[i][l] * ue[l];
#pragma unroll
    for (int l = 0; l < M; ++l) ao += et.So[i][l] * uo[l];
    ve[i] = alpha * ae + se * et.ee[i] + te * et.de[i];
    vo[i] = alpha * ao + so * et.eo[i] + to * et.dd[i];
  }
  if constexpr (O) {
    T am = T(0);
#pragma unroll
    for (int l = 0; l < ME; ++l) am += et.Sm[l] * ue[l];
    ve[M] = alpha * am + se * et.ee[M] + te * et.de[M];
  }
  if constexpr (REACT) {
    const T rc = cre * vol * stan;
#pragma unroll
    for (int i = 0; i < M; ++i) {
      ve[i] += rc * et.wh[i] * ue[i];
      vo[i] += rc * et.wh[i] * uo[i];
    }
    if constexpr (O) ve[M] += rc * et.wh[M] * ue[M];
  }
#pragma unroll
  for (int i = 0; i < M; ++i) {
    v[i] = ve[i] + vo[i];
    v[N - 1 - i] = ve[i] - vo[i];
  }
  if constexpr (O) v[M] = ve[M];
}

// Diagonal entry i of the line operator without neighbour couplings
// (line_apply with u = unit vector e_i and zero neighbour traces).
template <typename T, int N>
__host__ __device__ inline T line_diag(const DevTab<T, N> &tb, const AxisCoef<T> &f, T stan, T vol, T cre, bool hasb,
                                       const LineConv<T> &lc, int i) {
  const T ih = f.ih;
  T d = stan * vol * f.d * ih * ih * tb.S[i][i] + cre * vol * stan * tb.w[i];
  if (hasb) d += -stan * vol * ih * tb.Dt[i][i] * tb.w[i] * (lc.beta + lc.Bkk * (lc.xk0 + tb.xi[i] * lc.hk));
  const T WF = stan * vol * ih;
  if (f.fl & 2) {
    const T uM = tb.e1[i], gM = tb.d1[i];
    T s = -f.kR * gM * ih + f.gR * uM;
    if (hasb) {
      const T bnu = lc.beta + lc.Bkk * (lc.xk0 + lc.hk);
      s += bnu >= T(0) ? bnu * uM : T(0);
    }
    const T t = -f.kR * uM * ih;
    d += WF * (s * tb.e1[i] + t * tb.d1[i]);
  }
  if (f.fl & 1) {
    const T uP = tb.e0[i], gP = tb.d0[i];
    T s = -f.kL * gP * ih - f.gL * uP;
    if (hasb) {
      const T bk = lc.beta + lc.Bkk * lc.xk0;
      s += bk >= T(0) ? T(0) : bk * uP;
    }
    const T t = f.kL * uP * ih;
    d += -WF * s * tb.e0[i] + WF * t * tb.d0[i];
  }
  return d;
}

// Entry (i, l) of the line operator without neighbour couplings: component
// i of line_apply applied to the unit vector e_l with zero neighbour traces.
template <typename T, int N>
__host__ __device__ inline T line_entry(const DevTab<T, N> &tb, const AxisCoef<T> &f, T stan, T vol, T cre, bool hasb,
                                        const LineConv<T> &lc, int i, int l) {
  const T ih = f.ih;
  T m = stan * vol * f.d * ih * ih * tb.S[i][l];
  if (i == l) m += cre * vol * stan * tb.w[i];
  if (hasb) m += -stan * vol * ih * tb.Dt[i][l] * tb.w[l] * (lc.beta + lc.Bkk * (lc.xk0 + tb.xi[l] * lc.hk));
  const T WF = stan * vol * ih;
  if (f.fl & 2) {
    const T uM = tb.e1[l], gM = tb.d1[l];
    T s = -f.kR * gM * ih + f.gR * uM;
    if (hasb) {
      const T bnu = lc.beta + lc.Bkk * (lc.xk0 + lc.hk);
      s += bnu >= T(0) ? bnu * uM : T(0);
    }
    m += WF * (s * tb.e1[i] - f.kR * uM * ih * tb.d1[i]);
  }
  if (f.fl & 1) {
    const T uP = tb.e0[l], gP = tb.d0[l];
    T s = -f.kL * gP * ih - f.gL * uP;
    if (hasb) {
      const T bk = lc.beta + lc.Bkk * lc.xk0;
      s += bk >= T(0) ? T(0) : bk * uP;
    }
    m += -WF * s * tb.e0[i] + WF * f.kL * uP * ih * tb.d0[i];
  }
  return m;
}

// Entry (i, l) of the 1-D block operator along one axis for b = 0, without
// the tangential weight factor: the line part of D_T is stan * M u with
//   M = vol [ d/h^2 S + (1/h) (face at xi=1) + (1/h) (face at xi=0) ]
//       (+ c vol diag(w) on the axis that carries the reaction),
// i.e. line_apply with zero neighbour traces written as a matrix.  D_T is
// then the Kronecker sum  Mx (x) Wy (x) Wz + Wx (x) My (x) Wz + Wx (x) Wy (x) Mz
// with W = diag(w).
template <typename T, int N>
__host__ __device__ inline T line_matrix_entry(const DevTab<T, N> &tb, const AxisCoef<T> &f, T vol, T cre, int i,
                                               int l) {
  const T ih = f.ih;
  T m = f.d * ih * ih * tb.S[i][l];
  if (f.fl & 2) m += ih * (tb.e1[i] * (f.gR * tb.e1[l] - f.kR * ih * tb.d1[l]) - f.kR * ih * tb.d1[i] * tb.e1[l]);
  if (f.fl & 1) m += ih * (tb.e0[i] * (f.gL * tb.e0[l] + f.kL * ih * tb.d0[l]) + f.kL * ih * tb.d0[i] * tb.e0[l]);
  m *= vol;
  if (i == l) m += cre * vol * tb.w[i];
  return m;
}

}  // namespace dgmg
