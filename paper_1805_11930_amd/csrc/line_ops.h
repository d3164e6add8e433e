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
// omega- = d+/(d- + d+), omega+ = d-/(d- + d+), d = K_kk,
// gamma_F = sigma <d-,d+> |F| / min|T| with <a,b> = 2ab/(a+b) and
// |F|/|T| = 1/h_k on a uniform mesh; Dirichlet faces take omega = 1 and
// gamma_F = sigma d |F|/|T|; Neumann faces contribute nothing to A.
#pragma once

#include "dg_internal.h"

namespace dgmg {

template <typename T>
struct LineCtx {
  T stan;     // product of the tangential Gauss weights of the line
  T hk;       // cell size along the line
  T vol;      // cell volume
  T delta;    // K_kk of the cell
  T dL, dR;   // K_kk of the neighbours (interior faces only)
  T sigma;    // penalty prefactor
  T cre;      // reaction coefficient added on this line (0 except one axis)
  T beta;     // b_k on the line, without its x_k part
  T Bkk;      // d b_k / d x_k
  T xk0;      // cell origin along the line
  int left, right;  // FaceKind of the faces at xi_k = 0 and xi_k = 1
};

// v = (1-D operator along the line) u.  Neighbour traces enter through
// four numbers: tLu = e1.uL, tLd = d1.uL (left neighbour, its face at
// xi_k = 1) and tRu = e0.uR, tRd = d0.uR (right neighbour).  For the block
// diagonal D_T these are zero while the face stays interior.
template <typename T, int N>
__host__ __device__ inline void line_apply(const LineCtx<T> &c, const DevTab<T, N> &tb, const T (&u)[N], T tLu,
                                           T tLd, T tRu, T tRd, bool hasb, T (&v)[N]) {
  const T ih = T(1) / c.hk;
  const T alpha = c.stan * c.vol * c.delta * ih * ih;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T acc = T(0);
#pragma unroll
    for (int l = 0; l < N; ++l) acc += tb.S[i][l] * u[l];
    v[i] = alpha * acc;
  }
  if (c.cre != T(0)) {
    const T rc = c.cre * c.vol * c.stan;
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += rc * tb.w[i] * u[i];
  }
  if (hasb) {
    const T coef = -c.stan * c.vol * ih;
    T bu[N];
#pragma unroll
    for (int q = 0; q < N; ++q) bu[q] = tb.w[q] * (c.beta + c.Bkk * (c.xk0 + tb.xi[q] * c.hk)) * u[q];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      T acc = T(0);
#pragma unroll
      for (int q = 0; q < N; ++q) acc += tb.Dt[i][q] * bu[q];
      v[i] += coef * acc;
    }
  }
  const T WF = c.stan * c.vol * ih;
  if (c.right != FACE_NEUMANN) {
    T uM = T(0), gM = T(0);
#pragma unroll
    for (int l = 0; l < N; ++l) {
      uM += tb.e1[l] * u[l];
      gM += tb.d1[l] * u[l];
    }
    gM *= ih;
    const T bnu = hasb ? c.beta + c.Bkk * (c.xk0 + c.hk) : T(0);
    T s, t;
    if (c.right == FACE_INTERIOR) {
      const T uP = tRu, gP = tRd * ih;
      const T den = T(1) / (c.delta + c.dR);
      const T wM = c.dR * den, wP = c.delta * den;
      const T gam = c.sigma * T(2) * c.delta * c.dR * den * ih;
      const T flux = bnu >= T(0) ? bnu * uM : bnu * uP;
      const T jump = uM - uP;
      s = flux - (wM * c.delta * gM + wP * c.dR * gP) + gam * jump;
      t = -wM * c.delta * jump * ih;
    } else {
      const T gam = c.sigma * c.delta * ih;
      const T flux = bnu >= T(0) ? bnu * uM : T(0);
      s = flux - c.delta * gM + gam * uM;
      t = -c.delta * uM * ih;
    }
    s *= WF;
    t *= WF;
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += s * tb.e1[i] + t * tb.d1[i];
  }
  if (c.left != FACE_NEUMANN) {
    T uP = T(0), gP = T(0);
#pragma unroll
    for (int l = 0; l < N; ++l) {
      uP += tb.e0[l] * u[l];
      gP += tb.d0[l] * u[l];
    }
    gP *= ih;
    const T bk = hasb ? c.beta + c.Bkk * c.xk0 : T(0);
    T s, t;
    if (c.left == FACE_INTERIOR) {
      const T uM = tLu, gM = tLd * ih;
      const T den = T(1) / (c.dL + c.delta);
      const T wM = c.delta * den, wP = c.dL * den;
      const T gam = c.sigma * T(2) * c.dL * c.delta * den * ih;
      const T flux = bk >= T(0) ? bk * uM : bk * uP;
      const T jump = uM - uP;
      s = -(flux - (wM * c.dL * gM + wP * c.delta * gP) + gam * jump);
      t = -wP * c.delta * jump * ih;
    } else {
      const T bnu = -bk;  // outward normal -e_k
      const T gam = c.sigma * c.delta * ih;
      const T flux = bnu >= T(0) ? bnu * uP : T(0);
      s = flux + c.delta * gP + gam * uP;
      t = c.delta * uP * ih;
    }
    s *= WF;
    t *= WF;
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += s * tb.e0[i] + t * tb.d0[i];
  }
}

// Diagonal entry i of the line operator without neighbour couplings
// (the same expressions as line_apply with u = unit vector e_i).
template <typename T, int N>
__host__ __device__ inline T line_diag(const LineCtx<T> &c, const DevTab<T, N> &tb, int i, bool hasb) {
  const T ih = T(1) / c.hk;
  T d = c.stan * c.vol * c.delta * ih * ih * tb.S[i][i];
  d += c.cre * c.vol * c.stan * tb.w[i];
  if (hasb) d += -c.stan * c.vol * ih * tb.Dt[i][i] * tb.w[i] * (c.beta + c.Bkk * (c.xk0 + tb.xi[i] * c.hk));
  const T WF = c.stan * c.vol * ih;
  if (c.right != FACE_NEUMANN) {
    const T uM = tb.e1[i], gM = tb.d1[i] * ih;
    const T bnu = hasb ? c.beta + c.Bkk * (c.xk0 + c.hk) : T(0);
    const T flux = bnu >= T(0) ? bnu * uM : T(0);
    T s, t;
    if (c.right == FACE_INTERIOR) {
      const T den = T(1) / (c.delta + c.dR);
      const T wM = c.dR * den;
      const T gam = c.sigma * T(2) * c.delta * c.dR * den * ih;
      s = flux - wM * c.delta * gM + gam * uM;
      t = -wM * c.delta * uM * ih;
    } else {
      const T gam = c.sigma * c.delta * ih;
      s = flux - c.delta * gM + gam * uM;
      t = -c.delta * uM * ih;
    }
    d += WF * (s * tb.e1[i] + t * tb.d1[i]);
  }
  if (c.left != FACE_NEUMANN) {
    const T uP = tb.e0[i], gP = tb.d0[i] * ih;
    const T bk = hasb ? c.beta + c.Bkk * c.xk0 : T(0);
    T s, t;
    if (c.left == FACE_INTERIOR) {
      const T den = T(1) / (c.dL + c.delta);
      const T wP = c.dL * den;
      const T gam = c.sigma * T(2) * c.dL * c.delta * den * ih;
      const T flux = bk >= T(0) ? T(0) : bk * uP;
      const T jump = -uP;
      s = -(flux - wP * c.delta * gP + gam * jump);
      t = -wP * c.delta * jump * ih;
    } else {
      const T bnu = -bk;
      const T gam = c.sigma * c.delta * ih;
      const T flux = bnu >= T(0) ? bnu * uP : T(0);
      s = flux + c.delta * gP + gam * uP;
      t = c.delta * uP * ih;
    }
    d += WF * (s * tb.e0[i] + t * tb.d0[i]);
  }
  return d;
}

// Build the context of the line along axis k through cell (ix,iy,iz) with
// tangential node indices (ta, tb_) on the two other axes (in increasing
// axis order).  K is read from the device array g.K.
template <typename T, int N>
__host__ __device__ inline LineCtx<T> make_ctx(const Geo &g, const DevTab<T, N> &tb, int k, int ix, int iy, int iz,
                                               int ta, int tb_) {
  LineCtx<T> c;
  const int ijk[3] = {ix, iy, iz};
  const int nn[3] = {g.nx, g.ny, g.nz};
  const int cell = ix + g.nx * (iy + g.ny * iz);
  const int stride[3] = {1, g.nx, g.nx * g.ny};
  c.stan = tb.w[ta] * tb.w[tb_];
  c.hk = (T)g.h[k];
  c.vol = (T)g.vol;
  c.delta = (T)g.K[3 * cell + k];
  c.sigma = (T)g.sigma;
  c.cre = (k == 0 && g.has_c) ? (T)g.c[cell] : T(0);
  if (ijk[k] > 0) {
    c.left = FACE_INTERIOR;
    c.dL = (T)g.K[3 * (cell - stride[k]) + k];
  } else {
    c.left = g.bc[2 * k];
    c.dL = T(0);
  }
  if (ijk[k] < nn[k] - 1) {
    c.right = FACE_INTERIOR;
    c.dR = (T)g.K[3 * (cell + stride[k]) + k];
  } else {
    c.right = g.bc[2 * k + 1];
    c.dR = T(0);
  }
  // tangential axes t1 < t2 and their physical coordinates
  const int t1 = (k == 0) ? 1 : 0;
  const int t2 = (k == 2) ? 1 : 2;
  const double x1 = (ijk[t1] + (double)tb.xi[ta]) * g.h[t1];
  const double x2 = (ijk[t2] + (double)tb.xi[tb_]) * g.h[t2];
  c.beta = (T)(g.b0[k] + g.B[3 * k + t1] * x1 + g.B[3 * k + t2] * x2);
  c.Bkk = (T)g.B[3 * k + k];
  c.xk0 = (T)(ijk[k] * g.h[k]);
  return c;
}

}  // namespace dgmg
