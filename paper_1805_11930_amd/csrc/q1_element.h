// One row of the matrix of a_h on the trilinear corner functions of a cell
// (Sec. 2.2.2-2.2.3, App. A.2): row a of E_c with E_c[a][b] = a_h(phi_b,
// phi_a), corners q = qx + 2 qy + 4 qz.
//
// The trilinears are continuous, so every interior jump term vanishes and
// only the volume terms and the Dirichlet boundary-face terms of a_h
// remain.  Since they lie in the DG space, this equals the Galerkin product
// P^T A P of the DG matrix with the nodal interpolation P when the same
// quadrature is used: all terms have polynomial integrands of degree <= 3
// per direction (b affine), which every Gauss rule of >= 2 points
// integrates exactly, except the positive part of b.nu on a boundary face,
// which is taken at the DG operator's own face points.
//   volume diffusion / reaction: closed forms from the 1-D factors
//     stiffness (1/h) [[1,-1],[-1,1]], mass h [[1/3,1/6],[1/6,1/3]];
//   volume advection -(b phi_b, grad phi_a): 2-point Gauss per direction;
//   Dirichlet faces: -d phi_a dn phi_b - d dn phi_a phi_b
//     + (gamma + max(b.nu, 0)) phi_a phi_b at the (p+1)^2 face points.
#pragma once

#include "line_ops.h"

namespace dgmg {

template <int N>
__host__ __device__ inline void q1_element_row(const Geo &g, const DevTab<double, N> &tb, int c, const int (&ijk)[3],
                                               int a, double (&row)[8]) {
  const double K[3] = {g.K[3 * (size_t)c], g.K[3 * (size_t)c + 1], g.K[3 * (size_t)c + 2]};
  const double cr = g.has_c ? g.c[c] : 0.0;
  const int da[3] = {a & 1, (a >> 1) & 1, a >> 2};
  for (int b = 0; b < 8; ++b) {
    const int db[3] = {b & 1, (b >> 1) & 1, b >> 2};
    double st[3], ms[3];
    for (int k = 0; k < 3; ++k) {
      st[k] = (da[k] == db[k] ? 1.0 : -1.0) / g.h[k];
      ms[k] = (da[k] == db[k] ? 1.0 / 3.0 : 1.0 / 6.0) * g.h[k];
    }
    row[b] = K[0] * st[0] * ms[1] * ms[2] + K[1] * ms[0] * st[1] * ms[2] + K[2] * ms[0] * ms[1] * st[2] +
             cr * ms[0] * ms[1] * ms[2];
  }
  auto bfield = [&](const double (&x)[3], int k) {
    double v = g.b0[k];
    for (int l = 0; l < 3; ++l) v += g.B[3 * k + l] * x[l];
    return v;
  };
  if (g.has_b) {
    const double gp[2] = {0.5 - 0.5 / sqrt(3.0), 0.5 + 0.5 / sqrt(3.0)};
    const double W = 0.125 * g.vol;
    for (int qz = 0; qz < 2; ++qz)
      for (int qy = 0; qy < 2; ++qy)
        for (int qx = 0; qx < 2; ++qx) {
          const double xi[3] = {gp[qx], gp[qy], gp[qz]};
          double x[3];
          for (int k = 0; k < 3; ++k) x[k] = (ijk[k] + xi[k]) * g.h[k];
          double La[3], gra[3];
          for (int k = 0; k < 3; ++k) La[k] = da[k] ? xi[k] : 1.0 - xi[k];
          for (int k = 0; k < 3; ++k) {
            const double dL = (da[k] ? 1.0 : -1.0) / g.h[k];
            gra[k] = dL * La[(k + 1) % 3] * La[(k + 2) % 3];
          }
          const double bq[3] = {bfield(x, 0), bfield(x, 1), bfield(x, 2)};
          const double bg = bq[0] * gra[0] + bq[1] * gra[1] + bq[2] * gra[2];
          for (int b = 0; b < 8; ++b) {
            const int db[3] = {b & 1, (b >> 1) & 1, b >> 2};
            double phib = 1.0;
            for (int k = 0; k < 3; ++k) phib *= db[k] ? xi[k] : 1.0 - xi[k];
            row[b] -= W * bg * phib;
          }
        }
  }
  const int nn[3] = {g.nx, g.ny, g.nz};
  for (int k = 0; k < 3; ++k)
    for (int side = 0; side < 2; ++side) {
      const bool boundary = side ? ijk[k] == nn[k] - 1 : ijk[k] == 0;
      if (!boundary || g.bc[2 * k + side] != FACE_DIRICHLET) continue;
      const int t1 = (k == 0) ? 1 : 0, t2 = (k == 2) ? 1 : 2;
      const double area = g.vol / g.h[k];
      const double nu = side ? 1.0 : -1.0;
      const double d = K[k];
      const double gam = g.sigma * d / g.h[k];
      for (int ib = 0; ib < N; ++ib)
        for (int ia = 0; ia < N; ++ia) {
          double xi[3];
          xi[k] = side;
          xi[t1] = tb.xi[ia];
          xi[t2] = tb.xi[ib];
          double x[3];
          for (int l = 0; l < 3; ++l) x[l] = (ijk[l] + xi[l]) * g.h[l];
          const double WF = tb.w[ia] * tb.w[ib] * area;
          double La[3];
          for (int l = 0; l < 3; ++l) La[l] = da[l] ? xi[l] : 1.0 - xi[l];
          const double phia = La[0] * La[1] * La[2];
          const double dna = nu * (da[k] ? 1.0 : -1.0) / g.h[k] * La[t1] * La[t2];
          double up = 0.0;
          if (g.has_b) {
            const double bnu = nu * bfield(x, k);
            up = bnu >= 0.0 ? bnu : 0.0;
          }
          for (int b = 0; b < 8; ++b) {
            const int db[3] = {b & 1, (b >> 1) & 1, b >> 2};
            double Lb[3];
            for (int l = 0; l < 3; ++l) Lb[l] = db[l] ? xi[l] : 1.0 - xi[l];
            const double phib = Lb[0] * Lb[1] * Lb[2];
            const double dnb = nu * (db[k] ? 1.0 : -1.0) / g.h[k] * Lb[t1] * Lb[t2];
            row[b] += WF * (-d * phia * dnb - d * dna * phib + (gam + up) * phia * phib);
          }
        }
    }
}

}  // namespace dgmg
