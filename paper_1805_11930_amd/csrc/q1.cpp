// Host setup of the conforming Q1 coarse space (Sec. 2.2.2-2.2.3, App. A.2).
//
// The coarse space is the continuous trilinear functions on the DG mesh,
// one unknown per mesh vertex.  Its matrix A_hat_ij = a_h(psi_j, psi_i) is
// evaluated directly on the trilinear vertex functions: they are
// continuous, so every jump term of an interior face vanishes and only the
// volume terms and the boundary-face terms of Dirichlet faces remain.  Since
// the trilinears lie in the DG space, this equals the Galerkin product
// P^T A P of the DG matrix with the nodal interpolation P, provided the
// same quadrature is used: all terms here have polynomial integrands of
// degree <= 3 per direction (b is affine), which every Gauss rule of
// >= 2 points integrates exactly, except the positive part of b.nu on a
// boundary face, which is evaluated at the DG operator's own face points.
//
// Coarser levels of the vertex grid: Galerkin products with trilinear
// interpolation (every second vertex along each axis, and always the last
// one), until at most bottom_max unknowns remain; that level is inverted
// densely.
#include <cmath>
#include <vector>

#include "dg_internal.h"

namespace dgmg {

int dmalloc(dg_problem *pr, void **p, size_t bytes);
int upload_level(dg_problem *pr, CoarseLevel &L, const std::vector<double> &A, bool first);
int upload_bottom(dg_problem *pr, Hierarchy &H, const std::vector<double> &A);

namespace {

// Cell-independent parts of the volume terms on a uniform mesh:
// G[k][a][b] = (d phi_a/dx_k, d phi_b/dx_k)_T and M[a][b] = (phi_a, phi_b)_T.
// 1-D factors: stiffness (1/h) [[1,-1],[-1,1]], mass h [[1/3,1/6],[1/6,1/3]].
struct RefMatrices {
  double G[3][8][8], M[8][8];
};

RefMatrices ref_matrices(const Geo &g) {
  RefMatrices r;
  for (int a = 0; a < 8; ++a)
    for (int b = 0; b < 8; ++b) {
      double st[3], ms[3];
      for (int k = 0; k < 3; ++k) {
        const int da = (a >> k) & 1, db = (b >> k) & 1;
        st[k] = (da == db ? 1.0 : -1.0) / g.h[k];
        ms[k] = (da == db ? 1.0 / 3.0 : 1.0 / 6.0) * g.h[k];
      }
      r.M[a][b] = ms[0] * ms[1] * ms[2];
      r.G[0][a][b] = st[0] * ms[1] * ms[2];
      r.G[1][a][b] = ms[0] * st[1] * ms[2];
      r.G[2][a][b] = ms[0] * ms[1] * st[2];
    }
  return r;
}

// 8 x 8 matrix of a_h on the trilinear corner functions of one cell,
// corner q = qx + 2 qy + 4 qz; E[a][b] = a_h(phi_b, phi_a).
void q1_element(const dg_problem *pr, const RefMatrices &R, int64_t c, const int ijk[3], double E[8][8]) {
  const Geo &g = pr->geo;
  const Tables1D &t = pr->tab;
  const double *K = &pr->hK[3 * c];
  const double cr = pr->hc[c];
  for (int a = 0; a < 8; ++a)
    for (int b = 0; b < 8; ++b)
      E[a][b] = K[0] * R.G[0][a][b] + K[1] * R.G[1][a][b] + K[2] * R.G[2][a][b] + cr * R.M[a][b];
  auto bfield = [&](const double x[3], int k) {
    double v = g.b0[k];
    for (int l = 0; l < 3; ++l) v += g.B[3 * k + l] * x[l];
    return v;
  };
  // advection volume term -(b phi_b, grad phi_a): 2-point Gauss rule per
  // direction (exact, see above)
  const double gp[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
  for (int qz = 0; qz < 2 && g.has_b; ++qz)
    for (int qy = 0; qy < 2; ++qy)
      for (int qx = 0; qx < 2; ++qx) {
        const double xi[3] = {gp[qx], gp[qy], gp[qz]};
        double x[3];
        for (int k = 0; k < 3; ++k) x[k] = (ijk[k] + xi[k]) * g.h[k];
        double phi[8], grad[8][3];
        for (int q = 0; q < 8; ++q) {
          const int d[3] = {q & 1, (q >> 1) & 1, q >> 2};
          double L[3], dL[3];
          for (int k = 0; k < 3; ++k) {
            L[k] = d[k] ? xi[k] : 1.0 - xi[k];
            dL[k] = (d[k] ? 1.0 : -1.0) / g.h[k];
          }
          phi[q] = L[0] * L[1] * L[2];
          grad[q][0] = dL[0] * L[1] * L[2];
          grad[q][1] = L[0] * dL[1] * L[2];
          grad[q][2] = L[0] * L[1] * dL[2];
        }
        const double W = 0.125 * g.vol;
        double bq[3];
        for (int k = 0; k < 3; ++k) bq[k] = bfield(x, k);
        for (int a = 0; a < 8; ++a)
          for (int b = 0; b < 8; ++b) {
            double v = 0.0;
            for (int k = 0; k < 3; ++k) v -= bq[k] * phi[b] * grad[a][k];
            E[a][b] += W * v;
          }
      }
  // Dirichlet boundary faces, at the DG operator's face points
  const int nn[3] = {g.nx, g.ny, g.nz};
  const int N = pr->n;
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
          xi[t1] = t.xi[ia];
          xi[t2] = t.xi[ib];
          double x[3];
          for (int l = 0; l < 3; ++l) x[l] = (ijk[l] + xi[l]) * g.h[l];
          const double WF = t.w[ia] * t.w[ib] * area;
          double phi[8], dn[8];
          for (int q = 0; q < 8; ++q) {
            const int dd[3] = {q & 1, (q >> 1) & 1, q >> 2};
            double L[3];
            for (int l = 0; l < 3; ++l) L[l] = dd[l] ? xi[l] : 1.0 - xi[l];
            phi[q] = L[0] * L[1] * L[2];
            dn[q] = nu * (dd[k] ? 1.0 : -1.0) / g.h[k] * L[t1] * L[t2];
          }
          double up = 0.0;
          if (g.has_b) {
            const double bnu = nu * bfield(x, k);
            up = bnu >= 0.0 ? bnu : 0.0;
          }
          for (int a = 0; a < 8; ++a)
            for (int b = 0; b < 8; ++b)
              E[a][b] += WF * (-d * phi[a] * dn[b] - d * dn[a] * phi[b] + (gam + up) * phi[a] * phi[b]);
        }
    }
}

// 27-point stencil of the vertex-grid matrix on level 0.
void q1_level0(const dg_problem *pr, std::vector<double> &A) {
  const Geo &g = pr->geo;
  const int vx = g.nx + 1, vy = g.ny + 1;
  const int64_t nv = (int64_t)vx * vy * (g.nz + 1);
  A.assign(27 * nv, 0.0);
  const RefMatrices R = ref_matrices(g);
  double E[8][8];
  for (int64_t c = 0; c < pr->ncell; ++c) {
    const int ijk[3] = {(int)(c % g.nx), (int)((c / g.nx) % g.ny), (int)(c / ((int64_t)g.nx * g.ny))};
    q1_element(pr, R, c, ijk, E);
    for (int a = 0; a < 8; ++a) {
      const int da[3] = {a & 1, (a >> 1) & 1, a >> 2};
      const int64_t va = (ijk[0] + da[0]) + vx * ((int64_t)(ijk[1] + da[1]) + (int64_t)vy * (ijk[2] + da[2]));
      for (int b = 0; b < 8; ++b) {
        const int o = (b & 1) - da[0] + 1 + 3 * (((b >> 1) & 1) - da[1] + 1) + 9 * ((b >> 2) - da[2] + 1);
        A[(size_t)o * nv + va] += E[a][b];
      }
    }
  }
}

// 1-D interpolation from the coarser vertex line (vc = vf/2 + 1 points):
// fine i -> (coarse index, weight) pairs.
struct Interp1 {
  int n;
  int j[2];
  double w[2];
};
Interp1 interp1(int i, int vf, int vc) {
  if (i == vf - 1) return {1, {vc - 1, 0}, {1.0, 0.0}};
  if (i % 2 == 0) return {1, {i / 2, 0}, {1.0, 0.0}};
  return {2, {i / 2, i / 2 + 1}, {0.5, 0.5}};
}

// Ac = P^T A P for the 27-point stencil A on a vx * vy * vz grid.
void galerkin27(const std::vector<double> &A, int vx, int vy, int vz, std::vector<double> &Ac, int &cx, int &cy,
                int &cz) {
  cx = vx / 2 + 1;
  cy = vy / 2 + 1;
  cz = vz / 2 + 1;
  if (vx <= 2) cx = vx;
  if (vy <= 2) cy = vy;
  if (vz <= 2) cz = vz;
  const int64_t n = (int64_t)vx * vy * vz, nc = (int64_t)cx * cy * cz;
  Ac.assign(27 * nc, 0.0);
  std::vector<Interp1> px(vx), py(vy), pz(vz);
  for (int i = 0; i < vx; ++i) px[i] = interp1(i, vx, cx);
  for (int i = 0; i < vy; ++i) py[i] = interp1(i, vy, cy);
  for (int i = 0; i < vz; ++i) pz[i] = interp1(i, vz, cz);
  for (int iz = 0; iz < vz; ++iz)
    for (int iy = 0; iy < vy; ++iy)
      for (int ix = 0; ix < vx; ++ix) {
        const int64_t i = ix + (int64_t)vx * (iy + (int64_t)vy * iz);
        for (int o = 0; o < 27; ++o) {
          const double a = A[(size_t)o * n + i];
          if (a == 0.0) continue;
          const int jx = ix + o % 3 - 1, jy = iy + (o / 3) % 3 - 1, jz = iz + o / 9 - 1;
          const Interp1 &Ix = px[ix], &Iy = py[iy], &Iz = pz[iz];
          const Interp1 &Jx = px[jx], &Jy = py[jy], &Jz = pz[jz];
          for (int c3 = 0; c3 < Iz.n; ++c3)
            for (int c2 = 0; c2 < Iy.n; ++c2)
              for (int c1 = 0; c1 < Ix.n; ++c1) {
                const double wi = Ix.w[c1] * Iy.w[c2] * Iz.w[c3] * a;
                const int64_t I = Ix.j[c1] + (int64_t)cx * (Iy.j[c2] + (int64_t)cy * Iz.j[c3]);
                for (int d3 = 0; d3 < Jz.n; ++d3)
                  for (int d2 = 0; d2 < Jy.n; ++d2)
                    for (int d1 = 0; d1 < Jx.n; ++d1) {
                      const int oc = (Jx.j[d1] - Ix.j[c1] + 1) + 3 * (Jy.j[d2] - Iy.j[c2] + 1) +
                                     9 * (Jz.j[d3] - Iz.j[c3] + 1);
                      Ac[(size_t)oc * nc + I] += wi * Jx.w[d1] * Jy.w[d2] * Jz.w[d3];
                    }
              }
        }
      }
}

}  // namespace

int build_q1(dg_problem *pr, int bottom_max) {
  Hierarchy &H = pr->q1h;
  H.kind = COARSE_Q1;
  std::vector<double> A;
  q1_level0(pr, A);
  int vx = pr->geo.nx + 1, vy = pr->geo.ny + 1, vz = pr->geo.nz + 1;
  int rc;
  while (true) {
    CoarseLevel L;
    L.nx = vx;
    L.ny = vy;
    L.nz = vz;
    L.n = vx * vy * vz;
    L.ns = 27;
    rc = upload_level(pr, L, A, H.levels.empty());
    H.levels.push_back(L);
    if (rc) return rc;
    if (L.n <= bottom_max) break;
    std::vector<double> Ac;
    int cx, cy, cz;
    galerkin27(A, vx, vy, vz, Ac, cx, cy, cz);
    A.swap(Ac);
    vx = cx;
    vy = cy;
    vz = cz;
  }
  if ((rc = upload_bottom(pr, H, A))) return rc;
  for (int prec = 0; prec < 2; ++prec) {
    const size_t es = prec == DG_FP64 ? sizeof(double) : sizeof(float);
    if (!pr->corner_buf[prec] && (rc = dmalloc(pr, &pr->corner_buf[prec], 8 * (size_t)pr->ncell * es))) return rc;
  }
  return DG_OK;
}

}  // namespace dgmg
