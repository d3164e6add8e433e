// 1-D tables of the nodal Gauss-Legendre basis on [0,1].
//
// The basis of each cell is the tensor product of 1-D Lagrange polynomials
// (Sec. 2.1, basis paragraph), and sum factorisation works with the 1-D
// matrices of shape-function values and derivatives at the quadrature
// points (Sec. 3.1, Stage 1).  With nodes at the p+1 Gauss points and the
// same points used for quadrature, the value matrix is the identity and
// only the derivative matrix D, the end values and end derivatives (for
// face terms) and the 1-D stiffness S = D^T W D are needed.
//
// Nodes: Newton iteration on the Legendre polynomial P_n, evaluated with
// the three-term recurrence; weights 2 / ((1 - x^2) P_n'(x)^2); both mapped
// from [-1,1] to [0,1].  Derivatives of the Lagrange polynomials use the
// barycentric form.
#include <cmath>

#include "dg_internal.h"

namespace dgmg {

static void legendre(int n, double x, double &pn, double &dpn) {
  double p0 = 1.0, p1 = x;
  if (n == 0) {
    pn = 1.0;
    dpn = 0.0;
    return;
  }
  for (int k = 1; k < n; ++k) {
    double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  pn = p1;
  dpn = n * (x * p1 - p0) / (x * x - 1.0);
}

void build_tables(int n, Tables1D &t) {
  t.n = n;
  const double pi = 3.14159265358979323846;
  double x[kMaxN], wt[kMaxN];
  for (int i = 0; i < n; ++i) {
    double z = std::cos(pi * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double pn, dpn;
      legendre(n, z, pn, dpn);
      double dz = pn / dpn;
      z -= dz;
      if (std::fabs(dz) < 1e-17) break;
    }
    double pn, dpn;
    legendre(n, z, pn, dpn);
    x[i] = z;
    wt[i] = 2.0 / ((1.0 - z * z) * dpn * dpn);
  }
  // descending x -> ascending xi = (1 - x)/2 ... keep symmetric pairs exact
  for (int i = 0; i < n; ++i) {
    t.xi[i] = 0.5 * (1.0 - x[i]);
    t.w[i] = 0.5 * wt[i];
  }
  for (int i = 0; i < n / 2; ++i) {  // enforce exact symmetry of the rule
    double a = 0.5 * (t.xi[i] + (1.0 - t.xi[n - 1 - i]));
    t.xi[i] = a;
    t.xi[n - 1 - i] = 1.0 - a;
    double ww = 0.5 * (t.w[i] + t.w[n - 1 - i]);
    t.w[i] = t.w[n - 1 - i] = ww;
  }
  if (n % 2 == 1) t.xi[n / 2] = 0.5;
  // barycentric weights
  double lam[kMaxN];
  for (int j = 0; j < n; ++j) {
    double prod = 1.0;
    for (int m = 0; m < n; ++m)
      if (m != j) prod *= t.xi[j] - t.xi[m];
    lam[j] = 1.0 / prod;
  }
  for (int q = 0; q < n; ++q) {
    double diag = 0.0;
    for (int j = 0; j < n; ++j) {
      if (j == q) continue;
      t.D[q][j] = (lam[j] / lam[q]) / (t.xi[q] - t.xi[j]);
      diag -= t.D[q][j];
    }
    t.D[q][q] = diag;
  }
  // end values and end derivatives (the ends are not nodes)
  for (int side = 0; side < 2; ++side) {
    double xe = side ? 1.0 : 0.0;
    for (int j = 0; j < n; ++j) {
      double l = 1.0, s = 0.0;
      for (int m = 0; m < n; ++m) {
        if (m == j) continue;
        l *= (xe - t.xi[m]) / (t.xi[j] - t.xi[m]);
        s += 1.0 / (xe - t.xi[m]);
      }
      (side ? t.e1 : t.e0)[j] = l;
      (side ? t.d1 : t.d0)[j] = l * s;
    }
  }
  for (int i = 0; i < n; ++i)
    for (int l = 0; l < n; ++l) {
      double s = 0.0;
      for (int q = 0; q < n; ++q) s += t.w[q] * t.D[q][i] * t.D[q][l];
      t.S[i][l] = s;
    }
}

}  // namespace dgmg
