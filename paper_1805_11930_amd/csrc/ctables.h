// Compile-time 1-D tables of the nodal Gauss-Legendre basis on [0,1].
//
// The basis of each cell is the tensor product of 1-D Lagrange polynomials
// (Sec. 2.1, basis paragraph) and sum factorisation works with the 1-D
// matrices of shape-function values and derivatives at the quadrature
// points (Sec. 3.1, Stage 1).  With the nodes at the p+1 Gauss points and
// the same points used for quadrature the value matrix is the identity; the
// derivative matrix D, the end values / derivatives used by the face terms
// and the 1-D stiffness S = D^T W D remain.
//
// Everything is evaluated by the compiler (constexpr), so inside kernels
// every table entry is a literal: nothing is passed as a kernel argument
// or held in scalar registers.  The host copy (tables.cpp) is produced by
// the same functions.
//
// Nodes: Newton iteration on the Legendre polynomial P_n (three-term
// recurrence), started from cos(pi (i + 3/4) / (n + 1/2)); weights
// 2 / ((1 - x^2) P_n'(x)^2); both mapped from [-1,1] to [0,1].  Lagrange
// derivatives use the barycentric form.
#pragma once

namespace dgmg {
namespace ct {

constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double cabs(double x) { return x < 0 ? -x : x; }

// cosine by range reduction to [-pi, pi] and a Taylor series
constexpr double ccos(double x) {
  while (x > kPi) x -= 2 * kPi;
  while (x < -kPi) x += 2 * kPi;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 40; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}

constexpr void legendre(int n, double x, double &pn, double &dpn) {
  double p0 = 1.0, p1 = x;
  for (int k = 1; k < n; ++k) {
    const double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  pn = n == 0 ? 1.0 : p1;
  dpn = n == 0 ? 0.0 : n * (x * p1 - p0) / (x * x - 1.0);
}

template <int N>
struct Tab {
  double xi[N] = {}, w[N] = {};
  double D[N][N] = {};  // D[q][j] = l_j'(xi_q)
  double S[N][N] = {};  // D^T diag(w) D
  double e0[N] = {}, e1[N] = {}, d0[N] = {}, d1[N] = {};
};

template <int N>
constexpr Tab<N> make_tab() {
  Tab<N> t;
  double x[N] = {}, wt[N] = {};
  for (int i = 0; i < N; ++i) {
    double z = ccos(kPi * (i + 0.75) / (N + 0.5));
    for (int it = 0; it < 100; ++it) {
      double pn = 0, dpn = 0;
      legendre(N, z, pn, dpn);
      const double dz = pn / dpn;
      z -= dz;
      if (cabs(dz) < 1e-17) break;
    }
    double pn = 0, dpn = 0;
    legendre(N, z, pn, dpn);
    x[i] = z;
    wt[i] = 2.0 / ((1.0 - z * z) * dpn * dpn);
  }
  for (int i = 0; i < N; ++i) {
    t.xi[i] = 0.5 * (1.0 - x[i]);
    t.w[i] = 0.5 * wt[i];
  }
  for (int i = 0; i < N / 2; ++i) {  // exact mirror symmetry of the rule
    const double a = 0.5 * (t.xi[i] + (1.0 - t.xi[N - 1 - i]));
    t.xi[i] = a;
    t.xi[N - 1 - i] = 1.0 - a;
    const double ww = 0.5 * (t.w[i] + t.w[N - 1 - i]);
    t.w[i] = ww;
    t.w[N - 1 - i] = ww;
  }
  if (N % 2 == 1) t.xi[N / 2] = 0.5;
  double lam[N] = {};
  for (int j = 0; j < N; ++j) {
    double prod = 1.0;
    for (int m = 0; m < N; ++m)
      if (m != j) prod *= t.xi[j] - t.xi[m];
    lam[j] = 1.0 / prod;
  }
  for (int q = 0; q < N; ++q) {
    double diag = 0.0;
    for (int j = 0; j < N; ++j) {
      if (j == q) continue;
      t.D[q][j] = (lam[j] / lam[q]) / (t.xi[q] - t.xi[j]);
      diag -= t.D[q][j];
    }
    t.D[q][q] = diag;
  }
  for (int side = 0; side < 2; ++side) {
    const double xe = side ? 1.0 : 0.0;
    for (int j = 0; j < N; ++j) {
      double l = 1.0, s = 0.0;
      for (int m = 0; m < N; ++m) {
        if (m == j) continue;
        l *= (xe - t.xi[m]) / (t.xi[j] - t.xi[m]);
        s += 1.0 / (xe - t.xi[m]);
      }
      if (side) {
        t.e1[j] = l;
        t.d1[j] = l * s;
      } else {
        t.e0[j] = l;
        t.d0[j] = l * s;
      }
    }
  }
  for (int i = 0; i < N; ++i)
    for (int l = 0; l < N; ++l) {
      double s = 0.0;
      for (int q = 0; q < N; ++q) s += t.w[q] * t.D[q][i] * t.D[q][l];
      t.S[i][l] = s;
    }
  return t;
}

template <int N>
struct Tabs {
  static constexpr Tab<N> t = make_tab<N>();
};

// The paper's basis: nodal at the N Gauss-Lobatto points on [0,1] (the end
// points and the roots of P_(N-1)'), with the same N-point Gauss quadrature.
// A function with GLL nodal values u' has the Gauss-point values u = V u'
// along each axis, V[q][j] = lj(xq) for the GLL Lagrange polynomial lj at
// the Gauss point xq; in 3-D u = (V x V x V) u' (Stage 1 of Sec. 3.1 with
// the value matrix V).  Interior roots: Newton iteration on P_(N-1)' with
// P_(N-1)'' from the Legendre equation, started from -cos(pi k / (N-1)).
template <int N>
struct GllTab {
  double xi[N] = {};
  double V[N][N] = {};  // V[q][j] = l_j^GLL(xi_q^GL)
};

template <int N>
constexpr GllTab<N> make_gll_tab() {
  GllTab<N> g;
  constexpr Tab<N> t = make_tab<N>();
  double x[N] = {};
  x[0] = -1.0;
  x[N - 1] = 1.0;
  const int m = N - 1;  // roots of P_m'
  for (int k = 1; k < N - 1; ++k) {
    double z = -ccos(kPi * k / m);
    for (int it = 0; it < 100; ++it) {
      double pm = 0, dpm = 0;
      legendre(m, z, pm, dpm);
      const double d2 = (2.0 * z * dpm - m * (m + 1.0) * pm) / (1.0 - z * z);
      const double dz = dpm / d2;
      z -= dz;
      if (cabs(dz) < 1e-17) break;
    }
    x[k] = z;
  }
  for (int i = 0; i < N; ++i) g.xi[i] = 0.5 * (x[i] + 1.0);
  for (int i = 0; i < N / 2; ++i) {  // exact mirror symmetry
    const double a = 0.5 * (g.xi[i] + (1.0 - g.xi[N - 1 - i]));
    g.xi[i] = a;
    g.xi[N - 1 - i] = 1.0 - a;
  }
  if (N % 2 == 1) g.xi[N / 2] = 0.5;
  for (int q = 0; q < N; ++q)
    for (int j = 0; j < N; ++j) {
      double l = 1.0;
      for (int r = 0; r < N; ++r)
        if (r != j) l *= (t.xi[q] - g.xi[r]) / (g.xi[j] - g.xi[r]);
      g.V[q][j] = l;
    }
  return g;
}

}  // namespace ct
}  // namespace dgmg
