// Host copy of the 1-D Gauss-Legendre tables and of the Gauss-Lobatto
// nodes (see ctables.h for the definitions; both come from the same
// constexpr functions).
#include "dg_internal.h"

namespace dgmg {

template <int N>
static void copy_tab(Tables1D &t) {
  constexpr ct::Tab<N> c = ct::make_tab<N>();
  for (int i = 0; i < N; ++i) {
    t.xi[i] = c.xi[i];
    t.w[i] = c.w[i];
    t.e0[i] = c.e0[i];
    t.e1[i] = c.e1[i];
    t.d0[i] = c.d0[i];
    t.d1[i] = c.d1[i];
    for (int j = 0; j < N; ++j) {
      t.D[i][j] = c.D[i][j];
      t.S[i][j] = c.S[i][j];
    }
  }
}

template <int N>
static void copy_gll(double *xi) {
  constexpr ct::GllTab<N> g = ct::make_gll_tab<N>();
  for (int i = 0; i < N; ++i) xi[i] = g.xi[i];
}

// the n Gauss-Lobatto points on [0,1]
void gll_nodes(int n, double *xi) {
  switch (n) {
    case 2: copy_gll<2>(xi); break;
    case 3: copy_gll<3>(xi); break;
    case 4: copy_gll<4>(xi); break;
    case 5: copy_gll<5>(xi); break;
    case 6: copy_gll<6>(xi); break;
    default: break;
  }
}

void build_tables(int n, Tables1D &t) {
  t.n = n;
  switch (n) {
    case 2: copy_tab<2>(t); break;
    case 3: copy_tab<3>(t); break;
    case 4: copy_tab<4>(t); break;
    case 5: copy_tab<5>(t); break;
    case 6: copy_tab<6>(t); break;
    default: break;
  }
}

}  // namespace dgmg
