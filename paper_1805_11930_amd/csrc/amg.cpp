// Aggregation AMG for the coarse-space matrix of the hybrid V-cycle (alg
// hybrid_multigrid, coarse solve; Sec. 2.2, where the paper hands the
// P0 / Q1 problem to an algebraic multigrid).  The coarse solver is not
// specified beyond "AMG"; this one is smoothed aggregation (Vanek, Mandel,
// Brezina, "Algebraic multigrid by smoothed aggregation for second and
// fourth order elliptic problems", Computing 56, 1996), set up on the host
// once per problem and applied on the device:
//
//  * strength: j is a strong neighbour of i when
//    max(|a_ij|, |a_ji|) >= theta_l sqrt(|a_ii a_jj|), theta_l = 0.08 / 2^l;
//  * aggregation in three passes over the unknowns in index order: (1) an
//    unknown whose strong neighbours are all free starts an aggregate with
//    them; (2) a free unknown joins the aggregate of its strongest
//    aggregated neighbour of pass 1; (3) what is left forms aggregates of
//    itself and its free strong neighbours;
//  * tentative prolongation: the aggregates' indicator vectors;
//    prolongation P = (I - omega D_F^-1 A_F) P_tent with the filtered matrix
//    A_F (weak couplings moved onto the diagonal, so row sums are kept) and
//    omega = 4 / (3 rho), rho the Gershgorin bound of D_F^-1 A_F;
//  * restriction R = P^T, Galerkin product A_c = R A P;
//  * until at most 1024 unknowns remain (inverted densely).
//
// Level 0 is the structured level 0 of the geometric hierarchy of the same
// coarse space (its 7- or 27-point stencil, its buffers and smoothing
// diagonal); the levels below are CSR.  The cycle (api.cpp, coarse_cycle)
// is the same damped-Jacobi V-cycle as the geometric one, with
// 2 / sum_j |a_ij| as the smoothing diagonal on every level.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "dg_internal.h"

namespace dgmg {

int dmalloc(dg_problem *pr, void **p, size_t bytes);
int ensure_hierarchy(dg_problem *pr, int kind);
bool dense_inverse(std::vector<double> M, int n, std::vector<double> &inv);

namespace {

constexpr int kAmgBottomMax = 1024;
constexpr int kAmgMaxLevels = 24;
constexpr double kTheta0 = 0.08;

struct Csr {
  int n = 0, m = 0;  // rows, columns
  std::vector<int> rp, ci;
  std::vector<double> v;
  int64_t nnz() const { return (int64_t)ci.size(); }
};

// Structured level (7- or 27-point stencil [ns][n] on a vx * vy * vz grid)
// to CSR with sorted columns; couplings outside the grid and exact zeros
// are left out.
Csr stencil_to_csr(const std::vector<double> &A, const CoarseLevel &L) {
  Csr M;
  M.n = M.m = L.n;
  M.rp.assign((size_t)L.n + 1, 0);
  M.ci.reserve((size_t)L.n * L.ns);
  M.v.reserve((size_t)L.n * L.ns);
  std::vector<std::pair<int, double>> row;
  for (int i = 0; i < L.n; ++i) {
    const int ix = i % L.nx, iy = (i / L.nx) % L.ny, iz = i / (L.nx * L.ny);
    row.clear();
    if (L.ns == 7) {
      row.emplace_back(i, A[i]);
      const int off[6] = {-1, 1, -L.nx, L.nx, -L.nx * L.ny, L.nx * L.ny};
      const bool ok[6] = {ix > 0, ix < L.nx - 1, iy > 0, iy < L.ny - 1, iz > 0, iz < L.nz - 1};
      for (int d = 0; d < 6; ++d)
        if (ok[d]) row.emplace_back(i + off[d], A[(size_t)(1 + d) * L.n + i]);
    } else {
      for (int o = 0; o < 27; ++o) {
        const int jx = ix + o % 3 - 1, jy = iy + (o / 3) % 3 - 1, jz = iz + o / 9 - 1;
        if (jx < 0 || jy < 0 || jz < 0 || jx >= L.nx || jy >= L.ny || jz >= L.nz) continue;
        row.emplace_back(jx + L.nx * (jy + L.ny * jz), A[(size_t)o * L.n + i]);
      }
    }
    std::sort(row.begin(), row.end());
    for (auto &e : row) {
      if (e.second == 0.0 && e.first != i) continue;
      M.ci.push_back(e.first);
      M.v.push_back(e.second);
    }
    M.rp[i + 1] = (int)M.ci.size();
  }
  return M;
}

Csr transpose(const Csr &A) {
  Csr T;
  T.n = A.m;
  T.m = A.n;
  T.rp.assign((size_t)T.n + 1, 0);
  for (int c : A.ci) ++T.rp[c + 1];
  for (int i = 0; i < T.n; ++i) T.rp[i + 1] += T.rp[i];
  T.ci.resize(A.ci.size());
  T.v.resize(A.v.size());
  std::vector<int> pos(T.rp.begin(), T.rp.end() - 1);
  for (int i = 0; i < A.n; ++i)
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      const int p = pos[A.ci[k]]++;
      T.ci[p] = i;
      T.v[p] = A.v[k];
    }
  return T;  // rows come out sorted: i ascends
}

// C = A B (Gustavson, dense accumulator over the columns of B), sorted rows.
Csr multiply(const Csr &A, const Csr &B) {
  Csr C;
  C.n = A.n;
  C.m = B.m;
  C.rp.assign((size_t)C.n + 1, 0);
  std::vector<int> mark((size_t)B.m, -1);
  std::vector<double> acc((size_t)B.m, 0.0);
  std::vector<int> cols;
  for (int i = 0; i < A.n; ++i) {
    cols.clear();
    for (int ka = A.rp[i]; ka < A.rp[i + 1]; ++ka) {
      const int k = A.ci[ka];
      const double a = A.v[ka];
      for (int kb = B.rp[k]; kb < B.rp[k + 1]; ++kb) {
        const int j = B.ci[kb];
        if (mark[j] != i) {
          mark[j] = i;
          acc[j] = 0.0;
          cols.push_back(j);
        }
        acc[j] += a * B.v[kb];
      }
    }
    std::sort(cols.begin(), cols.end());
    for (int j : cols) {
      C.ci.push_back(j);
      C.v.push_back(acc[j]);
    }
    C.rp[i + 1] = (int)C.ci.size();
  }
  return C;
}

double diag_of(const Csr &A, int i) {
  for (int k = A.rp[i]; k < A.rp[i + 1]; ++k)
    if (A.ci[k] == i) return A.v[k];
  return 0.0;
}

// Strong-neighbour lists (symmetric measure max(|a_ij|, |a_ji|)).
void strength(const Csr &A, const Csr &AT, double theta, std::vector<int> &sp, std::vector<int> &sc,
              std::vector<double> &sv) {
  const int n = A.n;
  std::vector<double> d(n);
  for (int i = 0; i < n; ++i) d[i] = std::fabs(diag_of(A, i));
  sp.assign((size_t)n + 1, 0);
  sc.clear();
  sv.clear();
  for (int i = 0; i < n; ++i) {
    // merge row i of A and of A^T (both sorted)
    int ka = A.rp[i], kt = AT.rp[i];
    const int ea = A.rp[i + 1], et = AT.rp[i + 1];
    while (ka < ea || kt < et) {
      int j;
      double m;
      if (kt >= et || (ka < ea && A.ci[ka] < AT.ci[kt])) {
        j = A.ci[ka];
        m = std::fabs(A.v[ka++]);
      } else if (ka >= ea || AT.ci[kt] < A.ci[ka]) {
        j = AT.ci[kt];
        m = std::fabs(AT.v[kt++]);
      } else {
        j = A.ci[ka];
        m = std::max(std::fabs(A.v[ka++]), std::fabs(AT.v[kt++]));
      }
      if (j == i) continue;
      if (m >= theta * std::sqrt(d[i] * d[j]) && m > 0.0) {
        sc.push_back(j);
        sv.push_back(m);
      }
    }
    sp[i + 1] = (int)sc.size();
  }
}

// Aggregates (agg[i] = aggregate of unknown i); returns their number.
int aggregate(int n, const std::vector<int> &sp, const std::vector<int> &sc, const std::vector<double> &sv,
              std::vector<int> &agg) {
  agg.assign(n, -1);
  int na = 0;
  // pass 1: roots whose whole strong neighbourhood is free
  for (int i = 0; i < n; ++i) {
    if (agg[i] >= 0) continue;
    bool free_nb = true;
    for (int k = sp[i]; k < sp[i + 1] && free_nb; ++k) free_nb = agg[sc[k]] < 0;
    if (!free_nb) continue;
    agg[i] = na;
    for (int k = sp[i]; k < sp[i + 1]; ++k) agg[sc[k]] = na;
    ++na;
  }
  // pass 2: join the strongest neighbouring aggregate of pass 1
  std::vector<int> agg1(agg);
  for (int i = 0; i < n; ++i) {
    if (agg1[i] >= 0) continue;
    double best = -1.0;
    int a = -1;
    for (int k = sp[i]; k < sp[i + 1]; ++k)
      if (agg1[sc[k]] >= 0 && sv[k] > best) {
        best = sv[k];
        a = agg1[sc[k]];
      }
    if (a >= 0) agg[i] = a;
  }
  // pass 3: the rest with their free strong neighbours
  for (int i = 0; i < n; ++i) {
    if (agg[i] >= 0) continue;
    agg[i] = na;
    for (int k = sp[i]; k < sp[i + 1]; ++k)
      if (agg[sc[k]] < 0) agg[sc[k]] = na;
    ++na;
  }
  return na;
}

// Smoothed prolongation P = (I - omega D_F^-1 A_F) P_tent.
Csr smoothed_prolongation(const Csr &A, const std::vector<int> &sp, const std::vector<int> &sc,
                          const std::vector<int> &agg, int na) {
  const int n = A.n;
  // filtered matrix: strong couplings kept, weak ones added to the diagonal
  std::vector<double> dF(n);
  std::vector<char> strong;
  double rho = 0.0;
  for (int i = 0; i < n; ++i) {
    double d = 0.0, off = 0.0;
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      const int j = A.ci[k];
      if (j == i) {
        d += A.v[k];
        continue;
      }
      const bool s = std::binary_search(sc.begin() + sp[i], sc.begin() + sp[i + 1], j);
      if (s)
        off += std::fabs(A.v[k]);
      else
        d += A.v[k];
    }
    if (!(d > 0.0)) d = std::fabs(diag_of(A, i));
    if (!(d > 0.0)) d = 1.0;
    dF[i] = d;
    rho = std::max(rho, (std::fabs(d) + off) / std::fabs(d));
  }
  const double omega = 4.0 / (3.0 * rho);
  Csr P;
  P.n = n;
  P.m = na;
  P.rp.assign((size_t)n + 1, 0);
  std::vector<int> mark(na, -1);
  std::vector<double> acc(na, 0.0);
  std::vector<int> cols;
  for (int i = 0; i < n; ++i) {
    cols.clear();
    auto add = [&](int a, double v) {
      if (mark[a] != i) {
        mark[a] = i;
        acc[a] = 0.0;
        cols.push_back(a);
      }
      acc[a] += v;
    };
    add(agg[i], 1.0);
    const double s = omega / dF[i];
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      const int j = A.ci[k];
      double a;
      if (j == i) {
        a = dF[i];
      } else if (std::binary_search(sc.begin() + sp[i], sc.begin() + sp[i + 1], j)) {
        a = A.v[k];
      } else {
        continue;
      }
      add(agg[j], -s * a);
    }
    std::sort(cols.begin(), cols.end());
    for (int a : cols) {
      if (acc[a] == 0.0) continue;
      P.ci.push_back(a);
      P.v.push_back(acc[a]);
    }
    P.rp[i + 1] = (int)P.ci.size();
  }
  return P;
}

template <typename T>
int upload(dg_problem *pr, T **dst, const std::vector<T> &src) {
  int rc = dmalloc(pr, (void **)dst, std::max<size_t>(src.size(), 1) * sizeof(T));
  if (rc) return rc;
  if (!src.empty()) DG_HIP(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
  return DG_OK;
}

int upload_values(dg_problem *pr, double **d64, float **d32, const std::vector<double> &v) {
  int rc = upload(pr, d64, v);
  if (rc) return rc;
  std::vector<float> f(v.begin(), v.end());
  return upload(pr, d32, f);
}

// CSR level l >= 1: A, its smoothing diagonal, the transfers from the
// finer level, and the work vectors of both precisions.
int upload_csr_level(dg_problem *pr, CoarseLevel &L, const Csr &A, const Csr &P, const Csr &R) {
  int rc;
  L.n = A.n;
  L.nx = A.n;
  L.ny = L.nz = 1;
  L.ns = 0;
  L.nnz = (int)A.nnz();
  L.nf = P.n;
  L.pnnz = (int)P.nnz();
  std::vector<double> dinv(A.n);
  for (int i = 0; i < A.n; ++i) {
    double s = 0.0;
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) s += std::fabs(A.v[k]);
    dinv[i] = s > 0.0 ? 2.0 / s : 0.0;
  }
  if ((rc = upload(pr, &L.rp, A.rp)) || (rc = upload(pr, &L.ci, A.ci)) ||
      (rc = upload_values(pr, &L.A64, &L.A32, A.v)) || (rc = upload_values(pr, &L.dinv64, &L.dinv32, dinv)) ||
      (rc = upload(pr, &L.prp, P.rp)) || (rc = upload(pr, &L.pci, P.ci)) ||
      (rc = upload_values(pr, &L.pv64, &L.pv32, P.v)) || (rc = upload(pr, &L.rrp, R.rp)) ||
      (rc = upload(pr, &L.rci, R.ci)) || (rc = upload_values(pr, &L.rv64, &L.rv32, R.v)))
    return rc;
  for (double **p : {&L.r64, &L.x64, &L.t64})
    if ((rc = dmalloc(pr, (void **)p, (size_t)L.n * sizeof(double)))) return rc;
  for (float **p : {&L.r32, &L.x32, &L.t32})
    if ((rc = dmalloc(pr, (void **)p, (size_t)L.n * sizeof(float)))) return rc;
  return DG_OK;
}

int upload_dense_bottom(dg_problem *pr, Hierarchy &H, const Csr &A) {
  const int n = A.n;
  std::vector<double> M((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) M[(size_t)i * n + A.ci[k]] += A.v[k];
  std::vector<double> inv;
  if (!dense_inverse(M, n, inv)) {
    set_error("singular coarse matrix (pure Neumann problem without reaction?)");
    return DG_EINVAL;
  }
  int rc = upload_values(pr, &H.inv64, &H.inv32, inv);
  if (rc) return rc;
  H.bottom_n = n;
  return DG_OK;
}

int build_amg(dg_problem *pr, int kind) {
  int rc = ensure_hierarchy(pr, kind);
  if (rc) return rc;
  Hierarchy &G = kind == COARSE_Q1 ? pr->q1h : pr->p0h;
  Hierarchy &H = kind == COARSE_Q1 ? pr->q1amg : pr->p0amg;
  H.kind = kind;
  H.solver = SOLVER_AMG;
  CoarseLevel L0 = G.levels[0];
  L0.borrowed = true;
  H.levels.push_back(L0);
  std::vector<double> st((size_t)L0.ns * L0.n);
  DG_HIP(hipMemcpy(st.data(), L0.A64, st.size() * sizeof(double), hipMemcpyDeviceToHost));
  Csr A = stencil_to_csr(st, L0);
  st.clear();
  st.shrink_to_fit();
  double theta = kTheta0;
  while (A.n > kAmgBottomMax) {
    if ((int)H.levels.size() >= kAmgMaxLevels) {
      set_error("aggregation AMG: too many levels");
      return DG_EINVAL;
    }
    const Csr AT = transpose(A);
    std::vector<int> sp, sc, agg;
    std::vector<double> sv;
    strength(A, AT, theta, sp, sc, sv);
    const int na = aggregate(A.n, sp, sc, sv, agg);
    if (na >= A.n) {
      set_error("aggregation AMG: no coarsening (no strong couplings)");
      return DG_EINVAL;
    }
    const Csr P = smoothed_prolongation(A, sp, sc, agg, na);
    const Csr R = transpose(P);
    Csr Ac = multiply(R, multiply(A, P));
    CoarseLevel C;
    H.levels.push_back(C);
    if ((rc = upload_csr_level(pr, H.levels.back(), Ac, P, R))) return rc;
    A = std::move(Ac);
    theta *= 0.5;
  }
  if ((rc = upload_dense_bottom(pr, H, A))) return rc;
  DG_HIP(hipStreamSynchronize(0));
  return DG_OK;
}

}  // namespace

// The AMG hierarchy of a coarse space, built on first use.
int ensure_amg(dg_problem *pr, int kind) {
  Hierarchy &H = kind == COARSE_Q1 ? pr->q1amg : pr->p0amg;
  if (H.built == 1) return DG_OK;
  if (H.built < 0) {
    set_error("the AMG coarse solver could not be built for this problem");
    return H.built;
  }
  const int rc = build_amg(pr, kind);
  H.built = rc == DG_OK ? 1 : (rc < 0 ? rc : DG_EINVAL);
  return rc;
}

// CSR of level `level` of the AMG hierarchy (level 0: the structured level
// 0 as CSR; which = 0: A_l, 1: P into level l, 2: R = P^T), HOST output.
// dims: [4] = (rows, cols, nnz, nlevels).  With rp == NULL only dims.
int amg_level_csr(dg_problem *pr, int kind, int level, int which, int64_t *dims, int *rp, int *ci, double *v) {
  int rc = ensure_amg(pr, kind);
  if (rc) return rc;
  Hierarchy &H = kind == COARSE_Q1 ? pr->q1amg : pr->p0amg;
  if (level < 0 || level >= (int)H.levels.size() || which < 0 || which > 2 || (level == 0 && which != 0)) {
    set_error("dg_coarse_csr: level or matrix out of range");
    return DG_EINVAL;
  }
  const CoarseLevel &L = H.levels[level];
  dims[3] = (int64_t)H.levels.size();
  if (level == 0) {
    std::vector<double> st((size_t)L.ns * L.n);
    DG_HIP(hipMemcpy(st.data(), L.A64, st.size() * sizeof(double), hipMemcpyDeviceToHost));
    const Csr A = stencil_to_csr(st, L);
    dims[0] = A.n;
    dims[1] = A.m;
    dims[2] = A.nnz();
    if (rp) {
      std::memcpy(rp, A.rp.data(), A.rp.size() * sizeof(int));
      std::memcpy(ci, A.ci.data(), A.ci.size() * sizeof(int));
      std::memcpy(v, A.v.data(), A.v.size() * sizeof(double));
    }
    return DG_OK;
  }
  const int *drp = which == 0 ? L.rp : (which == 1 ? L.prp : L.rrp);
  const int *dci = which == 0 ? L.ci : (which == 1 ? L.pci : L.rci);
  const double *dv = which == 0 ? L.A64 : (which == 1 ? L.pv64 : L.rv64);
  const int rows = which == 0 ? L.n : (which == 1 ? L.nf : L.n);
  const int cols = which == 0 ? L.n : (which == 1 ? L.n : L.nf);
  int nnz = 0;
  DG_HIP(hipMemcpy(&nnz, drp + rows, sizeof(int), hipMemcpyDeviceToHost));
  dims[0] = rows;
  dims[1] = cols;
  dims[2] = nnz;
  if (rp) {
    DG_HIP(hipMemcpy(rp, drp, ((size_t)rows + 1) * sizeof(int), hipMemcpyDeviceToHost));
    DG_HIP(hipMemcpy(ci, dci, (size_t)nnz * sizeof(int), hipMemcpyDeviceToHost));
    DG_HIP(hipMemcpy(v, dv, (size_t)nnz * sizeof(double), hipMemcpyDeviceToHost));
  }
  return DG_OK;
}

}  // namespace dgmg
