// Problem handle: validation, device copies of the coefficients, 1-D
// tables and the P0 coarse hierarchy (Sec. 2.2.2-2.2.3, App. A.1).
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "dg_internal.h"

namespace dgmg {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

int hip_fail(hipError_t e, const char *what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? DG_ENOMEM : DG_EDEVICE;
}

// Device memory of a problem, released only by dg_problem_destroy.  Sizes
// are rounded up to 256 bytes; requests up to kChunkBytes / 4 are carved
// from shared chunks of kChunkBytes, larger ones get their own block.
constexpr size_t kChunkBytes = size_t(4) << 20;

int dmalloc(dg_problem *pr, void **p, size_t bytes) {
  *p = nullptr;
  const size_t b = (bytes + 255) & ~size_t(255);
  if (b > kChunkBytes / 4) {
    hipError_t e = hipMalloc(p, b);
    if (e != hipSuccess) {
      *p = nullptr;
      return hip_fail(e, "hipMalloc");
    }
    pr->blocks.push_back(*p);
  } else {
    if (pr->chunk_left < b) {
      void *c = nullptr;
      hipError_t e = hipMalloc(&c, kChunkBytes);
      if (e != hipSuccess) return hip_fail(e, "hipMalloc");
      pr->blocks.push_back(c);
      pr->chunk_cur = (char *)c;
      pr->chunk_left = kChunkBytes;
    }
    *p = pr->chunk_cur;
    pr->chunk_cur += b;
    pr->chunk_left -= b;
  }
  pr->held_bytes += bytes;
  return DG_OK;
}

// P0 coarse matrix A_hat_{T,T'} = a_h(1_T', 1_T) (App. A.1, eqn
// p0_galerkin1): gradients of P0 functions vanish, so only the reaction
// c |T|, the upwind terms and the penalty terms remain.  The face integrals
// of the upwind terms use the same tangential Gauss points as the DG
// operator, so A_hat equals P^T A P exactly.
static void p0_stencil(const dg_problem *pr, const std::vector<double> &K, const std::vector<double> &cc,
                       std::vector<double> &A) {
  const Geo &g = pr->geo;
  const int64_t n = pr->ncell;
  const int N = pr->n;
  const Tables1D &t = pr->tab;
  A.assign(7 * n, 0.0);
  const int nn[3] = {g.nx, g.ny, g.nz};
  const int64_t stride[3] = {1, g.nx, (int64_t)g.nx * g.ny};
  for (int64_t c = 0; c < n; ++c) {
    const int ijk[3] = {(int)(c % g.nx), (int)((c / g.nx) % g.ny), (int)(c / ((int64_t)g.nx * g.ny))};
    A[c] += cc[c] * g.vol;
    for (int k = 0; k < 3; ++k) {
      const int t1 = (k == 0) ? 1 : 0, t2 = (k == 2) ? 1 : 2;
      const double area = g.vol / g.h[k];
      for (int side = 0; side < 2; ++side) {
        const bool boundary = side ? (ijk[k] == nn[k] - 1) : (ijk[k] == 0);
        // sum over face points of W^F b_nu chi (outward / T- orientation)
        auto upwind = [&](double nu, bool positive_part) {
          double s = 0.0;
          if (!g.has_b) return 0.0;
          for (int a = 0; a < N; ++a)
            for (int b = 0; b < N; ++b) {
              double x[3];
              x[k] = (ijk[k] + side) * g.h[k];
              x[t1] = (ijk[t1] + t.xi[a]) * g.h[t1];
              x[t2] = (ijk[t2] + t.xi[b]) * g.h[t2];
              double bk = g.b0[k];
              for (int l = 0; l < 3; ++l) bk += g.B[3 * k + l] * x[l];
              const double bnu = nu * bk;
              const double WF = t.w[a] * t.w[b] * area;
              if (positive_part ? (bnu >= 0.0) : (bnu < 0.0)) s += WF * bnu;
            }
          return s;
        };
        if (boundary) {
          if (g.bc[2 * k + side] != FACE_DIRICHLET) continue;
          const double d = K[3 * c + k];
          const double gam = g.sigma * d / g.h[k];
          A[c] += gam * area + upwind(side ? 1.0 : -1.0, true);
        } else if (side == 1) {
          // interior face, this cell is T- (nu = +e_k), neighbour T+
          const int64_t cu = c + stride[k];
          const double dm = K[3 * c + k], dp = K[3 * cu + k];
          const double gam = g.sigma * 2.0 * dm * dp / (dm + dp) / g.h[k];
          const double up_pos = upwind(1.0, true);   // sum W b_nu chi-
          const double up_neg = upwind(1.0, false);  // sum W b_nu chi+
          A[c] += up_pos + gam * area;                          // (-,-)
          A[(2 + 2 * k) * n + c] += up_neg - gam * area;        // row T-, col T+ (+k)
          A[(1 + 2 * k) * n + cu] += -up_pos - gam * area;      // row T+, col T- (-k)
          A[cu] += -up_neg + gam * area;                        // (+,+)
        }
      }
    }
  }
}

// Galerkin product with piecewise-constant aggregation of 2x2x2 blocks.
static void aggregate(const std::vector<double> &A, int nx, int ny, int nz, std::vector<double> &Ac, int &cnx,
                      int &cny, int &cnz) {
  cnx = (nx + 1) / 2;
  cny = (ny + 1) / 2;
  cnz = (nz + 1) / 2;
  const int64_t n = (int64_t)nx * ny * nz, nc = (int64_t)cnx * cny * cnz;
  Ac.assign(7 * nc, 0.0);
  for (int iz = 0; iz < nz; ++iz)
    for (int iy = 0; iy < ny; ++iy)
      for (int ix = 0; ix < nx; ++ix) {
        const int64_t i = ix + (int64_t)nx * (iy + (int64_t)ny * iz);
        const int jx = ix / 2, jy = iy / 2, jz = iz / 2;
        const int64_t J = jx + (int64_t)cnx * (jy + (int64_t)cny * jz);
        Ac[J] += A[i];
        const int ii[3] = {ix, iy, iz};
        const int jj[3] = {jx, jy, jz};
        for (int dir = 0; dir < 6; ++dir) {
          const double a = A[(1 + dir) * n + i];
          if (a == 0.0) continue;
          const int k = dir / 2, sgn = (dir & 1) ? 1 : -1;
          const int nb = ii[k] + sgn;
          if ((nb / 2) == jj[k] && nb >= 0)
            Ac[J] += a;  // neighbour inside the same aggregate
          else
            Ac[(1 + dir) * nc + J] += a;
        }
      }
}

constexpr int kBottomMax = 128;

bool dense_inverse(std::vector<double> M, int n, std::vector<double> &inv) {
  inv.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (std::fabs(M[(size_t)r * n + col]) > std::fabs(M[(size_t)piv * n + col])) piv = r;
    if (M[(size_t)piv * n + col] == 0.0) return false;
    if (piv != col)
      for (int j = 0; j < n; ++j) {
        std::swap(M[(size_t)piv * n + j], M[(size_t)col * n + j]);
        std::swap(inv[(size_t)piv * n + j], inv[(size_t)col * n + j]);
      }
    const double d = 1.0 / M[(size_t)col * n + col];
    for (int j = 0; j < n; ++j) {
      M[(size_t)col * n + j] *= d;
      inv[(size_t)col * n + j] *= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      const double f = M[(size_t)r * n + col];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        M[(size_t)r * n + j] -= f * M[(size_t)col * n + j];
        inv[(size_t)r * n + j] -= f * inv[(size_t)col * n + j];
      }
    }
  }
  return true;
}

// Device buffers of one level: stencil (both precisions), work vectors
// and, for 27-point levels, the smoothing diagonal.
int alloc_level(dg_problem *pr, CoarseLevel &L, bool first) {
  const int64_t n = L.n, ns = L.ns;
  int rc;
  if ((rc = dmalloc(pr, (void **)&L.A64, ns * n * sizeof(double)))) return rc;
  if ((rc = dmalloc(pr, (void **)&L.A32, ns * n * sizeof(float)))) return rc;
  for (double **p : {&L.r64, &L.x64, &L.t64})
    if ((rc = dmalloc(pr, (void **)p, n * sizeof(double)))) return rc;
  for (float **p : {&L.r32, &L.x32, &L.t32})
    if ((rc = dmalloc(pr, (void **)p, n * sizeof(float)))) return rc;
  if (first) {
    for (double **p : {&L.acc64, &L.rs64})
      if ((rc = dmalloc(pr, (void **)p, n * sizeof(double)))) return rc;
    for (float **p : {&L.acc32, &L.rs32})
      if ((rc = dmalloc(pr, (void **)p, n * sizeof(float)))) return rc;
  }
  if (ns == 27) {
    if ((rc = dmalloc(pr, (void **)&L.dinv64, n * sizeof(double)))) return rc;
    if ((rc = dmalloc(pr, (void **)&L.dinv32, n * sizeof(float)))) return rc;
  }
  return DG_OK;
}

// Host stencil A (P0 levels) to a freshly allocated level.
int upload_level(dg_problem *pr, CoarseLevel &L, const std::vector<double> &A, bool first) {
  const int64_t n = L.n, ns = L.ns;
  int rc;
  if ((rc = alloc_level(pr, L, first))) return rc;
  std::vector<float> Af(A.begin(), A.end());
  DG_HIP(hipMemcpy(L.A64, A.data(), ns * n * sizeof(double), hipMemcpyHostToDevice));
  DG_HIP(hipMemcpy(L.A32, Af.data(), ns * n * sizeof(float), hipMemcpyHostToDevice));
  return DG_OK;
}

// Dense inverse of the coarsest level (stencil A with L.ns entries) on the
// device in both precisions.
int upload_bottom(dg_problem *pr, Hierarchy &H, const std::vector<double> &A) {
  const CoarseLevel &B = H.levels.back();
  const int n = B.n;
  std::vector<double> M((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    const int ix = i % B.nx, iy = (i / B.nx) % B.ny, iz = i / (B.nx * B.ny);
    if (B.ns == 7) {
      M[(size_t)i * n + i] = A[i];
      const int off[6] = {-1, 1, -B.nx, B.nx, -B.nx * B.ny, B.nx * B.ny};
      const bool ok[6] = {ix > 0, ix < B.nx - 1, iy > 0, iy < B.ny - 1, iz > 0, iz < B.nz - 1};
      for (int d = 0; d < 6; ++d)
        if (ok[d]) M[(size_t)i * n + i + off[d]] += A[(1 + d) * n + i];
    } else {
      for (int o = 0; o < 27; ++o) {
        const int jx = ix + o % 3 - 1, jy = iy + (o / 3) % 3 - 1, jz = iz + o / 9 - 1;
        if (jx < 0 || jy < 0 || jz < 0 || jx >= B.nx || jy >= B.ny || jz >= B.nz) continue;
        M[(size_t)i * n + jx + B.nx * (jy + B.ny * jz)] += A[(size_t)o * n + i];
      }
    }
  }
  std::vector<double> inv;
  if (!dense_inverse(M, n, inv)) {
    set_error("singular coarse matrix (pure Neumann problem without reaction?)");
    return DG_EINVAL;
  }
  int rc;
  if ((rc = dmalloc(pr, (void **)&H.inv64, (size_t)n * n * sizeof(double)))) return rc;
  if ((rc = dmalloc(pr, (void **)&H.inv32, (size_t)n * n * sizeof(float)))) return rc;
  std::vector<float> invf(inv.begin(), inv.end());
  DG_HIP(hipMemcpy(H.inv64, inv.data(), (size_t)n * n * sizeof(double), hipMemcpyHostToDevice));
  DG_HIP(hipMemcpy(H.inv32, invf.data(), (size_t)n * n * sizeof(float), hipMemcpyHostToDevice));
  H.bottom_n = n;
  return DG_OK;
}

static int build_p0(dg_problem *pr) {
  Hierarchy &H = pr->p0h;
  H.kind = COARSE_P0;
  std::vector<double> A;
  p0_stencil(pr, pr->hK, pr->hc, A);
  int nx = pr->geo.nx, ny = pr->geo.ny, nz = pr->geo.nz;
  while (true) {
    CoarseLevel L;
    L.nx = nx;
    L.ny = ny;
    L.nz = nz;
    L.n = nx * ny * nz;
    L.ns = 7;
    int rc = upload_level(pr, L, A, H.levels.empty());
    H.levels.push_back(L);
    if (rc) return rc;
    if (L.n <= kBottomMax) break;
    std::vector<double> Ac;
    int cnx, cny, cnz;
    aggregate(A, nx, ny, nz, Ac, cnx, cny, cnz);
    A.swap(Ac);
    nx = cnx;
    ny = cny;
    nz = cnz;
  }
  return upload_bottom(pr, H, A);
}

int build_q1(dg_problem *pr, int bottom_max);

int ensure_hierarchy(dg_problem *pr, int kind) {
  Hierarchy &H = kind == COARSE_Q1 ? pr->q1h : pr->p0h;
  if (H.built == 1) return DG_OK;
  if (H.built < 0) {
    set_error("the coarse space could not be built for this problem");
    return H.built;
  }
  const int rc = kind == COARSE_Q1 ? build_q1(pr, kBottomMax) : build_p0(pr);
  H.built = rc == DG_OK ? 1 : (rc < 0 ? rc : DG_EINVAL);
  return rc;
}

int alloc_tmp(dg_problem *pr, int prec, int k, void **out) {
  if (!pr->mg_tmp[prec][k]) {
    const size_t es = prec == DG_FP64 ? sizeof(double) : sizeof(float);
    int rc = dmalloc(pr, &pr->mg_tmp[prec][k], (size_t)pr->ndof * es);
    if (rc) return rc;
  }
  *out = pr->mg_tmp[prec][k];
  return DG_OK;
}

int alloc_small(dg_problem *pr) {
  int rc;
  if (!pr->iters_buf && (rc = dmalloc(pr, (void **)&pr->iters_buf, pr->ncell * sizeof(int)))) return rc;
  if (!pr->red_buf && (rc = dmalloc(pr, &pr->red_buf, 8 * 1024 * sizeof(double) + 64))) return rc;
  if (!pr->inner_acc && (rc = dmalloc(pr, (void **)&pr->inner_acc, 4 * sizeof(unsigned long long)))) return rc;
  return DG_OK;
}

}  // namespace dgmg

using namespace dgmg;

extern "C" {

const char *dg_last_error(void) { return g_last_error.c_str(); }

void dg_problem_destroy(dg_problem *pr) {
  if (!pr) return;
  for (auto &cg : pr->graphs) (void)hipGraphExecDestroy(cg.exec);
  if (pr->capture_stream) (void)hipStreamDestroy(pr->capture_stream);
  for (auto &m : pr->phase_marks) {
    (void)hipEventDestroy(m.a);
    (void)hipEventDestroy(m.b);
  }
  for (hipEvent_t e : pr->phase_spare) (void)hipEventDestroy(e);
  // every device buffer of the problem lives in one of its blocks (dmalloc)
  for (void *p : pr->blocks) (void)hipFree(p);
  delete pr;
}

int dg_problem_create(const dg_problem_desc *d, dg_problem **out) {
  if (!out) {
    set_error("dg_problem_create: out is NULL");
    return DG_EINVAL;
  }
  *out = nullptr;
  if (!d) {
    set_error("dg_problem_create: desc is NULL");
    return DG_EINVAL;
  }
  if (d->nx < 1 || d->ny < 1 || d->nz < 1) {
    set_error("cell counts must be >= 1");
    return DG_EINVAL;
  }
  if (!(d->lx > 0) || !(d->ly > 0) || !(d->lz > 0) || !std::isfinite(d->lx) || !std::isfinite(d->ly) ||
      !std::isfinite(d->lz)) {
    set_error("box lengths must be finite and > 0");
    return DG_EINVAL;
  }
  if (d->p < 1 || d->p > DG_MAX_P) {
    set_error("p must be in 1..DG_MAX_P");
    return DG_EINVAL;
  }
  const int64_t ncell = (int64_t)d->nx * d->ny * d->nz;
  const int n = d->p + 1;
  if (ncell * n * n * n > ((int64_t)1 << 31) - 1 || ncell > ((int64_t)1 << 30)) {
    set_error("problem too large for 32-bit cell indexing");
    return DG_EINVAL;
  }
  for (int f = 0; f < 6; ++f)
    if (d->bc[f] != DG_BC_DIRICHLET && d->bc[f] != DG_BC_NEUMANN) {
      set_error("bc entries must be DG_BC_DIRICHLET or DG_BC_NEUMANN");
      return DG_EINVAL;
    }
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(d->b0[i])) {
      set_error("b0 must be finite");
      return DG_EINVAL;
    }
  for (int i = 0; i < 9; ++i)
    if (!std::isfinite(d->B[i])) {
      set_error("B must be finite");
      return DG_EINVAL;
    }
  if (!std::isfinite(d->penalty_factor)) {
    set_error("penalty_factor must be finite");
    return DG_EINVAL;
  }
  if (d->basis != DG_BASIS_GL && d->basis != DG_BASIS_GLL) {
    set_error("basis must be DG_BASIS_GL or DG_BASIS_GLL");
    return DG_EINVAL;
  }
  if (d->field != DG_FIELD_NONE && d->field != DG_FIELD_AXIS_QUADRATIC && d->field != DG_FIELD_ROTATED_QUADRATIC) {
    set_error("field must be DG_FIELD_NONE, DG_FIELD_AXIS_QUADRATIC or DG_FIELD_ROTATED_QUADRATIC");
    return DG_EINVAL;
  }
  double nrot[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  if (d->field == DG_FIELD_ROTATED_QUADRATIC) {
    for (int i = 0; i < 9; ++i) nrot[i] = d->nrot[i];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        double s = 0.0;
        for (int i = 0; i < 3; ++i) s += nrot[3 * a + i] * nrot[3 * b + i];
        if (!std::isfinite(s) || std::fabs(s - (a == b ? 1.0 : 0.0)) > 1e-12) {
          set_error("field: the rows of nrot must be orthonormal");
          return DG_EINVAL;
        }
      }
  }
  const double len[3] = {d->lx, d->ly, d->lz};
  const int cnt[3] = {d->nx, d->ny, d->nz};
  if (d->field != DG_FIELD_NONE) {
    for (int i = 0; i < 9; ++i)
      if (!std::isfinite(d->kq[i])) {
        set_error("field coefficients kq must be finite");
        return DG_EINVAL;
      }
    for (int k = 0; k < 3; ++k) {
      // minimum of P_k on [0, L_k]: at an end or at the vertex
      const double a0 = d->kq[k], a1 = d->kq[3 + k], a2 = d->kq[6 + k];
      auto P = [&](double t) { return a0 + t * (a1 + t * a2); };
      double mn = std::min(P(0.0), P(len[k]));
      if (a2 != 0.0) {
        const double t = -a1 / (2.0 * a2);
        if (t > 0.0 && t < len[k]) mn = std::min(mn, P(t));
      }
      if (!(mn > 0.0)) {
        set_error("field: P_k must be > 0 on [0, L_k]");
        return DG_EINVAL;
      }
    }
    const double r2 = len[0] * len[0] + len[1] * len[1] + len[2] * len[2];
    if (!std::isfinite(d->cq[0]) || !std::isfinite(d->cq[1]) || !(d->cq[0] >= 0.0) ||
        !(d->cq[0] + d->cq[1] * r2 >= 0.0)) {
      set_error("field: c(x) = cq[0] + cq[1] |x|^2 must be finite and >= 0 on the box");
      return DG_EINVAL;
    }
  }
  std::vector<double> K(3 * ncell), cc(ncell, 0.0);
  bool has_c = false;
  if (d->field != DG_FIELD_NONE) {
    // cell-centre values for the preconditioner (the diagonal of K there)
    for (int64_t c = 0; c < ncell; ++c) {
      const int64_t ijk[3] = {c % d->nx, (c / d->nx) % d->ny, c / ((int64_t)d->nx * d->ny)};
      double xc[3], Pm[3];
      for (int k = 0; k < 3; ++k) {
        xc[k] = (ijk[k] + 0.5) * (len[k] / cnt[k]);
        Pm[k] = d->kq[k] + xc[k] * (d->kq[3 + k] + xc[k] * d->kq[6 + k]);
      }
      for (int k = 0; k < 3; ++k) {
        double s = 0.0;
        for (int m = 0; m < 3; ++m) s += Pm[m] * nrot[3 * m + k] * nrot[3 * m + k];
        K[3 * c + k] = s;
      }
      cc[c] = d->cq[0] + d->cq[1] * (xc[0] * xc[0] + xc[1] * xc[1] + xc[2] * xc[2]);
    }
    has_c = d->cq[0] != 0.0 || d->cq[1] != 0.0;
  } else {
    for (int64_t i = 0; i < 3 * ncell; ++i) {
      const double v = d->K ? d->K[i] : d->K_scalar;
      if (!(v > 0) || !std::isfinite(v)) {
        set_error("K must be finite and > 0");
        return DG_EINVAL;
      }
      K[i] = v;
    }
    for (int64_t i = 0; i < ncell; ++i) {
      const double v = d->c ? d->c[i] : d->c_scalar;
      if (!(v >= 0) || !std::isfinite(v)) {
        set_error("c must be finite and >= 0");
        return DG_EINVAL;
      }
      cc[i] = v;
      has_c = has_c || v != 0.0;
    }
  }
  dg_problem *pr = new dg_problem();
  pr->desc = *d;
  pr->desc.K = nullptr;
  pr->desc.c = nullptr;
  pr->p = d->p;
  pr->n = n;
  pr->nloc = n * n * n;
  pr->ncell = ncell;
  pr->ndof = ncell * pr->nloc;
  pr->basis = d->basis;
  (void)hipGetDevice(&pr->device);
  build_tables(n, pr->tab);
  Geo &g = pr->geo;
  g.nx = d->nx;
  g.ny = d->ny;
  g.nz = d->nz;
  g.ncell = (int)ncell;
  g.h[0] = d->lx / d->nx;
  g.h[1] = d->ly / d->ny;
  g.h[2] = d->lz / d->nz;
  g.vol = g.h[0] * g.h[1] * g.h[2];
  for (int k = 0; k < 3; ++k) g.ih[k] = 1.0 / g.h[k];
  g.fx = make_fastdiv((uint32_t)d->nx);
  g.fxy = make_fastdiv((uint32_t)(d->nx * d->ny));
  g.sigma = d->penalty_factor > 0 ? d->penalty_factor : 1.25 * d->p * (d->p + 2);
  for (int f = 0; f < 6; ++f) g.bc[f] = d->bc[f] == DG_BC_DIRICHLET ? FACE_DIRICHLET : FACE_NEUMANN;
  g.has_b = 0;
  for (int i = 0; i < 3; ++i) {
    g.b0[i] = d->b0[i];
    if (d->b0[i] != 0.0) g.has_b = 1;
  }
  for (int i = 0; i < 9; ++i) {
    g.B[i] = d->B[i];
    if (d->B[i] != 0.0) g.has_b = 1;
  }
  g.has_c = has_c ? 1 : 0;
  g.field = d->field;
  for (int i = 0; i < 9; ++i) g.kq[i] = d->field ? d->kq[i] : 0.0;
  for (int i = 0; i < 2; ++i) g.cq[i] = d->field ? d->cq[i] : 0.0;
  for (int i = 0; i < 9; ++i) g.nrot[i] = nrot[i];
  int rc = dmalloc(pr, (void **)&pr->dK, 3 * ncell * sizeof(double));
  if (!rc) rc = dmalloc(pr, (void **)&pr->dc, ncell * sizeof(double));
  if (!rc) {
    hipError_t e = hipMemcpy(pr->dK, K.data(), 3 * ncell * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(pr->dc, cc.data(), ncell * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) rc = hip_fail(e, "hipMemcpy");
  }
  g.K = pr->dK;
  g.c = pr->dc;
  for (int64_t c = 0; c < ncell; ++c) {
    double lo = 0.0, hi = 0.0;
    for (int k = 0; k < 3; ++k) {
      const double a = K[3 * c + k] * g.ih[k] * g.ih[k];
      lo = k == 0 ? a : std::min(lo, a);
      hi = k == 0 ? a : std::max(hi, a);
    }
    pr->aniso = std::max(pr->aniso, hi / lo);
  }
  pr->hK.swap(K);
  pr->hc.swap(cc);
  if (!rc) rc = alloc_small(pr);
  if (!rc && pr->basis == DG_BASIS_GLL) rc = gll_setup(pr);
  if (rc) {
    dg_problem_destroy(pr);
    return rc;
  }
  *out = pr;
  return DG_OK;
}

int64_t dg_ndof(const dg_problem *pr) { return pr ? pr->ndof : -1; }

int64_t dg_boundary_npoints(const dg_problem *pr) {
  if (!pr) return -1;
  const Geo &g = pr->geo;
  const int64_t n2 = (int64_t)pr->n * pr->n;
  return 2 * n2 * ((int64_t)g.ny * g.nz + (int64_t)g.nx * g.nz + (int64_t)g.nx * g.ny);
}

// the tensor points of the 1-D points xi in every cell, in DOF order
static void cell_points(const dg_problem *pr, const double *xi, double *xyz) {
  const Geo &g = pr->geo;
  const int N = pr->n;
  int64_t o = 0;
  for (int64_t c = 0; c < pr->ncell; ++c) {
    const int ix = (int)(c % g.nx), iy = (int)((c / g.nx) % g.ny), iz = (int)(c / ((int64_t)g.nx * g.ny));
    for (int k = 0; k < N; ++k)
      for (int j = 0; j < N; ++j)
        for (int i = 0; i < N; ++i) {
          xyz[3 * o + 0] = (ix + xi[i]) * g.h[0];
          xyz[3 * o + 1] = (iy + xi[j]) * g.h[1];
          xyz[3 * o + 2] = (iz + xi[k]) * g.h[2];
          ++o;
        }
  }
}

int dg_node_points(const dg_problem *pr, double *xyz) {
  if (!pr || !xyz) {
    set_error("dg_node_points: NULL argument");
    return DG_EINVAL;
  }
  if (pr->basis == DG_BASIS_GLL) {
    double xi[kMaxN];
    gll_nodes(pr->n, xi);
    cell_points(pr, xi, xyz);
  } else {
    cell_points(pr, pr->tab.xi, xyz);
  }
  return DG_OK;
}

int dg_quadrature_points(const dg_problem *pr, double *xyz) {
  if (!pr || !xyz) {
    set_error("dg_quadrature_points: NULL argument");
    return DG_EINVAL;
  }
  cell_points(pr, pr->tab.xi, xyz);
  return DG_OK;
}

int dg_boundary_points(const dg_problem *pr, double *xyz) {
  if (!pr || !xyz) {
    set_error("dg_boundary_points: NULL argument");
    return DG_EINVAL;
  }
  const Geo &g = pr->geo;
  const int N = pr->n;
  const int nn[3] = {g.nx, g.ny, g.nz};
  int64_t o = 0;
  for (int f = 0; f < 6; ++f) {
    const int k = f / 2, side = f % 2;
    const int t1 = (k == 0) ? 1 : 0, t2 = (k == 2) ? 1 : 2;
    for (int c2 = 0; c2 < nn[t2]; ++c2)
      for (int c1 = 0; c1 < nn[t1]; ++c1)
        for (int b = 0; b < N; ++b)
          for (int a = 0; a < N; ++a) {
            double x[3];
            x[k] = side ? nn[k] * g.h[k] : 0.0;
            x[t1] = (c1 + pr->tab.xi[a]) * g.h[t1];
            x[t2] = (c2 + pr->tab.xi[b]) * g.h[t2];
            xyz[3 * o + 0] = x[0];
            xyz[3 * o + 1] = x[1];
            xyz[3 * o + 2] = x[2];
            ++o;
          }
  }
  return DG_OK;
}

}  // extern "C"
