// Launchers of the vector, transfer and coarse-level kernels (vec.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

struct dg_problem;

namespace dgmg {

constexpr int kMaxDots = 4;
constexpr int kDotBlocks = 1024;

struct DotSet {
  int m;
  const double *a[kMaxDots];
  const double *b[kMaxDots];
};

// out_dev[j] = a_j . b_j ; part: device scratch of kMaxDots*kDotBlocks doubles
int dots(const DotSet &ds, int64_t n, double *part, double *out_dev, hipStream_t s);
// out_dev[j] = sum of part[j * nblk .. (j + 1) * nblk), j < m (partials
// written by another kernel; large nblk: part is overwritten)
int dots_final(int m, int nblk, double *part, double *out_dev, hipStream_t s);
int axpby(int64_t n, double a, const double *x, double b, double *y, hipStream_t s);
int sub(int64_t n, const double *x, const double *y, double *z, hipStream_t s);
// outer-iteration kernels with device scalars (no host round trip)
// x += a p (not when x is nullptr), r_out = r_in - a q with a = *rz / *pq
// (a breakdown sets *flag = 1 and leaves x, r unchanged) and
// *rr = r_out . r_out (same sum as dots) in
// one pass over the vectors; part: kDotBlocks doubles of scratch.  With r32: also
// r32 = (1 / sqrt(*rr_old)) r_out in FP32 and *rr_keep = *rr_old (rr_old is
// read before rr is written, so it may be the same slot)
int cg_update_rr(int64_t n, const double *rz, const double *pq, const double *p, const double *q, double *x,
                 const double *r_in, double *r_out, double *flag, double *part, double *rr, hipStream_t s,
                 float *r32 = nullptr, const double *rr_old = nullptr, double *rr_keep = nullptr);
// z = z32 scaled back by the inverse of the factor 1 / sqrt(*rr) and
// out[j] = z . b_j for j < m <= 2 (same sums as dots), in one pass
int cast_back_dots(int64_t n, const double *rr, const float *z32, double *z, int m, const double *b0,
                   const double *b1, double *part, double *out, hipStream_t s);
// p = z + beta p (see k_beta_update); with x and pq also x += a p of the
// old p, a = rz_old / pq (0 on a breakdown), for a cg_update_rr called
// with x == nullptr
int beta_update(int64_t n, const double *zr, const double *zro, const double *rz_old, double *rz_new, bool flex,
                const double *z, double *p, hipStream_t s, double *x = nullptr, const double *pq = nullptr);
int cast_d2f(int64_t n, double sc, const double *x, float *y, hipStream_t s);
int cast_f2d(int64_t n, double sc, const float *x, double *y, hipStream_t s);

template <typename T>
int restrict_p0(int64_t ncell, int nloc, const T *r, const T *ar, T *rh, hipStream_t s);
template <typename T>
int prolong_add_p0(int64_t n, int nloc, const T *zh, T *u, hipStream_t s);

template <typename T>
int coarse_jacobi(const T *A, int nx, int ny, int nz, T w, const T *r, const T *xi, T *xo, hipStream_t s);
template <typename T>
int coarse_restrict(const T *A, int nx, int ny, int nz, const T *r, const T *x, int cnx, int cny, int cnz, T *rc,
                    hipStream_t s);
template <typename T>
int coarse_prolong(int nx, int ny, int nz, int cnx, int cny, const T *xc, T *x, hipStream_t s);
template <typename T>
int dense_mv(int n, const T *Ainv, const T *r, T *x, hipStream_t s);

// Q1 vertex-grid levels and transfers (coarse.hip)
int q1_assemble(const dg_problem *pr, double *A, hipStream_t s);
int galerkin27(const double *A, int vx, int vy, int vz, double *Ac, int cx, int cy, int cz, hipStream_t s);
int level_finish(const double *A, int64_t n, float *A32, double *d64, float *d32, hipStream_t s);
template <typename T>
int jacobi27(const T *A, const T *dinv, int vx, int vy, int vz, T w, const T *r, const T *xi, T *xo, hipStream_t s);
template <typename T>
int residual27(const T *A, int vx, int vy, int vz, const T *r, const T *x, T *out, hipStream_t s);
template <typename T>
int restrict27(int vx, int vy, int vz, const T *t, int cx, int cy, int cz, T *rc, const T *dinv, T w, T *xz,
               hipStream_t s);
template <typename T>
int prolong27(int vx, int vy, int vz, int cx, int cy, int cz, const T *xc, T *x, hipStream_t s);
// One V-cycle of the small 27-point levels of a vertex-grid hierarchy in
// a single workgroup (k_coarse_tail): levels lv[0 .. nl-1], lv[nl-1] the
// bottom with the dense inverse inv (bn unknowns); reads lv[0].r, leaves
// the result in lv[0].x and no other vector of the levels (they are kept
// in LDS).  x_init: lv[0].x already holds the first damped sweep.
constexpr int kTailLevels = 8;
constexpr int kTailThreads = 1024;
constexpr int64_t kTailMaxUnknowns = 1024;  // largest level the cycle takes
constexpr int kTailBottomMax = 128;         // largest dense bottom it takes
constexpr int kTailLds = 1536;              // unknowns of all its levels together
constexpr int kTailPrefetch = 4;            // coefficient lines per thread pulled into L2
// Largest coefficient volume the cycle takes.  Measured on the 729-unknown
// level over a 125-unknown bottom: 144 KB (FP32) runs faster as one
// workgroup than as 8 launches, 288 KB (FP64) slower.
constexpr int64_t kTailCoefBytes = 192 * 1024;
template <typename T>
struct TailLevel {
  const T *A = nullptr, *dinv = nullptr;
  T *r = nullptr, *x = nullptr, *t = nullptr;
  int vx = 0, vy = 0, vz = 0;
};
template <typename T>
struct TailArgs {
  TailLevel<T> lv[kTailLevels];
  const T *inv = nullptr;
  int nl = 0, bn = 0, nu = 1, x_init = 0;
  T w = T(0);
  int off[kTailLevels + 1] = {};  // level k's vectors at off[k] in LDS (set by coarse_tail)
};
template <typename T>
int coarse_tail(const TailArgs<T> &a, hipStream_t s);
template <typename T>
int q1_gather(int nx, int ny, int nz, const T *cs, T *rv, const T *dinv, T w, T *xz, hipStream_t s);
template <typename T>
int q1_prolong_add(int p, int nx, int ny, int nz, const T *xv, T *u, hipStream_t s);
template <typename T>
int residual7(const T *A, int nx, int ny, int nz, const T *r, const T *x, T *out, hipStream_t s);
template <typename T>
int add_to(int64_t n, const T *x, T *y, hipStream_t s);
template <typename T>
int copy_vec(int64_t n, const T *x, T *y, hipStream_t s);

// CSR levels of the aggregation AMG (amg_kernels.hip)
// (n rows, nnz entries: the mean row length picks the lanes per row)
template <typename T>
int csr_jacobi(int n, int nnz, const int *rp, const int *ci, const T *v, const T *dinv, T w, const T *r, const T *xi,
               T *xo, hipStream_t s);
template <typename T>
int csr_residual(int n, int nnz, const int *rp, const int *ci, const T *v, const T *r, const T *x, T *out,
                 hipStream_t s);
template <typename T>
int csr_spmv(int n, int nnz, const int *rp, const int *ci, const T *v, const T *x, T *y, bool add, hipStream_t s);

constexpr int kMaxBasis = 32;
struct VecList {
  const double *v[kMaxBasis];
};
struct Coefs {
  double c[kMaxBasis];
};
// Gram-Schmidt passes over the basis V_0..V_{m-1} (1 <= m <= kMaxBasis);
// part: kMaxBasis*kDotBlocks doubles, h_dev and out_dev in device memory.
// out_dev[i] = V_i . w
int gs_dot(const VecList &vl, int m, const double *w, int64_t n, double *part, double *out_dev, hipStream_t s);
// w -= sum_i h_dev[i] V_i, then out_dev[i] = V_i . w
int gs_update_dot(const VecList &vl, int m, const double *h_dev, double *w, int64_t n, double *part,
                  double *out_dev, hipStream_t s);
// w -= sum_i h_dev[i] V_i, then out_dev[0] = w . w
int gs_update_norm(const VecList &vl, int m, const double *h_dev, double *w, int64_t n, double *part,
                   double *out_dev, hipStream_t s);
int mcombine(const VecList &vl, const Coefs &y, int m, int64_t n, double *x, hipStream_t s);

int iter_stats(int64_t n, const int *it, unsigned long long *out_dev, hipStream_t s);
// acc_dev[0] += sum it, acc_dev[1] = max(acc_dev[1], max it), acc_dev[2] += n
int iter_accum(int64_t n, const int *it, unsigned long long *acc_dev, hipStream_t s);

}  // namespace dgmg
