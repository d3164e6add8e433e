// Helpers shared by the outer solvers (solve.cpp, batch.cpp).
#pragma once

#include <chrono>
#include <vector>

#include "dg_internal.h"

namespace dgmg {

int alloc_tmp(dg_problem *pr, int prec, int k, void **out);
int precond_apply(dg_problem *pr, const dg_solve_opts *o, const double *r, double *z, double rnorm, float *r32,
                  float *z32, hipStream_t s);
// FP32 preconditioner on an r32 the caller already scaled by 1 / sqrt(*rr_dev),
// z scaled back, and out[j] = z . b_j (j < m <= 2) in the same pass
int precond_apply_fp32_dots(dg_problem *pr, const dg_solve_opts *o, const float *r32, float *z32, double *z,
                            const double *rr_dev, int m, const double *b0, const double *b1, double *part,
                            double *out, hipStream_t s);
// z = M(r) in FP64 and out[j] = z . b_j, j < m <= 2 (the dots in the last
// smoothing sweep where it can take them)
int precond_apply_fp64_dots(dg_problem *pr, const dg_solve_opts *o, const double *r, double *z, int m,
                            const double *b0, const double *b1, double *part, double *out, hipStream_t s);

// Device allocations owned by one solve; freed together.  reserve() takes
// one block for the buffers that follow (each rounded up to 256 bytes);
// get() carves from it while it lasts, else allocates on its own.
struct DevBuf {
  std::vector<void *> ptrs;
  size_t bytes = 0;
  char *cur = nullptr;
  size_t left = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() {
    for (void *p : ptrs) (void)hipFree(p);
  }
  static size_t round(size_t b) { return (b + 255) & ~size_t(255); }
  int reserve(size_t total) {
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, total);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc (solve workspace)");
    ptrs.push_back(p);
    cur = (char *)p;
    left = total;
    return DG_OK;
  }
  template <typename T>
  int get(T **out, size_t n) {
    const size_t b = round(n * sizeof(T));
    void *p = nullptr;
    if (b <= left) {
      p = cur;
      cur += b;
      left -= b;
    } else {
      hipError_t e = hipMalloc(&p, b);
      if (e != hipSuccess) return hip_fail(e, "hipMalloc (solve workspace)");
      ptrs.push_back(p);
    }
    bytes += n * sizeof(T);
    *out = (T *)p;
    return DG_OK;
  }
};

inline double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int validate_solve_opts(const dg_solve_opts *o);
// f, u (and opts->u_ref) are 16-byte aligned, distinct device vectors
int check_solve_vectors(const double *f, const double *u, const dg_solve_opts *o);
// counting of the preconditioner's inner iterations (opts->inner_stats)
int inner_count_begin(dg_problem *pr, const dg_solve_opts *o, hipStream_t s);
int inner_count_end(dg_problem *pr, const dg_solve_opts *o, dg_solve_result *res, hipStream_t s);
// *err = ||u - u_ref||_2 / ||u_ref||_2 (or -1 without u_ref); tmp: [n]
// scratch, part / dout: dot scratch; synchronises s
int solution_error(int64_t n, const double *u, const double *u_ref, double *tmp, double *part, double *dout,
                   hipStream_t s, double *err);
int validate_mg_opts(const dg_mg_opts *o);

}  // namespace dgmg
