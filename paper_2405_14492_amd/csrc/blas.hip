// Dense float64 library products of the build and the backward (rocBLAS):
// the whitening solve with L_m and the m x m by m x n product of the
// derivative factor.  Handles come from a process-wide pool per device, so
// building a context costs no handle creation and concurrent contexts never
// share one.
#include <map>
#include <mutex>
#include <vector>

#include <rocblas/rocblas.h>

#include "ops.hpp"

namespace fsa {

namespace {
std::mutex g_mu;
std::map<int, std::vector<rocblas_handle>> g_free;

fsa_status blas_status(rocblas_status s, const char* what) {
  if (s == rocblas_status_success) return FSA_OK;
  set_error("%s failed: %s", what, rocblas_status_to_string(s));
  return FSA_ERR_DEVICE;
}
}  // namespace

fsa_status blas_acquire(BlasHandle& b) {
  if (b.h) return FSA_OK;
  int dev = 0;
  FSA_HIP(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto& v = g_free[dev];
    if (!v.empty()) {
      b.h = v.back();
      v.pop_back();
      b.dev = dev;
      return FSA_OK;
    }
  }
  rocblas_handle h = nullptr;
  FSA_TRY(blas_status(rocblas_create_handle(&h), "rocblas_create_handle"));
  b.h = h;
  b.dev = dev;
  return FSA_OK;
}

void blas_release(BlasHandle& b) {
  if (!b.h) return;
  std::lock_guard<std::mutex> lk(g_mu);
  g_free[b.dev].push_back(static_cast<rocblas_handle>(b.h));
  b.h = nullptr;
}

void blas_trim() {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& kv : g_free) {
    for (auto h : kv.second) (void)rocblas_destroy_handle(h);
    kv.second.clear();
  }
}

// X := L^{-1} X.  L: row-major mp x mp lower triangular; X: point-major
// n x mp (column-major mp x n).  Column-major, row-major L is the upper
// triangular L^T, so the solve is op(L^T) = L with op = transpose.
fsa_status blas_solve_lower(BlasHandle& b, hipStream_t st, const double* L, int mp, double* X, int64_t n) {
  if (n <= 0) return FSA_OK;
  if (n > INT32_MAX) {
    set_error("blas_solve_lower: n too large");
    return FSA_ERR_INVALID_ARG;
  }
  auto h = static_cast<rocblas_handle>(b.h);
  FSA_TRY(blas_status(rocblas_set_stream(h, st), "rocblas_set_stream"));
  const double one = 1.0;
  return blas_status(rocblas_dtrsm(h, rocblas_side_left, rocblas_fill_upper, rocblas_operation_transpose,
                                   rocblas_diagonal_non_unit, mp, (rocblas_int)n, &one, L, mp, X, mp),
                     "rocblas_dtrsm");
}

// X := alpha M Y + beta X.  M: row-major mp x mp; X, Y: point-major n x mp
// (column-major mp x n), so M enters as the transpose of its column-major view.
fsa_status blas_left_mul(BlasHandle& b, hipStream_t st, const double* M, int mp, const double* Y, double* X, int64_t n,
                         double alpha, double beta) {
  if (n <= 0) return FSA_OK;
  if (n > INT32_MAX) {
    set_error("blas_left_mul: n too large");
    return FSA_ERR_INVALID_ARG;
  }
  auto h = static_cast<rocblas_handle>(b.h);
  FSA_TRY(blas_status(rocblas_set_stream(h, st), "rocblas_set_stream"));
  return blas_status(rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, mp, (rocblas_int)n, mp,
                                   &alpha, M, mp, Y, mp, &beta, X, mp),
                     "rocblas_dgemm");
}

// Y := Y + alpha K X with K row-major lower triangular (mp x mp); X, Y
// point-major n x mp (column-major mp x n).  One product per 128-row block
// of K over its nonzero columns [0, r0 + 128): 10/16 of the full product's
// work.  Row-major K read column-major is K^T, so each block enters
// transposed.
fsa_status blas_lower_mul_acc(BlasHandle& b, hipStream_t st, const double* K, int mp, const double* X, double* Y,
                              int64_t n, double alpha) {
  if (n <= 0) return FSA_OK;
  if (n > INT32_MAX) {
    set_error("blas_lower_mul_acc: n too large");
    return FSA_ERR_INVALID_ARG;
  }
  auto h = static_cast<rocblas_handle>(b.h);
  FSA_TRY(blas_status(rocblas_set_stream(h, st), "rocblas_set_stream"));
  const double one = 1.0;
  for (int r0 = 0; r0 < mp; r0 += 128) {
    const int bs = std::min(128, mp - r0), kr = r0 + bs;
    FSA_TRY(blas_status(rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, bs, (rocblas_int)n, kr,
                                      &alpha, K + (size_t)r0 * mp, mp, X, mp, &one, Y + r0, mp),
                        "rocblas_dgemm"));
  }
  return FSA_OK;
}

// Linv := L^{-1} for row-major lower-triangular L (mp x mp).  Column-major,
// row-major L is the upper-triangular L^T, whose inverse (L^{-1})^T read
// back row-major is L^{-1}.
fsa_status blas_tri_inverse(BlasHandle& b, hipStream_t st, const double* L, double* Linv, int mp) {
  auto h = static_cast<rocblas_handle>(b.h);
  FSA_TRY(blas_status(rocblas_set_stream(h, st), "rocblas_set_stream"));
  return blas_status(rocblas_dtrtri(h, rocblas_fill_upper, rocblas_diagonal_non_unit, mp, L, mp, Linv, mp),
                     "rocblas_dtrtri");
}

}  // namespace fsa
