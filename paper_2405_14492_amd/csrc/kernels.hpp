// Data structures and launchers shared by the FSA kernel files.
#pragma once

#include <cmath>

#include "common.hpp"

namespace fsa {

// Uniform grid over one point set: cell (cx, cy) = floor((x - x0)/h),
// floor((y - y0)/h); cell id = cy * gx + cx.
struct GridDesc {
  double x0, y0, h, gamma;
  int64_t gx, gy;
};

struct Grid {
  int64_t n = 0, ncell = 0;
  GridDesc desc{};
  Buf<double> bbox;
  Buf<int> cell, count;   // per original point / per cell
  Buf<int64_t> cstart;    // ncell + 1 offsets into the sorted order
  Buf<int> perm, iperm;   // sorted slot -> original index, and inverse
  Buf<double> xs;         // sorted coordinates (n x 2)
  void release() {
    bbox.release(); cell.release(); count.release(); cstart.release();
    perm.release(); iperm.release(); xs.release();
  }
};

struct Csr {
  int64_t nrows = 0, nnz = 0;
  Buf<int64_t> row_ptr;
  Buf<int> col;
  // Per nonzero: (row - first row of its cell) mod 32 in the top 5 bits,
  // position of the column in its row cell's 3x3 neighbourhood (the three
  // contiguous column ranges of cell_ranges, concatenated) in the low 27.
  Buf<int> key;
  // largest neighbourhood row window (rows between the first and last
  // candidate column of a row cell) and largest 32-row group entry count
  int64_t max_window = 0, max_group_nnz = 0;
  void release() { row_ptr.release(); col.release(); key.release(); }
};

constexpr int KEY_SLOT_BITS = 27;
constexpr int KEY_SLOT_MASK = (1 << KEY_SLOT_BITS) - 1;

// The column points that can neighbour row cell `cell`: the cells of rows
// cy-1, cy, cy+1 (clipped) and columns cx-1..cx+1 (clipped) of the column
// grid, which is laid out like the row grid.  Range t is [qb[t], qe[t]) in
// the column set's sorted order and starts at position off[t] of the
// concatenation; the return value is the total length.
__device__ __forceinline__ int cell_ranges(int64_t cell, const GridDesc& gd, const int64_t* __restrict__ ccs,
                                           int* qb, int* qe, int* off) {
  const int64_t cx = cell % gd.gx, cy = cell / gd.gx;
  const int64_t xlo = cx - 1 < 0 ? 0 : cx - 1;
  const int64_t xhi = cx + 1 >= gd.gx ? gd.gx - 1 : cx + 1;
  int tot = 0;
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    const int64_t yy = cy - 1 + t;
    qb[t] = qe[t] = 0;
    if (yy >= 0 && yy < gd.gy) {
      qb[t] = (int)ccs[yy * gd.gx + xlo];
      qe[t] = (int)ccs[yy * gd.gx + xhi + 1];
    }
    off[t] = tot;
    tot += qe[t] - qb[t];
  }
  return tot;
}

__global__ void k_cstart_to_cursor(const int64_t* cstart, int64_t ncell, int* cursor);

fsa_status scan_counts(const int* in, int64_t n, int64_t* out, Buf<int64_t>& scratch, hipStream_t st);
fsa_status build_grid(Grid& g, const double* locs, int64_t n, double gamma, hipStream_t st, int* bad_flag_dev,
                      const Grid* like);
fsa_status build_pattern(const Grid& rows, const Grid& cols, Csr& csr, hipStream_t st);
fsa_status export_csr(const Csr& csr, const Grid& rows, const Grid& cols, const double* val_dev, int64_t* row_ptr_h,
                      int* col_h, double* val_h, hipStream_t st);

// ---- small dense (mp x mp, float64, row-major) ----
// Sigma_m of the (padded) inducing points; identity on the padding.
fsa_status dense_sigma_m(const double* ind, int m, int mp, const Theta& th, double jitter, bool drho, double* out,
                         hipStream_t st);
// In-place lower Cholesky; *info_dev = 0 or (failed column + 1).
fsa_status dense_cholesky(double* A, int mp, int* info_dev, hipStream_t st);
// C = alpha * op(A) op(B), op = transpose if flag set; all mp x mp.
fsa_status dense_gemm(const double* A, bool ta, const double* B, bool tb, double* C, int mp, double alpha,
                      hipStream_t st);
// out = sum_k 2 log L_kk (mp entries)
fsa_status dense_logdet_chol(const double* L, int mp, double* out, hipStream_t st);
// out_f = (float) in
fsa_status to_float(const double* in, float* out, int64_t cnt, hipStream_t st);
fsa_status add_identity(double* A, int mp, hipStream_t st);
fsa_status transpose_scale(const double* A, double* out, int mp, double scale, hipStream_t st);

}  // namespace fsa
