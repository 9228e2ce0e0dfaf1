// Uniform-grid neighbour search for the taper pattern T(gamma) (Section 2.1:
// the taper is zero for distances >= gamma).
//
// Points are binned into square cells of side h >= gamma, sorted by cell
// (row-major cell order, ties by original index, so the order is
// deterministic), and each point scans the 3x3 block of cells around its own.
// A pair (i, j) is kept iff dx*dx + dy*dy < gamma*gamma in float64 without
// contraction.  Cells of one grid row are contiguous in the sorted order, so
// the 3x3 block is three contiguous index ranges and the columns of each CSR
// row come out ascending.
#include "common.hpp"
#include "kernels.hpp"

namespace fsa {

// ------------------------------------------------------------------ bbox
__global__ __launch_bounds__(1024) void k_bbox(const double* __restrict__ locs, int64_t n, double* out) {
  __shared__ double s[4][1024];
  double a = INFINITY, b = INFINITY, c = -INFINITY, d = -INFINITY;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    double x = locs[2 * i], y = locs[2 * i + 1];
    a = fmin(a, x); b = fmin(b, y); c = fmax(c, x); d = fmax(d, y);
  }
  s[0][threadIdx.x] = a; s[1][threadIdx.x] = b; s[2][threadIdx.x] = c; s[3][threadIdx.x] = d;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      s[0][threadIdx.x] = fmin(s[0][threadIdx.x], s[0][threadIdx.x + o]);
      s[1][threadIdx.x] = fmin(s[1][threadIdx.x], s[1][threadIdx.x + o]);
      s[2][threadIdx.x] = fmax(s[2][threadIdx.x], s[2][threadIdx.x + o]);
      s[3][threadIdx.x] = fmax(s[3][threadIdx.x], s[3][threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 4) out[threadIdx.x] = s[threadIdx.x][0];
}

// non-finite check folded in: counts NaN/inf coordinates
__global__ void k_count_nonfinite(const double* __restrict__ v, int64_t cnt, int* bad) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < cnt && !isfinite(v[i])) atomicAdd(bad, 1);
}

__device__ __forceinline__ int64_t cell_coord(double v, double v0, double h, int64_t g) {
  double q = floor((v - v0) / h);
  if (q < -2.0) q = -2.0;
  if (q > (double)(g + 1)) q = (double)(g + 1);
  return (int64_t)q;
}

__global__ void k_cell_of(const double* __restrict__ locs, int64_t n, GridDesc gd, int* __restrict__ cell,
                          int* __restrict__ count) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t cx = cell_coord(locs[2 * i], gd.x0, gd.h, gd.gx);
  int64_t cy = cell_coord(locs[2 * i + 1], gd.y0, gd.h, gd.gy);
  cx = cx < 0 ? 0 : (cx >= gd.gx ? gd.gx - 1 : cx);
  cy = cy < 0 ? 0 : (cy >= gd.gy ? gd.gy - 1 : cy);
  int c = (int)(cy * gd.gx + cx);
  cell[i] = c;
  atomicAdd(&count[c], 1);
}

__global__ void k_scatter_cell(const int* __restrict__ cell, int64_t n, int* __restrict__ cursor,
                               int* __restrict__ tmp) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int pos = atomicAdd(&cursor[cell[i]], 1);
  tmp[pos] = (int)i;
}

// Final slot of a point: start of its cell plus the number of points of the
// same cell with a smaller original index (stable, deterministic).
// Points of a cell in ascending y (ties by index): the sparse product's
// 16 x 16 blocks of a row group against a neighbour cell then often fall
// entirely outside the taper range and are skipped.
__global__ void k_rank_cell(const int* __restrict__ tmp, const int* __restrict__ cell, const double* __restrict__ locs,
                            const int64_t* __restrict__ cstart, int64_t n, int* __restrict__ perm) {
  int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= n) return;
  int i = tmp[s];
  int c = cell[i];
  const double yi = locs[2 * (int64_t)i + 1];
  int64_t b = cstart[c], e = cstart[c + 1];
  int64_t r = 0;
  for (int64_t k = b; k < e; ++k) {
    const int j = tmp[k];
    const double yj = locs[2 * (int64_t)j + 1];
    r += (yj < yi || (yj == yi && j < i)) ? 1 : 0;
  }
  perm[b + r] = i;
}

__global__ void k_gather_sorted(const double* __restrict__ locs, const int* __restrict__ perm, int64_t n,
                                double* __restrict__ xs, int* __restrict__ iperm) {
  int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= n) return;
  int i = perm[p];
  xs[2 * p] = locs[2 * i];
  xs[2 * p + 1] = locs[2 * i + 1];
  iperm[i] = (int)p;
}

// ------------------------------------------------------------------ scans
// Three-phase exclusive scan of int32 counts into int64 offsets (n+1 values).
constexpr int SCAN_TILE = 4096;

__global__ __launch_bounds__(1024) void k_scan_tiles(const int* __restrict__ in, int64_t n,
                                                     int64_t* __restrict__ tile_sum) {
  __shared__ int64_t s[1024];
  int64_t base = blockIdx.x * (int64_t)SCAN_TILE;
  int64_t acc = 0;
  for (int k = threadIdx.x; k < SCAN_TILE; k += 1024) {
    int64_t i = base + k;
    if (i < n) acc += in[i];
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(1024) void k_scan_tile_sums(int64_t* __restrict__ tile_sum, int64_t ntiles) {
  // sequential carry over chunks of 1024, block scan inside each chunk
  __shared__ int64_t s[1024];
  int64_t carry = 0;
  for (int64_t b = 0; b < ntiles; b += 1024) {
    int64_t i = b + threadIdx.x;
    int64_t v = i < ntiles ? tile_sum[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      int64_t t = threadIdx.x >= o ? s[threadIdx.x - o] : 0;
      __syncthreads();
      s[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < ntiles) tile_sum[i] = carry + s[threadIdx.x] - v;  // exclusive
    int64_t tot = s[1023];
    __syncthreads();
    carry += tot;
  }
  if (threadIdx.x == 0) tile_sum[ntiles] = carry;
}

__global__ __launch_bounds__(1024) void k_scan_apply(const int* __restrict__ in, int64_t n,
                                                     const int64_t* __restrict__ tile_off, int64_t ntiles,
                                                     int64_t* __restrict__ out) {
  __shared__ int64_t s[1024];
  int64_t base = blockIdx.x * (int64_t)SCAN_TILE;
  // each thread owns 4 consecutive elements
  int64_t v[4];
  int64_t loc = 0;
  for (int k = 0; k < 4; ++k) {
    int64_t i = base + threadIdx.x * 4 + k;
    v[k] = i < n ? in[i] : 0;
    loc += v[k];
  }
  s[threadIdx.x] = loc;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    int64_t t = threadIdx.x >= o ? s[threadIdx.x - o] : 0;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  int64_t run = tile_off[blockIdx.x] + s[threadIdx.x] - loc;
  for (int k = 0; k < 4; ++k) {
    int64_t i = base + threadIdx.x * 4 + k;
    if (i < n) out[i] = run;
    run += v[k];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = tile_off[ntiles];
}

fsa_status scan_counts(const int* in, int64_t n, int64_t* out, Buf<int64_t>& scratch, hipStream_t st) {
  int64_t ntiles = ceil_div(n > 0 ? n : 1, SCAN_TILE);
  if (scratch.count < (size_t)(ntiles + 1)) FSA_TRY(scratch.alloc(ntiles + 1));
  hipLaunchKernelGGL(k_scan_tiles, dim3(ntiles), dim3(1024), 0, st, in, n, scratch.p);
  hipLaunchKernelGGL(k_scan_tile_sums, dim3(1), dim3(1024), 0, st, scratch.p, ntiles);
  hipLaunchKernelGGL(k_scan_apply, dim3(ntiles), dim3(1024), 0, st, in, n, scratch.p, ntiles, out);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

// ------------------------------------------------------------------ grid build
__global__ void k_cstart_to_cursor(const int64_t* cstart, int64_t ncell, int* cursor) {
  int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c < ncell) cursor[c] = (int)cstart[c];
}

fsa_status build_grid(Grid& g, const double* locs, int64_t n, double gamma, hipStream_t st, int* bad_flag_dev,
                      const Grid* like) {
  g.n = n;
  FSA_TRY(g.bbox.alloc(4));
  hipLaunchKernelGGL(k_bbox, dim3(1), dim3(1024), 0, st, locs, n, g.bbox.p);
  double bb[4];
  FSA_HIP(hipMemcpyAsync(bb, g.bbox.p, sizeof(bb), hipMemcpyDeviceToHost, st));
  FSA_HIP(hipStreamSynchronize(st));
  if (!(std::isfinite(bb[0]) && std::isfinite(bb[1]) && std::isfinite(bb[2]) && std::isfinite(bb[3]))) {
    set_error("non-finite location coordinates");
    return FSA_ERR_INVALID_ARG;
  }
  GridDesc& gd = g.desc;
  if (like) {
    gd = like->desc;
  } else {
    double h = gamma * (1.0 + 1.0 / 1048576.0);
    double ex = bb[2] - bb[0], ey = bb[3] - bb[1];
    // cap the number of cells at ~4n (+1024): larger cells are still correct
    double cap = 4.0 * (double)n + 1024.0;
    if ((ex / h + 1.0) * (ey / h + 1.0) > cap) {
      double hmin = sqrt(fmax(ex * ey, 0.0) / cap);
      hmin = fmax(hmin, fmax(ex, ey) / cap);
      h = fmax(h, hmin * 1.01);
    }
    gd.x0 = bb[0];
    gd.y0 = bb[1];
    gd.h = h;
    gd.gx = (int64_t)floor(ex / h) + 1;
    gd.gy = (int64_t)floor(ey / h) + 1;
  }
  gd.gamma = gamma;
  int64_t ncell = gd.gx * gd.gy;
  if (ncell > (int64_t)2000000000) {
    set_error("grid too large (%lld cells)", (long long)ncell);
    return FSA_ERR_INVALID_ARG;
  }
  g.ncell = ncell;
  FSA_TRY(g.cell.alloc(n));
  FSA_TRY(g.count.alloc(ncell));
  FSA_TRY(g.cstart.alloc(ncell + 1));
  FSA_TRY(g.perm.alloc(n));
  FSA_TRY(g.iperm.alloc(n));
  FSA_TRY(g.xs.alloc(2 * n));
  Buf<int> tmp, cursor;
  FSA_TRY(tmp.alloc(n));
  FSA_TRY(cursor.alloc(ncell));
  FSA_HIP(hipMemsetAsync(g.count.p, 0, ncell * sizeof(int), st));
  int64_t nb = ceil_div(n, 256);
  hipLaunchKernelGGL(k_cell_of, dim3(nb), dim3(256), 0, st, locs, n, gd, g.cell.p, g.count.p);
  Buf<int64_t> scr;
  FSA_TRY(scan_counts(g.count.p, ncell, g.cstart.p, scr, st));
  hipLaunchKernelGGL(k_cstart_to_cursor, dim3(ceil_div(ncell, 256)), dim3(256), 0, st, g.cstart.p, ncell,
                     cursor.p);
  hipLaunchKernelGGL(k_scatter_cell, dim3(nb), dim3(256), 0, st, g.cell.p, n, cursor.p, tmp.p);
  hipLaunchKernelGGL(k_rank_cell, dim3(nb), dim3(256), 0, st, tmp.p, g.cell.p, locs, g.cstart.p, n, g.perm.p);
  hipLaunchKernelGGL(k_gather_sorted, dim3(nb), dim3(256), 0, st, locs, g.perm.p, n, g.xs.p, g.iperm.p);
  FSA_HIP(hipGetLastError());
  FSA_HIP(hipStreamSynchronize(st));  // tmp/cursor go back to the pool
  (void)bad_flag_dev;
  return FSA_OK;
}


// ------------------------------------------------------------------ pattern
// Rows: points of set R in R's sorted order (coordinates xr).  Columns:
// points of set C in C's sorted order, binned by grid gc.
template <bool FILL>
__global__ __launch_bounds__(256) void k_pattern(const double* __restrict__ xr, int64_t nr, const double* __restrict__ xc,
                                                 const int64_t* __restrict__ cstart, GridDesc gc,
                                                 int* __restrict__ count, const int64_t* __restrict__ row_ptr,
                                                 int* __restrict__ col) {
#pragma clang fp contract(off)
  int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= nr) return;
  const double px = xr[2 * p], py = xr[2 * p + 1];
  const double g2 = gc.gamma * gc.gamma;
  int64_t cx = cell_coord(px, gc.x0, gc.h, gc.gx);
  int64_t cy = cell_coord(py, gc.y0, gc.h, gc.gy);
  int64_t cnt = 0;
  int64_t out = FILL ? row_ptr[p] : 0;
  for (int64_t yy = cy - 1; yy <= cy + 1; ++yy) {
    if (yy < 0 || yy >= gc.gy) continue;
    int64_t xlo = cx - 1 < 0 ? 0 : cx - 1;
    int64_t xhi = cx + 1 >= gc.gx ? gc.gx - 1 : cx + 1;
    if (xlo > xhi) continue;
    int64_t b = cstart[yy * gc.gx + xlo], e = cstart[yy * gc.gx + xhi + 1];
    for (int64_t q = b; q < e; ++q) {
      double dx = px - xc[2 * q];
      double dy = py - xc[2 * q + 1];
      double dx2 = dx * dx;
      double dy2 = dy * dy;
      double d2 = dx2 + dy2;
      if (d2 < g2) {
        if (FILL) col[out++] = (int)q;
        else ++cnt;
      }
    }
  }
  if (!FILL) count[p] = (int)cnt;
}

// Sparse-product keys (see Csr::key): one workgroup per row cell.
__global__ __launch_bounds__(256) void k_pattern_keys(const int64_t* __restrict__ rcs, const int64_t* __restrict__ ccs,
                                                      GridDesc gd, const int64_t* __restrict__ rp,
                                                      const int* __restrict__ col, int* __restrict__ key,
                                                      unsigned long long* __restrict__ stats) {
  const int64_t cell = blockIdx.x;
  const int64_t rb = rcs[cell], re = rcs[cell + 1];
  if (rb >= re) return;
  int qb[3], qe[3], off[3];
  cell_ranges(cell, gd, ccs, qb, qe, off);
  if (threadIdx.x == 0) {
    int qlo = 0x7fffffff, qhi = 0;
    for (int t = 0; t < 3; ++t)
      if (qe[t] > qb[t]) {
        qlo = min(qlo, qb[t]);
        qhi = max(qhi, qe[t]);
      }
    atomicMax(&stats[0], (unsigned long long)(qhi > 0 ? qhi - qlo : 0));
    for (int64_t g0 = rb; g0 < re; g0 += 32)
      atomicMax(&stats[1], (unsigned long long)(rp[min(g0 + 32, re)] - rp[g0]));
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int64_t p = rb + w; p < re; p += 4) {
    const int rowbits = (int)((p - rb) & 31) << KEY_SLOT_BITS;
    for (int64_t e = rp[p] + lane; e < rp[p + 1]; e += 64) {
      const int q = col[e];
      int v;
      if (q >= qb[2] && q < qe[2]) v = q - qb[2] + off[2];
      else if (q >= qb[1] && q < qe[1]) v = q - qb[1] + off[1];
      else v = q - qb[0] + off[0];
      key[e] = rowbits | v;
    }
  }
}

fsa_status build_pattern(const Grid& rows, const Grid& cols, Csr& csr, hipStream_t st) {
  int64_t nr = rows.n;
  if (cols.n > KEY_SLOT_MASK) {
    set_error("at most %d points per point set", KEY_SLOT_MASK);
    return FSA_ERR_INVALID_ARG;
  }
  csr.nrows = nr;
  Buf<int> cnt;
  FSA_TRY(cnt.alloc(nr));
  FSA_TRY(csr.row_ptr.alloc(nr + 1));
  int64_t nb = ceil_div(nr, 256);
  hipLaunchKernelGGL(k_pattern<false>, dim3(nb), dim3(256), 0, st, rows.xs.p, nr, cols.xs.p, cols.cstart.p,
                     cols.desc, cnt.p, (const int64_t*)nullptr, (int*)nullptr);
  Buf<int64_t> scr;
  FSA_TRY(scan_counts(cnt.p, nr, csr.row_ptr.p, scr, st));
  int64_t nnz = 0;
  FSA_HIP(hipMemcpyAsync(&nnz, csr.row_ptr.p + nr, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  FSA_HIP(hipStreamSynchronize(st));
  if (nnz > (int64_t)INT32_MAX * 4) {
    set_error("taper pattern too large (%lld nonzeros)", (long long)nnz);
    return FSA_ERR_INVALID_ARG;
  }
  csr.nnz = nnz;
  FSA_TRY(csr.col.alloc(nnz));
  hipLaunchKernelGGL(k_pattern<true>, dim3(nb), dim3(256), 0, st, rows.xs.p, nr, cols.xs.p, cols.cstart.p,
                     cols.desc, (int*)nullptr, csr.row_ptr.p, csr.col.p);
  FSA_HIP(hipGetLastError());
  FSA_TRY(csr.key.alloc(nnz > 0 ? nnz : 1));
  csr.max_window = csr.max_group_nnz = 0;
  if (rows.ncell > 0 && nnz > 0) {
    Buf<unsigned long long> stats;
    FSA_TRY(stats.alloc(2));
    FSA_HIP(hipMemsetAsync(stats.p, 0, 2 * sizeof(unsigned long long), st));
    hipLaunchKernelGGL(k_pattern_keys, dim3(rows.ncell), dim3(256), 0, st, rows.cstart.p, cols.cstart.p, cols.desc,
                       csr.row_ptr.p, csr.col.p, csr.key.p, stats.p);
    FSA_HIP(hipGetLastError());
    unsigned long long h[2] = {0, 0};
    FSA_HIP(hipMemcpyAsync(h, stats.p, sizeof(h), hipMemcpyDeviceToHost, st));
    FSA_HIP(hipStreamSynchronize(st));
    csr.max_window = (int64_t)h[0];
    csr.max_group_nnz = (int64_t)h[1];
  }
  FSA_HIP(hipStreamSynchronize(st));
  return FSA_OK;
}

// ------------------------------------------------------------------ export
// Row i (caller order) = sorted row iperm[i]; its columns mapped through the
// column set's perm and sorted ascending (rows are short: insertion sort).
__global__ void k_export_counts(const int64_t* __restrict__ rp, const int* __restrict__ iperm, int64_t n,
                                int* __restrict__ cnt) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int p = iperm[i];
  cnt[i] = (int)(rp[p + 1] - rp[p]);
}

__global__ void k_export_fill(const int64_t* __restrict__ rp, const int* __restrict__ col, const double* __restrict__ val,
                              const int* __restrict__ iperm_rows, const int* __restrict__ perm_cols, int64_t n,
                              const int64_t* __restrict__ orp, int* __restrict__ ocol, double* __restrict__ oval) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int p = iperm_rows[i];
  int64_t b = rp[p], e = rp[p + 1], o = orp[i];
  for (int64_t k = b; k < e; ++k) {
    int c = perm_cols[col[k]];
    double v = val ? val[k] : 0.0;
    int64_t pos = o + (k - b);
    // insertion into the sorted prefix [o, pos)
    while (pos > o && ocol[pos - 1] > c) {
      ocol[pos] = ocol[pos - 1];
      if (val) oval[pos] = oval[pos - 1];
      --pos;
    }
    ocol[pos] = c;
    if (val) oval[pos] = v;
  }
}

fsa_status export_csr(const Csr& csr, const Grid& rows, const Grid& cols, const double* val_dev, int64_t* row_ptr_h,
                      int* col_h, double* val_h, hipStream_t st) {
  int64_t n = csr.nrows;
  Buf<int> cnt;
  Buf<int64_t> orp, scr;
  Buf<int> ocol;
  Buf<double> oval;
  FSA_TRY(cnt.alloc(n));
  FSA_TRY(orp.alloc(n + 1));
  FSA_TRY(ocol.alloc(csr.nnz));
  if (val_h) FSA_TRY(oval.alloc(csr.nnz));
  int64_t nb = ceil_div(n, 256);
  hipLaunchKernelGGL(k_export_counts, dim3(nb), dim3(256), 0, st, csr.row_ptr.p, rows.iperm.p, n, cnt.p);
  FSA_TRY(scan_counts(cnt.p, n, orp.p, scr, st));
  hipLaunchKernelGGL(k_export_fill, dim3(nb), dim3(256), 0, st, csr.row_ptr.p, csr.col.p,
                     val_h ? val_dev : (const double*)nullptr, rows.iperm.p, cols.perm.p, n, orp.p, ocol.p,
                     val_h ? oval.p : (double*)nullptr);
  FSA_HIP(hipGetLastError());
  FSA_HIP(hipMemcpyAsync(row_ptr_h, orp.p, (n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  FSA_HIP(hipMemcpyAsync(col_h, ocol.p, csr.nnz * sizeof(int), hipMemcpyDeviceToHost, st));
  if (val_h) FSA_HIP(hipMemcpyAsync(val_h, oval.p, csr.nnz * sizeof(double), hipMemcpyDeviceToHost, st));
  FSA_HIP(hipStreamSynchronize(st));
  return FSA_OK;
}

}  // namespace fsa
