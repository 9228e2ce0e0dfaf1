// Iterative methods for Vecchia approximations with the FITC preconditioner
// (Section 5): the Vecchia factor of the latent process, products with
// Sigma_V = B^{-1} D B^{-T} by level-scheduled triangular solves, block PCG
// on Sigma_V + W^{-1} preconditioned by P = Sigma_mn^T Sigma_m^{-1} Sigma_mn
// + D_s (D_s = diag(Sigma - Sigma_mn^T Sigma_m^{-1} Sigma_mn) + W^{-1}), the
// solve (Sigma_V^{-1} + W)^{-1} v = W^{-1} (Sigma_V + W^{-1})^{-1} Sigma_V v
// and the SLQ estimate of log det(Sigma_V^{-1} + W).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include <hipcub/hipcub.hpp>

#include "common.hpp"
#include "kernels.hpp"
#include "ops.hpp"

namespace fsa {
namespace {

constexpr int VMV_MAX = 32;   // largest neighbour count (lists held in LDS)
constexpr int KNN_TPB = 128;  // points per neighbour-search workgroup
constexpr int KNN_TILE = 256; // earlier points staged per LDS tile

// ---------------------------------------------------------------- neighbours
// N(i) = the min(mv, i) nearest of points 0 .. i-1, ordered by (squared
// distance, index), -1 past the list.  One thread per point scans the
// earlier points in LDS tiles and keeps its sorted list in LDS
// ([slot][thread]).  Squared distances are dx*dx + dy*dy without fused
// multiply-add, so that the choice is the one a plain float64 evaluation
// makes.
__global__ __launch_bounds__(KNN_TPB) void k_vknn(const double* __restrict__ xs, int64_t n, int mv,
                                                  int* __restrict__ nbr) {
#pragma clang fp contract(off)
  __shared__ double tx[KNN_TILE], ty[KNN_TILE];
  __shared__ double sd[VMV_MAX][KNN_TPB];
  __shared__ int sj[VMV_MAX][KNN_TPB];
  const int t = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * KNN_TPB;
  const int64_t i = i0 + t;
  const bool live = i < n;
  const double px = live ? xs[2 * i] : 0.0, py = live ? xs[2 * i + 1] : 0.0;
  const int k = live ? (int)min<int64_t>(mv, i) : 0;
  int cnt = 0;
  double worst = INFINITY;
  const int64_t jend = min(i0 + KNN_TPB, n);
  for (int64_t j0 = 0; j0 < jend; j0 += KNN_TILE) {
    __syncthreads();
    for (int q = t; q < KNN_TILE; q += KNN_TPB) {
      const int64_t j = j0 + q;
      tx[q] = j < n ? xs[2 * j] : 0.0;
      ty[q] = j < n ? xs[2 * j + 1] : 0.0;
    }
    __syncthreads();
    const int lim = k > 0 ? (int)min<int64_t>(KNN_TILE, i - j0) : 0;
    for (int q = 0; q < lim; ++q) {
      const double dx = tx[q] - px;
      const double dy = ty[q] - py;
      const double dx2 = dx * dx;
      const double dy2 = dy * dy;
      const double d2 = dx2 + dy2;
      if (cnt < k || d2 < worst) {
        // the new index is larger than every listed one: it goes after all
        // entries of equal distance; a full list drops its last entry
        int p = cnt < k ? cnt : k - 1;
        while (p > 0 && sd[p - 1][t] > d2) {
          sd[p][t] = sd[p - 1][t];
          sj[p][t] = sj[p - 1][t];
          --p;
        }
        sd[p][t] = d2;
        sj[p][t] = (int)(j0 + q);
        if (cnt < k) ++cnt;
        worst = cnt == k ? sd[k - 1][t] : INFINITY;
      }
    }
  }
  if (!live) return;
  for (int s = 0; s < mv; ++s) nbr[i * mv + s] = s < cnt ? sj[s][t] : -1;
}

// ---------------------------------------------------------------- factor
// A_i = Sigma_{N(i),i}^T Sigma_{N(i)}^{-1} and D_i = Sigma_ii - A_i
// Sigma_{N(i),i} (Section 5.1): one wave per point, Sigma_{N(i)} factored by
// Cholesky in LDS.  D_i is taken as sigma1^2 - |L^{-1} Sigma_{N(i),i}|^2 (the
// same number).  info[0] counts points whose matrix is not positive definite
// or whose D_i is not positive.
__global__ __launch_bounds__(64) void k_vfactor(const double* __restrict__ xs, int64_t n, int mv,
                                                const int* __restrict__ nbr, Theta th, double* __restrict__ coef,
                                                double* __restrict__ Dv, int* __restrict__ info) {
  __shared__ double S[VMV_MAX][VMV_MAX + 1];
  __shared__ double r[VMV_MAX];
  __shared__ double nx[VMV_MAX], ny[VMV_MAX];
  const int64_t i = blockIdx.x;
  const int lane = threadIdx.x;
  const int my = lane < mv ? nbr[i * mv + lane] : -1;
  const int k = __popcll(__ballot(my >= 0));
  const double px = xs[2 * i], py = xs[2 * i + 1];
  if (lane < k) {
    nx[lane] = xs[2 * (int64_t)my];
    ny[lane] = xs[2 * (int64_t)my + 1];
  }
  __syncthreads();
  for (int e = lane; e < k * k; e += 64) {
    const int a = e / k, b = e - a * k;
    const double dx = nx[a] - nx[b], dy = ny[a] - ny[b];
    S[a][b] = cov_d(sqrt(dx * dx + dy * dy), th);
  }
  if (lane < k) {
    const double dx = nx[lane] - px, dy = ny[lane] - py;
    r[lane] = cov_d(sqrt(dx * dx + dy * dy), th);
  }
  __syncthreads();
  bool ok = true;
  for (int j = 0; j < k; ++j) {
    const double djj = S[j][j];
    if (!(djj > 0.0) || !isfinite(djj)) {  // uniform: every lane read the same value
      ok = false;
      break;
    }
    const double l = sqrt(djj);
    __syncthreads();
    if (lane == j) S[j][j] = l;
    if (lane > j && lane < k) S[lane][j] /= l;
    __syncthreads();
    const int w = k - j - 1;
    for (int e = lane; e < w * w; e += 64) {
      const int a = j + 1 + e / w, b = j + 1 + e % w;
      if (b <= a) S[a][b] -= S[a][j] * S[b][j];
    }
    __syncthreads();
  }
  double D = th.s1;
  if (ok) {
    for (int j = 0; j < k; ++j) {  // L y = r (y overwrites r)
      const double yj = r[j] / S[j][j];
      __syncthreads();
      if (lane == j) r[j] = yj;
      if (lane > j && lane < k) r[lane] -= S[lane][j] * yj;
      __syncthreads();
    }
    D = th.s1 - wave_sum(lane < k ? r[lane] * r[lane] : 0.0);
    for (int j = k - 1; j >= 0; --j) {  // L^T a = y (a overwrites r)
      const double aj = r[j] / S[j][j];
      __syncthreads();
      if (lane == j) r[j] = aj;
      if (lane < j) r[lane] -= S[j][lane] * aj;
      __syncthreads();
    }
  }
  if (!(D > 0.0) || !isfinite(D)) ok = false;
  if (lane < mv) coef[i * mv + lane] = (ok && lane < k) ? r[lane] : 0.0;
  if (lane == 0) {
    Dv[i] = ok ? D : 1.0;
    if (!ok) atomicAdd(info, 1);
  }
}

// ---------------------------------------------------------------- schedule
// level[i] = 0 without neighbours, else 1 + max level of N(i): relaxed in
// place (values only grow toward the fixed point; every neighbour has a
// smaller index, so depth + 1 sweeps settle it).
__global__ void k_vlevel(const int* __restrict__ nbr, int64_t n, int mv, int* level, int* changed) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int L = 0;
  for (int s = 0; s < mv; ++s) {
    const int j = nbr[i * mv + s];
    if (j < 0) break;
    L = max(L, level[j] + 1);
  }
  if (L != level[i]) {
    level[i] = L;
    changed[0] = 1;
  }
}

__global__ void k_vlevel_hist(const int* __restrict__ level, int64_t n, int* cnt, int* maxlev) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  atomicAdd(&cnt[level[i]], 1);
  atomicMax(maxlev, level[i]);
}

__global__ void k_vmaxlevel(const int* __restrict__ level, int64_t n, int* maxlev) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) atomicMax(maxlev, level[i]);
}

__global__ void k_viota(int* __restrict__ p, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = (int)i;
}

// children of each point (the rows of B^T): counts, then fill, then each
// list sorted by child index so that sums run in a fixed order
__global__ void k_vchild_count(const int* __restrict__ nbr, int64_t n, int mv, int* cnt) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * mv) return;
  const int j = nbr[e];
  if (j >= 0) atomicAdd(&cnt[j], 1);
}

__global__ void k_vchild_fill(const int* __restrict__ nbr, const double* __restrict__ coef, int64_t n, int mv,
                              const int64_t* __restrict__ cptr, int* cursor, int* __restrict__ ci,
                              double* __restrict__ cv) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * mv) return;
  const int j = nbr[e];
  if (j < 0) return;
  const int64_t pos = cptr[j] + atomicAdd(&cursor[j], 1);
  ci[pos] = (int)(e / mv);
  cv[pos] = coef[e];
}

__global__ void k_vchild_sort(const int64_t* __restrict__ cptr, int64_t n, int* ci, double* cv) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int64_t b = cptr[j], e = cptr[j + 1];
  for (int64_t p = b + 1; p < e; ++p) {
    const int key = ci[p];
    const double val = cv[p];
    int64_t q = p - 1;
    while (q >= b && ci[q] > key) {
      ci[q + 1] = ci[q];
      cv[q + 1] = cv[q];
      --q;
    }
    ci[q + 1] = key;
    cv[q + 1] = val;
  }
}

// Child lists padded per level: every point of level l gets stride_l slots
// (the level's longest list), its children first and -1 after, at poff[p],
// so a product finds a list from the launch's level base and the position
// alone.  stride_l >= the list's length by construction.
__global__ void k_vchild_pad(const int64_t* __restrict__ cptr, int64_t n, const int* __restrict__ ci,
                             const double* __restrict__ cv, const int64_t* __restrict__ poff, int* __restrict__ pci,
                             double* __restrict__ pcv) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int64_t b = cptr[p], len = cptr[p + 1] - b;
  const int64_t o = poff[p], w = poff[p + 1] - o;
  for (int64_t j = 0; j < w; ++j) {
    pci[o + j] = j < len ? ci[b + j] : -1;
    pcv[o + j] = j < len ? cv[b + j] : 0.0;
  }
}

// ---------------------------------------------------------------- B products
__device__ __forceinline__ double readlane_d(double v, int l) {
  const int2 u = __builtin_bit_cast(int2, v);
  return __builtin_bit_cast(double, make_int2(__builtin_amdgcn_readlane(u.x, l), __builtin_amdgcn_readlane(u.y, l)));
}

// Points, lists and block rows are stored in level order, so level l is the
// range of positions [base, base + cnt) and a list holds positions.  The
// k-th point's list (neighbours, or children in the padded layout) is the
// stride slots at lbase + k * stride, valid entries first and -1 after.
// One workgroup (NW waves) per point of a level, one lane per column
// (64-column passes).  The list is cut into NW contiguous segments, one per
// wave; a wave loads its segment across its lanes (64 entries at a time) and
// broadcasts it entry by entry (readlane reads a lane whatever the exec
// mask), U row gathers at a time: the round issues the loads of its entries
// that exist before it uses any, so they are in flight together.  The NW
// partial sums are added in a fixed order.  No point of a level is on the
// list of another point of the same level, and only the point's own
// workgroup writes its row, so wave 0 reads that row together with the list:
// the read is off the dependent chain (list, gathers, store).
template <int NW, int U>
__device__ __forceinline__ void vtri_chunk(int iq, double vq, int nq, const double* X, int64_t ld, int c,
                                           double (&acc)[U]) {
  for (int q = 0; q < nq; q += U) {
    double xr[U];
#pragma unroll
    for (int k = 0; k < U; ++k)
      xr[k] = q + k < nq ? X[(int64_t)__builtin_amdgcn_readlane(iq, q + k) * ld + c] : 0.0;
#pragma unroll
    for (int k = 0; k < U; ++k)
      if (q + k < nq) acc[k] += readlane_d(vq, q + k) * xr[k];
  }
}

// Row i of X plus the list [b, e) of entries applied to X's rows; ends with
// a workgroup barrier after the row's store.
template <int NW, int U>
__device__ __forceinline__ void vtri_point(int64_t i, int64_t b, int64_t e, const int* __restrict__ idx,
                                           const double* __restrict__ val, double* X, int64_t ld, int ncols,
                                           double (&part)[NW][64]) {
  const int wq = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t seg = (e - b + NW - 1) / NW;
  const int64_t sb = b + wq * seg < e ? b + wq * seg : e;
  const int64_t se = sb + seg < e ? sb + seg : e;
  // the segment's first 64 entries serve every 64-column pass; the valid
  // entries of a list, and so of each segment, are a prefix
  const int m0 = (int)(se - sb < 64 ? se - sb : 64);
  const int iq0 = lane < m0 ? idx[sb + lane] : -1;
  const double vq0 = lane < m0 ? val[sb + lane] : 0.0;
  // the point's own row for the first pass, issued with the list
  double own = (wq == 0 && lane < ncols) ? X[i * ld + lane] : 0.0;
  for (int c0 = 0; c0 < ncols; c0 += 64) {
    const int c = c0 + lane;
    const bool live = c < ncols;
    const int nq0 = __popcll(__ballot(iq0 >= 0));
    double acc[U];
#pragma unroll
    for (int k = 0; k < U; ++k) acc[k] = 0.0;
    if (live) vtri_chunk<NW, U>(iq0, vq0, nq0, X, ld, c, acc);
    for (int64_t p0 = sb + 64; p0 < se; p0 += 64) {  // segments over 64 entries (lists over 64 NW)
      const int64_t rem = se - p0;
      const int m64 = (int)(rem < 64 ? rem : 64);
      const int iq = lane < m64 ? idx[p0 + lane] : -1;
      const double vq = lane < m64 ? val[p0 + lane] : 0.0;
      const int nq = __popcll(__ballot(iq >= 0));
      if (live) vtri_chunk<NW, U>(iq, vq, nq, X, ld, c, acc);
    }
    double a = acc[0];
#pragma unroll
    for (int k = 1; k < U; ++k) a += acc[k];
    part[wq][lane] = a;
    __syncthreads();
    if (wq == 0 && live) {
      double t = part[0][lane];
      for (int u = 1; u < NW; ++u) t += part[u][lane];
      X[i * ld + c] = own + t;
      own = c + 64 < ncols ? X[i * ld + c + 64] : 0.0;  // the next pass's
    }
    __syncthreads();
  }
}

template <int NW, int U>
__global__ __launch_bounds__(NW * 64) void k_vtri(int base, int cnt, int64_t lbase, int stride,
                                              const int* __restrict__ idx, const double* __restrict__ val, double* X,
                                              int64_t ld, int ncols) {
  __shared__ double part[NW][64];
  if ((int)blockIdx.x >= cnt) return;  // uniform per workgroup
  const int64_t b = lbase + (int64_t)blockIdx.x * stride;
  vtri_point<NW, U>(base + (int64_t)blockIdx.x, b, b + stride, idx, val, X, ld, ncols, part);
}

// A run of consecutive levels of one point each (positions [base, base +
// cnt)) in one workgroup, point after point: ascending over the neighbour
// lists (mv slots at position * mv), descending over the padded child lists
// ([poff[i], poff[i + 1])).  A point's row is stored before the barrier that
// ends its turn, so the later points of the run, whose lists may hold it,
// read it from the same compute unit after that barrier.
template <int NW, int U>
__global__ __launch_bounds__(NW * 64) void k_vtri_run(int base, int cnt, const int64_t* __restrict__ poff, int mv,
                                                  const int* __restrict__ idx, const double* __restrict__ val,
                                                  double* X, int64_t ld, int ncols) {
  __shared__ double part[NW][64];
  for (int k = 0; k < cnt; ++k) {
    const int64_t i = poff ? base + cnt - 1 - k : base + k;
    const int64_t b = poff ? poff[i] : i * mv;
    const int64_t e = poff ? poff[i + 1] : b + mv;
    vtri_point<NW, U>(i, b, e, idx, val, X, ld, ncols, part);
  }
}

// T = (B X) / D: t_i = (x_i - sum_s A_i[s] x_{N(i)[s]}) / D_i
__global__ __launch_bounds__(256) void k_vB_div(int64_t n, const int* __restrict__ nbr, const double* __restrict__ coef,
                                                int mv, const double* __restrict__ Dv, const double* __restrict__ X,
                                                int64_t ldx, int ncols, double* __restrict__ T, int64_t ldt) {
  const int64_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  for (int c = lane; c < ncols; c += 64) {
    double acc = X[i * ldx + c];
    for (int s = 0; s < mv; ++s) {
      const int j = nbr[i * mv + s];
      if (j < 0) break;
      acc -= coef[i * mv + s] * X[(int64_t)j * ldx + c];
    }
    T[i * ldt + c] = acc / Dv[i];
  }
}

// Y = B^T T: y_j = t_j - sum over children i of A_i[s] t_i
__global__ __launch_bounds__(256) void k_vBt(int64_t n, const int64_t* __restrict__ cptr, const int* __restrict__ ci,
                                             const double* __restrict__ cv, const double* __restrict__ T, int64_t ldt,
                                             int ncols, double* __restrict__ Y, int64_t ldy) {
  const int64_t j = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= n) return;
  const int64_t b = cptr[j], e = cptr[j + 1];
  for (int c = lane; c < ncols; c += 64) {
    double acc = T[j * ldt + c];
    for (int64_t p = b; p < e; ++p) acc -= cv[p] * T[(int64_t)ci[p] * ldt + c];
    Y[j * ldy + c] = acc;
  }
}

// ---------------------------------------------------------------- level order
__global__ void k_vposof(const int* __restrict__ order, int64_t n, int* __restrict__ posof) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p < n) posof[order[p]] = (int)p;
}

// the factor, D, W and the locations in level order; neighbour lists hold positions
__global__ void k_vperm(const int* __restrict__ order, const int* __restrict__ posof, int64_t n, int mv,
                        const int* __restrict__ nbr, const double* __restrict__ coef, const double* __restrict__ Dv,
                        const double* __restrict__ w, const double* __restrict__ xs, int* __restrict__ fnbr,
                        double* __restrict__ fcoef, double* __restrict__ Dvp, double* __restrict__ wp,
                        double* __restrict__ xsp) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int64_t i = order[p];
  for (int s = 0; s < mv; ++s) {
    const int j = nbr[i * mv + s];
    fnbr[p * mv + s] = j < 0 ? -1 : posof[j];
    fcoef[p * mv + s] = coef[i * mv + s];
  }
  Dvp[p] = Dv[i];
  wp[p] = w[i];
  xsp[2 * p] = xs[2 * i];
  xsp[2 * p + 1] = xs[2 * i + 1];
}

// Y[p] = X[order[p]] (into level order) / Y[order[p]] = X[p] (back)
__global__ void k_vgather(int64_t n, int ncols, const double* __restrict__ X, int64_t ldx,
                          const int* __restrict__ order, double* __restrict__ Y, int64_t ldy) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * ncols) return;
  const int64_t p = e / ncols;
  const int c = (int)(e - p * ncols);
  Y[p * ldy + c] = X[(int64_t)order[p] * ldx + c];
}

__global__ void k_vscatter(int64_t n, int ncols, const double* __restrict__ X, int64_t ldx,
                           const int* __restrict__ order, double* __restrict__ Y, int64_t ldy) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * ncols) return;
  const int64_t p = e / ncols;
  const int c = (int)(e - p * ncols);
  Y[(int64_t)order[p] * ldy + c] = X[p * ldx + c];
}

// ---------------------------------------------------------------- elementwise
__global__ void k_vcopy(int64_t n, int ncols, const double* __restrict__ X, int64_t ldx, double* __restrict__ Y,
                        int64_t ldy) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * ncols) return;
  const int64_t p = e / ncols;
  const int c = (int)(e - p * ncols);
  Y[p * ldy + c] = X[p * ldx + c];
}

// Y = Y * D (rows), or Y += X / w with addw
__global__ void k_vscale_rows(int64_t n, int ncols, double* __restrict__ Y, int64_t ldy, const double* __restrict__ D) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * ncols) return;
  const int64_t p = e / ncols;
  const int c = (int)(e - p * ncols);
  Y[p * ldy + c] *= D[p];
}

__global__ void k_vadd_winv(int64_t n, int ncols, const double* __restrict__ X, int64_t ldx,
                            const double* __restrict__ w, double* __restrict__ Y, int64_t ldy) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * ncols) return;
  const int64_t p = e / ncols;
  const int c = (int)(e - p * ncols);
  Y[p * ldy + c] += X[p * ldx + c] / w[p];
}

// D_s = sigma1^2 - |A_p|^2 + 1 / w_p (the FITC diagonal of Sigma + W^{-1})
__global__ void k_vds(const double* __restrict__ A, int64_t n, int mp, double s1, const double* __restrict__ w,
                      double* __restrict__ Ds) {
  const int64_t p = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (p >= n) return;
  double a = 0.0;
  for (int k = lane; k < mp; k += 64) {
    const double v = A[p * mp + k];
    a += v * v;
  }
  a = wave_sum(a);
  if (lane == 0) Ds[p] = s1 - a + 1.0 / w[p];
}

// Z = (R - T) / D_s
__global__ void k_vprec_finish(int64_t n, int ncols, int64_t ld, const double* __restrict__ R,
                               const double* __restrict__ T, const double* __restrict__ Ds, double* __restrict__ Z) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * ncols) return;
  const int64_t p = e / ncols;
  const int c = (int)(e - p * ncols);
  Z[p * ld + c] = (R[p * ld + c] - T[p * ld + c]) / Ds[p];
}

// sum of log x (count of entries not finite or <= 0 in bad), partials per block
__global__ __launch_bounds__(256) void k_vsumlog_part(const double* __restrict__ x, int64_t n, double* part,
                                                      int* bad) {
  __shared__ double s[256];
  double a = 0.0;
  int nb = 0;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double v = x[i];
    if (!(v > 0.0) || !isfinite(v)) ++nb;
    else a += log(v);
  }
  s[threadIdx.x] = a;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
  if (nb) atomicAdd(bad, nb);
}

__global__ void k_vsum_fixed(const double* __restrict__ part, int np, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double a = 0.0;
  for (int i = 0; i < np; ++i) a += part[i];
  *out = a;
}


// ---------------------------------------------------------------- PCG
// One thread per column.  rz = r^T z, bn2 = |b|^2, active iff |b| > 0.
__global__ void k_vpcg_init(int ncols, const double* __restrict__ rz0, const double* __restrict__ bn2, double* rz,
                            int* active, int* iters, int* flags) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c == 0) {
    flags[0] = 0;
    flags[1] = 0;
  }
  if (c >= ncols) return;
  rz[c] = rz0[c];
  active[c] = bn2[c] > 0.0 ? 1 : 0;
  iters[c] = 0;
}

// alpha = r^T z / h^T K h on active columns (0 elsewhere); a breakdown
// (h^T K h not positive or not finite) sets flags[1]
__global__ void k_vpcg_alpha(int ncols, const double* __restrict__ hv, const double* __restrict__ rz,
                             const int* __restrict__ active, double* alpha, int* flags) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncols) return;
  double a = 0.0;
  if (active[c]) {
    const double h = hv[c];
    if (!(h > 0.0) || !isfinite(h)) atomicOr(&flags[1], 1);
    else a = rz[c] / h;
  }
  alpha[c] = a;
}

// u += alpha h, r -= alpha v (alpha = 0 leaves frozen columns as they are)
__global__ void k_vpcg_update(int64_t n, int ncols, int64_t ld, const double* __restrict__ alpha,
                              const double* __restrict__ H, const double* __restrict__ V, double* __restrict__ U,
                              double* __restrict__ R) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * ncols) return;
  const int64_t p = e / ncols;
  const int c = (int)(e - p * ncols);
  const double a = alpha[c];
  if (a == 0.0) return;
  const int64_t o = p * ld + c;
  U[o] += a * H[o];
  R[o] -= a * V[o];
}

// beta = r'^T z' / r^T z on active columns; the iteration's (alpha, beta)
// appended to the Lanczos history; a column stays active while |r|^2 >=
// tol^2 |b|^2; flags[0] counts the active columns after the iteration
__global__ void k_vpcg_beta(int ncols, const double* __restrict__ rzn, const double* __restrict__ rr,
                            const double* __restrict__ bn2, const double* __restrict__ alpha, double* rz, double* beta,
                            int* active, int* iters, double* ah, double* bh, int max_iter, double tol2, int fixed,
                            int* flags) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncols) return;
  double b = 0.0;
  if (active[c]) {
    b = rzn[c] / rz[c];
    const int it = iters[c];
    if (it < max_iter) {
      ah[(int64_t)it * ncols + c] = alpha[c];
      bh[(int64_t)it * ncols + c] = b;
    }
    iters[c] = it + 1;
    rz[c] = rzn[c];
    if (!isfinite(rzn[c])) atomicOr(&flags[1], 1);
    const int still = (fixed || !(rr[c] < tol2 * bn2[c])) ? 1 : 0;
    active[c] = still;
    if (still) atomicAdd(&flags[0], 1);
  }
  beta[c] = b;
}

// h = z + beta h on the columns of this iteration (beta = 0 elsewhere
// leaves h = z, which no later step reads)
__global__ void k_vpcg_direction(int64_t n, int ncols, int64_t ld, const double* __restrict__ beta,
                                 const double* __restrict__ Z, double* __restrict__ H) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * ncols) return;
  const int64_t p = e / ncols;
  const int c = (int)(e - p * ncols);
  const int64_t o = p * ld + c;
  H[o] = Z[o] + beta[c] * H[o];
}

// x = u_0 / w, back to the caller's order
__global__ void k_vsolution(int64_t n, const double* __restrict__ U, int64_t ld, const double* __restrict__ wp,
                            const int* __restrict__ order, double* __restrict__ x) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p < n) x[order[p]] = U[p * ld] / wp[p];
}

// log det(Sigma_V^{-1} + W) = offset + log det P + mean of the SLQ terms
__global__ void k_vlogdet(const double* __restrict__ terms, int c_first, int ncols, const double* __restrict__ parts,
                          double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double a = 0.0;
  for (int c = c_first; c < ncols; ++c) a += terms[c];
  const double sw = a / (double)(ncols - c_first) + parts[0];
  out[0] = parts[1] + sw;
  out[1] = sw;
}

inline unsigned grid1(int64_t cnt, int tpb = 256) { return (unsigned)ceil_div(cnt > 0 ? cnt : 1, tpb); }

}  // namespace
}  // namespace fsa

using namespace fsa;

struct fsa_vecchia {
  hipStream_t st = nullptr;
  int64_t n = 0;
  int m = 0, mp = 0, mv = 0;
  Theta th{};
  Buf<double> xs, ind, w;
  Buf<int> nbr, level, order, info;  // nbr, coef, Dv, w, xs in the caller's order
  Buf<double> coef, Dv;
  // level order: position p holds point order[p]; fnbr/fcoef list positions
  Buf<int> posof, fnbr;
  Buf<double> fcoef, Dvp, wp, xsp;
  Buf<int64_t> cptr, scan_scratch;
  Buf<int> ci, pci;
  Buf<double> cv, pcv;     // pci, pcv: the child lists padded per level
  Buf<int64_t> ppos;       // position p's padded child list: [ppos[p], ppos[p + 1])
  std::vector<int> lptr;   // level l holds order[lptr[l] .. lptr[l+1])
  std::vector<int> lmaxc;  // longest child list among the points of level l
  std::vector<int64_t> lpoff;  // level l's padded child lists start at lpoff[l]
  // FITC preconditioner of Sigma + W^{-1}
  Buf<double> Sm, Lm, A, Ds, C, LCinv, Cinv, parts;  // parts: [0] log det P, [1] sum log w - sum log D
  Scratch scr;
  double logdet_P = 0.0, offset = 0.0, sum_log_dv = 0.0;
  ~fsa_vecchia() {
    if (st) (void)hipStreamSynchronize(st);
  }
};

// ---------------------------------------------------------------- Vecchia-Laplace (Bernoulli-logit)
// Newton data at latent values b (caller's order) for responses y in {0, 1}:
// pi = 1/(1 + e^{-b}), W = pi (1 - pi) (the negative second derivative of
// the log-likelihood), and rhs = W b + y - pi (with_wb) or y - pi.
__global__ void k_vnewton(int64_t n, const double* __restrict__ b, const double* __restrict__ y, int with_wb,
                          double* __restrict__ w, double* __restrict__ rhs) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double pi = 0.5 * (1.0 + tanh(0.5 * b[i]));
  const double wi = pi * (1.0 - pi);
  w[i] = wi;
  rhs[i] = (with_wb ? wi * b[i] : 0.0) + y[i] - pi;
}

// Per-workgroup partial sums, three per group:
//   mode 0: |x - b|^2, |x|^2, 0;  mode 1: sum y b - log(1 + e^b), 0, 0;  mode 2: x . b, 0, 0
__global__ __launch_bounds__(256) void k_vlaplace_parts(int64_t n, int mode, const double* __restrict__ x,
                                                        const double* __restrict__ b, const double* __restrict__ y,
                                                        double* __restrict__ part) {
  __shared__ double s[3][256];
  double a0 = 0.0, a1 = 0.0;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    if (mode == 0) {
      const double d = x[i] - b[i];
      a0 += d * d;
      a1 += x[i] * x[i];
    } else if (mode == 1) {
      const double bi = b[i];
      const double sp = bi > 0.0 ? bi + log1p(exp(-bi)) : log1p(exp(bi));  // log(1 + e^b)
      a0 += y[i] * bi - sp;
    } else {
      a0 += x[i] * b[i];
    }
  }
  s[0][threadIdx.x] = a0;
  s[1][threadIdx.x] = a1;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      s[0][threadIdx.x] += s[0][threadIdx.x + o];
      s[1][threadIdx.x] += s[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x] = s[0][0];
    part[3 * blockIdx.x + 1] = s[1][0];
    part[3 * blockIdx.x + 2] = 0.0;
  }
}

__global__ void k_vsum3(const double* __restrict__ part, int np, double* __restrict__ out) {
  const int j = threadIdx.x;
  if (j >= 3 || blockIdx.x != 0) return;
  double a = 0.0;
  for (int i = 0; i < np; ++i) a += part[3 * i + j];
  out[j] = a;
}

// count of responses not in {0, 1}
__global__ void k_vcount_nonbinary(int64_t n, const double* __restrict__ y, int* bad) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n && !(y[i] == 0.0 || y[i] == 1.0)) atomicAdd(bad, 1);
}

namespace {

fsa_status sum_log(const double* x, int64_t n, double* out_dev, int* bad_dev, hipStream_t st, Buf<double>& part) {
  const int nb = (int)std::min<int64_t>(grid1(n), 256);
  FSA_TRY(part.alloc(nb));
  hipLaunchKernelGGL(k_vsumlog_part, dim3(nb), dim3(256), 0, st, x, n, part.p, bad_dev);
  hipLaunchKernelGGL(k_vsum_fixed, dim3(1), dim3(64), 0, st, part.p, nb, out_dev);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

// Y = Sigma_V X = B^{-1} (D (B^{-T} X))
fsa_status sigma_v(fsa_vecchia* v, const double* X, int64_t ldx, int ncols, double* Y, int64_t ldy) {
  hipStream_t st = v->st;
  const int64_t n = v->n;
  hipLaunchKernelGGL(k_vcopy, dim3(grid1(n * ncols)), dim3(256), 0, st, n, ncols, X, ldx, Y, ldy);
  const int nlev = (int)v->lptr.size() - 1;
  const auto single = [&](int l) { return v->lptr[l + 1] - v->lptr[l] == 1; };
  // B^{-T}: levels in descending order, each point adding its children's rows
  for (int l = nlev - 1; l >= 0;) {
    const int b = v->lptr[l], cnt = v->lptr[l + 1] - b;
    if (l > 0 && single(l) && single(l - 1)) {
      // levels l0 .. l hold one point each: one workgroup, point after point
      int l0 = l - 1;
      while (l0 > 0 && single(l0 - 1)) --l0;
      hipLaunchKernelGGL((k_vtri_run<16, 8>), dim3(1), dim3(1024), 0, st, v->lptr[l0], l - l0 + 1, v->ppos.p, 0,
                         v->pci.p, v->pcv.p, Y, ldy, ncols);
      l = l0 - 1;
      continue;
    }
    // 16 waves per point where some list of the level exceeds 32 entries,
    // else 4; a wave has 8 row gathers in flight per round.  A level without
    // children (the last) leaves its rows as they are.
    const int w = v->lmaxc[l];
    if (w > 32)
      hipLaunchKernelGGL((k_vtri<16, 8>), dim3((unsigned)cnt), dim3(1024), 0, st, b, cnt, v->lpoff[l], w, v->pci.p,
                         v->pcv.p, Y, ldy, ncols);
    else if (w > 0)
      hipLaunchKernelGGL((k_vtri<4, 8>), dim3((unsigned)cnt), dim3(256), 0, st, b, cnt, v->lpoff[l], w, v->pci.p,
                         v->pcv.p, Y, ldy, ncols);
    --l;
  }
  hipLaunchKernelGGL(k_vscale_rows, dim3(grid1(n * ncols)), dim3(256), 0, st, n, ncols, Y, ldy, v->Dvp.p);
  // B^{-1}: levels in ascending order, each point adding its neighbours' rows
  for (int l = 0; l < nlev;) {
    const int b = v->lptr[l], cnt = v->lptr[l + 1] - b;
    if (l + 1 < nlev && single(l) && single(l + 1)) {
      // levels l .. l1 hold one point each
      int l1 = l + 1;
      while (l1 + 1 < nlev && single(l1 + 1)) ++l1;
      hipLaunchKernelGGL((k_vtri_run<8, 4>), dim3(1), dim3(512), 0, st, b, l1 - l + 1, (const int64_t*)nullptr,
                         v->mv, v->fnbr.p, v->fcoef.p, Y, ldy, ncols);
      l = l1 + 1;
      continue;
    }
    // at most 32 neighbours: 8 waves take four each, all gathers in one round
    hipLaunchKernelGGL((k_vtri<8, 4>), dim3((unsigned)cnt), dim3(512), 0, st, b, cnt, (int64_t)b * v->mv, v->mv,
                       v->fnbr.p, v->fcoef.p, Y, ldy, ncols);
    ++l;
  }
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

// Y = Sigma_V^{-1} X = B^T D^{-1} B X (T: n x ncols scratch)
fsa_status precision_v(fsa_vecchia* v, const double* X, int64_t ldx, int ncols, double* Y, int64_t ldy) {
  hipStream_t st = v->st;
  const int64_t n = v->n;
  Buf<double> T;
  FSA_TRY(T.alloc((size_t)n * ncols));
  hipLaunchKernelGGL(k_vB_div, dim3(grid1(n, 4)), dim3(256), 0, st, n, v->fnbr.p, v->fcoef.p, v->mv, v->Dvp.p, X, ldx,
                     ncols, T.p, (int64_t)ncols);
  hipLaunchKernelGGL(k_vBt, dim3(grid1(n, 4)), dim3(256), 0, st, n, v->cptr.p, v->ci.p, v->cv.p, T.p,
                     (int64_t)ncols, ncols, Y, ldy);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

// Z = P^{-1} R by Woodbury: (R - A C^{-1} A^T D_s^{-1} R) / D_s; T, Wm, G scratch
fsa_status precond(fsa_vecchia* v, const double* R, int64_t ld, int ncols, double* Z, double* T, double* Wm,
                   double* G, int ldw) {
  hipStream_t st = v->st;
  FSA_TRY(lowrank_reduce<double>(v->A.p, v->n, v->mp, R, (int)ld, ncols, v->Ds.p, v->scr, Wm, ldw, st));
  FSA_TRY(mspace_apply<double>(v->Cinv.p, Wm, ldw, v->mp, ncols, G, ldw, st));
  FSA_TRY(lowrank_expand<double>(v->A.p, nullptr, v->n, v->mp, G, ldw, ncols, T, (int)ld, st));
  hipLaunchKernelGGL(k_vprec_finish, dim3(grid1(v->n * ncols)), dim3(256), 0, st, v->n, ncols, ld, R, T, v->Ds.p, Z);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

// Y = (Sigma_V + W^{-1}) X
fsa_status operator_v(fsa_vecchia* v, const double* X, int64_t ldx, int ncols, double* Y, int64_t ldy) {
  FSA_TRY(sigma_v(v, X, ldx, ncols, Y, ldy));
  hipLaunchKernelGGL(k_vadd_winv, dim3(grid1(v->n * ncols)), dim3(256), 0, v->st, v->n, ncols, X, ldx, v->wp.p, Y,
                     ldy);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

// The FITC preconditioner of Sigma + W^{-1} (Section 5.1) for the weights in
// v->w (the caller's order), on the factor A built once: W in level order,
// D_s = sigma1^2 - |A_p|^2 + 1/W, C = I + A D_s^{-1} A^T with its Cholesky
// factor, inverse and log det, and the log-determinant offset
// sum log W - sum log D.  The Vecchia factor does not depend on W.
fsa_status set_weights(fsa_vecchia* v) {
  hipStream_t st = v->st;
  const int64_t n = v->n;
  const int mp = v->mp;
  int hinfo[2] = {0, 0};
  FSA_HIP(hipMemsetAsync(v->info.p, 0, 4 * sizeof(int), st));
  Buf<double> part, part2, part3;
  FSA_TRY(sum_log(v->w.p, n, v->parts.p + 2, v->info.p + 1, st, part3));
  hipLaunchKernelGGL(k_vgather, dim3(grid1(n)), dim3(256), 0, st, n, 1, v->w.p, (int64_t)1, v->order.p, v->wp.p,
                     (int64_t)1);
  FSA_TRY(v->Ds.alloc(n));
  hipLaunchKernelGGL(k_vds, dim3(grid1(n, 4)), dim3(256), 0, st, v->A.p, n, mp, v->th.s1, v->wp.p, v->Ds.p);
  FSA_TRY(v->C.alloc((size_t)mp * mp));
  FSA_TRY(capacitance(v->A.p, v->Ds.p, n, mp, v->C.p, v->scr, st));
  FSA_TRY(dense_cholesky(v->C.p, mp, v->info.p, st));
  FSA_TRY(dense_logdet_chol(v->C.p, mp, v->parts.p, st));
  FSA_TRY(v->LCinv.alloc((size_t)mp * mp));
  FSA_TRY(v->Cinv.alloc((size_t)mp * mp));
  FSA_TRY(tri_inverse(v->C.p, v->LCinv.p, mp, st));
  FSA_TRY(dense_gemm(v->LCinv.p, true, v->LCinv.p, false, v->Cinv.p, mp, 1.0, st));
  // sums of logs: [1] log D_s, [2] log W, [3] log D (Vecchia)
  FSA_TRY(sum_log(v->Ds.p, n, v->parts.p + 1, v->info.p + 1, st, part));
  FSA_TRY(sum_log(v->Dv.p, n, v->parts.p + 3, v->info.p + 1, st, part2));
  double hp[4];
  FSA_HIP(hipMemcpyAsync(hp, v->parts.p, sizeof(hp), hipMemcpyDeviceToHost, st));
  FSA_HIP(hipMemcpyAsync(hinfo, v->info.p, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
  FSA_HIP(hipStreamSynchronize(st));
  if (hinfo[0]) {
    set_error("Cholesky of the FITC capacitance failed at column %d", hinfo[0] - 1);
    return FSA_ERR_NOT_SPD;
  }
  if (hinfo[1]) {
    set_error("a weight W or the FITC diagonal D_s is not finite and positive");
    return FSA_ERR_NOT_SPD;
  }
  v->logdet_P = hp[0] + hp[1];
  v->offset = hp[2] - hp[3];
  v->sum_log_dv = hp[3];
  // parts[0] = log det P, parts[1] = sum log w - sum log D (read by k_vlogdet)
  const double hp2[2] = {v->logdet_P, v->offset};
  FSA_HIP(hipMemcpyAsync(v->parts.p, hp2, sizeof(hp2), hipMemcpyHostToDevice, st));
  FSA_HIP(hipStreamSynchronize(st));
  return FSA_OK;
}

fsa_status build(fsa_vecchia* v, const double* locs, const double* inducing, const double* w) {
  hipStream_t st = v->st;
  const int64_t n = v->n;
  const int mv = v->mv, mp = v->mp;
  FSA_TRY(v->info.alloc(4));
  FSA_HIP(hipMemsetAsync(v->info.p, 0, 4 * sizeof(int), st));
  FSA_TRY(v->xs.alloc(2 * (size_t)n));
  FSA_TRY(v->w.alloc(n));
  FSA_TRY(v->ind.alloc(2 * (size_t)mp));
  FSA_HIP(hipMemcpyAsync(v->xs.p, locs, 2 * n * sizeof(double), hipMemcpyDeviceToDevice, st));
  FSA_HIP(hipMemcpyAsync(v->w.p, w, n * sizeof(double), hipMemcpyDeviceToDevice, st));
  FSA_HIP(hipMemsetAsync(v->ind.p, 0, 2 * (size_t)mp * sizeof(double), st));
  FSA_HIP(hipMemcpyAsync(v->ind.p, inducing, 2 * (size_t)v->m * sizeof(double), hipMemcpyDeviceToDevice, st));
  // sum log w (also rejects w not finite and positive)
  FSA_TRY(v->parts.alloc(4));
  Buf<double> part;
  FSA_TRY(sum_log(v->w.p, n, v->parts.p + 2, v->info.p + 1, st, part));
  // neighbours, factor
  FSA_TRY(v->nbr.alloc((size_t)n * std::max(mv, 1)));
  FSA_TRY(v->coef.alloc((size_t)n * std::max(mv, 1)));
  FSA_TRY(v->Dv.alloc(n));
  if (mv > 0) {
    hipLaunchKernelGGL(k_vknn, dim3(grid1(n, KNN_TPB)), dim3(KNN_TPB), 0, st, v->xs.p, n, mv, v->nbr.p);
  }
  hipLaunchKernelGGL(k_vfactor, dim3((unsigned)n), dim3(64), 0, st, v->xs.p, n, mv, v->nbr.p, v->th, v->coef.p,
                     v->Dv.p, v->info.p);
  FSA_HIP(hipGetLastError());
  int hinfo[2] = {0, 0};
  FSA_HIP(hipMemcpyAsync(hinfo, v->info.p, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
  FSA_HIP(hipStreamSynchronize(st));
  if (hinfo[1]) {
    set_error("%d weights W are not finite and positive", hinfo[1]);
    return FSA_ERR_INVALID_ARG;
  }
  if (hinfo[0]) {
    set_error("Vecchia factor: %d points have a conditioning matrix that is not positive definite "
              "(duplicate locations?)", hinfo[0]);
    return FSA_ERR_NOT_SPD;
  }
  // level schedule: relax until a batch of sweeps changes nothing
  FSA_TRY(v->level.alloc(n));
  FSA_HIP(hipMemsetAsync(v->level.p, 0, n * sizeof(int), st));
  {
    const int batch = 16;
    int64_t sweeps = 0;
    for (;;) {
      FSA_HIP(hipMemsetAsync(v->info.p + 2, 0, sizeof(int), st));
      for (int b = 0; b < batch; ++b)
        hipLaunchKernelGGL(k_vlevel, dim3(grid1(n)), dim3(256), 0, st, v->nbr.p, n, mv, v->level.p, v->info.p + 2);
      FSA_HIP(hipGetLastError());
      int changed = 0;
      FSA_HIP(hipMemcpyAsync(&changed, v->info.p + 2, sizeof(int), hipMemcpyDeviceToHost, st));
      FSA_HIP(hipStreamSynchronize(st));
      sweeps += batch;
      if (!changed) break;
      if (sweeps > n + 2 * batch) {
        set_error("Vecchia level schedule did not settle");
        return FSA_ERR_DEVICE;
      }
    }
  }
  int maxlev = 0;
  FSA_HIP(hipMemsetAsync(v->info.p + 3, 0, sizeof(int), st));
  hipLaunchKernelGGL(k_vmaxlevel, dim3(grid1(n)), dim3(256), 0, st, v->level.p, n, v->info.p + 3);
  FSA_HIP(hipMemcpyAsync(&maxlev, v->info.p + 3, sizeof(int), hipMemcpyDeviceToHost, st));
  FSA_HIP(hipStreamSynchronize(st));
  const int nlev = maxlev + 1;
  {
    Buf<int> cnt;
    FSA_TRY(cnt.alloc(nlev));
    FSA_HIP(hipMemsetAsync(cnt.p, 0, nlev * sizeof(int), st));
    hipLaunchKernelGGL(k_vlevel_hist, dim3(grid1(n)), dim3(256), 0, st, v->level.p, n, cnt.p, v->info.p + 3);
    std::vector<int> hc(nlev);
    FSA_HIP(hipMemcpyAsync(hc.data(), cnt.p, nlev * sizeof(int), hipMemcpyDeviceToHost, st));
    FSA_HIP(hipStreamSynchronize(st));
    v->lptr.assign(nlev + 1, 0);
    for (int l = 0; l < nlev; ++l) v->lptr[l + 1] = v->lptr[l] + hc[l];
    if (v->lptr[nlev] != n) {
      set_error("Vecchia level schedule: %d points counted of %lld", v->lptr[nlev], (long long)n);
      return FSA_ERR_DEVICE;
    }
    // points grouped by level, in index order inside a level: a stable radix
    // sort of (level, index), so positions, and every sum over them, are the
    // same on every build
    FSA_TRY(v->order.alloc(n));
    {
      Buf<int> keys_out, idx;
      FSA_TRY(keys_out.alloc(n));
      FSA_TRY(idx.alloc(n));
      hipLaunchKernelGGL(k_viota, dim3(grid1(n)), dim3(256), 0, st, idx.p, n);
      FSA_HIP(hipGetLastError());
      int end_bit = 1;
      while (end_bit < 31 && (1 << end_bit) <= maxlev) ++end_bit;
      size_t tb = 0;
      FSA_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, v->level.p, keys_out.p, idx.p, v->order.p, (int)n, 0,
                                                 end_bit, st));
      Buf<char> tmp;
      FSA_TRY(tmp.alloc(tb));
      FSA_HIP(hipcub::DeviceRadixSort::SortPairs((void*)tmp.p, tb, v->level.p, keys_out.p, idx.p, v->order.p, (int)n, 0,
                                                 end_bit, st));
      FSA_HIP(hipStreamSynchronize(st));  // the sort's buffers and cnt leave scope
    }
  }
  // level order
  FSA_TRY(v->posof.alloc(n));
  FSA_TRY(v->fnbr.alloc((size_t)n * std::max(mv, 1)));
  FSA_TRY(v->fcoef.alloc((size_t)n * std::max(mv, 1)));
  FSA_TRY(v->Dvp.alloc(n));
  FSA_TRY(v->wp.alloc(n));
  FSA_TRY(v->xsp.alloc(2 * (size_t)n));
  hipLaunchKernelGGL(k_vposof, dim3(grid1(n)), dim3(256), 0, st, v->order.p, n, v->posof.p);
  hipLaunchKernelGGL(k_vperm, dim3(grid1(n)), dim3(256), 0, st, v->order.p, v->posof.p, n, mv, v->nbr.p, v->coef.p,
                     v->Dv.p, v->w.p, v->xs.p, v->fnbr.p, v->fcoef.p, v->Dvp.p, v->wp.p, v->xsp.p);
  FSA_HIP(hipGetLastError());
  // children lists (rows of B^T), by position
  {
    Buf<int> ccnt, cur;
    FSA_TRY(ccnt.alloc(n));
    FSA_TRY(cur.alloc(n));
    FSA_TRY(v->cptr.alloc(n + 1));
    FSA_HIP(hipMemsetAsync(ccnt.p, 0, n * sizeof(int), st));
    FSA_HIP(hipMemsetAsync(cur.p, 0, n * sizeof(int), st));
    if (mv > 0)
      hipLaunchKernelGGL(k_vchild_count, dim3(grid1(n * mv)), dim3(256), 0, st, v->fnbr.p, n, mv, ccnt.p);
    FSA_TRY(scan_counts(ccnt.p, n, v->cptr.p, v->scan_scratch, st));
    int64_t nnz = 0;
    FSA_HIP(hipMemcpyAsync(&nnz, v->cptr.p + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    FSA_HIP(hipStreamSynchronize(st));
    FSA_TRY(v->ci.alloc(std::max<int64_t>(nnz, 1)));
    FSA_TRY(v->cv.alloc(std::max<int64_t>(nnz, 1)));
    // per level, the longest child list (host-side launch planning)
    {
      std::vector<int64_t> hcp(n + 1);
      FSA_HIP(hipMemcpyAsync(hcp.data(), v->cptr.p, (n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, st));
      FSA_HIP(hipStreamSynchronize(st));
      const int nl = (int)v->lptr.size() - 1;
      v->lmaxc.assign(nl, 0);
      for (int l = 0; l < nl; ++l)
        for (int q = v->lptr[l]; q < v->lptr[l + 1]; ++q)
          v->lmaxc[l] = std::max(v->lmaxc[l], (int)(hcp[q + 1] - hcp[q]));
    }
    if (mv > 0) {
      hipLaunchKernelGGL(k_vchild_fill, dim3(grid1(n * mv)), dim3(256), 0, st, v->fnbr.p, v->fcoef.p, n, mv, v->cptr.p,
                         cur.p, v->ci.p, v->cv.p);
      hipLaunchKernelGGL(k_vchild_sort, dim3(grid1(n)), dim3(256), 0, st, v->cptr.p, n, v->ci.p, v->cv.p);
    }
    // the padded copy: position p of level l at lpoff[l] + (p - lptr[l]) lmaxc[l]
    {
      const int nl = (int)v->lptr.size() - 1;
      std::vector<int64_t> hpo(n + 1);
      v->lpoff.assign(nl, 0);
      int64_t at = 0;
      for (int l = 0; l < nl; ++l) {
        v->lpoff[l] = at;
        for (int q = v->lptr[l]; q < v->lptr[l + 1]; ++q, at += v->lmaxc[l]) hpo[q] = at;
      }
      hpo[n] = at;
      FSA_TRY(v->ppos.alloc(n + 1));
      FSA_TRY(v->pci.alloc(std::max<int64_t>(at, 1)));
      FSA_TRY(v->pcv.alloc(std::max<int64_t>(at, 1)));
      FSA_HIP(hipMemcpyAsync(v->ppos.p, hpo.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st));
      hipLaunchKernelGGL(k_vchild_pad, dim3(grid1(n)), dim3(256), 0, st, v->cptr.p, n, v->ci.p, v->cv.p, v->ppos.p,
                         v->pci.p, v->pcv.p);
      FSA_HIP(hipGetLastError());
      FSA_HIP(hipStreamSynchronize(st));  // hpo leaves scope
    }
  }
  // FITC preconditioner of Sigma + W^{-1}: A = L_m^{-1} Sigma_mn, D_s, C = I + A D_s^{-1} A^T
  FSA_TRY(v->Sm.alloc((size_t)mp * mp));
  FSA_TRY(v->Lm.alloc((size_t)mp * mp));
  FSA_TRY(dense_sigma_m(v->ind.p, v->m, mp, v->th, 0.0, false, v->Sm.p, st));
  FSA_HIP(hipMemcpyAsync(v->Lm.p, v->Sm.p, (size_t)mp * mp * sizeof(double), hipMemcpyDeviceToDevice, st));
  FSA_TRY(dense_cholesky(v->Lm.p, mp, v->info.p, st));
  FSA_HIP(hipMemcpyAsync(hinfo, v->info.p, sizeof(int), hipMemcpyDeviceToHost, st));
  FSA_HIP(hipStreamSynchronize(st));
  if (hinfo[0]) {
    set_error("Cholesky of Sigma_m failed at column %d (duplicate inducing points?)", hinfo[0] - 1);
    return FSA_ERR_NOT_SPD;
  }
  FSA_TRY(v->A.alloc((size_t)n * mp));
  {
    Buf<double> Li, LiT;  // L_m^{-1} and its transpose
    FSA_TRY(Li.alloc((size_t)mp * mp));
    FSA_TRY(LiT.alloc((size_t)mp * mp));
    FSA_TRY(tri_inverse(v->Lm.p, Li.p, mp, st));
    FSA_TRY(transpose_scale(Li.p, LiT.p, mp, 1.0, st));
    FSA_TRY(whiten(v->xsp.p, n, v->ind.p, v->m, mp, v->th, LiT.p, v->A.p, st));
  }
  return set_weights(v);
}

// One block PCG run on Sigma_V + W^{-1} over [Sigma_V rhs, z_1 .. z_t]
// (num_probes = t >= 0; with t = 0 the solve alone, logdet unused):
// x = (Sigma_V^{-1} + W)^{-1} rhs, *logdet = the SLQ estimate of
// log det(Sigma_V^{-1} + W).  rhs and x in the caller's order.
fsa_status vsolve(fsa_vecchia* v, const double* rhs, double* x, int32_t num_probes, uint64_t seed, double tol,
                  int32_t max_iter, int fixed, double* logdet, fsa_vecchia_stats* stats) {
  hipStream_t st = v->st;
  const auto t0 = std::chrono::steady_clock::now();
  const int64_t n = v->n;
  const int ncols = num_probes + 1;
  const int64_t ld = round_up(ncols, 64);
  const int ldw = (int)round_up(ncols, 64);
  const size_t blk = (size_t)n * ld;
  Buf<double> mem, Wm, G, Emat, col, hist;
  Buf<int> ivec;
  FSA_TRY(mem.alloc(8 * blk));
  double* Bk = mem.p;
  double* R = mem.p + blk;
  double* H = mem.p + 2 * blk;
  double* V = mem.p + 3 * blk;
  double* Z = mem.p + 4 * blk;
  double* U = mem.p + 5 * blk;
  double* Q0 = mem.p + 6 * blk;
  double* T = mem.p + 7 * blk;
  FSA_TRY(Wm.alloc((size_t)v->mp * ldw));
  FSA_TRY(G.alloc((size_t)v->mp * ldw));
  FSA_TRY(Emat.alloc((size_t)v->mp * ldw));
  // per column: [0] rz [1] bn2 [2] hv [3] alpha [4] beta [5] rzn [6] rr [7] weight [8] slq terms, then 2 results
  FSA_TRY(col.alloc(9 * (size_t)ncols + 2));
  double* c_rz = col.p;
  double* c_bn2 = col.p + ncols;
  double* c_hv = col.p + 2 * ncols;
  double* c_alpha = col.p + 3 * ncols;
  double* c_beta = col.p + 4 * ncols;
  double* c_rzn = col.p + 5 * ncols;
  double* c_rr = col.p + 6 * ncols;
  double* c_w = col.p + 7 * ncols;
  double* c_slq = col.p + 8 * ncols;
  double* res = col.p + 9 * ncols;
  FSA_TRY(hist.alloc(2 * (size_t)max_iter * ncols));
  double* ah = hist.p;
  double* bh = hist.p + (size_t)max_iter * ncols;
  FSA_TRY(ivec.alloc(2 * (size_t)ncols + 2));
  int* active = ivec.p;
  int* iters = ivec.p + ncols;
  int* flags = ivec.p + 2 * ncols;
  FSA_HIP(hipMemsetAsync(mem.p, 0, 8 * blk * sizeof(double), st));
  FSA_HIP(hipMemsetAsync(hist.p, 0, hist.bytes(), st));
  // right-hand sides [Sigma_V v, z_1 .. z_t], z ~ (0, P) (App. F sampling recipe)
  hipLaunchKernelGGL(k_vgather, dim3(grid1(n)), dim3(256), 0, st, n, 1, rhs, (int64_t)1, v->order.p, Q0, ld);
  FSA_TRY(sigma_v(v, Q0, ld, 1, T, ld));
  FSA_HIP(hipMemsetAsync(Q0, 0, blk * sizeof(double), st));
  {
    Buf<double> y;
    FSA_TRY(y.alloc(n));
    FSA_HIP(hipMemcpy2DAsync(y.p, sizeof(double), T, ld * sizeof(double), sizeof(double), n,
                             hipMemcpyDeviceToDevice, st));
    FSA_HIP(hipMemsetAsync(T, 0, blk * sizeof(double), st));
    // the Rademacher draws are keyed by the caller's point index (order[p])
    FSA_TRY(make_probes(v->A.p, n, v->m, v->mp, v->Ds.p, y.p, v->order.p, seed, num_probes, Bk, (int)ld, Emat.p, st));
    FSA_HIP(hipStreamSynchronize(st));  // y leaves scope
  }
  // init: R = B, Z = P^{-1} R, H = Q0 = Z
  hipLaunchKernelGGL(k_vcopy, dim3(grid1(n * ncols)), dim3(256), 0, st, n, ncols, Bk, ld, R, ld);
  FSA_TRY(precond(v, R, ld, ncols, Z, T, Wm.p, G.p, ldw));
  hipLaunchKernelGGL(k_vcopy, dim3(grid1(n * ncols)), dim3(256), 0, st, n, ncols, Z, ld, H, ld);
  hipLaunchKernelGGL(k_vcopy, dim3(grid1(n * ncols)), dim3(256), 0, st, n, ncols, Z, ld, Q0, ld);
  FSA_TRY((coldot<double, double>(R, Z, n, (int)ld, ncols, c_rzn, v->scr, st)));
  FSA_TRY((coldot<double, double>(Bk, Bk, n, (int)ld, ncols, c_bn2, v->scr, st)));
  FSA_TRY((coldot<double, double>(Bk, Q0, n, (int)ld, ncols, c_w, v->scr, st)));
  hipLaunchKernelGGL(k_vpcg_init, dim3(grid1(ncols)), dim3(256), 0, st, ncols, c_rzn, c_bn2, c_rz, active, iters, flags);
  FSA_HIP(hipGetLastError());
  const double tol2 = tol * tol;
  int hflags[2] = {0, 0};
  int it = 0;
  bool converged = false;
  for (; it < max_iter; ++it) {
    FSA_TRY(operator_v(v, H, ld, ncols, V, ld));
    FSA_TRY((coldot<double, double>(H, V, n, (int)ld, ncols, c_hv, v->scr, st)));
    hipLaunchKernelGGL(k_vpcg_alpha, dim3(grid1(ncols)), dim3(256), 0, st, ncols, c_hv, c_rz, active, c_alpha, flags);
    hipLaunchKernelGGL(k_vpcg_update, dim3(grid1(n * ncols)), dim3(256), 0, st, n, ncols, ld, c_alpha, H, V, U, R);
    FSA_TRY(precond(v, R, ld, ncols, Z, T, Wm.p, G.p, ldw));
    FSA_TRY((coldot<double, double>(R, Z, n, (int)ld, ncols, c_rzn, v->scr, st)));
    FSA_TRY((coldot<double, double>(R, R, n, (int)ld, ncols, c_rr, v->scr, st)));
    FSA_HIP(hipMemsetAsync(flags, 0, sizeof(int), st));
    hipLaunchKernelGGL(k_vpcg_beta, dim3(grid1(ncols)), dim3(256), 0, st, ncols, c_rzn, c_rr, c_bn2, c_alpha, c_rz,
                       c_beta, active, iters, ah, bh, max_iter, tol2, fixed, flags);
    hipLaunchKernelGGL(k_vpcg_direction, dim3(grid1(n * ncols)), dim3(256), 0, st, n, ncols, ld, c_beta, Z, H);
    FSA_HIP(hipGetLastError());
    if (fixed && it + 1 < max_iter) continue;  // breakdowns are read after the last iteration
    FSA_HIP(hipMemcpyAsync(hflags, flags, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
    FSA_HIP(hipStreamSynchronize(st));
    if (hflags[1]) {
      set_error("CG breakdown in the Vecchia solve (h^T K h <= 0 or non-finite)");
      return FSA_ERR_BREAKDOWN;
    }
    if (hflags[0] == 0 || fixed) {
      converged = true;
      ++it;
      break;
    }
  }
  // solution and log det
  hipLaunchKernelGGL(k_vsolution, dim3(grid1(n)), dim3(256), 0, st, n, U, ld, v->wp.p, v->order.p, x);
  double hres[2] = {0.0, 0.0};
  if (ncols > 1) {
    FSA_TRY(slq_terms(ah, bh, iters, ncols, 1, c_w, c_slq, nullptr, max_iter, st));
    hipLaunchKernelGGL(k_vlogdet, dim3(1), dim3(64), 0, st, c_slq, 1, ncols, v->parts.p, res);
    FSA_HIP(hipGetLastError());
  }
  std::vector<int> hit(ncols);
  if (ncols > 1) FSA_HIP(hipMemcpyAsync(hres, res, sizeof(hres), hipMemcpyDeviceToHost, st));
  FSA_HIP(hipMemcpyAsync(hit.data(), iters, ncols * sizeof(int), hipMemcpyDeviceToHost, st));
  FSA_HIP(hipStreamSynchronize(st));
  if (logdet) *logdet = hres[0];
  if (stats) {
    *stats = fsa_vecchia_stats{};
    stats->nlevels = (int32_t)v->lptr.size() - 1;
    stats->iters_rhs = hit[0];
    stats->iters_max = *std::max_element(hit.begin(), hit.end());
    stats->converged = converged ? 1 : 0;
    for (int c = 0; c < ncols; ++c) stats->probe_iters += hit[c];
    stats->logdet_P = v->logdet_P;
    stats->logdet_offset = v->offset;
    stats->logdet_sw = hres[1];
    stats->ms_solve = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  if (!converged) {
    set_error("Vecchia solve: max_iter (%d) reached", max_iter);
    return FSA_ERR_NOT_CONVERGED;
  }
  return FSA_OK;
}

// the three sums of k_vlaplace_parts (fixed order), read back to the host
fsa_status laplace_sums(fsa_vecchia* v, int mode, const double* x, const double* b, const double* y, double out[3]) {
  hipStream_t st = v->st;
  const int G = (int)std::min<int64_t>(grid1(v->n), 256);
  Buf<double> part;
  FSA_TRY(part.alloc(3 * (size_t)G + 3));
  hipLaunchKernelGGL(k_vlaplace_parts, dim3(G), dim3(256), 0, st, v->n, mode, x, b, y, part.p);
  hipLaunchKernelGGL(k_vsum3, dim3(1), dim3(64), 0, st, part.p, G, part.p + 3 * (size_t)G);
  FSA_HIP(hipGetLastError());
  FSA_HIP(hipMemcpyAsync(out, part.p + 3 * (size_t)G, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
  FSA_HIP(hipStreamSynchronize(st));
  return FSA_OK;
}

}  // namespace

extern "C" {

fsa_status fsa_vecchia_build_dev(const double* locs, int64_t n, const double* inducing, int32_t m, int32_t kind,
                                 double sigma1_sq, double rho, int32_t mv, const double* w, void* hip_stream,
                                 fsa_vecchia** out) {
  if (!out) { set_error("null argument"); return FSA_ERR_INVALID_ARG; }
  *out = nullptr;
  if (!locs || !inducing || !w) { set_error("null argument"); return FSA_ERR_INVALID_ARG; }
  if (n < 1 || n > (int64_t)INT32_MAX) { set_error("n must be in [1, 2^31)"); return FSA_ERR_INVALID_ARG; }
  if (m < 1 || m > 512) { set_error("m must be in [1, 512]"); return FSA_ERR_INVALID_ARG; }
  if (mv < 0 || mv > VMV_MAX) { set_error("m_v must be in [0, %d]", VMV_MAX); return FSA_ERR_INVALID_ARG; }
  if (kind != FSA_COV_EXPONENTIAL && kind != FSA_COV_MATERN32) { set_error("unknown covariance"); return FSA_ERR_INVALID_ARG; }
  if (!(sigma1_sq > 0.0) || !(rho > 0.0) || !std::isfinite(sigma1_sq) || !std::isfinite(rho)) {
    set_error("sigma1^2 and rho must be finite and positive");
    return FSA_ERR_INVALID_ARG;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  PoolStream ps(st);
  fsa_vecchia* v = new (std::nothrow) fsa_vecchia();
  if (!v) { set_error("out of host memory"); return FSA_ERR_OOM; }
  v->st = st;
  v->n = n;
  v->m = m;
  v->mp = (int)round_up(m, 64);
  v->mv = mv;
  v->th = Theta{kind, sigma1_sq, rho, 0.0};
  fsa_status s = build(v, locs, inducing, w);
  if (s != FSA_OK) {
    delete v;
    return s;
  }
  *out = v;
  return FSA_OK;
}

fsa_status fsa_vecchia_factor_dev(fsa_vecchia* v, int32_t* nbr, double* coef, double* d) {
  if (!v || !nbr || !coef || !d) { set_error("null argument"); return FSA_ERR_INVALID_ARG; }
  PoolStream ps(v->st);
  const size_t cnt = (size_t)v->n * v->mv;
  if (cnt) {
    FSA_HIP(hipMemcpyAsync(nbr, v->nbr.p, cnt * sizeof(int), hipMemcpyDeviceToDevice, v->st));
    FSA_HIP(hipMemcpyAsync(coef, v->coef.p, cnt * sizeof(double), hipMemcpyDeviceToDevice, v->st));
  }
  FSA_HIP(hipMemcpyAsync(d, v->Dv.p, v->n * sizeof(double), hipMemcpyDeviceToDevice, v->st));
  FSA_HIP(hipStreamSynchronize(v->st));
  return FSA_OK;
}

fsa_status fsa_vecchia_apply_dev(fsa_vecchia* v, int32_t which, const double* X, int64_t ldx, int32_t ncols,
                                 double* Y, int64_t ldy) {
  if (!v || !X || !Y) { set_error("null argument"); return FSA_ERR_INVALID_ARG; }
  if (ncols < 1 || ldx < ncols || ldy < ncols) { set_error("need 1 <= ncols <= ldx, ldy"); return FSA_ERR_INVALID_ARG; }
  if (X == Y) { set_error("X and Y must not alias"); return FSA_ERR_INVALID_ARG; }
  if (which < FSA_V_SIGMA || which > FSA_V_P_INV) {
    set_error("unknown operator %d", which);
    return FSA_ERR_INVALID_ARG;
  }
  PoolStream ps(v->st);
  hipStream_t st = v->st;
  const int64_t n = v->n;
  // into level order, apply, back to the caller's order
  const int ld = (int)round_up(ncols, 4), ldw = (int)round_up(ncols, 64);
  Buf<double> Xp, Yp;
  FSA_TRY(Xp.alloc((size_t)n * ld));
  FSA_TRY(Yp.alloc((size_t)n * ld));
  hipLaunchKernelGGL(k_vgather, dim3(grid1(n * ncols)), dim3(256), 0, st, n, ncols, X, ldx, v->order.p, Xp.p,
                     (int64_t)ld);
  switch (which) {
    case FSA_V_SIGMA:
      FSA_TRY(sigma_v(v, Xp.p, ld, ncols, Yp.p, ld));
      break;
    case FSA_V_PRECISION:
      FSA_TRY(precision_v(v, Xp.p, ld, ncols, Yp.p, ld));
      break;
    case FSA_V_OPERATOR:
      FSA_TRY(operator_v(v, Xp.p, ld, ncols, Yp.p, ld));
      break;
    default: {
      Buf<double> T, Wm, G;
      FSA_TRY(T.alloc((size_t)n * ld));
      FSA_TRY(Wm.alloc((size_t)v->mp * ldw));
      FSA_TRY(G.alloc((size_t)v->mp * ldw));
      FSA_TRY(precond(v, Xp.p, ld, ncols, Yp.p, T.p, Wm.p, G.p, ldw));
      FSA_HIP(hipStreamSynchronize(st));  // T, Wm, G leave scope
      break;
    }
  }
  hipLaunchKernelGGL(k_vscatter, dim3(grid1(n * ncols)), dim3(256), 0, st, n, ncols, Yp.p, (int64_t)ld, v->order.p, Y,
                     ldy);
  FSA_HIP(hipGetLastError());
  FSA_HIP(hipStreamSynchronize(st));
  return FSA_OK;
}

fsa_status fsa_vecchia_solve_logdet_dev(fsa_vecchia* v, const double* rhs, double* x, int32_t num_probes,
                                        uint64_t seed, double tol, int32_t max_iter, int32_t fixed_iter,
                                        double* logdet, fsa_vecchia_stats* stats) {
  if (!v || !rhs || !x || !logdet) { set_error("null argument"); return FSA_ERR_INVALID_ARG; }
  if (num_probes < 1 || num_probes > 1023) { set_error("num_probes must be in [1, 1023]"); return FSA_ERR_INVALID_ARG; }
  if (fixed_iter < 0 || fixed_iter > 6000) { set_error("fixed_iter must be in [0, 6000]"); return FSA_ERR_INVALID_ARG; }
  const int fixed = fixed_iter > 0 ? 1 : 0;
  if (fixed) max_iter = fixed_iter;
  if (!fixed && (!(tol > 0.0) || !std::isfinite(tol))) { set_error("tol must be finite and positive"); return FSA_ERR_INVALID_ARG; }
  if (max_iter < 1 || max_iter > 6000) { set_error("max_iter must be in [1, 6000]"); return FSA_ERR_INVALID_ARG; }
  PoolStream ps(v->st);
  return vsolve(v, rhs, x, num_probes, seed, tol, max_iter, fixed, logdet, stats);
}

fsa_status fsa_vecchia_laplace_dev(fsa_vecchia* v, const double* y, int32_t num_probes, uint64_t seed, double tol,
                                   int32_t max_iter, int32_t fixed_iter, double newton_tol, int32_t max_newton,
                                   int32_t fixed_newton, double* mode, double* nll,
                                   fsa_vecchia_laplace_stats* stats) {
  if (!v || !y || !mode || !nll) { set_error("null argument"); return FSA_ERR_INVALID_ARG; }
  if (num_probes < 1 || num_probes > 1023) { set_error("num_probes must be in [1, 1023]"); return FSA_ERR_INVALID_ARG; }
  if (fixed_iter < 0 || fixed_iter > 6000) { set_error("fixed_iter must be in [0, 6000]"); return FSA_ERR_INVALID_ARG; }
  const int fixed = fixed_iter > 0 ? 1 : 0;
  if (fixed) max_iter = fixed_iter;
  if (!fixed && (!(tol > 0.0) || !std::isfinite(tol))) { set_error("tol must be finite and positive"); return FSA_ERR_INVALID_ARG; }
  if (max_iter < 1 || max_iter > 6000) { set_error("max_iter must be in [1, 6000]"); return FSA_ERR_INVALID_ARG; }
  if (fixed_newton < 0 || fixed_newton > 200) { set_error("fixed_newton must be in [0, 200]"); return FSA_ERR_INVALID_ARG; }
  if (fixed_newton == 0 && (max_newton < 1 || max_newton > 200 || !(newton_tol > 0.0) || !std::isfinite(newton_tol))) {
    set_error("need 1 <= max_newton <= 200 and a finite positive newton_tol");
    return FSA_ERR_INVALID_ARG;
  }
  PoolStream ps(v->st);
  hipStream_t st = v->st;
  const auto t0 = std::chrono::steady_clock::now();
  const int64_t n = v->n;
  {
    int bad = 0;
    FSA_HIP(hipMemsetAsync(v->info.p + 2, 0, sizeof(int), st));
    hipLaunchKernelGGL(k_vcount_nonbinary, dim3(grid1(n)), dim3(256), 0, st, n, y, v->info.p + 2);
    FSA_HIP(hipGetLastError());
    FSA_HIP(hipMemcpyAsync(&bad, v->info.p + 2, sizeof(int), hipMemcpyDeviceToHost, st));
    FSA_HIP(hipStreamSynchronize(st));
    if (bad) { set_error("%d responses are not 0 or 1", bad); return FSA_ERR_INVALID_ARG; }
  }
  Buf<double> b, rhs, xn;
  FSA_TRY(b.alloc(n));
  FSA_TRY(rhs.alloc(n));
  FSA_TRY(xn.alloc(n));
  FSA_HIP(hipMemsetAsync(b.p, 0, n * sizeof(double), st));
  fsa_vecchia_laplace_stats ls{};
  bool soft_fail = false;
  const int limit = fixed_newton > 0 ? fixed_newton : max_newton;
  for (int k = 0; k < limit; ++k) {
    // b <- (Sigma_V^{-1} + W)^{-1} (W b + y - pi), W and the preconditioner at the current b
    hipLaunchKernelGGL(k_vnewton, dim3(grid1(n)), dim3(256), 0, st, n, b.p, y, 1, v->w.p, rhs.p);
    FSA_HIP(hipGetLastError());
    FSA_TRY(set_weights(v));
    fsa_vecchia_stats vs{};
    const fsa_status rc = vsolve(v, rhs.p, xn.p, 0, seed, tol, max_iter, fixed, nullptr, &vs);
    if (rc == FSA_ERR_NOT_CONVERGED) soft_fail = true;
    else FSA_TRY(rc);
    ls.cg_iters_max = std::max(ls.cg_iters_max, vs.iters_max);
    ls.probe_iters += vs.probe_iters;
    double nrm[3];
    FSA_TRY(laplace_sums(v, 0, xn.p, b.p, y, nrm));
    FSA_HIP(hipMemcpyAsync(b.p, xn.p, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    ++ls.newton_steps;
    if (fixed_newton == 0 && std::sqrt(nrm[0]) <= newton_tol * std::sqrt(nrm[1])) {
      ls.converged = 1;
      break;
    }
  }
  // at the mode: W there, log det(Sigma_V^{-1} + W) by SLQ, the log-likelihood and b^T Sigma_V^{-1} b
  hipLaunchKernelGGL(k_vnewton, dim3(grid1(n)), dim3(256), 0, st, n, b.p, y, 0, v->w.p, rhs.p);
  FSA_HIP(hipGetLastError());
  FSA_TRY(set_weights(v));
  fsa_vecchia_stats vs{};
  double ld = 0.0;
  {
    const fsa_status rc = vsolve(v, rhs.p, xn.p, num_probes, seed, tol, max_iter, fixed, &ld, &vs);
    if (rc == FSA_ERR_NOT_CONVERGED) soft_fail = true;
    else FSA_TRY(rc);
  }
  ls.cg_iters_max = std::max(ls.cg_iters_max, vs.iters_max);
  ls.probe_iters += vs.probe_iters;
  double ll[3], qd[3];
  FSA_TRY(laplace_sums(v, 1, nullptr, b.p, y, ll));
  {
    Buf<double> bp, qb;
    FSA_TRY(bp.alloc(n));
    FSA_TRY(qb.alloc(n));
    hipLaunchKernelGGL(k_vgather, dim3(grid1(n)), dim3(256), 0, st, n, 1, b.p, (int64_t)1, v->order.p, bp.p,
                       (int64_t)1);
    FSA_TRY(precision_v(v, bp.p, 1, 1, qb.p, 1));
    FSA_TRY(laplace_sums(v, 2, qb.p, bp.p, nullptr, qd));
  }
  FSA_HIP(hipMemcpyAsync(mode, b.p, n * sizeof(double), hipMemcpyDeviceToDevice, st));
  FSA_HIP(hipStreamSynchronize(st));
  ls.loglik = ll[0];
  ls.quad = qd[0];
  ls.sum_log_d = v->sum_log_dv;
  ls.logdet = ld;
  *nll = -ls.loglik + 0.5 * ls.quad + 0.5 * (ls.sum_log_d + ls.logdet);
  ls.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (stats) *stats = ls;
  if (soft_fail) {
    set_error("Vecchia-Laplace: a PCG solve reached max_iter (%d)", max_iter);
    return FSA_ERR_NOT_CONVERGED;
  }
  if (fixed_newton == 0 && !ls.converged) {
    set_error("Vecchia-Laplace: the mode did not converge in %d Newton steps", max_newton);
    return FSA_ERR_NOT_CONVERGED;
  }
  return FSA_OK;
}

fsa_status fsa_vecchia_destroy(fsa_vecchia* v) {
  if (!v) return FSA_OK;
  PoolStream ps(v->st);
  delete v;
  return FSA_OK;
}

}  // extern "C"
