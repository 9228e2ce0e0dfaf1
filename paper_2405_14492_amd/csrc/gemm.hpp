// MFMA (16x16x4, f64 or f32) kernels for the three dense contractions of the
// FSA path.  All point-indexed matrices are stored point-major: row i holds
// the kdim (multiple of 64) values of point i contiguously.
//
//  k_rows_gemm   OUT(i, c) = sum_k Aop(i, k) G[k][c]          (n x K) (K x 64)
//                e.g. A^T g (the low-rank half of the operator / Woodbury
//                solve), the whitening L_m^{-1} Sigma_mn, the probe block.
//  k_reduce_gemm W[k][c]   = sum_i Acol(i, k) X(i, c)          (K x n) (n x 64)
//                split over point chunks; deterministic second-stage sum.
//                e.g. A D^{-1} r, the capacitance A D^{-1} A^T.
//  k_sddmm       V(p, q)   = fn(d_pq, Xrow(p) . Yrow(q)) for the taper
//                pattern, by dense 16x16 blocks between a grid cell's points
//                and the points of its 3x3 neighbourhood.
//
// K-permutation: inside every block of 16 consecutive k, lane group
// q = lane/16 owns k = 4q..4q+3 and feeds element j to MFMA number j, so each
// lane fetches its four values with one vector load.  Any order of the k
// terms is a valid contraction order.
#pragma once

#include "common.hpp"
#include "kernels.hpp"

namespace fsa {

constexpr int GS_LD = 80;  // LDS row stride of the G tile (bank spread)
constexpr int XS_LD = 68;  // LDS row stride of the X chunk

// ------------------------------------------------------------------ operand loaders
template <typename T>
struct RowsOp {  // row i of a point-major matrix
  const T* a;
  int64_t lda;
  __device__ __forceinline__ V4<T> operator()(int64_t i, int k) const { return load4(a + i * lda + k); }
};

template <typename T>
struct Rows2Op {  // row i of [a1 | a2] (two point-major matrices, kseg each)
  const T* a1;
  const T* a2;
  int64_t lda;
  int kseg;
  __device__ __forceinline__ V4<T> operator()(int64_t i, int k) const {
    return k < kseg ? load4(a1 + i * lda + k) : load4(a2 + i * lda + (k - kseg));
  }
};

// ------------------------------------------------------------------ rows GEMM
// grid: (ceil(nrows / (64*RT)), ceil(ncols / 64)); block 256 (4 waves).
// Wave w handles rows [blk*64RT + w*16RT, +16RT) x 64 columns.
template <typename T, int RT, bool DOT, class AOp, class Epi>
__global__ __launch_bounds__(256) void k_rows_gemm(int64_t nrows, int kdim, const T* __restrict__ G, int ldg, int ncols,
                                                   int upper_g, AOp aop, Epi epi, double* __restrict__ dot_part,
                                                   int ld_dot) {
  __shared__ __attribute__((aligned(16))) T Gs[64 * GS_LD];
  __shared__ double red[4][64];
  typedef typename Mfma<T>::acc acc_t;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int q = lane >> 4, r16 = lane & 15;
  const int c0 = blockIdx.y * 64;
  const int64_t row0 = (int64_t)blockIdx.x * (64 * RT) + w * 16 * RT;
  acc_t acc[RT][4];
#pragma unroll
  for (int a = 0; a < RT; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
  const int kend = upper_g ? min(kdim, c0 + 64) : kdim;
  for (int kc = 0; kc < kend; kc += 64) {
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
      int rr = e >> 6, cc = e & 63;
      int gc = c0 + cc;
      Gs[rr * GS_LD + cc] = (gc < ncols) ? G[(int64_t)(kc + rr) * ldg + gc] : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 64; ks += 16) {
      V4<T> av[RT];
#pragma unroll
      for (int a = 0; a < RT; ++a) {
        int64_t i = row0 + a * 16 + r16;
        if (i < nrows) av[a] = aop(i, kc + ks + 4 * q);
        else av[a] = V4<T>{{T(0), T(0), T(0), T(0)}};
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        T bv[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) bv[b] = Gs[(ks + 4 * q + j) * GS_LD + b * 16 + r16];
#pragma unroll
        for (int a = 0; a < RT; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] = Mfma<T>::op(av[a].v[j], bv[b], acc[a][b]);
      }
    }
  }
  double dsum[4] = {0, 0, 0, 0};
#pragma unroll
  for (int a = 0; a < RT; ++a) {
    typename Epi::In in[4][4];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int64_t i = row0 + a * 16 + Mfma<T>::orow(q, r);
        int c = c0 + b * 16 + r16;
        if (i < nrows && c < ncols) in[b][r] = epi.load(i, c);
      }
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int64_t i = row0 + a * 16 + Mfma<T>::orow(q, r);
        int c = c0 + b * 16 + r16;
        if (i < nrows && c < ncols) dsum[b] += epi.apply(i, c, acc[a][b][r], in[b][r]);
      }
  }
  if constexpr (DOT) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      double v = dsum[b];
      v += __shfl_xor(v, 16, 64);
      v += __shfl_xor(v, 32, 64);
      if (q == 0) red[w][b * 16 + r16] = v;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
      double s = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
      dot_part[(int64_t)blockIdx.x * ld_dot + c0 + threadIdx.x] = s;
    }
  }
}

// ------------------------------------------------------------------ rows GEMM, float32, resident G
// OUT(i, c) = sum_k A[i][k] G[k][c] for one 64-column block: the whole
// kdim x 64 block of G (kdim <= 512) stays in LDS as [k/4][c][k%4], so a lane
// fetches the four k of one MFMA group with one 16-byte read.  Waves are
// persistent over 32-row tiles (no barrier in the main loop) and prefetch A
// two 16-k steps ahead.
template <bool DOT, class Epi>
__global__ __launch_bounds__(1024) void k_rows_gemm_f32(int64_t nrows, int kdim, const float* __restrict__ A,
                                                        int64_t lda, const float* __restrict__ G, int ldg, int ncols,
                                                        Epi epi, double* __restrict__ dot_part, int ld_dot) {
  extern __shared__ __attribute__((aligned(16))) float gres[];
  __shared__ double red[16][64];
  typedef Mfma<float>::acc acc_t;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const int q = lane >> 4, r16 = lane & 15;
  const int c0 = blockIdx.y * 64;
  for (int e = threadIdx.x; e < kdim * 64; e += blockDim.x) {
    int k = e >> 6, cc = e & 63;
    float v = (c0 + cc < ncols) ? G[(int64_t)k * ldg + c0 + cc] : 0.f;
    gres[(((k >> 2) * 64 + cc) << 2) + (k & 3)] = v;
  }
  __syncthreads();
  double dsum[4] = {0, 0, 0, 0};
  const int64_t ntile = (nrows + 31) / 32;
  for (int64_t tile = (int64_t)blockIdx.x * nw + w; tile < ntile; tile += (int64_t)gridDim.x * nw) {
    const int64_t row0 = tile * 32;
    const int64_t ia = min(row0 + r16, nrows - 1), ib = min(row0 + 16 + r16, nrows - 1);
    const float* pa = A + ia * lda + 4 * q;
    const float* pb = A + ib * lda + 4 * q;
    acc_t acc[2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
    f4 fa0 = *reinterpret_cast<const f4*>(pa), fb0 = *reinterpret_cast<const f4*>(pb);
    f4 fa1 = kdim > 16 ? *reinterpret_cast<const f4*>(pa + 16) : f4{0, 0, 0, 0};
    f4 fb1 = kdim > 16 ? *reinterpret_cast<const f4*>(pb + 16) : f4{0, 0, 0, 0};
    for (int ks = 0; ks < kdim; ks += 16) {
      f4 ca = fa0, cb = fb0;
      fa0 = fa1;
      fb0 = fb1;
      if (ks + 32 < kdim) {
        fa1 = *reinterpret_cast<const f4*>(pa + ks + 32);
        fb1 = *reinterpret_cast<const f4*>(pb + ks + 32);
      }
      f4 g[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) g[b] = *reinterpret_cast<const f4*>(&gres[((((ks >> 2) + q) * 64) + b * 16 + r16) << 2]);
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          acc[0][b] = Mfma<float>::op(ca[j], g[b][j], acc[0][b]);
          acc[1][b] = Mfma<float>::op(cb[j], g[b][j], acc[1][b]);
        }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        typename Epi::In in[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int64_t i = row0 + a * 16 + Mfma<float>::orow(q, r);
          int c = c0 + b * 16 + r16;
          if (i < nrows && c < ncols) in[r] = epi.load(i, c);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int64_t i = row0 + a * 16 + Mfma<float>::orow(q, r);
          int c = c0 + b * 16 + r16;
          if (i < nrows && c < ncols) dsum[b] += epi.apply(i, c, acc[a][b][r], in[r]);
        }
      }
  }
  if constexpr (DOT) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      double v = dsum[b];
      v += __shfl_xor(v, 16, 64);
      v += __shfl_xor(v, 32, 64);
      if (q == 0) red[w][b * 16 + r16] = v;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
      double sacc = 0.0;
      for (int k = 0; k < nw; ++k) sacc += red[k][threadIdx.x];
      dot_part[(int64_t)blockIdx.x * ld_dot + c0 + threadIdx.x] = sacc;
    }
  }
}

// ------------------------------------------------------------------ reduce GEMM
// grid: (nchunks, ncb = ceil(ncols/64), ceil(kdim / 512)); block 64*NW.
// Partial tile layout: part[((chunk*ncb + cb)*nmb + mb)*4096 + (tile*4 + r)*64 + lane]
// with tile = tau*4 + ct, k = mb*64 + 4*orow(lane/16, r) + tau, c = cb*64 + 4*(lane%16) + ct.
template <typename T, bool DOT, class AOp, class Pro>
__global__ __launch_bounds__(512) void k_reduce_gemm(int64_t npts, int pts_per_chunk, int kdim, int ncols, AOp acol,
                                                     Pro pro, T* __restrict__ part, double* __restrict__ dot_part,
                                                     int ld_dot, int lower_only) {
  __shared__ __attribute__((aligned(16))) T Xs[64 * XS_LD];
  __shared__ double red[512];
  typedef typename Mfma<T>::acc acc_t;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const int q = lane >> 4, r16 = lane & 15;
  const int c0 = blockIdx.y * 64;
  const int ncb = gridDim.y;
  const int nmb = kdim / 64;
  const int mb = blockIdx.z * 8 + w;
  const bool mactive = mb < nmb && (!lower_only || mb >= (int)blockIdx.y);
  const int kb = mb * 64;
  const int64_t pbeg = (int64_t)blockIdx.x * pts_per_chunk;
  const int64_t pend = min(npts, pbeg + pts_per_chunk);
  acc_t acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
  // prologue thread mapping: column tc, points tp0 + k*(nthreads/64)
  const int tc = threadIdx.x & 63;
  const int tp0 = threadIdx.x >> 6;
  double dacc = 0.0;
  for (int64_t p0 = pbeg; p0 < pend; p0 += 64) {
    __syncthreads();
    constexpr int PB = sizeof(T) == 8 ? 4 : 8;
    for (int pb = tp0; pb < 64; pb += PB * nw) {
      typename Pro::In in[PB];
      const int c = c0 + tc;
#pragma unroll
      for (int u = 0; u < PB; ++u) {
        int pp = pb + u * nw;
        int64_t p = p0 + pp;
        if (pp < 64 && p < pend && c < ncols) in[u] = pro.load(p, c);
      }
#pragma unroll
      for (int u = 0; u < PB; ++u) {
        int pp = pb + u * nw;
        if (pp < 64) {
          int64_t p = p0 + pp;
          T xv = T(0);
          if (p < pend && c < ncols) xv = pro.apply(p, c, in[u], dacc);
          Xs[pp * XS_LD + tc] = xv;
        }
      }
    }
    __syncthreads();
    if (mactive) {
#pragma unroll 4
      for (int kk = 0; kk < 64; kk += 4) {
        int64_t i = p0 + kk + q;
        V4<T> av;
        if (i < pend) av = acol(i, kb + 4 * r16);
        else av = V4<T>{{T(0), T(0), T(0), T(0)}};
        V4<T> xv = load4(&Xs[(kk + q) * XS_LD + 4 * r16]);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] = Mfma<T>::op(av.v[a], xv.v[b], acc[a][b]);
      }
    }
  }
  if (mactive) {
    T* dst = part + (((int64_t)blockIdx.x * ncb + blockIdx.y) * nmb + mb) * 4096;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) dst[((a * 4 + b) * 4 + r) * 64 + lane] = acc[a][b][r];
  }
  if constexpr (DOT) {
    red[threadIdx.x] = dacc;
    __syncthreads();
    if (threadIdx.x < 64) {
      double s = 0.0;
      for (int k = 0; k < nw; ++k) s += red[k * 64 + threadIdx.x];
      dot_part[(int64_t)blockIdx.x * ld_dot + c0 + threadIdx.x] = s;
    }
  }
}

// Sum the per-chunk partial tiles (fixed order, eight interleaved partial
// sums) into W (float64, row-major kdim x ldw); optionally add the identity.
template <typename T>
__global__ void k_reduce_parts(const T* __restrict__ part, int nchunks, int ncb, int nmb, double* __restrict__ W,
                               int ldw, int add_identity, int lower_only) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t per = (int64_t)ncb * nmb * 4096;
  if (e >= per) return;
  if (lower_only && (int)((e >> 12) % nmb) < (int)((e >> 12) / nmb)) return;
  double s8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int ch = 0;
  for (; ch + 8 <= nchunks; ch += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) s8[u] += (double)part[(int64_t)(ch + u) * per + e];
  }
  for (int u = 0; ch < nchunks; ++ch, ++u) s8[u] += (double)part[(int64_t)ch * per + e];
  double s = ((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]));
  int lane = (int)(e & 63);
  int r = (int)((e >> 6) & 3);
  int tile = (int)((e >> 8) & 15);
  int64_t blk = e >> 12;
  int mb = (int)(blk % nmb);
  int cb = (int)(blk / nmb);
  int tau = tile >> 2, ct = tile & 3;
  int k = mb * 64 + 4 * Mfma<T>::orow(lane >> 4, r) + tau;
  int c = cb * 64 + 4 * (lane & 15) + ct;
  if (add_identity && k == c) s += 1.0;
  W[(int64_t)k * ldw + c] = s;
}

// Column sums of per-workgroup partials: out[c] = sum_k part[k*ldp + c],
// one workgroup per column, fixed order.
__global__ __launch_bounds__(256) void k_colsum(const double* __restrict__ part, int nparts, int ldp,
                                                double* __restrict__ out);

// ------------------------------------------------------------------ SpMM
// Y(p, c) = sum_q S_pq X(q, c) for the rows of one grid cell per workgroup.
// The candidate columns are the points of the 3x3 block of cells (three
// contiguous ranges); their block rows are staged in LDS in chunks of CH
// rows, and every row reads its neighbours from LDS.  Waves own rows; lanes
// own columns (64-column block per grid.y).
// Position of column q in the concatenation of the three neighbour ranges
// (empty ranges never match).
__device__ __forceinline__ int64_t spmm_v_of_q(int64_t q, const int64_t* qb, const int64_t* qe, const int64_t* off) {
  if (q >= qb[2] && q < qe[2]) return q - qb[2] + off[2];
  if (q >= qb[1] && q < qe[1]) return q - qb[1] + off[1];
  return q - qb[0] + off[0];
}
__device__ __forceinline__ double readlane_t(double v, int j) {
  int64_t b = __double_as_longlong(v);
  int lo = __builtin_amdgcn_readlane((int)b, j);
  int hi = __builtin_amdgcn_readlane((int)(b >> 32), j);
  return __longlong_as_double(((int64_t)hi << 32) | (uint32_t)lo);
}
__device__ __forceinline__ float readlane_t(float v, int j) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), j));
}

template <typename T, bool DOT, int R, class Epi>
__global__ __launch_bounds__(256) void k_spmm_cell(const int64_t* __restrict__ rcs, const int64_t* __restrict__ ccs,
                                                   GridDesc gd, const int64_t* __restrict__ rp,
                                                   const int* __restrict__ col, const T* __restrict__ val,
                                                   const T* __restrict__ X, int ldx, int ncols, int CH, Epi epi,
                                                   double* __restrict__ dot_part, int ld_dot) {
  extern __shared__ __attribute__((aligned(16))) unsigned char spmm_smem[];
  T* Xs = reinterpret_cast<T*>(spmm_smem);
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t cell = blockIdx.x;
  const int c0 = blockIdx.y * 64;
  const int c = c0 + lane;
  const int64_t rb = rcs[cell], re = rcs[cell + 1];
  double dacc = 0.0;
  if (rb < re) {
    const int64_t cx = cell % gd.gx, cy = cell / gd.gx;
    int64_t qb[3], qe[3], off[3];
    int64_t V = 0;
    for (int t = 0; t < 3; ++t) {
      int64_t yy = cy - 1 + t;
      qb[t] = qe[t] = 0;
      if (yy >= 0 && yy < gd.gy) {
        int64_t xlo = cx - 1 < 0 ? 0 : cx - 1;
        int64_t xhi = cx + 1 >= gd.gx ? gd.gx - 1 : cx + 1;
        qb[t] = ccs[yy * gd.gx + xlo];
        qe[t] = ccs[yy * gd.gx + xhi + 1];
      }
      off[t] = V;
      V += qe[t] - qb[t];
    }
    for (int64_t g0 = rb; g0 < re; g0 += 4 * R) {
      // prefetch up to 128 entries of each of this wave's R rows: slot index
      // in the neighbourhood and value, two per lane
      T acc[R];
      int vq0[R], vq1[R];
      T vv0[R], vv1[R];
      int nent[R];
      int64_t ebeg[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        acc[r] = T(0);
        int64_t p = g0 + w + 4 * r;
        int64_t e0 = p < re ? rp[p] : 0;
        int64_t e1 = p < re ? rp[p + 1] : 0;
        ebeg[r] = e0;
        nent[r] = (int)(e1 - e0);
        int ne = nent[r];
        int qa = lane < ne ? col[e0 + lane] : 0;
        int qc = lane + 64 < ne ? col[e0 + 64 + lane] : 0;
        vv0[r] = lane < ne ? val[e0 + lane] : T(0);
        vv1[r] = lane + 64 < ne ? val[e0 + 64 + lane] : T(0);
        vq0[r] = lane < ne ? (int)spmm_v_of_q(qa, qb, qe, off) : 0x7fffffff;
        vq1[r] = lane + 64 < ne ? (int)spmm_v_of_q(qc, qb, qe, off) : 0x7fffffff;
      }
      for (int64_t vb = 0; vb < V; vb += CH) {
        __syncthreads();
        const int vn = (int)min((int64_t)CH, V - vb);
        // 16 four-element vectors per staged row; batches of 8 loads in flight
        for (int u0 = threadIdx.x; u0 < vn * 16; u0 += 256 * 8) {
          V4<T> tmp[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            int u = u0 + 256 * k;
            tmp[k] = V4<T>{{T(0), T(0), T(0), T(0)}};
            if (u < vn * 16) {
              int vr = u >> 4, c4 = (u & 15) * 4;
              int64_t v = vb + vr;
              int64_t q = v >= off[2] ? v - off[2] + qb[2] : (v >= off[1] ? v - off[1] + qb[1] : v - off[0] + qb[0]);
              if (c0 + c4 < ncols) tmp[k] = load4(X + q * ldx + c0 + c4);
            }
          }
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            int u = u0 + 256 * k;
            if (u < vn * 16) {
              int vr = u >> 4, c4 = (u & 15) * 4;
#pragma unroll
              for (int z = 0; z < 4; ++z) Xs[vr * 64 + c4 + z] = (c0 + c4 + z < ncols) ? tmp[k].v[z] : T(0);
            }
          }
        }
        __syncthreads();
        const int lo = (int)vb, hi = (int)vb + vn;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (nent[r] == 0) continue;
          // entries are sorted, so the ones in [lo, hi) are a contiguous run
          uint64_t m0 = __ballot(vq0[r] >= lo && vq0[r] < hi);
          uint64_t m1 = __ballot(vq1[r] >= lo && vq1[r] < hi);
          int j = m0 ? __ffsll((unsigned long long)m0) - 1 : 64;
          int jn = 64 - __clzll((unsigned long long)m0);
          if (!m0) jn = 64;
          T a0 = T(0), a1 = T(0);
          if (m0) {
            for (; j + 2 <= jn; j += 2) {
              int v0 = __builtin_amdgcn_readlane(vq0[r], j) - lo;
              int v1 = __builtin_amdgcn_readlane(vq0[r], j + 1) - lo;
              T w0 = readlane_t(vv0[r], j), w1 = readlane_t(vv0[r], j + 1);
              a0 += w0 * Xs[v0 * 64 + lane];
              a1 += w1 * Xs[v1 * 64 + lane];
            }
            if (j < jn) {
              int v0 = __builtin_amdgcn_readlane(vq0[r], j) - lo;
              a0 += readlane_t(vv0[r], j) * Xs[v0 * 64 + lane];
            }
          }
          if (m1) {
            j = __ffsll((unsigned long long)m1) - 1;
            jn = 64 - __clzll((unsigned long long)m1);
            for (; j + 2 <= jn; j += 2) {
              int v0 = __builtin_amdgcn_readlane(vq1[r], j) - lo;
              int v1 = __builtin_amdgcn_readlane(vq1[r], j + 1) - lo;
              T w0 = readlane_t(vv1[r], j), w1 = readlane_t(vv1[r], j + 1);
              a0 += w0 * Xs[v0 * 64 + lane];
              a1 += w1 * Xs[v1 * 64 + lane];
            }
            if (j < jn) {
              int v0 = __builtin_amdgcn_readlane(vq1[r], j) - lo;
              a0 += readlane_t(vv1[r], j) * Xs[v0 * 64 + lane];
            }
          }
          // rows with more than 128 entries: the rest straight from memory
          if (nent[r] > 128) {
            for (int64_t e = ebeg[r] + 128; e < ebeg[r] + nent[r]; ++e) {
              int v0 = (int)spmm_v_of_q(col[e], qb, qe, off);
              if (v0 >= lo && v0 < hi) a0 += val[e] * Xs[(v0 - lo) * 64 + lane];
            }
          }
          acc[r] += a0 + a1;
        }
      }
      typename Epi::In in[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        int64_t p = g0 + w + 4 * r;
        if (p < re && c < ncols) in[r] = epi.load(p, c);
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        int64_t p = g0 + w + 4 * r;
        if (p < re && c < ncols) dacc += epi.apply(p, c, acc[r], in[r]);
      }
    }
  }
  if constexpr (DOT) {
    __shared__ double red[4][64];
    __syncthreads();
    red[w][lane] = dacc;
    __syncthreads();
    if (threadIdx.x < 64)
      dot_part[(int64_t)blockIdx.x * ld_dot + c0 + threadIdx.x] =
          red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
  }
}

// ------------------------------------------------------------------ SDDMM
// One workgroup per row cell; rows are the row set's points in that cell,
// candidate columns the column set's points in the 3x3 block of cells.
template <typename T, class XOp, class YOp, class Fn>
__global__ __launch_bounds__(256) void k_sddmm(const int64_t* __restrict__ rcs, const double* __restrict__ rxs,
                                               const int64_t* __restrict__ ccs, const double* __restrict__ cxs,
                                               GridDesc gd, const int64_t* __restrict__ row_ptr,
                                               const int* __restrict__ col, int kdim, XOp xop, YOp yop, Fn fn,
                                               double* __restrict__ vals) {
#pragma clang fp contract(off)
  typedef typename Mfma<T>::acc acc_t;
  const int64_t cell = blockIdx.x;
  const int64_t rb = rcs[cell], re = rcs[cell + 1];
  if (rb >= re) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int q = lane >> 4, r16 = lane & 15;
  const int64_t cx = cell % gd.gx, cy = cell / gd.gx;
  int64_t qb[3], qe[3], nt[3];
  int64_t ntot = 0;
  for (int t = 0; t < 3; ++t) {
    int64_t yy = cy - 1 + t;
    qb[t] = qe[t] = 0;
    if (yy >= 0 && yy < gd.gy) {
      int64_t xlo = cx - 1 < 0 ? 0 : cx - 1;
      int64_t xhi = cx + 1 >= gd.gx ? gd.gx - 1 : cx + 1;
      qb[t] = ccs[yy * gd.gx + xlo];
      qe[t] = ccs[yy * gd.gx + xhi + 1];
    }
    nt[t] = (qe[t] - qb[t] + 15) / 16;
    ntot += nt[t];
  }
  const int64_t nrt = (re - rb + 15) / 16;
  const int64_t items = nrt * ntot;
  const double g2 = gd.gamma * gd.gamma;
  for (int64_t it = w; it < items; it += 4) {
    int64_t rt = it / ntot, ti = it % ntot;
    int t = 0;
    while (ti >= nt[t]) { ti -= nt[t]; ++t; }
    const int64_t p0 = rb + rt * 16;
    const int64_t q0 = qb[t] + ti * 16;
    const int64_t qend = qe[t];
    const int64_t pa = min(p0 + r16, re - 1);
    const int64_t qa = min(q0 + r16, qend - 1);
    acc_t acc = acc_t{0, 0, 0, 0};
    for (int ks = 0; ks < kdim; ks += 16) {
      V4<T> a = xop(pa, ks + 4 * q);
      V4<T> b = yop(qa, ks + 4 * q);
#pragma unroll
      for (int j = 0; j < 4; ++j) acc = Mfma<T>::op(a.v[j], b.v[j], acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int64_t p = p0 + Mfma<T>::orow(q, r);
      int64_t qq = q0 + r16;
      if (p < re && qq < qend) {
        double dx = rxs[2 * p] - cxs[2 * qq];
        double dy = rxs[2 * p + 1] - cxs[2 * qq + 1];
        double dx2 = dx * dx;
        double dy2 = dy * dy;
        double d2 = dx2 + dy2;
        if (d2 < g2) {
          int64_t lo = row_ptr[p], hi = row_ptr[p + 1] - 1;
          while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if (col[mid] < qq) lo = mid + 1;
            else hi = mid;
          }
          if (lo <= hi && col[lo] == qq) vals[lo] = fn(p, qq, sqrt(d2), (double)acc[r]);
        }
      }
    }
  }
}

}  // namespace fsa
