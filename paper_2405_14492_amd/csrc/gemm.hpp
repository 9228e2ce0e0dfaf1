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
  typedef T value_type;
  const T* a;
  int64_t lda;
  __device__ __forceinline__ V4<T> operator()(int64_t i, int k) const { return load4(a + i * lda + k); }
};

template <typename T>
struct Rows2Op {  // row i of [a1 | a2] (two point-major matrices, kseg each)
  typedef T value_type;
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

// Buffer resource over [base, base + bytes): loads past the end return zero,
// stores past the end are dropped (gfx9 raw buffer, stride 0).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc_of(const void* base, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
constexpr int BUF_OOR = 0x7ff00000;  // a buffer offset past every range used here

typedef unsigned u2v __attribute__((ext_vector_type(2)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));
template <typename T>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, unsigned off) {
  if constexpr (sizeof(T) == 8) return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
  else return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <typename T>
__device__ __forceinline__ void bstore(T v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  if constexpr (sizeof(T) == 8) __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2v, v), r, off, 0, 0);
  else __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 0);
}
// The low-rank factor A is float32 or bfloat16 (stored as its upper 16 bits;
// widened to float32 exactly by a shift).
typedef uint16_t bf16_t;
__device__ __forceinline__ float bf16_lo(unsigned x) { return __uint_as_float(x << 16); }
__device__ __forceinline__ float bf16_hi(unsigned x) { return __uint_as_float(x & 0xffff0000u); }
// four consecutive A entries at byte offset off
template <typename TA>
__device__ __forceinline__ f4 load_a4(__amdgpu_buffer_rsrc_t r, unsigned off) {
  if constexpr (sizeof(TA) == 4) {
    return __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
  } else {
    const u2v x = __builtin_bit_cast(u2v, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    return f4{bf16_lo(x[0]), bf16_hi(x[0]), bf16_lo(x[1]), bf16_hi(x[1])};
  }
}

template <typename T>
__device__ __forceinline__ V4<T> bload4(__amdgpu_buffer_rsrc_t r, unsigned off) {
  V4<T> o;
  if constexpr (sizeof(T) == 8) {
    const d2 a = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
    const d2 b = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(r, off + 16u, 0, 0));
    o.v[0] = a[0]; o.v[1] = a[1]; o.v[2] = b[0]; o.v[3] = b[1];
  } else {
    const f4 a = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
    o.v[0] = a[0]; o.v[1] = a[1]; o.v[2] = a[2]; o.v[3] = a[3];
  }
  return o;
}


// ------------------------------------------------------------------ rows GEMM, float32, resident G
// Epilogue of the float32 rows GEMM, out-of-place over row-major n x ld
// blocks.  Modes: ROWS_STORE Y = acc; ROWS_ACC Y += acc; ROWS_PCG t = acc
// written to Y, dot += r (r - t) Dinv; ROWS_PCG_INIT q = (r - acc) Dinv,
// H = Q0 = q, P = acc, dot += r q.
enum { ROWS_STORE = 0, ROWS_ACC = 1, ROWS_PCG = 2, ROWS_PCG_INIT = 3 };
struct F32RowsEpi {
  float* Y;  // ROWS_STORE / ROWS_ACC / ROWS_PCG output
  const float* R;
  const double* Dinv;
  float* H;
  float* P;
  float* Q0;
  int64_t ld;
};

// OUT(i, c) = sum_k A[i][k] G[k][c] for one 64-column block: the whole
// kdim x 64 block of G (kdim <= 512) stays in LDS as [k/4][c][k%4].  Each of
// the 16 waves is persistent over 16-row tiles and walks k in steps of 64: a
// lane loads 64 contiguous bytes of its row (k = 64 kb + 16 q' + 4 t + j for
// MFMA t, j) through a range-checked buffer resource over the tile's rows.
// The A loads of the step two ahead in the flattened (tile, k block) stream
// are issued before the matrix cores take the current step, and the
// epilogue reads and writes through buffer resources too, so no divergent
// branch in the loop forces the memory pipeline to drain.
template <typename TA, bool DOT, int EM>
__global__ __launch_bounds__(1024) void k_rows_gemm_f32(int64_t nrows, int kdim, const TA* __restrict__ A,
                                                        int64_t lda, const float* __restrict__ G, int ldg, int ncols,
                                                        F32RowsEpi epi, double* __restrict__ dot_part, int ld_dot) {
  extern __shared__ __attribute__((aligned(16))) float gres[];
  __shared__ double red[16][64];
  typedef Mfma<float>::acc acc_t;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int q = lane >> 4, r16 = lane & 15;
  const int c0 = blockIdx.y * 64;
  for (int e = tid; e < kdim * 64; e += 1024) {
    const int k = e >> 6, cc = e & 63;
    const float v = (c0 + cc < ncols) ? G[(int64_t)k * ldg + c0 + cc] : 0.f;
    gres[(((k >> 2) * 64 + cc) << 2) + (k & 3)] = v;
  }
  __syncthreads();
  const int nkb = kdim / 64;
  const int64_t ntile = (nrows + 15) / 16;
  const int64_t gw = (int64_t)blockIdx.x * 16 + w, GW = (int64_t)gridDim.x * 16;
  const int64_t ntw = gw < ntile ? (ntile - gw + GW - 1) / GW : 0;  // tiles of this wave
  constexpr unsigned EB = sizeof(TA);
  const unsigned lane_off = (unsigned)(r16 * lda + 16 * q) * EB;
  double dsum[4] = {0, 0, 0, 0};
  // load cursor: tile ordinal lj, k block lkb
  int64_t lj = 0;
  int lkb = 0;
  auto load_next = [&](f4* ab) {
    const int64_t row0 = (gw + lj * GW) * 16;
    const int64_t nr = lj < ntw ? min((int64_t)16, nrows - row0) : 0;
    const __amdgpu_buffer_rsrc_t rs = rsrc_of(A + (lj < ntw ? row0 * lda : 0), nr * lda * EB);
    const unsigned o = lane_off + (unsigned)lkb * 64u * EB;
#pragma unroll
    for (int t = 0; t < 4; ++t) ab[t] = load_a4<TA>(rs, o + 4u * EB * t);
    if (++lkb == nkb) {
      lkb = 0;
      ++lj;
    }
  };
  acc_t acc[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) acc[b] = acc_t{0, 0, 0, 0};
  // compute cursor: tile ordinal cj, k block ckb
  int64_t cj = 0;
  int ckb = 0;
  auto epilogue = [&]() {
    const int64_t row0 = (gw + cj * GW) * 16;
    const int64_t nr = min((int64_t)16, nrows - row0);
    const __amdgpu_buffer_rsrc_t ry = rsrc_of(epi.Y ? epi.Y + row0 * epi.ld : (const void*)A, epi.Y ? nr * epi.ld * 4 : 0);
    const __amdgpu_buffer_rsrc_t rr = rsrc_of(epi.R ? epi.R + row0 * epi.ld : (const void*)A, epi.R ? nr * epi.ld * 4 : 0);
    const __amdgpu_buffer_rsrc_t rd = rsrc_of(epi.Dinv ? epi.Dinv + row0 : (const double*)A, epi.Dinv ? nr * 8 : 0);
    const __amdgpu_buffer_rsrc_t rh = rsrc_of(EM == ROWS_PCG_INIT ? epi.H + row0 * epi.ld : (const void*)A, EM == ROWS_PCG_INIT ? nr * epi.ld * 4 : 0);
    const __amdgpu_buffer_rsrc_t rp = rsrc_of(EM == ROWS_PCG_INIT ? epi.P + row0 * epi.ld : (const void*)A, EM == ROWS_PCG_INIT ? nr * epi.ld * 4 : 0);
    const __amdgpu_buffer_rsrc_t rq = rsrc_of(EM == ROWS_PCG_INIT ? epi.Q0 + row0 * epi.ld : (const void*)A, EM == ROWS_PCG_INIT ? nr * epi.ld * 4 : 0);
    float xin[4][4];
    double di[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if constexpr (EM >= ROWS_PCG)
        di[r] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rd, (unsigned)(4 * q + r) * 8u, 0, 0));
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int c = c0 + b * 16 + r16;
        const unsigned o = c < ncols ? (unsigned)((4 * q + r) * (int)epi.ld + c) * 4u : (unsigned)BUF_OOR;
        if constexpr (EM == ROWS_ACC)
          xin[r][b] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(ry, o, 0, 0));
        if constexpr (EM >= ROWS_PCG)
          xin[r][b] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rr, o, 0, 0));
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int c = c0 + b * 16 + r16;
        const unsigned o = c < ncols ? (unsigned)((4 * q + r) * (int)epi.ld + c) * 4u : (unsigned)BUF_OOR;
        const float v = acc[b][r];
        if constexpr (EM == ROWS_STORE) {
          __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), ry, o, 0, 0);
        } else if constexpr (EM == ROWS_ACC) {
          __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v + xin[r][b]), ry, o, 0, 0);
        } else {
          const double rv = (double)xin[r][b];
          const double qv = (rv - (double)v) * di[r];
          // zero for points past the tile and padding columns (r = 0, Dinv = 0)
          dsum[b] += rv * qv;
          if constexpr (EM == ROWS_PCG) {
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), ry, o, 0, 0);
          } else {
            const unsigned qb = __builtin_bit_cast(unsigned, (float)qv);
            __builtin_amdgcn_raw_buffer_store_b32(qb, rh, o, 0, 0);
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), rp, o, 0, 0);
            __builtin_amdgcn_raw_buffer_store_b32(qb, rq, o, 0, 0);
          }
        }
      }
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[b] = acc_t{0, 0, 0, 0};
  };
  // one step of the flattened (tile, k block) stream: the loads of the step
  // two ahead go into `ahead`, the matrix cores take `cur`
  auto step = [&](const f4* cur, f4* ahead) {
    load_next(ahead);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      f4 g[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) g[b] = *reinterpret_cast<const f4*>(&gres[((ckb * 16 + 4 * q + t) * 64 + b * 16 + r16) << 2]);
#pragma unroll
      for (int jj = 0; jj < 4; ++jj)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[b] = Mfma<float>::op(cur[t][jj], g[b][jj], acc[b]);
    }
    if (++ckb == nkb) {
      epilogue();
      ckb = 0;
      ++cj;
    }
  };
  const int64_t nflat = ntw * nkb;
  f4 b0[4], b1[4], b2[4];
  load_next(b0);
  load_next(b1);
  int64_t f = 0;
  for (; f + 2 < nflat; f += 3) {
    step(b0, b2);
    step(b1, b0);
    step(b2, b1);
  }
  if (f < nflat) step(b0, b2);
  if (f + 1 < nflat) step(b1, b0);
  if constexpr (DOT) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      double v = dsum[b];
      v += __shfl_xor(v, 16, 64);
      v += __shfl_xor(v, 32, 64);
      if (q == 0) red[w][b * 16 + r16] = v;
    }
    __syncthreads();
    if (tid < 64) {
      double sacc = 0.0;
      for (int k = 0; k < 16; ++k) sacc += red[k][tid];
      dot_part[(int64_t)blockIdx.x * ld_dot + c0 + tid] = sacc;
    }
  }
}

// ------------------------------------------------------------------ rows GEMM, float64, resident G slice
// OUT(i, c) = sum_k A[i][acol0 + k] G[grow0 + k][c], k < kh <= 256, one
// 64-column block: the kh x 64 slice of G stays in LDS as [k/4][c][k%4]
// (128 KB).  A product with a longer k runs as passes over 256-k slices:
// the first stores its partial sums in `part`, middle passes add to them,
// the last adds them and applies the epilogue (PM: 0 single pass, 1 first,
// 2 middle, 3 last).  The 16 waves are persistent over 16-row tiles and
// walk k in steps of 32: a lane loads 64 contiguous bytes of its row
// (k = 32 s + 8 q' + 4 t + j for MFMA t, j) through a per-tile buffer
// resource, one step ahead across tile boundaries.  Epilogue modes as in
// the float32 kernel (ROWS_STORE, ROWS_PCG, ROWS_PCG_INIT).
struct F64RowsEpi {
  double* Y;
  const double* R;
  const double* Dinv;
  double* H;
  double* P;
  double* Q0;
  int64_t ld;
};

template <bool DOT, int EM, int PM>
__global__ __launch_bounds__(1024) void k_rows_gemm_f64(int64_t nrows, const double* __restrict__ A, int64_t lda,
                                                        int acol0, int kh, const double* __restrict__ G, int ldg,
                                                        int grow0, int ncols, F64RowsEpi epi,
                                                        double* __restrict__ part, double* __restrict__ dot_part,
                                                        int ld_dot) {
  extern __shared__ __attribute__((aligned(16))) double gres64[];
  __shared__ double red[16][64];
  typedef Mfma<double>::acc acc_t;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int q = lane >> 4, r16 = lane & 15;
  const int c0 = blockIdx.y * 64;
  for (int e = tid; e < kh * 64; e += 1024) {
    const int k = e >> 6, cc = e & 63;
    const double v = (c0 + cc < ncols) ? G[(int64_t)(grow0 + k) * ldg + c0 + cc] : 0.0;
    gres64[(((k >> 2) * 64 + cc) << 2) + (k & 3)] = v;
  }
  __syncthreads();
  const int nks = kh / 32;
  const int64_t ntile = (nrows + 15) / 16;
  const int64_t gw = (int64_t)blockIdx.x * 16 + w, GW = (int64_t)gridDim.x * 16;
  const int64_t ntw = gw < ntile ? (ntile - gw + GW - 1) / GW : 0;
  const unsigned lane_off = (unsigned)(r16 * (int)lda + acol0 + 8 * q) * 8u;
  double dsum[4] = {0, 0, 0, 0};
  int64_t lj = 0;
  int lks = 0;
  auto load_next = [&](d2* ab) {
    const int64_t row0 = (gw + lj * GW) * 16;
    const int64_t nr = lj < ntw ? min((int64_t)16, nrows - row0) : 0;
    const __amdgpu_buffer_rsrc_t rs = rsrc_of(A + (lj < ntw ? row0 * lda : 0), nr * lda * 8);
    const unsigned o = lane_off + (unsigned)lks * 256u;
#pragma unroll
    for (int t = 0; t < 4; ++t) ab[t] = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(rs, o + 16u * t, 0, 0));
    if (++lks == nks) {
      lks = 0;
      ++lj;
    }
  };
  acc_t acc[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) acc[b] = acc_t{0, 0, 0, 0};
  int64_t cj = 0;
  int cks = 0;
  auto epilogue = [&]() {
    const int64_t row0 = (gw + cj * GW) * 16;
    const int64_t nr = min((int64_t)16, nrows - row0);
    const int64_t bytes = nr * epi.ld * 8;
    const __amdgpu_buffer_rsrc_t rpart = rsrc_of(part ? part + row0 * epi.ld : A, part ? bytes : 0);
    const __amdgpu_buffer_rsrc_t ry = rsrc_of(epi.Y ? epi.Y + row0 * epi.ld : A, epi.Y ? bytes : 0);
    const __amdgpu_buffer_rsrc_t rr = rsrc_of(epi.R ? epi.R + row0 * epi.ld : A, epi.R ? bytes : 0);
    const __amdgpu_buffer_rsrc_t rd = rsrc_of(epi.Dinv ? epi.Dinv + row0 : A, epi.Dinv ? nr * 8 : 0);
    const __amdgpu_buffer_rsrc_t rh = rsrc_of(EM == ROWS_PCG_INIT ? epi.H + row0 * epi.ld : A, EM == ROWS_PCG_INIT ? bytes : 0);
    const __amdgpu_buffer_rsrc_t rp = rsrc_of(EM == ROWS_PCG_INIT ? epi.P + row0 * epi.ld : A, EM == ROWS_PCG_INIT ? bytes : 0);
    const __amdgpu_buffer_rsrc_t rq = rsrc_of(EM == ROWS_PCG_INIT ? epi.Q0 + row0 * epi.ld : A, EM == ROWS_PCG_INIT ? bytes : 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = Mfma<double>::orow(q, r);
      double di = 0.0;
      if constexpr ((PM == 0 || PM == 3) && EM >= ROWS_PCG) di = bload<double>(rd, (unsigned)i * 8u);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int c = c0 + b * 16 + r16;
        const unsigned o = c < ncols ? (unsigned)(i * (int)epi.ld + c) * 8u : (unsigned)BUF_OOR;
        double v = acc[b][r];
        if constexpr (PM >= 2) v += bload<double>(rpart, o);
        if constexpr (PM == 1 || PM == 2) {
          bstore<double>(v, rpart, o);
        } else if constexpr (EM == ROWS_STORE) {
          bstore<double>(v, ry, o);
        } else {
          const double rv = bload<double>(rr, o);
          const double qv = (rv - v) * di;
          dsum[b] += rv * qv;  // zero past the tile's rows and columns
          if constexpr (EM == ROWS_PCG) {
            bstore<double>(v, ry, o);
          } else {
            bstore<double>(qv, rh, o);
            bstore<double>(v, rp, o);
            bstore<double>(qv, rq, o);
          }
        }
      }
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[b] = acc_t{0, 0, 0, 0};
  };
  auto step = [&](const d2* cur, d2* nxt) {
    load_next(nxt);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      V4<double> g[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) g[b] = load4(&gres64[((cks * 8 + 2 * q + t) * 64 + b * 16 + r16) << 2]);
      const double av[4] = {cur[2 * t][0], cur[2 * t][1], cur[2 * t + 1][0], cur[2 * t + 1][1]};
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[b] = Mfma<double>::op(av[j], g[b].v[j], acc[b]);
    }
    if (++cks == nks) {
      epilogue();
      cks = 0;
      ++cj;
    }
  };
  const int64_t nflat = ntw * nks;
  d2 b0[4], b1[4];
  load_next(b0);
  int64_t f = 0;
  for (; f + 1 < nflat; f += 2) {
    step(b0, b1);
    step(b1, b0);
  }
  if (f < nflat) step(b0, b1);
  if constexpr (DOT) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      double v = dsum[b];
      v += __shfl_xor(v, 16, 64);
      v += __shfl_xor(v, 32, 64);
      if (q == 0) red[w][b * 16 + r16] = v;
    }
    __syncthreads();
    if (tid < 64) {
      double sacc = 0.0;
      for (int k = 0; k < 16; ++k) sacc += red[k][tid];
      dot_part[(int64_t)blockIdx.x * ld_dot + c0 + tid] = sacc;
    }
  }
}

// ------------------------------------------------------------------ reduce GEMM
// Prologue of the float32 reduce GEMM: X(p, c) = x(p, c) * scale, where
// x = S(p, c), or with UPD the updated residual x = S - alpha_c V (written
// back to S, and |x|^2 accumulated per column), and scale = 1 (SC = 0),
// sc[p] (SC = 1) or 1 / sc[p] (SC = 2).
struct F32Pro {
  float* S;
  const float* V;        // with UPD
  const double* alpha;   // with UPD
  const double* sc;      // with SC != 0
  int64_t ld;
};


// Float32 reduce GEMM, software-pipelined.  grid (nchunks, ncb, zb), 512
// threads; wave w owns the 64 rows 512 z + 64 w .. +63 of the kdim side
// (four 16-row MFMA tiles, rows interleaved by four so that a lane loads four
// adjacent A entries) and the workgroup's 64-column block.  Points are taken
// 24 per step; the A rows of the next two steps are in flight in registers
// while the matrix cores work on the current one, and the next step's
// prologue inputs load meanwhile and land in the other half of a
// double-buffered LDS block (one barrier per step).  Every load and store in
// the loop is an unconditional buffer access over the chunk's rows (zero
// fill and dropped stores past the last point or column), so no branch
// forces the memory pipeline to drain.  Partials are row-major:
// part[((chunk * ncb + cb) * kdim + k) * 64 + c - 64 cb].
template <typename TA, bool UPD, int SC>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2))) void k_reduce_gemm_f32(
    int64_t npts, int pts_per_chunk, int kdim, int ncols, const TA* __restrict__ A, F32Pro pro,
    float* __restrict__ part, double* __restrict__ dot_part, int ld_dot) {
  constexpr int SP = 24;        // points per step
  constexpr int NA = SP / 4;    // A loads per lane per step
  constexpr int NP = SP / 8;    // prologue elements per thread per step
  __shared__ __attribute__((aligned(16))) float Xs[2][SP * XS_LD];
  __shared__ double red[512];
  typedef Mfma<float>::acc acc_t;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int q = lane >> 4, r16 = lane & 15;
  const int c0 = blockIdx.x * 64;
  const int ncb = gridDim.x;
  const int chunk = blockIdx.y;
  const int kb = blockIdx.z * 512 + w * 64;
  const bool mactive = kb < kdim;
  const int64_t pbeg = (int64_t)chunk * pts_per_chunk;
  const int64_t pend = min(npts, pbeg + pts_per_chunk);
  const int np = pend > pbeg ? (int)(pend - pbeg) : 0;
  const int nsteps = (np + SP - 1) / SP;
  const int tc = tid & 63, tp = tid >> 6;  // prologue: column c0 + tc, points tp + 8 u
  const int c = c0 + tc;
  const bool cval = c < ncols;
  acc_t acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
  double dacc = 0.0;
  f4 ab0[NA] = {}, ab1[NA] = {}, ab2[NA] = {};
  constexpr unsigned EB = sizeof(TA);
  const __amdgpu_buffer_rsrc_t arsrc = rsrc_of(A + pbeg * kdim, (int64_t)np * kdim * EB);
  const __amdgpu_buffer_rsrc_t srsrc = rsrc_of(pro.S + pbeg * pro.ld, (int64_t)np * pro.ld * 4);
  const __amdgpu_buffer_rsrc_t vrsrc = rsrc_of(UPD ? pro.V + pbeg * pro.ld : pro.S, UPD ? (int64_t)np * pro.ld * 4 : 0);
  const __amdgpu_buffer_rsrc_t drsrc = rsrc_of(SC ? pro.sc + pbeg : (const double*)pro.S, SC ? (int64_t)np * 8 : 0);
  const double a_c = (UPD && cval) ? pro.alpha[c] : 0.0;
  // byte offsets into the chunk (unsigned: BUF_OOR plus an offset stays out of range)
  const unsigned a_off = mactive ? (unsigned)(q * kdim + kb + 4 * r16) * EB : (unsigned)BUF_OOR;
  const unsigned s_off = cval ? (unsigned)(tp * (int)pro.ld + c) * 4u : (unsigned)BUF_OOR;  // element (tp, c)
  const unsigned s_step = 8u * (unsigned)pro.ld * 4u;                                       // + 8 points
  float sv[NP], vv[NP];
  double dv[NP];
  auto load_a = [&](int s, f4* ab) {
    const unsigned so = a_off + (unsigned)(s * SP * kdim) * EB;
#pragma unroll
    for (int k = 0; k < NA; ++k) ab[k] = load_a4<TA>(arsrc, so + 4u * EB * k * kdim);
  };
  auto pro_load = [&](int s) {
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      const int pr = s * SP + tp + 8 * u;
      const unsigned o = s_off + (unsigned)(s * SP / 8 + u) * s_step;
      sv[u] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(srsrc, o, 0, 0));
      vv[u] = UPD ? __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(vrsrc, o, 0, 0)) : 0.f;
      dv[u] = SC ? __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(drsrc, (unsigned)pr * 8u, 0, 0)) : 1.0;
    }
  };
  auto pro_apply = [&](int s, float* xs) {
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      const int pr = s * SP + tp + 8 * u;
      double x = (double)sv[u];
      if constexpr (UPD) {
        const float rt = (float)(x - a_c * (double)vv[u]);
        const unsigned o = s_off + (unsigned)(s * SP / 8 + u) * s_step;
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, rt), srsrc, o, 0, 0);
        x = (double)rt;
        dacc += x * x;  // zero for padding columns and points past the chunk
      }
      const double y = SC == 0 ? x : (SC == 1 ? x * dv[u] : x / dv[u]);
      xs[(tp + 8 * u) * XS_LD + tc] = (pr < np && cval) ? (float)y : 0.f;
    }
  };
  auto mma = [&](const f4* ab, const float* xs) {
    if (!mactive) return;
#pragma unroll
    for (int k = 0; k < NA; ++k) {
      const V4<float> xv = load4(&xs[(4 * k + q) * XS_LD + 4 * r16]);
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = Mfma<float>::op(ab[k][a], xv.v[b], acc[a][b]);
    }
  };
  // step s: prologue inputs of step s + 1 and A of step s + 2 load (in that
  // order, so that the prologue's wait leaves the A loads in flight), the
  // matrix cores take step s from (abc, Xs[s & 1])
  auto step = [&](int s, const f4* abc, f4* abn) {
    pro_load(s + 1);
    load_a(s + 2, abn);
    mma(abc, Xs[s & 1]);
    pro_apply(s + 1, Xs[(s + 1) & 1]);
    __syncthreads();
  };
  if (nsteps > 0) {
    pro_load(0);
    load_a(0, ab0);
    load_a(1, ab1);
    pro_apply(0, Xs[0]);
    __syncthreads();
    int s = 0;
    for (; s + 2 < nsteps; s += 3) {
      step(s, ab0, ab2);
      step(s + 1, ab1, ab0);
      step(s + 2, ab2, ab1);
    }
    if (s < nsteps) step(s, ab0, ab2);
    if (s + 1 < nsteps) step(s + 1, ab1, ab0);
  }
  if (mactive) {
    // tile (a, b) row i = 4 q' + r, column r16: k = kb + 4 i + a, c = 4 r16 + b
    float* dst = part + (((int64_t)chunk * ncb + blockIdx.x) * kdim + kb) * 64 + 4 * r16;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        *reinterpret_cast<f4*>(dst + (4 * (4 * q + r) + a) * 64) =
            f4{acc[a][0][r], acc[a][1][r], acc[a][2][r], acc[a][3][r]};
  }
  if constexpr (UPD) {
    red[tid] = dacc;
    __syncthreads();
    if (tid < 64) {
      double sum = 0.0;
      for (int k = 0; k < 8; ++k) sum += red[k * 64 + tid];
      dot_part[(int64_t)chunk * ld_dot + c0 + tid] = sum;
    }
  }
}

// Float64 version: grid (ncb, nchunks, zb), 1024 threads; wave w owns the
// 32 rows 512 z + 32 w .. +31 of the kdim side (two 16-row MFMA tiles, rows
// interleaved by two so that a lane loads two adjacent A entries with one
// 16-byte buffer load) for the workgroup's 64-column block.  Points are taken
// 16 per step; the next step's A rows and prologue inputs are in flight
// while the matrix cores work on the current step (double-buffered
// registers and LDS).  Same prologue modes and partial layout as the float32
// kernel.  With lower_only, rows below the column block's diagonal block are
// skipped (symmetric products).
struct F64Pro {
  double* S;
  const double* V;
  const double* alpha;
  const double* sc;
  int64_t ld;
};

template <bool UPD, int SC>
__global__ __launch_bounds__(1024) void k_reduce_gemm_f64(int64_t npts, int pts_per_chunk, int kdim, int ncols,
                                                          const double* __restrict__ A, F64Pro pro,
                                                          double* __restrict__ part, double* __restrict__ dot_part,
                                                          int ld_dot, int lower_only, int nchunks) {
  constexpr int SP = 16;       // points per step
  constexpr int NA = SP / 4;   // A loads per lane per step
  __shared__ __attribute__((aligned(16))) double Xs[2][SP * XS_LD];
  __shared__ double red[1024];
  typedef Mfma<double>::acc acc_t;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int q = lane >> 4, r16 = lane & 15;
  // XCD-aware order: linear workgroup b runs on XCD b % 8, and the column
  // blocks of one chunk go to the same XCD back to back, so that the
  // chunk's A rows come from HBM once and from that XCD's L2 after (the
  // grid's y extent is the chunk count rounded up to a multiple of 8)
  const int ncb = gridDim.x;
  const int bl = blockIdx.x + ncb * blockIdx.y;
  const int cbx = (bl >> 3) % ncb;
  const int chunk = (bl & 7) + 8 * ((bl >> 3) / ncb);
  if (chunk >= nchunks) return;
  const int c0 = cbx * 64;
  const int kb = blockIdx.z * 512 + w * 32;
  const bool mactive = kb < kdim && (!lower_only || kb >= c0);
  const int64_t pbeg = (int64_t)chunk * pts_per_chunk;
  const int64_t pend = min(npts, pbeg + pts_per_chunk);
  const int np = pend > pbeg ? (int)(pend - pbeg) : 0;
  const int nsteps = (np + SP - 1) / SP;
  const int tc = tid & 63, tp = tid >> 6;  // prologue: column c0 + tc, point tp of the step
  const int c = c0 + tc;
  const bool cval = c < ncols;
  acc_t acc[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
  double dacc = 0.0;
  d2 ab0[NA] = {}, ab1[NA] = {};
  const __amdgpu_buffer_rsrc_t arsrc = rsrc_of(A + pbeg * kdim, (int64_t)np * kdim * 8);
  const __amdgpu_buffer_rsrc_t srsrc = rsrc_of(pro.S + pbeg * pro.ld, (int64_t)np * pro.ld * 8);
  const __amdgpu_buffer_rsrc_t vrsrc = rsrc_of(UPD ? pro.V + pbeg * pro.ld : pro.S, UPD ? (int64_t)np * pro.ld * 8 : 0);
  const __amdgpu_buffer_rsrc_t drsrc = rsrc_of(SC ? pro.sc + pbeg : (const double*)pro.S, SC ? (int64_t)np * 8 : 0);
  const double a_c = (UPD && cval) ? pro.alpha[c] : 0.0;
  const unsigned a_off = mactive ? (unsigned)(q * kdim + kb + 2 * r16) * 8u : (unsigned)BUF_OOR;
  const unsigned s_off = cval ? (unsigned)(tp * (int)pro.ld + c) * 8u : (unsigned)BUF_OOR;
  const unsigned s_step = (unsigned)SP * (unsigned)pro.ld * 8u;
  double sv = 0.0, vv = 0.0, dv = 1.0;
  auto load_a = [&](int s, d2* ab) {
    const unsigned so = a_off + (unsigned)(s * SP * kdim) * 8u;
#pragma unroll
    for (int k = 0; k < NA; ++k)
      ab[k] = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(arsrc, so + 32u * k * kdim, 0, 0));
  };
  auto pro_load = [&](int s) {
    const unsigned o = s_off + (unsigned)s * s_step;
    sv = bload<double>(srsrc, o);
    if constexpr (UPD) vv = bload<double>(vrsrc, o);
    if constexpr (SC != 0) dv = bload<double>(drsrc, (unsigned)(s * SP + tp) * 8u);
  };
  auto pro_apply = [&](int s, double* xs) {
    const int pr = s * SP + tp;
    double x = sv;
    if constexpr (UPD) {
      x = x - a_c * vv;
      bstore<double>(x, srsrc, s_off + (unsigned)s * s_step);
      dacc += x * x;  // zero for padding columns and points past the chunk
    }
    const double y = SC == 0 ? x : (SC == 1 ? x * dv : x / dv);
    xs[tp * XS_LD + tc] = (pr < np && cval) ? y : 0.0;
  };
  auto mma = [&](const d2* ab, const double* xs) {
    if (!mactive) return;
#pragma unroll
    for (int k = 0; k < NA; ++k) {
      const V4<double> xv = load4(&xs[(4 * k + q) * XS_LD + 4 * r16]);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = Mfma<double>::op(ab[k][a], xv.v[b], acc[a][b]);
    }
  };
  auto step = [&](int s, const d2* abc, d2* abn) {
    pro_load(s + 1);
    load_a(s + 1, abn);
    mma(abc, Xs[s & 1]);
    pro_apply(s + 1, Xs[(s + 1) & 1]);
    __syncthreads();
  };
  if (nsteps > 0) {
    pro_load(0);
    load_a(0, ab0);
    pro_apply(0, Xs[0]);
    __syncthreads();
    int s = 0;
    for (; s + 1 < nsteps; s += 2) {
      step(s, ab0, ab1);
      step(s + 1, ab1, ab0);
    }
    if (s < nsteps) step(s, ab0, ab1);
  }
  if (mactive) {
    // tile (a, b) row i = orow(q, r), column r16: k = kb + 2 i + a, c = 4 r16 + b
    double* dst = part + (((int64_t)chunk * ncb + cbx) * kdim + kb) * 64 + 4 * r16;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double* o = dst + (2 * Mfma<double>::orow(q, r) + a) * 64;
        *reinterpret_cast<d2*>(o) = d2{acc[a][0][r], acc[a][1][r]};
        *reinterpret_cast<d2*>(o + 2) = d2{acc[a][2][r], acc[a][3][r]};
      }
  }
  if constexpr (UPD) {
    red[tid] = dacc;
    __syncthreads();
    if (tid < 64) {
      double sum = 0.0;
      for (int k = 0; k < 16; ++k) sum += red[k * 64 + tid];
      dot_part[(int64_t)chunk * ld_dot + c0 + tid] = sum;
    }
  }
}

// Sum the row-major per-chunk partials of the reduce GEMMs into W (float64,
// row-major kdim x ldw, all 64 ncb columns); optionally add the identity.
// One workgroup per 64-element row (column block cb, kdim row k): wave w
// sums the w-th quarter of the chunks (eight interleaved running sums), and
// the four quarters are added in LDS, all in a fixed order.  With
// lower_only, rows k < 64 cb (above the diagonal block) are left alone.
template <typename TP>
__global__ __launch_bounds__(256) void k_reduce_parts_rm(const TP* __restrict__ part, int nchunks, int ncb, int kdim,
                                                         double* __restrict__ W, int ldw, int add_identity,
                                                         int lower_only) {
  __shared__ double red[4][64];
  const int64_t row = blockIdx.x;
  const int k = (int)(row % kdim), cb = (int)(row / kdim);
  if (lower_only && k < 64 * cb) return;  // uniform over the workgroup
  const int cl = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t per = (int64_t)ncb * kdim * 64;
  const int64_t e = row * 64 + cl;
  const int q0 = (int)((int64_t)nchunks * wv / 4), q1 = (int)((int64_t)nchunks * (wv + 1) / 4);
  double s8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int ch = q0;
  for (; ch + 8 <= q1; ch += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) s8[u] += (double)part[(int64_t)(ch + u) * per + e];
  }
  for (int u = 0; ch < q1; ++ch, ++u) s8[u] += (double)part[(int64_t)ch * per + e];
  red[wv][cl] = ((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]));
  __syncthreads();
  if (wv == 0) {
    double sum = (red[0][cl] + red[1][cl]) + (red[2][cl] + red[3][cl]);
    const int cc = cb * 64 + cl;
    if (add_identity && k == cc) sum += 1.0;
    W[(int64_t)k * ldw + cc] = sum;
  }
}

// Column sums of per-workgroup partials: out[c] = sum_k part[k*ldp + c],
// one workgroup per column, fixed order.
__global__ __launch_bounds__(256) void k_colsum(const double* __restrict__ part, int nparts, int ldp,
                                                double* __restrict__ out);

// ------------------------------------------------------------------ SpMM
// Y(p, c) = sum_q S_pq X(q, c), one workgroup per (row cell, 64-column block).
// The rows of the cell are taken 32 at a time; for each chunk of CH
// positions of the cell's 3x3 neighbourhood (Csr::key), the group's sparse
// rows are scattered into a dense 32 x CH LDS tile, the matching block rows
// of X are staged in LDS, and the tile product runs on MFMA 16x16x4 (four
// waves, each two 16x16 output tiles).  The zero entries of the tile cost
// matrix-core cycles only; every nonzero costs one coalesced load and one
// LDS store.  All global accesses go through range-checked buffer resources
// (the group's entries, the neighbourhood's row window of X, the group's
// output rows), so the loop has no divergent branch around a memory access:
// the entries and epilogue inputs load before the first chunk, and the next
// chunk's block rows load while the current chunk is scattered and
// multiplied.  Workgroups are mapped so that each XCD (dispatched
// round-robin) walks a contiguous run of cells, keeping the shared block
// rows of neighbouring cells in its own L2.
template <typename T>
struct SpmmShape {
  static constexpr int CH = 64;                         // neighbourhood positions per chunk
  static constexpr int XLD = 68;                        // LDS row stride of staged block rows
  static constexpr int SLD = CH + 4;                    // LDS row stride of the sparse tile
  static constexpr int XU = CH * 16 / 256;              // 4-column units per thread per chunk
  static constexpr int EPT = 8;                         // entries per thread per batch
};

// Workgroup b -> cell of a gx-wide grid (ncell = gx * gy, row-major cells).
// Workgroups are dispatched to the 8 XCDs round-robin; XCD b & 7 takes the
// (b & 7)-th eighth of a walk over the grid in vertical strips of sw cell
// columns, each strip row by row.  The 3x3 neighbourhoods of the cells in
// flight on one XCD then overlap within a few strip rows, so the block rows
// they share are read from that XCD's L2; only the cell columns bordering a
// strip are read again by the next strip (traffic (sw + 2) / sw of one
// pass).  Returns ncell past the end.
__device__ __forceinline__ int64_t xcd_cell(int64_t b, int64_t ncell, int64_t gx, int sw) {
  const int64_t per = (ncell + 7) >> 3;
  const int64_t j = (b & 7) * per + (b >> 3);
  if (j >= ncell) return ncell;
  const int64_t strip = (int64_t)sw * (ncell / gx);  // cells of a full strip
  const int64_t s = j / strip;                       // every strip before s is full
  const int64_t rem = j - s * strip;
  const int64_t wd = min((int64_t)sw, gx - s * sw);
  const int64_t iy = rem / wd;
  return iy * gx + s * sw + (rem - iy * wd);
}

// Epilogue of the sparse product over row-major n x ld blocks.  Modes:
// SP_STORE Y = acc; SP_ACC Y += acc; SP_PCG Y = acc + P (P may be null),
// dot += H . Y per column; SP_DOT dot += H . acc per column (Y not written).
enum { SP_STORE = 0, SP_ACC = 1, SP_PCG = 2, SP_DOT = 3 };
template <typename T>
struct SpmmEpi {
  T* Y;
  const T* H;
  const T* P;
  int64_t ld;
};

template <typename T, int EM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 3 : 5))) void k_spmm_dense(
    const int64_t* __restrict__ rcs, int64_t ncell, const int64_t* __restrict__ ccs, GridDesc gd,
    const int64_t* __restrict__ rp, const int* __restrict__ key, const T* __restrict__ val, const T* __restrict__ X,
    int ldx, int ncols, SpmmEpi<T> epi, double* __restrict__ dot_part, int ld_dot, int sw) {
  typedef SpmmShape<T> Sh;
  constexpr int CH = Sh::CH, XLD = Sh::XLD, SLD = Sh::SLD, XU = Sh::XU, EPT = Sh::EPT;
  constexpr unsigned TS = sizeof(T);
  __shared__ __attribute__((aligned(16))) T Xs[CH * XLD];
  __shared__ __attribute__((aligned(16))) T Ss[32 * SLD];
  typedef typename Mfma<T>::acc acc_t;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int q = lane >> 4, r16 = lane & 15;
  const int64_t cell = xcd_cell(blockIdx.x, ncell, gd.gx, sw);
  if (cell >= ncell) return;
  const int c0 = blockIdx.y * 64;
  const int64_t rb = rcs[cell], re = rcs[cell + 1];
  const int rt = w >> 1, ct0 = (w & 1) * 2;  // this wave's tiles: rows rt*16.., columns (ct0, ct0+1)*16..
  double dsum0 = 0.0, dsum1 = 0.0;
  if (rb < re) {
    int qb[3], qe[3], off[3];
    const int V = cell_ranges(cell, gd, ccs, qb, qe, off);
    int qlo = 0x7fffffff, qhi = 0;
#pragma unroll
    for (int t = 0; t < 3; ++t)
      if (qe[t] > qb[t]) {
        qlo = min(qlo, qb[t]);
        qhi = max(qhi, qe[t]);
      }
    if (qhi == 0) qlo = 0;
    // the neighbourhood's row window of X
    const __amdgpu_buffer_rsrc_t xrs = rsrc_of(X + (int64_t)qlo * ldx, (int64_t)(qhi - qlo) * ldx * TS);
    // staging unit u = tid + 256 k: chunk row (tid >> 4) + 16 k, columns 4 (tid & 15)..+3
    const int sc4 = (tid & 15) * 4;
    const bool col_ok = c0 + sc4 < ncols;
    auto load_chunk = [&](int vb, V4<T>* xr) {
#pragma unroll
      for (int k = 0; k < XU; ++k) {
        const int v = vb + (tid >> 4) + 16 * k;
        const int qq = v >= off[2] ? v - off[2] + qb[2] : (v >= off[1] ? v - off[1] + qb[1] : v - off[0] + qb[0]);
        const unsigned o = (v < V && col_ok) ? (unsigned)((qq - qlo) * ldx + c0 + sc4) * TS : (unsigned)BUF_OOR;
        xr[k] = bload4<T>(xrs, o);
      }
    };
    auto stage = [&](const V4<T>* xr) {
#pragma unroll
      for (int k = 0; k < XU; ++k) {
        T* dst = &Xs[((tid >> 4) + 16 * k) * XLD + sc4];
        if constexpr (sizeof(T) == 8) {
          *reinterpret_cast<d2*>(dst) = d2{xr[k].v[0], xr[k].v[1]};
          *reinterpret_cast<d2*>(dst + 2) = d2{xr[k].v[2], xr[k].v[3]};
        } else {
          *reinterpret_cast<f4*>(dst) = f4{xr[k].v[0], xr[k].v[1], xr[k].v[2], xr[k].v[3]};
        }
      }
      for (int i = tid; i < 32 * SLD / 4; i += 256) {
        if constexpr (sizeof(T) == 8) {
          *reinterpret_cast<d2*>(&Ss[4 * i]) = d2{0.0, 0.0};
          *reinterpret_cast<d2*>(&Ss[4 * i + 2]) = d2{0.0, 0.0};
        } else {
          *reinterpret_cast<f4*>(&Ss[4 * i]) = f4{0.f, 0.f, 0.f, 0.f};
        }
      }
    };
    auto mma = [&](acc_t& acc0, acc_t& acc1) {
#pragma unroll 4
      for (int ks = 0; ks < CH; ks += 16) {
        const V4<T> a = load4(&Ss[(rt * 16 + r16) * SLD + ks + 4 * q]);
        const T* xb = &Xs[(ks + 4 * q) * XLD + ct0 * 16 + r16];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          acc0 = Mfma<T>::op(a.v[j], xb[j * XLD], acc0);
          acc1 = Mfma<T>::op(a.v[j], xb[j * XLD + 16], acc1);
        }
      }
    };
    for (int64_t g0 = rb; g0 < re; g0 += 32) {
      const int64_t E0 = rp[g0];
      const int ne = (int)(rp[min(g0 + 32, re)] - E0);
      const int nrg = (int)min((int64_t)32, re - g0);
      const __amdgpu_buffer_rsrc_t krs = rsrc_of(key + E0, (int64_t)ne * 4);
      const __amdgpu_buffer_rsrc_t vrs = rsrc_of(val + E0, (int64_t)ne * TS);
      int kk[EPT];
      T vv[EPT];
      auto load_batch = [&](int bi) {
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
          const unsigned i = (unsigned)(bi * 256 * EPT + 256 * k + tid);
          kk[k] = (int)__builtin_amdgcn_raw_buffer_load_b32(krs, i * 4u, 0, 0);
          vv[k] = bload<T>(vrs, i * TS);
        }
      };
      auto scatter = [&](int bi, int vb) {
        const int lim = ne - bi * 256 * EPT - tid;  // entry k of this thread exists iff 256 k < lim
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
          const unsigned kv = (unsigned)kk[k];
          const int sl = (int)(kv & KEY_SLOT_MASK) - vb;
          if (256 * k < lim && (unsigned)sl < (unsigned)CH) Ss[(kv >> KEY_SLOT_BITS) * SLD + sl] = vv[k];
        }
      };
      // epilogue inputs of this wave's two tiles
      const __amdgpu_buffer_rsrc_t yrs = rsrc_of(epi.Y + g0 * epi.ld, (int64_t)nrg * epi.ld * TS);
      constexpr bool HD = EM == SP_PCG || EM == SP_DOT;  // the epilogue reads H
      const __amdgpu_buffer_rsrc_t hrs = rsrc_of(HD ? epi.H + g0 * epi.ld : epi.Y, HD ? (int64_t)nrg * epi.ld * TS : 0);
      const __amdgpu_buffer_rsrc_t prs = rsrc_of(EM == SP_PCG && epi.P ? epi.P + g0 * epi.ld : epi.Y, EM == SP_PCG && epi.P ? (int64_t)nrg * epi.ld * TS : 0);
      unsigned eo[2][4];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int c = c0 + (ct0 + t) * 16 + r16;
#pragma unroll
        for (int r = 0; r < 4; ++r)
          eo[t][r] = c < ncols ? (unsigned)((rt * 16 + Mfma<T>::orow(q, r)) * (int)epi.ld + c) * TS : (unsigned)BUF_OOR;
      }
      T in0[2][4], in1[2][4];
      acc_t acc0 = acc_t{0, 0, 0, 0}, acc1 = acc_t{0, 0, 0, 0};
      V4<T> xr[XU];
      if (ne <= 256 * EPT) {
        // one batch of entries, re-read from cache per chunk (no registers
        // held across the chunk loop); epilogue inputs load at the end
        load_chunk(0, xr);
        for (int vb = 0; vb < V; vb += CH) {
          __syncthreads();  // the previous chunk's products are done with Xs and Ss
          stage(xr);
          __syncthreads();
          load_batch(0);
          load_chunk(vb + CH, xr);  // past the neighbourhood: zero, no traffic
          scatter(0, vb);
          __syncthreads();
          mma(acc0, acc1);
        }
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            if constexpr (EM == SP_ACC) in0[t][r] = bload<T>(yrs, eo[t][r]);
            if constexpr (EM == SP_PCG) {
              in0[t][r] = bload<T>(hrs, eo[t][r]);
              in1[t][r] = bload<T>(prs, eo[t][r]);
            }
            if constexpr (EM == SP_DOT) in0[t][r] = bload<T>(hrs, eo[t][r]);
          }
      } else {
        // long rows: entries re-read per chunk in batches
        const int nbatch = (ne + 256 * EPT - 1) / (256 * EPT);
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            if constexpr (EM == SP_ACC) in0[t][r] = bload<T>(yrs, eo[t][r]);
            if constexpr (EM == SP_PCG) {
              in0[t][r] = bload<T>(hrs, eo[t][r]);
              in1[t][r] = bload<T>(prs, eo[t][r]);
            }
            if constexpr (EM == SP_DOT) in0[t][r] = bload<T>(hrs, eo[t][r]);
          }
        for (int vb = 0; vb < V; vb += CH) {
          load_chunk(vb, xr);
          __syncthreads();
          stage(xr);
          __syncthreads();
          for (int bi = 0; bi < nbatch; ++bi) {
            load_batch(bi);
            scatter(bi, vb);
          }
          __syncthreads();
          mma(acc0, acc1);
        }
      }
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        double d = 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const T a = t == 0 ? acc0[r] : acc1[r];
          if constexpr (EM == SP_STORE) {
            bstore<T>(a, yrs, eo[t][r]);
          } else if constexpr (EM == SP_ACC) {
            bstore<T>(a + in0[t][r], yrs, eo[t][r]);
          } else if constexpr (EM == SP_DOT) {
            d += (double)in0[t][r] * (double)a;  // zero past the group's rows and columns
          } else {
            const T v = (T)((double)a + (double)in1[t][r]);
            bstore<T>(v, yrs, eo[t][r]);
            d += (double)in0[t][r] * (double)v;  // zero past the group's rows and columns
          }
        }
        if (t == 0) dsum0 += d;
        else dsum1 += d;
      }
    }
  }
  if constexpr (EM >= SP_PCG) {
    // column c0 + 16 b + r16 gathers the q groups of the two waves owning tile column b
    dsum0 += __shfl_xor(dsum0, 16, 64);
    dsum0 += __shfl_xor(dsum0, 32, 64);
    dsum1 += __shfl_xor(dsum1, 16, 64);
    dsum1 += __shfl_xor(dsum1, 32, 64);
    double* red = reinterpret_cast<double*>(Ss);
    __syncthreads();
    if (q == 0) {
      red[w * 32 + r16] = dsum0;
      red[w * 32 + 16 + r16] = dsum1;
    }
    __syncthreads();
    if (tid < 64) {
      // wave w holds columns (2 (w & 1)) * 16 .. +31 of row tile w >> 1
      const int half = tid >> 5, o = tid & 31;
      dot_part[cell * ld_dot + c0 + tid] = red[half * 32 + o] + red[(half + 2) * 32 + o];
    }
  }
}

// ------------------------------------------------------------------ SpMM on pre-scattered tiles
// The float32 operator's pattern and values are fixed for a whole solve, so
// the build scatters them once into dense 64 x 64 tiles.  The rows are taken
// by cell pairs: cells 2 sx and 2 sx + 1 of a cell row (one cell at an odd
// grid's right edge), whose rows are contiguous.  The pair's neighbourhood
// is cell rows sy - 1 .. sy + 1 by cell columns 2 sx - 1 .. 2 sx + 2
// (clipped): three contiguous column ranges, 12 cells against 18 for the
// two cells' own neighbourhoods, so a staged chunk of X serves twice the
// rows of a single cell.  A pair has a tile per (64-row group, 64-position
// chunk of its neighbourhood), tiles in (group, chunk) order.  Inside a tile
// the values sit in the order the MFMA 16x16x4 reads them: for row tile rt
// (0..3), 16-position step ks and lane (q, r16), the four positions
// 16 ks + 4 q + j (j = 0..3) of row 16 rt + r16 are one 16-byte word.  The
// product then loads its sparse operand straight into registers (no
// scatter, no tile clearing, no keys); the chunk's block rows of X go
// through LDS, double-buffered, so a chunk costs one workgroup barrier.
// A per-tile mask marks the 16 x 16 blocks (row tile, 16-position step)
// that hold a nonzero, and a wave neither loads nor multiplies the others
// (padding rows and positions, and neighbour points beyond the taper range
// of all 16 rows; the points of each cell are in ascending y).
struct SpmmTile {
  static constexpr int ROWS = 64, CH = 64, FLOATS = ROWS * CH;
  __host__ __device__ static int offset(int r, int v) {
    const int rt = r >> 4, r16 = r & 15, ks = v >> 4, q = (v >> 2) & 3, j = v & 3;
    return (((rt * 4 + ks) * 64 + q * 16 + r16) << 2) + j;
  }
};

// Cell pairs of a gx-wide grid: gxs = ceil(gx / 2) pairs per cell row.
__host__ __device__ __forceinline__ int64_t pair_cols(int64_t gx) { return (gx + 1) >> 1; }

// Rows [rb, re) of pair `pair` (cs: the row grid's cell starts).
__device__ __forceinline__ void pair_rows(int64_t pair, const GridDesc& gd, const int64_t* __restrict__ cs,
                                          int64_t& rb, int64_t& re) {
  const int64_t gxs = pair_cols(gd.gx), sx = pair % gxs, sy = pair / gxs;
  const int64_t c0 = sy * gd.gx + 2 * sx;
  const int64_t c1 = sy * gd.gx + (2 * sx + 2 < gd.gx ? 2 * sx + 2 : gd.gx);
  rb = cs[c0];
  re = cs[c1];
}

// The column points that can neighbour a row of pair `pair`, as cell_ranges
// for a cell: range t is [qb[t], qe[t]) (cell row sy - 1 + t, cell columns
// 2 sx - 1 .. 2 sx + 2, clipped) and starts at position off[t] of the
// concatenation; the return value is the total length.
__device__ __forceinline__ int pair_ranges(int64_t pair, const GridDesc& gd, const int64_t* __restrict__ ccs, int* qb,
                                           int* qe, int* off) {
  const int64_t gxs = pair_cols(gd.gx), sx = pair % gxs, sy = pair / gxs;
  const int64_t xlo = 2 * sx - 1 < 0 ? 0 : 2 * sx - 1;
  const int64_t xhi = 2 * sx + 2 >= gd.gx ? gd.gx - 1 : 2 * sx + 2;
  int tot = 0;
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    const int64_t yy = sy - 1 + t;
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

// One workgroup (4 waves) per cell pair and 64-column block; wave w owns row
// tile w of every 64-row group and the block's first NCT 16-column tiles
// (NCT < 4: a single block of at most 16 NCT columns).
template <int EM, int NCT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_spmm_tiled(
    const int64_t* __restrict__ rcs, int64_t npair, const int64_t* __restrict__ ccs, GridDesc gd,
    const int64_t* __restrict__ toff, const float* __restrict__ tiles, const unsigned* __restrict__ tmask,
    const float* __restrict__ X, int ldx, int ncols, SpmmEpi<float> epi, double* __restrict__ dot_part, int ld_dot,
    int sw) {
  constexpr int CH = SpmmTile::CH, XLD = 68, XU = CH * 16 / 256;
  constexpr unsigned TB = SpmmTile::FLOATS * 4;  // bytes per tile
  constexpr bool HD = EM == SP_PCG || EM == SP_DOT;
  __shared__ __attribute__((aligned(16))) float Xs[2][CH * XLD];
  typedef Mfma<float>::acc acc_t;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int q = lane >> 4, r16 = lane & 15;
  const int64_t pair = xcd_cell(blockIdx.x, npair, pair_cols(gd.gx), sw);
  if (pair >= npair) return;
  const int c0 = blockIdx.y * 64;
  int64_t rb, re;
  pair_rows(pair, gd, rcs, rb, re);
  const int rt = w;  // this wave's row tile
  double dsum[NCT];
#pragma unroll
  for (int t = 0; t < NCT; ++t) dsum[t] = 0.0;
  if (rb < re) {
    int qb[3], qe[3], off[3];
    const int V = pair_ranges(pair, gd, ccs, qb, qe, off);
    int qlo = 0x7fffffff, qhi = 0;
#pragma unroll
    for (int t = 0; t < 3; ++t)
      if (qe[t] > qb[t]) {
        qlo = min(qlo, qb[t]);
        qhi = max(qhi, qe[t]);
      }
    if (qhi == 0) qlo = 0;
    const __amdgpu_buffer_rsrc_t xrs = rsrc_of(X + (int64_t)qlo * ldx, (int64_t)(qhi - qlo) * ldx * 4);
    const int nk = (V + CH - 1) / CH;
    const int ng = (int)((re - rb + SpmmTile::ROWS - 1) / SpmmTile::ROWS);
    const int nt = ng * nk;  // this pair's tiles, (group, chunk) order
    const int64_t t0 = toff[pair];
    const __amdgpu_buffer_rsrc_t trs = rsrc_of(tiles + t0 * SpmmTile::FLOATS, (int64_t)nt * TB);
    // staging unit u = tid + 256 k: chunk row (tid >> 4) + 16 k, columns 4 (tid & 15)..+3
    const int sc4 = (tid & 15) * 4;
    const bool col_ok = c0 + sc4 < ncols;
    auto load_chunk = [&](int vb, V4<float>* xr) {
#pragma unroll
      for (int k = 0; k < XU; ++k) {
        const int v = vb + (tid >> 4) + 16 * k;
        const int qq = v >= off[2] ? v - off[2] + qb[2] : (v >= off[1] ? v - off[1] + qb[1] : v - off[0] + qb[0]);
        const unsigned o = (v < V && col_ok) ? (unsigned)((qq - qlo) * ldx + c0 + sc4) * 4u : (unsigned)BUF_OOR;
        xr[k] = bload4<float>(xrs, o);
      }
    };
    // the sparse operand of tile i for this wave: its four blocks' bits of
    // the tile mask, and the blocks that hold a nonzero (no load for the others)
    auto load_a = [&](int i, f4* ar) -> unsigned {
      const unsigned mk = i < nt ? (tmask[t0 + i] >> (rt * 4)) & 15u : 0u;
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const unsigned o = (mk >> ks) & 1u ? (unsigned)i * TB + (unsigned)(((rt * 4 + ks) * 64 + lane) * 16)
                                           : (unsigned)BUF_OOR;
        ar[ks] = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(trs, o, 0, 0));
      }
      return mk;
    };
    auto stage = [&](float* xs, const V4<float>* xr) {
#pragma unroll
      for (int k = 0; k < XU; ++k)
        *reinterpret_cast<f4*>(&xs[((tid >> 4) + 16 * k) * XLD + sc4]) = f4{xr[k].v[0], xr[k].v[1], xr[k].v[2], xr[k].v[3]};
    };
    auto mma = [&](const float* xs, const f4* a, unsigned mk, acc_t* acc) {
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        if (!((mk >> ks) & 1u)) continue;  // uniform over the wave
        const float* xb = &xs[(ks * 16 + 4 * q) * XLD + r16];
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int t = 0; t < NCT; ++t) acc[t] = Mfma<float>::op(a[ks][j], xb[j * XLD + 16 * t], acc[t]);
      }
    };
    // epilogue offset of this lane's element r of column tile t (past the block's columns: out of range)
    auto eoff = [&](int t, int r) -> unsigned {
      const int c = c0 + 16 * t + r16;
      return c < ncols ? (unsigned)((rt * 16 + Mfma<float>::orow(q, r)) * (int)epi.ld + c) * 4u : (unsigned)BUF_OOR;
    };
    V4<float> xr[XU];
    f4 ar[4], ac[4];
    load_chunk(0, xr);
    unsigned mnext = load_a(0, ar);
    acc_t acc[NCT];
#pragma unroll
    for (int t = 0; t < NCT; ++t) acc[t] = acc_t{0, 0, 0, 0};
    for (int i = 0; i < nt; ++i) {
      const int g = i / nk, k = i - g * nk;
      // chunk buffers alternate over the whole (group, chunk) sequence: the
      // barrier of step i - 1 orders the products of step i - 2 before this write
      float* xs = Xs[i & 1];
      stage(xs, xr);
      __syncthreads();
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) ac[ks] = ar[ks];
      const unsigned mcur = mnext;
      if (i + 1 < nt) {
        const int kn = k + 1 < nk ? k + 1 : 0;  // the next group starts again at chunk 0
        load_chunk(kn * CH, xr);
        mnext = load_a(i + 1, ar);
      }
      const int64_t g0 = rb + (int64_t)g * SpmmTile::ROWS;
      const int nrg = (int)min((int64_t)SpmmTile::ROWS, re - g0);
      const __amdgpu_buffer_rsrc_t yrs = rsrc_of(epi.Y + g0 * epi.ld, (int64_t)nrg * epi.ld * 4);
      const __amdgpu_buffer_rsrc_t hrs = rsrc_of(HD ? epi.H + g0 * epi.ld : epi.Y, HD ? (int64_t)nrg * epi.ld * 4 : 0);
      const __amdgpu_buffer_rsrc_t prs = rsrc_of(EM == SP_PCG && epi.P ? epi.P + g0 * epi.ld : epi.Y,
                                                 EM == SP_PCG && epi.P ? (int64_t)nrg * epi.ld * 4 : 0);
      const bool last = k == nk - 1;
      mma(xs, ac, mcur, acc);
      if (last) {
        // epilogue inputs of this wave's tiles (loaded after the products:
        // with four column tiles in flight they would not fit the registers)
        float in0[NCT][4], in1[NCT][4];
#pragma unroll
        for (int t = 0; t < NCT; ++t)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const unsigned o = eoff(t, r);
            if constexpr (EM == SP_ACC) in0[t][r] = bload<float>(yrs, o);
            if constexpr (HD) in0[t][r] = bload<float>(hrs, o);
            if constexpr (EM == SP_PCG) in1[t][r] = bload<float>(prs, o);
          }
#pragma unroll
        for (int t = 0; t < NCT; ++t) {
          double d = 0.0;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const unsigned o = eoff(t, r);
            const float a = acc[t][r];
            if constexpr (EM == SP_STORE) {
              bstore<float>(a, yrs, o);
            } else if constexpr (EM == SP_ACC) {
              bstore<float>(a + in0[t][r], yrs, o);
            } else if constexpr (EM == SP_DOT) {
              d += (double)in0[t][r] * (double)a;  // zero past the group's rows and columns
            } else {
              const float v = (float)((double)a + (double)in1[t][r]);
              bstore<float>(v, yrs, o);
              d += (double)in0[t][r] * (double)v;  // zero past the group's rows and columns
            }
          }
          dsum[t] += d;
          acc[t] = acc_t{0, 0, 0, 0};
        }
      }
    }
  }
  if constexpr (HD) {
    // column c0 + 16 t + r16 gathers the q groups of the wave, then the four waves (row tiles)
#pragma unroll
    for (int t = 0; t < NCT; ++t) {
      dsum[t] += __shfl_xor(dsum[t], 16, 64);
      dsum[t] += __shfl_xor(dsum[t], 32, 64);
    }
    double* red = reinterpret_cast<double*>(&Xs[0][0]);  // [wave][64 columns]
    __syncthreads();
    if (q == 0) {
#pragma unroll
      for (int t = 0; t < 4; ++t) red[w * 64 + 16 * t + r16] = t < NCT ? dsum[t < NCT ? t : 0] : 0.0;
    }
    __syncthreads();
    if (tid < 64) dot_part[pair * ld_dot + c0 + tid] = (red[tid] + red[64 + tid]) + (red[128 + tid] + red[192 + tid]);
  }
}

// ------------------------------------------------------------------ SDDMM (cell-blocked)
// vals[e] = fn(p, q, d_pq, X_p . Y_q) for every nonzero e = (p, q) of the
// pattern, float64.  One workgroup (8 waves) per row cell; its rows are
// taken 32 at a time and the candidate columns (the 3x3 neighbourhood, in
// Csr::key positions) 256 at a time.  For each 256-wide k chunk the 32 row
// operands are staged in LDS once; wave w owns column tiles w and w + 8 of
// the block and keeps their 2 x 2 (row tile x column tile) MFMA 16x16x4
// accumulators in registers across the chunks, reading its column operands
// from global memory one step ahead.  The dense 32 x 256 block then goes to
// LDS in place of the row operands, and a coalesced pass over the group's
// nonzeros picks each value by its key and applies fn.
template <class XOp, class YOp, class Fn>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_sddmm_cell(const int64_t* __restrict__ rcs, int64_t ncell,
                                                    const double* __restrict__ rxs, const int64_t* __restrict__ ccs,
                                                    const double* __restrict__ cxs, GridDesc gd,
                                                    const int64_t* __restrict__ rp, const int* __restrict__ col,
                                                    const int* __restrict__ key, int kdim, XOp xop, YOp yop, Fn fn,
                                                    double* __restrict__ vals, int sw) {
#pragma clang fp contract(off)
  constexpr int KC = 256, XLD = KC + 2, VB = 256, DLD = VB + 2;
  // the dense block Dv reuses the row-operand tile once the products are
  // done (66 KB of LDS: two workgroups per CU)
  static_assert(DLD == XLD, "Dv aliases Xs");
  __shared__ __attribute__((aligned(16))) double Xs[32 * XLD];
  double* const Dv = Xs;
  typedef Mfma<double>::acc acc_t;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int q = lane >> 4, r16 = lane & 15;
  const int64_t cell = xcd_cell(blockIdx.x, ncell, gd.gx, sw);
  if (cell >= ncell) return;
  const int64_t rb = rcs[cell], re = rcs[cell + 1];
  if (rb >= re) return;
  int qb[3], qe[3], off[3];
  const int V = cell_ranges(cell, gd, ccs, qb, qe, off);
  if (V == 0) return;
  for (int64_t g0 = rb; g0 < re; g0 += 32) {
    const int nrg = (int)min((int64_t)32, re - g0);
    const int64_t E0 = rp[g0], E1 = rp[g0 + nrg];
    for (int vb0 = 0; vb0 < V; vb0 += VB) {
      const int vn = min(VB, V - vb0);
      // this lane's candidate column in each of the wave's two tiles (clamped into range)
      int64_t qcol[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        int v = vb0 + 16 * (w + 8 * t) + r16;
        if (v >= V) v = V - 1;
        qcol[t] = v >= off[2] ? v - off[2] + qb[2] : (v >= off[1] ? v - off[1] + qb[1] : v - off[0] + qb[0]);
      }
      const bool tile_on[2] = {16 * w < vn, 16 * (w + 8) < vn};
      acc_t acc[2][2];
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int a = 0; a < 2; ++a) acc[t][a] = acc_t{0, 0, 0, 0};
      for (int kc0 = 0; kc0 < kdim; kc0 += KC) {
        const int kn = min(KC, kdim - kc0);
        __syncthreads();
        // stage rows g0 .. g0+31 (clamped), k in [kc0, kc0 + kn): 4 k per thread item
        for (int u = tid; u < 32 * (kn / 4); u += 512) {
          const int r = u / (kn / 4), k4 = (u - r * (kn / 4)) * 4;
          const int64_t p = g0 + min(r, nrg - 1);
          const V4<double> x = xop(p, kc0 + k4);
          double* dst = &Xs[r * XLD + k4];
          *reinterpret_cast<d2*>(dst) = d2{x.v[0], x.v[1]};
          *reinterpret_cast<d2*>(dst + 2) = d2{x.v[2], x.v[3]};
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          if (!tile_on[t]) continue;
          V4<double> b0 = yop(qcol[t], kc0 + 4 * q), b1;
          for (int ks = 0; ks < kn; ks += 32) {
            b1 = yop(qcol[t], kc0 + min(ks + 16, kn - 16) + 4 * q);
#pragma unroll
            for (int a = 0; a < 2; ++a) {
              const double* xa = &Xs[(a * 16 + r16) * XLD + ks + 4 * q];
#pragma unroll
              for (int j = 0; j < 4; ++j) acc[t][a] = Mfma<double>::op(xa[j], b0.v[j], acc[t][a]);
            }
            // kn is a multiple of 64, so the second half-step always exists
            b0 = yop(qcol[t], kc0 + min(ks + 32, kn - 16) + 4 * q);
#pragma unroll
            for (int a = 0; a < 2; ++a) {
              const double* xa = &Xs[(a * 16 + r16) * XLD + ks + 16 + 4 * q];
#pragma unroll
              for (int j = 0; j < 4; ++j) acc[t][a] = Mfma<double>::op(xa[j], b1.v[j], acc[t][a]);
            }
          }
        }
      }
      // dense block to LDS: row a*16 + orow(q, r), position 16 (w + 8 t) + r16
      __syncthreads();  // every wave is done reading Xs
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        if (!tile_on[t]) continue;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int r = 0; r < 4; ++r) Dv[(a * 16 + Mfma<double>::orow(q, r)) * DLD + 16 * (w + 8 * t) + r16] = acc[t][a][r];
      }
      __syncthreads();
      for (int64_t e = E0 + tid; e < E1; e += 512) {
        const unsigned kv = (unsigned)key[e];
        const int sl = (int)(kv & KEY_SLOT_MASK) - vb0;
        if ((unsigned)sl < (unsigned)vn) {
          const int row = (int)(kv >> KEY_SLOT_BITS);
          const int64_t p = g0 + row;
          const int64_t qq = col[e];
          const double dx = rxs[2 * p] - cxs[2 * qq];
          const double dy = rxs[2 * p + 1] - cxs[2 * qq + 1];
          const double dx2 = dx * dx;
          const double dy2 = dy * dy;
          const double d2v = dx2 + dy2;
          vals[e] = fn(p, qq, sqrt(d2v), Dv[row * DLD + sl]);
        }
      }
      __syncthreads();  // Dv and Xs are reused by the next block
    }
  }
}

// Symmetric SDDMM over one point set (rows = columns, X_p . Y_q = X_q . Y_p
// and fn symmetric off the diagonal): each unordered pair of cells is
// computed once.  The workgroup of cell c = (cx, cy) forms the dense block
// of its rows against its forward neighbourhood only, the cells (cx, cy),
// (cx + 1, cy) and (cx - 1 .. cx + 1, cy + 1), two contiguous column ranges
// [c, right neighbour] and [row cy + 1]; it writes (a) every nonzero of its
// rows whose column lies in that set, and (b) the mirror nonzeros (p', q)
// with p' in a forward cell other than c and q among its rows, from the
// transposed block entry.  A nonzero (p, q) with q behind c is written by
// the workgroup of q's cell under (b).  Same blocking and MFMA scheme as
// k_sddmm_cell on half the columns.
template <class XOp, class YOp, class Fn>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_sddmm_sym(const int64_t* __restrict__ cs, int64_t ncell,
                                                   const double* __restrict__ xs, GridDesc gd,
                                                   const int64_t* __restrict__ rp, const int* __restrict__ col,
                                                   const int* __restrict__ key, int kdim, XOp xop, YOp yop, Fn fn,
                                                   double* __restrict__ vals, int sw) {
#pragma clang fp contract(off)
  constexpr int KC = 256, XLD = KC + 2, VB = 256, DLD = VB + 2;
  // the dense block Dv reuses the row-operand tile once the products are
  // done (66 KB of LDS: two workgroups per CU)
  static_assert(DLD == XLD, "Dv aliases Xs");
  // operand arithmetic: the rows' element type (float64, or float32 with
  // float32 MFMA); the dense block is float64 either way
  typedef typename XOp::value_type T;
  __shared__ __attribute__((aligned(16))) double Sm[32 * XLD];
  T* const Xs = reinterpret_cast<T*>(Sm);
  double* const Dv = Sm;
  typedef typename Mfma<T>::acc acc_t;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int q = lane >> 4, r16 = lane & 15;
  const int64_t cell = xcd_cell(blockIdx.x, ncell, gd.gx, sw);
  if (cell >= ncell) return;
  const int64_t rb = cs[cell], re = cs[cell + 1];
  if (rb >= re) return;
  const int64_t cx = cell % gd.gx, cy = cell / gd.gx;
  const int64_t xlo = cx - 1 < 0 ? 0 : cx - 1;
  const int64_t xhi = cx + 1 >= gd.gx ? gd.gx - 1 : cx + 1;
  // forward ranges: [f1b, f1e) = this cell and its right neighbour,
  // [f2b, f2e) = the three cells of the next cell row (empty on the last)
  const int64_t f1b = rb, f1e = cs[cy * gd.gx + xhi + 1];
  int64_t f2b = 0, f2e = 0;
  if (cy + 1 < gd.gy) {
    f2b = cs[(cy + 1) * gd.gx + xlo];
    f2e = cs[(cy + 1) * gd.gx + xhi + 1];
  }
  const int n1 = (int)(f1e - f1b);
  const int V = n1 + (int)(f2e - f2b);
  for (int64_t g0 = rb; g0 < re; g0 += 32) {
    const int nrg = (int)min((int64_t)32, re - g0);
    const int64_t E0 = rp[g0], E1 = rp[g0 + nrg];
    for (int vb0 = 0; vb0 < V; vb0 += VB) {
      const int vn = min(VB, V - vb0);
      int64_t qcol[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        int v = vb0 + 16 * (w + 8 * t) + r16;
        if (v >= V) v = V - 1;
        qcol[t] = v < n1 ? f1b + v : f2b + (v - n1);
      }
      const bool tile_on[2] = {16 * w < vn, 16 * (w + 8) < vn};
      acc_t acc[2][2];
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int a = 0; a < 2; ++a) acc[t][a] = acc_t{0, 0, 0, 0};
      for (int kc0 = 0; kc0 < kdim; kc0 += KC) {
        const int kn = min(KC, kdim - kc0);
        __syncthreads();
        for (int u = tid; u < 32 * (kn / 4); u += 512) {
          const int r = u / (kn / 4), k4 = (u - r * (kn / 4)) * 4;
          const int64_t p = g0 + min(r, nrg - 1);
          const V4<T> x = xop(p, kc0 + k4);
          T* dst = &Xs[r * XLD + k4];
          if constexpr (sizeof(T) == 8) {
            *reinterpret_cast<d2*>(dst) = d2{x.v[0], x.v[1]};
            *reinterpret_cast<d2*>(dst + 2) = d2{x.v[2], x.v[3]};
          } else {  // float rows of XLD = 258 are 8-byte aligned
            *reinterpret_cast<float2*>(dst) = float2{x.v[0], x.v[1]};
            *reinterpret_cast<float2*>(dst + 2) = float2{x.v[2], x.v[3]};
          }
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          if (!tile_on[t]) continue;
          V4<T> b0 = yop(qcol[t], kc0 + 4 * q), b1;
          for (int ks = 0; ks < kn; ks += 32) {
            b1 = yop(qcol[t], kc0 + min(ks + 16, kn - 16) + 4 * q);
#pragma unroll
            for (int a = 0; a < 2; ++a) {
              const T* xa = &Xs[(a * 16 + r16) * XLD + ks + 4 * q];
#pragma unroll
              for (int j = 0; j < 4; ++j) acc[t][a] = Mfma<T>::op(xa[j], b0.v[j], acc[t][a]);
            }
            b0 = yop(qcol[t], kc0 + min(ks + 32, kn - 16) + 4 * q);
#pragma unroll
            for (int a = 0; a < 2; ++a) {
              const T* xa = &Xs[(a * 16 + r16) * XLD + ks + 16 + 4 * q];
#pragma unroll
              for (int j = 0; j < 4; ++j) acc[t][a] = Mfma<T>::op(xa[j], b1.v[j], acc[t][a]);
            }
          }
        }
      }
      __syncthreads();  // every wave is done reading Xs
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        if (!tile_on[t]) continue;
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            Dv[(a * 16 + Mfma<T>::orow(q, r)) * DLD + 16 * (w + 8 * t) + r16] = (double)acc[t][a][r];
      }
      __syncthreads();
      // (a) this group's nonzeros with a forward column
      for (int64_t e = E0 + tid; e < E1; e += 512) {
        const int64_t qq = col[e];
        const int fp = (qq >= f1b && qq < f1e) ? (int)(qq - f1b) : ((qq >= f2b && qq < f2e) ? n1 + (int)(qq - f2b) : -1);
        const int sl = fp - vb0;
        if (fp >= 0 && (unsigned)sl < (unsigned)vn) {
          const int row = (int)((unsigned)key[e] >> KEY_SLOT_BITS);
          const int64_t p = g0 + row;
          const double dx = xs[2 * p] - xs[2 * qq];
          const double dy = xs[2 * p + 1] - xs[2 * qq + 1];
          const double dx2 = dx * dx;
          const double dy2 = dy * dy;
          vals[e] = fn(p, qq, sqrt(dx2 + dy2), Dv[row * DLD + sl]);
        }
      }
      // (b) mirror nonzeros: rows p' of the forward cells after this one
      // whose column is in this group; wave w takes rows w, w + 8, ...
      {
        const int64_t m1 = cs[cell + 1];  // first row after this cell
        const int nm1 = (int)(f1e - m1), nm = nm1 + (int)(f2e - f2b);
        for (int j = w; j < nm; j += 8) {
          const int64_t pp = j < nm1 ? m1 + j : f2b + (j - nm1);
          const int fp = pp < f1e ? (int)(pp - f1b) : n1 + (int)(pp - f2b);
          const int sl = fp - vb0;
          if ((unsigned)sl >= (unsigned)vn) continue;
          const int64_t a0 = rp[pp], a1 = rp[pp + 1];
          for (int64_t e = a0 + lane; e < a1; e += 64) {
            const int64_t qq = col[e];
            if (qq >= g0 && qq < g0 + nrg) {
              const double dx = xs[2 * pp] - xs[2 * qq];
              const double dy = xs[2 * pp + 1] - xs[2 * qq + 1];
              const double dx2 = dx * dx;
              const double dy2 = dy * dy;
              vals[e] = fn(pp, qq, sqrt(dx2 + dy2), Dv[(int)(qq - g0) * DLD + sl]);
            }
          }
        }
      }
      __syncthreads();  // Dv and Xs are reused by the next block
    }
  }
}

// ------------------------------------------------------------------ bfloat16 MFMA passes (MIXED_BF16A)
// v_mfma_f32_16x16x32_bf16: lane l supplies A[l % 16][8 (l / 16) + j] and
// B[8 (l / 16) + j][l % 16], j = 0..7, and holds D[4 (l / 16) + r][l % 16],
// r = 0..3.  A (the rounded factor) is exact in bfloat16; the float32 block
// operand x is split into three bfloat16 parts, hi = bf16(x), mid =
// bf16(x - hi), lo = bf16(x - hi - mid) (each difference exact in float32),
// which leave |x - hi - mid - lo| <= 2^-27 |x|.  The three products per tile
// are exact and accumulate in float32, so a pass agrees with the float32
// product of the widened factor to float32 accumulation order.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ unsigned bf16_rne_bits(float x) {
  const unsigned u = __float_as_uint(x);
  return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}
// the three bfloat16 parts of x
__device__ __forceinline__ void bf16_split3(float x, uint16_t& hi, uint16_t& mid, uint16_t& lo) {
  const unsigned h = bf16_rne_bits(x);
  const float r1 = x - __uint_as_float(h << 16);
  const unsigned m = bf16_rne_bits(r1);
  const float r2 = r1 - __uint_as_float(m << 16);
  hi = (uint16_t)h;
  mid = (uint16_t)m;
  lo = (uint16_t)bf16_rne_bits(r2);
}
__device__ __forceinline__ f4 mfma_bf16(u4v a, u4v b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c, 0, 0,
                                                 0);
}

// Residual pass on the bfloat16 MFMA: same contract, prologue modes and
// partial layout as k_reduce_gemm_f32 (grid (ncb, nchunks), 512 threads,
// wave w owns kdim rows 64 w .. 64 w + 63 as four 16-row tiles against the
// workgroup's 64 columns).  A comes point-interleaved, [n/8][kdim][8], so
// one 16-byte load gives a lane the eight points of its MFMA k slice for
// one kdim row.  Points are taken 32 per step (one MFMA k extent); the
// prologue of the next step writes the three parts of X to the other half
// of a double-buffered LDS block as [part][column][point], and the A loads
// of the step two ahead are in flight while the matrix cores work.
template <bool UPD, int SC>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2))) void k_reduce_bf16(
    int64_t npts, int pts_per_chunk, int kdim, int ncols, const uint16_t* __restrict__ A8, F32Pro pro,
    float* __restrict__ part, double* __restrict__ dot_part, int ld_dot) {
  constexpr int SP = 32;       // points per step
  constexpr int NP = SP / 8;   // prologue elements per thread per step
  constexpr int XST = 40;      // LDS stride (bfloat16) of one column's points
  __shared__ __attribute__((aligned(16))) uint16_t Xs[2][3][64 * XST];
  __shared__ double red[512];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int q = lane >> 4, r16 = lane & 15;
  const int c0 = blockIdx.x * 64;
  const int ncb = gridDim.x;
  const int chunk = blockIdx.y;
  const int kb = w * 64;
  const bool mactive = kb < kdim;
  const int64_t pbeg = (int64_t)chunk * pts_per_chunk;  // a multiple of 8
  const int64_t pend = min(npts, pbeg + pts_per_chunk);
  const int np = pend > pbeg ? (int)(pend - pbeg) : 0;
  const int nsteps = (np + SP - 1) / SP;
  const int tc = tid & 63, tp = tid >> 6;  // prologue: column c0 + tc, points tp + 8 u
  const int c = c0 + tc;
  const bool cval = c < ncols;
  f4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f4{0, 0, 0, 0};
  double dacc = 0.0;
  u4v ab0[4] = {}, ab1[4] = {}, ab2[4] = {};
  const int ngr = (np + 7) / 8;  // point groups of the chunk (zero-padded past npts)
  const __amdgpu_buffer_rsrc_t arsrc = rsrc_of(A8 + (pbeg / 8) * kdim * 8, (int64_t)ngr * kdim * 16);
  const __amdgpu_buffer_rsrc_t srsrc = rsrc_of(pro.S + pbeg * pro.ld, (int64_t)np * pro.ld * 4);
  const __amdgpu_buffer_rsrc_t vrsrc = rsrc_of(UPD ? pro.V + pbeg * pro.ld : pro.S, UPD ? (int64_t)np * pro.ld * 4 : 0);
  const __amdgpu_buffer_rsrc_t drsrc = rsrc_of(SC ? pro.sc + pbeg : (const double*)pro.S, SC ? (int64_t)np * 8 : 0);
  const double a_c = (UPD && cval) ? pro.alpha[c] : 0.0;
  // byte offset of (group q of step 0, kdim row kb + r16)
  const unsigned a_off = mactive ? (unsigned)(q * kdim + kb + r16) * 16u : (unsigned)BUF_OOR;
  const unsigned a_step = (unsigned)(4 * kdim) * 16u;
  const unsigned s_off = cval ? (unsigned)(tp * (int)pro.ld + c) * 4u : (unsigned)BUF_OOR;
  const unsigned s_step = 8u * (unsigned)pro.ld * 4u;
  float sv[NP], vv[NP];
  double dv[NP];
  auto load_a = [&](int s, u4v* ab) {
    const unsigned so = a_off + (unsigned)s * a_step;
#pragma unroll
    for (int a = 0; a < 4; ++a) ab[a] = __builtin_bit_cast(u4v, __builtin_amdgcn_raw_buffer_load_b128(arsrc, so + 256u * a, 0, 0));
  };
  auto pro_load = [&](int s) {
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      const int pr = s * SP + tp + 8 * u;
      const unsigned o = s_off + (unsigned)(s * NP + u) * s_step;
      sv[u] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(srsrc, o, 0, 0));
      vv[u] = UPD ? __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(vrsrc, o, 0, 0)) : 0.f;
      dv[u] = SC ? __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(drsrc, (unsigned)pr * 8u, 0, 0)) : 1.0;
    }
  };
  auto pro_apply = [&](int s, int buf) {
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      const int pl = tp + 8 * u;
      const int pr = s * SP + pl;
      double x = (double)sv[u];
      if constexpr (UPD) {
        const float rt = (float)(x - a_c * (double)vv[u]);
        const unsigned o = s_off + (unsigned)(s * NP + u) * s_step;
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, rt), srsrc, o, 0, 0);
        x = (double)rt;
        dacc += x * x;  // zero for padding columns and points past the chunk
      }
      const double y = SC == 0 ? x : (SC == 1 ? x * dv[u] : x / dv[u]);
      const float yf = (pr < np && cval) ? (float)y : 0.f;
      uint16_t h, m, l;
      bf16_split3(yf, h, m, l);
      Xs[buf][0][tc * XST + pl] = h;
      Xs[buf][1][tc * XST + pl] = m;
      Xs[buf][2][tc * XST + pl] = l;
    }
  };
  auto mma = [&](const u4v* ab, int buf) {
    if (!mactive) return;
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int P = 0; P < 3; ++P) {
        const u4v bop = *reinterpret_cast<const u4v*>(&Xs[buf][P][(16 * b + r16) * XST + 8 * q]);
#pragma unroll
        for (int a = 0; a < 4; ++a) acc[a][b] = mfma_bf16(ab[a], bop, acc[a][b]);
      }
  };
  auto step = [&](int s, const u4v* abc, u4v* abn) {
    pro_load(s + 1);
    load_a(s + 2, abn);
    mma(abc, s & 1);
    pro_apply(s + 1, (s + 1) & 1);
    __syncthreads();
  };
  if (nsteps > 0) {
    pro_load(0);
    load_a(0, ab0);
    load_a(1, ab1);
    pro_apply(0, 0);
    __syncthreads();
    int s = 0;
    for (; s + 2 < nsteps; s += 3) {
      step(s, ab0, ab2);
      step(s + 1, ab1, ab0);
      step(s + 2, ab2, ab1);
    }
    if (s < nsteps) step(s, ab0, ab2);
    if (s + 1 < nsteps) step(s + 1, ab1, ab0);
  }
  if (mactive) {
    // tile (a, b) element r: k = kb + 16 a + 4 q + r, column 16 b + r16
    float* dst = part + (((int64_t)chunk * ncb + blockIdx.x) * kdim + kb) * 64 + r16;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int b = 0; b < 4; ++b) dst[(16 * a + 4 * q + r) * 64 + 16 * b] = acc[a][b][r];
  }
  if constexpr (UPD) {
    red[tid] = dacc;
    __syncthreads();
    if (tid < 64) {
      double sum = 0.0;
      for (int k = 0; k < 8; ++k) sum += red[k * 64 + tid];
      dot_part[(int64_t)chunk * ld_dot + c0 + tid] = sum;
    }
  }
}

// Woodbury expansion on the bfloat16 MFMA: same contract and epilogue as
// k_rows_gemm_f32 for a column block of at most BF16_ROWS_NC columns.  The
// three parts of the kdim x 64 block of G live in LDS as [part][column][k]
// (row stride kdim + 8) for the first BF16_ROWS_NC columns, with a zero row
// standing in for the padding columns; that fits kdim <= 512 in 160 KB.
// Each of the 16 waves is persistent over 16-row tiles and walks k in steps
// of 64: a lane loads 32 contiguous bytes of its row (k = 64 kb + 16 q' +
// 8 t + j for MFMA t, j), two steps ahead in the flattened (tile, k block)
// stream.
constexpr int BF16_ROWS_NC = 52;
inline size_t bf16_rows_lds(int kdim) { return (size_t)(3 * BF16_ROWS_NC + 1) * (kdim + 8) * 2; }

template <int EM>
__global__ __launch_bounds__(1024) void k_rows_bf16(int64_t nrows, int kdim, const uint16_t* __restrict__ A,
                                                    int64_t lda, const float* __restrict__ G, int ldg, int ncols,
                                                    F32RowsEpi epi, double* __restrict__ dot_part, int ld_dot) {
  extern __shared__ __attribute__((aligned(16))) uint16_t gsh[];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int q = lane >> 4, r16 = lane & 15;
  const int c0 = blockIdx.y * 64;
  const int gst = kdim + 8;
  for (int e = tid; e < kdim * BF16_ROWS_NC; e += 1024) {
    const int k = e / BF16_ROWS_NC, cc = e - k * BF16_ROWS_NC;
    const float v = (c0 + cc < ncols) ? G[(int64_t)k * ldg + c0 + cc] : 0.f;
    uint16_t h, m, l;
    bf16_split3(v, h, m, l);
    gsh[(0 * BF16_ROWS_NC + cc) * gst + k] = h;
    gsh[(1 * BF16_ROWS_NC + cc) * gst + k] = m;
    gsh[(2 * BF16_ROWS_NC + cc) * gst + k] = l;
  }
  for (int e = tid; e < gst; e += 1024) gsh[3 * BF16_ROWS_NC * gst + e] = 0;
  __syncthreads();
  // element offsets of this lane's G rows (column 16 b + r16, part P)
  int brow[4][3];
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int P = 0; P < 3; ++P) {
      const int cc = 16 * b + r16;
      brow[b][P] = (cc < BF16_ROWS_NC ? (P * BF16_ROWS_NC + cc) : 3 * BF16_ROWS_NC) * gst + 16 * q;
    }
  const int nkb = kdim / 64;
  const int64_t ntile = (nrows + 15) / 16;
  const int64_t gw = (int64_t)blockIdx.x * 16 + w, GW = (int64_t)gridDim.x * 16;
  const int64_t ntw = gw < ntile ? (ntile - gw + GW - 1) / GW : 0;
  const unsigned lane_off = (unsigned)(r16 * lda + 16 * q) * 2u;
  double dsum[4] = {0, 0, 0, 0};
  int64_t lj = 0;
  int lkb = 0;
  auto load_next = [&](u4v* ab) {
    const int64_t row0 = (gw + lj * GW) * 16;
    const int64_t nr = lj < ntw ? min((int64_t)16, nrows - row0) : 0;
    const __amdgpu_buffer_rsrc_t rs = rsrc_of(A + (lj < ntw ? row0 * lda : 0), nr * lda * 2);
    const unsigned o = lane_off + (unsigned)lkb * 128u;
    ab[0] = __builtin_bit_cast(u4v, __builtin_amdgcn_raw_buffer_load_b128(rs, o, 0, 0));
    ab[1] = __builtin_bit_cast(u4v, __builtin_amdgcn_raw_buffer_load_b128(rs, o + 16u, 0, 0));
    if (++lkb == nkb) {
      lkb = 0;
      ++lj;
    }
  };
  f4 acc[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) acc[b] = f4{0, 0, 0, 0};
  int64_t cj = 0;
  int ckb = 0;
  auto epilogue = [&]() {
    const int64_t row0 = (gw + cj * GW) * 16;
    const int64_t nr = min((int64_t)16, nrows - row0);
    const __amdgpu_buffer_rsrc_t ry = rsrc_of(epi.Y ? epi.Y + row0 * epi.ld : (const void*)A, epi.Y ? nr * epi.ld * 4 : 0);
    const __amdgpu_buffer_rsrc_t rr = rsrc_of(epi.R + row0 * epi.ld, nr * epi.ld * 4);
    const __amdgpu_buffer_rsrc_t rd = rsrc_of(epi.Dinv + row0, nr * 8);
    const __amdgpu_buffer_rsrc_t rh = rsrc_of(EM == ROWS_PCG_INIT ? epi.H + row0 * epi.ld : (const void*)A, EM == ROWS_PCG_INIT ? nr * epi.ld * 4 : 0);
    const __amdgpu_buffer_rsrc_t rp = rsrc_of(EM == ROWS_PCG_INIT ? epi.P + row0 * epi.ld : (const void*)A, EM == ROWS_PCG_INIT ? nr * epi.ld * 4 : 0);
    const __amdgpu_buffer_rsrc_t rq = rsrc_of(EM == ROWS_PCG_INIT ? epi.Q0 + row0 * epi.ld : (const void*)A, EM == ROWS_PCG_INIT ? nr * epi.ld * 4 : 0);
    float xin[4][4];
    double di[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      di[r] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rd, (unsigned)(4 * q + r) * 8u, 0, 0));
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int cc = c0 + b * 16 + r16;
        const unsigned o = cc < ncols ? (unsigned)((4 * q + r) * (int)epi.ld + cc) * 4u : (unsigned)BUF_OOR;
        xin[r][b] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rr, o, 0, 0));
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int cc = c0 + b * 16 + r16;
        const unsigned o = cc < ncols ? (unsigned)((4 * q + r) * (int)epi.ld + cc) * 4u : (unsigned)BUF_OOR;
        const float v = acc[b][r];
        const double rv = (double)xin[r][b];
        const double qv = (rv - (double)v) * di[r];
        dsum[b] += rv * qv;  // zero for points past the tile and padding columns
        if constexpr (EM == ROWS_PCG) {
          __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), ry, o, 0, 0);
        } else {
          const unsigned qb = __builtin_bit_cast(unsigned, (float)qv);
          __builtin_amdgcn_raw_buffer_store_b32(qb, rh, o, 0, 0);
          __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), rp, o, 0, 0);
          __builtin_amdgcn_raw_buffer_store_b32(qb, rq, o, 0, 0);
        }
      }
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[b] = f4{0, 0, 0, 0};
  };
  auto step = [&](const u4v* cur, u4v* ahead) {
    load_next(ahead);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int P = 0; P < 3; ++P) {
          const u4v g = *reinterpret_cast<const u4v*>(&gsh[brow[b][P] + ckb * 64 + 8 * t]);
          acc[b] = mfma_bf16(cur[t], g, acc[b]);
        }
    if (++ckb == nkb) {
      epilogue();
      ckb = 0;
      ++cj;
    }
  };
  const int64_t nflat = ntw * nkb;
  u4v b0[2], b1[2], b2[2];
  load_next(b0);
  load_next(b1);
  int64_t f = 0;
  for (; f + 2 < nflat; f += 3) {
    step(b0, b2);
    step(b1, b0);
    step(b2, b1);
  }
  if (f < nflat) step(b0, b2);
  if (f + 1 < nflat) step(b1, b0);
  // column dots: the four row groups of each wave, then the 16 waves
  __syncthreads();  // G is no longer read: reuse its LDS
  double* red = reinterpret_cast<double*>(gsh);
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    double v = dsum[b];
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    if (q == 0) red[w * 64 + b * 16 + r16] = v;
  }
  __syncthreads();
  if (tid < 64) {
    double sacc = 0.0;
    for (int k = 0; k < 16; ++k) sacc += red[k * 64 + tid];
    dot_part[(int64_t)blockIdx.x * ld_dot + c0 + tid] = sacc;
  }
}


// ------------------------------------------------------------------ float32 passes on the bfloat16 MFMA
// The float32 PCG passes (MIXED_FP32) are bound by the float32 matrix cores
// (16x16x4, 2048 flop per 32 cycles) at the 500k x 512 shape.  The bfloat16
// 16x16x32 instruction does sixteen times the flops per cycle, so the passes
// run there with every float32 operand split into three bfloat16 parts:
// h = bf16(x), m = bf16(x - h), l = bf16(x - h - m), each to nearest even.
// For a normal float32 x the split is exact, x = h + m + l (x - h is a
// multiple of x's last place below 2^-8 |x|, so x - h - m has at most eight
// significant bits).  Each partial product a_i x_j is exact in float32.  Of
// the nine, the six with i + j <= 2 are taken, smallest first; the three
// dropped ones (m l, l m, l l) are below 2^-23 |a x| together, under the
// float32 accumulation error of a k-long sum (about 2^-24 sqrt(k) of the
// sum of |terms|).  Taking m l and l m as well (eight products) did not
// spare the float32 iteration its breakdowns on strongly low-rank problems
// (those go to float64) and cost 14 us per expansion.  The six take 6/16 of the
// float32 matrix-core time, so the passes are bound by the HBM stream of A.
typedef float split_f2 __attribute__((ext_vector_type(2)));
typedef __bf16 split_b2 __attribute__((ext_vector_type(2)));
// two floats rounded to bfloat16 (nearest even, one v_cvt_pk_bf16_f32), a in the low half
__device__ __forceinline__ unsigned bf16_pk2(float a, float b) {
  return __builtin_bit_cast(unsigned, __builtin_convertvector((split_f2){a, b}, split_b2));
}
// the three bfloat16 parts of two floats (h, m, l: one packed pair each)
__device__ __forceinline__ void bf16_split_pair(float a, float b, unsigned& h, unsigned& m, unsigned& l) {
  h = bf16_pk2(a, b);
  const float ra = a - __uint_as_float(h << 16), rb = b - __uint_as_float(h & 0xffff0000u);
  m = bf16_pk2(ra, rb);
  const float sa = ra - __uint_as_float(m << 16), sb = rb - __uint_as_float(m & 0xffff0000u);
  l = bf16_pk2(sa, sb);
}

// Residual pass with split operands: same contract, prologue modes and
// partial layout as k_reduce_gemm_f32, grid (ncb, nchunks), 512 threads.
// Only the first NB 16-column tiles of a column block are multiplied (a
// single block of at most 16 NB columns; the others stay zero).
// Wave w owns kdim rows 64 w .. 64 w + 63 as four 16-row tiles interleaved by
// four (tile a, row i: kdim row 64 w + 4 i + a), so a lane reads its four
// rows of one point with one 16-byte load from the point-major float32 A and
// splits them in registers; a step takes 32 points (one MFMA k extent).  The
// prologue writes the three parts of X to a double-buffered LDS block as
// [part][column][point].  A loads run one step ahead of their use, the
// prologue inputs one step ahead of the prologue that writes them to LDS.
template <bool UPD, int SC, int NB>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2))) void k_reduce_split(
    int64_t npts, int pts_per_chunk, int kdim, int ncols, const float* __restrict__ A, F32Pro pro,
    float* __restrict__ part, double* __restrict__ dot_part, int ld_dot) {
  constexpr int SP = 32;       // points per step (one MFMA k extent)
  constexpr int NP = SP / 8;   // prologue elements per thread per step
  constexpr int XST = 40;      // LDS stride (bfloat16) of one column's points
  __shared__ __attribute__((aligned(16))) uint16_t Xs[2][3][64 * XST];
  __shared__ double red[512];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int q = lane >> 4, r16 = lane & 15;
  const int c0 = blockIdx.x * 64;
  const int ncb = gridDim.x;
  const int chunk = blockIdx.y;
  const int kb = w * 64;
  const bool mactive = kb < kdim;
  const int64_t pbeg = (int64_t)chunk * pts_per_chunk;
  const int64_t pend = min(npts, pbeg + pts_per_chunk);
  const int np = pend > pbeg ? (int)(pend - pbeg) : 0;
  const int nsteps = (np + SP - 1) / SP;
  const int tc = tid & 63, tp = tid >> 6;
  const int c = c0 + tc;
  const bool cval = c < ncols;
  f4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f4{0, 0, 0, 0};
  double dacc = 0.0;
  const __amdgpu_buffer_rsrc_t arsrc = rsrc_of(A + pbeg * kdim, (int64_t)np * kdim * 4);
  const __amdgpu_buffer_rsrc_t srsrc = rsrc_of(pro.S + pbeg * pro.ld, (int64_t)np * pro.ld * 4);
  const __amdgpu_buffer_rsrc_t vrsrc = rsrc_of(UPD ? pro.V + pbeg * pro.ld : pro.S, UPD ? (int64_t)np * pro.ld * 4 : 0);
  const __amdgpu_buffer_rsrc_t drsrc = rsrc_of(SC ? pro.sc + pbeg : (const double*)pro.S, SC ? (int64_t)np * 8 : 0);
  const double a_c = (UPD && cval) ? pro.alpha[c] : 0.0;
  // lane's A: points 8 q + j of the step, kdim rows kb + 4 r16 .. + 3 (one 16-byte load per point)
  const unsigned a_off = mactive ? (unsigned)((8 * q) * kdim + kb + 4 * r16) * 4u : (unsigned)BUF_OOR;
  const unsigned a_pt = (unsigned)kdim * 4u;
  const unsigned a_step = (unsigned)(SP * kdim) * 4u;
  const unsigned s_off = cval ? (unsigned)(tp * (int)pro.ld + c) * 4u : (unsigned)BUF_OOR;
  const unsigned s_step = 8u * (unsigned)pro.ld * 4u;
  float sv[2][NP], vv[2][NP];
  double dv[2][NP];
  auto load_a = [&](int s, f4* ab) {
    const unsigned so = a_off + (unsigned)s * a_step;
#pragma unroll
    for (int j = 0; j < 8; ++j) ab[j] = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(arsrc, so + a_pt * j, 0, 0));
  };
  auto pro_load = [&](int s, int set) {
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      const int pr = s * SP + tp + 8 * u;
      const unsigned o = s_off + (unsigned)(s * NP + u) * s_step;
      sv[set][u] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(srsrc, o, 0, 0));
      vv[set][u] = UPD ? __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(vrsrc, o, 0, 0)) : 0.f;
      dv[set][u] = SC ? __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(drsrc, (unsigned)pr * 8u, 0, 0)) : 1.0;
    }
  };
  auto pro_apply = [&](int s, int set, int buf) {
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      const int pl = tp + 8 * u;
      const int pr = s * SP + pl;
      double x = (double)sv[set][u];
      if constexpr (UPD) {
        const float rt = (float)(x - a_c * (double)vv[set][u]);
        const unsigned o = s_off + (unsigned)(s * NP + u) * s_step;
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, rt), srsrc, o, 0, 0);
        x = (double)rt;
        dacc += x * x;
      }
      const double y = SC == 0 ? x : (SC == 1 ? x * dv[set][u] : x / dv[set][u]);
      const float yf = (pr < np && cval) ? (float)y : 0.f;
      const unsigned h = bf16_pk2(yf, 0.f);
      const float r1 = yf - __uint_as_float(h << 16);
      const unsigned m = bf16_pk2(r1, 0.f);
      const float r2 = r1 - __uint_as_float(m << 16);
      const unsigned l = bf16_pk2(r2, 0.f);
      Xs[buf][0][tc * XST + pl] = (uint16_t)h;
      Xs[buf][1][tc * XST + pl] = (uint16_t)m;
      Xs[buf][2][tc * XST + pl] = (uint16_t)l;
    }
  };
  // the three parts of the lane's A operand for tile a (kdim row kb + 4 r16 + a, points 8 q .. 8 q + 7)
  u4v sa[4][3];
  auto split_a = [&](const f4* ab) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        unsigned h, m, l;
        bf16_split_pair(ab[2 * i][a], ab[2 * i + 1][a], h, m, l);
        sa[a][0][i] = h;
        sa[a][1][i] = m;
        sa[a][2][i] = l;
      }
  };
  auto mma = [&](int buf) {
    if (!mactive) return;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      u4v xo[3];
#pragma unroll
      for (int P = 0; P < 3; ++P) xo[P] = *reinterpret_cast<const u4v*>(&Xs[buf][P][(16 * b + r16) * XST + 8 * q]);
      // the six partial products with i + j <= 2, smallest first: (l,h) (m,m) (h,l) (m,h) (h,m) (h,h)
#pragma unroll
      for (int a = 0; a < 4; ++a) acc[a][b] = mfma_bf16(sa[a][2], xo[0], acc[a][b]);
#pragma unroll
      for (int a = 0; a < 4; ++a) acc[a][b] = mfma_bf16(sa[a][1], xo[1], acc[a][b]);
#pragma unroll
      for (int a = 0; a < 4; ++a) acc[a][b] = mfma_bf16(sa[a][0], xo[2], acc[a][b]);
#pragma unroll
      for (int a = 0; a < 4; ++a) acc[a][b] = mfma_bf16(sa[a][1], xo[0], acc[a][b]);
#pragma unroll
      for (int a = 0; a < 4; ++a) acc[a][b] = mfma_bf16(sa[a][0], xo[1], acc[a][b]);
#pragma unroll
      for (int a = 0; a < 4; ++a) acc[a][b] = mfma_bf16(sa[a][0], xo[0], acc[a][b]);
    }
  };
  // step s (parity par = s & 1): A(s) is split, its registers then take
  // A(s + 1); the prologue inputs of step s + 2 load; the matrix cores take
  // step s; the prologue of step s + 1 (inputs loaded a step ago) fills the
  // other LDS half
  f4 ab[8];
  auto step = [&](int s, int par) {
    split_a(ab);
    load_a(s + 1, ab);
    pro_load(s + 2, par);
    mma(par);
    pro_apply(s + 1, par ^ 1, par ^ 1);
    __syncthreads();
  };
  if (nsteps > 0) {
    pro_load(0, 0);
    load_a(0, ab);
    pro_load(1, 1);
    pro_apply(0, 0, 0);
    __syncthreads();
    int s = 0;
    for (; s + 1 < nsteps; s += 2) {
      step(s, 0);
      step(s + 1, 1);
    }
    if (s < nsteps) step(s, 0);
  }
  if (mactive) {
    // tile (a, b) element r: kdim row kb + 4 (4 q + r) + a, column 16 b + r16
    float* dst = part + (((int64_t)chunk * ncb + blockIdx.x) * kdim + kb) * 64 + r16;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int b = 0; b < 4; ++b) dst[(4 * (4 * q + r) + a) * 64 + 16 * b] = acc[a][b][r];
  }
  if constexpr (UPD) {
    red[tid] = dacc;
    __syncthreads();
    if (tid < 64) {
      double sum = 0.0;
      for (int k = 0; k < 8; ++k) sum += red[k * 64 + tid];
      dot_part[(int64_t)chunk * ld_dot + c0 + tid] = sum;
    }
  }
}

// Woodbury expansion with split operands: the ROWS_PCG / ROWS_PCG_INIT
// epilogues of k_rows_gemm_f32 for a column block of at most SPLIT_ROWS_NC
// columns.  The three parts of G live in LDS as [part][column][k] (row
// stride kdim + 8), a zero row standing in for the padding columns (160 KB at
// kdim = 512, one workgroup of NW waves per CU).  Each wave is persistent over
// 16-row tiles and walks k in steps of 64: a lane loads 64 contiguous bytes
// of its row (k = 64 kb + 16 q' + 8 t + j for MFMA t, j) two steps ahead and
// splits them when the step starts; the epilogue's residual and D^{-1} rows
// load two steps before the tile ends.  Only the first NB 16-column tiles
// of the block are multiplied (the launch takes NB = ceil(ncols / 16), 3
// rounded up to 4); the others stay zero.
constexpr int SPLIT_ROWS_NC = 52;
inline size_t split_rows_lds(int kdim) { return (size_t)(3 * SPLIT_ROWS_NC + 1) * (kdim + 8) * 2; }

template <int EM, int NW, int NB>
__global__ __launch_bounds__(64 * NW) void k_rows_split(int64_t nrows, int kdim, const float* __restrict__ A,
                                                     int64_t lda, const float* __restrict__ G, int ldg, int ncols,
                                                     F32RowsEpi epi, double* __restrict__ dot_part, int ld_dot) {
  extern __shared__ __attribute__((aligned(16))) uint16_t gsh[];
  constexpr int NT = 64 * NW;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int q = lane >> 4, r16 = lane & 15;
  const int c0 = blockIdx.y * 64;
  const int gst = kdim + 8;
  for (int e = tid; e < kdim * SPLIT_ROWS_NC; e += NT) {
    const int k = e / SPLIT_ROWS_NC, cc = e - k * SPLIT_ROWS_NC;
    const float v = (c0 + cc < ncols) ? G[(int64_t)k * ldg + c0 + cc] : 0.f;
    unsigned h, m, l;
    bf16_split_pair(v, 0.f, h, m, l);
    gsh[(0 * SPLIT_ROWS_NC + cc) * gst + k] = (uint16_t)h;
    gsh[(1 * SPLIT_ROWS_NC + cc) * gst + k] = (uint16_t)m;
    gsh[(2 * SPLIT_ROWS_NC + cc) * gst + k] = (uint16_t)l;
  }
  for (int e = tid; e < gst; e += NT) gsh[3 * SPLIT_ROWS_NC * gst + e] = 0;
  __syncthreads();
  int brow[4][3];
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int P = 0; P < 3; ++P) {
      const int cc = 16 * b + r16;
      brow[b][P] = (cc < SPLIT_ROWS_NC ? (P * SPLIT_ROWS_NC + cc) : 3 * SPLIT_ROWS_NC) * gst + 16 * q;
    }
  const int nkb = kdim / 64;
  const int64_t ntile = (nrows + 15) / 16;
  const int64_t gw = (int64_t)blockIdx.x * NW + w, GW = (int64_t)gridDim.x * NW;
  const int64_t ntw = gw < ntile ? (ntile - gw + GW - 1) / GW : 0;
  const unsigned lane_off = (unsigned)(r16 * lda + 16 * q) * 4u;
  double dsum[4] = {0, 0, 0, 0};
  int64_t lj = 0;
  int lkb = 0;
  auto load_next = [&](f4* ab) {
    const int64_t row0 = (gw + lj * GW) * 16;
    const int64_t nr = lj < ntw ? min((int64_t)16, nrows - row0) : 0;
    const __amdgpu_buffer_rsrc_t rs = rsrc_of(A + (lj < ntw ? row0 * lda : 0), nr * lda * 4);
    const unsigned o = lane_off + (unsigned)lkb * 256u;
#pragma unroll
    for (int i = 0; i < 4; ++i) ab[i] = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(rs, o + 16u * i, 0, 0));
    if (++lkb == nkb) {
      lkb = 0;
      ++lj;
    }
  };
  f4 acc[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) acc[b] = f4{0, 0, 0, 0};
  int64_t cj = 0;
  int ckb = 0;
  // epilogue inputs of the current tile, loaded two steps before its end
  float xin[4][4];
  double di[4];
  auto epi_load = [&]() {
    const int64_t row0 = (gw + cj * GW) * 16;
    const int64_t nr = min((int64_t)16, nrows - row0);
    const __amdgpu_buffer_rsrc_t rr = rsrc_of(epi.R + row0 * epi.ld, nr * epi.ld * 4);
    const __amdgpu_buffer_rsrc_t rd = rsrc_of(epi.Dinv + row0, nr * 8);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      di[r] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rd, (unsigned)(4 * q + r) * 8u, 0, 0));
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int cc = c0 + b * 16 + r16;
        const unsigned o = cc < ncols ? (unsigned)((4 * q + r) * (int)epi.ld + cc) * 4u : (unsigned)BUF_OOR;
        xin[r][b] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rr, o, 0, 0));
      }
    }
  };
  auto epilogue = [&]() {
    const int64_t row0 = (gw + cj * GW) * 16;
    const int64_t nr = min((int64_t)16, nrows - row0);
    const __amdgpu_buffer_rsrc_t ry = rsrc_of(epi.Y ? epi.Y + row0 * epi.ld : (const void*)A, epi.Y ? nr * epi.ld * 4 : 0);
    const __amdgpu_buffer_rsrc_t rh = rsrc_of(EM == ROWS_PCG_INIT ? epi.H + row0 * epi.ld : (const void*)A, EM == ROWS_PCG_INIT ? nr * epi.ld * 4 : 0);
    const __amdgpu_buffer_rsrc_t rp = rsrc_of(EM == ROWS_PCG_INIT ? epi.P + row0 * epi.ld : (const void*)A, EM == ROWS_PCG_INIT ? nr * epi.ld * 4 : 0);
    const __amdgpu_buffer_rsrc_t rq = rsrc_of(EM == ROWS_PCG_INIT ? epi.Q0 + row0 * epi.ld : (const void*)A, EM == ROWS_PCG_INIT ? nr * epi.ld * 4 : 0);
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int cc = c0 + b * 16 + r16;
        const unsigned o = cc < ncols ? (unsigned)((4 * q + r) * (int)epi.ld + cc) * 4u : (unsigned)BUF_OOR;
        const float v = acc[b][r];
        const double rv = (double)xin[r][b];
        const double qv = (rv - (double)v) * di[r];
        dsum[b] += rv * qv;
        if constexpr (EM == ROWS_PCG) {
          __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), ry, o, 0, 0);
        } else {
          const unsigned qb = __builtin_bit_cast(unsigned, (float)qv);
          __builtin_amdgcn_raw_buffer_store_b32(qb, rh, o, 0, 0);
          __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), rp, o, 0, 0);
          __builtin_amdgcn_raw_buffer_store_b32(qb, rq, o, 0, 0);
        }
      }
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[b] = f4{0, 0, 0, 0};
  };
  auto step = [&](f4* cur) {
    // the lane's 16 k (64 kb + 16 q + 8 t + j): parts of the two MFMA operands
    u4v sa[2][3];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int e = 8 * t + 2 * i;
        unsigned h, m, l;
        bf16_split_pair(cur[e >> 2][e & 3], cur[e >> 2][(e & 3) + 1], h, m, l);
        sa[t][0][i] = h;
        sa[t][1][i] = m;
        sa[t][2][i] = l;
      }
    load_next(cur);
    if (ckb == nkb - 2 || (nkb == 1 && ckb == 0)) epi_load();
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      u4v g[NB][3];
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int P = 0; P < 3; ++P) g[b][P] = *reinterpret_cast<const u4v*>(&gsh[brow[b][P] + ckb * 64 + 8 * t]);
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[b] = mfma_bf16(sa[t][2], g[b][0], acc[b]);
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[b] = mfma_bf16(sa[t][1], g[b][1], acc[b]);
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[b] = mfma_bf16(sa[t][0], g[b][2], acc[b]);
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[b] = mfma_bf16(sa[t][1], g[b][0], acc[b]);
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[b] = mfma_bf16(sa[t][0], g[b][1], acc[b]);
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[b] = mfma_bf16(sa[t][0], g[b][0], acc[b]);
    }
    if (++ckb == nkb) {
      epilogue();
      ckb = 0;
      ++cj;
    }
  };
  const int64_t nflat = ntw * nkb;
  f4 b0[4], b1[4];
  load_next(b0);
  load_next(b1);
  int64_t f = 0;
  for (; f + 1 < nflat; f += 2) {
    step(b0);
    step(b1);
  }
  if (f < nflat) step(b0);
  __syncthreads();
  double* red = reinterpret_cast<double*>(gsh);
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    double v = dsum[b];
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    if (q == 0) red[w * 64 + b * 16 + r16] = v;
  }
  __syncthreads();
  if (tid < 64) {
    double sacc = 0.0;
    for (int k = 0; k < NW; ++k) sacc += red[k * 64 + tid];
    dot_part[(int64_t)blockIdx.x * ld_dot + c0 + tid] = sacc;
  }
}

}  // namespace fsa
