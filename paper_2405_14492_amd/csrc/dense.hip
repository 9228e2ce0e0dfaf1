// Small dense float64 kernels on mp x mp matrices (mp = m rounded up to a
// multiple of 64; the padding is the identity): Sigma_m and its Cholesky
// factor (Section 2.1), the FITC capacitance factor (App. F), triangular
// inverses and small products.
#include "common.hpp"
#include "kernels.hpp"

namespace fsa {

__global__ void k_sigma_m(const double* __restrict__ ind, int m, int mp, Theta th, double jitter, int drho,
                          double* __restrict__ out) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)mp * mp) return;
  int k = (int)(e / mp), l = (int)(e % mp);
  double v;
  if (k < m && l < m) {
    double dx = ind[2 * k] - ind[2 * l], dy = ind[2 * k + 1] - ind[2 * l + 1];
    double d = sqrt(dx * dx + dy * dy);
    if (drho) {
      v = dcov_drho(d, th);
    } else {
      v = cov_d(d, th);
      if (k == l) v += jitter * th.s1;
    }
  } else {
    v = (k == l && !drho) ? 1.0 : 0.0;
  }
  out[e] = v;
}

fsa_status dense_sigma_m(const double* ind, int m, int mp, const Theta& th, double jitter, bool drho, double* out,
                         hipStream_t st) {
  int64_t tot = (int64_t)mp * mp;
  hipLaunchKernelGGL(k_sigma_m, dim3(ceil_div(tot, 256)), dim3(256), 0, st, ind, m, mp, th, jitter, (int)drho, out);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

// Blocked right-looking Cholesky in one workgroup (n <= 512, n % 32 == 0).
// Per 32-column block: factor the diagonal block in LDS, solve the panel
// below it (one thread per row, panel kept in LDS), then update the trailing
// lower triangle in 4x4 register tiles.  The matrix stays in L2.
constexpr int CH_NB = 32;
__global__ __launch_bounds__(1024) void k_cholesky(double* __restrict__ A, int n, int* __restrict__ info) {
  __shared__ double Dk[CH_NB][CH_NB + 1];
  __shared__ double P[512 - CH_NB][CH_NB + 1];
  __shared__ int fail;
  const int tid = threadIdx.x;
  if (tid == 0) fail = 0;
  __syncthreads();
  for (int kb = 0; kb < n; kb += CH_NB) {
    // 1. diagonal block
    for (int e = tid; e < CH_NB * CH_NB; e += 1024) {
      int i = e / CH_NB, j = e % CH_NB;
      Dk[i][j] = A[(int64_t)(kb + i) * n + kb + j];
    }
    __syncthreads();
    for (int j = 0; j < CH_NB; ++j) {
      if (tid == 0) {
        double a = Dk[j][j];
        if (!(a > 0.0) || !isfinite(a)) {
          if (!fail) fail = kb + j + 1;
          a = 1.0;
        }
        Dk[j][j] = sqrt(a);
      }
      __syncthreads();
      if (tid > j && tid < CH_NB) Dk[tid][j] /= Dk[j][j];
      __syncthreads();
      {
        int i = tid / CH_NB, k = tid % CH_NB;
        if (i > j && k > j && k <= i) Dk[i][k] -= Dk[i][j] * Dk[k][j];
      }
      __syncthreads();
    }
    if (fail) break;
    for (int e = tid; e < CH_NB * CH_NB; e += 1024) {
      int i = e / CH_NB, j = e % CH_NB;
      A[(int64_t)(kb + i) * n + kb + j] = j <= i ? Dk[i][j] : 0.0;
    }
    // 2. panel rows below: x Dk^T = a  (forward substitution per row)
    const int r0 = kb + CH_NB;
    const int rem = n - r0;
    if (tid < rem) {
      int i = r0 + tid;
      double x[CH_NB];
#pragma unroll
      for (int j = 0; j < CH_NB; ++j) {
        double v = A[(int64_t)i * n + kb + j];
#pragma unroll
        for (int k = 0; k < j; ++k) v -= x[k] * Dk[j][k];
        x[j] = v / Dk[j][j];
      }
#pragma unroll
      for (int j = 0; j < CH_NB; ++j) {
        P[tid][j] = x[j];
        A[(int64_t)i * n + kb + j] = x[j];
      }
    }
    __syncthreads();
    // 3. trailing update of the lower triangle, 4x4 tiles
    const int tb = (rem + 3) / 4;
    const int ntile = tb * (tb + 1) / 2;
    for (int t = tid; t < ntile; t += 1024) {
      // t -> (bi, bj), bj <= bi
      int bi = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
      while (bi * (bi + 1) / 2 > t) --bi;
      while ((bi + 1) * (bi + 2) / 2 <= t) ++bi;
      int bj = t - bi * (bi + 1) / 2;
      double acc[4][4] = {};
#pragma unroll 4
      for (int k = 0; k < CH_NB; ++k) {
        double pi[4], pj[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          int ii = 4 * bi + u, jj = 4 * bj + u;
          pi[u] = ii < rem ? P[ii][k] : 0.0;
          pj[u] = jj < rem ? P[jj][k] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[u][v] += pi[u] * pj[v];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          int ii = 4 * bi + u, jj = 4 * bj + v;
          if (ii < rem && jj <= ii) A[(int64_t)(r0 + ii) * n + r0 + jj] -= acc[u][v];
        }
    }
    __syncthreads();
  }
  __syncthreads();
  // zero the strict upper triangle
  for (int64_t e = tid; e < (int64_t)n * n; e += 1024) {
    int i = (int)(e / n), j = (int)(e % n);
    if (j > i) A[e] = 0.0;
  }
  if (tid == 0) *info = fail;
}

fsa_status dense_cholesky(double* A, int mp, int* info_dev, hipStream_t st) {
  if (mp > 512 || mp % CH_NB) {
    set_error("cholesky: unsupported order %d", mp);
    return FSA_ERR_INVALID_ARG;
  }
  hipLaunchKernelGGL(k_cholesky, dim3(1), dim3(1024), 0, st, A, mp, info_dev);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

// C[i][j] = alpha * sum_k op(A)[i][k] op(B)[k][j]; 16x16 tiles through LDS.
__global__ __launch_bounds__(256) void k_dense_gemm(const double* __restrict__ A, int ta, const double* __restrict__ B,
                                                    int tb, double* __restrict__ C, int n, double alpha) {
  __shared__ double As[16][17], Bs[16][17];
  int ty = threadIdx.x / 16, tx = threadIdx.x % 16;
  int i = blockIdx.y * 16 + ty, j = blockIdx.x * 16 + tx;
  double acc = 0.0;
  for (int k0 = 0; k0 < n; k0 += 16) {
    int ka = k0 + tx, kb = k0 + ty;
    As[ty][tx] = (i < n && ka < n) ? (ta ? A[(int64_t)ka * n + i] : A[(int64_t)i * n + ka]) : 0.0;
    Bs[ty][tx] = (kb < n && j < n) ? (tb ? B[(int64_t)j * n + kb] : B[(int64_t)kb * n + j]) : 0.0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) acc += As[ty][k] * Bs[k][tx];
    __syncthreads();
  }
  if (i < n && j < n) C[(int64_t)i * n + j] = alpha * acc;
}

fsa_status dense_gemm(const double* A, bool ta, const double* B, bool tb, double* C, int mp, double alpha,
                      hipStream_t st) {
  dim3 g(ceil_div(mp, 16), ceil_div(mp, 16));
  hipLaunchKernelGGL(k_dense_gemm, g, dim3(256), 0, st, A, (int)ta, B, (int)tb, C, mp, alpha);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

__global__ __launch_bounds__(1024) void k_logdet_chol(const double* __restrict__ L, int n, double* out) {
  __shared__ double s[1024];
  double a = 0.0;
  for (int k = threadIdx.x; k < n; k += blockDim.x) a += 2.0 * log(L[(int64_t)k * n + k]);
  s[threadIdx.x] = a;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s[0];
}

fsa_status dense_logdet_chol(const double* L, int mp, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_logdet_chol, dim3(1), dim3(1024), 0, st, L, mp, out);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

__global__ void k_to_float(const double* __restrict__ in, float* __restrict__ out, int64_t cnt) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < cnt) out[i] = (float)in[i];
}

__global__ void k_to_bf16(const double* in, uint16_t* out, double* rounded, int64_t cnt) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  // the float32 value rounded to the nearest bfloat16, ties to even (finite inputs)
  const unsigned u = __float_as_uint((float)in[i]);
  const unsigned h = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
  if (out) out[i] = (uint16_t)h;
  if (rounded) rounded[i] = (double)__uint_as_float(h << 16);
}
fsa_status to_bf16(const double* in, uint16_t* out, double* rounded, int64_t cnt, hipStream_t st) {
  if (cnt <= 0) return FSA_OK;
  hipLaunchKernelGGL(k_to_bf16, dim3(ceil_div(cnt, 256)), dim3(256), 0, st, in, out, rounded, cnt);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

__global__ void k_bf16_interleave8(const uint16_t* __restrict__ A, int64_t n, int kdim, uint16_t* __restrict__ out,
                                   int64_t tot) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;  // output element
  if (e >= tot) return;
  const int j = (int)(e & 7);
  const int64_t gk = e >> 3;
  const int k = (int)(gk % kdim);
  const int64_t p = (gk / kdim) * 8 + j;
  out[e] = p < n ? A[p * kdim + k] : (uint16_t)0;
}
fsa_status bf16_interleave8(const uint16_t* A, int64_t n, int kdim, uint16_t* out, hipStream_t st) {
  const int64_t tot = ceil_div(n, 8) * 8 * kdim;
  if (tot <= 0) return FSA_OK;
  hipLaunchKernelGGL(k_bf16_interleave8, dim3(ceil_div(tot, 256)), dim3(256), 0, st, A, n, kdim, out, tot);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

fsa_status to_float(const double* in, float* out, int64_t cnt, hipStream_t st) {
  if (cnt <= 0) return FSA_OK;
  hipLaunchKernelGGL(k_to_float, dim3(ceil_div(cnt, 256)), dim3(256), 0, st, in, out, cnt);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

__global__ void k_add_identity(double* A, int n) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) A[(int64_t)k * n + k] += 1.0;
}

fsa_status add_identity(double* A, int mp, hipStream_t st) {
  hipLaunchKernelGGL(k_add_identity, dim3(ceil_div(mp, 256)), dim3(256), 0, st, A, mp);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

__global__ void k_transpose_scale(const double* __restrict__ A, double* __restrict__ out, int n, double s) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  int i = (int)(e / n), j = (int)(e % n);
  out[(int64_t)j * n + i] = s * A[e];
}

fsa_status transpose_scale(const double* A, double* out, int mp, double scale, hipStream_t st) {
  int64_t tot = (int64_t)mp * mp;
  hipLaunchKernelGGL(k_transpose_scale, dim3(ceil_div(tot, 256)), dim3(256), 0, st, A, out, mp, scale);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

}  // namespace fsa
