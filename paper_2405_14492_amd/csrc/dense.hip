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

// Right-looking Cholesky in one workgroup.  The matrix (<= 1024^2 doubles)
// lives in global memory and stays in L2; a 64-column panel of the current
// trailing matrix is factored with the pivot column cached in LDS.
__global__ __launch_bounds__(1024) void k_cholesky(double* __restrict__ A, int n, int* __restrict__ info) {
  __shared__ double colk[1024];
  __shared__ int fail;
  if (threadIdx.x == 0) fail = 0;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (threadIdx.x == 0) {
      double a = A[(int64_t)k * n + k];
      if (!(a > 0.0) || !isfinite(a)) {
        fail = k + 1;
        a = 1.0;
      }
      A[(int64_t)k * n + k] = sqrt(a);
    }
    __syncthreads();
    if (fail) break;
    double dkk = A[(int64_t)k * n + k];
    for (int i = k + 1 + threadIdx.x; i < n; i += blockDim.x) {
      double v = A[(int64_t)i * n + k] / dkk;
      A[(int64_t)i * n + k] = v;
      colk[i] = v;
    }
    __syncthreads();
    // trailing update of the lower triangle: A[i][j] -= l_i l_j, k < j <= i
    int rem = n - k - 1;
    int64_t tot = (int64_t)rem * rem;
    for (int64_t e = threadIdx.x; e < tot; e += blockDim.x) {
      int i = k + 1 + (int)(e / rem);
      int j = k + 1 + (int)(e % rem);
      if (j <= i) A[(int64_t)i * n + j] -= colk[i] * colk[j];
    }
    __syncthreads();
  }
  // zero the strict upper triangle
  __syncthreads();
  for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += blockDim.x) {
    int i = (int)(e / n), j = (int)(e % n);
    if (j > i) A[e] = 0.0;
  }
  if (threadIdx.x == 0) *info = fail;
}

fsa_status dense_cholesky(double* A, int mp, int* info_dev, hipStream_t st) {
  hipLaunchKernelGGL(k_cholesky, dim3(1), dim3(1024), 0, st, A, mp, info_dev);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

// Column j of L^{-1}: forward substitution L x = e_j, one thread per column.
__global__ void k_tri_inverse(const double* __restrict__ L, double* __restrict__ X, int n) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  for (int i = 0; i < j; ++i) X[(int64_t)i * n + j] = 0.0;
  X[(int64_t)j * n + j] = 1.0 / L[(int64_t)j * n + j];
  for (int i = j + 1; i < n; ++i) {
    double s = 0.0;
    for (int k = j; k < i; ++k) s += L[(int64_t)i * n + k] * X[(int64_t)k * n + j];
    X[(int64_t)i * n + j] = -s / L[(int64_t)i * n + i];
  }
}

fsa_status dense_tri_inverse(const double* L, double* Linv, int mp, hipStream_t st) {
  hipLaunchKernelGGL(k_tri_inverse, dim3(ceil_div(mp, 64)), dim3(64), 0, st, L, Linv, mp);
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
