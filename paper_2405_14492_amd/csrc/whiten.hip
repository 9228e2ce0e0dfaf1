// Hand-written float64 kernels of the low-rank factor (Section 2.1) and its
// derivative (eq. NEGLLDNEGLLFSA):
//  - the inverse of a lower-triangular mp x mp factor (L_m, L_C, the
//    prediction factor of Algorithm 1), blocked by 64;
//  - products Y = X W^T of a tall point-major block X (n x K) with the
//    transpose of a lower-triangular mp x K matrix W, on the float64 MFMA,
//    with X either read from memory or generated on the fly as the
//    covariance (or its rho-derivative) between the points and the inducing
//    points.  The whitened factor A = L_m^{-1} Sigma_mn is Sigma_nm L_m^{-T}
//    with Sigma_nm never stored; the derivative factor
//    F = L_m^{-1} dSigma_mn - Phi(E) A is one product over [dSigma_nm | A]
//    against [L_m^{-T} ; -Phi(E)^T].
#include "common.hpp"
#include "kernels.hpp"
#include <type_traits>
#include "ops.hpp"

namespace fsa {

// ---------------------------------------------------------------- triangular inverse
// Inverse of each 64 x 64 diagonal block of a lower-triangular L (row-major,
// mp x mp): forward substitution, one thread per column of the block.
__global__ __launch_bounds__(64) void k_trinv_diag(const double* __restrict__ L, int mp, double* __restrict__ Linv) {
  __shared__ double Lb[64][65];
  __shared__ double Xb[64][65];
  const int c = threadIdx.x;
  const int64_t o = (int64_t)blockIdx.x * 64;
  for (int r = 0; r < 64; ++r) Lb[r][c] = L[(o + r) * mp + o + c];
  __syncthreads();
  for (int r = 0; r < 64; ++r) {
    double s = 0.0;
    if (r >= c) {
      s = r == c ? 1.0 : 0.0;
      for (int k = c; k < r; ++k) s -= Lb[r][k] * Xb[k][c];
      s /= Lb[r][r];
    }
    Xb[r][c] = s;
  }
  __syncthreads();
  for (int r = 0; r < 64; ++r) Linv[(o + r) * mp + o + c] = Xb[r][c];
}

// Block column j of L^{-1} below the diagonal block, in order i = j+1..nb-1:
// X_ij = -inv(L_ii) sum_{k=j}^{i-1} L_ik X_kj (X_jj from k_trinv_diag); the
// blocks above the diagonal are cleared.  256 threads, a 4 x 4 register tile
// each.  X_kj is read back after this workgroup wrote it (workgroup scope).
__global__ __launch_bounds__(256) void k_trinv_off(const double* __restrict__ L, int mp, double* __restrict__ Linv) {
  __shared__ double As[64][65];
  __shared__ double Bs[64][65];
  const int j = blockIdx.x, nb = mp / 64, tid = threadIdx.x;
  const int tr = tid / 16, tc = tid % 16;
  for (int i = 0; i < j; ++i)
    for (int e = tid; e < 64 * 64; e += 256)
      Linv[(int64_t)(i * 64 + e / 64) * mp + j * 64 + e % 64] = 0.0;
  for (int i = j + 1; i < nb; ++i) {
    double acc[4][4] = {};
    for (int k = j; k < i; ++k) {
      for (int e = tid; e < 64 * 64; e += 256) {
        const int r = e / 64, q = e % 64;
        As[r][q] = L[(int64_t)(i * 64 + r) * mp + k * 64 + q];
        Bs[r][q] = Linv[(int64_t)(k * 64 + r) * mp + j * 64 + q];
      }
      __syncthreads();
      for (int q = 0; q < 64; ++q) {
        double a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          a[u] = As[tr * 4 + u][q];
          b[u] = Bs[q][tc * 4 + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * b[v];
      }
      __syncthreads();
    }
    // X_ij = -inv(L_ii) T
    for (int e = tid; e < 64 * 64; e += 256) {
      const int r = e / 64, q = e % 64;
      As[r][q] = Linv[(int64_t)(i * 64 + r) * mp + i * 64 + q];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) Bs[tr * 4 + u][tc * 4 + v] = acc[u][v];
    __syncthreads();
    double out[4][4] = {};
    for (int q = 0; q < 64; ++q) {
      double a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = As[tr * 4 + u][q];
        b[u] = Bs[q][tc * 4 + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) out[u][v] -= a[u] * b[v];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) Linv[(int64_t)(i * 64 + tr * 4 + u) * mp + j * 64 + tc * 4 + v] = out[u][v];
    __syncthreads();
  }
}

fsa_status tri_inverse(const double* L, double* Linv, int mp, hipStream_t st) {
  if (mp % 64 || mp <= 0 || mp > 512) {
    set_error("tri_inverse: mp must be a multiple of 64 in [64, 512]");
    return FSA_ERR_INVALID_ARG;
  }
  hipLaunchKernelGGL(k_trinv_diag, dim3(mp / 64), dim3(64), 0, st, L, mp, Linv);
  hipLaunchKernelGGL(k_trinv_off, dim3(mp / 64), dim3(256), 0, st, L, mp, Linv);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

// ---------------------------------------------------------------- Y = X W^T, W lower triangular
// Workgroup: 128 points x 256 output columns, 8 waves.  Wave w takes point
// half ph = w / 4 (64 points, four 16-row MFMA tiles) and column quarter
// cq = w % 4 for w < 4, 3 - w % 4 for w >= 4 (64 columns, four 16-column
// tiles), so the two waves on one SIMD (w and w + 4) together cover
// quarters q and 3 - q: with W lower triangular, the column quarter
// [c0, c0 + 64) needs k < c0 + 64 only, and the pair's work is the same on
// every SIMD.  K runs in chunks of 16 through double-buffered LDS: X as
// Xs[k][point], W^T as Ws[k][column], both read by the MFMA 16x16x4 lanes
// (lane l: A[l % 16][l / 16], B[l / 16][l % 16]).
constexpr int WG_PTS = 128;
constexpr int WG_RT = WG_PTS / 32;  // 16-row MFMA tiles per wave
constexpr int WG_COLS = 256;
constexpr int WG_KC = 16;
constexpr int XS_LD = WG_PTS + 2;
constexpr int WS_LD = WG_COLS + 4;

enum { XSRC_MEM = 0, XSRC_COV = 1, XSRC_DCOV = 2 };

// float32 versions of cov_d and dcov_drho (the float32 derivative factor)
__device__ __forceinline__ float cov_f(float d, const Theta& th) {
  const float s1 = (float)th.s1, rho = (float)th.rho;
  if (th.kind == FSA_COV_EXPONENTIAL) return s1 * expf(-d / rho);
  const float x = 1.7320508f * d / rho;
  return s1 * (1.0f + x) * expf(-x);
}
__device__ __forceinline__ float dcov_drho_f(float d, const Theta& th) {
  const float s1 = (float)th.s1, rho = (float)th.rho;
  if (th.kind == FSA_COV_EXPONENTIAL) return s1 * (d / (rho * rho)) * expf(-d / rho);
  const float x = 1.7320508f * d / rho;
  return s1 * (x * x / rho) * expf(-x);
}

struct WgemmSeg {
  int src;             // XSRC_*
  const double* X;     // XSRC_MEM: point-major n x ldx
  int64_t ldx;
  const double* Wt;    // K x mp row-major (Wt[k][j] = W[j][k]), zero for k > j
  const float* Xf;     // float32 products only: X in float32 (null: X rounded when staged)
};

struct WgemmArgs {
  int64_t n;
  int mp, m, nseg;
  WgemmSeg seg[2];
  const double* xs;    // point coordinates (covariance sources)
  const double* ind;   // inducing coordinates (padded to mp)
  Theta th;
  double* Y;           // n x mp point-major
  float* Yf;           // optional: the same, rounded to float32 (nearest)
};

// SRC0: the source of segment 0 (XSRC_*); segment 1, if TWO, is read from memory.
// T: the arithmetic of the product (double: float64 MFMA with the covariance
// generated in float64; float: float32 MFMA, the covariance generated in
// float32 and W rounded to float32 when staged).
template <int SRC0, bool TWO, typename T>
__global__ __launch_bounds__(512) void k_wgemm(WgemmArgs a) {
  __shared__ T Xs[2][WG_KC][XS_LD];
  __shared__ T Ws[2][WG_KC][WS_LD];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int ph = w >> 2, cq = w < 4 ? (w & 3) : 3 - (w & 3);
  const int64_t p0 = (int64_t)blockIdx.x * WG_PTS;
  const int jb = blockIdx.y * WG_COLS;
  const int ncolw = min(WG_COLS, a.mp - jb);  // 64, 128, 192 or 256
  const int jw = jb + cq * 64;                // this wave's first column
  const bool wave_on = cq * 64 < ncolw;
  // the chunks each segment needs: k < jb + ncolw (W lower triangular)
  const int kneed = min(a.mp, jb + ncolw);
  const int nch_seg = kneed / WG_KC;
  const int nch = nch_seg * (TWO ? 2 : 1);

  // staging of one chunk: X (128 x 16) and W^T (16 x ncolw)
  // X: thread t < 512 takes points t / 8 and t / 8 + 64, k pair 2 (t % 8)
  const int xp = tid >> 3, xk = (tid & 7) * 2;
  double px[2] = {0.0, 0.0}, py[2] = {0.0, 0.0};
  bool xrow_ok[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    xrow_ok[h] = p0 + xp + 64 * h < a.n;
    if (xrow_ok[h] && a.xs) {
      px[h] = a.xs[2 * (p0 + xp + 64 * h)];
      py[h] = a.xs[2 * (p0 + xp + 64 * h) + 1];
    }
  }
  // W: thread t takes k row t / 32 and columns 8 (t % 32) .. + 8
  const int wk = tid >> 5, wc = (tid & 31) * 8;
  T xr[2][2], wr[8];
  auto load = [&](int c) {
    const int s = TWO ? c / nch_seg : 0, k0 = (c % nch_seg) * WG_KC;
    const WgemmSeg& sg = a.seg[s];
    const bool mem = SRC0 == XSRC_MEM || s == 1;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (mem) {
        xr[h][0] = xr[h][1] = T(0);
        if (xrow_ok[h]) {
          const int64_t o = (p0 + xp + 64 * h) * sg.ldx + k0 + xk;
          if (std::is_same<T, float>::value && sg.Xf) {
            const float2 v = *reinterpret_cast<const float2*>(sg.Xf + o);
            xr[h][0] = (T)v.x;
            xr[h][1] = (T)v.y;
          } else {
            const d2 v = *reinterpret_cast<const d2*>(sg.X + o);
            xr[h][0] = (T)v[0];
            xr[h][1] = (T)v[1];
          }
        }
      } else {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int k = k0 + xk + u;
          T v = T(0);
          if (xrow_ok[h] && k < a.m) {
            if constexpr (std::is_same<T, double>::value) {
              const double dx = px[h] - a.ind[2 * k], dy = py[h] - a.ind[2 * k + 1];
              const double d = sqrt(dx * dx + dy * dy);
              v = SRC0 == XSRC_COV ? cov_d(d, a.th) : dcov_drho(d, a.th);
            } else {
              const float dx = (float)(px[h] - a.ind[2 * k]), dy = (float)(py[h] - a.ind[2 * k + 1]);
              const float d = sqrtf(dx * dx + dy * dy);
              v = SRC0 == XSRC_COV ? cov_f(d, a.th) : dcov_drho_f(d, a.th);
            }
          }
          xr[h][u] = v;
        }
      }
    }
    if (wc < ncolw) {
      const d2* src = reinterpret_cast<const d2*>(sg.Wt + (int64_t)(k0 + wk) * a.mp + jb + wc);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const d2 v = src[u];
        wr[2 * u] = (T)v[0];
        wr[2 * u + 1] = (T)v[1];
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      Xs[buf][xk][xp + 64 * h] = xr[h][0];
      Xs[buf][xk + 1][xp + 64 * h] = xr[h][1];
    }
    if (wc < ncolw) {
#pragma unroll
      for (int u = 0; u < 8; ++u) Ws[buf][wk][wc + u] = wr[u];
    }
  };

  typedef typename Mfma<T>::acc acc_t;
  acc_t acc[WG_RT][4];
#pragma unroll
  for (int r = 0; r < WG_RT; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = acc_t{T(0), T(0), T(0), T(0)};

  if (nch > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  for (int c = 0; c < nch; ++c) {
    const int buf = c & 1;
    if (c + 1 < nch) load(c + 1);
    const int k0 = (c % nch_seg) * WG_KC;
    // W lower triangular: columns [jw, jw + 64) need k < jw + 64
    if (wave_on && k0 < jw + 64) {
#pragma unroll
      for (int ks = 0; ks < WG_KC / 4; ++ks) {
        const int kk = ks * 4 + (lane >> 4);
        T av[WG_RT], bv[4];
#pragma unroll
        for (int r = 0; r < WG_RT; ++r) av[r] = Xs[buf][kk][ph * (WG_PTS / 2) + r * 16 + (lane & 15)];
#pragma unroll
        for (int q = 0; q < 4; ++q) bv[q] = Ws[buf][kk][cq * 64 + q * 16 + (lane & 15)];
#pragma unroll
        for (int r = 0; r < WG_RT; ++r)
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[r][q] = Mfma<T>::op(av[r], bv[q], acc[r][q]);
      }
    }
    if (c + 1 < nch) store(buf ^ 1);
    __syncthreads();
  }
  if (!wave_on) return;
  // lane l, register e holds row orow(l / 16, e), column l % 16 of each tile
#pragma unroll
  for (int r = 0; r < WG_RT; ++r)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t p = p0 + ph * (WG_PTS / 2) + r * 16 + Mfma<T>::orow(lane >> 4, e);
      if (p >= a.n) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t o = p * a.mp + jw + q * 16 + (lane & 15);
        if (a.Y) a.Y[o] = (double)acc[r][q][e];
        if (a.Yf) a.Yf[o] = (float)acc[r][q][e];
      }
    }
}

template <typename T>
static fsa_status launch_wgemm(const WgemmArgs& a, hipStream_t st) {
  if (a.n <= 0) return FSA_OK;
  if (a.mp % 64 || a.mp <= 0 || a.mp > 512) {
    set_error("wgemm: mp must be a multiple of 64 in [64, 512]");
    return FSA_ERR_INVALID_ARG;
  }
  for (int s = 0; s < a.nseg; ++s)
    if (a.seg[s].src == XSRC_MEM && ((a.seg[s].ldx & 1) || (reinterpret_cast<uintptr_t>(a.seg[s].X) & 15))) {
      set_error("wgemm: X rows must be 16-byte aligned");
      return FSA_ERR_INVALID_ARG;
    }
  dim3 grid((unsigned)ceil_div(a.n, WG_PTS), (unsigned)ceil_div(a.mp, WG_COLS));
  const int src0 = a.seg[0].src;
  if (a.nseg == 2) {
    if (src0 != XSRC_DCOV || a.seg[1].src != XSRC_MEM) {
      set_error("wgemm: two segments are [dSigma_nm | X]");
      return FSA_ERR_INVALID_ARG;
    }
    hipLaunchKernelGGL((k_wgemm<XSRC_DCOV, true, T>), grid, dim3(512), 0, st, a);
  } else if (src0 == XSRC_COV) {
    hipLaunchKernelGGL((k_wgemm<XSRC_COV, false, T>), grid, dim3(512), 0, st, a);
  } else if (src0 == XSRC_DCOV) {
    hipLaunchKernelGGL((k_wgemm<XSRC_DCOV, false, T>), grid, dim3(512), 0, st, a);
  } else {
    hipLaunchKernelGGL((k_wgemm<XSRC_MEM, false, T>), grid, dim3(512), 0, st, a);
  }
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

// A = Sigma_nm L_m^{-T} (point-major n x mp): LminvT = (L_m^{-1})^T, mp x mp row-major.
fsa_status whiten(const double* xs, int64_t n, const double* ind, int m, int mp, const Theta& th,
                  const double* LminvT, double* A_out, hipStream_t st, float* Af_out) {
  WgemmArgs a{};
  a.n = n;
  a.mp = mp;
  a.m = m;
  a.nseg = 1;
  a.seg[0] = WgemmSeg{XSRC_COV, nullptr, 0, LminvT, nullptr};
  a.xs = xs;
  a.ind = ind;
  a.th = th;
  a.Y = A_out;
  a.Yf = Af_out;
  return launch_wgemm<double>(a, st);
}

// F = dSigma_nm L_m^{-T} - A Phi(E)^T: LminvT as above, PhiT_neg = -Phi(E)^T (mp x mp row-major).
// Af non-null: the product in float32 arithmetic from the float32 copy of A
// (F_out gets the float32 result widened, Ff_out, if non-null, the float32 one).
fsa_status derivative_factor(const double* xs, int64_t n, const double* ind, int m, int mp, const Theta& th,
                             const double* LminvT, const double* A, const double* PhiT_neg, double* F_out,
                             hipStream_t st, const float* Af, float* Ff_out) {
  WgemmArgs a{};
  a.n = n;
  a.mp = mp;
  a.m = m;
  a.nseg = 2;
  a.seg[0] = WgemmSeg{XSRC_DCOV, nullptr, 0, LminvT, nullptr};
  a.seg[1] = WgemmSeg{XSRC_MEM, A, mp, PhiT_neg, Af};
  a.xs = xs;
  a.ind = ind;
  a.th = th;
  a.Y = F_out;
  a.Yf = Ff_out;
  return Af ? launch_wgemm<float>(a, st) : launch_wgemm<double>(a, st);
}

// Y = X W^T for point-major X (n x mp) and lower-triangular W given as WT = W^T.
fsa_status rows_times_lower_t(const double* X, int64_t n, int mp, const double* WT, double* Y, hipStream_t st) {
  WgemmArgs a{};
  a.n = n;
  a.mp = mp;
  a.m = mp;
  a.nseg = 1;
  a.seg[0] = WgemmSeg{XSRC_MEM, X, mp, WT, nullptr};
  a.Y = Y;
  return launch_wgemm<double>(a, st);
}

}  // namespace fsa
