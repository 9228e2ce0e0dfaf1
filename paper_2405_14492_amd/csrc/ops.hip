// FSA operations: covariance generation + whitening, residual values,
// capacitance, sparse and low-rank block products, the fused PCG steps of
// Algorithm 2, and the Lanczos-quadrature eigensolve.
#include <algorithm>
#include <type_traits>
#include "gemm.hpp"
#include "ops.hpp"

#include <mutex>

namespace fsa {

constexpr int RT_ROWS = 2;  // row tiles per wave in k_rows_gemm

static int64_t rows_grid(int64_t n) { return ceil_div(n, 64 * RT_ROWS); }
static int64_t f32_rows_grid() { return 256; }

// ================================================================ functors
struct CovRowsOp {
  const double* xs;
  const double* ind;
  int m, mp, mode;
  Theta th;
  __device__ __forceinline__ V4<double> operator()(int64_t i, int k) const {
    V4<double> r;
    const double px = xs[2 * i], py = xs[2 * i + 1];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int kk = k + j;
      bool der = false;
      if (mode == 1) {
        if (kk < mp) der = true;
        else kk -= mp;
      }
      double v = 0.0;
      if (kk < m) {
        double dx = px - ind[2 * kk], dy = py - ind[2 * kk + 1];
        double d = sqrt(dx * dx + dy * dy);
        v = der ? dcov_drho(d, th) : cov_d(d, th);
      }
      r.v[j] = v;
    }
    return r;
  }
};

// Epilogues / prologues are split into load() (all global reads of an
// element) and apply() (arithmetic and stores), so that a thread issues the
// loads of a whole batch before its first store.
template <typename T>
struct StoreEpi {
  T* out;
  int64_t ld;
  int accumulate;
  struct In { T prev; };
  __device__ __forceinline__ In load(int64_t i, int c) const { return In{accumulate ? out[i * ld + c] : T(0)}; }
  __device__ __forceinline__ double apply(int64_t i, int c, T v, const In& x) const {
    out[i * ld + c] = accumulate ? x.prev + v : v;
    return 0.0;
  }
};

namespace {
std::mutex g_tev_mu;
std::vector<hipEvent_t> g_tev;
}  // namespace
hipEvent_t timer_event_get() {
  {
    std::lock_guard<std::mutex> lk(g_tev_mu);
    if (!g_tev.empty()) {
      hipEvent_t e = g_tev.back();
      g_tev.pop_back();
      return e;
    }
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}
void timer_event_put(hipEvent_t e) {
  if (!e) return;
  std::lock_guard<std::mutex> lk(g_tev_mu);
  g_tev.push_back(e);
}

struct ValFn {
  Theta th;
  double gamma;
  int self;
  double* D;
  __device__ __forceinline__ double operator()(int64_t p, int64_t q, double d, double dot) const {
    double v = (cov_d(d, th) - dot) * taper(d, gamma);
    if (self && p == q) {
      v += th.s2;
      D[p] = v;
    }
    return v;
  }
};

struct DValFn {
  Theta th;
  double gamma;
  __device__ __forceinline__ double operator()(int64_t, int64_t, double d, double dot) const {
    return (dcov_drho(d, th) - dot) * taper(d, gamma);
  }
};

// X(p, c) = S[p][c] / D[p]
template <typename T>
struct DivDPro {
  const T* S;
  int64_t ld;
  const double* D;
  struct In { T s; double d; };
  static constexpr bool kUpd = false;
  static constexpr int kSc = 2;
  F32Pro f32() const { return F32Pro{(float*)S, nullptr, nullptr, D, ld}; }
  F64Pro f64() const { return F64Pro{(double*)S, nullptr, nullptr, D, ld}; }
  __device__ __forceinline__ In load(int64_t p, int c) const { return In{S[p * ld + c], D[p]}; }
  __device__ __forceinline__ T apply(int64_t, int, const In& x, double&) const { return (T)((double)x.s / x.d); }
};
// X(p, c) = S[p][c] * Dinv[p]
template <typename T>
struct MulDinvPro {
  const T* S;
  int64_t ld;
  const double* Dinv;
  struct In { T s; double d; };
  static constexpr bool kUpd = false;
  static constexpr int kSc = 1;
  F32Pro f32() const { return F32Pro{(float*)S, nullptr, nullptr, Dinv, ld}; }
  F64Pro f64() const { return F64Pro{(double*)S, nullptr, nullptr, Dinv, ld}; }
  __device__ __forceinline__ In load(int64_t p, int c) const { return In{S[p * ld + c], Dinv[p]}; }
  __device__ __forceinline__ T apply(int64_t, int, const In& x, double&) const { return (T)((double)x.s * x.d); }
};
// X(p, c) = S[p][c]
template <typename T, typename TS>
struct PlainPro {
  const TS* S;
  int64_t ld;
  struct In { TS s; };
  static constexpr bool kUpd = false;
  static constexpr int kSc = 0;
  F32Pro f32() const {
    static_assert(std::is_same<TS, float>::value, "float32 prologue reads float32");
    return F32Pro{(float*)S, nullptr, nullptr, nullptr, ld};
  }
  F64Pro f64() const {
    static_assert(std::is_same<TS, double>::value, "float64 prologue reads float64");
    return F64Pro{(double*)S, nullptr, nullptr, nullptr, ld};
  }
  __device__ __forceinline__ In load(int64_t p, int c) const { return In{S[p * ld + c]}; }
  __device__ __forceinline__ T apply(int64_t, int, const In& x, double&) const { return (T)x.s; }
};

// ================================================================ build-time
// out[i][k] = c(x_i, ind_k) or dc/drho for k < m, 0 on the padding; each
// thread writes four consecutive k of one row.
__global__ __launch_bounds__(256) void k_cov_block(const double* __restrict__ xs, int64_t n,
                                                   const double* __restrict__ ind, int m, int mp, Theta th, int deriv,
                                                   double* __restrict__ out) {
  const int nq = mp / 4;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * nq) return;
  const int64_t i = e / nq;
  const int k0 = (int)(e - i * nq) * 4;
  const double px = xs[2 * i], py = xs[2 * i + 1];
  double v[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int k = k0 + u;
    v[u] = 0.0;
    if (k < m) {
      const double dx = px - ind[2 * k], dy = py - ind[2 * k + 1];
      const double d = sqrt(dx * dx + dy * dy);
      v[u] = deriv ? dcov_drho(d, th) : cov_d(d, th);
    }
  }
  d2* o = reinterpret_cast<d2*>(out + i * mp + k0);
  o[0] = d2{v[0], v[1]};
  o[1] = d2{v[2], v[3]};
}

fsa_status cov_block(const double* xs, int64_t n, const double* ind, int m, int mp, const Theta& th, bool deriv,
                     double* out, hipStream_t st) {
  if (mp % 4) {
    set_error("cov_block: padded m must be a multiple of 4");
    return FSA_ERR_INVALID_ARG;
  }
  const int64_t tot = n * (mp / 4);
  if (tot == 0) return FSA_OK;
  hipLaunchKernelGGL(k_cov_block, dim3(ceil_div(tot, 256)), dim3(256), 0, st, xs, n, ind, m, mp, th, deriv ? 1 : 0,
                     out);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

fsa_status residual_values(const Grid& rg, const Grid& cg, const Csr& csr, const double* Xr, const double* Yc,
                           const double* Fr, const double* Fc, int mp, const Theta& th, double gamma, bool self,
                           bool deriv, double* vals, double* D, hipStream_t st) {
  if (rg.ncell == 0) return FSA_OK;
  GridDesc gd = cg.desc;
  gd.gamma = gamma;
  if (csr.nnz == 0) return FSA_OK;
  dim3 grid(8 * ceil_div(rg.ncell, 8));
  const int sw = 16;  // cell columns per strip of the workgroup walk (measured best of 1..64)
  // one point set with symmetric dot products (X = Y, or [F|A] against
  // [A|F]): each pair of cells once
  const bool sym = self && Xr == Yc && (!deriv || Fr == Fc);
  if (!deriv) {
    RowsOp<double> xo{Xr, mp}, yo{Yc, mp};
    ValFn fn{th, gamma, self ? 1 : 0, D};
    if (sym)
      hipLaunchKernelGGL((k_sddmm_sym<RowsOp<double>, RowsOp<double>, ValFn>), grid, dim3(512), 0, st, rg.cstart.p,
                         rg.ncell, rg.xs.p, gd, csr.row_ptr.p, csr.col.p, csr.key.p, mp, xo, yo, fn, vals, sw);
    else
      hipLaunchKernelGGL((k_sddmm_cell<RowsOp<double>, RowsOp<double>, ValFn>), grid, dim3(512), 0, st, rg.cstart.p,
                         rg.ncell, rg.xs.p, cg.cstart.p, cg.xs.p, gd, csr.row_ptr.p, csr.col.p, csr.key.p, mp, xo, yo,
                         fn, vals, sw);
  } else {
    Rows2Op<double> xo{Fr, Xr, mp, mp}, yo{Yc, Fc, mp, mp};
    DValFn fn{th, gamma};
    if (sym)
      hipLaunchKernelGGL((k_sddmm_sym<Rows2Op<double>, Rows2Op<double>, DValFn>), grid, dim3(512), 0, st,
                         rg.cstart.p, rg.ncell, rg.xs.p, gd, csr.row_ptr.p, csr.col.p, csr.key.p, 2 * mp, xo, yo, fn,
                         vals, sw);
    else
      hipLaunchKernelGGL((k_sddmm_cell<Rows2Op<double>, Rows2Op<double>, DValFn>), grid, dim3(512), 0, st,
                         rg.cstart.p, rg.ncell, rg.xs.p, cg.cstart.p, cg.xs.p, gd, csr.row_ptr.p, csr.col.p,
                         csr.key.p, 2 * mp, xo, yo, fn, vals, sw);
  }
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

// The derivative values of one point set from float32 rows: [Ff | Af]_p .
// [Af | Ff]_q on the float32 MFMA, the rest of DValFn in float64.
fsa_status derivative_values_f32(const Grid& g, const Csr& csr, const float* Af, const float* Ff, int mp,
                                 const Theta& th, double gamma, double* vals, hipStream_t st) {
  if (g.ncell == 0 || csr.nnz == 0) return FSA_OK;
  GridDesc gd = g.desc;
  gd.gamma = gamma;
  dim3 grid(8 * ceil_div(g.ncell, 8));
  const int sw = 16;
  Rows2Op<float> xo{Ff, Af, mp, mp}, yo{Af, Ff, mp, mp};
  DValFn fn{th, gamma};
  hipLaunchKernelGGL((k_sddmm_sym<Rows2Op<float>, Rows2Op<float>, DValFn>), grid, dim3(512), 0, st, g.cstart.p,
                     g.ncell, g.xs.p, gd, csr.row_ptr.p, csr.col.p, csr.key.p, 2 * mp, xo, yo, fn, vals, sw);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

struct ReduceShape {
  int nchunks, ppc, ncb, nmb, zb, threads;
};
// wg_target: about how many workgroups to launch (one per CU by default;
// more where workgroups carry unequal work and the scheduler must balance)
static ReduceShape reduce_shape(int64_t n, int kdim, int ncols, int wg_target = 256) {
  ReduceShape r;
  r.ncb = (int)ceil_div(ncols, 64);
  r.nmb = kdim / 64;
  r.zb = (int)ceil_div(r.nmb, 8);
  r.threads = 64 * (r.nmb < 8 ? r.nmb : 8);
  int64_t target = wg_target / (r.ncb * r.zb);
  if (target < 16) target = 16;
  int64_t nch = ceil_div(n, 256);  // chunks of at least 256 points: enough workgroups at small n too
  if (nch > target) nch = target;
  if (nch < 1) nch = 1;
  r.ppc = (int)round_up(ceil_div(n, nch), 64);
  r.nchunks = (int)ceil_div(n, r.ppc);
  if (r.nchunks < 1) r.nchunks = 1;
  return r;
}

template <typename T>
static fsa_status ensure_part(Scratch& s, const ReduceShape& r) {
  size_t need = (size_t)r.nchunks * r.ncb * r.nmb * 4096 * sizeof(T);
  if (s.part.count < need) FSA_TRY(s.part.alloc(need));
  size_t needd = (size_t)r.nchunks * r.ncb * 64;
  if (s.dot.count < needd) FSA_TRY(s.dot.alloc(needd));
  if (s.dot2.count < needd) FSA_TRY(s.dot2.alloc(needd));
  return FSA_OK;
}

// Reduce GEMM launch: the pipelined kernel for float32, the general one for
// float64.  Prologues that write their input (the PCG residual update) need a
// single workgroup along z, which kdim <= 512 guarantees.
template <typename T, bool DOT, class Pro>
static fsa_status launch_reduce(const ReduceShape& r, int64_t n, int kdim, int ncols, const T* A, const Pro& pro,
                                T* part, double* dot_part, int ld_dot, hipStream_t st, int lower_only = 0,
                                const uint16_t* Abf = nullptr, const uint16_t* Abf8 = nullptr, bool split = false) {
  if (DOT && r.zb != 1) {
    set_error("reduce GEMM with a dot prologue needs kdim <= 512 (got %d)", kdim);
    return FSA_ERR_INVALID_ARG;
  }
  // grid (column blocks, chunks, kdim blocks): the column blocks of one chunk run back to back
  if constexpr (std::is_same<T, double>::value) {
    dim3 grid(r.ncb, (int)round_up(r.nchunks, 8), (kdim + 511) / 512);
    F64Pro fp = pro.f64();
    if constexpr (Pro::kUpd) {
      hipLaunchKernelGGL((k_reduce_gemm_f64<true, Pro::kSc>), grid, dim3(1024), 0, st, n, r.ppc, kdim, ncols, A, fp,
                         part, dot_part, ld_dot, lower_only, r.nchunks);
    } else {
      hipLaunchKernelGGL((k_reduce_gemm_f64<false, Pro::kSc>), grid, dim3(1024), 0, st, n, r.ppc, kdim, ncols, A,
                         fp, part, dot_part, ld_dot, lower_only, r.nchunks);
    }
  } else if constexpr (std::is_same<T, float>::value) {
    if (lower_only) {
      set_error("reduce GEMM: lower-only products are float64");
      return FSA_ERR_INVALID_ARG;
    }
    dim3 grid(r.ncb, r.nchunks, (kdim + 511) / 512);
    F32Pro fp = pro.f32();
    if (Abf8 && r.zb == 1 && r.ppc % 32 == 0) {
      hipLaunchKernelGGL((k_reduce_bf16<Pro::kUpd, Pro::kSc>), dim3(r.ncb, r.nchunks), dim3(512), 0, st, n, r.ppc, kdim,
                         ncols, Abf8, fp, part, dot_part, ld_dot);
    } else if (Abf) {
      hipLaunchKernelGGL((k_reduce_gemm_f32<bf16_t, Pro::kUpd, Pro::kSc>), grid, dim3(512), 0, st, n, r.ppc, kdim,
                         ncols, Abf, fp, part, dot_part, ld_dot);
    } else if (split && r.zb == 1) {
      auto go = [&](auto nb) {
        hipLaunchKernelGGL((k_reduce_split<Pro::kUpd, Pro::kSc, decltype(nb)::value>), dim3(r.ncb, r.nchunks),
                           dim3(512), 0, st, n, r.ppc, kdim, ncols, (const float*)A, fp, part, dot_part, ld_dot);
      };
      // a single column block multiplies only the column tiles that hold a column
      if (r.ncb == 1 && ncols <= 16) go(std::integral_constant<int, 1>{});
      else if (r.ncb == 1 && ncols <= 32) go(std::integral_constant<int, 2>{});
      else go(std::integral_constant<int, 4>{});
    } else {
      hipLaunchKernelGGL((k_reduce_gemm_f32<float, Pro::kUpd, Pro::kSc>), grid, dim3(512), 0, st, n, r.ppc, kdim,
                         ncols, (const float*)A, fp, part, dot_part, ld_dot);
    }
  } else {
    static_assert(std::is_same<T, float>::value || std::is_same<T, double>::value, "float32 or float64 only");
  }
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

template <typename T>
static fsa_status reduce_finish(Scratch& s, const ReduceShape& r, double* W, int ldw, int add_id, hipStream_t st,
                                int lower_only = 0) {
  // row-major partials of the pipelined kernels (all of kdim): a workgroup per 64-column row
  const int64_t rows = (int64_t)r.ncb * r.nmb * 64;
  hipLaunchKernelGGL(k_reduce_parts_rm<T>, dim3(rows), dim3(256), 0, st, (const T*)s.part.p, r.nchunks, r.ncb,
                     r.nmb * 64, W, ldw, add_id, lower_only);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

fsa_status capacitance(const double* A, const double* D, int64_t n, int mp, double* C, Scratch& s, hipStream_t st) {
  // lower blocks only: column block cb works on mp - 64 cb rows, so four
  // workgroups per CU let the scheduler even out the triangle
  ReduceShape r = reduce_shape(n, mp, mp, 1024);
  FSA_TRY(ensure_part<double>(s, r));
  DivDPro<double> pro{A, mp, D};
  FSA_TRY((launch_reduce<double, false>(r, n, mp, mp, A, pro, (double*)s.part.p, nullptr, 0, st, 1)));
  return reduce_finish<double>(s, r, C, mp, 1, st, 1);
}

// ================================================================ block products
template <typename T>
fsa_status lowrank_reduce(const T* A, int64_t n, int kdim, const T* X, int ldx, int ncols, const double* Dinv_src,
                          Scratch& s, double* W, int ldw, hipStream_t st) {
  ReduceShape r = reduce_shape(n, kdim, ncols);
  FSA_TRY(ensure_part<T>(s, r));
  if (Dinv_src) {
    DivDPro<T> pro{X, ldx, Dinv_src};
    FSA_TRY((launch_reduce<T, false>(r, n, kdim, ncols, A, pro, (T*)s.part.p, nullptr, 0, st)));
  } else {
    PlainPro<T, T> pro{X, ldx};
    FSA_TRY((launch_reduce<T, false>(r, n, kdim, ncols, A, pro, (T*)s.part.p, nullptr, 0, st)));
  }
  return reduce_finish<T>(s, r, W, ldw, 0, st);
}

// Float64 rows GEMM over [A | A2] (kseg columns each, A2 optional) in passes
// of at most 256 k; `part` holds the partial sums between passes (it may be
// the epilogue's own output block).
template <int EM, int PM>
static void launch_rows_f64(dim3 grid, size_t smem, hipStream_t st, int64_t n, const double* M, int kseg, int acol0,
                            int kh, const double* G, int ldg, int grow0, int ncols, const F64RowsEpi& epi,
                            double* part, double* dot, int ld_dot) {
  hipLaunchKernelGGL((k_rows_gemm_f64<(EM >= ROWS_PCG), EM, PM>), grid, dim3(1024), smem, st, n, M, (int64_t)kseg,
                     acol0, kh, G, ldg, grow0, ncols, epi, part, dot, ld_dot);
}
template <int EM>
static fsa_status rows_f64(const double* A, const double* A2, int64_t n, int kseg, const double* G, int ldg,
                           int ncols, const F64RowsEpi& epi, double* part, double* dot, int ld_dot, int64_t gx,
                           hipStream_t st) {
  struct Slice { const double* M; int acol0, kh, grow0; };
  Slice sl[16];
  int ns = 0;
  for (int mat = 0; mat < (A2 ? 2 : 1); ++mat)
    for (int k0 = 0; k0 < kseg; k0 += 256) {
      if (ns == 16) {
        set_error("rows GEMM: k too long");
        return FSA_ERR_INVALID_ARG;
      }
      sl[ns++] = Slice{mat ? A2 : A, k0, std::min(256, kseg - k0), mat * kseg + k0};
    }
  if (kseg % 32) {
    set_error("rows GEMM: k must be a multiple of 32");
    return FSA_ERR_INVALID_ARG;
  }
  if (ns > 1 && !part) {
    set_error("rows GEMM: multi-pass product needs a partial-sum block");
    return FSA_ERR_INVALID_ARG;
  }
  dim3 grid(gx, ceil_div(ncols, 64));
  for (int i = 0; i < ns; ++i) {
    const Slice& x = sl[i];
    const size_t smem = (size_t)x.kh * 64 * sizeof(double);
    if (ns == 1) launch_rows_f64<EM, 0>(grid, smem, st, n, x.M, kseg, x.acol0, x.kh, G, ldg, x.grow0, ncols, epi, part, dot, ld_dot);
    else if (i == 0) launch_rows_f64<EM, 1>(grid, smem, st, n, x.M, kseg, x.acol0, x.kh, G, ldg, x.grow0, ncols, epi, part, dot, ld_dot);
    else if (i + 1 < ns) launch_rows_f64<EM, 2>(grid, smem, st, n, x.M, kseg, x.acol0, x.kh, G, ldg, x.grow0, ncols, epi, part, dot, ld_dot);
    else launch_rows_f64<EM, 3>(grid, smem, st, n, x.M, kseg, x.acol0, x.kh, G, ldg, x.grow0, ncols, epi, part, dot, ld_dot);
    FSA_HIP(hipGetLastError());
  }
  return FSA_OK;
}

template <typename T>
fsa_status lowrank_expand(const T* A, const T* A2, int64_t n, int kdim, const T* G, int ldg, int ncols, T* OUT,
                          int ldo, hipStream_t st) {
  StoreEpi<T> epi{OUT, ldo, 0};
  dim3 grid(rows_grid(n), ceil_div(ncols, 64));
  if constexpr (sizeof(T) == 4) {
    if (!A2 && kdim <= 512) {
      F32RowsEpi fe{(float*)OUT, nullptr, nullptr, nullptr, nullptr, nullptr, ldo};
      hipLaunchKernelGGL((k_rows_gemm_f32<float, false, ROWS_STORE>), dim3(f32_rows_grid(), ceil_div(ncols, 64)),
                         dim3(1024), (size_t)kdim * 64 * sizeof(float), st, n, kdim, (const float*)A, (int64_t)kdim,
                         (const float*)G, ldg, ncols, fe, (double*)nullptr, 0);
      FSA_HIP(hipGetLastError());
      return FSA_OK;
    }
  }
  if constexpr (sizeof(T) == 8) {
    F64RowsEpi fe{(double*)OUT, nullptr, nullptr, nullptr, nullptr, nullptr, ldo};
    return rows_f64<ROWS_STORE>((const double*)A, (const double*)A2, n, A2 ? kdim / 2 : kdim, (const double*)G, ldg,
                                ncols, fe, (double*)OUT, nullptr, 0, f32_rows_grid(), st);
  } else {
    if (A2) {
      Rows2Op<T> op{A, A2, kdim / 2, kdim / 2};
      hipLaunchKernelGGL((k_rows_gemm<T, RT_ROWS, false, Rows2Op<T>, StoreEpi<T>>), grid, dim3(256), 0, st, n, kdim,
                         G, ldg, ncols, 0, op, epi, (double*)nullptr, 0);
    } else {
      RowsOp<T> op{A, kdim};
      hipLaunchKernelGGL((k_rows_gemm<T, RT_ROWS, false, RowsOp<T>, StoreEpi<T>>), grid, dim3(256), 0, st, n, kdim,
                         G, ldg, ncols, 0, op, epi, (double*)nullptr, 0);
    }
    FSA_HIP(hipGetLastError());
    return FSA_OK;
  }
}

// ---------------------------------------------------------------- SpMM
static int64_t spmm_grid(int64_t n) {
  int64_t g = ceil_div(n, 4 * 8);
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return g;
}

template <typename T, int EM>
static fsa_status launch_spmm_cell(const Csr& S, const Grid& rg, const Grid& cg, const T* val, const T* X, int ldx,
                                   int ncols, const SpmmEpi<T>& epi, double* dot_part, int ld_dot, hipStream_t st) {
  if (rg.ncell == 0) return FSA_OK;
  if ((ldx & 3) || (reinterpret_cast<uintptr_t>(X) & 15)) {
    set_error("spmm: block rows must be 16-byte aligned (ld multiple of 4)");
    return FSA_ERR_INVALID_ARG;
  }
  // buffer resources span 32-bit byte ranges
  if (S.max_window * ldx * (int64_t)sizeof(T) > INT32_MAX || S.max_group_nnz * (int64_t)sizeof(T) > INT32_MAX) {
    set_error("spmm: a cell neighbourhood of %lld rows or a row group of %lld nonzeros exceeds the 2 GiB window",
              (long long)S.max_window, (long long)S.max_group_nnz);
    return FSA_ERR_INVALID_ARG;
  }
  dim3 grid(8 * ceil_div(rg.ncell, 8), ceil_div(ncols, 64));
  GridDesc gd = cg.desc;
  const int sw = 32;  // cell columns per strip of the workgroup walk (measured best of 4..64)
  hipLaunchKernelGGL((k_spmm_dense<T, EM>), grid, dim3(256), 0, st, rg.cstart.p, rg.ncell, cg.cstart.p, gd,
                     S.row_ptr.p, S.key.p, val, X, ldx, ncols, epi, dot_part, ld_dot, sw);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

// ---------------------------------------------------------------- pre-scattered tiles
// tiles of cell pair p: ceil(rows / 64) groups x ceil(V / 64) neighbourhood chunks
__global__ void k_tile_counts(const int64_t* __restrict__ cs, int64_t npair, GridDesc gd, int* __restrict__ cnt) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= npair) return;
  int64_t rb, re;
  pair_rows(p, gd, cs, rb, re);
  int qb[3], qe[3], off[3];
  const int V = re > rb ? pair_ranges(p, gd, cs, qb, qe, off) : 0;
  cnt[p] = re > rb ? (int)((re - rb + SpmmTile::ROWS - 1) / SpmmTile::ROWS) * ((V + SpmmTile::CH - 1) / SpmmTile::CH)
                   : 0;
}

// one workgroup per cell pair: the pair's tiles are cleared, then, one wave
// per row at a time, every nonzero of the pair's rows goes to its (group,
// chunk) tile at its MFMA-order slot (its column's position in the pair's
// neighbourhood ranges), and the tile's mask gets the bit of the 16 x 16
// block (row tile, step) it lands in (bit rt * 4 + ks; a nonzero value, so
// a block with only zeros stays off).  The masks of the pair's first
// TILE_MASK_LDS tiles gather in LDS, the rest (pairs of very many points) in
// global memory.
constexpr int TILE_MASK_LDS = 512;
__global__ __launch_bounds__(256) void k_tile_fill(const int64_t* __restrict__ cs, int64_t npair, GridDesc gd,
                                                   const int64_t* __restrict__ toff, const int64_t* __restrict__ rp,
                                                   const int* __restrict__ col, const float* __restrict__ val,
                                                   float* __restrict__ tiles, unsigned* __restrict__ mask) {
  __shared__ unsigned msk[TILE_MASK_LDS];
  const int64_t pr = blockIdx.x;
  if (pr >= npair) return;
  int64_t rb, re;
  pair_rows(pr, gd, cs, rb, re);
  if (rb >= re) return;
  int qb[3], qe[3], off[3];
  const int V = pair_ranges(pr, gd, cs, qb, qe, off);
  const int nk = (V + SpmmTile::CH - 1) / SpmmTile::CH;
  const int nt = (int)((re - rb + SpmmTile::ROWS - 1) / SpmmTile::ROWS) * nk;
  float* base = tiles + toff[pr] * SpmmTile::FLOATS;
  unsigned* gmask = mask + toff[pr];
  for (int i = threadIdx.x; i < nt; i += 256) {
    if (i < TILE_MASK_LDS) msk[i] = 0u;
    else gmask[i] = 0u;
  }
  // the pair's tiles start from zero (written here, so the scattered
  // entries below update lines this workgroup has just written)
  f4* base4 = reinterpret_cast<f4*>(base);
  for (int64_t i = threadIdx.x; i < (int64_t)nt * (SpmmTile::FLOATS / 4); i += 256) base4[i] = f4{0.f, 0.f, 0.f, 0.f};
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int64_t p = rb + w; p < re; p += 4) {
    const int g = (int)((p - rb) / SpmmTile::ROWS), r = (int)((p - rb) % SpmmTile::ROWS);
    for (int64_t e = rp[p] + lane; e < rp[p + 1]; e += 64) {
      // the column's range in the pair's neighbourhood (it lies in one: a
      // row's own cell neighbourhood is inside its pair's)
      const int qc = col[e];
      const int rg = (qc >= qb[2] && qc < qe[2]) ? 2 : ((qc >= qb[1] && qc < qe[1]) ? 1 : 0);
      if (qc < qb[rg] || qc >= qe[rg]) continue;
      const int slot = qc - qb[rg] + off[rg];
      const int t = g * nk + slot / SpmmTile::CH, v = slot % SpmmTile::CH;
      const float x = val[e];
      base[(int64_t)t * SpmmTile::FLOATS + SpmmTile::offset(r, v)] = x;
      if (x != 0.f) {
        const unsigned bit = 1u << ((r >> 4) * 4 + (v >> 4));
        if (t < TILE_MASK_LDS) atomicOr(&msk[t], bit);
        else atomicOr(&gmask[t], bit);
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nt && i < TILE_MASK_LDS; i += 256) gmask[i] = msk[i];
}

int64_t spmm_tile_pairs(const Grid& g) { return pair_cols(g.desc.gx) * g.desc.gy; }

fsa_status build_spmm_tiles(const Csr& S, const Grid& g, const float* val, Buf<int64_t>& toff, Buf<float>& tiles,
                            Buf<unsigned>& tmask, hipStream_t st) {
  const int64_t np = g.ncell > 0 ? spmm_tile_pairs(g) : 0;
  FSA_TRY(toff.alloc(np + 1));
  Buf<int> cnt;
  Buf<int64_t> scr;
  FSA_TRY(cnt.alloc(np > 0 ? np : 1));
  hipLaunchKernelGGL(k_tile_counts, dim3(ceil_div(np > 0 ? np : 1, 256)), dim3(256), 0, st, g.cstart.p, np, g.desc,
                     cnt.p);
  FSA_TRY(scan_counts(cnt.p, np, toff.p, scr, st));
  int64_t ntile = 0;
  FSA_HIP(hipMemcpyAsync(&ntile, toff.p + np, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  FSA_HIP(hipStreamSynchronize(st));
  const size_t nf = (size_t)(ntile > 0 ? ntile : 1) * SpmmTile::FLOATS;
  FSA_TRY(tiles.alloc(nf));  // cleared pair by pair by the fill
  FSA_TRY(tmask.alloc(ntile > 0 ? ntile : 1));
  if (np > 0)
    hipLaunchKernelGGL(k_tile_fill, dim3(np), dim3(256), 0, st, g.cstart.p, np, g.desc, toff.p, S.row_ptr.p, S.col.p,
                       val, tiles.p, tmask.p);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

static fsa_status launch_spmm_tiled(const Grid& g, const int64_t* toff, const float* tiles, const unsigned* tmask,
                                    const float* X, int ldx, int ncols, const SpmmEpi<float>& epi, double* dot_part,
                                    int ld_dot, hipStream_t st) {
  if (g.ncell == 0) return FSA_OK;
  if ((ldx & 3) || (reinterpret_cast<uintptr_t>(X) & 15)) {
    set_error("spmm: block rows must be 16-byte aligned (ld multiple of 4)");
    return FSA_ERR_INVALID_ARG;
  }
  const int64_t np = spmm_tile_pairs(g);
  dim3 grid(8 * ceil_div(np, 8), ceil_div(ncols, 64));
  const int sw = 16;  // pair columns per strip of the workgroup walk
  auto go = [&](auto nct) {
    hipLaunchKernelGGL((k_spmm_tiled<SP_PCG, decltype(nct)::value>), grid, dim3(256), 0, st, g.cstart.p, np,
                       g.cstart.p, g.desc, toff, tiles, tmask, X, ldx, ncols, epi, dot_part, ld_dot, sw);
  };
  // a single block multiplies only the column tiles that hold a column
  if (ncols <= 16) go(std::integral_constant<int, 1>{});
  else if (ncols <= 32) go(std::integral_constant<int, 2>{});
  else go(std::integral_constant<int, 4>{});
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

template <typename T>
fsa_status spmm(const Csr& S, const Grid& rg, const Grid& cg, const T* val, const T* X, int ldx, int ncols, T* Y,
                int ldy, bool accumulate, hipStream_t st) {
  SpmmEpi<T> epi{Y, nullptr, nullptr, ldy};
  if (accumulate) return launch_spmm_cell<T, SP_ACC>(S, rg, cg, val, X, ldx, ncols, epi, nullptr, 0, st);
  return launch_spmm_cell<T, SP_STORE>(S, rg, cg, val, X, ldx, ncols, epi, nullptr, 0, st);
}

__global__ __launch_bounds__(256) void k_colsum(const double* __restrict__ part, int nparts, int ldp,
                                                double* __restrict__ out) {
  __shared__ double red[256];
  const int c = blockIdx.x;
  double s = 0.0;
  for (int k = threadIdx.x; k < nparts; k += 256) s += part[(int64_t)k * ldp + c];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = red[0];
}

fsa_status colsum(const double* part, int nparts, int ldp, int ncols, double* out, hipStream_t st) {
  if (ncols <= 0) return FSA_OK;
  hipLaunchKernelGGL(k_colsum, dim3(ncols), dim3(256), 0, st, part, nparts, ldp, out);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

// block-wide fixed-order sum of nparts partials of column c (256 threads)
__device__ __forceinline__ double block_colsum(const double* __restrict__ part, int nparts, int ldp, int c,
                                               double* red) {
  double s = 0.0;
  for (int k = threadIdx.x; k < nparts; k += 256) s += part[(int64_t)k * ldp + c];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------- column dots
template <typename TX, typename TY>
__global__ __launch_bounds__(256) void k_coldot(const TX* __restrict__ X, const TY* __restrict__ Y, int64_t n, int ld,
                                                int ncols, double* __restrict__ part) {
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int c = blockIdx.y * 64 + lane;
  double a = 0.0;
  if (c < ncols) {
    // four rows in flight per wave, summed in a fixed order
    const int64_t st = (int64_t)gridDim.x * 4;
    int64_t p = (int64_t)blockIdx.x * 4 + w;
    double a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (; p + 3 * st < n; p += 4 * st) {
      a += (double)X[p * ld + c] * (double)Y[p * ld + c];
      a1 += (double)X[(p + st) * ld + c] * (double)Y[(p + st) * ld + c];
      a2 += (double)X[(p + 2 * st) * ld + c] * (double)Y[(p + 2 * st) * ld + c];
      a3 += (double)X[(p + 3 * st) * ld + c] * (double)Y[(p + 3 * st) * ld + c];
    }
    for (; p < n; p += st) a += (double)X[p * ld + c] * (double)Y[p * ld + c];
    a = (a + a1) + (a2 + a3);
  }
  red[w][lane] = a;
  __syncthreads();
  if (threadIdx.x < 64)
    part[(int64_t)blockIdx.x * (gridDim.y * 64) + blockIdx.y * 64 + threadIdx.x] =
        red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
}

template <typename TX, typename TY>
fsa_status coldot(const TX* X, const TY* Y, int64_t n, int ld, int ncols, double* out, Scratch& s, hipStream_t st) {
  int ncb = (int)ceil_div(ncols, 64);
  int64_t g = ceil_div(n, 64);
  if (g > 1024) g = 1024;
  if (g < 1) g = 1;
  size_t need = (size_t)g * ncb * 64;
  if (s.dot.count < need) FSA_TRY(s.dot.alloc(need));
  hipLaunchKernelGGL((k_coldot<TX, TY>), dim3(g, ncb), dim3(256), 0, st, X, Y, n, ld, ncols, s.dot.p);
  hipLaunchKernelGGL(k_colsum, dim3(ncols), dim3(256), 0, st, s.dot.p, (int)g, ncb * 64, out);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

// ---------------------------------------------------------------- m-space
// G (kdim x ldg, type T) = M (kdim x kdim) W (kdim x ldw, columns < ncols),
// float64 MFMA 16x16x4: one workgroup per 16 x 16 output tile; its eight
// waves take the 16-wide k blocks round robin (a few steps each, so the
// loads of a wave are few and in flight together) and their partial tiles
// are summed in LDS in a fixed order.  (Sixteen waves were no faster alone
// and waited longer for a free CU beside other work.)  Lane (q, r) of a wave reads four
// consecutive k of row r of M.
constexpr int MSPACE_WAVES = 8;
template <typename T>
__global__ __launch_bounds__(64 * MSPACE_WAVES) void k_mspace(const double* __restrict__ M,
                                                              const double* __restrict__ W, int ldw, int kdim,
                                                              int ncols, T* __restrict__ G, int ldg) {
  __shared__ double red[MSPACE_WAVES][4][64];
  typedef Mfma<double>::acc acc_t;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int q = lane >> 4, r16 = lane & 15;
  const int k0 = blockIdx.y * 16, c0 = blockIdx.x * 16;
  const int cc = c0 + r16;
  const bool cok = cc < ncols;
  const double* mrow = M + (int64_t)(k0 + r16) * kdim;
  acc_t acc = acc_t{0, 0, 0, 0};
  for (int kb = 16 * w; kb < kdim; kb += 16 * MSPACE_WAVES) {
    const V4<double> a = load4(mrow + kb + 4 * q);
    double bv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) bv[j] = cok ? W[(int64_t)(kb + 4 * q + j) * ldw + cc] : 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) acc = Mfma<double>::op(a.v[j], bv[j], acc);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) red[w][r][lane] = acc[r];
  __syncthreads();
  if (w == 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double p[MSPACE_WAVES / 2];
#pragma unroll
      for (int i = 0; i < MSPACE_WAVES / 2; ++i) p[i] = red[2 * i][r][lane] + red[2 * i + 1][r][lane];
#pragma unroll
      for (int h = MSPACE_WAVES / 4; h >= 1; h /= 2)
#pragma unroll
        for (int i = 0; i < h; ++i) p[i] = p[2 * i] + p[2 * i + 1];
      const int k = k0 + Mfma<double>::orow(q, r);
      if (cc < ldg) G[(int64_t)k * ldg + cc] = (T)(cok ? p[0] : 0.0);
    }
  }
}

template <typename T>
fsa_status mspace_apply(const double* M, const double* W, int ldw, int kdim, int ncols, T* G, int ldg,
                        hipStream_t st) {
  if (kdim % 64) {
    set_error("mspace: kdim must be a multiple of 64");
    return FSA_ERR_INVALID_ARG;
  }
  dim3 grid(ceil_div(ldg, 16), kdim / 16);
  hipLaunchKernelGGL(k_mspace<T>, grid, dim3(64 * MSPACE_WAVES), 0, st, M, W, ldw, kdim, ncols, G, ldg);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

// ================================================================ PCG (Algorithm 2)
#define KT_BEGIN(b, cls) int _kt = (b).timer ? (b).timer->start((cls), st) : -1
#define KT_END(b, cls) \
  if ((b).timer) (b).timer->stop((cls), _kt, st)

// Pass-1 prologue of an iteration: r -= alpha v, |r|^2, X = r / D.
template <typename T>
struct PcgPass1Pro {
  T* R;
  const T* V;
  const double* Dinv;
  const double* alpha;
  int64_t ld;
  struct In { T r, v; double di, a; };
  static constexpr bool kUpd = true;
  static constexpr int kSc = 1;
  F32Pro f32() const { return F32Pro{(float*)R, (const float*)V, alpha, Dinv, ld}; }
  F64Pro f64() const { return F64Pro{(double*)R, (const double*)V, alpha, Dinv, ld}; }
  __device__ __forceinline__ In load(int64_t p, int c) const {
    int64_t o = p * ld + c;
    return In{R[o], V[o], Dinv[p], alpha[c]};
  }
  __device__ __forceinline__ T apply(int64_t p, int c, const In& x, double& dot) const {
    T rt = (T)((double)x.r - x.a * (double)x.v);
    R[p * ld + c] = rt;
    double r = (double)rt;
    dot += r * r;
    return (T)(r * x.di);
  }
};

// Pass-2 epilogue: t = (A^T g)_i, q = (r - t)/D; on init h = q, p = t, q0 = q.
template <typename T>
struct PcgPass2Epi {
  T* Tt;
  const T* R;
  const double* Dinv;
  T* H;
  T* P;
  T* Q0;
  int64_t ld;
  int init;
  struct In { T r; double di; };
  __device__ __forceinline__ In load(int64_t i, int c) const { return In{R[i * ld + c], Dinv[i]}; }
  __device__ __forceinline__ double apply(int64_t i, int c, T v, const In& x) const {
    int64_t o = i * ld + c;
    double r = (double)x.r;
    double qv = (r - (double)v) * x.di;
    if (init) {
      H[o] = (T)qv;
      P[o] = v;
      Q0[o] = (T)qv;
    } else {
      Tt[o] = v;
    }
    return r * qv;
  }
};

// Sparse-only variants (no low-rank part): elementwise
template <typename T>
__global__ __launch_bounds__(256) void k_pcg_sparse_update(int64_t n, int ncols, int64_t ld, T* R, const T* V,
                                                           const double* Dinv, const double* alpha, int update,
                                                           int init, T* Hout, T* Q0, double* rr_part,
                                                           double* rq_part, int ld_dot) {
  __shared__ double red1[4][64], red2[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int c = blockIdx.y * 64 + lane;
  double a1 = 0.0, a2 = 0.0;
  if (c < ncols) {
    for (int64_t p = (int64_t)blockIdx.x * 4 + w; p < n; p += (int64_t)gridDim.x * 4) {
      int64_t o = p * ld + c;
      double r;
      if (update) {
        T rt = (T)((double)R[o] - alpha[c] * (double)V[o]);
        R[o] = rt;
        r = (double)rt;
      } else {
        r = (double)R[o];
      }
      double qv = r * Dinv[p];
      if (init) {
        Hout[o] = (T)qv;
        Q0[o] = (T)qv;
      }
      a1 += r * r;
      a2 += r * qv;
    }
  }
  red1[w][lane] = a1;
  red2[w][lane] = a2;
  __syncthreads();
  if (threadIdx.x < 64) {
    int64_t o = (int64_t)blockIdx.x * ld_dot + blockIdx.y * 64 + threadIdx.x;
    rr_part[o] = red1[0][threadIdx.x] + red1[1][threadIdx.x] + red1[2][threadIdx.x] + red1[3][threadIdx.x];
    rq_part[o] = red2[0][threadIdx.x] + red2[1][threadIdx.x] + red2[2][threadIdx.x] + red2[3][threadIdx.x];
  }
}

// u += alpha h (the direction of this iteration), then h = q + beta h with
// q = (r - t)/D (t = 0 when there is no low-rank part) and p = t + beta p.
// A thread takes the E = 16 / sizeof(T) consecutive entries of one 16-byte
// group of the row-major n x ld blocks (ld a multiple of E): group e holds
// entries E e .. E e + E - 1, in row e / (ld / E), so every access is 16
// bytes wide and a row's groups are contiguous.  Entries of padding columns
// (c >= ncols) are written back unchanged, and so are those of a frozen
// column (alpha 0): it keeps its direction, so that if a float64 residual
// check reactivates it, its Krylov sequence continues where it stopped.
template <typename T>
struct Vec16 {
  static constexpr int E = 16 / sizeof(T);
  T v[E];
};
template <typename T>
__device__ __forceinline__ Vec16<T> ld16(const T* p) {
  Vec16<T> q;
  if constexpr (sizeof(T) == 4) {
    const f4 a = *reinterpret_cast<const f4*>(p);
    q.v[0] = a[0]; q.v[1] = a[1]; q.v[2] = a[2]; q.v[3] = a[3];
  } else {
    const d2 a = *reinterpret_cast<const d2*>(p);
    q.v[0] = a[0]; q.v[1] = a[1];
  }
  return q;
}
template <typename T>
__device__ __forceinline__ void st16(T* p, const Vec16<T>& q) {
  if constexpr (sizeof(T) == 4) *reinterpret_cast<f4*>(p) = f4{q.v[0], q.v[1], q.v[2], q.v[3]};
  else *reinterpret_cast<d2*>(p) = d2{q.v[0], q.v[1]};
}
template <typename T, typename TU>
__global__ __launch_bounds__(256) void k_pcg_hupdate(int64_t ngroups, int64_t gpr, int ncols, const T* __restrict__ R,
                                                     const T* __restrict__ Tt, const double* __restrict__ Dinv,
                                                     const double* __restrict__ alpha, const double* __restrict__ beta,
                                                     T* __restrict__ H, T* __restrict__ P, TU* __restrict__ U,
                                                     int has_lr) {
  static_assert(sizeof(T) == sizeof(TU), "U has the block's element size");
  constexpr int E = Vec16<T>::E;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= ngroups) return;
  // row of group e (32-bit division while the group count allows)
  const int64_t p = ngroups <= 0xffffffffll ? (int64_t)((unsigned)e / (unsigned)gpr) : e / gpr;
  const int c0 = E * (int)(e - p * gpr);
  const int64_t o = E * e;
  const double di = Dinv[p];
  Vec16<T> h = ld16(H + o), r = ld16(R + o);
  Vec16<T> t{}, pv{};
  if (has_lr) {
    t = ld16(Tt + o);
    pv = ld16(P + o);
  }
  Vec16<TU> u = ld16(U + o);
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int c = c0 + j;
    const double a = c < ncols ? alpha[c] : 0.0;
    if (a == 0.0) continue;
    const double b = beta[c];
    const double hj = (double)h.v[j];
    const double tj = has_lr ? (double)t.v[j] : 0.0;
    u.v[j] = (TU)((double)u.v[j] + a * hj);
    h.v[j] = (T)(((double)r.v[j] - tj) * di + b * hj);
    if (has_lr) pv.v[j] = (T)(tj + b * (double)pv.v[j]);
  }
  st16(U + o, u);
  st16(H + o, h);
  if (has_lr) st16(P + o, pv);
}

// One workgroup per column c (flags zeroed beforehand): |b|^2, r^T q and the
// column's activity; flags[0] counts the active columns.
__global__ __launch_bounds__(256) void k_pcg_setup(const double* __restrict__ bn2_part, int nb, int ldb,
                                                   const double* __restrict__ rq_part, int nr, int ldr, double* bn2,
                                                   double* rz, double* rz0, double* rr, int* active, int* iters,
                                                   int* flags) {
  __shared__ double red[256];
  const int c = blockIdx.x;
  const double b = block_colsum(bn2_part, nb, ldb, c, red);
  const double r = block_colsum(rq_part, nr, ldr, c, red);
  if (threadIdx.x != 0) return;
  bn2[c] = b;
  rr[c] = b;
  rz[c] = r;
  rz0[c] = r;
  iters[c] = 0;
  const int a = b > 0.0 ? 1 : 0;
  active[c] = a;
  if (a) atomicAdd(&flags[0], 1);
}

// First stage of a fixed-order column sum over many partial rows: workgroup
// g sums rows g, g + G, g + 2G, ... of part (coalesced: 64 columns per row
// block), out[g][c].  The second stage sums the G rows per column.
constexpr int COLSUM_G = 512;
__global__ __launch_bounds__(256) void k_colsum_stage1(const double* __restrict__ part, int nparts, int ldp, int ncols,
                                                       double* __restrict__ out, int ldo) {
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int c0 = 0; c0 < ncols; c0 += 64) {
    const int c = c0 + lane;
    double s = 0.0;
    if (c < ncols)
      for (int k = blockIdx.x + COLSUM_G * w; k < nparts; k += 4 * COLSUM_G) s += part[(int64_t)k * ldp + c];
    red[w][lane] = s;
    __syncthreads();
    if (w == 0 && c < ncols) out[(int64_t)blockIdx.x * ldo + c] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
    __syncthreads();
  }
}

template <typename T>
fsa_status spmm_dot(const Csr& S, const Grid& g, const T* val, const T* X, const T* H, int ld, int ncols,
                    double* out, Scratch& s, hipStream_t st) {
  if (ncols <= 0) return FSA_OK;
  const int ldd = (int)ceil_div(ncols, 64) * 64;
  const int64_t np = std::max<int64_t>(g.ncell, 1);
  if (s.dot.count < (size_t)np * ldd) FSA_TRY(s.dot.alloc((size_t)np * ldd));
  if (s.dot1.count < (size_t)COLSUM_G * ldd) FSA_TRY(s.dot1.alloc((size_t)COLSUM_G * ldd));
  if (g.ncell == 0) FSA_HIP(hipMemsetAsync(s.dot.p, 0, (size_t)ldd * sizeof(double), st));
  SpmmEpi<T> epi{const_cast<T*>(H), H, nullptr, ld};  // Y is not written in this mode
  FSA_TRY((launch_spmm_cell<T, SP_DOT>(S, g, g, val, X, ld, ncols, epi, s.dot.p, ldd, st)));
  hipLaunchKernelGGL(k_colsum_stage1, dim3(COLSUM_G), dim3(256), 0, st, s.dot.p, (int)np, ldd, ncols, s.dot1.p, ldd);
  hipLaunchKernelGGL(k_colsum, dim3(ncols), dim3(256), 0, st, s.dot1.p, COLSUM_G, ldd, out);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}
template fsa_status spmm_dot<double>(const Csr&, const Grid&, const double*, const double*, const double*, int, int,
                                     double*, Scratch&, hipStream_t);

// One workgroup per column: alpha = r^T q / h^T v for active columns.
__global__ __launch_bounds__(256) void k_pcg_alpha(int ncols, const double* __restrict__ hv_part, int np, int ldp,
                                                   const double* __restrict__ rz, const int* __restrict__ active,
                                                   double* __restrict__ alpha, int* flags) {
  __shared__ double red[256];
  const int c = blockIdx.x;
  double hv = block_colsum(hv_part, np, ldp, c, red);
  if (threadIdx.x == 0) {
    if (c == 0) flags[0] = 0;
    double a = 0.0;
    if (active[c]) {
      if (!(hv > 0.0) || !isfinite(hv)) atomicOr(&flags[1], 1);
      else a = rz[c] / hv;
    }
    alpha[c] = a;
  }
}

// One workgroup per column: beta = r'^T q' / r^T q, Lanczos coefficients of
// the iteration, convergence test on |r'|^2 / |b|^2; flags[0] counts the
// columns still active afterwards.
__global__ __launch_bounds__(256) void k_pcg_beta(int ncols, const double* __restrict__ rq_part, int nq, int ldq,
                                                  const double* __restrict__ rr_part, int nr, int ldr, double* rz,
                                                  const double* __restrict__ alpha, double* beta, int* active,
                                                  int* iters, double* ah, double* bh, const double* __restrict__ bn2,
                                                  double* rr_out, double tol2, int fixed, int max_iter, int* flags) {
  __shared__ double red[256];
  const int c = blockIdx.x;
  const bool act = active[c] != 0;
  double rq = 0.0, rr = 0.0;
  if (act) {
    rq = block_colsum(rq_part, nq, ldq, c, red);
    rr = block_colsum(rr_part, nr, ldr, c, red);
  }
  if (threadIdx.x == 0) {
    double b = 0.0;
    int still = 0;
    if (act) {
      b = rq / rz[c];
      int it = iters[c];
      if (it < max_iter) {
        ah[(int64_t)it * ncols + c] = alpha[c];
        bh[(int64_t)it * ncols + c] = b;
      }
      iters[c] = it + 1;
      rz[c] = rq;
      rr_out[c] = rr;
      if (!isfinite(rq)) atomicOr(&flags[1], 1);
      still = (fixed || !(rr < tol2 * bn2[c])) ? 1 : 0;
      active[c] = still;
    }
    beta[c] = b;
    if (still) atomicAdd(&flags[0], 1);
  }
}

template <typename T>
static fsa_status pcg_precond_and_dots(PcgBlock<T>& b, const OpDesc<T>& op, int init, Scratch& s, int& nparts_rq,
                                       hipStream_t st) {
  // m-space: g = Cinv (A D^{-1} r), then q = (r - A^T g)/D
  {
    KT_BEGIN(b, KT_SMALL);
    FSA_TRY(mspace_apply<T>(op.Cinv, s.w.p, b.ldw, op.kdim, b.ncols, b.g, b.ldw, st));
    KT_END(b, KT_SMALL);
  }
  [[maybe_unused]] PcgPass2Epi<T> epi{b.Tt, b.R, op.Dinv, b.H, b.P, b.Q0, b.ld, init};
  int ncb = (int)ceil_div(b.ncols, 64);
  int64_t gx;
  if constexpr (sizeof(T) == 4) {
    gx = f32_rows_grid();
    size_t need = (size_t)gx * ncb * 64;
    if (s.dot.count < need) FSA_TRY(s.dot.alloc(need));
    KT_BEGIN(b, KT_PASS2);
    F32RowsEpi fe{init ? nullptr : (float*)b.Tt, (const float*)b.R, op.Dinv, (float*)b.H, (float*)b.P, (float*)b.Q0,
                  (int64_t)b.ld};
    const size_t smem = (size_t)op.kdim * 64 * sizeof(float);
    dim3 grid2(gx, ncb);
    if (op.Abf8 && b.ncols <= BF16_ROWS_NC && op.kdim <= 512) {
      // bfloat16 MFMA (op.Abf8 set means the bfloat16 kernels are in use)
      const size_t smem16 = bf16_rows_lds(op.kdim);
      if (init)
        hipLaunchKernelGGL((k_rows_bf16<ROWS_PCG_INIT>), grid2, dim3(1024), smem16, st, b.n, op.kdim, op.Abf,
                           (int64_t)op.kdim, (const float*)b.g, b.ldw, b.ncols, fe, s.dot.p, ncb * 64);
      else
        hipLaunchKernelGGL((k_rows_bf16<ROWS_PCG>), grid2, dim3(1024), smem16, st, b.n, op.kdim, op.Abf,
                           (int64_t)op.kdim, (const float*)b.g, b.ldw, b.ncols, fe, s.dot.p, ncb * 64);
    } else if (op.split && b.ncols <= SPLIT_ROWS_NC && op.kdim <= 512) {
      // float32 operands split in three bfloat16 parts, one 8-wave workgroup per CU
      const size_t smem16 = split_rows_lds(op.kdim);
      auto go = [&](auto em, auto nb) {
        hipLaunchKernelGGL((k_rows_split<decltype(em)::value, 8, decltype(nb)::value>), grid2, dim3(512), smem16, st,
                           b.n, op.kdim, (const float*)op.A, (int64_t)op.kdim, (const float*)b.g, b.ldw, b.ncols, fe,
                           s.dot.p, ncb * 64);
      };
      // the column tiles that hold a column
      auto go_nb = [&](auto em) {
        if (b.ncols <= 16) go(em, std::integral_constant<int, 1>{});
        else if (b.ncols <= 32) go(em, std::integral_constant<int, 2>{});
        else go(em, std::integral_constant<int, 4>{});
      };
      if (init) go_nb(std::integral_constant<int, ROWS_PCG_INIT>{});
      else go_nb(std::integral_constant<int, ROWS_PCG>{});
    } else if (op.Abf) {
      if (init)
        hipLaunchKernelGGL((k_rows_gemm_f32<bf16_t, true, ROWS_PCG_INIT>), grid2, dim3(1024), smem, st, b.n, op.kdim,
                           op.Abf, (int64_t)op.kdim, (const float*)b.g, b.ldw, b.ncols, fe, s.dot.p, ncb * 64);
      else
        hipLaunchKernelGGL((k_rows_gemm_f32<bf16_t, true, ROWS_PCG>), grid2, dim3(1024), smem, st, b.n, op.kdim,
                           op.Abf, (int64_t)op.kdim, (const float*)b.g, b.ldw, b.ncols, fe, s.dot.p, ncb * 64);
    } else {
      if (init)
        hipLaunchKernelGGL((k_rows_gemm_f32<float, true, ROWS_PCG_INIT>), grid2, dim3(1024), smem, st, b.n, op.kdim,
                           (const float*)op.A, (int64_t)op.kdim, (const float*)b.g, b.ldw, b.ncols, fe, s.dot.p,
                           ncb * 64);
      else
        hipLaunchKernelGGL((k_rows_gemm_f32<float, true, ROWS_PCG>), grid2, dim3(1024), smem, st, b.n, op.kdim,
                           (const float*)op.A, (int64_t)op.kdim, (const float*)b.g, b.ldw, b.ncols, fe, s.dot.p,
                           ncb * 64);
    }
    KT_END(b, KT_PASS2);
  } else {
    gx = f32_rows_grid();
    size_t need = (size_t)gx * ncb * 64;
    if (s.dot.count < need) FSA_TRY(s.dot.alloc(need));
    F64RowsEpi fe{init ? nullptr : (double*)b.Tt, (const double*)b.R, op.Dinv, (double*)b.H, (double*)b.P,
                  (double*)b.Q0, (int64_t)b.ld};
    double* part = init ? (double*)b.P : (double*)b.Tt;  // partial sums between the k passes
    KT_BEGIN(b, KT_PASS2);
    if (init)
      FSA_TRY(rows_f64<ROWS_PCG_INIT>((const double*)op.A, nullptr, b.n, op.kdim, (const double*)b.g, b.ldw, b.ncols,
                                      fe, part, s.dot.p, ncb * 64, gx, st));
    else
      FSA_TRY(rows_f64<ROWS_PCG>((const double*)op.A, nullptr, b.n, op.kdim, (const double*)b.g, b.ldw, b.ncols, fe,
                                 part, s.dot.p, ncb * 64, gx, st));
    KT_END(b, KT_PASS2);
  }
  FSA_HIP(hipGetLastError());
  nparts_rq = (int)gx;
  return FSA_OK;
}

template <typename T>
fsa_status pcg_init(PcgBlock<T>& b, const OpDesc<T>& op, const double* B, double tol, Scratch& s, hipStream_t st) {
  (void)tol;
  if (b.ncols <= 0) {
    set_error("PCG needs at least one right-hand side");
    return FSA_ERR_INVALID_ARG;
  }
  FSA_TRY((copy_block<double, T>(B, b.ld, b.R, b.ld, b.n, b.ncols, st)));
  FSA_HIP(hipMemsetAsync(b.U, 0, (size_t)b.n * b.ld * sizeof(double), st));
  if (sizeof(T) == 4 && b.U32) FSA_HIP(hipMemsetAsync(b.U32, 0, (size_t)b.n * b.ld * sizeof(float), st));
  int ncb = (int)ceil_div(b.ncols, 64);
  int nparts_rq = 0, nparts_rr = 0;
  if (op.kdim > 0) {
    ReduceShape r = reduce_shape(b.n, op.kdim, b.ncols);
    FSA_TRY(ensure_part<T>(s, r));
    MulDinvPro<T> pro{b.R, b.ld, op.Dinv};
    FSA_TRY((launch_reduce<T, false>(r, b.n, op.kdim, b.ncols, op.A, pro, (T*)s.part.p, nullptr, 0, st, 0, op.Abf,
                                     op.Abf8, op.split)));
    FSA_TRY(reduce_finish<T>(s, r, s.w.p, b.ldw, 0, st));
    FSA_TRY(pcg_precond_and_dots<T>(b, op, 1, s, nparts_rq, st));
    // |b|^2 partials
    int64_t g = ceil_div(b.n, 64);
    if (g > 1024) g = 1024;
    size_t need = (size_t)g * ncb * 64;
    if (s.dot2.count < need) FSA_TRY(s.dot2.alloc(need));
    hipLaunchKernelGGL((k_coldot<double, double>), dim3(g, ncb), dim3(256), 0, st, B, B, b.n, b.ld, b.ncols, s.dot2.p);
    nparts_rr = (int)g;
    FSA_HIP(hipGetLastError());
    FSA_HIP(hipMemsetAsync(b.flags, 0, 2 * sizeof(int), st));
    hipLaunchKernelGGL(k_pcg_setup, dim3(b.ncols), dim3(256), 0, st, s.dot2.p, nparts_rr, ncb * 64, s.dot.p,
                       nparts_rq, ncb * 64, b.bn2, b.rz, b.rz0, b.rr, b.active, b.iters, b.flags);
  } else {
    int64_t g = spmm_grid(b.n);
    size_t need = (size_t)g * ncb * 64;
    if (s.dot.count < need) FSA_TRY(s.dot.alloc(need));
    if (s.dot2.count < need) FSA_TRY(s.dot2.alloc(need));
    hipLaunchKernelGGL((k_pcg_sparse_update<T>), dim3(g, ncb), dim3(256), 0, st, b.n, b.ncols, (int64_t)b.ld, b.R,
                       (const T*)b.V, op.Dinv, b.alpha, 0, 1, b.H, b.Q0, s.dot2.p, s.dot.p, ncb * 64);
    FSA_HIP(hipGetLastError());
    FSA_HIP(hipMemsetAsync(b.flags, 0, 2 * sizeof(int), st));
    hipLaunchKernelGGL(k_pcg_setup, dim3(b.ncols), dim3(256), 0, st, s.dot2.p, (int)g, ncb * 64, s.dot.p, (int)g,
                       ncb * 64, b.bn2, b.rz, b.rz0, b.rr, b.active, b.iters, b.flags);
  }
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

template <typename T>
fsa_status pcg_iter(PcgBlock<T>& b, const OpDesc<T>& op, double tol, int fixed, Scratch& s, hipStream_t st) {
  const int ncb = (int)ceil_div(b.ncols, 64);
  const int ldd = ncb * 64;
  const bool lr = op.kdim > 0;
  // 1. V = S H + P, h^T v
  {
    SpmmEpi<T> epi{b.V, b.H, lr ? b.P : nullptr, b.ld};
    // partial dot rows: one per cell, or one per cell pair of the tiled product
    const bool tiled = sizeof(T) == 4 && op.tiles;
    int64_t g = tiled ? spmm_tile_pairs(*op.grid) : op.grid->ncell;
    size_t need = (size_t)g * ldd;
    if (s.dot.count < need) FSA_TRY(s.dot.alloc(need));
    {
      KT_BEGIN(b, KT_SPMM);
      if constexpr (sizeof(T) == 4) {
        if (tiled)
          FSA_TRY(launch_spmm_tiled(*op.grid, op.tile_off, op.tiles, op.tile_mask, (const float*)b.H, b.ld, b.ncols,
                                    reinterpret_cast<const SpmmEpi<float>&>(epi), s.dot.p, ldd, st));
        else
          FSA_TRY((launch_spmm_cell<T, SP_PCG>(*op.S, *op.grid, *op.grid, op.val, b.H, b.ld, b.ncols, epi, s.dot.p,
                                               ldd, st)));
      } else {
        FSA_TRY((launch_spmm_cell<T, SP_PCG>(*op.S, *op.grid, *op.grid, op.val, b.H, b.ld, b.ncols, epi, s.dot.p,
                                             ldd, st)));
      }
      KT_END(b, KT_SPMM);
    }
    KT_BEGIN(b, KT_SMALL);
    if (s.dot1.count < (size_t)COLSUM_G * ldd) FSA_TRY(s.dot1.alloc((size_t)COLSUM_G * ldd));
    hipLaunchKernelGGL(k_colsum_stage1, dim3(COLSUM_G), dim3(256), 0, st, s.dot.p, (int)g, ldd, b.ncols, s.dot1.p,
                       ldd);
    hipLaunchKernelGGL(k_pcg_alpha, dim3(b.ncols), dim3(256), 0, st, b.ncols, s.dot1.p, COLSUM_G, ldd, b.rz,
                       b.active, b.alpha, b.flags);
    KT_END(b, KT_SMALL);
    FSA_HIP(hipGetLastError());
  }
  int nparts_rq = 0, nparts_rr = 0;
  if (lr) {
    // 2. u += alpha h, r -= alpha v, |r|^2, W = A D^{-1} r
    ReduceShape r = reduce_shape(b.n, op.kdim, b.ncols);
    FSA_TRY(ensure_part<T>(s, r));
    PcgPass1Pro<T> pro{b.R, b.V, op.Dinv, b.alpha, b.ld};
    {
      KT_BEGIN(b, KT_PASS1);
      FSA_TRY((launch_reduce<T, true>(r, b.n, op.kdim, b.ncols, op.A, pro, (T*)s.part.p, s.dot2.p, ldd, st, 0,
                                      op.Abf, op.Abf8, op.split)));
      KT_END(b, KT_PASS1);
    }
    nparts_rr = r.nchunks;
    {
      KT_BEGIN(b, KT_SMALL);
      FSA_TRY(reduce_finish<T>(s, r, s.w.p, b.ldw, 0, st));
      KT_END(b, KT_SMALL);
    }
    // 3. g = Cinv W; t = A^T g; q = (r - t)/D; r^T q
    FSA_TRY(pcg_precond_and_dots<T>(b, op, 0, s, nparts_rq, st));
  } else {
    int64_t g = spmm_grid(b.n);
    hipLaunchKernelGGL((k_pcg_sparse_update<T>), dim3(g, ncb), dim3(256), 0, st, b.n, b.ncols, (int64_t)b.ld, b.R,
                       (const T*)b.V, op.Dinv, b.alpha, 1, 0, b.H, b.Q0, s.dot2.p, s.dot.p, ldd);
    FSA_HIP(hipGetLastError());
    nparts_rq = nparts_rr = (int)g;
  }
  // 4. beta, Lanczos entries, convergence
  {
    KT_BEGIN(b, KT_SMALL);
    hipLaunchKernelGGL(k_pcg_beta, dim3(b.ncols), dim3(256), 0, st, b.ncols, s.dot.p, nparts_rq, ldd, s.dot2.p, nparts_rr,
                       ldd, b.rz, b.alpha, b.beta, b.active, b.iters, b.alpha_hist, b.beta_hist, b.bn2, b.rr,
                       tol * tol, fixed, b.max_iter, b.flags);
    KT_END(b, KT_SMALL);
  }
  // 5. h = q + beta h, p = t + beta p
  constexpr int E = Vec16<T>::E;
  const uintptr_t al = reinterpret_cast<uintptr_t>(b.R) | reinterpret_cast<uintptr_t>(b.H) |
                       reinterpret_cast<uintptr_t>(b.P) | reinterpret_cast<uintptr_t>(b.Tt) |
                       reinterpret_cast<uintptr_t>(b.U) | reinterpret_cast<uintptr_t>(b.U32);
  if ((b.ld % E) || (al & 15)) {
    set_error("PCG blocks must be 16-byte aligned with a stride that is a multiple of %d (ld %d)", E, b.ld);
    return FSA_ERR_INVALID_ARG;
  }
  const int64_t gpr = b.ld / E, ngroups = b.n * gpr;
  KT_BEGIN(b, KT_UPDATE);
  if constexpr (sizeof(T) == 4) {
    if (!b.U32) {
      set_error("float32 PCG block without its float32 solution increment");
      return FSA_ERR_INVALID_ARG;
    }
    hipLaunchKernelGGL((k_pcg_hupdate<T, float>), dim3(ceil_div(ngroups, 256)), dim3(256), 0, st, ngroups, gpr,
                       b.ncols, (const T*)b.R, (const T*)b.Tt, op.Dinv, b.alpha, b.beta, b.H, b.P, b.U32,
                       lr ? 1 : 0);
  } else {
    hipLaunchKernelGGL((k_pcg_hupdate<T, double>), dim3(ceil_div(ngroups, 256)), dim3(256), 0, st, ngroups, gpr,
                       b.ncols, (const T*)b.R, (const T*)b.Tt, op.Dinv, b.alpha, b.beta, b.H, b.P, b.U, lr ? 1 : 0);
  }
  KT_END(b, KT_UPDATE);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

// R = B - (S U + A^T (A U)) in float64, then rounded to float.
__global__ void k_residual_f32(int64_t n, int ncols, int64_t ld, const double* __restrict__ B, const double* __restrict__ SU,
                               const double* __restrict__ LU, float* __restrict__ R) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t p = e / ncols;
  int c = (int)(e % ncols);
  if (p >= n) return;
  int64_t o = p * ld + c;
  R[o] = (float)(B[o] - SU[o] - LU[o]);
}

__global__ void k_fold_u(int64_t n, int ncols, int64_t ld, double* __restrict__ U, float* __restrict__ U32) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t p = e / ncols;
  int c = (int)(e % ncols);
  if (p >= n) return;
  int64_t o = p * ld + c;
  U[o] += (double)U32[o];
  U32[o] = 0.f;
}

// After a float64 residual replacement: rr_true[c] = |r_c|^2 of the replaced
// residual; a column at or above the tolerance is active again (its
// direction was kept while it was frozen), flags[0] = the active count.
__global__ __launch_bounds__(256) void k_pcg_reactivate(int ncols, const double* __restrict__ rr_true,
                                                        const double* __restrict__ bn2, double tol2, double* rr,
                                                        int* active, int* flags) {
  __shared__ int red[256];
  int cnt = 0;
  for (int c = threadIdx.x; c < ncols; c += 256) {
    const double v = rr_true[c];
    rr[c] = v;
    const int a = (bn2[c] > 0.0 && !(v < tol2 * bn2[c])) ? 1 : 0;
    active[c] = a;
    cnt += a;
  }
  red[threadIdx.x] = cnt;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) flags[0] = red[0];
}

fsa_status pcg_recheck_true_residual(PcgBlock<float>& b, double tol, Scratch& s, hipStream_t st) {
  Buf<double> rrt;
  FSA_TRY(rrt.alloc(b.ncols));
  FSA_TRY((coldot<float, float>(b.R, b.R, b.n, b.ld, b.ncols, rrt.p, s, st)));
  hipLaunchKernelGGL(k_pcg_reactivate, dim3(1), dim3(256), 0, st, b.ncols, rrt.p, b.bn2, tol * tol, b.rr, b.active,
                     b.flags);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

fsa_status pcg_fold_u(PcgBlock<float>& b, hipStream_t st) {
  if (!b.U32) return FSA_OK;
  int64_t tot = b.n * b.ncols;
  hipLaunchKernelGGL(k_fold_u, dim3(ceil_div(tot, 256)), dim3(256), 0, st, b.n, b.ncols, (int64_t)b.ld, b.U, b.U32);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

fsa_status pcg_replace_residual_f32(PcgBlock<float>& b, const OpDesc<double>& op64, const OpDesc<float>& op32,
                                    const double* B, Scratch& s, hipStream_t st) {
  (void)op32;
  FSA_TRY(pcg_fold_u(b, st));
  Buf<double> SU, LU;
  FSA_TRY(SU.alloc((size_t)b.n * b.ld));
  FSA_TRY(LU.alloc((size_t)b.n * b.ld));
  FSA_TRY(spmm<double>(*op64.S, *op64.grid, *op64.grid, op64.val, b.U, b.ld, b.ncols, SU.p, b.ld, false, st));
  if (op64.kdim > 0) {
    FSA_TRY(lowrank_reduce<double>(op64.A, b.n, op64.kdim, b.U, b.ld, b.ncols, nullptr, s, s.w.p, b.ldw, st));
    FSA_TRY(lowrank_expand<double>(op64.A, nullptr, b.n, op64.kdim, s.w.p, b.ldw, b.ncols, LU.p, b.ld, st));
  } else {
    FSA_HIP(hipMemsetAsync(LU.p, 0, (size_t)b.n * b.ld * sizeof(double), st));
  }
  int64_t tot = b.n * b.ncols;
  hipLaunchKernelGGL(k_residual_f32, dim3(ceil_div(tot, 256)), dim3(256), 0, st, b.n, b.ncols, (int64_t)b.ld, B, SU.p,
                     LU.p, b.R);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

// ================================================================ SLQ
// e_1^T log(T) e_1 of the Lanczos tridiagonal built from the CG
// coefficients: T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1}, T_{j,j+1} =
// sqrt(beta_j)/alpha_j (Algorithm 2).  Eigenvalues by the implicit QL
// iteration with Wilkinson-type shifts (Bowdler, Martin, Reinsch &
// Wilkinson 1968), tracking only the first row of the eigenvector matrix.
// The rotation lengths use sqrt(f^2 + g^2) directly: the Lanczos entries
// are of the order of the preconditioned spectrum, far from overflow.
__global__ __launch_bounds__(64) void k_slq(const double* __restrict__ ah, const double* __restrict__ bh,
                                            const int* __restrict__ iters, int ncols, int c_first,
                                            const double* __restrict__ weight, double* __restrict__ out,
                                            int max_iter) {
  extern __shared__ double slq_smem[];
  const int c = c_first + blockIdx.x;
  int k = iters[c];
  if (k > max_iter) k = max_iter;
  double* d = slq_smem;
  double* e = d + max_iter;
  double* z = e + max_iter;
  for (int j = threadIdx.x; j < k; j += 64) {
    double a = ah[(int64_t)j * ncols + c];
    d[j] = 1.0 / a + (j > 0 ? bh[(int64_t)(j - 1) * ncols + c] / ah[(int64_t)(j - 1) * ncols + c] : 0.0);
    e[j] = (j < k - 1) ? sqrt(bh[(int64_t)j * ncols + c]) / a : 0.0;
    z[j] = (j == 0) ? 1.0 : 0.0;
  }
  __syncthreads();
  __shared__ int ok_s;
  if (threadIdx.x == 0) {
    bool ok = k > 0;
    for (int l = 0; l < k && ok; ++l) {
      int iter = 0;
      int mm;
      do {
        for (mm = l; mm < k - 1; ++mm) {
          double dd = fabs(d[mm]) + fabs(d[mm + 1]);
          if (fabs(e[mm]) <= 2.220446049250313e-16 * dd) break;
        }
        if (mm != l) {
          if (iter++ == 200) { ok = false; break; }
          double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
          double r = sqrt(g * g + 1.0);
          g = d[mm] - d[l] + e[l] / (g + copysign(r, g));
          double s = 1.0, cc = 1.0, p = 0.0;
          bool deflated = false;
          for (int i = mm - 1; i >= l; --i) {
            double f = s * e[i], bb = cc * e[i];
            r = sqrt(f * f + g * g);
            e[i + 1] = r;
            if (r == 0.0) {
              d[i + 1] -= p;
              e[mm] = 0.0;
              deflated = true;
              break;
            }
            const double rinv = 1.0 / r;
            s = f * rinv;
            cc = g * rinv;
            g = d[i + 1] - p;
            r = (d[i] - g) * s + 2.0 * cc * bb;
            p = s * r;
            d[i + 1] = g + p;
            g = cc * r - bb;
            double zf = z[i + 1];
            z[i + 1] = s * z[i] + cc * zf;
            z[i] = cc * z[i] - s * zf;
          }
          if (deflated) continue;
          d[l] -= p;
          e[l] = g;
          e[mm] = 0.0;
        }
      } while (mm != l);
    }
    ok_s = ok ? 1 : 0;
  }
  __syncthreads();
  double v = 0.0;
  int bad = 0;
  if (ok_s) {
    for (int j = threadIdx.x; j < k; j += 64) {
      if (!(d[j] > 0.0)) bad = 1;
      else v += z[j] * z[j] * log(d[j]);
    }
  }
  v = wave_sum(v);
  bad = __any(bad);
  if (threadIdx.x == 0) out[c] = (ok_s && !bad) ? weight[c] * v : NAN;
}

fsa_status slq_terms(const double* alpha_hist, const double* beta_hist, const int* iters, int ncols, int c_first,
                     const double* weight, double* out, double* scratch, int max_iter, hipStream_t st) {
  int cnt = ncols - c_first;
  if (cnt <= 0) return FSA_OK;
  (void)scratch;
  size_t smem = (size_t)3 * max_iter * sizeof(double);
  if (smem > 150 * 1024) {
    set_error("slq: max_iter too large for the on-chip eigensolve");
    return FSA_ERR_INVALID_ARG;
  }
  hipLaunchKernelGGL(k_slq, dim3(cnt), dim3(64), smem, st, alpha_hist, beta_hist, iters, ncols, c_first, weight, out,
                     max_iter);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

// ================================================================ probes
__global__ void k_probe_e(int m, int mp, int nprobe, uint64_t seed, double* E, int ldb) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)mp * ldb) return;
  int k = (int)(e / ldb), c = (int)(e % ldb);
  double v = 0.0;
  if (k < m && c >= 1 && c <= nprobe) v = rademacher(seed, STREAM_E, (uint64_t)(c - 1), (uint64_t)k);
  E[e] = v;
}

// B[p][0] = y[p]; B[p][c] += sqrt(D[p]) rho_{c-1}(perm[p]) for 1 <= c < ncols
__global__ void k_probe_finish(double* __restrict__ B, int64_t ldb, const double* __restrict__ y,
                               const double* __restrict__ D, const int* __restrict__ perm, uint64_t seed, int64_t n,
                               int ncols) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t p = e / ncols;
  const int c = (int)(e % ncols);
  if (p >= n) return;
  if (c == 0) B[p * ldb] = y[p];
  else B[p * ldb + c] += sqrt(D[p]) * rademacher(seed, STREAM_RHO, (uint64_t)(c - 1), (uint64_t)perm[p]);
}

fsa_status make_probes(const double* A, int64_t n, int m, int mp, const double* D, const double* y, const int* perm,
                       uint64_t seed, int nprobe, double* B, int ldb, double* Emat, hipStream_t st) {
  int ncols = nprobe + 1;
  int ldE = (int)round_up(ncols, 64);
  hipLaunchKernelGGL(k_probe_e, dim3(ceil_div((int64_t)mp * ldE, 256)), dim3(256), 0, st, m, mp, nprobe, seed, Emat,
                     ldE);
  // A^T-side products A E (column 0 of E is zero), then y and sqrt(D) rho
  F64RowsEpi fe{B, nullptr, nullptr, nullptr, nullptr, nullptr, ldb};
  FSA_TRY(rows_f64<ROWS_STORE>(A, nullptr, n, mp, Emat, ldE, ncols, fe, B, nullptr, 0, f32_rows_grid(), st));
  hipLaunchKernelGGL(k_probe_finish, dim3(ceil_div(n * ncols, 256)), dim3(256), 0, st, B, (int64_t)ldb, y, D, perm,
                     seed, n, ncols);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

// ================================================================ elementwise
template <typename TI, typename TO>
__global__ void k_copy_block(const TI* __restrict__ in, int ldi, TO* __restrict__ out, int ldo, int64_t n, int ncols) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t p = e / ncols;
  int c = (int)(e % ncols);
  if (p >= n) return;
  out[p * ldo + c] = (TO)in[p * ldi + c];
}

template <typename TI, typename TO>
fsa_status copy_block(const TI* in, int ldi, TO* out, int ldo, int64_t n, int ncols, hipStream_t st) {
  int64_t tot = n * ncols;
  if (tot == 0) return FSA_OK;
  hipLaunchKernelGGL((k_copy_block<TI, TO>), dim3(ceil_div(tot, 256)), dim3(256), 0, st, in, ldi, out, ldo, n, ncols);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

__global__ void k_permute_rows(const double* __restrict__ in, int ldi, double* __restrict__ out, int ldo,
                               const int* __restrict__ idx, int64_t n, int ncols) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t p = e / ncols;
  int c = (int)(e % ncols);
  if (p >= n) return;
  out[p * ldo + c] = in[(int64_t)idx[p] * ldi + c];
}

fsa_status permute_rows(const double* in, int ldi, double* out, int ldo, const int* idx, int64_t n, int ncols,
                        hipStream_t st) {
  int64_t tot = n * ncols;
  if (tot == 0) return FSA_OK;
  hipLaunchKernelGGL(k_permute_rows, dim3(ceil_div(tot, 256)), dim3(256), 0, st, in, ldi, out, ldo, idx, n, ncols);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

__global__ void k_scale_rows(double* X, int ld, const double* __restrict__ D, int64_t n, int ncols, int invert) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t p = e / ncols;
  int c = (int)(e % ncols);
  if (p >= n) return;
  X[p * ld + c] = invert ? X[p * ld + c] / D[p] : X[p * ld + c] * D[p];
}

fsa_status scale_rows(double* X, int ld, const double* D, int64_t n, int ncols, int invert, hipStream_t st) {
  int64_t tot = n * ncols;
  if (tot == 0) return FSA_OK;
  hipLaunchKernelGGL(k_scale_rows, dim3(ceil_div(tot, 256)), dim3(256), 0, st, X, ld, D, n, ncols, invert);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

__global__ void k_axpy_block(const double* __restrict__ X, double a, double* __restrict__ Y, int ld, int64_t n, int ncols) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t p = e / ncols;
  int c = (int)(e % ncols);
  if (p >= n) return;
  Y[p * ld + c] += a * X[p * ld + c];
}

fsa_status axpy_block(const double* X, double a, double* Y, int ld, int64_t n, int ncols, hipStream_t st) {
  int64_t tot = n * ncols;
  if (tot == 0) return FSA_OK;
  hipLaunchKernelGGL(k_axpy_block, dim3(ceil_div(tot, 256)), dim3(256), 0, st, X, a, Y, ld, n, ncols);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

__global__ void k_scal_block(double* X, int ld, int64_t n, int ncols, double a) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t p = e / ncols;
  int c = (int)(e % ncols);
  if (p >= n) return;
  X[p * ld + c] *= a;
}

fsa_status scal_block(double* X, int ld, int64_t n, int ncols, double a, hipStream_t st) {
  int64_t tot = n * ncols;
  if (tot == 0) return FSA_OK;
  hipLaunchKernelGGL(k_scal_block, dim3(ceil_div(tot, 256)), dim3(256), 0, st, X, ld, n, ncols, a);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

__global__ void k_reciprocal(const double* __restrict__ D, double* __restrict__ Dinv, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) Dinv[i] = 1.0 / D[i];
}

fsa_status reciprocal(const double* D, double* Dinv, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_reciprocal, dim3(ceil_div(n, 256)), dim3(256), 0, st, D, Dinv, n);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

// ================================================================ predictive variances
// Z[p][c] = Rademacher(seed, stream 2, column c, original index perm[p]) (Algorithm 1 z^(1))
__global__ void k_pred_rademacher(const int* __restrict__ perm, int64_t np, int s, uint64_t seed, double* __restrict__ Z,
                                  int ldz) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t p = e / s;
  int c = (int)(e % s);
  if (p >= np) return;
  Z[p * ldz + c] = rademacher(seed, STREAM_PRED, (uint64_t)c, (uint64_t)perm[p]);
}

fsa_status pred_rademacher(const int* perm, int64_t np, int s, uint64_t seed, double* Z, int ldz, hipStream_t st) {
  int64_t tot = np * s;
  if (tot == 0) return FSA_OK;
  hipLaunchKernelGGL(k_pred_rademacher, dim3(ceil_div(tot, 256)), dim3(256), 0, st, perm, np, s, seed, Z, ldz);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

// One wave per prediction point (sorted slot p):
// D1 = |a|^2 - |y|^2, D2 = z . y, D3 = |z|^2 with a = A_p row, y = L_M^{-1} a,
// z = L_M^{-1} (S_p^T V~) row; D_l = mean_c z1_c (S_p^T W_l)_c; the variance
// sigma1^2 + sigma^2 - D1 - 2 D2 + D3 - D_l goes to the caller's slot perm[p].
__global__ __launch_bounds__(256) void k_pred_combine(int64_t np, int mp, const double* __restrict__ Ap,
                                                      const double* __restrict__ Y, const double* __restrict__ Z2,
                                                      const double* __restrict__ Z1, const double* __restrict__ Zl,
                                                      int ldl, int s, double s1, double s2, const int* __restrict__ perm,
                                                      double* __restrict__ var_out, double* __restrict__ parts) {
  const int lane = threadIdx.x & 63;
  const int64_t p = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (p >= np) return;
  double aa = 0, yy = 0, zy = 0, zz = 0, dl = 0;
  for (int k = lane; k < mp; k += 64) {
    double a = Ap[p * mp + k], y = Y[p * mp + k], z = Z2[p * mp + k];
    aa += a * a;
    yy += y * y;
    zy += z * y;
    zz += z * z;
  }
  for (int c = lane; c < s; c += 64) dl += Z1[p * ldl + c] * Zl[p * ldl + c];
  aa = wave_sum(aa);
  yy = wave_sum(yy);
  zy = wave_sum(zy);
  zz = wave_sum(zz);
  dl = wave_sum(dl);
  if (lane == 0) {
    double D1 = aa - yy, D2 = zy, D3 = zz, Dl = s > 0 ? dl / s : 0.0;
    int o = perm[p];
    var_out[o] = s1 + s2 - D1 - 2.0 * D2 + D3 - Dl;
    if (parts) {
      parts[4 * (int64_t)o + 0] = D1;
      parts[4 * (int64_t)o + 1] = D2;
      parts[4 * (int64_t)o + 2] = D3;
      parts[4 * (int64_t)o + 3] = Dl;
    }
  }
}

fsa_status pred_combine(int64_t np, int mp, const double* Ap, const double* Y, const double* Z2, const double* Z1,
                        const double* Zl, int ldl, int s, double s1, double s2, const int* perm, double* var_out,
                        double* parts, hipStream_t st) {
  hipLaunchKernelGGL(k_pred_combine, dim3(ceil_div(np, 4)), dim3(256), 0, st, np, mp, Ap, Y, Z2, Z1, Zl, ldl, s, s1, s2,
                     perm, var_out, parts);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

// mean[perm[p]] = A_p row . w + (S_p^T u)_p
__global__ void k_pred_mean(int64_t np, int mp, const double* __restrict__ Ap, const double* __restrict__ w,
                            const double* __restrict__ su, const int* __restrict__ perm, double* __restrict__ out) {
  int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= np) return;
  double v = su[p];
  for (int k = 0; k < mp; ++k) v += Ap[p * mp + k] * w[k];
  out[perm[p]] = v;
}

fsa_status pred_mean(int64_t np, int mp, const double* Ap, const double* w, const double* su, const int* perm,
                     double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_pred_mean, dim3(ceil_div(np, 256)), dim3(256), 0, st, np, mp, Ap, w, su, perm, out);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

__global__ void k_symmetrize(double* A, int n) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  int i = (int)(e / n), j = (int)(e % n);
  if (j < i) {
    double v = 0.5 * (A[(int64_t)i * n + j] + A[(int64_t)j * n + i]);
    A[(int64_t)i * n + j] = v;
    A[(int64_t)j * n + i] = v;
  }
}

fsa_status symmetrize(double* A, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_symmetrize, dim3(ceil_div((int64_t)n * n, 256)), dim3(256), 0, st, A, n);
  FSA_HIP(hipGetLastError());
  return FSA_OK;
}

// ================================================================ instantiations
template fsa_status lowrank_reduce<double>(const double*, int64_t, int, const double*, int, int, const double*, Scratch&,
                                           double*, int, hipStream_t);
template fsa_status lowrank_reduce<float>(const float*, int64_t, int, const float*, int, int, const double*, Scratch&,
                                          double*, int, hipStream_t);
template fsa_status lowrank_expand<double>(const double*, const double*, int64_t, int, const double*, int, int, double*,
                                           int, hipStream_t);
template fsa_status lowrank_expand<float>(const float*, const float*, int64_t, int, const float*, int, int, float*, int,
                                          hipStream_t);
template fsa_status spmm<double>(const Csr&, const Grid&, const Grid&, const double*, const double*, int, int, double*,
                                 int, bool, hipStream_t);
template fsa_status spmm<float>(const Csr&, const Grid&, const Grid&, const float*, const float*, int, int, float*, int,
                                bool, hipStream_t);
template fsa_status coldot<double, double>(const double*, const double*, int64_t, int, int, double*, Scratch&,
                                           hipStream_t);
template fsa_status coldot<float, float>(const float*, const float*, int64_t, int, int, double*, Scratch&,
                                        hipStream_t);
template fsa_status coldot<double, float>(const double*, const float*, int64_t, int, int, double*, Scratch&,
                                          hipStream_t);
template fsa_status mspace_apply<double>(const double*, const double*, int, int, int, double*, int, hipStream_t);
template fsa_status mspace_apply<float>(const double*, const double*, int, int, int, float*, int, hipStream_t);
template fsa_status pcg_init<double>(PcgBlock<double>&, const OpDesc<double>&, const double*, double, Scratch&,
                                     hipStream_t);
template fsa_status pcg_init<float>(PcgBlock<float>&, const OpDesc<float>&, const double*, double, Scratch&,
                                    hipStream_t);
template fsa_status pcg_iter<double>(PcgBlock<double>&, const OpDesc<double>&, double, int, Scratch&, hipStream_t);
template fsa_status pcg_iter<float>(PcgBlock<float>&, const OpDesc<float>&, double, int, Scratch&, hipStream_t);
template fsa_status copy_block<double, double>(const double*, int, double*, int, int64_t, int, hipStream_t);
template fsa_status copy_block<double, float>(const double*, int, float*, int, int64_t, int, hipStream_t);
template fsa_status copy_block<float, double>(const float*, int, double*, int, int64_t, int, hipStream_t);

}  // namespace fsa
