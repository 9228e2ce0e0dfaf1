// Launchers of the FSA operations (float64 or float32 element type T).
#pragma once

#include "common.hpp"
#include "kernels.hpp"

namespace fsa {

// Scratch for split reductions, grown on demand.
struct Scratch {
  Buf<double> dot;   // per-workgroup column partials
  Buf<double> dot2;
  Buf<char> part;    // reduce-GEMM partial tiles
  Buf<double> w;     // reduced m-space block (kdim x ldw)
  Buf<double> dot1;  // first-stage column sums of many partials
};

// Timing events are kept in a process-wide free list across contexts.
hipEvent_t timer_event_get();  // nullptr if none can be created
void timer_event_put(hipEvent_t e);

// HIP-event timing of kernel classes on one stream (enabled per context).
// Only the classes in `mask` (bit k: class k) are timed: each timed launch
// costs two event records on the stream.
struct KernelTimer {
  static constexpr int NCLS = 5;
  bool on = false;
  unsigned mask = 0;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<int> cls;
  void reset() { used = 0; cls.clear(); }
  int start(int k, hipStream_t st) {
    if (!on || !((mask >> k) & 1u)) return -1;
    if (used + 2 > pool.size()) {
      for (int k = 0; k < 256; ++k) {
        hipEvent_t e = timer_event_get();
        if (!e) return -1;
        pool.push_back(e);
      }
    }
    int i = (int)used;
    used += 2;
    (void)hipEventRecord(pool[i], st);
    return i;
  }
  void stop(int k, int i, hipStream_t st) {
    if (i < 0) return;
    (void)hipEventRecord(pool[i + 1], st);
    if ((int)cls.size() <= i / 2) cls.resize(i / 2 + 1, -1);
    cls[i / 2] = k;
  }
  // after the stream has drained
  void collect(double* ms, int* cnt) {
    for (size_t j = 0; j < cls.size(); ++j) {
      if (cls[j] < 0) continue;
      float t = 0.f;
      if (hipEventElapsedTime(&t, pool[2 * j], pool[2 * j + 1]) == hipSuccess) {
        ms[cls[j]] += t;
        cnt[cls[j]] += 1;
      }
    }
    reset();
  }
  ~KernelTimer() {
    for (auto e : pool) timer_event_put(e);
  }
};
enum { KT_SPMM = 0, KT_PASS1 = 1, KT_PASS2 = 2, KT_UPDATE = 3, KT_SMALL = 4 };

// ---- float64 factor kernels (whiten.hip) ----
// Linv := L^{-1} for row-major lower-triangular L (mp x mp, mp % 64 == 0, mp <= 512)
fsa_status tri_inverse(const double* L, double* Linv, int mp, hipStream_t st);
// Y := X W^T for point-major X (n x mp) and lower-triangular W given as WT = W^T (row-major mp x mp)
fsa_status rows_times_lower_t(const double* X, int64_t n, int mp, const double* WT, double* Y, hipStream_t st);
// F := dSigma_nm L_m^{-T} - A Phi(E)^T (point-major n x mp), dSigma_nm generated on the fly;
// LminvT = (L_m^{-1})^T, PhiT_neg = -Phi(E)^T, both row-major mp x mp
// Af non-null: in float32 arithmetic from the float32 copy of A (F_out gets the
// float32 result widened; Ff_out, if non-null, the float32 one)
fsa_status derivative_factor(const double* xs, int64_t n, const double* ind, int m, int mp, const Theta& th,
                             const double* LminvT, const double* A, const double* PhiT_neg, double* F_out,
                             hipStream_t st, const float* Af = nullptr, float* Ff_out = nullptr);

// ---- build-time contractions (float64) ----
// out[i][k] = c(x_i, ind_k) (deriv: dc/drho) for k < m, 0 for m <= k < mp
// (point-major n x mp, Section 2.1)
fsa_status cov_block(const double* xs, int64_t n, const double* ind, int m, int mp, const Theta& th, bool deriv,
                     double* out, hipStream_t st);
// A = L_m^{-1} Sigma_mn = Sigma_nm L_m^{-T} (point-major n x mp): whitened low-rank factor,
// Sigma_nm generated on the fly (never stored); LminvT = (L_m^{-1})^T (row-major mp x mp)
// (Af_out: optionally the same factor rounded to float32, written by the same kernel)
fsa_status whiten(const double* xs, int64_t n, const double* ind, int m, int mp, const Theta& th,
                  const double* LminvT, double* A_out, hipStream_t st, float* Af_out = nullptr);
// Residual values of a taper pattern (rows of grid rg, columns of grid cg):
// v = (c(d) - Xr_p . Yc_q) W(d/gamma) (+ s2 on the self diagonal, D[p] = v_pp).
// deriv: v = (dc/drho(d) - [F|A]_p . [A|F]_q) W(d/gamma).
fsa_status residual_values(const Grid& rg, const Grid& cg, const Csr& csr, const double* Xr, const double* Yc,
                           const double* Fr, const double* Fc, int mp, const Theta& th, double gamma, bool self,
                           bool deriv, double* vals, double* D, hipStream_t st);
// deriv values of one point set (grid g against itself) from float32 rows:
// v = (dc/drho(d) - [Ff|Af]_p . [Af|Ff]_q) W(d/gamma), the dot on the float32 MFMA
fsa_status derivative_values_f32(const Grid& g, const Csr& csr, const float* Af, const float* Ff, int mp,
                                 const Theta& th, double gamma, double* vals, hipStream_t st);
// C = I + A D^{-1} A^T (mp x mp float64)
fsa_status capacitance(const double* A, const double* D, int64_t n, int mp, double* C, Scratch& s, hipStream_t st);

// ---- block operations on n x ld point-major blocks ----
// W (float64, kdim x ldw) = A^T-side reduction sum_i A_i^T X_i with X = src / D (scale_by_dinv)
template <typename T>
fsa_status lowrank_reduce(const T* A, int64_t n, int kdim, const T* X, int ldx, int ncols, const double* Dinv_src,
                          Scratch& s, double* W, int ldw, hipStream_t st);
// OUT = A G (+ beta_out * OUT_prev handled by caller), G row-major kdim x ldg (type T)
template <typename T>
fsa_status lowrank_expand(const T* A, const T* A2, int64_t n, int kdim, const T* G, int ldg, int ncols, T* OUT,
                          int ldo, hipStream_t st);
// Y = S X (+ Y if accumulate) ; S in CSR with values val, rows of grid rg,
// columns of grid cg (cell-aligned grids)
template <typename T>
fsa_status spmm(const Csr& S, const Grid& rg, const Grid& cg, const T* val, const T* X, int ldx, int ncols, T* Y,
                int ldy, bool accumulate, hipStream_t st);
// The float32 sparse part as dense 64 x 64 tiles in MFMA order, one per
// (64-row group, 64-position neighbourhood chunk) of each cell pair (cells
// 2 sx, 2 sx + 1 of a cell row); toff (spmm_tile_pairs(g) + 1) gives each
// pair's first tile.  The pattern's rows and columns are both the grid g.
fsa_status build_spmm_tiles(const Csr& S, const Grid& g, const float* val, Buf<int64_t>& toff, Buf<float>& tiles,
                            Buf<unsigned>& tmask, hipStream_t st);
// Cell pairs of grid g (ceil(gx / 2) per cell row); also the number of
// partial dot rows the tiled product writes.
int64_t spmm_tile_pairs(const Grid& g);
// out[c] = sum_p H[p][c] (S X)[p][c] for c < ncols (float64 result; S X is
// not stored), S with the pattern of grid g on both sides
template <typename T>
fsa_status spmm_dot(const Csr& S, const Grid& g, const T* val, const T* X, const T* H, int ld, int ncols,
                    double* out, Scratch& s, hipStream_t st);
// out[c] = sum_k part[k * ldp + c], k < nparts, for c < ncols (fixed order)
fsa_status colsum(const double* part, int nparts, int ldp, int ncols, double* out, hipStream_t st);
// out[c] = sum_p X[p][c] Y[p][c] (float64 result, c < ncols)
template <typename TX, typename TY>
fsa_status coldot(const TX* X, const TY* Y, int64_t n, int ld, int ncols, double* out, Scratch& s, hipStream_t st);
// G (type T, kdim x ldg) = M (kdim x kdim f64) * W (kdim x ldw f64), columns < ncols
template <typename T>
fsa_status mspace_apply(const double* M, const double* W, int ldw, int kdim, int ncols, T* G, int ldg,
                        hipStream_t st);

// ---- PCG (Algorithm 2) on a block of columns ----
template <typename T>
struct PcgBlock {
  int64_t n = 0;
  int ncols = 0, ld = 0, ldw = 0;
  int max_iter = 0;
  // block vectors (n x ld)
  T *R = nullptr, *H = nullptr, *V = nullptr, *P = nullptr, *Tt = nullptr, *Q0 = nullptr;
  double* U = nullptr;  // solution accumulator (float64)
  // float32 operator only (may be null): the solution increments since the
  // last fold into U, accumulated in float32 (half the bytes of U per
  // iteration); pcg_fold_u adds them to U and clears them
  float* U32 = nullptr;
  // per column
  double *rz = nullptr, *rz0 = nullptr, *alpha = nullptr, *beta = nullptr, *rr = nullptr, *bn2 = nullptr;
  int *active = nullptr, *iters = nullptr, *flags = nullptr;  // flags[0] = #active, flags[1] = breakdown
  double *alpha_hist = nullptr, *beta_hist = nullptr;
  T* g = nullptr;  // m-space block in T (kdim x ldw)
  KernelTimer* timer = nullptr;
};

// Operator description: sparse part (CSR values valT, diagonal D) plus an
// optional low-rank part A (point-major n x kdim) with Woodbury capacitance
// inverse Cinv (kdim x kdim f64); kdim == 0 gives the sparse operator with
// the diagonal preconditioner.
template <typename T>
struct OpDesc {
  const Grid* grid = nullptr;  // row = column grid of S
  const Csr* S = nullptr;
  const T* val = nullptr;
  const double* D = nullptr;
  const double* Dinv = nullptr;  // 1 / D
  const T* A = nullptr;
  const uint16_t* Abf = nullptr;  // float32 operator only: A in bfloat16 for the PCG passes (else null)
  // with Abf: the same values point-interleaved, [ceil(n/8)][kdim][8] (zero
  // past n), for the bfloat16-MFMA residual pass (null: widen Abf instead)
  const uint16_t* Abf8 = nullptr;
  // float32 operator with A in float32: the low-rank passes on the bfloat16
  // matrix cores with operands split in three parts (k_reduce_split,
  // k_rows_split) instead of the float32 matrix cores
  bool split = false;
  int kdim = 0;
  const double* Cinv = nullptr;
  // float32 operator only (may be null): the sparse part pre-scattered into
  // dense MFMA-order tiles (build_spmm_tiles), used by the sparse product
  const int64_t* tile_off = nullptr;
  const float* tiles = nullptr;
  const unsigned* tile_mask = nullptr;  // per tile: its 16 x 16 blocks that hold a nonzero
};

// Initialise: R = B, U = 0, Q0 = H = P^{-1} R, P = A^T A H, rz = r^T q.
template <typename T>
fsa_status pcg_init(PcgBlock<T>& b, const OpDesc<T>& op, const double* B, double tol, Scratch& s, hipStream_t st);
// One iteration on all active columns; the Lanczos coefficients of the
// iteration are appended to alpha_hist/beta_hist.
template <typename T>
fsa_status pcg_iter(PcgBlock<T>& b, const OpDesc<T>& op, double tol, int fixed, Scratch& s, hipStream_t st);
// Stopping test on the float64 residual (mixed precision), after R has just
// been replaced by B - A_op U: rr = |R|^2 per column; the columns at or above
// tol^2 |b|^2 become active again and flags[0] counts them.
fsa_status pcg_recheck_true_residual(PcgBlock<float>& b, double tol, Scratch& s, hipStream_t st);
// U += U32, U32 = 0 (no-op when U32 is null).
fsa_status pcg_fold_u(PcgBlock<float>& b, hipStream_t st);
// Replace R by B - A_op U with the float64 operator (mixed precision); folds
// U32 into U first.
fsa_status pcg_replace_residual_f32(PcgBlock<float>& b, const OpDesc<double>& op64, const OpDesc<float>& op32,
                                    const double* B, Scratch& s, hipStream_t st);

// out[c] = w_c e_1^T log(T_c) e_1 for c in [c_first, ncols) (tridiagonal QL)
fsa_status slq_terms(const double* alpha_hist, const double* beta_hist, const int* iters, int ncols, int c_first,
                     const double* weight, double* out, double* scratch, int max_iter, hipStream_t st);

// B[:,0] = y, B[:,1+i] = sqrt(D) rho_i + A^T e_i  (probe block, Section 3.3 / App. F)
fsa_status make_probes(const double* A, int64_t n, int m, int mp, const double* D, const double* y, const int* perm,
                       uint64_t seed, int nprobe, double* B, int ldb, double* Emat, hipStream_t st);

// predictive variances (Algorithm 1)
fsa_status pred_rademacher(const int* perm, int64_t np, int s, uint64_t seed, double* Z, int ldz, hipStream_t st);
fsa_status pred_combine(int64_t np, int mp, const double* Ap, const double* Y, const double* Z2, const double* Z1,
                        const double* Zl, int ldl, int s, double s1, double s2, const int* perm, double* var_out,
                        double* parts, hipStream_t st);
fsa_status pred_mean(int64_t np, int mp, const double* Ap, const double* w, const double* su, const int* perm,
                     double* out, hipStream_t st);
fsa_status symmetrize(double* A, int n, hipStream_t st);

// out[((p/8) kdim + k) 8 + p%8] = A[p][k] (bfloat16, n x kdim point-major),
// zero for the padding points up to a multiple of 8
fsa_status bf16_interleave8(const uint16_t* A, int64_t n, int kdim, uint16_t* out, hipStream_t st);
// bfloat16 (round to nearest even, through float32) of a float64 array: the
// bits to out and/or the rounded value to rounded (either may be null;
// rounded may alias in)
fsa_status to_bf16(const double* in, uint16_t* out, double* rounded, int64_t cnt, hipStream_t st);

// elementwise helpers
template <typename TI, typename TO>
fsa_status copy_block(const TI* in, int ldi, TO* out, int ldo, int64_t n, int ncols, hipStream_t st);
fsa_status permute_rows(const double* in, int ldi, double* out, int ldo, const int* idx, int64_t n, int ncols,
                        hipStream_t st);  // out[p] = in[idx[p]]
fsa_status scale_rows(double* X, int ld, const double* D, int64_t n, int ncols, int invert, hipStream_t st);
fsa_status scal_block(double* X, int ld, int64_t n, int ncols, double a, hipStream_t st);
fsa_status axpy_block(const double* X, double a, double* Y, int ld, int64_t n, int ncols, hipStream_t st);
fsa_status reciprocal(const double* D, double* Dinv, int64_t n, hipStream_t st);

}  // namespace fsa
