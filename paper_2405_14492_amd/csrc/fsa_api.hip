// C ABI of the FSA library: context lifetime, build and revaluation, the
// PCG/SLQ likelihood with its stochastic gradient, predictive variances and
// inspection hooks.  All arithmetic runs in the kernels of geom/dense/ops;
// this file orders launches and moves scalars.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <vector>

#include "ops.hpp"

namespace fsa {

// ---------------------------------------------------------------- errors
static thread_local char g_err[1024] = "";
void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}
const char* get_error() { return g_err; }

// ---------------------------------------------------------------- pool
namespace {
struct FreeBlock {
  void* p;
  hipStream_t st;  // stream current when the block was released
  hipEvent_t ev;   // recorded on st at the release
};
// A block from the caller's allocator (fsa_set_allocator) and where it goes back.
struct UserAlloc {
  fsa_alloc_fn alloc = nullptr;
  fsa_release_fn release = nullptr;
  void* user = nullptr;
};
struct LiveBlock {
  size_t bytes;
  UserAlloc from;  // from.release == nullptr: the library's own pool
};
// A released block of the caller's allocator, handed back once the event
// recorded at its release (after every use the library enqueued) has passed.
struct Pending {
  void* p;
  hipEvent_t ev;
  UserAlloc to;
};
std::mutex g_pool_mu;
std::multimap<size_t, FreeBlock> g_free;  // rounded size -> block
std::map<void*, LiveBlock> g_live;        // block -> rounded size and origin
std::vector<hipEvent_t> g_events;         // idle events
std::vector<Pending> g_pending;
UserAlloc g_user;                         // the registered allocator (alloc == nullptr: none)
thread_local hipStream_t t_stream = nullptr;
size_t pool_round(size_t b) {
  const size_t g = b < (1u << 20) ? 4096 : (size_t(2) << 20);
  return (b + g - 1) / g * g;
}
// with g_pool_mu held
void release_cached_locked() {
  for (auto& kv : g_free) {
    (void)hipEventSynchronize(kv.second.ev);
    (void)hipFree(kv.second.p);
    g_events.push_back(kv.second.ev);
  }
  g_free.clear();
}
hipEvent_t event_get_locked() {
  if (!g_events.empty()) {
    hipEvent_t e = g_events.back();
    g_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}
// Hand the caller's blocks whose last use has completed back to their
// allocator (all of them, waiting, with wait = true).  The callbacks run
// without the pool lock held.
void flush_pending(bool wait) {
  std::vector<Pending> ready;
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    for (size_t i = 0; i < g_pending.size();) {
      Pending& q = g_pending[i];
      bool done = true;
      if (q.ev) {
        if (wait) (void)hipEventSynchronize(q.ev);
        const hipError_t e = hipEventQuery(q.ev);
        done = e == hipSuccess;
        if (e != hipSuccess && e != hipErrorNotReady) (void)hipGetLastError();
      }
      if (done) {
        if (q.ev) g_events.push_back(q.ev);
        ready.push_back(q);
        g_pending[i] = g_pending.back();
        g_pending.pop_back();
      } else {
        ++i;
      }
    }
  }
  for (auto& q : ready) q.to.release(q.p, q.to.user);
}
}  // namespace

hipStream_t pool_stream() { return t_stream; }
void pool_set_stream(hipStream_t st) { t_stream = st; }

// ---- regions
namespace {
thread_local Region* t_region = nullptr;
constexpr size_t kRegionAlign = 256;
}  // namespace
Region* pool_region() { return t_region; }
void pool_set_region(Region* r) { t_region = r; }

Region::Region(void* base, size_t bytes) : base_(static_cast<char*>(base)), size_(bytes / kRegionAlign * kRegionAlign) {
  if (size_) free_.emplace_back(0, size_);
}

Region::~Region() { settle(); }

bool Region::owns(const void* p) const {
  const char* c = static_cast<const char*>(p);
  return c >= base_ && c < base_ + size_;
}

void Region::insert_free(size_t off, size_t len) {
  auto it = std::lower_bound(free_.begin(), free_.end(), std::make_pair(off, (size_t)0));
  it = free_.insert(it, {off, len});
  // coalesce with the successor, then with the predecessor
  auto nx = it + 1;
  if (nx != free_.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    free_.erase(nx);
  }
  if (it != free_.begin()) {
    auto pv = it - 1;
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      free_.erase(it);
    }
  }
}

void Region::reclaim(bool wait) {
  for (size_t i = 0; i < pend_.size();) {
    Pend& q = pend_[i];
    bool done = true;
    if (q.ev) {
      if (wait) (void)hipEventSynchronize(q.ev);
      const hipError_t e = hipEventQuery(q.ev);
      done = e == hipSuccess;
      if (e != hipSuccess && e != hipErrorNotReady) (void)hipGetLastError();
    }
    if (done) {
      if (q.ev) {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        g_events.push_back(q.ev);
      }
      insert_free(q.off, q.len);
      pend_[i] = pend_.back();
      pend_.pop_back();
    } else {
      ++i;
    }
  }
}

void Region::settle() { reclaim(true); }

void* Region::alloc(size_t bytes) {
  const size_t r = (std::max<size_t>(bytes, 1) + kRegionAlign - 1) / kRegionAlign * kRegionAlign;
  for (int pass = 0; pass < 2; ++pass) {
    reclaim(pass == 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < r) continue;
      const size_t off = it->first;
      if (it->second == r) free_.erase(it);
      else {
        it->first += r;
        it->second -= r;
      }
      used_.insert(std::lower_bound(used_.begin(), used_.end(), std::make_pair(off, (size_t)0)), {off, r});
      live_ += r;
      peak_ = std::max(peak_, live_);
      return base_ + off;
    }
  }
  return nullptr;
}

void Region::release(void* p, hipStream_t st) {
  const size_t off = (size_t)(static_cast<char*>(p) - base_);
  auto it = std::lower_bound(used_.begin(), used_.end(), std::make_pair(off, (size_t)0));
  if (it == used_.end() || it->first != off) return;
  const size_t len = it->second;
  used_.erase(it);
  live_ -= len;
  hipEvent_t ev = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    ev = event_get_locked();
  }
  if (ev && hipEventRecord(ev, st) != hipSuccess) {
    (void)hipGetLastError();
    std::lock_guard<std::mutex> lk(g_pool_mu);
    g_events.push_back(ev);
    ev = nullptr;
  }
  if (!ev) (void)hipStreamSynchronize(st);
  pend_.push_back(Pend{off, len, ev});
}

void* pool_alloc(size_t bytes) {
  if (t_region) return t_region->alloc(bytes);
  size_t r = pool_round(bytes);
  UserAlloc ua;
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    ua = g_user;
  }
  if (ua.alloc) {
    flush_pending(false);
    void* p = ua.alloc(r, reinterpret_cast<void*>(t_stream), ua.user);
    if (!p) return nullptr;
    std::lock_guard<std::mutex> lk(g_pool_mu);
    g_live[p] = LiveBlock{r, ua};
    return p;
  }
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    auto it = g_free.find(r);
    if (it != g_free.end()) {
      FreeBlock fb = it->second;
      g_free.erase(it);
      if (fb.st != t_stream) (void)hipStreamWaitEvent(t_stream, fb.ev, 0);
      g_events.push_back(fb.ev);
      g_live[fb.p] = LiveBlock{r, UserAlloc{}};
      return fb.p;
    }
  }
  void* p = nullptr;
  if (hipMalloc(&p, r) != hipSuccess) {
    (void)hipGetLastError();
    // release cached blocks and retry once
    std::lock_guard<std::mutex> lk(g_pool_mu);
    release_cached_locked();
    if (hipMalloc(&p, r) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
  }
  std::lock_guard<std::mutex> lk(g_pool_mu);
  g_live[p] = LiveBlock{r, UserAlloc{}};
  return p;
}

void pool_free(void* p) {
  if (!p) return;
  if (t_region && t_region->owns(p)) {
    t_region->release(p, t_stream);
    return;
  }
  bool user = false;
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    auto it = g_live.find(p);
    if (it == g_live.end()) return;
    const LiveBlock lb = it->second;
    g_live.erase(it);
    hipEvent_t ev = event_get_locked();
    if (ev) (void)hipEventRecord(ev, t_stream);
    if (lb.from.release) {
      // the caller's block: back to its allocator once this event has passed
      if (!ev) (void)hipStreamSynchronize(t_stream);
      g_pending.push_back(Pending{p, ev, lb.from});
      user = true;
    } else if (ev) {
      g_free.emplace(lb.bytes, FreeBlock{p, t_stream, ev});
    } else {
      // no event: make the block safe to reuse anywhere by draining its stream
      (void)hipStreamSynchronize(t_stream);
      (void)hipFree(p);
    }
  }
  if (user) flush_pending(false);
}

void pool_flush() { flush_pending(true); }

void pool_trim() {
  flush_pending(true);
  std::lock_guard<std::mutex> lk(g_pool_mu);
  release_cached_locked();
}

// ---------------------------------------------------------------- small kernels
// sum_i log D_i in two fixed-order stages: part[b] over the points
// b, b + G, b + 2G, ... (G = gridDim.x), then the G partials; flags a
// non-positive or non-finite D_i.
__global__ __launch_bounds__(256) void k_sum_log_part(const double* __restrict__ D, int64_t n, double* part, int* bad) {
  __shared__ double s[256];
  double a = 0.0;
  int b = 0;
  for (int64_t i = blockIdx.x + (int64_t)gridDim.x * threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double v = D[i];
    if (!(v > 0.0) || !isfinite(v)) b = 1;
    a += log(v);
  }
  s[threadIdx.x] = a;
  if (b) atomicOr(bad, 1);
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}
__global__ __launch_bounds__(256) void k_sum_fixed(const double* __restrict__ part, int np, double* out) {
  __shared__ double s[256];
  double a = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) a += part[i];
  s[threadIdx.x] = a;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s[0];
}

__global__ void k_count_bad(const double* __restrict__ v, int64_t cnt, int* bad) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < cnt && !isfinite(v[i])) atomicOr(bad, 1);
}

__global__ void k_pad_inducing(const double* __restrict__ in, int m, int mp, double* __restrict__ out) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= mp) return;
  out[2 * k] = k < m ? in[2 * k] : 0.0;
  out[2 * k + 1] = k < m ? in[2 * k + 1] : 0.0;
}

// results[0] = log det, [1] = quad, [2] = nll
__global__ void k_finalize_nll(const double* __restrict__ slq, int ncols, const double* __restrict__ logdet_parts,
                               const double* __restrict__ quad, int64_t n, double* out) {
  double s = 0.0;
  for (int c = 1; c < ncols; ++c) s += slq[c];
  double logdet = s / (double)(ncols - 1) + logdet_parts[0] + logdet_parts[1];
  out[0] = logdet;
  out[1] = quad[0];
  out[2] = 0.5 * (double)n * 1.8378770664093453 + 0.5 * logdet + 0.5 * quad[0];
}

// grad from column dots: uSX = U.(Sigma X), uX = U.X, uDX = U.(dSigma/drho X)
__global__ void k_finalize_grad(int ncols, const double* __restrict__ uSX, const double* __restrict__ uX,
                                const double* __restrict__ uDX, double s1, double s2, double* out) {
  double tr[3] = {0, 0, 0};
  for (int c = 1; c < ncols; ++c) {
    tr[0] += (uSX[c] - s2 * uX[c]) / s1;
    tr[1] += uDX[c];
    tr[2] += uX[c];
  }
  double t = (double)(ncols - 1);
  double qd[3] = {(uSX[0] - s2 * uX[0]) / s1, uDX[0], uX[0]};
  for (int k = 0; k < 3; ++k) {
    out[k] = 0.5 * tr[k] / t - 0.5 * qd[k];
    out[3 + k] = tr[k] / t;
    out[6 + k] = qd[k];
  }
}

// Low-rank parts of the gradient's column dots from the m-space blocks
// (kdim x ldw, row-major): with a = A^T x, f = F^T x, au = A^T u, fu = F^T u,
// u.(A A^T x) = au . a and u.((F A^T + A F^T) x) = fu . a + au . f.
// One workgroup (256 threads) per column, fixed-order tree sum over k.
// Also |a|^2 and f . a (the control variate's low-rank terms).
__global__ __launch_bounds__(256) void k_grad_mdots(const double* __restrict__ a, const double* __restrict__ f,
                                                    const double* __restrict__ au, const double* __restrict__ fu,
                                                    int kdim, int ldw, double* __restrict__ lr_sigma,
                                                    double* __restrict__ lr_drho, double* __restrict__ aa,
                                                    double* __restrict__ fa) {
  __shared__ double r[4][256];
  const int c = blockIdx.x, t = threadIdx.x;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  for (int k = t; k < kdim; k += 256) {
    const int64_t o = (int64_t)k * ldw + c;
    s0 += au[o] * a[o];
    s1 += fu[o] * a[o] + au[o] * f[o];
    s2 += a[o] * a[o];
    s3 += f[o] * a[o];
  }
  r[0][t] = s0;
  r[1][t] = s1;
  r[2][t] = s2;
  r[3][t] = s3;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h)
      for (int j = 0; j < 4; ++j) r[j][t] += r[j][t + h];
    __syncthreads();
  }
  if (t == 0) {
    lr_sigma[c] = r[0][0];
    lr_drho[c] = r[1][0];
    aa[c] = r[2][0];
    fa[c] = r[3][0];
  }
}

// ---- control variate (App. E) ----
// A coefficient is taken as 0 when its b_i hardly vary (centred sum of
// squares at most this fraction of sum_i b_i^2): then any c leaves the
// estimate unchanged up to rounding, and the ratio is noise.
constexpr double CV_DEGENERATE = 1e-12;
// out[p] = the value of row p's diagonal entry (0 if the pattern has none)
__global__ void k_csr_diag(const int64_t* __restrict__ rp, const int* __restrict__ col, const double* __restrict__ v,
                           int64_t n, double* __restrict__ out) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= n) return;
  double d = 0.0;
  for (int64_t e = rp[p]; e < rp[p + 1]; ++e)
    if (col[e] == (int)p) d = v[e];
  out[p] = d;
}

// Per-workgroup partial sums for the exact Tr(P^{-1} dP/dtheta): with rows
// ba_p = L_C^{-1} A_p and bf_p = L_C^{-1} F_p (so s_p = |ba_p|^2 = A_p C^{-1} A_p^T and
// r_p = ba_p . bf_p = A_p C^{-1} F_p^T),
//   [0] sum 1/D_p  [1] sum s_p/D_p^2  [2] sum dD_p/D_p  [3] sum dD_p s_p/D_p^2  [4] sum r_p/D_p.
// One wave per point (kdim a multiple of 64), fixed order throughout.
__global__ __launch_bounds__(256) void k_cv_trace_parts(const double* __restrict__ BA, const double* __restrict__ BF,
                                                        const double* __restrict__ D, const double* __restrict__ dD,
                                                        int64_t n, int kdim, double* __restrict__ part) {
  __shared__ double red[4][5];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double acc[5] = {0, 0, 0, 0, 0};
  for (int64_t p = blockIdx.x * 4 + w; p < n; p += (int64_t)gridDim.x * 4) {
    double sa = 0.0, sr = 0.0;
    for (int k = lane; k < kdim; k += 64) {
      const double a = BA[p * kdim + k];
      sa += a * a;
      sr += a * BF[p * kdim + k];
    }
    for (int o = 32; o > 0; o >>= 1) {
      sa += __shfl_xor(sa, o, 64);
      sr += __shfl_xor(sr, o, 64);
    }
    const double d = D[p], dd = dD[p];
    acc[0] += 1.0 / d;
    acc[1] += sa / (d * d);
    acc[2] += dd / d;
    acc[3] += dd * sa / (d * d);
    acc[4] += sr / d;
  }
  if (lane == 0)
    for (int j = 0; j < 5; ++j) red[w][j] = acc[j];
  __syncthreads();
  if (threadIdx.x < 5) {
    const int j = threadIdx.x;
    part[(int64_t)blockIdx.x * 5 + j] = (red[0][j] + red[1][j]) + (red[2][j] + red[3][j]);
  }
}

__global__ void k_cv_trace_final(const double* __restrict__ part, int nparts, double* __restrict__ out) {
  const int j = threadIdx.x;
  if (j >= 5) return;
  double s = 0.0;
  for (int b = 0; b < nparts; ++b) s += part[(int64_t)b * 5 + j];
  out[j] = s;
}

// Per column c of X (n x ld): partial sums of x^2, D x^2 and dD x^2 per
// workgroup, planes [3][gridDim.x][ldp] (coalesced over columns).
__global__ __launch_bounds__(256) void k_cv_xdots(const double* __restrict__ X, int64_t n, int ld, int ncols,
                                                  const double* __restrict__ D, const double* __restrict__ dD,
                                                  double* __restrict__ part, int ldp) {
  __shared__ double red[3][4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int c = blockIdx.y * 64 + lane;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  if (c < ncols)
    for (int64_t p = (int64_t)blockIdx.x * 4 + w; p < n; p += (int64_t)gridDim.x * 4) {
      const double x = X[p * ld + c];
      const double x2 = x * x;
      a0 += x2;
      a1 += D[p] * x2;
      a2 += dD[p] * x2;
    }
  red[0][w][lane] = a0;
  red[1][w][lane] = a1;
  red[2][w][lane] = a2;
  __syncthreads();
  if (threadIdx.x < 64) {
    const int64_t o = (int64_t)blockIdx.x * ldp + blockIdx.y * 64 + threadIdx.x;
    const int64_t plane = (int64_t)gridDim.x * ldp;
    for (int j = 0; j < 3; ++j)
      part[j * plane + o] = (red[j][0][threadIdx.x] + red[j][1][threadIdx.x]) + (red[j][2][threadIdx.x] + red[j][3][threadIdx.x]);
  }
}

// The gradient with the control variate (App. E, eq. Troptc), one thread.
// Per probe column i >= 1: samples a_k and control terms b_k,
//   a_0 = (u.Sx - s2 u.x)/s1, a_1 = u.dx, a_2 = u.x;
//   b_0 = (x.Dx + |A^T x|^2 - s2 |x|^2)/s1, b_1 = x.dD x + 2 (F^T x).(A^T x), b_2 = |x|^2;
// exact traces from tr5 (k_cv_trace_parts): T_2 = Tr P^{-1} = tr5[0] - tr5[1],
// T_0 = (n - s2 T_2)/s1, T_1 = tr5[2] - tr5[3] + 2 tr5[4].
// out: [0..2] gradient, [3..5] trace estimates, [6..8] quadratic terms,
// [9..11] coefficients c, [12..14] T.
__global__ void k_finalize_control_variate(int ncols, const double* __restrict__ uSX, const double* __restrict__ uX,
                                   const double* __restrict__ uDX, const double* __restrict__ xx,
                                   const double* __restrict__ xDx, const double* __restrict__ xdDx,
                                   const double* __restrict__ ax2, const double* __restrict__ fax,
                                   const double* __restrict__ tr5, double n, double s1, double s2, int mode,
                                   double* __restrict__ out) {
  const double T2 = tr5[0] - tr5[1];
  const double T[3] = {(n - s2 * T2) / s1, tr5[2] - tr5[3] + 2.0 * tr5[4], T2};
  const double t = (double)(ncols - 1);
  double ma[3] = {0, 0, 0}, mb[3] = {0, 0, 0};
  for (int c = 1; c < ncols; ++c) {
    const double a[3] = {(uSX[c] - s2 * uX[c]) / s1, uDX[c], uX[c]};
    const double b[3] = {(xDx[c] + ax2[c] - s2 * xx[c]) / s1, xdDx[c] + 2.0 * fax[c], xx[c]};
    for (int k = 0; k < 3; ++k) {
      ma[k] += a[k];
      mb[k] += b[k];
    }
  }
  for (int k = 0; k < 3; ++k) {
    ma[k] /= t;
    mb[k] /= t;
  }
  double num[3] = {0, 0, 0}, den[3] = {0, 0, 0}, bb[3] = {0, 0, 0};
  for (int c = 1; c < ncols; ++c) {
    const double a[3] = {(uSX[c] - s2 * uX[c]) / s1, uDX[c], uX[c]};
    const double b[3] = {(xDx[c] + ax2[c] - s2 * xx[c]) / s1, xdDx[c] + 2.0 * fax[c], xx[c]};
    for (int k = 0; k < 3; ++k) {
      const double bc = mode == FSA_CV_OPT ? b[k] - mb[k] : b[k];
      num[k] += (a[k] - ma[k]) * bc;
      den[k] += bc * bc;
      bb[k] += b[k] * b[k];
    }
  }
  const double qd[3] = {(uSX[0] - s2 * uX[0]) / s1, uDX[0], uX[0]};
  for (int k = 0; k < 3; ++k) {
    const double cc = mode == FSA_CV_ONE ? 1.0 : (den[k] > CV_DEGENERATE * bb[k] ? num[k] / den[k] : 0.0);
    const double est = ma[k] - cc * mb[k] + cc * T[k];
    out[k] = 0.5 * est - 0.5 * qd[k];
    out[3 + k] = est;
    out[6 + k] = qd[k];
    out[9 + k] = cc;
    out[12 + k] = T[k];
  }
}

// E[j] = sum over row j of the cross pattern of v^2 / D[col]: diag(S^T D_s^{-1} S)
// for the prediction points (rows of S^T)
__global__ void k_cross_diag_w(const int64_t* __restrict__ rp, const int* __restrict__ col, const double* __restrict__ v,
                               const double* __restrict__ D, int64_t np_, double* __restrict__ E) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= np_) return;
  double e = 0.0;
  for (int64_t k = rp[j]; k < rp[j + 1]; ++k) e += v[k] * v[k] / D[col[k]];
  E[j] = e;
}

// Algorithm 1's stochastic diagonal with D_s as control variate, in place:
// per prediction point j, a_i = z_i Zl_i, b_i = z_i Zv_i (i < s), c by mode,
// Zl_i <- Zl_i - c Zv_i + c E z_i, so that mean_i z_i Zl_i becomes
// mean(a) - c mean(b) + c E (z_i = +-1).
__global__ void k_pred_cv(int64_t np_, int s, const double* __restrict__ Z1, double* __restrict__ Zl,
                          const double* __restrict__ Zv, int ld, const double* __restrict__ E, int mode) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= np_) return;
  const double* z = Z1 + j * ld;
  double* zl = Zl + j * ld;
  const double* zv = Zv + j * ld;
  double ma = 0.0, mb = 0.0;
  for (int i = 0; i < s; ++i) {
    ma += z[i] * zl[i];
    mb += z[i] * zv[i];
  }
  ma /= s;
  mb /= s;
  double c = 1.0;
  if (mode != FSA_CV_ONE) {
    double num = 0.0, den = 0.0, bb = 0.0;
    for (int i = 0; i < s; ++i) {
      const double a = z[i] * zl[i], b = z[i] * zv[i];
      const double bc = mode == FSA_CV_OPT ? b - mb : b;
      num += (a - ma) * bc;
      den += bc * bc;
      bb += b * b;
    }
    c = den > CV_DEGENERATE * bb ? num / den : 0.0;
  }
  for (int i = 0; i < s; ++i) zl[i] = zl[i] - c * zv[i] + c * E[j] * z[i];
}

// ---- scores (Section 4) ----
// per-workgroup partial sums of the log-score, CRPS and squared-error terms,
// and a count of variances that are not finite and positive
__global__ __launch_bounds__(256) void k_score_parts(const double* __restrict__ y, const double* __restrict__ mu,
                                                     const double* __restrict__ var, int64_t n,
                                                     double* __restrict__ part, int* __restrict__ bad) {
  __shared__ double red[3][256];
  const int t = threadIdx.x;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  int nb = 0;
  for (int64_t i = blockIdx.x * 256 + t; i < n; i += (int64_t)gridDim.x * 256) {
    const double v = var[i];
    if (!(v > 0.0) || !isfinite(v)) {
      ++nb;
      continue;
    }
    const double sd = sqrt(v), e = y[i] - mu[i], z = e / sd;
    a0 += 0.5 * log(2.0 * M_PI * v) + 0.5 * z * z;
    const double phi = exp(-0.5 * z * z) / sqrt(2.0 * M_PI);
    const double Phi = 0.5 * erfc(-z / sqrt(2.0));
    a1 += sd * (-1.0 / sqrt(M_PI) + 2.0 * phi + z * (2.0 * Phi - 1.0));
    a2 += e * e;
  }
  if (nb) atomicAdd(bad, nb);
  red[0][t] = a0;
  red[1][t] = a1;
  red[2][t] = a2;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h)
      for (int j = 0; j < 3; ++j) red[j][t] += red[j][t + h];
    __syncthreads();
  }
  if (t < 3) part[(int64_t)blockIdx.x * 3 + t] = red[t][0];
}

// the scores from the partials (fixed order): mean log-score, mean CRPS, RMSE
__global__ void k_score_final(const double* __restrict__ part, int nparts, int64_t n, double* __restrict__ out) {
  const int j = threadIdx.x;
  if (j >= 3) return;
  double s = 0.0;
  for (int b = 0; b < nparts; ++b) s += part[(int64_t)b * 3 + j];
  s /= (double)n;
  out[j] = j == 2 ? sqrt(s) : s;
}

__global__ void k_add_cols(int ncols, const double* __restrict__ x, double* __restrict__ y) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < ncols) y[c] += x[c];
}

// The gradient's block X (n x 2 ld): columns [0, ld) hold x = [u | P^{-1} z]
// (u = U's column 0), columns [ld, 2 ld) hold U, both zero past ncols, so
// that one reduction over A (or F) serves x and u together.
__global__ void k_grad_block(int64_t n, int ncols, int64_t ld, const double* __restrict__ U, const void* Q0, int q0_f32,
                             double* __restrict__ X) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t p = e / (2 * ld);
  const int c = (int)(e % (2 * ld));
  if (p >= n) return;
  double v = 0.0;
  if (c < ld) {
    if (c < ncols) {
      const int64_t o = p * ld + c;
      v = c == 0 ? U[o] : (q0_f32 ? (double)((const float*)Q0)[o] : ((const double*)Q0)[o]);
    }
  } else if (c - ld < ncols) {
    v = U[p * ld + (c - ld)];
  }
  X[e] = v;
}

// The solver's small per-solve readback in one block: flags[2] (int), then
// rr[tp], bn2[tp] (double), then iters[tp] (int, if given).
__global__ void k_pack_status(const int* __restrict__ flags, const double* __restrict__ rr,
                              const double* __restrict__ bn2, const int* __restrict__ iters, int tp,
                              char* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  int* fo = reinterpret_cast<int*>(out);
  double* ro = reinterpret_cast<double*>(out + 8);
  double* bo = ro + tp;
  int* io = reinterpret_cast<int*>(bo + tp);
  if (i < 2) fo[i] = flags[i];
  if (i < tp) {
    ro[i] = rr[i];
    bo[i] = bn2[i];
    if (iters) io[i] = iters[i];
  }
}

__global__ void k_fill_weight_n(double* w, int ncols, double n) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < ncols) w[c] = n;
}

}  // namespace fsa

using namespace fsa;

struct fsa_ctx {
  bool mixed_stalled = false;  // the last float32 solve made no progress (see run_pcg)
  int64_t n = 0;
  int m = 0, mp = 0;
  int t = 0, tp = 0, ld = 0, ldw = 0;
  Theta th{};
  double gamma = 0;
  fsa_options opt{};
  hipStream_t st = nullptr;
  Grid grid;
  Csr csr;
  Buf<double> ind, y;
  Buf<double> Sm, Lm, Lminv, LminvT, C, LCinv, Cinv;
  Buf<double> A, vals, D, Dinv;
  Buf<float> Af, valsf;
  Buf<int64_t> tile_off;  // the float32 sparse part as MFMA-order tiles (mixed modes)
  Buf<float> tiles;
  Buf<unsigned> tile_mask;
  Buf<uint16_t> Abf;   // bfloat16 copy of A (MIXED_BF16A), point-major
  Buf<uint16_t> Abf8;  // the same, point-interleaved by 8 (bfloat16-MFMA residual pass)
  Buf<double> logdet_parts;  // [0] = 2 sum log diag L_C, [1] = sum log D
  Buf<int> info;
  // PCG / SLQ
  Buf<double> B, U, Emat;
  Buf<char> blockmem;
  Buf<double> colbuf;   // per-column scalars
  Buf<int> colint;
  Buf<double> hist;
  Buf<double> slq_scratch, results;
  const double* lanczos_weight = nullptr;  // quadrature weights of the last solve (in colbuf)
  // A second, non-blocking stream (default priority) for build and
  // quadrature work beside the main stream; ev_ready orders it behind st
  hipStream_t st2 = nullptr;
  hipEvent_t ev_ready = nullptr;
  // the quadrature of a solve also runs on st2, beside the gradient: ev_solve
  // marks the solve's end on st, ev_slq the quadrature's end on st2
  hipEvent_t ev_solve = nullptr, ev_slq = nullptr;
  bool slq_pending = false;
  // the two Cholesky factorizations of a build run on st2 beside other
  // build work: ev_fact marks the end of the one in flight
  hipEvent_t ev_fact = nullptr;
  bool lm_pending = false;  // Sigma_m -> L_m enqueued on st2
  // small device-to-host readbacks: a device staging block and its pinned
  // host mirror (one asynchronous copy each)
  Buf<char> dstage;
  char* hstage = nullptr;
  size_t hstage_bytes = 0;
  // the derivative factor and values (backward) depend on theta only: built
  // once per theta, after the solve, on st (beside the solve they only
  // shared the CUs with its kernels, each of which fills the chip)
  bool deriv_ready = false;
  bool timer_pending = false;  // the last solve's kernel events are not yet summed
  // gradient
  Buf<double> F, dvals, Xb, tmp, dSm, Ework;
  // control variate (options.control_variate): diagonal of the derivative values,
  // L_C^{-1} A and L_C^{-1} F by rows, and the five trace sums (per theta)
  Buf<double> dD, cvBA, cvBF, cvpart, cvtr;
  Scratch scr;
  KernelTimer timer;
  bool solved = false;
  double last_logdet_P = 0;
  // last statistics
  fsa_stats stats{};
};

static hipStream_t as_stream(void* p) { return reinterpret_cast<hipStream_t>(p); }

static double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

static fsa_status check_theta(const fsa_theta* th) {
  if (!th) return FSA_OK;
  if (th->cov != FSA_COV_EXPONENTIAL && th->cov != FSA_COV_MATERN32) {
    set_error("unknown covariance %d", th->cov);
    return FSA_ERR_INVALID_ARG;
  }
  if (!(th->sigma1_sq > 0) || !(th->rho > 0) || !(th->sigma_sq > 0) || !std::isfinite(th->sigma1_sq) ||
      !std::isfinite(th->rho) || !std::isfinite(th->sigma_sq)) {
    set_error("covariance parameters must be finite and > 0");
    return FSA_ERR_INVALID_ARG;
  }
  return FSA_OK;
}

// Sigma_m, L_m, whitened factor, residual values, D_s, FITC capacitance.
static fsa_status side_stream(fsa_ctx* c);

// Sigma_m and its Cholesky factor L_m on the side stream, behind everything
// enqueued on st so far (ev_fact marks the end): one workgroup's work that
// runs beside the grid and pattern build or the cross-covariance block.
static fsa_status launch_sigma_m(fsa_ctx* c) {
  FSA_TRY(side_stream(c));
  const int mp = c->mp;
  FSA_HIP(hipEventRecord(c->ev_ready, c->st));
  FSA_HIP(hipStreamWaitEvent(c->st2, c->ev_ready, 0));
  FSA_TRY(dense_sigma_m(c->ind.p, c->m, mp, c->th, c->opt.sigma_m_jitter, false, c->Sm.p, c->st2));
  FSA_HIP(hipMemcpyAsync(c->Lm.p, c->Sm.p, (size_t)mp * mp * sizeof(double), hipMemcpyDeviceToDevice, c->st2));
  FSA_TRY(dense_cholesky(c->Lm.p, mp, c->info.p, c->st2));
  // L_m^{-1} and its transpose for the whitening, still beside the main stream
  // (meaningless if the factorization failed; the build then stops on info)
  FSA_TRY(tri_inverse(c->Lm.p, c->Lminv.p, mp, c->st2));
  FSA_TRY(transpose_scale(c->Lminv.p, c->LminvT.p, mp, 1.0, c->st2));
  FSA_HIP(hipEventRecord(c->ev_fact, c->st2));
  c->lm_pending = true;
  return FSA_OK;
}

static fsa_status build_values(fsa_ctx* c) {
  c->deriv_ready = false;
  hipStream_t st = c->st;
  const int mp = c->mp;
  if (!c->lm_pending) FSA_TRY(launch_sigma_m(c));
  FSA_HIP(hipStreamWaitEvent(st, c->ev_fact, 0));
  c->lm_pending = false;
  int info = 0;
  FSA_HIP(hipMemcpyAsync(&info, c->info.p, sizeof(int), hipMemcpyDeviceToHost, st));
  FSA_HIP(hipStreamSynchronize(st));
  if (info) {
    set_error("Cholesky of Sigma_m failed at column %d (duplicate inducing points?)", info - 1);
    return FSA_ERR_NOT_SPD;
  }
  FSA_TRY(whiten(c->grid.xs.p, c->n, c->ind.p, c->m, mp, c->th, c->LminvT.p, c->A.p, st,
                 c->opt.precision == FSA_MIXED_FP32 ? c->Af.p : nullptr));  // the float32 copy in the same pass
  // MIXED_BF16A: the model takes the bfloat16-rounded factor from here on
  // (residual values, D_s, capacitance, probes, gradient and prediction), so
  // the PCG operator read in bfloat16 is the float64 operator of that model
  if (c->opt.precision == FSA_MIXED_BF16A) {
    FSA_TRY(to_bf16(c->A.p, c->Abf.p, c->A.p, c->n * (int64_t)mp, st));
    FSA_TRY(bf16_interleave8(c->Abf.p, c->n, mp, c->Abf8.p, st));
  }
  FSA_TRY(residual_values(c->grid, c->grid, c->csr, c->A.p, c->A.p, nullptr, nullptr, mp, c->th, c->gamma, true, false,
                          c->vals.p, c->D.p, st));
  FSA_TRY(reciprocal(c->D.p, c->Dinv.p, c->n, st));
  FSA_TRY(capacitance(c->A.p, c->D.p, c->n, mp, c->C.p, c->scr, st));
  // On the side stream: C -> L_C (in place), log det, L_C^{-1} and
  // C^{-1} = L_C^{-T} L_C^{-1}; meanwhile st converts the factor and values
  // and forms the probe block (none of which reads C).
  FSA_HIP(hipMemsetAsync(c->info.p, 0, 2 * sizeof(int), st));
  FSA_HIP(hipEventRecord(c->ev_ready, st));
  FSA_HIP(hipStreamWaitEvent(c->st2, c->ev_ready, 0));
  FSA_TRY(dense_cholesky(c->C.p, mp, c->info.p, c->st2));
  FSA_TRY(dense_logdet_chol(c->C.p, mp, c->logdet_parts.p, c->st2));
  FSA_TRY(tri_inverse(c->C.p, c->LCinv.p, mp, c->st2));
  FSA_TRY(dense_gemm(c->LCinv.p, true, c->LCinv.p, false, c->Cinv.p, mp, 1.0, c->st2));
  FSA_HIP(hipEventRecord(c->ev_fact, c->st2));
  {
    const int nb = 256;
    FSA_TRY(c->scr.dot1.alloc(nb));
    hipLaunchKernelGGL(k_sum_log_part, dim3(nb), dim3(256), 0, st, c->D.p, c->n, c->scr.dot1.p, c->info.p + 1);
    hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(256), 0, st, c->scr.dot1.p, nb, c->logdet_parts.p + 1);
  }
  if (c->opt.precision != FSA_FP64) {
    FSA_TRY(to_float(c->vals.p, c->valsf.p, c->csr.nnz, st));
    FSA_TRY(build_spmm_tiles(c->csr, c->grid, c->valsf.p, c->tile_off, c->tiles, c->tile_mask, st));
  }
  // probe block [y, z_1 .. z_t] (Section 3.3)
  FSA_TRY(c->B.alloc((size_t)c->n * c->ld));
  FSA_TRY(c->Emat.alloc((size_t)mp * c->ldw));
  FSA_TRY(make_probes(c->A.p, c->n, c->m, mp, c->D.p, c->y.p, c->grid.perm.p, c->opt.seed, c->t, c->B.p, c->ld,
                      c->Emat.p, st));
  FSA_HIP(hipStreamWaitEvent(st, c->ev_fact, 0));
  FSA_HIP(hipMemcpyAsync(&info, c->info.p, sizeof(int), hipMemcpyDeviceToHost, st));
  int bad = 0;
  FSA_HIP(hipMemcpyAsync(&bad, c->info.p + 1, sizeof(int), hipMemcpyDeviceToHost, st));
  double ld2[2];
  FSA_HIP(hipMemcpyAsync(ld2, c->logdet_parts.p, sizeof(ld2), hipMemcpyDeviceToHost, st));
  FSA_HIP(hipStreamSynchronize(st));
  if (info) {
    set_error("Cholesky of the FITC capacitance failed at column %d", info - 1);
    return FSA_ERR_NOT_SPD;
  }
  if (bad) {
    set_error("residual diagonal D_s has a non-positive or non-finite entry");
    return FSA_ERR_NOT_SPD;
  }
  c->last_logdet_P = ld2[0] + ld2[1];
  c->solved = false;
  return FSA_OK;
}

static fsa_status build_core(fsa_ctx* c, const double* locs, const double* y, const double* inducing) {
  hipStream_t st = c->st;
  const int64_t n = c->n;
  const int mp = c->mp;
  // input checks on the device
  FSA_TRY(c->info.alloc(4));
  FSA_HIP(hipMemsetAsync(c->info.p, 0, 4 * sizeof(int), st));
  hipLaunchKernelGGL(k_count_bad, dim3(ceil_div(2 * n, 256)), dim3(256), 0, st, locs, 2 * n, c->info.p + 2);
  hipLaunchKernelGGL(k_count_bad, dim3(ceil_div(n, 256)), dim3(256), 0, st, y, n, c->info.p + 2);
  hipLaunchKernelGGL(k_count_bad, dim3(ceil_div(2 * c->m, 256)), dim3(256), 0, st, inducing, (int64_t)2 * c->m,
                     c->info.p + 2);
  int bad = 0;
  FSA_HIP(hipMemcpyAsync(&bad, c->info.p + 2, sizeof(int), hipMemcpyDeviceToHost, st));
  FSA_HIP(hipStreamSynchronize(st));
  if (bad) {
    set_error("non-finite value in locations, responses or inducing points");
    return FSA_ERR_INVALID_ARG;
  }
  FSA_TRY(c->ind.alloc(2 * (size_t)mp));
  hipLaunchKernelGGL(k_pad_inducing, dim3(ceil_div(mp, 256)), dim3(256), 0, st, inducing, c->m, mp, c->ind.p);
  size_t mm = (size_t)mp * mp;
  FSA_TRY(c->Sm.alloc(mm));
  FSA_TRY(c->Lm.alloc(mm));
  FSA_TRY(c->Lminv.alloc(mm));
  FSA_TRY(c->LminvT.alloc(mm));
  FSA_TRY(launch_sigma_m(c));  // beside the grid and pattern build
  FSA_TRY(build_grid(c->grid, locs, n, c->gamma, st, nullptr, nullptr));
  FSA_TRY(build_pattern(c->grid, c->grid, c->csr, st));
  FSA_TRY(c->y.alloc(n));
  FSA_TRY(permute_rows(y, 1, c->y.p, 1, c->grid.perm.p, n, 1, st));
  FSA_TRY(c->C.alloc(mm));
  FSA_TRY(c->LCinv.alloc(mm));
  FSA_TRY(c->Cinv.alloc(mm));
  FSA_TRY(c->A.alloc((size_t)n * mp));
  FSA_TRY(c->vals.alloc(c->csr.nnz));
  FSA_TRY(c->D.alloc(n));
  FSA_TRY(c->Dinv.alloc(n));
  FSA_TRY(c->logdet_parts.alloc(2));
  if (c->opt.precision == FSA_MIXED_FP32) FSA_TRY(c->Af.alloc((size_t)n * mp));
  if (c->opt.precision == FSA_MIXED_BF16A) {
    FSA_TRY(c->Abf.alloc((size_t)n * mp));
    FSA_TRY(c->Abf8.alloc((size_t)ceil_div(n, 8) * 8 * mp));
  }
  if (c->opt.precision != FSA_FP64) FSA_TRY(c->valsf.alloc(c->csr.nnz));
  return build_values(c);
}

static fsa_status validate_build(int64_t n, int32_t d, const fsa_theta* theta, int32_t m, double gamma,
                                 const fsa_options* opt) {
  if (n < 2) { set_error("n must be >= 2 (got %lld)", (long long)n); return FSA_ERR_INVALID_ARG; }
  if (n > (int64_t)INT32_MAX / 2) { set_error("n too large"); return FSA_ERR_INVALID_ARG; }
  if (d != 2) { set_error("only d == 2 is supported (got %d)", d); return FSA_ERR_INVALID_ARG; }
  if (!theta) { set_error("theta is required"); return FSA_ERR_INVALID_ARG; }
  FSA_TRY(check_theta(theta));
  if (m < 1 || m > n || m > 512) { set_error("need 1 <= m <= min(n, 512) (got m=%d)", m); return FSA_ERR_INVALID_ARG; }
  if (!(gamma > 0) || !std::isfinite(gamma)) { set_error("taper range must be finite and > 0"); return FSA_ERR_INVALID_ARG; }
  if (opt) {
    if (opt->num_probes < 1 || opt->num_probes > 4096) { set_error("num_probes must be in [1, 4096]"); return FSA_ERR_INVALID_ARG; }
    if (opt->max_iter < 1 && opt->fixed_iter < 1) { set_error("max_iter must be >= 1"); return FSA_ERR_INVALID_ARG; }
    if (!(opt->cg_rel_tol >= 0)) { set_error("cg_rel_tol must be >= 0"); return FSA_ERR_INVALID_ARG; }
    if (opt->precision != FSA_FP64 && opt->precision != FSA_MIXED_FP32 && opt->precision != FSA_MIXED_BF16A) { set_error("unknown precision"); return FSA_ERR_INVALID_ARG; }
    if (opt->control_variate < FSA_CV_NONE || opt->control_variate > FSA_CV_OPT_PRINTED) { set_error("unknown control_variate"); return FSA_ERR_INVALID_ARG; }
    if (opt->fp32_products != FSA_F32P_SPLIT && opt->fp32_products != FSA_F32P_MFMA) { set_error("unknown fp32_products"); return FSA_ERR_INVALID_ARG; }
    if (!(opt->sigma_m_jitter >= 0)) { set_error("sigma_m_jitter must be >= 0"); return FSA_ERR_INVALID_ARG; }
  }
  return FSA_OK;
}

static fsa_status new_ctx(int64_t n, int32_t m, const fsa_theta* theta, double gamma, const fsa_options* opt,
                          fsa_ctx** out) {
  fsa_ctx* c = new fsa_ctx();
  c->n = n;
  c->m = m;
  c->mp = (int)round_up(m, 64);
  if (opt) c->opt = *opt;
  else fsa_default_options(&c->opt);
  if (c->opt.max_iter < 1) c->opt.max_iter = c->opt.fixed_iter;
  c->t = c->opt.num_probes;
  c->tp = c->t + 1;
  c->ld = (int)round_up(c->tp, 4);
  c->ldw = (int)round_up(c->tp, 64);
  c->th = Theta{theta->cov, theta->sigma1_sq, theta->rho, theta->sigma_sq};
  c->gamma = gamma;
  c->st = as_stream(c->opt.hip_stream);
  *out = c;
  return FSA_OK;
}

extern "C" {

void fsa_default_options(fsa_options* o) {
  memset(o, 0, sizeof(*o));
  o->num_probes = 50;
  o->seed = 0;
  o->cg_rel_tol = 1e-8;
  o->max_iter = 1000;
  o->fixed_iter = 0;
  o->precision = FSA_FP64;
  o->rr_period = 10;
  o->slq_weight_n = 0;
  o->sigma_m_jitter = 0.0;
  o->hip_stream = nullptr;
  o->fp32_products = FSA_F32P_SPLIT;
}

const char* fsa_last_error(void) { return get_error(); }

// Pinned host blocks for the small readbacks of a solve.  A context holds
// one while it lives and returns it at destroy, after draining its streams,
// so a block on the free list has no copy in flight.
static std::mutex g_pinned_mu;
static std::vector<std::pair<char*, size_t>> g_pinned;

static char* pinned_get(size_t bytes, size_t* got) {
  {
    std::lock_guard<std::mutex> lk(g_pinned_mu);
    for (size_t i = 0; i < g_pinned.size(); ++i)
      if (g_pinned[i].second >= bytes) {
        char* p = g_pinned[i].first;
        *got = g_pinned[i].second;
        g_pinned.erase(g_pinned.begin() + (ptrdiff_t)i);
        return p;
      }
  }
  const size_t sz = (bytes + 4095) & ~(size_t)4095;
  char* p = nullptr;
  if (hipHostMalloc((void**)&p, sz, hipHostMallocDefault) != hipSuccess) return nullptr;
  *got = sz;
  return p;
}

static void pinned_put(char* p, size_t bytes) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_pinned_mu);
  g_pinned.emplace_back(p, bytes);
}

static void pinned_trim() {
  std::lock_guard<std::mutex> lk(g_pinned_mu);
  for (auto& b : g_pinned) (void)hipHostFree(b.first);
  g_pinned.clear();
}

fsa_status fsa_scores(const double* y, const double* mean, const double* var, int64_t n, double* out) {
  if (!y || !mean || !var || !out) { set_error("null argument"); return FSA_ERR_INVALID_ARG; }
  if (n < 1) { set_error("n must be >= 1"); return FSA_ERR_INVALID_ARG; }
  hipStream_t st = nullptr;
  PoolStream ps(st);
  Buf<double> d;
  Buf<int> bad;
  const int G = (int)std::min<int64_t>(ceil_div(n, 256), 1024);
  FSA_TRY(d.alloc(3 * (size_t)n + 3 * (size_t)G + 3));
  FSA_TRY(bad.alloc(1));
  FSA_HIP(hipMemcpyAsync(d.p, y, n * sizeof(double), hipMemcpyHostToDevice, st));
  FSA_HIP(hipMemcpyAsync(d.p + n, mean, n * sizeof(double), hipMemcpyHostToDevice, st));
  FSA_HIP(hipMemcpyAsync(d.p + 2 * n, var, n * sizeof(double), hipMemcpyHostToDevice, st));
  FSA_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), st));
  double* part = d.p + 3 * n;
  hipLaunchKernelGGL(k_score_parts, dim3(G), dim3(256), 0, st, d.p, d.p + n, d.p + 2 * n, n, part, bad.p);
  hipLaunchKernelGGL(k_score_final, dim3(1), dim3(64), 0, st, part, G, n, part + 3 * (size_t)G);
  FSA_HIP(hipGetLastError());
  double res[3];
  int hb = 0;
  FSA_HIP(hipMemcpyAsync(res, part + 3 * (size_t)G, sizeof(res), hipMemcpyDeviceToHost, st));
  FSA_HIP(hipMemcpyAsync(&hb, bad.p, sizeof(int), hipMemcpyDeviceToHost, st));
  FSA_HIP(hipStreamSynchronize(st));
  if (hb) { set_error("%d predictive variances are not finite and positive", hb); return FSA_ERR_INVALID_ARG; }
  for (int j = 0; j < 3; ++j) out[j] = res[j];
  return FSA_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- scores without allocation
// fsa_scores_noalloc stages its inputs, its per-workgroup partials, its
// result and its counter in one file-scope device array.  In host code the
// array's name is only a host-side stand-in: the device address comes from
// hipGetSymbolAddress, taken once per device with that device current, and
// only that address is ever passed to kernels or copies.
namespace {
constexpr int64_t kScoresNoallocMaxN = int64_t(1) << 18;  // 262,144 points
constexpr int kScoresMaxGroups = 1024;                      // grid cap of k_score_parts
constexpr size_t kScoresPartOff = 3 * (size_t)kScoresNoallocMaxN;
constexpr size_t kScoresOutOff = kScoresPartOff + 3 * (size_t)kScoresMaxGroups;
constexpr size_t kScoresBadOff = kScoresOutOff + 4;          // an int in the slot of one double
constexpr size_t kScoresScratchDoubles = kScoresBadOff + 4;  // 6.32 MB in all
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) double scratch[kScoresScratchDoubles];

namespace {
std::mutex g_scratch_mu[kMaxDevices];  // one call at a time per device: the array is shared
double* g_scratch_ptr[kMaxDevices] = {};

__global__ void k_zero_int(int* p) {
  if (threadIdx.x == 0) *p = 0;
}
}  // namespace

extern "C" {

fsa_status fsa_scores_noalloc(const double* y, const double* mean, const double* var, int64_t n, double* out) {
  if (!y || !mean || !var || !out) { set_error("null argument"); return FSA_ERR_INVALID_ARG; }
  if (n < 1) { set_error("n must be >= 1"); return FSA_ERR_INVALID_ARG; }
  if (n > kScoresNoallocMaxN) {
    set_error("fsa_scores_noalloc: n = %lld exceeds its fixed scratch of %lld points (use fsa_scores)",
              (long long)n, (long long)kScoresNoallocMaxN);
    return FSA_ERR_INVALID_ARG;
  }
  int dev = 0;
  FSA_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) { set_error("device %d out of range", dev); return FSA_ERR_INVALID_ARG; }
  std::lock_guard<std::mutex> lk(g_scratch_mu[dev]);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    FSA_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  double* base = g_scratch_ptr[dev];
  double* dy = base;
  double* dmu = base + n;
  double* dvar = base + 2 * n;
  double* part = base + kScoresPartOff;
  double* res_d = base + kScoresOutOff;
  int* bad = reinterpret_cast<int*>(base + kScoresBadOff);
  hipStream_t st = nullptr;  // the default stream, as fsa_scores
  const int G = (int)std::min<int64_t>(ceil_div(n, 256), kScoresMaxGroups);
  FSA_HIP(hipMemcpyAsync(dy, y, n * sizeof(double), hipMemcpyHostToDevice, st));
  FSA_HIP(hipMemcpyAsync(dmu, mean, n * sizeof(double), hipMemcpyHostToDevice, st));
  FSA_HIP(hipMemcpyAsync(dvar, var, n * sizeof(double), hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, st, bad);  // the counter keeps the last call's value
  hipLaunchKernelGGL(k_score_parts, dim3(G), dim3(256), 0, st, dy, dmu, dvar, n, part, bad);
  hipLaunchKernelGGL(k_score_final, dim3(1), dim3(64), 0, st, part, G, n, res_d);
  FSA_HIP(hipGetLastError());
  double res[3];
  int hb = 0;
  FSA_HIP(hipMemcpyAsync(res, res_d, sizeof(res), hipMemcpyDeviceToHost, st));
  FSA_HIP(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, st));
  FSA_HIP(hipStreamSynchronize(st));
  if (hb) { set_error("%d predictive variances are not finite and positive", hb); return FSA_ERR_INVALID_ARG; }
  for (int j = 0; j < 3; ++j) out[j] = res[j];
  return FSA_OK;
}

fsa_status fsa_set_allocator(fsa_alloc_fn alloc, fsa_release_fn release, void* user) {
  if ((alloc == nullptr) != (release == nullptr)) {
    set_error("fsa_set_allocator needs both callbacks or neither");
    return FSA_ERR_INVALID_ARG;
  }
  std::lock_guard<std::mutex> lk(g_pool_mu);
  g_user = UserAlloc{alloc, release, user};
  return FSA_OK;
}

void fsa_pool_trim(void) {
  pool_trim();
  pinned_trim();
}

fsa_status fsa_build_dev(const double* locs, int64_t n, int32_t d, const double* y, const fsa_theta* theta,
                         const double* inducing, int32_t m, double gamma, const fsa_options* opt, fsa_ctx** out) {
  if (!out || !locs || !y || !inducing) { set_error("null argument"); return FSA_ERR_INVALID_ARG; }
  *out = nullptr;
  FSA_TRY(validate_build(n, d, theta, m, gamma, opt));
  PoolStream ps(opt ? as_stream(opt->hip_stream) : nullptr);
  fsa_ctx* c = nullptr;
  FSA_TRY(new_ctx(n, m, theta, gamma, opt, &c));
  fsa_status s = build_core(c, locs, y, inducing);
  if (s != FSA_OK) {
    fsa_destroy(c);
    return s;
  }
  *out = c;
  return FSA_OK;
}

fsa_status fsa_build(const double* locs, int64_t n, int32_t d, const double* y, const fsa_theta* theta,
                     const double* inducing, int32_t m, double gamma, const fsa_options* opt, fsa_ctx** out) {
  if (!out || !locs || !y || !inducing) { set_error("null argument"); return FSA_ERR_INVALID_ARG; }
  *out = nullptr;
  FSA_TRY(validate_build(n, d, theta, m, gamma, opt));
  hipStream_t st = opt ? as_stream(opt->hip_stream) : nullptr;
  PoolStream ps(st);
  Buf<double> dl, dy, di;
  FSA_TRY(dl.alloc(2 * (size_t)n));
  FSA_TRY(dy.alloc(n));
  FSA_TRY(di.alloc(2 * (size_t)m));
  FSA_HIP(hipMemcpyAsync(dl.p, locs, 2 * n * sizeof(double), hipMemcpyHostToDevice, st));
  FSA_HIP(hipMemcpyAsync(dy.p, y, n * sizeof(double), hipMemcpyHostToDevice, st));
  FSA_HIP(hipMemcpyAsync(di.p, inducing, 2 * (size_t)m * sizeof(double), hipMemcpyHostToDevice, st));
  fsa_status s = fsa_build_dev(dl.p, n, d, dy.p, theta, di.p, m, gamma, opt, out);
  (void)hipStreamSynchronize(st);
  return s;
}

void fsa_destroy(fsa_ctx* c) {
  if (!c) return;
  PoolStream ps(c->st);
  (void)hipStreamSynchronize(c->st);
  if (c->st2) {
    (void)hipStreamSynchronize(c->st2);
    (void)hipEventDestroy(c->ev_ready);
    (void)hipEventDestroy(c->ev_solve);
    (void)hipEventDestroy(c->ev_slq);
    (void)hipEventDestroy(c->ev_fact);
    (void)hipStreamDestroy(c->st2);
  }
  pinned_put(c->hstage, c->hstage_bytes);
  delete c;  // Buf members return their blocks to the pool
  pool_flush();  // and blocks of a registered allocator go back to it now
}

int64_t fsa_nnz(const fsa_ctx* c) { return c ? c->csr.nnz : -1; }

}  // extern "C"

// ---------------------------------------------------------------- PCG driver
// The side stream (non-blocking, default priority) and its events.
static fsa_status side_stream(fsa_ctx* c) {
  if (!c->st2) {
    FSA_HIP(hipStreamCreateWithFlags(&c->st2, hipStreamNonBlocking));
    FSA_HIP(hipEventCreateWithFlags(&c->ev_ready, hipEventDisableTiming));
    FSA_HIP(hipEventCreateWithFlags(&c->ev_solve, hipEventDisableTiming));
    FSA_HIP(hipEventCreateWithFlags(&c->ev_slq, hipEventDisableTiming));
    FSA_HIP(hipEventCreateWithFlags(&c->ev_fact, hipEventDisableTiming));
  }
  return FSA_OK;
}

// Make the last solve's quadrature (results: slq, fin) visible to work on st.
static fsa_status join_slq(fsa_ctx* c) {
  if (c->slq_pending) {
    FSA_HIP(hipStreamWaitEvent(c->st, c->ev_slq, 0));
    c->slq_pending = false;
  }
  return FSA_OK;
}

// Stage the solver status (flags, rr, bn2 and, if given, iters) for the host:
// packed on the device and copied to pinned host memory in one asynchronous
// copy on st; the caller synchronises st before reading it.
struct HostStatus {
  const int* flags;
  const double* rr;
  const double* bn;
  const int* iters;
};
static fsa_status stage_status(fsa_ctx* c, const int* flags, const double* rr, const double* bn2, const int* iters,
                               int tp, HostStatus* hs) {
  const size_t bytes = 8 + 16 * (size_t)tp + 4 * (size_t)tp;
  if (c->hstage_bytes < bytes) {
    FSA_HIP(hipStreamSynchronize(c->st));  // no copy into the old block is in flight
    pinned_put(c->hstage, c->hstage_bytes);
    c->hstage = pinned_get(bytes, &c->hstage_bytes);
    if (!c->hstage) {
      c->hstage_bytes = 0;
      set_error("hipHostMalloc of %zu bytes failed", bytes);
      return FSA_ERR_OOM;
    }
  }
  FSA_TRY(c->dstage.alloc(bytes));
  hipLaunchKernelGGL(k_pack_status, dim3(ceil_div(std::max(tp, 2), 256)), dim3(256), 0, c->st, flags, rr, bn2, iters,
                     tp, c->dstage.p);
  FSA_HIP(hipGetLastError());
  FSA_HIP(hipMemcpyAsync(c->hstage, c->dstage.p, bytes, hipMemcpyDeviceToHost, c->st));
  hs->flags = reinterpret_cast<const int*>(c->hstage);
  hs->rr = reinterpret_cast<const double*>(c->hstage + 8);
  hs->bn = hs->rr + tp;
  hs->iters = iters ? reinterpret_cast<const int*>(hs->bn + tp) : nullptr;
  return FSA_OK;
}

// One PCG iteration replayed from a HIP graph: captured on first use, then
// launched once per iteration.  The iteration's launches and arguments are
// the same every iteration (its state lives in device memory), and its
// scratch is sized by the eager first iteration, so the capture allocates
// nothing and holds no memset.
template <typename T>
struct IterGraph {
  hipStream_t st = nullptr;
  hipGraph_t g = nullptr;
  hipGraphExec_t x = nullptr;
  explicit IterGraph(hipStream_t s) : st(s) {}
  IterGraph(const IterGraph&) = delete;
  IterGraph& operator=(const IterGraph&) = delete;
  ~IterGraph() {
    if (!x && !g) return;
    (void)hipStreamSynchronize(st);
    if (x) (void)hipGraphExecDestroy(x);
    if (g) (void)hipGraphDestroy(g);
  }
  fsa_status run(PcgBlock<T>& b, const OpDesc<T>& op, double tol, int fixed, Scratch& s) {
    if (!x) {
      FSA_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      const fsa_status cs = pcg_iter<T>(b, op, tol, fixed, s, st);
      const hipError_t ce = hipStreamEndCapture(st, &g);
      if (cs != FSA_OK) return cs;
      FSA_HIP(ce);
      FSA_HIP(hipGraphInstantiate(&x, g, nullptr, nullptr, 0));
    }
    FSA_HIP(hipGraphLaunch(x, st));
    return FSA_OK;
  }
};

template <typename T>
static fsa_status run_pcg(fsa_ctx* c, double* ms_pcg) {
  hipStream_t st = c->st;
  const int64_t n = c->n;
  const int tp = c->tp, ld = c->ld, ldw = c->ldw, mp = c->mp;
  const int max_iter = c->opt.fixed_iter > 0 ? c->opt.fixed_iter : c->opt.max_iter;
  size_t blk = (size_t)n * ld;
  const int nblk = sizeof(T) == 4 ? 7 : 6;
  FSA_TRY(c->blockmem.alloc(nblk * blk * sizeof(T)));
  T* base = reinterpret_cast<T*>(c->blockmem.p);
  PcgBlock<T> b;
  b.n = n;
  b.ncols = tp;
  b.ld = ld;
  b.ldw = ldw;
  b.max_iter = max_iter;
  b.R = base;
  b.H = base + blk;
  b.V = base + 2 * blk;
  b.P = base + 3 * blk;
  b.Tt = base + 4 * blk;
  b.Q0 = base + 5 * blk;
  if constexpr (sizeof(T) == 4) b.U32 = base + 6 * blk;
  FSA_TRY(c->U.alloc(blk));
  b.U = c->U.p;
  FSA_TRY(c->colbuf.alloc(8 * (size_t)ldw));
  b.rz = c->colbuf.p;
  b.rz0 = b.rz + ldw;
  b.alpha = b.rz + 2 * ldw;
  b.beta = b.rz + 3 * ldw;
  b.rr = b.rz + 4 * ldw;
  b.bn2 = b.rz + 5 * ldw;
  FSA_TRY(c->colint.alloc(2 * (size_t)ldw + 4));
  b.active = c->colint.p;
  b.iters = c->colint.p + ldw;
  b.flags = c->colint.p + 2 * ldw;
  FSA_TRY(c->hist.alloc(2 * (size_t)max_iter * tp));
  b.alpha_hist = c->hist.p;
  b.beta_hist = c->hist.p + (size_t)max_iter * tp;
  FSA_TRY(c->scr.w.alloc((size_t)mp * ldw * 2));
  Buf<T> gbuf;
  FSA_TRY(gbuf.alloc((size_t)mp * ldw));
  b.g = gbuf.p;
  OpDesc<T> op;
  op.grid = &c->grid;
  op.S = &c->csr;
  op.D = c->D.p;
  op.Dinv = c->Dinv.p;
  op.kdim = mp;
  op.Cinv = c->Cinv.p;
  OpDesc<double> op64;
  op64.grid = &c->grid;
  op64.S = &c->csr;
  op64.val = c->vals.p;
  op64.D = c->D.p;
  op64.Dinv = c->Dinv.p;
  op64.A = c->A.p;
  op64.kdim = mp;
  op64.Cinv = c->Cinv.p;
  if constexpr (sizeof(T) == 8) {
    op.val = reinterpret_cast<const T*>(c->vals.p);
    op.A = reinterpret_cast<const T*>(c->A.p);
  } else {
    op.val = reinterpret_cast<const T*>(c->valsf.p);
    op.tile_off = c->tile_off.p;
    op.tiles = c->tiles.p;
    op.tile_mask = c->tile_mask.p;
    op.A = reinterpret_cast<const T*>(c->Af.p);  // null in MIXED_BF16A
    op.Abf = c->Abf.p;                            // null unless MIXED_BF16A
    op.Abf8 = c->Abf8.p;
    op.split = c->opt.precision == FSA_MIXED_FP32 && c->opt.fp32_products == FSA_F32P_SPLIT;
  }
  const double tol = c->opt.cg_rel_tol;
  const int fixed = c->opt.fixed_iter > 0 ? 1 : 0;
  FSA_TRY(join_slq(c));  // the last solve's quadrature reads the buffers reused here
  c->timer.mask = (unsigned)c->opt.profile & ((1u << KernelTimer::NCLS) - 1u);
  c->timer.on = c->timer.mask != 0;
  c->timer.reset();
  c->timer_pending = false;
  b.timer = c->timer.on ? &c->timer : nullptr;
  double t0 = now_ms();
  FSA_TRY(pcg_init<T>(b, op, c->B.p, tol, c->scr, st));
  int flags[2] = {0, 0};
  int it = 0;
  // Convergence is read back at checkpoints only (each one drains the
  // stream).  The next checkpoint comes where the slowest column's
  // recurrence residual, at the log-linear rate seen since the last one,
  // reaches the tolerance (between 1 and 8 iterations on): few drains while
  // far from convergence, and no idle iterations once every column is done.
  int next_check = 4, prev_it = 0;
  double prev_res = -1.0, rate = 0.0;
  // Float32 stall: the slowest column's residual (the float64 one right after
  // a replacement) has not halved over three replacement periods.  Where
  // |A A^T| exceeds D by ~10^5 the float32 Woodbury application cancels
  // most of its digits, and the float32 iteration can stall or break down.
  double stall_best = INFINITY;
  int stall_it = 0;
  const int stall_span = 3 * std::max(c->opt.rr_period, 10);
  c->mixed_stalled = false;
  IterGraph<T> ig(st);
  const bool use_graph = c->opt.graph != 0 && !c->timer.on && st != nullptr;  // the null stream cannot be captured
  for (it = 0; it < max_iter; ++it) {
    if (use_graph && it > 0) FSA_TRY(ig.run(b, op, tol, fixed, c->scr));
    else FSA_TRY(pcg_iter<T>(b, op, tol, fixed, c->scr, st));
    bool replaced = false;
    if constexpr (sizeof(T) == 4) {
      if (c->opt.rr_period > 0 && (it + 1) % c->opt.rr_period == 0 && it + 1 < max_iter) {
        FSA_TRY(pcg_replace_residual_f32(reinterpret_cast<PcgBlock<float>&>(b), op64,
                                         reinterpret_cast<const OpDesc<float>&>(op), c->B.p, c->scr, st));
        replaced = true;
      }
    }
    if (!fixed && (it + 1 == next_check || it + 1 == max_iter)) {
      HostStatus hs;
      FSA_TRY(stage_status(c, b.flags, b.rr, b.bn2, nullptr, tp, &hs));
      FSA_HIP(hipStreamSynchronize(st));
      if (hs.flags[1]) break;
      if (hs.flags[0] == 0) {
        // Mixed precision: the float32 recurrence residual has drifted from
        // b - Sigma~ u since the last float64 replacement, so the stop is
        // confirmed on the float64 residual; columns still above the
        // tolerance continue (same Krylov sequence, replaced residual).
        bool done = true;
        if constexpr (sizeof(T) == 4) {
          auto& bf = reinterpret_cast<PcgBlock<float>&>(b);
          if (!replaced)
            FSA_TRY(pcg_replace_residual_f32(bf, op64, reinterpret_cast<const OpDesc<float>&>(op), c->B.p, c->scr,
                                             st));
          FSA_TRY(pcg_recheck_true_residual(bf, tol, c->scr, st));
          FSA_TRY(stage_status(c, b.flags, b.rr, b.bn2, nullptr, tp, &hs));
          FSA_HIP(hipStreamSynchronize(st));
          done = hs.flags[0] == 0;
        }
        if (done) {
          ++it;
          break;
        }
        // the columns above the tolerance continue from the float64
        // residual; the next check comes where the slowest of them is
        // predicted to reach it at the last rate seen
        double worst = 0.0;
        for (int k = 0; k < tp; ++k)
          if (hs.bn[k] > 0.0) worst = std::max(worst, std::sqrt(std::max(hs.rr[k], 0.0) / hs.bn[k]));
        int step = 2;
        if (rate < 0.0 && worst > tol && tol > 0.0)
          step = (int)std::min(8.0, std::max(1.0, std::ceil(std::log(tol / worst) / rate)));
        prev_res = worst;
        prev_it = it + 1;
        next_check = it + 1 + step;
        continue;
      }
      double worst = 0.0;
      for (int k = 0; k < tp; ++k)
        if (hs.bn[k] > 0.0) worst = std::max(worst, std::sqrt(std::max(hs.rr[k], 0.0) / hs.bn[k]));
      if constexpr (sizeof(T) == 4) {
        if (worst < 0.5 * stall_best) {
          stall_best = worst;
          stall_it = it + 1;
        } else if (it + 1 - stall_it >= stall_span) {
          c->mixed_stalled = true;
          ++it;
          break;
        }
      }
      int step = 4;
      if (prev_res > 0.0 && worst > 0.0 && worst < prev_res && tol > 0.0) {
        rate = std::log(worst / prev_res) / (double)(it + 1 - prev_it);  // < 0
        const double remain = std::log(tol / worst) / rate;
        step = (int)std::min(8.0, std::max(1.0, std::floor(remain)));
      }
      prev_res = worst;
      prev_it = it + 1;
      next_check = it + 1 + step;
    }
  }
  if constexpr (sizeof(T) == 4) FSA_TRY(pcg_fold_u(reinterpret_cast<PcgBlock<float>&>(b), st));
  // The quadratic term and the gradient block go in behind the solve on st,
  // the quadrature and the likelihood on the side stream, where they run
  // beside the gradient; all of it is enqueued before the host-side
  // bookkeeping below (on a breakdown it runs on meaningless coefficients
  // and is discarded).
  FSA_TRY(c->slq_scratch.alloc((size_t)tp * 3 * max_iter));
  FSA_TRY(c->results.alloc(4 * (size_t)ldw + 16));
  double* slq = c->results.p;
  double* quad = c->results.p + ldw;
  double* fin = c->results.p + 2 * ldw;
  const double* weight = b.rz0;
  if (c->opt.slq_weight_n) {
    double* wn = c->colbuf.p + 6 * ldw;  // spare per-column slot
    hipLaunchKernelGGL(k_fill_weight_n, dim3(ceil_div(tp, 64)), dim3(64), 0, st, wn, tp, (double)n);
    weight = wn;
  }
  c->lanczos_weight = weight;
  FSA_TRY((coldot<double, double>(c->B.p, c->U.p, n, ld, 1, quad, c->scr, st)));
  FSA_TRY(side_stream(c));
  FSA_HIP(hipEventRecord(c->ev_solve, st));
  FSA_HIP(hipStreamWaitEvent(c->st2, c->ev_solve, 0));
  FSA_TRY(slq_terms(b.alpha_hist, b.beta_hist, b.iters, tp, 1, weight, slq, c->slq_scratch.p, max_iter, c->st2));
  hipLaunchKernelGGL(k_finalize_nll, dim3(1), dim3(1), 0, c->st2, slq, tp, c->logdet_parts.p, quad, n, fin);
  FSA_HIP(hipGetLastError());
  FSA_HIP(hipEventRecord(c->ev_slq, c->st2));
  c->slq_pending = true;
  // keep Q0 (P^{-1} z) for the gradient in float64
  FSA_TRY(c->Xb.alloc(2 * blk));
  hipLaunchKernelGGL(k_grad_block, dim3(ceil_div((int64_t)n * 2 * ld, 256)), dim3(256), 0, st, n, tp, (int64_t)ld,
                     c->U.p, (const void*)b.Q0, sizeof(T) == 4 ? 1 : 0, c->Xb.p);
  FSA_HIP(hipGetLastError());
  // iteration statistics (staged behind the work above)
  HostStatus hs;
  FSA_TRY(stage_status(c, b.flags, b.rr, b.bn2, b.iters, tp, &hs));
  FSA_HIP(hipStreamSynchronize(st));
  const int* iters = hs.iters;
  const double *rr = hs.rr, *bn = hs.bn;
  flags[0] = hs.flags[0];
  flags[1] = hs.flags[1];
  *ms_pcg = now_ms() - t0;
  c->timer_pending = c->timer.on;  // collected while the device runs the next work
  int imin = 1 << 30, imax = 0;
  int64_t tot = 0;
  for (int k = 0; k < tp; ++k) {
    imin = std::min(imin, iters[k]);
    imax = std::max(imax, iters[k]);
    tot += iters[k];
  }
  c->stats.iters_min = imin;
  c->stats.iters_max = imax;
  c->stats.probe_iters = tot;
  double rmax = 0.0;
  for (int k = 0; k < tp; ++k)
    if (bn[k] > 0.0) rmax = std::max(rmax, std::sqrt(std::max(rr[k], 0.0) / bn[k]));
  c->stats.rel_res_max = rmax;
  if (flags[1]) {
    c->lanczos_weight = nullptr;
    set_error("CG breakdown (h^T Sigma h <= 0 or non-finite)");
    return FSA_ERR_BREAKDOWN;
  }
  c->solved = true;
  if (c->mixed_stalled) {
    set_error("float32 PCG stalled at relative residual %.3g after %d iterations", rmax, imax);
    return FSA_ERR_NOT_CONVERGED;
  }
  if (!fixed && flags[0] > 0) {
    set_error("PCG did not converge in %d iterations (%d columns active)", max_iter, flags[0]);
    return FSA_ERR_NOT_CONVERGED;
  }
  return FSA_OK;
}

// Y = Sigma~_dagger X (float64), X/Y n x ld blocks in sorted order.
static fsa_status apply_sigma(fsa_ctx* c, const double* X, double* Y, int ncols, int ldx) {
  hipStream_t st = c->st;
  int ldw = (int)round_up(ncols, 64);
  FSA_TRY(c->scr.w.alloc((size_t)c->mp * ldw * 2));
  FSA_TRY(c->tmp.alloc((size_t)c->n * ldx));
  FSA_TRY(spmm<double>(c->csr, c->grid, c->grid, c->vals.p, X, ldx, ncols, Y, ldx, false, st));
  FSA_TRY(lowrank_reduce<double>(c->A.p, c->n, c->mp, X, ldx, ncols, nullptr, c->scr, c->scr.w.p, ldw, st));
  FSA_TRY(lowrank_expand<double>(c->A.p, nullptr, c->n, c->mp, c->scr.w.p, ldw, ncols, c->tmp.p, ldx, st));
  FSA_TRY(axpy_block(c->tmp.p, 1.0, Y, ldx, c->n, ncols, st));
  return FSA_OK;
}

// F = L^{-1} dSigma_mn - Phi(E) A (whitened rho-derivative factor) and the derivative values.
// K = Phi(E): the lower triangle of the symmetric E with half its diagonal
// (row-major mp x mp), so that K + K^T = E.
__global__ void k_lower_half(const double* __restrict__ E, int mp, double* __restrict__ K) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)mp * mp) return;
  const int r = (int)(e / mp), col = (int)(e % mp);
  K[e] = col < r ? E[e] : (col == r ? 0.5 * E[e] : 0.0);
}

static fsa_status build_derivative(fsa_ctx* c, hipStream_t st) {
  const int mp = c->mp;
  size_t mm = (size_t)mp * mp;
  FSA_TRY(c->dSm.alloc(mm));
  FSA_TRY(c->Ework.alloc(2 * mm));
  FSA_TRY(dense_sigma_m(c->ind.p, c->m, mp, c->th, 0.0, true, c->dSm.p, st));
  double* T1 = c->Ework.p;
  double* E = c->Ework.p + mm;
  FSA_TRY(dense_gemm(c->Lminv.p, false, c->dSm.p, false, T1, mp, 1.0, st));   // L^{-1} dSm
  FSA_TRY(dense_gemm(T1, false, c->Lminv.p, true, E, mp, 1.0, st));           // E = L^{-1} dSm L^{-T}
  // F = L^{-1} dSigma_mn - Phi(E) A (point-major n x mp), the derivative of
  // the whitened factor A = L^{-1} Sigma_mn (dL = L Phi(E)); every use of F
  // goes through A F^T + F A^T = dSigma_nm Sigma_m^{-1} Sigma_mn + ... (or
  // Tr(C^{-1} A^T D^{-1} F)), which any F = L^{-1} dSigma_mn - K A with
  // K + K^T = E gives alike; the triangular K costs n mp^2 flop where the
  // symmetric K = E/2 costs 2 n mp^2 (taken here in 128-row blocks: 1.25 n mp^2)
  hipLaunchKernelGGL(k_lower_half, dim3(ceil_div((int64_t)mp * mp, 256)), dim3(256), 0, st, E, mp, T1);
  FSA_HIP(hipGetLastError());
  FSA_TRY(transpose_scale(T1, E, mp, -1.0, st));  // -Phi(E)^T (E is not needed past here)
  FSA_TRY(c->F.alloc((size_t)c->n * mp));
  // MIXED_FP32: F and the derivative values only enter the gradient (its 1e-4
  // bar), so both run in float32 arithmetic from the float32 copy of A, at
  // twice the float64 MFMA rate (F is kept in float64 too, widened, for the
  // gradient's float64 passes)
  const bool f32 = c->opt.precision == FSA_MIXED_FP32;
  Buf<float> Ff;
  if (f32) FSA_TRY(Ff.alloc((size_t)c->n * mp));
  FSA_TRY(derivative_factor(c->grid.xs.p, c->n, c->ind.p, c->m, mp, c->th, c->LminvT.p, c->A.p, E, c->F.p, st,
                            f32 ? c->Af.p : nullptr, f32 ? Ff.p : nullptr));
  FSA_TRY(c->dvals.alloc(c->csr.nnz));
  if (f32)
    FSA_TRY(derivative_values_f32(c->grid, c->csr, c->Af.p, Ff.p, mp, c->th, c->gamma, c->dvals.p, st));
  else
    FSA_TRY(residual_values(c->grid, c->grid, c->csr, c->A.p, c->A.p, c->F.p, c->F.p, mp, c->th, c->gamma, true,
                            true, c->dvals.p, nullptr, st));
  if (c->opt.control_variate != FSA_CV_NONE) {
    // Tr(P^{-1} dP/dtheta) by Woodbury (App. E, F): with C = L_C L_C^T,
    // Tr P^{-1} = sum 1/D - sum |L_C^{-1} A_p|^2 / D^2, Tr(P^{-1} dD) likewise
    // weighted by dD, and Tr(P^{-1}(F A^T + A F^T)) = 2 Tr(C^{-1} A^T D^{-1} F)
    const int64_t n = c->n;
    FSA_TRY(c->dD.alloc(n));
    hipLaunchKernelGGL(k_csr_diag, dim3(ceil_div(n, 256)), dim3(256), 0, st, c->csr.row_ptr.p, c->csr.col.p,
                       c->dvals.p, n, c->dD.p);
    // rows of L_C^{-1} A and L_C^{-1} F: A L_C^{-T} and F L_C^{-T}
    FSA_TRY(c->cvBA.alloc((size_t)n * mp));
    FSA_TRY(c->cvBF.alloc((size_t)n * mp));
    FSA_TRY(transpose_scale(c->LCinv.p, T1, mp, 1.0, st));  // L_C^{-T}
    FSA_TRY(rows_times_lower_t(c->A.p, n, mp, T1, c->cvBA.p, st));
    FSA_TRY(rows_times_lower_t(c->F.p, n, mp, T1, c->cvBF.p, st));
    const int G = 1024;
    FSA_TRY(c->cvpart.alloc((size_t)G * 5));
    FSA_TRY(c->cvtr.alloc(8));
    hipLaunchKernelGGL(k_cv_trace_parts, dim3(G), dim3(256), 0, st, c->cvBA.p, c->cvBF.p, c->D.p, c->dD.p, n, mp,
                       c->cvpart.p);
    hipLaunchKernelGGL(k_cv_trace_final, dim3(1), dim3(64), 0, st, c->cvpart.p, G, c->cvtr.p);
    FSA_HIP(hipGetLastError());
  }
  return FSA_OK;
}

// Y = dSigma~/drho X = dS X + F^T (A X) + A^T (F X)
static fsa_status apply_drho(fsa_ctx* c, const double* X, double* Y, int ncols, int ldx) {
  hipStream_t st = c->st;
  const int mp = c->mp;
  int ldw = (int)round_up(ncols, 64);
  FSA_TRY(c->scr.w.alloc((size_t)mp * ldw * 2));
  FSA_TRY(c->tmp.alloc((size_t)c->n * ldx));
  FSA_TRY(spmm<double>(c->csr, c->grid, c->grid, c->dvals.p, X, ldx, ncols, Y, ldx, false, st));
  FSA_TRY(lowrank_reduce<double>(c->A.p, c->n, mp, X, ldx, ncols, nullptr, c->scr, c->scr.w.p, ldw, st));
  FSA_TRY(lowrank_reduce<double>(c->F.p, c->n, mp, X, ldx, ncols, nullptr, c->scr, c->scr.w.p + (size_t)mp * ldw, ldw,
                                 st));
  FSA_TRY(lowrank_expand<double>(c->F.p, c->A.p, c->n, 2 * mp, c->scr.w.p, ldw, ncols, c->tmp.p, ldx, st));
  FSA_TRY(axpy_block(c->tmp.p, 1.0, Y, ldx, c->n, ncols, st));
  return FSA_OK;
}

// Make the derivative factor and values available to work on st.
static fsa_status ensure_derivative(fsa_ctx* c) {
  if (!c->deriv_ready) {
    FSA_TRY(build_derivative(c, c->st));
    c->deriv_ready = true;
  }
  return FSA_OK;
}

// Sum the solve's per-kernel event times into the stats (the events have
// completed once the solve was read back).
static void collect_timer(fsa_ctx* c) {
  if (!c->timer_pending) return;
  c->timer.collect(c->stats.kernel_ms, c->stats.kernel_launches);
  c->timer_pending = false;
}

static fsa_status run_gradient(fsa_ctx* c, double* grad, double* parts6, double* grad_dev = nullptr) {
  hipStream_t st = c->st;
  const int64_t n = c->n;
  const int tp = c->tp, ld = c->ld;
  FSA_TRY(ensure_derivative(c));
  // Only the column dots u.(Sigma~ x), u.x and u.(dSigma~/drho x) are
  // needed (u = U, x = Xb, column by column): the sparse parts come from the
  // sparse product's epilogue without storing it, the low-rank parts from
  // m-space reductions of x and u (no n x t expansion).
  const int mp = c->mp;
  // x and u side by side in one n x 2 ld block (k_grad_block): one reduction
  // over A and one over F give A^T x, A^T u, F^T x, F^T u (two launches, not
  // four; the float64 reduction's cost is its MFMA work per 64-column block,
  // which does not change)
  const int ldx = 2 * ld;
  const double* X = c->Xb.p;
  const double* Ux = c->Xb.p + ld;
  const int ldw = (int)round_up(ld + tp, 64);
  Buf<double> dd, wm;
  // dd: [0] u.Sx [1] u.x [2] u.dx [3] low-rank u.Sx [4] low-rank u.dx [5] |A^T x|^2
  // [6] (F^T x).(A^T x) [7] |x|^2 [8] x.Dx [9] x.dDx (tp each), then the results
  FSA_TRY(dd.alloc(10 * (size_t)tp + 15));
  FSA_TRY(wm.alloc(2 * (size_t)mp * ldw));
  double* w_a = wm.p;                     // columns [0, tp): A^T x; [ld, ld + tp): A^T u
  double* w_f = wm.p + (size_t)mp * ldw;  // the same with F
  FSA_TRY(spmm_dot<double>(c->csr, c->grid, c->vals.p, X, Ux, ldx, tp, dd.p, c->scr, st));
  FSA_TRY((coldot<double, double>(Ux, X, n, ldx, tp, dd.p + tp, c->scr, st)));
  FSA_TRY(spmm_dot<double>(c->csr, c->grid, c->dvals.p, X, Ux, ldx, tp, dd.p + 2 * tp, c->scr, st));
  FSA_TRY(lowrank_reduce<double>(c->A.p, n, mp, X, ldx, ld + tp, nullptr, c->scr, w_a, ldw, st));
  FSA_TRY(lowrank_reduce<double>(c->F.p, n, mp, X, ldx, ld + tp, nullptr, c->scr, w_f, ldw, st));
  hipLaunchKernelGGL(k_grad_mdots, dim3(tp), dim3(256), 0, st, w_a, w_f, w_a + ld, w_f + ld, mp, ldw, dd.p + 3 * tp,
                     dd.p + 4 * tp, dd.p + 5 * tp, dd.p + 6 * tp);
  hipLaunchKernelGGL(k_add_cols, dim3(ceil_div(tp, 64)), dim3(64), 0, st, tp, dd.p + 3 * tp, dd.p);
  hipLaunchKernelGGL(k_add_cols, dim3(ceil_div(tp, 64)), dim3(64), 0, st, tp, dd.p + 4 * tp, dd.p + 2 * tp);
  double* res = dd.p + 10 * (size_t)tp;
  const int cv = c->opt.control_variate;
  if (cv == FSA_CV_NONE) {
    hipLaunchKernelGGL(k_finalize_grad, dim3(1), dim3(1), 0, st, tp, dd.p, dd.p + tp, dd.p + 2 * tp, c->th.s1,
                       c->th.s2, res);
  } else {
    // |x|^2, x.Dx, x.dDx per column of the probe block
    const int ncb = (int)ceil_div(tp, 64);
    const int ldp = ncb * 64;
    const int64_t g = std::min<int64_t>(std::max<int64_t>(ceil_div(n, 64), 1), 1024);
    Buf<double> xp;
    FSA_TRY(xp.alloc(3 * (size_t)g * ldp));
    hipLaunchKernelGGL(k_cv_xdots, dim3(g, ncb), dim3(256), 0, st, X, n, ldx, tp, c->D.p, c->dD.p, xp.p, ldp);
    for (int j = 0; j < 3; ++j)
      FSA_TRY(colsum(xp.p + (size_t)j * g * ldp, (int)g, ldp, tp, dd.p + (7 + j) * (size_t)tp, st));
    hipLaunchKernelGGL(k_finalize_control_variate, dim3(1), dim3(1), 0, st, tp, dd.p, dd.p + tp, dd.p + 2 * tp, dd.p + 7 * tp,
                       dd.p + 8 * tp, dd.p + 9 * tp, dd.p + 5 * tp, dd.p + 6 * tp, c->cvtr.p, (double)n, c->th.s1,
                       c->th.s2, cv, res);
  }
  FSA_HIP(hipGetLastError());
  if (grad_dev) FSA_HIP(hipMemcpyAsync(grad_dev, res, 3 * sizeof(double), hipMemcpyDeviceToDevice, st));
  collect_timer(c);  // host work while the gradient kernels run
  double g9[15];
  FSA_HIP(hipMemcpyAsync(g9, res, (cv == FSA_CV_NONE ? 9 : 15) * sizeof(double), hipMemcpyDeviceToHost, st));
  FSA_HIP(hipStreamSynchronize(st));
  for (int k = 0; k < 3; ++k) grad[k] = g9[k];
  if (parts6)
    for (int k = 0; k < 6; ++k) parts6[k] = g9[3 + k];
  for (int k = 0; k < 3; ++k) {
    c->stats.cv_c[k] = cv == FSA_CV_NONE ? 0.0 : g9[9 + k];
    c->stats.trace_P[k] = cv == FSA_CV_NONE ? 0.0 : g9[12 + k];
  }
  return FSA_OK;
}

// ---------------------------------------------------------------- sparse block PCG
// Sigma~_s W = B with the diagonal preconditioner D_s (Section 3.3), every
// column independent; W (float64, n x ld) receives the solutions.
template <typename T>
static fsa_status run_sparse_pcg(fsa_ctx* c, const double* B, int ncols, int ld, double* W, int* iters_max) {
  hipStream_t st = c->st;
  const int64_t n = c->n;
  const int max_iter = c->opt.fixed_iter > 0 ? c->opt.fixed_iter : c->opt.max_iter;
  const int ldw = (int)round_up(ncols, 64);
  size_t blk = (size_t)n * ld;
  Buf<T> mem;
  FSA_TRY(mem.alloc((sizeof(T) == 4 ? 7 : 6) * blk));
  PcgBlock<T> b;
  b.n = n;
  b.ncols = ncols;
  b.ld = ld;
  b.ldw = ldw;
  b.max_iter = max_iter;
  b.R = mem.p;
  b.H = mem.p + blk;
  b.V = mem.p + 2 * blk;
  b.P = mem.p + 3 * blk;
  b.Tt = mem.p + 4 * blk;
  b.Q0 = mem.p + 5 * blk;
  if constexpr (sizeof(T) == 4) b.U32 = mem.p + 6 * blk;
  b.U = W;
  Buf<double> colb, hist;
  Buf<int> coli;
  FSA_TRY(colb.alloc(8 * (size_t)ldw));
  FSA_TRY(coli.alloc(2 * (size_t)ldw + 4));
  FSA_TRY(hist.alloc(2 * (size_t)max_iter * ncols));
  b.rz = colb.p;
  b.rz0 = colb.p + ldw;
  b.alpha = colb.p + 2 * ldw;
  b.beta = colb.p + 3 * ldw;
  b.rr = colb.p + 4 * ldw;
  b.bn2 = colb.p + 5 * ldw;
  b.active = coli.p;
  b.iters = coli.p + ldw;
  b.flags = coli.p + 2 * ldw;
  b.alpha_hist = hist.p;
  b.beta_hist = hist.p + (size_t)max_iter * ncols;
  OpDesc<T> op;
  op.grid = &c->grid;
  op.S = &c->csr;
  op.D = c->D.p;
  op.Dinv = c->Dinv.p;
  op.kdim = 0;
  if constexpr (sizeof(T) == 8) {
    op.val = reinterpret_cast<const T*>(c->vals.p);
  } else {
    op.val = reinterpret_cast<const T*>(c->valsf.p);
    op.tile_off = c->tile_off.p;
    op.tiles = c->tiles.p;
    op.tile_mask = c->tile_mask.p;
  }
  OpDesc<double> op64;
  op64.grid = &c->grid;
  op64.S = &c->csr;
  op64.val = c->vals.p;
  op64.D = c->D.p;
  op64.Dinv = c->Dinv.p;
  op64.kdim = 0;
  const double tol = c->opt.cg_rel_tol;
  const int fixed = c->opt.fixed_iter > 0 ? 1 : 0;
  FSA_TRY(pcg_init<T>(b, op, B, tol, c->scr, st));
  int flags[2] = {0, 0};
  IterGraph<T> ig(st);
  for (int it = 0; it < max_iter; ++it) {
    if (c->opt.graph != 0 && st != nullptr && it > 0) FSA_TRY(ig.run(b, op, tol, fixed, c->scr));
    else FSA_TRY(pcg_iter<T>(b, op, tol, fixed, c->scr, st));
    if constexpr (sizeof(T) == 4) {
      if (c->opt.rr_period > 0 && (it + 1) % c->opt.rr_period == 0 && it + 1 < max_iter)
        FSA_TRY(pcg_replace_residual_f32(reinterpret_cast<PcgBlock<float>&>(b), op64,
                                         reinterpret_cast<const OpDesc<float>&>(op), B, c->scr, st));
    }
    if (!fixed && ((it + 1) % 4 == 0 || it + 1 == max_iter)) {
      FSA_HIP(hipMemcpyAsync(flags, b.flags, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
      FSA_HIP(hipStreamSynchronize(st));
      if (flags[1]) break;
      if (flags[0] == 0) {
        // mixed precision: stop only on the float64 residual (as in run_pcg)
        if constexpr (sizeof(T) == 4) {
          auto& bf = reinterpret_cast<PcgBlock<float>&>(b);
          if (!(c->opt.rr_period > 0 && (it + 1) % c->opt.rr_period == 0 && it + 1 < max_iter))
            FSA_TRY(pcg_replace_residual_f32(bf, op64, reinterpret_cast<const OpDesc<float>&>(op), B, c->scr, st));
          FSA_TRY(pcg_recheck_true_residual(bf, tol, c->scr, st));
          FSA_HIP(hipMemcpyAsync(flags, b.flags, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
          FSA_HIP(hipStreamSynchronize(st));
          if (flags[0] == 0) break;
        } else {
          break;
        }
      }
    }
  }
  if constexpr (sizeof(T) == 4) FSA_TRY(pcg_fold_u(reinterpret_cast<PcgBlock<float>&>(b), st));
  FSA_HIP(hipMemcpyAsync(flags, b.flags, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
  std::vector<int> its(ncols);
  FSA_HIP(hipMemcpyAsync(its.data(), b.iters, ncols * sizeof(int), hipMemcpyDeviceToHost, st));
  FSA_HIP(hipStreamSynchronize(st));
  int mx = 0;
  for (int k = 0; k < ncols; ++k) mx = std::max(mx, its[k]);
  if (iters_max) *iters_max = mx;
  if (flags[1]) {
    set_error("CG breakdown in a Sigma~_s solve");
    return FSA_ERR_BREAKDOWN;
  }
  if (!fixed && flags[0] > 0) {
    set_error("Sigma~_s PCG did not converge in %d iterations (%d columns active)", max_iter, flags[0]);
    return FSA_ERR_NOT_CONVERGED;
  }
  return FSA_OK;
}

// Algorithm 1 with the whitened factors: A = L_m^{-1} Sigma_mn (training),
// A_p = L_m^{-1} Sigma_{m n_p}, V~ = Sigma~_s^{-1} A^T and
// M~ = I + A V~ (= L_m^{-1} M L_m^{-T}), so that
//   D1 = diag(A_p^T A_p) - diag(A_p^T M~^{-1} A_p),
//   D2 = diag(S_p^T V~ M~^{-1} A_p),  D3 = diag(S_p^T V~ M~^{-1} V~^T S_p),
// S_p = Sigma^s_{n n_p}; D_l by simulation with Rademacher z (Algorithm 1).
static fsa_status predict_core(fsa_ctx* c, const double* pred_locs_h, int64_t n_p, int s, double* var_out,
                               double* mean_out, fsa_stats* st_out, double* parts_out) {
  double t0 = now_ms();
  hipStream_t st = c->st;
  const int64_t n = c->n;
  const int mp = c->mp;
  Buf<double> pl;
  FSA_TRY(pl.alloc(2 * (size_t)n_p));
  FSA_HIP(hipMemcpyAsync(pl.p, pred_locs_h, 2 * n_p * sizeof(double), hipMemcpyHostToDevice, st));
  Buf<int> bad;
  FSA_TRY(bad.alloc(1));
  FSA_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), st));
  hipLaunchKernelGGL(k_count_bad, dim3(ceil_div(2 * n_p, 256)), dim3(256), 0, st, pl.p, 2 * n_p, bad.p);
  int hbad = 0;
  FSA_HIP(hipMemcpyAsync(&hbad, bad.p, sizeof(int), hipMemcpyDeviceToHost, st));
  FSA_HIP(hipStreamSynchronize(st));
  if (hbad) { set_error("non-finite prediction location"); return FSA_ERR_INVALID_ARG; }
  Grid pg;
  FSA_TRY(build_grid(pg, pl.p, n_p, c->gamma, st, nullptr, &c->grid));
  Csr cPT, cTP;
  FSA_TRY(build_pattern(pg, c->grid, cPT, st));
  FSA_TRY(build_pattern(c->grid, pg, cTP, st));
  // whitened prediction factor and the cross residual values
  Buf<double> Ap, vPT, vTP;
  FSA_TRY(Ap.alloc((size_t)n_p * mp));
  FSA_TRY(vPT.alloc(cPT.nnz));
  FSA_TRY(vTP.alloc(cTP.nnz));
  FSA_TRY(whiten(pg.xs.p, n_p, c->ind.p, c->m, mp, c->th, c->LminvT.p, Ap.p, st));
  if (c->opt.precision == FSA_MIXED_BF16A) FSA_TRY(to_bf16(Ap.p, nullptr, Ap.p, n_p * (int64_t)mp, st));
  FSA_TRY(residual_values(pg, c->grid, cPT, Ap.p, c->A.p, nullptr, nullptr, mp, c->th, c->gamma, false, false, vPT.p,
                          nullptr, st));
  FSA_TRY(residual_values(c->grid, pg, cTP, c->A.p, Ap.p, nullptr, nullptr, mp, c->th, c->gamma, false, false, vTP.p,
                          nullptr, st));
  // right-hand sides [A^T | S_p z^(1)]
  const int ncols = mp + s;
  const int ld = (int)round_up(ncols, 4);
  const int lds = (int)round_up(s, 4);
  Buf<double> B, W, Z1;
  FSA_TRY(B.alloc((size_t)n * ld));
  FSA_TRY(W.alloc((size_t)n * ld));
  FSA_TRY(Z1.alloc((size_t)n_p * lds));
  FSA_HIP(hipMemsetAsync(Z1.p, 0, (size_t)n_p * lds * sizeof(double), st));
  FSA_TRY((copy_block<double, double>(c->A.p, mp, B.p, ld, n, mp, st)));
  FSA_TRY(pred_rademacher(pg.perm.p, n_p, s, c->opt.seed, Z1.p, lds, st));
  FSA_TRY(spmm<double>(cTP, c->grid, pg, vTP.p, Z1.p, lds, s, B.p + mp, ld, false, st));
  int its = 0;
  double t1 = now_ms();
  fsa_status ps = c->opt.precision != FSA_FP64 ? run_sparse_pcg<float>(c, B.p, ncols, ld, W.p, &its)
                                                      : run_sparse_pcg<double>(c, B.p, ncols, ld, W.p, &its);
  if (ps != FSA_OK && ps != FSA_ERR_NOT_CONVERGED) return ps;
  double t2 = now_ms();
  // M~ = I + A V~ and its Cholesky factor
  size_t mm = (size_t)mp * mp;
  Buf<double> Mt, LMi, G;
  FSA_TRY(Mt.alloc(mm));
  FSA_TRY(LMi.alloc(mm));
  FSA_TRY(G.alloc(mm));
  FSA_TRY(c->scr.w.alloc(mm));
  FSA_TRY(lowrank_reduce<double>(c->A.p, n, mp, W.p, ld, mp, nullptr, c->scr, Mt.p, mp, st));
  FSA_TRY(add_identity(Mt.p, mp, st));
  FSA_TRY(symmetrize(Mt.p, mp, st));
  FSA_TRY(dense_cholesky(Mt.p, mp, c->info.p, st));
  int info = 0;
  FSA_HIP(hipMemcpyAsync(&info, c->info.p, sizeof(int), hipMemcpyDeviceToHost, st));
  FSA_HIP(hipStreamSynchronize(st));
  if (info) { set_error("Cholesky of I + A Sigma~_s^{-1} A^T failed at column %d", info - 1); return FSA_ERR_NOT_SPD; }
  FSA_TRY(tri_inverse(Mt.p, LMi.p, mp, st));
  FSA_TRY(transpose_scale(LMi.p, G.p, mp, 1.0, st));
  // Y = A_p L_M^{-T}, Z2 = (S_p^T V~) L_M^{-T}, Z_l = S_p^T W_l
  Buf<double> Y, Y2, Z2, Zl;
  FSA_TRY(Y.alloc((size_t)n_p * mp));
  FSA_TRY(Y2.alloc((size_t)n_p * mp));
  FSA_TRY(Z2.alloc((size_t)n_p * mp));
  FSA_TRY(Zl.alloc((size_t)n_p * lds));
  FSA_HIP(hipMemsetAsync(Zl.p, 0, (size_t)n_p * lds * sizeof(double), st));
  FSA_TRY(lowrank_expand<double>(Ap.p, nullptr, n_p, mp, G.p, mp, mp, Y.p, mp, st));
  FSA_TRY(spmm<double>(cPT, pg, c->grid, vPT.p, W.p, ld, mp, Y2.p, mp, false, st));
  FSA_TRY(lowrank_expand<double>(Y2.p, nullptr, n_p, mp, G.p, mp, mp, Z2.p, mp, st));
  FSA_TRY(spmm<double>(cPT, pg, c->grid, vPT.p, W.p + mp, ld, s, Zl.p, lds, false, st));
  if (c->opt.control_variate != FSA_CV_NONE) {
    // D_s as control variate (App. E): Zv = S^T D_s^{-1} S z and diag(S^T D_s^{-1} S)
    Buf<double> Xd, Zv, Ev;
    FSA_TRY(Xd.alloc((size_t)n * lds));
    FSA_TRY(Zv.alloc((size_t)n_p * lds));
    FSA_TRY(Ev.alloc(n_p));
    FSA_HIP(hipMemsetAsync(Xd.p, 0, (size_t)n * lds * sizeof(double), st));
    FSA_TRY((copy_block<double, double>(B.p + mp, ld, Xd.p, lds, n, s, st)));
    FSA_TRY(scale_rows(Xd.p, lds, c->D.p, n, s, 1, st));
    FSA_HIP(hipMemsetAsync(Zv.p, 0, (size_t)n_p * lds * sizeof(double), st));
    FSA_TRY(spmm<double>(cPT, pg, c->grid, vPT.p, Xd.p, lds, s, Zv.p, lds, false, st));
    hipLaunchKernelGGL(k_cross_diag_w, dim3(ceil_div(n_p, 256)), dim3(256), 0, st, cPT.row_ptr.p, cPT.col.p, vPT.p,
                       c->D.p, n_p, Ev.p);
    hipLaunchKernelGGL(k_pred_cv, dim3(ceil_div(n_p, 256)), dim3(256), 0, st, n_p, s, Z1.p, Zl.p, Zv.p, lds, Ev.p,
                       c->opt.control_variate);
    FSA_HIP(hipGetLastError());
  }
  Buf<double> vdev;
  FSA_TRY(vdev.alloc(n_p));
  Buf<double> pdev;
  if (parts_out) FSA_TRY(pdev.alloc(4 * (size_t)n_p));
  FSA_TRY(pred_combine(n_p, mp, Ap.p, Y.p, Z2.p, Z1.p, Zl.p, lds, s, c->th.s1, c->th.s2, pg.perm.p, vdev.p,
                       parts_out ? pdev.p : nullptr, st));
  FSA_HIP(hipMemcpyAsync(var_out, vdev.p, n_p * sizeof(double), hipMemcpyDeviceToHost, st));
  if (parts_out) FSA_HIP(hipMemcpyAsync(parts_out, pdev.p, 4 * n_p * sizeof(double), hipMemcpyDeviceToHost, st));
  if (mean_out) {
    // mu = A_p (A u) + S_p^T u, u = Sigma~_dagger^{-1} y from the last likelihood solve
    Buf<double> wu, su, mdev;
    FSA_TRY(wu.alloc((size_t)mp * 64));
    FSA_TRY(su.alloc((size_t)n_p * 4));
    FSA_TRY(mdev.alloc(n_p));
    FSA_TRY(lowrank_reduce<double>(c->A.p, n, mp, c->U.p, c->ld, 1, nullptr, c->scr, wu.p, 64, st));
    FSA_TRY(spmm<double>(cPT, pg, c->grid, vPT.p, c->U.p, c->ld, 1, su.p, 1, false, st));
    Buf<double> wcol;
    FSA_TRY(wcol.alloc(mp));
    FSA_TRY((copy_block<double, double>(wu.p, 64, wcol.p, 1, mp, 1, st)));
    FSA_TRY(pred_mean(n_p, mp, Ap.p, wcol.p, su.p, pg.perm.p, mdev.p, st));
    FSA_HIP(hipMemcpyAsync(mean_out, mdev.p, n_p * sizeof(double), hipMemcpyDeviceToHost, st));
    FSA_HIP(hipStreamSynchronize(st));
  }
  FSA_HIP(hipStreamSynchronize(st));
  double t3 = now_ms();
  if (st_out) {
    memset(st_out, 0, sizeof(*st_out));
    st_out->iters_max = its;
    st_out->ms_build = t1 - t0;
    st_out->ms_pcg = t2 - t1;
    st_out->ms_backward = t3 - t2;
    st_out->ms_total = t3 - t0;
    st_out->nnz = cPT.nnz;
  }
  return ps;
}

// The likelihood call behind fsa_nll_grad and fsa_nll_grad_dev: host
// outputs (nll, grad) and/or device outputs (nll_dev, grad_dev), each may be
// null except one of nll / nll_dev; a gradient is computed if grad or
// grad_dev is given.
static fsa_status nll_grad_core(fsa_ctx* c, const fsa_theta* theta, double* nll, double* grad, double* nll_dev,
                                double* grad_dev, fsa_stats* st_out) {
  PoolStream ps(c->st);
  double t0 = now_ms();
  hipStream_t st = c->st;
  memset(&c->stats, 0, sizeof(c->stats));
  if (theta) {
    FSA_TRY(check_theta(theta));
    Theta nt{theta->cov, theta->sigma1_sq, theta->rho, theta->sigma_sq};
    if (nt.kind != c->th.kind || nt.s1 != c->th.s1 || nt.rho != c->th.rho || nt.s2 != c->th.s2) {
      c->th = nt;
      FSA_TRY(build_values(c));
    }
  }
  double t_build = now_ms();
  const bool want_grad = grad || grad_dev;
  double ms_pcg = 0;
  fsa_status s;
  if (c->opt.precision != FSA_FP64) {
    s = run_pcg<float>(c, &ms_pcg);
    if (s == FSA_ERR_BREAKDOWN || (s == FSA_ERR_NOT_CONVERGED && c->mixed_stalled)) {
      // the float32 iteration cannot resolve this system: the solve is
      // repeated in float64 on the float64 operator the replacements use
      const int64_t wasted = c->stats.probe_iters;
      double ms64 = 0;
      s = run_pcg<double>(c, &ms64);
      ms_pcg += ms64;
      c->stats.fp64_fallback = 1;
      c->stats.fallback_probe_iters = wasted;
    }
  } else {
    s = run_pcg<double>(c, &ms_pcg);
  }
  if (s != FSA_OK && s != FSA_ERR_NOT_CONVERGED) {
    FSA_TRY(join_slq(c));
    collect_timer(c);
    if (nll) *nll = INFINITY;
    if (nll_dev) {
      const double inf = INFINITY;
      FSA_HIP(hipMemcpyAsync(nll_dev, &inf, sizeof(double), hipMemcpyHostToDevice, st));
      FSA_HIP(hipStreamSynchronize(st));
    }
    return s;
  }
  double t_b0 = now_ms();
  if (want_grad) {
    double parts6[6];
    double gh[3];
    fsa_status gs = run_gradient(c, grad ? grad : gh, parts6, grad_dev);
    if (gs != FSA_OK) {
      FSA_TRY(join_slq(c));
      return gs;
    }
    for (int k = 0; k < 3; ++k) {
      c->stats.grad_trace[k] = parts6[k];
      c->stats.grad_quad[k] = parts6[3 + k];
    }
  }
  // the likelihood from the side stream (the quadrature ran beside the gradient)
  FSA_TRY(join_slq(c));
  double fin[3];
  if (nll_dev)
    FSA_HIP(hipMemcpyAsync(nll_dev, c->results.p + 2 * c->ldw + 2, sizeof(double), hipMemcpyDeviceToDevice, st));
  FSA_HIP(hipMemcpyAsync(fin, c->results.p + 2 * c->ldw, sizeof(fin), hipMemcpyDeviceToHost, st));
  FSA_HIP(hipStreamSynchronize(st));
  if (nll) *nll = fin[2];
  collect_timer(c);
  double t1 = now_ms();
  c->stats.logdet = fin[0];
  c->stats.quad = fin[1];
  c->stats.logdet_P = c->last_logdet_P;
  c->stats.ms_build = t_build - t0;
  c->stats.ms_pcg = ms_pcg;
  c->stats.ms_backward = want_grad ? t1 - t_b0 : 0.0;
  c->stats.ms_total = t1 - t0;
  c->stats.nnz = c->csr.nnz;
  if (st_out) *st_out = c->stats;
  return s;
}

extern "C" {

fsa_status fsa_nll_grad(fsa_ctx* c, const fsa_theta* theta, double* nll, double* grad, fsa_stats* st_out) {
  if (!c || !nll) { set_error("null argument"); return FSA_ERR_INVALID_ARG; }
  return nll_grad_core(c, theta, nll, grad, nullptr, nullptr, st_out);
}

fsa_status fsa_nll_grad_dev(fsa_ctx* c, const fsa_theta* theta, double* nll_dev, double* grad_dev,
                            fsa_stats* st_out) {
  if (!c || !nll_dev) { set_error("null argument"); return FSA_ERR_INVALID_ARG; }
  return nll_grad_core(c, theta, nullptr, nullptr, nll_dev, grad_dev, st_out);
}

fsa_status fsa_grad(fsa_ctx* c, double* grad, fsa_stats* st_out) {
  if (!c || !grad) { set_error("null argument"); return FSA_ERR_INVALID_ARG; }
  PoolStream ps(c->st);
  if (!c->solved) { set_error("fsa_grad needs a preceding fsa_nll_grad on this context"); return FSA_ERR_INVALID_ARG; }
  double t0 = now_ms();
  double parts6[6];
  FSA_TRY(run_gradient(c, grad, parts6));
  for (int k = 0; k < 3; ++k) {
    c->stats.grad_trace[k] = parts6[k];
    c->stats.grad_quad[k] = parts6[3 + k];
  }
  c->stats.ms_backward = now_ms() - t0;
  if (st_out) *st_out = c->stats;
  return FSA_OK;
}

fsa_status fsa_export_csr(fsa_ctx* c, int64_t* row_ptr, int32_t* col_idx, double* vals) {
  if (!c || !row_ptr || !col_idx) { set_error("null argument"); return FSA_ERR_INVALID_ARG; }
  PoolStream ps(c->st);
  return export_csr(c->csr, c->grid, c->grid, c->vals.p, row_ptr, col_idx, vals, c->st);
}

fsa_status fsa_export_diag(fsa_ctx* c, double* D, double* logdet_P) {
  if (!c) { set_error("null argument"); return FSA_ERR_INVALID_ARG; }
  PoolStream ps(c->st);
  if (D) {
    Buf<double> tmp;
    FSA_TRY(tmp.alloc(c->n));
    FSA_TRY(permute_rows(c->D.p, 1, tmp.p, 1, c->grid.iperm.p, c->n, 1, c->st));
    FSA_HIP(hipMemcpyAsync(D, tmp.p, c->n * sizeof(double), hipMemcpyDeviceToHost, c->st));
    FSA_HIP(hipStreamSynchronize(c->st));
  }
  if (logdet_P) *logdet_P = c->last_logdet_P;
  return FSA_OK;
}

fsa_status fsa_export_lanczos(fsa_ctx* c, int32_t* iters, double* alpha, double* beta, double* weight,
                              double* slq) {
  if (!c) { set_error("null argument"); return FSA_ERR_INVALID_ARG; }
  PoolStream ps(c->st);
  if (!c->solved || !c->lanczos_weight) { set_error("no likelihood solve to export"); return FSA_ERR_INVALID_ARG; }
  FSA_TRY(join_slq(c));
  const int tp = c->tp;
  const int L = c->opt.fixed_iter > 0 ? c->opt.fixed_iter : c->opt.max_iter;
  hipStream_t st = c->st;
  if (iters) FSA_HIP(hipMemcpyAsync(iters, c->colint.p + c->ldw, tp * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  if (alpha) FSA_HIP(hipMemcpyAsync(alpha, c->hist.p, (size_t)L * tp * sizeof(double), hipMemcpyDeviceToHost, st));
  if (beta)
    FSA_HIP(hipMemcpyAsync(beta, c->hist.p + (size_t)L * tp, (size_t)L * tp * sizeof(double), hipMemcpyDeviceToHost,
                           st));
  if (weight) FSA_HIP(hipMemcpyAsync(weight, c->lanczos_weight, tp * sizeof(double), hipMemcpyDeviceToHost, st));
  if (slq) FSA_HIP(hipMemcpyAsync(slq, c->results.p, tp * sizeof(double), hipMemcpyDeviceToHost, st));
  FSA_HIP(hipStreamSynchronize(st));
  if (slq) slq[0] = 0.0;
  return FSA_OK;
}

fsa_status fsa_export_solution(fsa_ctx* c, double* U) {
  if (!c || !U) { set_error("null argument"); return FSA_ERR_INVALID_ARG; }
  PoolStream ps(c->st);
  if (!c->solved) { set_error("no likelihood solve to export"); return FSA_ERR_INVALID_ARG; }
  FSA_TRY(join_slq(c));
  const int64_t n = c->n;
  const int tp = c->tp;
  Buf<double> tmp;
  FSA_TRY(tmp.alloc((size_t)n * tp));
  FSA_TRY(permute_rows(c->U.p, c->ld, tmp.p, tp, c->grid.iperm.p, n, tp, c->st));
  FSA_HIP(hipMemcpyAsync(U, tmp.p, (size_t)n * tp * sizeof(double), hipMemcpyDeviceToHost, c->st));
  FSA_HIP(hipStreamSynchronize(c->st));
  return FSA_OK;
}

fsa_status fsa_apply(fsa_ctx* c, int32_t which, const double* X, double* Y, int32_t ncols) {
  if (!c || !Y || ncols < 1 || (which != FSA_OP_PROBES && !X)) { set_error("bad argument"); return FSA_ERR_INVALID_ARG; }
  PoolStream ps(c->st);
  hipStream_t st = c->st;
  const int64_t n = c->n;
  int ld = (int)round_up(ncols, 4);
  Buf<double> xh, xs, ys;
  FSA_TRY(xh.alloc((size_t)n * ncols));
  FSA_TRY(xs.alloc((size_t)n * ld));
  FSA_TRY(ys.alloc((size_t)n * ld));
  if (which != FSA_OP_PROBES) {
    FSA_HIP(hipMemcpyAsync(xh.p, X, (size_t)n * ncols * sizeof(double), hipMemcpyHostToDevice, st));
    FSA_TRY(permute_rows(xh.p, ncols, xs.p, ld, c->grid.perm.p, n, ncols, st));
  }
  int ldw = (int)round_up(ncols + 1, 64);
  switch (which) {
    case FSA_OP_SIGMA_S:
      FSA_TRY(spmm<double>(c->csr, c->grid, c->grid, c->vals.p, xs.p, ld, ncols, ys.p, ld, false, st));
      break;
    case FSA_OP_SIGMA_DAGGER:
      FSA_TRY(apply_sigma(c, xs.p, ys.p, ncols, ld));
      break;
    case FSA_OP_D_SIGMA1:
      FSA_TRY(apply_sigma(c, xs.p, ys.p, ncols, ld));
      FSA_TRY(axpy_block(xs.p, -c->th.s2, ys.p, ld, n, ncols, st));
      FSA_TRY(scal_block(ys.p, ld, n, ncols, 1.0 / c->th.s1, st));
      break;
    case FSA_OP_D_RHO:
      FSA_TRY(ensure_derivative(c));
      FSA_TRY(apply_drho(c, xs.p, ys.p, ncols, ld));
      break;
    case FSA_OP_P_INV: {
      int ldw2 = (int)round_up(ncols, 64);
      FSA_TRY(c->scr.w.alloc((size_t)c->mp * ldw2 * 2));
      Buf<double> g, tt;
      FSA_TRY(g.alloc((size_t)c->mp * ldw2));
      FSA_TRY(tt.alloc((size_t)n * ld));
      FSA_TRY(lowrank_reduce<double>(c->A.p, n, c->mp, xs.p, ld, ncols, c->D.p, c->scr, c->scr.w.p, ldw2, st));
      FSA_TRY(mspace_apply<double>(c->Cinv.p, c->scr.w.p, ldw2, c->mp, ncols, g.p, ldw2, st));
      FSA_TRY(lowrank_expand<double>(c->A.p, nullptr, n, c->mp, g.p, ldw2, ncols, tt.p, ld, st));
      FSA_TRY((copy_block<double, double>(xs.p, ld, ys.p, ld, n, ncols, st)));
      FSA_TRY(axpy_block(tt.p, -1.0, ys.p, ld, n, ncols, st));
      FSA_TRY(scale_rows(ys.p, ld, c->D.p, n, ncols, 1, st));
      FSA_HIP(hipStreamSynchronize(st));
      break;
    }
    case FSA_OP_PROBES: {
      int ldb = (int)round_up(ncols + 1, 4);
      Buf<double> Bp, Em;
      FSA_TRY(Bp.alloc((size_t)n * ldb));
      FSA_TRY(Em.alloc((size_t)c->mp * ldw));
      FSA_TRY(make_probes(c->A.p, n, c->m, c->mp, c->D.p, c->y.p, c->grid.perm.p, c->opt.seed, ncols, Bp.p, ldb, Em.p,
                          st));
      FSA_TRY((copy_block<double, double>(Bp.p + 1, ldb, ys.p, ld, n, ncols, st)));
      FSA_HIP(hipStreamSynchronize(st));
      break;
    }
    default:
      set_error("unknown operator %d", which);
      return FSA_ERR_INVALID_ARG;
  }
  FSA_TRY(permute_rows(ys.p, ld, xh.p, ncols, c->grid.iperm.p, n, ncols, st));
  FSA_HIP(hipMemcpyAsync(Y, xh.p, (size_t)n * ncols * sizeof(double), hipMemcpyDeviceToHost, st));
  FSA_HIP(hipStreamSynchronize(st));
  return FSA_OK;
}

fsa_status fsa_predict_var(fsa_ctx* c, const double* pred_locs, int64_t n_p, int32_t num_samples, double* var_out,
                           double* mean_out, fsa_stats* st_out) {
  if (!c || !pred_locs || !var_out) { set_error("null argument"); return FSA_ERR_INVALID_ARG; }
  PoolStream ps(c->st);
  if (n_p < 1 || n_p > (int64_t)INT32_MAX / 2) { set_error("n_p out of range"); return FSA_ERR_INVALID_ARG; }
  if (num_samples < 1 || num_samples > 4096) { set_error("num_samples must be in [1, 4096]"); return FSA_ERR_INVALID_ARG; }
  if (mean_out && !c->solved) { set_error("the predictive mean needs a preceding fsa_nll_grad"); return FSA_ERR_INVALID_ARG; }
  return predict_core(c, pred_locs, n_p, num_samples, var_out, mean_out, st_out, nullptr);
}

}  // extern "C"
