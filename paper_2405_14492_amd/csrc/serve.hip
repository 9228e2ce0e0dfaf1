// Serving: likelihood + gradient (Section 3.1, eq. NEGLLDNEGLLFSA) and
// predictive-variance (Algorithm 1) requests of uneven size on one GPU.
//
// One device block of hbm_budget bytes is taken at creation.  A request is
// admitted in arrival order once its arrival time has come, a worker is free
// and a contiguous range of the block holds its footprint; the worker then
// runs it on its own stream with every device allocation served from that
// range (a Region current on the worker's thread), and gives the range back
// after the request's streams have drained.  Requests on different workers
// overlap on the device; each one's arithmetic is that of the request alone.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "ops.hpp"

using namespace fsa;

namespace {

// ---------------------------------------------------------------- footprint
// The device's binning (cells of side gamma (1 + 2^-20) over the bounding
// box, at most ~4n cells), mirrored on the host for the size of the pattern.
struct HostGrid {
  double x0 = 0, y0 = 0, h = 0;
  int64_t gx = 0, gy = 0;
  std::vector<int32_t> cnt;  // points per cell
};

int64_t host_cell(double v, double v0, double h, int64_t g) {
  double q = std::floor((v - v0) / h);
  if (q < -2.0) q = -2.0;
  if (q > (double)(g + 1)) q = (double)(g + 1);
  int64_t c = (int64_t)q;
  return c < 0 ? 0 : (c >= g ? g - 1 : c);
}

bool host_grid(const double* locs, int64_t n, double gamma, HostGrid& g) {
  double x0 = INFINITY, y0 = INFINITY, x1 = -INFINITY, y1 = -INFINITY;
  for (int64_t i = 0; i < n; ++i) {
    const double x = locs[2 * i], y = locs[2 * i + 1];
    if (!std::isfinite(x) || !std::isfinite(y)) return false;
    x0 = std::min(x0, x);
    x1 = std::max(x1, x);
    y0 = std::min(y0, y);
    y1 = std::max(y1, y);
  }
  double h = gamma * (1.0 + 1.0 / 1048576.0);
  const double ex = x1 - x0, ey = y1 - y0;
  const double cap = 4.0 * (double)n + 1024.0;
  if ((ex / h + 1.0) * (ey / h + 1.0) > cap) {
    double hmin = std::sqrt(std::fmax(ex * ey, 0.0) / cap);
    hmin = std::fmax(hmin, std::fmax(ex, ey) / cap);
    h = std::fmax(h, hmin * 1.01);
  }
  g.x0 = x0;
  g.y0 = y0;
  g.h = h;
  g.gx = (int64_t)std::floor(ex / h) + 1;
  g.gy = (int64_t)std::floor(ey / h) + 1;
  if (g.gx * g.gy > (int64_t)2000000000) return false;
  g.cnt.assign((size_t)(g.gx * g.gy), 0);
  for (int64_t i = 0; i < n; ++i)
    ++g.cnt[(size_t)(host_cell(locs[2 * i + 1], g.y0, g.h, g.gy) * g.gx + host_cell(locs[2 * i], g.x0, g.h, g.gx))];
  return true;
}

// points of `cnt` in the 3 x 3 neighbourhood of every cell
std::vector<int64_t> nbhd_sums(const HostGrid& g) {
  const int64_t gx = g.gx, gy = g.gy;
  std::vector<int64_t> row((size_t)(gx * gy)), out((size_t)(gx * gy));
  for (int64_t y = 0; y < gy; ++y)
    for (int64_t x = 0; x < gx; ++x) {
      int64_t s = g.cnt[(size_t)(y * gx + x)];
      if (x > 0) s += g.cnt[(size_t)(y * gx + x - 1)];
      if (x + 1 < gx) s += g.cnt[(size_t)(y * gx + x + 1)];
      row[(size_t)(y * gx + x)] = s;
    }
  for (int64_t y = 0; y < gy; ++y)
    for (int64_t x = 0; x < gx; ++x) {
      int64_t s = row[(size_t)(y * gx + x)];
      if (y > 0) s += row[(size_t)((y - 1) * gx + x)];
      if (y + 1 < gy) s += row[(size_t)((y + 1) * gx + x)];
      out[(size_t)(y * gx + x)] = s;
    }
  return out;
}

struct Tally {
  double bytes = 0;
  void add(double b) { bytes += std::ceil(std::max(b, 1.0) / 256.0) * 256.0 + 256.0; }
};

fsa_status check_request(const fsa_request* r, const fsa_options* opt) {
  if (!r || !opt) { set_error("null argument"); return FSA_ERR_INVALID_ARG; }
  if (r->kind != FSA_REQ_NLL_GRAD && r->kind != FSA_REQ_PREDICT_VAR) {
    set_error("unknown request kind %d", r->kind);
    return FSA_ERR_INVALID_ARG;
  }
  if (!r->locs || !r->y || !r->inducing) { set_error("null request array"); return FSA_ERR_INVALID_ARG; }
  if (r->n < 2 || r->n > (int64_t)INT32_MAX / 2) { set_error("need 2 <= n (got %lld)", (long long)r->n); return FSA_ERR_INVALID_ARG; }
  if (r->m < 1 || r->m > r->n || r->m > 512) { set_error("need 1 <= m <= min(n, 512) (got m=%d)", r->m); return FSA_ERR_INVALID_ARG; }
  if (!(r->taper_range > 0) || !std::isfinite(r->taper_range)) { set_error("taper range must be finite and > 0"); return FSA_ERR_INVALID_ARG; }
  const fsa_theta& th = r->theta;
  if ((th.cov != FSA_COV_EXPONENTIAL && th.cov != FSA_COV_MATERN32) || !(th.sigma1_sq > 0) || !(th.rho > 0) ||
      !(th.sigma_sq > 0) || !std::isfinite(th.sigma1_sq) || !std::isfinite(th.rho) || !std::isfinite(th.sigma_sq)) {
    set_error("bad covariance parameters");
    return FSA_ERR_INVALID_ARG;
  }
  if (r->kind == FSA_REQ_PREDICT_VAR && (r->n_p < 1 || !r->pred_locs || r->num_samples < 1)) {
    set_error("a prediction request needs n_p >= 1 locations and num_samples >= 1");
    return FSA_ERR_INVALID_ARG;
  }
  if (!std::isfinite(r->arrival_ms)) { set_error("arrival time must be finite"); return FSA_ERR_INVALID_ARG; }
  if (opt->num_probes < 1 || opt->num_probes > 4096) { set_error("num_probes must be in [1, 4096]"); return FSA_ERR_INVALID_ARG; }
  return FSA_OK;
}

fsa_status footprint(const fsa_request* r, const fsa_options* opt, uint64_t* out) {
  FSA_TRY(check_request(r, opt));
  HostGrid g;
  if (!host_grid(r->locs, r->n, r->taper_range, g)) {
    set_error("non-finite locations or too many grid cells");
    return FSA_ERR_INVALID_ARG;
  }
  const std::vector<int64_t> nb = nbhd_sums(g);
  double cand = 0, tiles = 0;
  for (size_t c = 0; c < g.cnt.size(); ++c) {
    const double k = g.cnt[c];
    if (k > 0) cand += k * (double)nb[c];
  }
  // the sparse product's 64 x 64 tiles per cell pair (cells 2 sx, 2 sx + 1
  // of a row); the pair's neighbourhood holds at most its cells' two
  for (int64_t y = 0; y < g.gy; ++y)
    for (int64_t x = 0; x < g.gx; x += 2) {
      const size_t cl = (size_t)(y * g.gx + x), cr = cl + 1;
      const bool right = x + 1 < g.gx;
      const double k = (double)g.cnt[cl] + (right ? (double)g.cnt[cr] : 0.0);
      if (k <= 0) continue;
      const double v = (double)nb[cl] + (right ? (double)nb[cr] : 0.0);
      tiles += std::ceil(k / 64.0) * std::ceil(v / 64.0);
    }
  const double n = (double)r->n, ncell = (double)(g.gx * g.gy);
  const double mp = (double)round_up(r->m, 64);
  const double tp = opt->num_probes + 1.0, ld = (double)round_up((int64_t)tp, 4), ldw = (double)round_up((int64_t)tp, 64);
  const int prec = opt->precision;
  const bool mixed = prec != FSA_FP64;
  const double maxit = opt->fixed_iter > 0 ? opt->fixed_iter : std::max(opt->max_iter, 1);
  const double nnz = cand;
  Tally T;
  // inputs (host-input build), grid, pattern
  T.add(16 * n); T.add(8 * n); T.add(16 * mp);
  T.add(16 * n); T.add(4 * n); T.add(4 * n); T.add(4 * n); T.add(4 * n);  // xs, cell, perm, iperm, scatter tmp
  T.add(4 * ncell); T.add(8 * (ncell + 1)); T.add(4 * ncell); T.add(8 * (ncell / 1024 + 2));
  T.add(8 * (n + 1)); T.add(4 * nnz); T.add(4 * nnz); T.add(4 * n); T.add(16);
  // factors and values
  for (int k = 0; k < 8; ++k) T.add(8 * mp * mp);  // Sigma_m, L_m, L_m^-1, C, L_C^-1, C^-1, and two work blocks
  T.add(8 * n);                                    // y
  T.add(16 * n); T.add(16 * n);                    // D, D^-1 (and a spare pair)
  T.add(8 * n * mp);                               // A
  if (prec == FSA_MIXED_FP32) T.add(4 * n * mp);
  if (prec == FSA_MIXED_BF16A) { T.add(2 * n * mp); T.add(2 * (n + 8) * mp); }
  T.add(8 * nnz);
  if (mixed) { T.add(4 * nnz); T.add(16384.0 * tiles); T.add(4 * tiles); T.add(8 * (ncell + 1)); T.add(4 * ncell); }
  T.add(8 * n * ld); T.add(8 * mp * ldw);          // probe block, E
  // the library's reduction scratch: column partials and reduce-GEMM tiles
  const double ncb_max = std::max({std::ceil(ldw / 64.0), mp / 64.0,
                                   r->kind == FSA_REQ_PREDICT_VAR ? std::ceil((mp + r->num_samples) / 64.0) : 0.0});
  T.add(8 * std::max(ncell + 1.0, 4096.0) * 64 * ncb_max);                   // dot
  T.add(8 * std::max(ncell + 1.0, 4096.0) * 64 * ncb_max);                   // dot2
  T.add(8 * 512.0 * 64 * ncb_max);                                            // dot1
  T.add(8 * 4096.0 * (mp / 64.0) * (16 * ncb_max + 1024));                    // reduce-GEMM partial tiles
  T.add(16 * mp * 64 * ncb_max);                                              // m-space block
  if (r->kind == FSA_REQ_NLL_GRAD) {
    T.add((mixed ? 28 : 48) * n * ld);             // PCG blocks R, H, V, P, T, Q0 (+ float32 increments)
    T.add(8 * n * ld);                             // U
    T.add(8 * mp * ldw);                           // G
    T.add(16 * maxit * tp); T.add(64 * ldw); T.add(24 * maxit * tp); T.add(64 * ldw);
    if (mixed) { T.add(8 * n * ld); T.add(8 * n * ld); T.add(8 * n * ld); }  // float64 residual replacement
    T.add(16 * n * ld);                            // gradient block [x | u]
    T.add(8 * n * mp);                             // derivative factor F
    T.add(8 * nnz);                                // derivative values
    T.add(16 * n * ld);                            // operator temporaries
    T.add(8 * mp * mp); T.add(8 * mp * mp);
    if (opt->control_variate != FSA_CV_NONE) { T.add(8 * n * mp); T.add(8 * n * mp); T.add(8 * n); T.add(8 * n * 8); }
  } else {
    HostGrid gp = g;  // the prediction points binned on the training grid
    std::fill(gp.cnt.begin(), gp.cnt.end(), 0);
    for (int64_t i = 0; i < r->n_p; ++i) {
      const double x = r->pred_locs[2 * i], y = r->pred_locs[2 * i + 1];
      if (!std::isfinite(x) || !std::isfinite(y)) { set_error("non-finite prediction location"); return FSA_ERR_INVALID_ARG; }
      ++gp.cnt[(size_t)(host_cell(y, g.y0, g.h, g.gy) * g.gx + host_cell(x, g.x0, g.h, g.gx))];
    }
    double candx = 0;
    for (size_t c = 0; c < gp.cnt.size(); ++c) candx += (double)gp.cnt[c] * (double)nb[c];
    const double np = (double)r->n_p, s = r->num_samples;
    const double ldp = (double)round_up((int64_t)(mp + s), 4), lds = (double)round_up((int64_t)s, 4);
    T.add(16 * np); T.add(4);                                                      // locations, flag
    T.add(16 * np); T.add(4 * np); T.add(4 * np); T.add(4 * np); T.add(4 * np);   // prediction grid
    T.add(4 * ncell); T.add(8 * (ncell + 1)); T.add(4 * ncell); T.add(8 * (ncell / 1024 + 2));
    T.add(8 * (np + 1)); T.add(8 * candx); T.add(4 * np);                         // two cross patterns
    T.add(8 * (n + 1)); T.add(8 * candx); T.add(4 * n);
    T.add(8 * np * mp); T.add(8 * candx); T.add(8 * candx);                        // A_p and cross values
    T.add(8 * n * ldp); T.add(8 * n * ldp); T.add(8 * np * lds);                   // B, W, z(1)
    T.add((mixed ? 28 : 48) * n * ldp);                                            // sparse PCG blocks
    T.add(64 * ldp); T.add(16 * maxit * (mp + s)); T.add(16 * ldp);
    if (mixed) { T.add(8 * n * ldp); T.add(8 * n * ldp); T.add(8 * ldp); }         // float64 residual replacement
    T.add(3 * 8 * mp * mp);                                                        // M~, L_M^-1, G
    T.add(3 * 8 * np * mp); T.add(8 * np * lds); T.add(8 * np); T.add(32 * np);    // Y, Y2, Z2, Z_l, out
    if (opt->control_variate != FSA_CV_NONE) { T.add(8 * n * lds); T.add(8 * np * lds); T.add(8 * np); }
  }
  // headroom for the free ranges a request's release order leaves between its
  // blocks, and for small blocks not itemised
  *out = (uint64_t)(T.bytes * 1.08) + (uint64_t(16) << 20);
  return FSA_OK;
}

double clock_ms(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// ---------------------------------------------------------------- jobs
struct Job {
  fsa_request r{};
  std::vector<double> locs, y, ind, pred;
  std::vector<double> var;
  fsa_result res{};
  uint64_t fp = 0;
  size_t off = 0;
  bool done = false;
};

}  // namespace

struct fsa_server {
  fsa_server_options o{};
  int device = 0;
  char* block = nullptr;
  size_t block_bytes = 0;
  std::vector<std::pair<size_t, size_t>> free_ranges;  // (offset, length), sorted, coalesced
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv;       // queue, memory and workers changed
  std::condition_variable cv_done;  // a request finished
  std::deque<Job*> queue;           // by arrival time, then id
  std::map<int64_t, Job*> jobs;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;
  bool stop = false;
  int64_t next_id = 1;
  uint64_t reserved = 0;
  int active = 0;
  fsa_server_stats stats{};

  // first fit of a contiguous range (host bookkeeping only; lock held)
  bool take(size_t bytes, size_t* off) {
    for (auto it = free_ranges.begin(); it != free_ranges.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      if (it->second == bytes) free_ranges.erase(it);
      else {
        it->first += bytes;
        it->second -= bytes;
      }
      return true;
    }
    return false;
  }
  void give(size_t off, size_t len) {
    auto it = std::lower_bound(free_ranges.begin(), free_ranges.end(), std::make_pair(off, (size_t)0));
    it = free_ranges.insert(it, {off, len});
    auto nx = it + 1;
    if (nx != free_ranges.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_ranges.erase(nx);
    }
    if (it != free_ranges.begin()) {
      auto pv = it - 1;
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_ranges.erase(it);
      }
    }
  }
};

namespace {

void run_job(fsa_server* s, Job* j, int w) {
  hipStream_t st = s->streams[(size_t)w];
  Region region(s->block + j->off, (size_t)j->fp);
  fsa_status rc;
  {
    PoolRegion pr(&region);
    fsa_options o = s->o.opt;
    o.hip_stream = st;
    fsa_ctx* c = nullptr;
    const fsa_request& r = j->r;
    rc = fsa_build(j->locs.data(), r.n, 2, j->y.data(), &r.theta, j->ind.data(), r.m, r.taper_range, &o, &c);
    fsa_stats stt{};
    if (rc == FSA_OK) {
      if (r.kind == FSA_REQ_NLL_GRAD) {
        rc = fsa_nll_grad(c, nullptr, &j->res.nll, j->res.grad, &stt);
        j->res.iters_max = stt.iters_max;
        j->res.probe_iters = stt.probe_iters;
      } else {
        j->var.assign((size_t)r.n_p, 0.0);
        rc = fsa_predict_var(c, j->pred.data(), r.n_p, r.num_samples, j->var.data(), nullptr, &stt);
        j->res.iters_max = stt.iters_max;
        j->res.probe_iters = stt.probe_iters;
      }
    }
    if (rc != FSA_OK) snprintf(j->res.message, sizeof(j->res.message), "%s", get_error());
    fsa_destroy(c);
    (void)hipStreamSynchronize(st);
    region.settle();
  }
  j->res.status = rc;
  j->res.peak_bytes = region.peak_bytes();
  if (region.live_bytes() != 0 && rc == FSA_OK) {
    j->res.status = FSA_ERR_DEVICE;
    snprintf(j->res.message, sizeof(j->res.message), "%zu device bytes not released", region.live_bytes());
  }
}

void worker_main(fsa_server* s, int w) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    Job* j = nullptr;
    size_t off = 0;
    for (;;) {
      if (s->queue.empty()) {
        if (s->stop) return;
        s->cv.wait(lk);
        continue;
      }
      Job* h = s->queue.front();
      const double now = clock_ms(s->t0);
      if (h->r.arrival_ms > now) {
        s->cv.wait_for(lk, std::chrono::duration<double, std::milli>(h->r.arrival_ms - now));
        continue;
      }
      if (s->take((size_t)h->fp, &off)) {
        j = h;
        s->queue.pop_front();
        break;
      }
      s->cv.wait(lk);  // memory comes back when a request finishes
    }
    j->off = off;
    j->res.admit_ms = clock_ms(s->t0);
    j->res.worker = w;
    s->reserved += j->fp;
    s->active += 1;
    s->stats.peak_reserved = std::max<uint64_t>(s->stats.peak_reserved, s->reserved);
    s->stats.peak_active = std::max(s->stats.peak_active, s->active);
    s->cv.notify_all();  // the next request may fit beside this one
    lk.unlock();
    run_job(s, j, w);
    lk.lock();
    s->give(j->off, (size_t)j->fp);
    s->reserved -= j->fp;
    s->active -= 1;
    j->res.done_ms = clock_ms(s->t0);
    s->stats.last_done_ms = std::max(s->stats.last_done_ms, j->res.done_ms);
    s->stats.completed += 1;
    if (j->res.status != FSA_OK) s->stats.failed += 1;
    j->done = true;
    s->cv.notify_all();
    s->cv_done.notify_all();
  }
}

}  // namespace

extern "C" {

fsa_status fsa_request_footprint(const fsa_request* r, const fsa_options* opt, uint64_t* bytes) {
  if (!bytes) { set_error("null argument"); return FSA_ERR_INVALID_ARG; }
  return footprint(r, opt, bytes);
}

fsa_status fsa_server_create(const fsa_server_options* o, fsa_server** out) {
  if (!o || !out) { set_error("null argument"); return FSA_ERR_INVALID_ARG; }
  *out = nullptr;
  if (o->slots < 1 || o->slots > 64) { set_error("slots must be in [1, 64]"); return FSA_ERR_INVALID_ARG; }
  if (o->hbm_budget < (uint64_t(1) << 20)) { set_error("hbm_budget must be at least 1 MiB"); return FSA_ERR_INVALID_ARG; }
  const fsa_options& op = o->opt;
  if (op.precision != FSA_FP64 && op.precision != FSA_MIXED_FP32 && op.precision != FSA_MIXED_BF16A) {
    set_error("unknown precision");
    return FSA_ERR_INVALID_ARG;
  }
  if (op.num_probes < 1 || op.num_probes > 4096 || (op.max_iter < 1 && op.fixed_iter < 1) || !(op.cg_rel_tol >= 0)) {
    set_error("bad solver options");
    return FSA_ERR_INVALID_ARG;
  }
  fsa_server* s = new fsa_server();
  s->o = *o;
  FSA_HIP(hipGetDevice(&s->device));
  s->block_bytes = (size_t)o->hbm_budget / 256 * 256;
  if (hipMalloc((void**)&s->block, s->block_bytes) != hipSuccess) {
    (void)hipGetLastError();
    set_error("could not allocate the serving budget of %llu bytes", (unsigned long long)o->hbm_budget);
    delete s;
    return FSA_ERR_OOM;
  }
  s->free_ranges.emplace_back(0, s->block_bytes);
  for (int w = 0; w < o->slots; ++w) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      for (auto x : s->streams) (void)hipStreamDestroy(x);
      (void)hipFree(s->block);
      delete s;
      set_error("stream creation failed");
      return FSA_ERR_DEVICE;
    }
    s->streams.push_back(st);
  }
  s->stats.hbm_budget = s->block_bytes;
  s->stats.slots = o->slots;
  s->stats.first_arrival_ms = INFINITY;
  s->t0 = std::chrono::steady_clock::now();
  for (int w = 0; w < o->slots; ++w) s->workers.emplace_back(worker_main, s, w);
  *out = s;
  return FSA_OK;
}

double fsa_server_clock_ms(const fsa_server* s) { return s ? clock_ms(s->t0) : 0.0; }

fsa_status fsa_server_submit(fsa_server* s, const fsa_request* r, int64_t* id) {
  if (!s || !r || !id) { set_error("null argument"); return FSA_ERR_INVALID_ARG; }
  uint64_t fp = 0;
  FSA_TRY(footprint(r, &s->o.opt, &fp));
  Job* j = new Job();
  j->r = *r;
  j->locs.assign(r->locs, r->locs + 2 * r->n);
  j->y.assign(r->y, r->y + r->n);
  j->ind.assign(r->inducing, r->inducing + 2 * (size_t)r->m);
  if (r->kind == FSA_REQ_PREDICT_VAR) j->pred.assign(r->pred_locs, r->pred_locs + 2 * r->n_p);
  j->r.locs = j->r.y = j->r.inducing = j->r.pred_locs = nullptr;  // the copies above are used
  j->fp = (fp + 255) / 256 * 256;
  j->res.kind = r->kind;
  j->res.arrival_ms = r->arrival_ms;
  j->res.footprint = j->fp;
  j->res.worker = -1;
  j->res.n_p = r->kind == FSA_REQ_PREDICT_VAR ? r->n_p : 0;
  std::lock_guard<std::mutex> lk(s->mu);
  j->res.id = s->next_id++;
  *id = j->res.id;
  s->jobs[j->res.id] = j;
  s->stats.submitted += 1;
  s->stats.first_arrival_ms = std::min(s->stats.first_arrival_ms, r->arrival_ms);
  if (j->fp > s->block_bytes) {
    j->res.status = FSA_ERR_OOM;
    snprintf(j->res.message, sizeof(j->res.message), "footprint of %llu bytes exceeds the budget of %llu",
             (unsigned long long)j->fp, (unsigned long long)s->block_bytes);
    j->res.done_ms = j->res.admit_ms = clock_ms(s->t0);
    j->done = true;
    s->stats.completed += 1;
    s->stats.failed += 1;
    s->cv_done.notify_all();
    return FSA_OK;
  }
  auto it = s->queue.end();
  while (it != s->queue.begin() && (*(it - 1))->r.arrival_ms > r->arrival_ms) --it;
  s->queue.insert(it, j);
  s->cv.notify_all();
  return FSA_OK;
}

fsa_status fsa_server_wait(fsa_server* s, int64_t id, fsa_result* res, double* var_out) {
  if (!s || !res) { set_error("null argument"); return FSA_ERR_INVALID_ARG; }
  Job* j = nullptr;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->jobs.find(id);
    if (it == s->jobs.end()) { set_error("unknown request id %lld", (long long)id); return FSA_ERR_INVALID_ARG; }
    j = it->second;
    s->cv_done.wait(lk, [j] { return j->done; });
    s->jobs.erase(it);
  }
  *res = j->res;
  if (var_out && !j->var.empty()) memcpy(var_out, j->var.data(), j->var.size() * sizeof(double));
  delete j;
  return FSA_OK;
}

fsa_status fsa_server_get_stats(fsa_server* s, fsa_server_stats* st) {
  if (!s || !st) { set_error("null argument"); return FSA_ERR_INVALID_ARG; }
  std::lock_guard<std::mutex> lk(s->mu);
  *st = s->stats;
  return FSA_OK;
}

void fsa_server_destroy(fsa_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv.notify_all();
  }
  for (auto& t : s->workers) t.join();
  for (auto& kv : s->jobs) delete kv.second;
  for (auto st : s->streams) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  (void)hipFree(s->block);
  delete s;
}

}  // extern "C"
