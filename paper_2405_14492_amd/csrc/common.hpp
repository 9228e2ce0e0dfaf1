// Internal definitions shared by the FSA HIP kernels and the C-ABI host code.
// gfx950 (CDNA4) only: 64-wide wavefronts, MFMA 16x16x4 for f64/f32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>

#include <string>
#include <vector>

#include "../../include/fsa.h"

namespace fsa {

constexpr int WAVE = 64;

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------- MFMA 16x16x4
// Lane l supplies A[l%16][l/16] and B[l/16][l%16]; accumulator register r of
// lane l holds D[orow(l/16, r)][l%16] with orow = 4q + r for f32 and
// q + 4r for f64 (checked on gfx950).
template <typename T> struct Mfma;
template <> struct Mfma<double> {
  typedef d4 acc;
  static __device__ __forceinline__ int orow(int q, int r) { return q + 4 * r; }
  static __device__ __forceinline__ acc op(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma<float> {
  typedef f4 acc;
  static __device__ __forceinline__ int orow(int q, int r) { return 4 * q + r; }
  static __device__ __forceinline__ acc op(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// Four consecutive elements, loaded with one (or two) vector loads.
template <typename T> struct V4 { T v[4]; };
template <typename T>
__device__ __forceinline__ V4<T> load4(const T* p) {
  V4<T> r;
  if constexpr (sizeof(T) == 8) {
    const d2* q = reinterpret_cast<const d2*>(p);
    d2 a = q[0], b = q[1];
    r.v[0] = a[0]; r.v[1] = a[1]; r.v[2] = b[0]; r.v[3] = b[1];
  } else {
    f4 a = *reinterpret_cast<const f4*>(p);
    r.v[0] = a[0]; r.v[1] = a[1]; r.v[2] = a[2]; r.v[3] = a[3];
  }
  return r;
}

// ---------------------------------------------------------------- covariance
// c(d) = s1 exp(-d/rho)                          (Matérn smoothness 1/2)
// c(d) = s1 (1 + sqrt3 d/rho) exp(-sqrt3 d/rho)  (Matérn smoothness 3/2)
struct Theta {
  int kind;
  double s1, rho, s2;
};

__device__ __forceinline__ double cov_d(double d, const Theta& th) {
  if (th.kind == FSA_COV_EXPONENTIAL) return th.s1 * exp(-d / th.rho);
  double x = 1.7320508075688772 * d / th.rho;
  return th.s1 * (1.0 + x) * exp(-x);
}
// dc/drho
__device__ __forceinline__ double dcov_drho(double d, const Theta& th) {
  if (th.kind == FSA_COV_EXPONENTIAL) return th.s1 * (d / (th.rho * th.rho)) * exp(-d / th.rho);
  double x = 1.7320508075688772 * d / th.rho;
  return th.s1 * (x * x / th.rho) * exp(-x);
}
// Wendland taper (1-r)^4 (1+4r) for r = d/gamma < 1, else 0.
__device__ __forceinline__ double taper(double d, double gamma) {
  double r = d / gamma;
  if (r >= 1.0) return 0.0;
  double a = 1.0 - r;
  a = a * a;
  return a * a * (1.0 + 4.0 * r);
}

// ---------------------------------------------------------------- SplitMix64
// Output number (c+1) of SplitMix64 started from state `seed`.
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t c) {
  uint64_t z = seed + (c + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
// +1 or -1 from the top bit of the counter stream<<60 | col<<40 | idx.
__device__ __forceinline__ double rademacher(uint64_t seed, uint64_t stream, uint64_t col, uint64_t idx) {
  uint64_t v = splitmix64(seed, (stream << 60) | (col << 40) | idx);
  return (v >> 63) ? -1.0 : 1.0;
}
enum { STREAM_RHO = 0, STREAM_E = 1, STREAM_PRED = 2 };

// ---------------------------------------------------------------- reductions
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
const char* get_error();

#define FSA_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t _e = (call);                                                             \
    if (_e != hipSuccess) {                                                             \
      ::fsa::set_error("%s:%d %s: %s", __FILE__, __LINE__, #call, hipGetErrorString(_e)); \
      return FSA_ERR_DEVICE;                                                            \
    }                                                                                   \
  } while (0)

#define FSA_TRY(call)                    \
  do {                                   \
    fsa_status _s = (call);              \
    if (_s != FSA_OK) return _s;         \
  } while (0)

// ---------------------------------------------------------------- memory pool
// Process-wide, stream-ordered caching allocator: a released block is
// reused by the next allocation of the same rounded size, so rebuilding a
// context of the same shape performs no hipMalloc.  A release records an
// event on the calling thread's current stream (set by PoolStream at each
// entry point, and around work enqueued on a side stream); an allocation
// from another stream makes that stream wait for the event, so a block is
// never handed to new work while earlier work that used it can still run.
// With a caller's allocator registered (fsa_set_allocator), blocks come from
// it for the current stream and go back to it once the release event has
// passed.
void* pool_alloc(size_t bytes);
void pool_free(void* p);
// hand every released block of a registered allocator back to it, waiting
// for the work that used it
void pool_flush();
hipStream_t pool_stream();
void pool_set_stream(hipStream_t st);
struct PoolStream {  // scope guard: the current stream of this thread
  hipStream_t prev;
  explicit PoolStream(hipStream_t st) : prev(pool_stream()) { pool_set_stream(st); }
  ~PoolStream() { pool_set_stream(prev); }
  PoolStream(const PoolStream&) = delete;
  PoolStream& operator=(const PoolStream&) = delete;
};

// A fixed range of device memory that serves every pool allocation of one
// host thread while it is current (serving: the device memory reserved for
// one request at its admission).  Blocks are 256-byte aligned and carved
// first-fit from the free ranges; a released block becomes free again once
// the event recorded at its release (on the releasing stream) has passed,
// so a reuse never overlaps earlier work on any stream.  An allocation that
// no free range can hold waits for pending releases, then fails (OOM).
class Region {
 public:
  Region(void* base, size_t bytes);
  ~Region();
  Region(const Region&) = delete;
  Region& operator=(const Region&) = delete;
  void* alloc(size_t bytes);
  bool owns(const void* p) const;
  void release(void* p, hipStream_t st);
  // wait for every pending release (the region is then whole if nothing is live)
  void settle();
  size_t live_bytes() const { return live_; }
  size_t peak_bytes() const { return peak_; }
  size_t size() const { return size_; }

 private:
  struct Pend {
    size_t off, len;
    hipEvent_t ev;
  };
  void reclaim(bool wait);
  void insert_free(size_t off, size_t len);
  char* base_;
  size_t size_, live_ = 0, peak_ = 0;
  std::vector<std::pair<size_t, size_t>> free_;  // (offset, length), sorted by offset, coalesced
  std::vector<std::pair<size_t, size_t>> used_;  // (offset, length) of live blocks
  std::vector<Pend> pend_;
};
Region* pool_region();
void pool_set_region(Region* r);
struct PoolRegion {  // scope guard: the current region of this thread
  Region* prev;
  explicit PoolRegion(Region* r) : prev(pool_region()) { pool_set_region(r); }
  ~PoolRegion() { pool_set_region(prev); }
  PoolRegion(const PoolRegion&) = delete;
  PoolRegion& operator=(const PoolRegion&) = delete;
};

// Device buffer owned by its holder: released to the pool when it is
// reallocated, released explicitly, or destroyed.
template <typename T>
struct Buf {
  T* p = nullptr;
  size_t count = 0;
  Buf() = default;
  Buf(const Buf&) = delete;
  Buf& operator=(const Buf&) = delete;
  Buf(Buf&& o) noexcept : p(o.p), count(o.count) { o.p = nullptr; o.count = 0; }
  Buf& operator=(Buf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      count = o.count;
      o.p = nullptr;
      o.count = 0;
    }
    return *this;
  }
  ~Buf() { release(); }
  fsa_status alloc(size_t n) {
    release();
    if (n == 0) n = 1;
    p = static_cast<T*>(pool_alloc(n * sizeof(T)));
    if (!p) {
      set_error("device allocation of %zu bytes failed", n * sizeof(T));
      return FSA_ERR_OOM;
    }
    count = n;
    return FSA_OK;
  }
  void release() {
    if (p) pool_free(p);
    p = nullptr;
    count = 0;
  }
  size_t bytes() const { return count * sizeof(T); }
};

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

}  // namespace fsa
