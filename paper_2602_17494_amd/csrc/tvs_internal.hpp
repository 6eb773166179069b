// Internal definitions shared by the HIP translation units of libtvs.
//
// Grids: an image grid Omega has N2 rows (y, index i) and N1 columns (x,
// index j); the Step-1 grid Omega-tilde has (N2+1) x (N1+1) points and holds
// Omega as its first N2 rows and N1 columns (Section 4.1).  All device arrays
// are row-major and planar: plane-major, then row, then column.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

namespace tvs {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define TVS_HIP(call)                                                          \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess)                                                      \
      throw ::tvs::Error(-3, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define TVS_LAUNCH_CHECK()                                                     \
  do {                                                                         \
    hipError_t e_ = hipGetLastError();                                         \
    if (e_ != hipSuccess)                                                      \
      throw ::tvs::Error(-3, std::string("kernel launch: ") + hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// complex arithmetic on float2 / double2
// ---------------------------------------------------------------------------
template <typename T> struct alignas(2 * sizeof(T)) cx {
  T x, y;
};
template <typename T> using cplx = cx<T>;

template <typename C>
__device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C>
__device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C>
__device__ __forceinline__ C cmul(C a, C b) {
  return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename C>
__device__ __forceinline__ C cconj(C a) { return C{a.x, -a.y}; }

// ---------------------------------------------------------------------------
// device buffer (RAII, owned by the library)
// ---------------------------------------------------------------------------
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  explicit DevBuf(size_t n) { alloc(n); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; bytes = o.bytes; o.p = nullptr; o.bytes = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t n) {
    release();
    if (n == 0) n = 256;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
      p = nullptr;
      throw Error(-2, "device allocation of " + std::to_string(n) + " bytes failed");
    }
    bytes = n;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <typename U> U* as() const { return static_cast<U*>(p); }
};
template <typename U> U* dptr(const DevBuf& b) { return static_cast<U*>(b.p); }

// ---------------------------------------------------------------------------
// optional kernel timing: HIP events recorded around instrumented launches
// on the launch stream, each with the launch's algorithmic bytes
// ---------------------------------------------------------------------------
struct KernelTimer {
  struct Rec {
    hipEvent_t a, b;
    double bytes;
  };
  struct Acc {
    std::vector<Rec> pending;
    long long calls = 0;     // instrumented calls seen, timed or not
    long long launches = 0;  // timed launches folded in
    double ms = 0, bytes = 0;
  };
  bool on = false;
  int every = 1;  // time one launch in `every` of each class
  std::vector<std::pair<std::string, Acc>> accs;
  std::vector<hipEvent_t> pool;

  Acc& acc(const std::string& name) {
    for (auto& kv : accs)
      if (kv.first == name) return kv.second;
    accs.emplace_back(name, Acc{});
    return accs.back().second;
  }
  hipEvent_t get_event() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) throw Error(-3, "hipEventCreate failed");
    return e;
  }
  // Wrap a launch: timer may be null or off.
  template <typename F>
  static void time(KernelTimer* t, const char* name, double bytes, hipStream_t s, F&& launch) {
    if (!t || !t->on) {
      launch();
      return;
    }
    Acc& a = t->acc(name);
    if (a.calls++ % t->every != 0) {
      launch();
      return;
    }
    // keep the number of outstanding events bounded: the oldest records
    // are long finished when this many have queued up behind them
    if (a.pending.size() >= 64) t->fold_front(a, a.pending.size() / 2);
    Rec r{t->get_event(), t->get_event(), bytes};
    if (hipEventRecord(r.a, s) != hipSuccess) throw Error(-3, "hipEventRecord failed");
    launch();
    if (hipEventRecord(r.b, s) != hipSuccess) throw Error(-3, "hipEventRecord failed");
    a.pending.push_back(r);
  }
  // Fold the first n pending records of a into its totals (waits for them).
  void fold_front(Acc& a, size_t n) {
    for (size_t i = 0; i < n; ++i) {
      Rec& r = a.pending[i];
      if (hipEventSynchronize(r.b) != hipSuccess) throw Error(-3, "hipEventSynchronize failed");
      float ms = 0;
      if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) throw Error(-3, "hipEventElapsedTime failed");
      a.ms += ms;
      a.bytes += r.bytes;
      a.launches += 1;
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    a.pending.erase(a.pending.begin(), a.pending.begin() + static_cast<long>(n));
  }
  // Fold finished records into the totals (waits for their events).
  void collect() {
    for (auto& kv : accs) fold_front(kv.second, kv.second.pending.size());
  }
  void reset() {
    collect();
    accs.clear();
  }
  ~KernelTimer() {
    for (auto& kv : accs)
      for (auto& r : kv.second.pending) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
      }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

// ---------------------------------------------------------------------------
// one axis of a subdomain layout (Section 6.1)
// ---------------------------------------------------------------------------
constexpr int kMaxSub = 32;  // subdomains per axis

struct AxisLayout {
  int n;        // points on the Omega-tilde axis
  int m;        // subdomains on this axis
  int s;        // width of the stripe shared by two neighbours
  int cut[kMaxSub + 1];
  int start[kMaxSub];
  int end[kMaxSub];
};

// One-dimensional partition-of-unity weight (linear ramps across each shared
// stripe, 1 on the rest of the core, 0 outside the subdomain).
template <typename T>
__host__ __device__ __forceinline__ T axis_theta(const AxisLayout& a, int m, int x) {
  if (x < a.start[m] || x >= a.end[m]) return T(0);
  const int lo = a.s / 2, hi = a.s - a.s / 2;
  if (m > 0 && x < a.cut[m] + hi) return (T(x - (a.cut[m] - lo)) + T(0.5)) / T(a.s);
  if (m < a.m - 1 && x >= a.cut[m + 1] - lo)
    return T(1) - (T(x - (a.cut[m + 1] - lo)) + T(0.5)) / T(a.s);
  return T(1);
}

// ---------------------------------------------------------------------------
// FFT plan data passed to kernels by value
// ---------------------------------------------------------------------------
constexpr int kMaxPass = 16;

// Division by a runtime divisor d (1 <= d < 2^16) of numerators x < 2^16 by
// a multiply-high with m = ceil(2^32 / d); exact in that range.
struct FastDiv {
  int d;
  unsigned m;
  __host__ __device__ __forceinline__ int div(int x) const {
#ifdef __HIP_DEVICE_COMPILE__
    return d == 1 ? x : int(__umulhi(unsigned(x), m));
#else
    return x / d;
#endif
  }
};
FastDiv make_fastdiv(int d);

struct FftDesc {
  int n;
  int npass;
  int radix[kMaxPass];
  int twstep[kMaxPass];   // n / (Ls * R)
  FastDiv ls[kMaxPass];   // Ls before the pass (product of earlier radices)
  FastDiv nbf[kMaxPass];  // butterflies per sequence, n / R
};

// smallest even integer >= n whose only prime factors are 2, 3 and 5
int smooth_even_at_least(int n);
// radices 8, 4, 2, 9, 3, 5 in that order of preference, none above max_radix
FftDesc make_fft_desc(int n, int max_radix = 9);

}  // namespace tvs
