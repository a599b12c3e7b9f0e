// Shared host/device definitions of the crk library (gfx950 only).
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>

#include "../../include/crk.h"

// Thread-local last-error text of the C ABI (defined in capi.cpp).
void crk_set_error_(const std::string& msg);
void crk_clear_error_();

namespace crk {

// ------------------------------------------------------------------ errors
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(int code, const std::string& msg) { throw Error(code, msg); }

// On failure the runtime's sticky last error is read back (cleared) so that a
// handled error (e.g. an allocation that did not fit) is not reported again by
// the next launch check.
#define CRK_HIP(call)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess) {                                                                 \
      (void)hipGetLastError();                                                              \
      ::crk::fail(e_ == hipErrorOutOfMemory ? CRK_ENOMEM : CRK_EHIP,                        \
                  std::string(#call) + ": " + hipGetErrorString(e_) + " (" __FILE__ ":" +   \
                      std::to_string(__LINE__) + ")");                                      \
    }                                                                                       \
  } while (0)

#define CRK_REQUIRE(cond, msg)                                  \
  do {                                                          \
    if (!(cond)) ::crk::fail(CRK_EINVAL, std::string(msg));     \
  } while (0)

// A call made out of order (e.g. an operator before the gauge field is loaded).
#define CRK_REQUIRE_STATE(cond, msg)                            \
  do {                                                          \
    if (!(cond)) ::crk::fail(CRK_ESTATE, std::string(msg));     \
  } while (0)

#define CRK_LAUNCH_CHECK() CRK_HIP(hipGetLastError())

// ------------------------------------------------------------------ device buffer
// Device memory comes from a process-wide cache (pool.cpp): device_free keeps
// the buffer for a later device_alloc of about the same size, after waiting for
// the device as hipFree does.  device_free_bytes counts the cached bytes of the
// current device as free.
void* device_alloc(size_t n);
void device_free(void* p) noexcept;
size_t device_cached_bytes(int dev);
size_t device_free_bytes();
void device_release_cached();

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
    if (n == 0) return;
    p = device_alloc(n);
    bytes = n;
  }
  void ensure(size_t n) { if (bytes < n) alloc(n); }
  void release() {
    if (p) device_free(p);
    p = nullptr;
    bytes = 0;
  }
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// ------------------------------------------------------------------ complex arithmetic
template <class T> struct cplx_t;
template <> struct cplx_t<double> { using type = double2; };
template <> struct cplx_t<float> { using type = float2; };
template <class T> using cplx = typename cplx_t<T>::type;

template <class C> __host__ __device__ __forceinline__ C mk(decltype(C::x) r, decltype(C::x) i) {
  C c; c.x = r; c.y = i; return c;
}
__host__ __device__ __forceinline__ double2 operator+(double2 a, double2 b) { return mk<double2>(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ double2 operator-(double2 a, double2 b) { return mk<double2>(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ float2 operator+(float2 a, float2 b) { return mk<float2>(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ float2 operator-(float2 a, float2 b) { return mk<float2>(a.x - b.x, a.y - b.y); }

template <class C> __host__ __device__ __forceinline__ C cmul(C a, C b) {
  return mk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
template <class C> __host__ __device__ __forceinline__ C cmulc(C a, C b) {
  return mk<C>(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
// acc += a * b
template <class C> __host__ __device__ __forceinline__ void cfma(C& acc, C a, C b) {
  acc.x = fma(a.x, b.x, acc.x); acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y); acc.y = fma(a.y, b.x, acc.y);
}
// acc += conj(a) * b
template <class C> __host__ __device__ __forceinline__ void cfmac(C& acc, C a, C b) {
  acc.x = fma(a.x, b.x, acc.x); acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y); acc.y = fma(-a.y, b.x, acc.y);
}
template <class C> __host__ __device__ __forceinline__ C cscale(C a, decltype(C::x) s) { return mk<C>(a.x * s, a.y * s); }
template <class C> __host__ __device__ __forceinline__ C cconj(C a) { return mk<C>(a.x, -a.y); }
// multiply by i
template <class C> __host__ __device__ __forceinline__ C cmuli(C a) { return mk<C>(-a.y, a.x); }
template <class C> __host__ __device__ __forceinline__ C czero() { return mk<C>(0, 0); }

template <class D, class S> __host__ __device__ __forceinline__ D ccast(S a) {
  return mk<D>(static_cast<decltype(D::x)>(a.x), static_cast<decltype(D::x)>(a.y));
}

// ------------------------------------------------------------------ launch helpers
constexpr int kNumXcd = 8;

// Map the hardware workgroup id to a logical id so that each XCD (which
// receives workgroups round-robin) processes one contiguous range of logical
// work, keeping neighbouring tiles in the same L2.
__device__ __forceinline__ uint32_t xcd_swizzle(uint32_t bid, uint32_t nb) {
  uint32_t q = nb / kNumXcd, r = nb % kNumXcd;
  uint32_t x = bid % kNumXcd, i = bid / kNumXcd;
  return x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
}

inline unsigned ceil_div(int64_t a, int64_t b) { return static_cast<unsigned>((a + b - 1) / b); }

}  // namespace crk
