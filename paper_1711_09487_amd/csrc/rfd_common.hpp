// Common definitions of the RF-DDES gfx950 library: device matrix handles,
// status plumbing and the launch helpers shared by every translation unit.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

namespace rfd {

// A strided batch of dense column-major matrices, complex as planar (re, im).
// Element (i, j) of item b is re[b * bs + i + j * ld] (+ im at the same
// offset); im == nullptr for real data.
template <typename T>
struct DMat {
  T* re = nullptr;
  T* im = nullptr;
  int64_t ld = 0;
  int64_t bs = 0;
  __host__ __device__ DMat sub(int64_t r, int64_t c) const {
    DMat o = *this;
    o.re = re ? re + r + c * ld : nullptr;
    o.im = im ? im + r + c * ld : nullptr;
    return o;
  }
  __host__ __device__ DMat item(int64_t b) const {
    DMat o = *this;
    o.re = re ? re + b * bs : nullptr;
    o.im = im ? im + b * bs : nullptr;
    return o;
  }
  __host__ __device__ bool cplx() const { return im != nullptr; }
};

// Error carried from the orchestration code to the C ABI.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

enum { ST_OK = 0, ST_EINVAL = 1, ST_ENOMEM = 2, ST_EBREAKDOWN = 3, ST_ENOCONV = 4,
       ST_EDEVICE = 5, ST_ESTATE = 6, ST_EPENDING = 7 };

#define RFD_HIP(call)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      throw ::rfd::Error(::rfd::ST_EDEVICE, std::string(#call) + ": " +               \
                                               hipGetErrorString(e_));                 \
  } while (0)

#define RFD_CHECK_LAUNCH() RFD_HIP(hipGetLastError())

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }
inline unsigned grid1(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

// Owning device allocation (hipMalloc / hipFree), grown on demand.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) {
    o.p = nullptr;
    o.bytes = 0;
  }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      bytes = o.bytes;
      o.p = nullptr;
      o.bytes = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  // Makes room for at least n bytes (contents are not preserved).
  void alloc(size_t n) {
    if (n <= bytes && p) return;
    release();
    if (n == 0) n = 16;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      throw Error(ST_ENOMEM, "device allocation of " + std::to_string(n) + " bytes failed");
    }
    bytes = n;
  }
  template <typename T>
  T* as() const { return static_cast<T*>(p); }
};

// Device flag word written by kernels that detect a breakdown (tiny pivot,
// non-finite value).  Bit 0: tiny pivot, bit 1: non-finite.
struct Flags {
  unsigned* d = nullptr;
};

}  // namespace rfd
