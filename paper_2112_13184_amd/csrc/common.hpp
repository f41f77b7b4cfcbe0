// Shared host/device definitions of the CTMRG library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>

namespace ctm {

// Error raised inside the library; converted to a ctm_status at the C ABI.
struct Error : std::runtime_error {
  int status;
  Error(int st, const std::string& msg) : std::runtime_error(msg), status(st) {}
};

#define CTM_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      throw ::ctm::Error(-3, std::string(#call) + ": " + hipGetErrorString(e_) + " at " \
                                 + __FILE__ + ":" + std::to_string(__LINE__));          \
  } while (0)

#define CTM_CHECK(cond, st, msg)                  \
  do {                                            \
    if (!(cond)) throw ::ctm::Error((st), (msg)); \
  } while (0)

inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

// Device buffer owned by a context (released with hipFree).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void alloc(size_t b) {
    release();
    if (b == 0) b = 8;
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
      p = nullptr;
      throw Error(-2, "hipMalloc of " + std::to_string(b) + " bytes failed: " + hipGetErrorString(e));
    }
    bytes = b;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

// Pinned (page-locked) host memory, so that stream-ordered copies from it
// are asynchronous.
struct PinnedBuf {
  void* p = nullptr;
  size_t bytes = 0;
  PinnedBuf() = default;
  PinnedBuf(const PinnedBuf&) = delete;
  PinnedBuf& operator=(const PinnedBuf&) = delete;
  ~PinnedBuf() { release(); }
  void alloc(size_t b) {
    release();
    hipError_t e = hipHostMalloc(&p, b, hipHostMallocDefault);
    if (e != hipSuccess) {
      p = nullptr;
      throw Error(-2, "hipHostMalloc of " + std::to_string(b) + " bytes failed: " + hipGetErrorString(e));
    }
    bytes = b;
  }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

}  // namespace ctm
