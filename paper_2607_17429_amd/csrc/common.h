// Shared host-side definitions of the FTLM library: error type, last-error
// storage, HIP status checks.
#pragma once

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "ftlm.h"

namespace ftlm {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(int code, const std::string& msg) { throw Error(code, msg); }

void set_last_error(const std::string& msg);

#define FTLM_HIP(expr)                                                                   \
  do {                                                                                   \
    hipError_t _e = (expr);                                                              \
    if (_e != hipSuccess) {                                                              \
      if (_e == hipErrorOutOfMemory)                                                     \
        ::ftlm::fail(FTLM_ERR_OUT_OF_MEMORY, std::string(#expr) + ": out of device memory"); \
      ::ftlm::fail(FTLM_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(_e));     \
    }                                                                                    \
  } while (0)

// Device buffer owned by a host object (freed in the destructor).
template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t count) {
    release();
    if (count == 0) return;
    FTLM_HIP(hipMalloc(reinterpret_cast<void**>(&p), count * sizeof(T)));
    n = count;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  size_t bytes() const { return n * sizeof(T); }
  void upload(const T* h, size_t count, hipStream_t s = nullptr) {
    alloc(count);
    if (count) FTLM_HIP(hipMemcpyAsync(p, h, count * sizeof(T), hipMemcpyHostToDevice, s));
  }
  void upload(const std::vector<T>& v, hipStream_t s = nullptr) { upload(v.data(), v.size(), s); }
  std::vector<T> download(hipStream_t s = nullptr) const {
    std::vector<T> h(n);
    if (n) {
      FTLM_HIP(hipMemcpyAsync(h.data(), p, n * sizeof(T), hipMemcpyDeviceToHost, s));
      FTLM_HIP(hipStreamSynchronize(s));
    }
    return h;
  }
};

}  // namespace ftlm
