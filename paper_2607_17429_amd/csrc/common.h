// Shared host-side definitions of the FTLM library: error type, last-error
// storage, HIP status checks.
#pragma once

#include <algorithm>
#include <cstdint>
#include <exception>
#include <mutex>
#include <stdexcept>
#include <string>
#include <thread>
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

// Stream for stream-ordered allocation on this thread (nullptr: plain
// hipMalloc/hipFree).  The job server sets it so that building one job's
// tables never waits for other jobs' kernels (hipFree synchronizes the device).
inline thread_local hipStream_t tl_alloc_stream = nullptr;

struct AllocStreamScope {
  hipStream_t prev;
  explicit AllocStreamScope(hipStream_t s) : prev(tl_alloc_stream) { tl_alloc_stream = s; }
  ~AllocStreamScope() { tl_alloc_stream = prev; }
};

// Device buffer owned by a host object (freed in the destructor).
template <typename T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  hipStream_t s = nullptr;  // allocation stream when stream-ordered
  bool async = false;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n), s(o.s), async(o.async) { o.p = nullptr; o.n = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p; n = o.n; s = o.s; async = o.async;
      o.p = nullptr; o.n = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t count) {
    release();
    if (count == 0) return;
    if (tl_alloc_stream) {
      FTLM_HIP(hipMallocAsync(reinterpret_cast<void**>(&p), count * sizeof(T), tl_alloc_stream));
      s = tl_alloc_stream;
      async = true;
    } else {
      FTLM_HIP(hipMalloc(reinterpret_cast<void**>(&p), count * sizeof(T)));
      s = nullptr;
      async = false;
    }
    n = count;
  }
  void release() {
    if (p) {
      if (async)
        (void)hipFreeAsync(p, s);
      else
        (void)hipFree(p);
    }
    p = nullptr;
    n = 0;
  }
  size_t bytes() const { return n * sizeof(T); }
  // Synchronous host -> device copy (the host array may go away afterwards).
  void upload(const T* h, size_t count, hipStream_t st = nullptr) {
    alloc(count);
    if (!st) st = tl_alloc_stream;
    if (count) {
      FTLM_HIP(hipMemcpyAsync(p, h, count * sizeof(T), hipMemcpyHostToDevice, st));
      FTLM_HIP(hipStreamSynchronize(st));
    }
  }
  void upload(const std::vector<T>& v, hipStream_t st = nullptr) { upload(v.data(), v.size(), st); }
  // Asynchronous host -> device copy: the host array must stay unchanged
  // until the stream has passed the copy.
  void upload_async(const T* h, size_t count, hipStream_t st) {
    alloc(count);
    if (count) FTLM_HIP(hipMemcpyAsync(p, h, count * sizeof(T), hipMemcpyHostToDevice, st));
  }
  void upload_async(const std::vector<T>& v, hipStream_t st) { upload_async(v.data(), v.size(), st); }
  std::vector<T> download(hipStream_t st = nullptr) const {
    std::vector<T> h(n);
    if (!st) st = tl_alloc_stream;
    if (n) {
      FTLM_HIP(hipMemcpyAsync(h.data(), p, n * sizeof(T), hipMemcpyDeviceToHost, st));
      FTLM_HIP(hipStreamSynchronize(st));
    }
    return h;
  }
};

// fn(i) for 0 <= i < n on up to 16 host threads (static contiguous ranges;
// results written per index are independent of the split).  The first
// exception thrown by any fn is rethrown on the calling thread.
template <typename F>
void parallel_for(int64_t n, int64_t min_per_thread, F fn) {
  const int64_t hw = std::max<int64_t>(1, (int64_t)std::thread::hardware_concurrency());
  const int64_t nt = std::max<int64_t>(1, std::min<int64_t>({hw, 16, n / std::max<int64_t>(min_per_thread, 1)}));
  if (nt <= 1) {
    for (int64_t i = 0; i < n; ++i) fn(i);
    return;
  }
  std::exception_ptr err;
  std::mutex mu;
  std::vector<std::thread> th;
  for (int64_t t = 0; t < nt; ++t)
    th.emplace_back([&, t] {
      try {
        for (int64_t i = n * t / nt; i < n * (t + 1) / nt; ++i) fn(i);
      } catch (...) {
        std::lock_guard<std::mutex> lk(mu);
        if (!err) err = std::current_exception();
      }
    });
  for (auto& x : th) x.join();
  if (err) std::rethrow_exception(err);
}

}  // namespace ftlm
