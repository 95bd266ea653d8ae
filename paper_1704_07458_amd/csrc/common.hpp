// Shared definitions for the LOBPCG HIP library: error handling, status codes,
// small RAII device buffers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>

#include "lobpcg.h"

namespace lobpcg {

// Error carried across internal layers; converted to a status code at the ABI.
struct Error : public std::runtime_error {
  int code;
  Error(int c, const std::string& msg) : std::runtime_error(msg), code(c) {}
};

#define LOBPCG_HIP(call)                                                              \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      throw ::lobpcg::Error(LOBPCG_ERR_HIP, std::string(#call) + ": " +               \
                                                hipGetErrorString(e_) + " at " +      \
                                                __FILE__ + ":" + std::to_string(__LINE__)); \
  } while (0)

#define LOBPCG_CHECK(cond, code, msg)                  \
  do {                                                 \
    if (!(cond)) throw ::lobpcg::Error((code), (msg)); \
  } while (0)

// Device allocator of a solver handle: the caller's hooks of lobpcg_options
// (dev_alloc / dev_free / alloc_user) or, when they are NULL, hipMalloc /
// hipFree.
struct DevAllocator {
  void* (*alloc)(size_t, void*) = nullptr;
  void (*free)(void*, void*) = nullptr;
  void* user = nullptr;
  bool hooked() const { return alloc != nullptr && free != nullptr; }
};

// The allocator DevBuf::alloc uses on this thread (null = hipMalloc); set for
// the extent of a solver call by AllocatorScope.
inline const DevAllocator*& current_allocator() {
  thread_local const DevAllocator* a = nullptr;
  return a;
}

class AllocatorScope {
 public:
  explicit AllocatorScope(const DevAllocator* a) : prev_(current_allocator()) {
    current_allocator() = a;
  }
  ~AllocatorScope() { current_allocator() = prev_; }
  AllocatorScope(const AllocatorScope&) = delete;
  AllocatorScope& operator=(const AllocatorScope&) = delete;

 private:
  const DevAllocator* prev_;
};

// Owning device allocation.  The allocator in force when the buffer is
// allocated (current_allocator(), else hipMalloc) is remembered and frees it.
class DevBuf {
 public:
  DevBuf() = default;
  explicit DevBuf(size_t bytes) { alloc(bytes); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p_(o.p_), n_(o.n_), a_(o.a_) { o.p_ = nullptr; o.n_ = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p_ = o.p_;
      n_ = o.n_;
      a_ = o.a_;
      o.p_ = nullptr;
      o.n_ = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }

  void alloc(size_t bytes) {
    release();
    if (bytes == 0) return;
    const DevAllocator* a = current_allocator();
    if (a && a->hooked()) {
      a_ = *a;
      p_ = a_.alloc(bytes, a_.user);
      if (!p_)
        throw Error(LOBPCG_ERR_ALLOC, "dev_alloc of " + std::to_string(bytes) + " bytes failed");
    } else {
      a_ = DevAllocator{};
      hipError_t e = hipMalloc(&p_, bytes);
      if (e != hipSuccess) {
        p_ = nullptr;
        throw Error(LOBPCG_ERR_ALLOC, "hipMalloc of " + std::to_string(bytes) +
                                          " bytes failed: " + hipGetErrorString(e));
      }
    }
    n_ = bytes;
  }
  // Grow-only reallocation (contents are not preserved).
  void ensure(size_t bytes) {
    if (bytes > n_) alloc(bytes);
  }
  void release() {
    if (p_) {
      if (a_.hooked()) a_.free(p_, a_.user);
      else (void)hipFree(p_);
    }
    p_ = nullptr;
    n_ = 0;
  }
  template <typename T>
  T* as() const { return static_cast<T*>(p_); }
  void* get() const { return p_; }
  size_t size() const { return n_; }

 private:
  void* p_ = nullptr;
  size_t n_ = 0;
  DevAllocator a_{};
};

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

}  // namespace lobpcg
