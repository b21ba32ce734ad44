// Device buffers that take their memory from the allocator in force.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

namespace hfmm {

// Device memory of a plan comes from the caller's allocator (hfmm_options_t
// alloc / free / alloc_ctx) or from hipMalloc. The allocator in force is set
// for the duration of each library call that may allocate (AllocScope); every
// buffer keeps the allocator that gave it its memory and returns it there.
struct Allocator {
  void* (*alloc)(size_t, void*) = nullptr;
  void (*free)(void*, void*) = nullptr;
  void* ctx = nullptr;
};
inline thread_local const Allocator* tl_alloc = nullptr;
struct AllocScope {
  const Allocator* prev;
  explicit AllocScope(const Allocator* a) : prev(tl_alloc) { tl_alloc = a; }
  ~AllocScope() { tl_alloc = prev; }
};

template <class T>
struct DevBuf {
  T* p = nullptr;
  size_t n = 0;
  Allocator al{};  // the allocator p came from (alloc == nullptr: hipMalloc)
  hipError_t alloc(size_t count) {
    release();
    n = count;
    if (count == 0) return hipSuccess;
    if (tl_alloc && tl_alloc->alloc) {
      al = *tl_alloc;
      p = (T*)al.alloc(count * sizeof(T), al.ctx);
      if (!p) {
        n = 0;
        return hipErrorOutOfMemory;
      }
      return hipSuccess;
    }
    al = Allocator{};
    return hipMalloc((void**)&p, count * sizeof(T));
  }
  // grow only: keeps the buffer when it already holds count elements
  hipError_t ensure(size_t count) { return n >= count && p ? hipSuccess : alloc(count); }
  hipError_t upload(const std::vector<T>& v, hipStream_t s) {
    hipError_t e = alloc(v.size());
    if (e != hipSuccess || v.empty()) return e;
    return hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
  }
  void release() {
    if (p) {
      if (al.free)
        al.free(p, al.ctx);
      else
        (void)hipFree(p);
    }
    p = nullptr;
    n = 0;
  }
};

}  // namespace hfmm
