// Device memory of the library's grids: every buffer a grid owns is allocated through dmalloc and
// released through dfree.  While a grid's call runs (AllocScope), dmalloc uses that grid's
// allocator hook (wt_set_allocator) or hipMalloc when it has none; dfree returns a buffer to
// whichever allocator produced it.  A registry of live buffers keeps the owner and size of each.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace wt {

struct AllocHook {
  void* (*alloc)(size_t bytes, void* stream, void* ctx) = nullptr;
  void (*free_)(void* p, void* ctx) = nullptr;
  void* ctx = nullptr;
};

// The allocator and owner used by dmalloc on the calling thread until the scope ends (scopes nest).
class AllocScope {
 public:
  AllocScope(const AllocHook* hook, const void* owner, hipStream_t stream);
  ~AllocScope();
  AllocScope(const AllocScope&) = delete;
  AllocScope& operator=(const AllocScope&) = delete;

 private:
  const AllocHook* prev_hook_;
  const void* prev_owner_;
  hipStream_t prev_stream_;
};

hipError_t dmalloc_bytes(void** p, size_t bytes);
template <typename X>
inline hipError_t dmalloc(X** p, size_t bytes) {
  return dmalloc_bytes(reinterpret_cast<void**>(p), bytes);
}
hipError_t dfree(const void* p);

// Live buffers of `owner`: count and bytes that came from a hook and from hipMalloc.
void alloc_stats(const void* owner, int64_t* n_hook, int64_t* bytes_hook, int64_t* n_direct,
                 int64_t* bytes_direct);

// Process-wide hook for grids created later (alloc == nullptr: hipMalloc).
void set_default_hook(const AllocHook& h);
AllocHook default_hook();

}  // namespace wt
