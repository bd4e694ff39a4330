// Device allocation of the grids (see wt_alloc.hpp).
#include "wt_alloc.hpp"

#include <mutex>
#include <unordered_map>

namespace wt {

namespace {
struct Cur {
  const AllocHook* hook = nullptr;
  const void* owner = nullptr;
  hipStream_t stream = nullptr;
};
thread_local Cur t_cur;

struct Rec {
  AllocHook hook;   // alloc == nullptr: hipMalloc
  const void* owner;
  size_t bytes;
};
std::mutex g_mu;
std::unordered_map<const void*, Rec>* g_live = nullptr;   // never destroyed (frees may run at exit)
AllocHook g_default;

std::unordered_map<const void*, Rec>& live() {
  if (!g_live) g_live = new std::unordered_map<const void*, Rec>();
  return *g_live;
}
}  // namespace

AllocScope::AllocScope(const AllocHook* hook, const void* owner, hipStream_t stream)
    : prev_hook_(t_cur.hook), prev_owner_(t_cur.owner), prev_stream_(t_cur.stream) {
  t_cur.hook = hook;
  t_cur.owner = owner;
  t_cur.stream = stream;
}

AllocScope::~AllocScope() {
  t_cur.hook = prev_hook_;
  t_cur.owner = prev_owner_;
  t_cur.stream = prev_stream_;
}

hipError_t dmalloc_bytes(void** p, size_t bytes) {
  *p = nullptr;
  const AllocHook* h = t_cur.hook;
  Rec r{};
  r.owner = t_cur.owner;
  r.bytes = bytes;
  if (h && h->alloc) {
    // a zero-byte request still yields a distinct buffer that can be freed
    void* q = h->alloc(bytes ? bytes : 256, static_cast<void*>(t_cur.stream), h->ctx);
    if (!q) return hipErrorOutOfMemory;
    r.hook = *h;
    *p = q;
  } else {
    const hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) return e;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  live()[*p] = r;
  return hipSuccess;
}

hipError_t dfree(const void* p) {
  if (!p) return hipSuccess;
  Rec r{};
  bool found = false;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = live().find(p);
    if (it != live().end()) {
      r = it->second;
      found = true;
      live().erase(it);
    }
  }
  if (found && r.hook.alloc) {
    // the hook's free may hand the memory to other work at once: nothing of the owner may still
    // use it (the owner's stream has been synchronised by the caller)
    r.hook.free_(const_cast<void*>(p), r.hook.ctx);
    return hipSuccess;
  }
  return hipFree(const_cast<void*>(p));
}

void alloc_stats(const void* owner, int64_t* n_hook, int64_t* bytes_hook, int64_t* n_direct,
                 int64_t* bytes_direct) {
  int64_t a = 0, b = 0, c = 0, d = 0;
  std::lock_guard<std::mutex> lk(g_mu);
  for (const auto& kv : live()) {
    if (kv.second.owner != owner) continue;
    if (kv.second.hook.alloc) {
      ++a;
      b += int64_t(kv.second.bytes);
    } else {
      ++c;
      d += int64_t(kv.second.bytes);
    }
  }
  if (n_hook) *n_hook = a;
  if (bytes_hook) *bytes_hook = b;
  if (n_direct) *n_direct = c;
  if (bytes_direct) *bytes_direct = d;
}

void set_default_hook(const AllocHook& h) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_default = h;
}

AllocHook default_hook() {
  std::lock_guard<std::mutex> lk(g_mu);
  return g_default;
}

}  // namespace wt
