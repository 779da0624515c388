// Allocation registry, dry-run switch and copy wrappers (see common.h).
#include <cstdlib>
#include <malloc.h>
#include <cstring>
#include <map>
#include <mutex>

#include "common.h"

namespace qtt {
namespace rt {

static std::mutex g_mu;
// every device range the library may touch: bytes, and whether it came from
// the caller's allocator (returned to it on free)
struct Range {
  size_t bytes = 0;
  bool hooked = false;
  bool slab = false;  // carved from a slab: nothing to free
};
static std::map<uintptr_t, Range>& registry() {
  static std::map<uintptr_t, Range> m;
  return m;
}

// the caller's allocator (tt_set_allocator); null: hipMalloc / hipFree
static tt_alloc_fn g_alloc = nullptr;
static tt_free_fn g_free = nullptr;
static void* g_user = nullptr;

void set_allocator(tt_alloc_fn a, tt_free_fn f, void* user) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_alloc = a;
  g_free = f;
  g_user = user;
}

bool dry() {
  static int v = -1;
  if (v < 0) {
    const char* e = std::getenv("QTTPDF_DRYRUN");
    v = (e && e[0] == '1') ? 1 : 0;
    // Dry runs stand host memory in for thousands of workspaces of up to
    // gigabytes: a fixed mmap threshold gives each large one its own fresh
    // zero pages, instead of heap chunks that glibc would search and clear
    // (its adaptive threshold otherwise grows after the first large frees).
    if (v == 1) mallopt(M_MMAP_THRESHOLD, 256 * 1024);
  }
  return v == 1;
}

namespace {
struct Slab {
  char* base = nullptr;
  size_t cap = 0, used = 0;
};
thread_local Slab* t_slab = nullptr;
thread_local size_t t_count = 0;
thread_local Fuse t_fuse;
constexpr size_t kSlabAlign = 256;
size_t slab_round(size_t b) { return (std::max<size_t>(b, 1) + kSlabAlign - 1) & ~(kSlabAlign - 1); }
}  // namespace

SlabScope::SlabScope(void* base, size_t cap) {
  QTT_REQUIRE(t_slab == nullptr, "slab scopes do not nest");
  QTT_REQUIRE(((uintptr_t)base & (kSlabAlign - 1)) == 0, "slab base not aligned");
  t_slab = new Slab{static_cast<char*>(base), cap, 0};
}
SlabScope::~SlabScope() {
  delete t_slab;
  t_slab = nullptr;
}
size_t SlabScope::used() const { return t_slab ? t_slab->used : 0; }

void alloc_count_reset() { t_count = 0; }
size_t alloc_count() { return t_count; }

Fuse& fuse() { return t_fuse; }

void fuse_check(const void* p, size_t bytes, const char* what) {
  const Fuse& f = t_fuse;
  if (f.n <= 1 || bytes == 0) return;
  const uintptr_t a = (uintptr_t)p;
  if (!(a >= f.lo && a + bytes <= f.hi))
    QTT_THROW(TT_ERR_INVALID_ARG, "%s: a fused launch needs its data inside the instance slab", what);
}

void fuse_refuse(const char* what) {
  if (t_fuse.n > 1) QTT_THROW(TT_ERR_INVALID_ARG, "%s has no fused form for batched instances", what);
}

void* dev_alloc(size_t bytes) {
  void* p = nullptr;
  bool hooked = false;
  t_count += slab_round(bytes);
  if (t_slab) {
    Slab& sl = *t_slab;
    const size_t n = slab_round(bytes);
    if (sl.used + n > sl.cap)
      QTT_THROW(TT_ERR_OOM, "slab of %zu bytes exhausted (%zu more needed)", sl.cap, sl.used + n - sl.cap);
    p = sl.base + sl.used;
    sl.used += n;
    std::lock_guard<std::mutex> lk(g_mu);
    registry()[(uintptr_t)p] = Range{bytes, false, true};
    return p;
  }
  if (dry()) {
    p = std::calloc(1, bytes);
    if (!p) QTT_THROW(TT_ERR_OOM, "host allocation of %zu bytes failed", bytes);
  } else {
    tt_alloc_fn a;
    void* user;
    {
      std::lock_guard<std::mutex> lk(g_mu);
      a = g_alloc;
      user = g_user;
    }
    if (a) {
      int dev = 0;
      QTT_HIP(hipGetDevice(&dev));
      p = a(bytes, dev, nullptr, user);
      if (!p) QTT_THROW(TT_ERR_OOM, "the registered allocator returned no memory for %zu bytes", bytes);
      hooked = true;
    } else {
      hipError_t e = hipMalloc(&p, bytes);
      if (e != hipSuccess) QTT_THROW(TT_ERR_OOM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
  }
  std::lock_guard<std::mutex> lk(g_mu);
  registry()[(uintptr_t)p] = Range{bytes, hooked};
  return p;
}

void dev_free(void* p) {
  if (!p) return;
  Range r;
  tt_free_fn f;
  void* user;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = registry().find((uintptr_t)p);
    if (it != registry().end()) {
      r = it->second;
      registry().erase(it);
    }
    f = g_free;
    user = g_user;
  }
  if (r.slab) {
    return;  // the slab's owner frees it as a whole
  } else if (dry()) {
    std::free(p);
  } else if (r.hooked) {
    // the caller's allocator may hand the block to other streams at once:
    // no kernel of the library may still use it
    (void)hipDeviceSynchronize();
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (f) f(p, r.bytes, dev, nullptr, user);
  } else {
    (void)hipFree(p);
  }
}

void register_range(const void* p, size_t bytes) {
  std::lock_guard<std::mutex> lk(g_mu);
  registry()[(uintptr_t)p] = Range{bytes, false};
}

void unregister_range(const void* p) {
  std::lock_guard<std::mutex> lk(g_mu);
  registry().erase((uintptr_t)p);
}

void check_range(const void* p, int64_t lo, int64_t hi, size_t esize, const char* what) {
  if (hi < lo) return;  // empty range
  uintptr_t a = (uintptr_t)p + (uintptr_t)(lo * (int64_t)esize);
  uintptr_t b = (uintptr_t)p + (uintptr_t)((hi + 1) * (int64_t)esize);
  std::lock_guard<std::mutex> lk(g_mu);
  auto& m = registry();
  auto it = m.upper_bound(a);
  if (it == m.begin()) QTT_THROW(TT_ERR_INVALID_ARG, "%s: pointer outside every allocation", what);
  --it;
  if (a < it->first || b > it->first + it->second.bytes)
    QTT_THROW(TT_ERR_INVALID_ARG, "%s: access [%ld, %ld] x %zu B overruns its allocation of %zu B",
              what, (long)lo, (long)hi, esize, it->second.bytes);
}

void copy(void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return;
  if (dry()) {
    std::memcpy(dst, src, bytes);
    return;
  }
  QTT_HIP(hipMemcpy(dst, src, bytes, hipMemcpyDefault));
}

void copy_async(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (bytes == 0) return;
  const Fuse& f = t_fuse;
  if (f.n > 1) {
    fuse_check(dst, bytes, "copy destination");
    fuse_check(src, bytes, "copy source");
  }
  if (dry()) {
    std::memcpy(dst, src, bytes);
    return;
  }
  for (int i = 0; i < f.n; ++i)
    QTT_HIP(hipMemcpyAsync(ishift(dst, i * f.stride), ishift(src, i * f.stride), bytes, hipMemcpyDefault, s));
}

void sync(hipStream_t s) {
  if (dry()) return;
  QTT_HIP(hipStreamSynchronize(s));
}

}  // namespace rt
}  // namespace qtt
