// Allocation registry, dry-run switch and copy wrappers (see common.h).
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>

#include "common.h"

namespace qtt {
namespace rt {

static std::mutex g_mu;
static std::map<uintptr_t, size_t>& registry() {
  static std::map<uintptr_t, size_t> m;
  return m;
}

bool dry() {
  static int v = -1;
  if (v < 0) {
    const char* e = std::getenv("QTTPDF_DRYRUN");
    v = (e && e[0] == '1') ? 1 : 0;
  }
  return v == 1;
}

void* dev_alloc(size_t bytes) {
  void* p = nullptr;
  if (dry()) {
    p = std::calloc(1, bytes);
    if (!p) QTT_THROW(TT_ERR_OOM, "host allocation of %zu bytes failed", bytes);
  } else {
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) QTT_THROW(TT_ERR_OOM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  }
  std::lock_guard<std::mutex> lk(g_mu);
  registry()[(uintptr_t)p] = bytes;
  return p;
}

void dev_free(void* p) {
  if (!p) return;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    registry().erase((uintptr_t)p);
  }
  if (dry()) std::free(p);
  else (void)hipFree(p);
}

void register_range(const void* p, size_t bytes) {
  std::lock_guard<std::mutex> lk(g_mu);
  registry()[(uintptr_t)p] = bytes;
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
  if (a < it->first || b > it->first + it->second)
    QTT_THROW(TT_ERR_INVALID_ARG, "%s: access [%ld, %ld] x %zu B overruns its allocation of %zu B",
              what, (long)lo, (long)hi, esize, it->second);
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
  if (dry()) {
    std::memcpy(dst, src, bytes);
    return;
  }
  QTT_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDefault, s));
}

void sync(hipStream_t s) {
  if (dry()) return;
  QTT_HIP(hipStreamSynchronize(s));
}

}  // namespace rt
}  // namespace qtt
