// Shared definitions of the qttpdf HIP library: error state, device
// allocation, fast integer division and the 2-mode tensor-contraction
// descriptor used by every contraction kernel.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/qttpdf.h"

namespace qtt {

// ---------------------------------------------------------------------------
// error state (thread local, read back through tt_last_error)
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
const char* get_error();

struct Error {
  tt_status code;
  std::string msg;
};

#define QTT_THROW(code, ...)                                   \
  do {                                                         \
    char _buf[512];                                            \
    snprintf(_buf, sizeof(_buf), __VA_ARGS__);                 \
    throw ::qtt::Error{code, std::string(_buf)};               \
  } while (0)

#define QTT_HIP(call)                                                             \
  do {                                                                            \
    hipError_t _e = (call);                                                       \
    if (_e != hipSuccess)                                                         \
      QTT_THROW(TT_ERR_HIP, "%s failed: %s (%s:%d)", #call, hipGetErrorString(_e), \
                __FILE__, __LINE__);                                              \
  } while (0)

#define QTT_REQUIRE(cond, ...)                         \
  do {                                                 \
    if (!(cond)) QTT_THROW(TT_ERR_INVALID_ARG, __VA_ARGS__); \
  } while (0)

// Runs `body` and converts exceptions into a status code + error message.
template <class F>
tt_status guard(F&& body) {
  try {
    body();
    return TT_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return TT_ERR_OOM;
  } catch (const std::exception& e) {
    set_error(e.what());
    return TT_ERR_INVALID_ARG;
  }
}

// ---------------------------------------------------------------------------
// runtime shim: allocation registry (every launch is bounds-checked against
// it on the host) and a dry-run mode (QTTPDF_DRYRUN=1) in which "device"
// buffers are host memory and no kernel is launched -- used to validate all
// launch geometry on machines without a GPU.
// ---------------------------------------------------------------------------
namespace rt {
bool dry();
// routes dev_alloc / dev_free through the caller's allocator (null: hipMalloc)
void set_allocator(tt_alloc_fn a, tt_free_fn f, void* user);
void* dev_alloc(size_t bytes);
void dev_free(void* p);
// throws unless [p + lo*esize, p + (hi+1)*esize) lies inside one allocation
void check_range(const void* p, int64_t lo, int64_t hi, size_t esize, const char* what);
// enters memory the library did not allocate (a static device buffer) into
// the registry that check_range consults; idempotent
void register_range(const void* p, size_t bytes);
void unregister_range(const void* p);
void copy(void* dst, const void* src, size_t bytes);  // synchronous, any direction
// asynchronous copy; while launches are fused (below), one copy per instance
void copy_async(void* dst, const void* src, size_t bytes, hipStream_t s);
void sync(hipStream_t s);

// Fused launches over identically laid-out instances (batched stepping).
// Every buffer of instance i lies at the same offset in slab i as instance
// 0's in slab 0; the slabs are `stride` bytes apart and slab 0 is [lo, hi).
// While n > 1 on the calling thread, the launch wrappers that support it run
// each launch for the n instances at once (the kernels shift every data
// pointer, given or read from a device table, by instance * stride; device
// tables of sizes and pointers are read unshifted, from slab 0), and the
// others refuse.
struct Fuse {
  int n = 1;
  int64_t stride = 0;
  uintptr_t lo = 0, hi = 0;
};
Fuse& fuse();  // this thread's setting
// with fusing on: throws unless [p, p + bytes) lies inside slab 0
void fuse_check(const void* p, size_t bytes, const char* what);
// throws when fusing is on (launches without instance support)
void fuse_refuse(const char* what);
// allocation from a slab instead of the device allocator while a slab scope
// is active on this thread: bump allocation, 256-byte aligned, no free
struct SlabScope {
  SlabScope(void* base, size_t cap);
  ~SlabScope();
  size_t used() const;
};
// bytes handed out by dev_alloc on this thread since the last reset (with
// the 256-byte rounding a slab applies)
void alloc_count_reset();
size_t alloc_count();
}  // namespace rt

// pointer shifted by a byte offset (null stays null).  The offset is added to
// a byte pointer, not to an integer: in device code the result then keeps the
// global address space the compiler infers for a kernel argument, so the
// accesses through it stay global loads and stores (a round trip through an
// integer would turn them into flat accesses, which also wait on LDS traffic)
template <class T>
__host__ __device__ inline T* ishift(T* p, int64_t bytes) {
  using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
  return p ? reinterpret_cast<T*>(reinterpret_cast<B*>(p) + bytes) : p;
}

// p taken as a pointer into device (global) memory, which every buffer a
// kernel here receives is.  For pointers the compiler cannot trace to a
// kernel argument (fields of a descriptor passed by value, pointer tables in
// device memory) accesses through the result are global instead of flat ones
// (a flat load also holds up every later wait for LDS traffic).
typedef __attribute__((address_space(1))) double gdouble;
template <class T>
__device__ inline __attribute__((address_space(1))) T* as_global(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// ---------------------------------------------------------------------------
// device buffers
// ---------------------------------------------------------------------------
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  explicit DevBuf(size_t n) { alloc(n); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; bytes = o.bytes; o.p = nullptr; o.bytes = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t n) {
    release();
    if (n == 0) n = 8;
    p = rt::dev_alloc(n);
    bytes = n;
  }
  void release() {
    if (p) rt::dev_free(p);
    p = nullptr;
    bytes = 0;
  }
  double* d() const { return static_cast<double*>(p); }
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// ---------------------------------------------------------------------------
// fast unsigned division by a runtime constant (round-up multiply-shift)
// valid for dividend < 2^31
// ---------------------------------------------------------------------------
struct FastDiv {
  uint32_t d = 1, m = 0, s = 0;
  FastDiv() = default;
  explicit FastDiv(uint32_t div) {
    d = div;
    s = 0;
    while ((1ull << s) < div) ++s;
    uint64_t one = 1;
    m = (uint32_t)(((one << 32) * ((one << s) - div)) / div + 1);
  }
  __host__ __device__ inline uint32_t div(uint32_t x) const {
#if defined(__HIP_DEVICE_COMPILE__)
    uint32_t t = __umulhi(x, m);
#else
    uint32_t t = (uint32_t)(((uint64_t)x * m) >> 32);
#endif
    return (t + x) >> s;
  }
};

// An index i of a contraction dimension that is really two tensor modes:
// offset(i) = (i / n2) * s1 + (i % n2) * s2.  A single mode has n2 == 0 and
// offset(i) = i * s2.
struct Mode2 {
  FastDiv fd;
  int32_t n2 = 0;
  int64_t s1 = 0, s2 = 0;
  __host__ __device__ inline int64_t off(int32_t i) const {
    if (n2 == 0) return (int64_t)i * s2;
    uint32_t q = fd.div((uint32_t)i);
    uint32_t r = (uint32_t)i - q * (uint32_t)n2;
    return (int64_t)q * s1 + (int64_t)r * s2;
  }
};

// largest offset of indices 0..n-1 (non-negative strides)
inline int64_t mode_max(const Mode2& m, int32_t n) {
  if (n <= 0) return 0;
  if (m.n2 == 0) return (int64_t)(n - 1) * m.s2;
  int64_t q = (n - 1) / m.n2;
  int64_t r = std::min<int64_t>(m.n2 - 1, n - 1);
  return q * m.s1 + r * m.s2;
}

inline Mode2 mode1(int64_t stride) {
  Mode2 m;
  m.n2 = 0;
  m.s2 = stride;
  return m;
}
inline Mode2 mode2(int32_t n2, int64_t s1, int64_t s2) {
  Mode2 m;
  if (n2 <= 1) {  // a single outer mode
    m.n2 = 0;
    m.s2 = s1;
    return m;
  }
  m.n2 = n2;
  m.fd = FastDiv((uint32_t)n2);
  m.s1 = s1;
  m.s2 = s2;
  return m;
}

// C[b](m,n) = alpha * sum_k A[b](m,k) B[b](k,n) + beta * C[b](m,n)
// With ksplit > 1 the K range is cut into ksplit chunks whose raw partial
// sums go to part ([batch][ng][ksplit][M][N], dense) and a second kernel adds
// them in a fixed order into C; summed pointer groups (gsum) take the same
// route even without a K split.
// Pointer groups: with ng > 1 the launch covers ng operand sets with the same
// shapes and strides but their own base pointers gA[g], gB[g], gC[g] (e.g. the
// terms of a rounding, whose cores live in different allocations).  With
// gsum = 1 the groups are one more reduction index: C = sum_g A_g B_g (gC
// unused), added in group order by the partial-sum reduction.  The kernels
// read the pointers from the device table gdev = [gA[0..ng), gB[0..ng),
// gC[0..ng)] (the host arrays serve the bounds checks).
constexpr int TC_MAXG = 6;

struct TcDesc {
  int32_t M = 0, N = 0, K = 0, batch = 1;
  Mode2 am, ak, ab;
  Mode2 bk, bn, bb;
  Mode2 cm, cn, cb;
  double alpha = 1.0, beta = 0.0;
  const double* A = nullptr;
  const double* B = nullptr;
  double* C = nullptr;
  int32_t ksplit = 1;
  double* part = nullptr;
  int32_t ng = 1, gsum = 0;
  int32_t ninst = 1;    // fused instances (grid z = batch * groups * K chunks * ninst)
  int64_t istride = 0;  // bytes between the instances' data
  int32_t tile = 0;  // FP64 tile: 0 by size, 1 64x64, 2 64x32, 3 32x64, 4 32x32; MFMA pipeline: 0 K tile 32,
                     // 1 K tile 32 double-buffered, 2 K tile 64 double-buffered
  const double* gA[TC_MAXG] = {};
  const double* gB[TC_MAXG] = {};
  double* gC[TC_MAXG] = {};
  const double* const* gdev = nullptr;
};

// precision of the contraction kernels (inputs are rounded to it, accumulation
// is FP32 for the FP32 / BF16 paths and FP64 otherwise)
enum class Prec { F64 = 0, F32 = 1, BF16 = 2 };

void tc_launch(const TcDesc& d, Prec p, hipStream_t s);
// number of K chunks worth splitting a contraction into (1: no split); the
// caller provides the partial-sum buffer of tc_part_size(d) doubles when
// tc_uses_part(d) (set d.ksplit first)
int tc_choose_ksplit(const TcDesc& d, Prec p);
// Sets d.ksplit and d.tile (FP64 tile; MFMA pipeline and tile) for a launch: with measure, the fastest
// of the candidate tiles and K splits timed on the device with scratch
// outputs (the operands are only read), cached per shape for the process;
// without, a cached choice for the shape or the rule of tc_choose_ksplit.
// QTTPDF_AUTOTUNE=0 keeps the rule everywhere.  Returns whether the choice
// came from a measurement.
bool tc_configure(TcDesc& d, Prec p, bool measure);
// number of launch shapes measured so far and the time spent measuring (s)
void tc_autotune_stats(int* shapes, double* seconds);
inline bool tc_uses_part(const TcDesc& d) { return d.ksplit > 1 || (d.ng > 1 && d.gsum); }
inline int64_t tc_part_size(const TcDesc& d) { return (int64_t)d.batch * d.ng * d.ksplit * d.M * d.N; }
// name of the kernel (template instantiation) a launch uses
std::string tc_kernel_name(const TcDesc& d, Prec p);
std::string qr_kernel_name(int m, int n);
// what factorises one m x n matrix given qr_work_size(1, m, n) of workspace:
// a register kernel's name, "qr_blocked", or "qr_kernel"
std::string qr_path_name(int m, int n);
std::string eig_kernel_name(int max_n);
// host-side bounds check of a contraction against the allocation registry
void tc_validate(const TcDesc& d);

// plain row-major GEMM helper: C(MxN) = alpha*op(A)*op(B) + beta*C
TcDesc gemm_desc(int M, int N, int K, const double* A, int64_t lda, bool transA,
                 const double* B, int64_t ldb, bool transB, double* C, int64_t ldc,
                 double alpha = 1.0, double beta = 0.0);

// ---------------------------------------------------------------------------
// factorisations (FP64)
// ---------------------------------------------------------------------------
// Householder QR of `count` matrices A_i (m x n, m >= n, element (r,c) at
// A + i*strideA + r*rs + c*cs).  Writes the thin explicit Q_i (m x n,
// row-major, leading dimension ldq, default n, at Q + i*strideQ) and, if
// R != nullptr, R_i (n x n upper triangular, row-major, same leading
// dimension).  `work` must hold count*m*n doubles.
// With sq != nullptr (m == n required), matrix i is sq[i] x sq[i] (<= m; none
// when <= 0) in the top-left corner of its m x n layout.  `work` is used only
// when no register configuration fits (qr_kernel_name(m, n) == "qr_kernel");
// then one matrix with m <= 576 and work_size >= qr_work_size(1, m, n) is
// factorised by blocked Householder (32-column register panels, compact WY
// updates on the whole chip) instead of the single-workgroup kernel.
void qr_launch(int count, int m, int n, const double* A, int64_t strideA, int64_t rs, int64_t cs,
               double* Q, int64_t strideQ, double* R, int64_t strideR, double* work,
               hipStream_t s, const int* sq = nullptr, int ldq = 0, int64_t work_size = -1);
// One m x n matrix, thin Q only, in two launches: the factorising workgroup
// leaves the reflectors (V, row-major with unit diagonal, then tau: m n + n
// doubles of work), and one wavefront per column forms Q from them.  Whether
// a shape and workspace take this path (qr_launch takes it by itself when
// they do; QTTPDF_QR_SPLIT=0 turns it off):
bool qr_split(int m, int n, int64_t work_size);
void qr_reflectors_launch(int m, int n, const double* A, int64_t rs, int64_t cs, double* work, hipStream_t s);
void qr_form_q_launch(int m, int n, const double* work, double* Q, int ldq, hipStream_t s);
std::string qr_q_kernel_name(int m, int n);

// workspace that lets a single matrix beyond the register kernels (m <= 576)
// take the blocked Householder QR (pass it as work_size); otherwise
// count * m * n doubles suffice
inline int64_t qr_work_size(int count, int m, int n) {
  return (int64_t)count * m * n + (count == 1 ? (int64_t)m * n + 97 * (int64_t)n + 64 * 32 * (int64_t)n : 0);
}

// Eigen-decomposition of `count` symmetric PSD matrices G_i (n_i x n_i,
// row-major, ld = ldg, at G + i*strideG); n_i = dims[i] (device array).
// Writes the eigenvectors of the k_i = keep[i] largest eigenvalues as the
// columns of P_i (n_i x k_i, row-major, ld = ldp, at P + i*strideP) and all
// eigenvalues in descending order to lam + i*strideL.  `work` holds
// eig_work_size(count, ldg) doubles.  `unoise` is the relative noise of the entries
// of G (the machine epsilon of the arithmetic that produced it): couplings
// below unoise * lambda_max times the column norm are not resolved.
// With `preconditioned`, `work` must hold what eig_precondition_launch wrote
// for the same G: the sweeps then start from W = R2^T, V = Q2 instead of
// W = G, V = I.
void eig_launch(int count, const int* dims, const int* keep, const double* G, int64_t strideG,
                int ldg, double* P, int64_t strideP, int ldp, double* lam, int64_t strideL,
                double* work, int max_n, double unoise, hipStream_t s, bool preconditioned = false);

// Whether matrices of size <= max_n can start the sweeps from a QR
// factorisation of G (every size the kernels take).
bool eig_uses_precondition(int max_n);

// workspace of eig_launch / eig_precondition_launch, in doubles: Q, R1, R2
// and the workspace of the global-memory QR, count * ldg^2 each
inline int64_t eig_work_size(int count, int ldg) { return 4 * (int64_t)count * ldg * ldg; }

// Two QR factorisations, G_i = Q1_i R1_i and R1_i^T = Q2_i R2_i (n_i =
// dims[i]), into `work` (eig_work_size(count, ldg) doubles): Q2_i at
// work + i*ldg^2, R1_i at work + (count + i)*ldg^2, R2_i at
// work + (2 count + i)*ldg^2, row-major with leading dimension max_n; the
// last quarter is the workspace of the global-memory QR (max_n > 160).
void eig_precondition_launch(int count, const int* dims, const double* G, int64_t strideG, int ldg,
                             double* work, int max_n, hipStream_t s);
// relative precision of a contraction precision's products: the machine
// epsilon of FP64 / FP32, and 2^-16 for BF16 (operands split into high and
// low BF16 parts, the low-low product dropped)
inline double machine_eps(Prec p) {
  return p == Prec::F64 ? 2.220446049250313e-16 : (p == Prec::F32 ? 1.1920928955078125e-07 : 1.52587890625e-05);
}

}  // namespace qtt
