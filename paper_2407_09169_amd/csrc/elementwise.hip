// Streaming kernels of the MPS arithmetic: block copies (block-diagonal MPS
// addition, operator assembly), the explicit MPO x MPS core product, and fills.
// Each launch processes a table of per-site jobs (blockIdx.y = job) so that a
// whole chain is one launch; threads stream the elements of a core in order,
// so global reads and writes are coalesced along the right bond.
#include <cmath>

#include "elementwise.h"

namespace qtt {

namespace {

// Fused launches (batched instances): grid y or z is the instance, whose data
// lie istride bytes after the previous one's; job tables and size tables are
// shared, the pointers they hold are shifted.
__global__ void fill_kernel(double* p, int64_t n, double v, int64_t istride) {
  p = ishift(p, (int64_t)blockIdx.y * istride);
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

__global__ void copy_jobs_kernel(const CopyJob* jobs, int64_t istride) {
  CopyJob j = jobs[blockIdx.y];
  const int64_t io = (int64_t)blockIdx.z * istride;
  j.src = ishift(j.src, io);
  j.dst = ishift(j.dst, io);
  j.dscale = ishift(j.dscale, io);
  const int64_t n = (int64_t)j.rl * j.sp * j.rr;
  double sc = j.scale;
  if (j.dscale) sc *= *as_global(j.dscale);
  const gdouble* src = as_global(j.src);  // table pointers: global accesses
  gdouble* dst = as_global(j.dst);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    int b = (int)(e % j.rr);
    int64_t q = e / j.rr;
    int s = (int)(q % j.sp);
    int a = (int)(q / j.sp);
    int ds = j.diag ? (s * 2 + s) : s;  // MPS digit s -> MPO entry (t = s, s)
    dst[((int64_t)(j.ro + a) * j.dp + ds) * j.drr + j.co + b] = sc * src[e];
  }
}

// product of two operands at contraction precision PR: FP64, FP32 inputs, or
// BF16 high + low parts (three products, the low-low one dropped)
template <int PR>
__device__ inline double prec_mul(double w, double x) {
  if constexpr (PR == 0) {
    return w * x;
  } else if constexpr (PR == 1) {
    return (double)((float)w * (float)x);
  } else {
    const float wf = (float)w, xf = (float)x;
    const float wh = (float)(__bf16)wf, xh = (float)(__bf16)xf;
    const float wl = (float)(__bf16)(wf - wh), xl = (float)(__bf16)(xf - xh);
    return (double)(wh * xh + (wh * xl + wl * xh));
  }
}

template <int PR>
__global__ void apply_jobs_kernel(const ApplyJob* jobs) {
  const ApplyJob j = jobs[blockIdx.y];
  // out[(a,alpha), t, (b,beta)] = sum_s W[alpha,t,s,beta] x[a,s,b]
  const int OL = j.xl * j.Dl, OR = j.xr * j.Dr;
  const int64_t n = (int64_t)OL * 2 * OR;
  const gdouble* W = as_global(j.W);  // table pointers: global accesses
  const gdouble* x = as_global(j.x);
  gdouble* out = as_global(j.out);
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    int col = (int)(e % OR);
    int64_t q = e / OR;
    int t = (int)(q % 2);
    int row = (int)(q / 2);
    int a = row / j.Dl, al = row % j.Dl;
    int b = col / j.Dr, be = col % j.Dr;
    double v = 0.0;
#pragma unroll
    for (int s = 0; s < 2; ++s)
      v += prec_mul<PR>(W[(((int64_t)al * 2 + t) * 2 + s) * j.Dr + be], x[((int64_t)a * 2 + s) * j.xr + b]);
    out[e] = v;
  }
}

// Rank cut of a batch of truncations: matrix i keeps its first keep[i]
// eigenvector columns; those whose eigenvalue is at most tol2 * lam[0] (all but
// the first) are zeroed, so the rounding keeps only singular values above
// sqrt(tol2) sigma_1.
__global__ void rank_cut_kernel(double* P, int64_t strideP, int ldp, const double* lam, int64_t strideL,
                                const int* dims, const int* keep, double tol2, int64_t istride) {
  const int i = blockIdx.x;
  P = ishift(P, (int64_t)blockIdx.y * istride);
  lam = ishift(lam, (int64_t)blockIdx.y * istride);
  const double* l = lam + i * strideL;
  const int kp = keep[i], rows = dims[i];
  const double cut = tol2 * l[0];
  int k = 1;
  while (k < kp && l[k] > cut) ++k;
  double* Pi = P + i * strideP;
  const int64_t n = (int64_t)rows * (kp - k);
  for (int64_t e = threadIdx.x; e < n; e += blockDim.x) {
    const int r = (int)(e / (kp - k)), c = k + (int)(e % (kp - k));
    Pi[(int64_t)r * ldp + c] = 0.0;
  }
}

// Sets *flag to 1 if any of the n values is NaN or infinite.
__global__ void nonfinite_kernel(const double* p, int64_t n, int* flag, int64_t istride) {
  p = ishift(p, (int64_t)blockIdx.y * istride);
  flag = ishift(flag, (int64_t)blockIdx.y * istride);
  bool bad = false;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    bad |= !isfinite(p[e]);
  if (bad) *flag = 1;
}

__global__ void transpose_kernel(const double* src, int rows, int cols, double* dst) {
  int64_t n = (int64_t)rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    int r = (int)(e / cols), c = (int)(e % cols);
    dst[(int64_t)c * rows + r] = src[e];
  }
}

__global__ void eye_kernel(double* dst, int m) {
  int64_t n = (int64_t)m * m;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = (e / m == e % m) ? 1.0 : 0.0;
}

__global__ void scalar_comb_kernel(double* out, const double* a, const double* b, double cb,
                                   double scale, int n) {
  int i = threadIdx.x;
  if (i < n) out[i] = scale * (a[i] + (b ? cb * b[i] : 0.0));
}

}  // namespace

void transpose(const double* src, int rows, int cols, double* dst, hipStream_t s) {
  int64_t n = (int64_t)rows * cols;
  if (n <= 0) return;
  rt::check_range(src, 0, n - 1, sizeof(double), "transpose src");
  rt::check_range(dst, 0, n - 1, sizeof(double), "transpose dst");
  rt::fuse_refuse("transpose");
  if (rt::dry()) return;
  int64_t blocks = std::min<int64_t>((n + 255) / 256, 2048);
  hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)blocks), dim3(256), 0, s, src, rows, cols, dst);
  QTT_HIP(hipGetLastError());
}

void eye(double* dst, int m, hipStream_t s) {
  int64_t n = (int64_t)m * m;
  rt::check_range(dst, 0, n - 1, sizeof(double), "eye dst");
  rt::fuse_refuse("eye");
  if (rt::dry()) return;
  int64_t blocks = std::min<int64_t>((n + 255) / 256, 2048);
  hipLaunchKernelGGL(eye_kernel, dim3((unsigned)blocks), dim3(256), 0, s, dst, m);
  QTT_HIP(hipGetLastError());
}

void scalar_comb(double* out, const double* a, const double* b, double cb, double scale, int n,
                 hipStream_t s) {
  QTT_REQUIRE(n <= 64, "scalar_comb: n <= 64");
  rt::check_range(out, 0, n - 1, sizeof(double), "scalar out");
  rt::check_range(a, 0, n - 1, sizeof(double), "scalar a");
  if (b) rt::check_range(b, 0, n - 1, sizeof(double), "scalar b");
  rt::fuse_refuse("scalar_comb");
  if (rt::dry()) return;
  hipLaunchKernelGGL(scalar_comb_kernel, dim3(1), dim3(64), 0, s, out, a, b, cb, scale, n);
  QTT_HIP(hipGetLastError());
}

void fill(double* p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return;
  rt::check_range(p, 0, n - 1, sizeof(double), "fill");
  rt::fuse_check(p, 8 * n, "fill");
  if (rt::dry()) return;
  const rt::Fuse& fu = rt::fuse();
  int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks, fu.n), dim3(256), 0, s, p, n, v, fu.stride);
  QTT_HIP(hipGetLastError());
}

void validate(const CopyJob& j) {
  QTT_REQUIRE(j.sp == 2 || j.sp == 4, "copy job: bad physical size");
  QTT_REQUIRE(!j.diag || (j.sp == 2 && j.dp == 4), "copy job: diag needs MPS -> MPO");
  QTT_REQUIRE(j.co + j.rr <= j.drr, "copy job: block exceeds the destination bond");
  rt::check_range(j.src, 0, (int64_t)j.rl * j.sp * j.rr - 1, sizeof(double), "copy job source");
  int64_t hi = ((int64_t)(j.ro + j.rl - 1) * j.dp + (j.dp - 1)) * j.drr + j.co + j.rr - 1;
  rt::check_range(j.dst, 0, hi, sizeof(double), "copy job destination");
  if (j.dscale) rt::check_range(j.dscale, 0, 0, sizeof(double), "copy job scale");
}

void validate(const ApplyJob& j) {
  rt::check_range(j.W, 0, (int64_t)j.Dl * 4 * j.Dr - 1, sizeof(double), "apply operator");
  rt::check_range(j.x, 0, (int64_t)j.xl * 2 * j.xr - 1, sizeof(double), "apply state");
  rt::check_range(j.out, 0, (int64_t)j.xl * j.Dl * 2 * j.xr * j.Dr - 1, sizeof(double), "apply out");
}

void fuse_check(const std::vector<CopyJob>& jobs) {
  if (rt::fuse().n <= 1) return;
  for (const CopyJob& j : jobs) {
    rt::fuse_check(j.src, 8 * (int64_t)j.rl * j.sp * j.rr, "copy job source");
    const int64_t hi = ((int64_t)(j.ro + j.rl - 1) * j.dp + (j.dp - 1)) * j.drr + j.co + j.rr - 1;
    rt::fuse_check(j.dst, 8 * (hi + 1), "copy job destination");
    if (j.dscale) rt::fuse_check(j.dscale, 8, "copy job scale");
  }
}

void copy_jobs(const CopyJob* d_jobs, int njobs, int64_t max_elems, hipStream_t s) {
  if (njobs <= 0) return;
  rt::check_range(d_jobs, 0, njobs - 1, sizeof(CopyJob), "copy job table");
  if (rt::dry()) return;
  const rt::Fuse& fu = rt::fuse();
  int64_t bx = std::min<int64_t>((max_elems + 255) / 256, 1024);
  if (bx < 1) bx = 1;
  hipLaunchKernelGGL(copy_jobs_kernel, dim3((unsigned)bx, njobs, fu.n), dim3(256), 0, s, d_jobs, fu.stride);
  QTT_HIP(hipGetLastError());
}

void rank_cut(double* P, int64_t strideP, int ldp, const double* lam, int64_t strideL, const int* d_dims,
              const int* d_keep, const std::vector<int>& dims, const std::vector<int>& keep, double tol2,
              hipStream_t s) {
  const int count = (int)dims.size();
  if (count == 0) return;
  for (int i = 0; i < count; ++i) {
    QTT_REQUIRE(keep[i] >= 1 && keep[i] <= ldp && keep[i] <= dims[i], "rank cut: keep %d of %d", keep[i], dims[i]);
    rt::check_range(P, i * strideP, i * strideP + (int64_t)(dims[i] - 1) * ldp + keep[i] - 1, sizeof(double),
                    "rank cut vectors");
    rt::check_range(lam, i * strideL, i * strideL + keep[i] - 1, sizeof(double), "rank cut values");
  }
  rt::check_range(d_dims, 0, count - 1, sizeof(int), "rank cut dims");
  rt::check_range(d_keep, 0, count - 1, sizeof(int), "rank cut keep");
  const rt::Fuse& fu = rt::fuse();
  if (fu.n > 1) {
    for (int i = 0; i < count; ++i) {
      rt::fuse_check(P + i * strideP, 8 * ((int64_t)(dims[i] - 1) * ldp + keep[i]), "rank cut vectors");
      rt::fuse_check(lam + i * strideL, 8 * (int64_t)keep[i], "rank cut values");
    }
  }
  if (rt::dry()) return;
  hipLaunchKernelGGL(rank_cut_kernel, dim3(count, fu.n), dim3(256), 0, s, P, strideP, ldp, lam, strideL, d_dims,
                     d_keep, tol2, fu.stride);
  QTT_HIP(hipGetLastError());
}

void check_finite(const double* p, int64_t n, int* flag, hipStream_t s) {
  if (n <= 0) return;
  rt::check_range(p, 0, n - 1, sizeof(double), "finite check");
  rt::check_range(flag, 0, 0, sizeof(int), "finite check flag");
  rt::fuse_check(p, 8 * n, "finite check");
  rt::fuse_check(flag, sizeof(int), "finite check flag");
  if (rt::dry()) {  // host memory stands in for device memory: scan it here
    for (int64_t e = 0; e < n; ++e)
      if (!std::isfinite(p[e])) *flag = 1;
    return;
  }
  const rt::Fuse& fu = rt::fuse();
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(nonfinite_kernel, dim3((unsigned)blocks, fu.n), dim3(256), 0, s, p, n, flag, fu.stride);
  QTT_HIP(hipGetLastError());
}

void apply_jobs(const ApplyJob* d_jobs, int njobs, int64_t max_elems, hipStream_t s, Prec prec) {
  if (njobs <= 0) return;
  rt::check_range(d_jobs, 0, njobs - 1, sizeof(ApplyJob), "apply job table");
  rt::fuse_refuse("the explicit MPO x MPS product");
  if (rt::dry()) return;
  int64_t bx = std::min<int64_t>((max_elems + 255) / 256, 1024);
  if (bx < 1) bx = 1;
  const dim3 grid((unsigned)bx, njobs);
  if (prec == Prec::F64) hipLaunchKernelGGL(apply_jobs_kernel<0>, grid, dim3(256), 0, s, d_jobs);
  else if (prec == Prec::F32) hipLaunchKernelGGL(apply_jobs_kernel<1>, grid, dim3(256), 0, s, d_jobs);
  else hipLaunchKernelGGL(apply_jobs_kernel<2>, grid, dim3(256), 0, s, d_jobs);
  QTT_HIP(hipGetLastError());
}

}  // namespace qtt
