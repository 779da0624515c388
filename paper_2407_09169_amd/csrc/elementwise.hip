// Streaming kernels of the MPS arithmetic: block copies (block-diagonal MPS
// addition, operator assembly), the explicit MPO x MPS core product, and fills.
// Each launch processes a table of per-site jobs (blockIdx.y = job) so that a
// whole chain is one launch; threads stream the elements of a core in order,
// so global reads and writes are coalesced along the right bond.
#include "elementwise.h"

namespace qtt {

namespace {

__global__ void fill_kernel(double* p, int64_t n, double v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

__global__ void copy_jobs_kernel(const CopyJob* jobs) {
  const CopyJob j = jobs[blockIdx.y];
  const int64_t n = (int64_t)j.rl * j.sp * j.rr;
  double sc = j.scale;
  if (j.dscale) sc *= *j.dscale;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    int b = (int)(e % j.rr);
    int64_t q = e / j.rr;
    int s = (int)(q % j.sp);
    int a = (int)(q / j.sp);
    int ds = j.diag ? (s * 2 + s) : s;  // MPS digit s -> MPO entry (t = s, s)
    j.dst[((int64_t)(j.ro + a) * j.dp + ds) * j.drr + j.co + b] = sc * j.src[e];
  }
}

__global__ void apply_jobs_kernel(const ApplyJob* jobs) {
  const ApplyJob j = jobs[blockIdx.y];
  // out[(a,alpha), t, (b,beta)] = sum_s W[alpha,t,s,beta] x[a,s,b]
  const int OL = j.xl * j.Dl, OR = j.xr * j.Dr;
  const int64_t n = (int64_t)OL * 2 * OR;
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
      v += j.W[(((int64_t)al * 2 + t) * 2 + s) * j.Dr + be] * j.x[((int64_t)a * 2 + s) * j.xr + b];
    j.out[e] = v;
  }
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
  if (rt::dry()) return;
  int64_t blocks = std::min<int64_t>((n + 255) / 256, 2048);
  hipLaunchKernelGGL(transpose_kernel, dim3((unsigned)blocks), dim3(256), 0, s, src, rows, cols, dst);
  QTT_HIP(hipGetLastError());
}

void eye(double* dst, int m, hipStream_t s) {
  int64_t n = (int64_t)m * m;
  rt::check_range(dst, 0, n - 1, sizeof(double), "eye dst");
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
  if (rt::dry()) return;
  hipLaunchKernelGGL(scalar_comb_kernel, dim3(1), dim3(64), 0, s, out, a, b, cb, scale, n);
  QTT_HIP(hipGetLastError());
}

void fill(double* p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return;
  rt::check_range(p, 0, n - 1, sizeof(double), "fill");
  if (rt::dry()) return;
  int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
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

void copy_jobs(const CopyJob* d_jobs, int njobs, int64_t max_elems, hipStream_t s) {
  if (njobs <= 0) return;
  rt::check_range(d_jobs, 0, njobs - 1, sizeof(CopyJob), "copy job table");
  if (rt::dry()) return;
  int64_t bx = std::min<int64_t>((max_elems + 255) / 256, 1024);
  if (bx < 1) bx = 1;
  hipLaunchKernelGGL(copy_jobs_kernel, dim3((unsigned)bx, njobs), dim3(256), 0, s, d_jobs);
  QTT_HIP(hipGetLastError());
}

void apply_jobs(const ApplyJob* d_jobs, int njobs, int64_t max_elems, hipStream_t s) {
  if (njobs <= 0) return;
  rt::check_range(d_jobs, 0, njobs - 1, sizeof(ApplyJob), "apply job table");
  if (rt::dry()) return;
  int64_t bx = std::min<int64_t>((max_elems + 255) / 256, 1024);
  if (bx < 1) bx = 1;
  hipLaunchKernelGGL(apply_jobs_kernel, dim3((unsigned)bx, njobs), dim3(256), 0, s, d_jobs);
  QTT_HIP(hipGetLastError());
}

}  // namespace qtt
