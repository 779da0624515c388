// FP64 factorisation kernels: Householder QR (thin explicit Q, optional R)
// and the symmetric eigen-decomposition used by the bond truncation.
//
// One workgroup per matrix; the matrix is staged column-major in a global
// workspace (L2 resident for the sizes used here) so that each Householder
// reflector or Jacobi rotation touches contiguous columns.  Reductions over
// a column use wavefront shuffles, then one LDS slot per wavefront.
#include "common.h"

namespace qtt {

namespace {

constexpr int FT = 256;  // threads per factorisation workgroup
constexpr int FW = FT / 64;

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < FW; ++w) s += red[w];
  return s;
}

// ---------------------------------------------------------------------------
// Householder QR:  A (m x n, m >= n) = Q R,  H_j = I - tau_j v_j v_j^T,
// v_j(j) = 1, beta_j = -sign(a_jj) ||a_{j:,j}||.  Q formed in place by
// backward accumulation (apply H_j to columns j+1.., then set column j).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(FT) void qr_kernel(int m, int n, const double* __restrict__ A0,
                                                int64_t strideA, int64_t rs, int64_t cs,
                                                double* __restrict__ Q0, int64_t strideQ,
                                                double* __restrict__ R0, int64_t strideR,
                                                double* __restrict__ work) {
  __shared__ double red[FW];
  __shared__ double taus[1024];
  __shared__ double betas[1024];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t b = blockIdx.x;
  const double* A = A0 + b * strideA;
  double* W = work + b * (int64_t)m * n;  // column-major, W[c*m + r]
  for (int64_t e = tid; e < (int64_t)m * n; e += FT) {
    int r = (int)(e % m), c = (int)(e / m);
    W[e] = A[r * rs + c * cs];
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    double* cj = W + (int64_t)j * m;
    double part = 0.0;
    for (int r = j + 1 + tid; r < m; r += FT) part += cj[r] * cj[r];
    double sig = block_sum(part, red);  // sum of squares below the diagonal
    double x0 = cj[j];
    double tau, beta, scale;
    if (sig == 0.0) {
      tau = 0.0;
      beta = x0;
      scale = 0.0;
    } else {
      double nrm = sqrt(x0 * x0 + sig);
      beta = x0 >= 0.0 ? -nrm : nrm;
      tau = (beta - x0) / beta;
      scale = 1.0 / (x0 - beta);
    }
    __syncthreads();
    for (int r = j + 1 + tid; r < m; r += FT) cj[r] *= scale;
    if (tid == 0) {
      taus[j] = tau;
      betas[j] = beta;
    }
    __syncthreads();
    if (tau != 0.0) {
      for (int c = j + 1 + wave; c < n; c += FW) {
        double* cc = W + (int64_t)c * m;
        double p = (lane == 0) ? cc[j] : 0.0;
        for (int r = j + 1 + lane; r < m; r += 64) p += cj[r] * cc[r];
        double w = wave_sum(p) * tau;
        if (lane == 0) cc[j] -= w;
        for (int r = j + 1 + lane; r < m; r += 64) cc[r] -= w * cj[r];
      }
    }
    __syncthreads();
  }
  if (R0 != nullptr) {
    double* R = R0 + b * strideR;
    for (int e = tid; e < n * n; e += FT) {
      int r = e / n, c = e % n;
      double v = 0.0;
      if (r == c) v = betas[r];
      else if (r < c) v = W[(int64_t)c * m + r];
      R[e] = v;
    }
  }
  __syncthreads();
  for (int j = n - 1; j >= 0; --j) {
    const double tau = taus[j];
    double* cj = W + (int64_t)j * m;
    for (int c = j + 1 + wave; c < n; c += FW) {
      double* cc = W + (int64_t)c * m;
      double p = (lane == 0) ? cc[j] : 0.0;
      for (int r = j + 1 + lane; r < m; r += 64) p += cj[r] * cc[r];
      double w = wave_sum(p) * tau;
      if (lane == 0) cc[j] -= w;
      for (int r = j + 1 + lane; r < m; r += 64) cc[r] -= w * cj[r];
    }
    __syncthreads();
    for (int r = tid; r < m; r += FT) {
      double v;
      if (r < j) v = 0.0;
      else if (r == j) v = 1.0 - tau;
      else v = -tau * cj[r];
      cj[r] = v;
    }
    __syncthreads();
  }
  double* Q = Q0 + b * strideQ;
  for (int64_t e = tid; e < (int64_t)m * n; e += FT) {
    int r = (int)(e / n), c = (int)(e % n);
    Q[e] = W[(int64_t)c * m + r];
  }
}

// ---------------------------------------------------------------------------
// Symmetric PSD eigen-decomposition by one-sided (Hestenes) Jacobi on G:
// G J = U S with J accumulated; for PSD G the columns of J are eigenvectors
// and the column norms of G J the eigenvalues.  Round-robin pair ordering,
// sweeps until no pair needs a rotation.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(FT) void eig_kernel(const int* dims, const int* keep,
                                                 const double* __restrict__ G0, int64_t strideG,
                                                 int ldg, double* __restrict__ P0, int64_t strideP,
                                                 int ldp, double* __restrict__ L0, int64_t strideL,
                                                 double* __restrict__ work) {
  __shared__ int changed;
  __shared__ double nrm[1024];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t b = blockIdx.x;
  const int n = dims[b];
  const int k = keep[b];
  const double* G = G0 + b * strideG;
  double* P = P0 + b * strideP;
  double* L = L0 + b * strideL;
  double* Wm = work + b * (int64_t)ldg * ldg * 2;  // G J, column-major
  double* V = Wm + (int64_t)ldg * ldg;              // J, column-major
  if (n <= 0) return;
  for (int e = tid; e < n * n; e += FT) {
    int r = e % n, c = e / n;
    Wm[(int64_t)c * n + r] = G[(int64_t)r * ldg + c];
    V[(int64_t)c * n + r] = (r == c) ? 1.0 : 0.0;
  }
  __syncthreads();
  const int np = n + (n & 1);  // even number of players (a dummy when n is odd)
  const int K = np - 1;
  for (int sweep = 0; sweep < 40 && np > 1; ++sweep) {
    if (tid == 0) changed = 0;
    __syncthreads();
    for (int rnd = 0; rnd < K; ++rnd) {
      for (int i = wave; i < np / 2; i += FW) {
        int p, q;
        if (i == 0) { p = rnd % K; q = K; }
        else { p = (rnd + i) % K; q = (rnd + K - i) % K; }
        if (p >= n || q >= n) continue;
        double* wp = Wm + (int64_t)p * n;
        double* wq = Wm + (int64_t)q * n;
        double a = 0.0, bb = 0.0, g = 0.0;
        for (int r = lane; r < n; r += 64) {
          double x = wp[r], y = wq[r];
          a += x * x;
          bb += y * y;
          g += x * y;
        }
        a = wave_sum(a);
        bb = wave_sum(bb);
        g = wave_sum(g);
        if (fabs(g) <= 1e-15 * sqrt(a * bb) || g == 0.0) continue;
        double zeta = (bb - a) / (2.0 * g);
        double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
        for (int r = lane; r < n; r += 64) {
          double x = wp[r], y = wq[r];
          wp[r] = c * x - s * y;
          wq[r] = s * x + c * y;
        }
        double* vp = V + (int64_t)p * n;
        double* vq = V + (int64_t)q * n;
        for (int r = lane; r < n; r += 64) {
          double x = vp[r], y = vq[r];
          vp[r] = c * x - s * y;
          vq[r] = s * x + c * y;
        }
        if (lane == 0) changed = 1;
      }
      __syncthreads();
    }
    if (!changed) break;
    __syncthreads();
  }
  // eigenvalues = column norms of G J
  for (int c = wave; c < n; c += FW) {
    double s = 0.0;
    for (int r = lane; r < n; r += 64) s += Wm[(int64_t)c * n + r] * Wm[(int64_t)c * n + r];
    s = wave_sum(s);
    if (lane == 0) nrm[c] = sqrt(s);
  }
  __syncthreads();
  // rank of each column by descending eigenvalue (ties by index)
  for (int c = tid; c < n; c += FT) {
    double v = nrm[c];
    int rank = 0;
    for (int o = 0; o < n; ++o) rank += (nrm[o] > v) || (nrm[o] == v && o < c);
    L[rank] = v;
    if (rank < k)
      for (int r = 0; r < n; ++r) P[(int64_t)r * ldp + rank] = V[(int64_t)c * n + r];
  }
}

}  // namespace

void qr_launch(int count, int m, int n, const double* A, int64_t strideA, int64_t rs, int64_t cs,
               double* Q, int64_t strideQ, double* R, int64_t strideR, double* work,
               hipStream_t s) {
  if (count <= 0) return;
  QTT_REQUIRE(m >= n && n >= 1 && n <= 1024, "qr: need m >= n, 1 <= n <= 1024 (m=%d n=%d)", m, n);
  rt::check_range(A, 0, (int64_t)(count - 1) * strideA + (int64_t)(m - 1) * rs + (int64_t)(n - 1) * cs,
                  sizeof(double), "qr input");
  rt::check_range(Q, 0, (int64_t)(count - 1) * strideQ + (int64_t)m * n - 1, sizeof(double), "qr Q");
  if (R) rt::check_range(R, 0, (int64_t)(count - 1) * strideR + (int64_t)n * n - 1, sizeof(double), "qr R");
  rt::check_range(work, 0, (int64_t)count * m * n - 1, sizeof(double), "qr workspace");
  if (rt::dry()) return;
  hipLaunchKernelGGL(qr_kernel, dim3(count), dim3(FT), 0, s, m, n, A, strideA, rs, cs, Q, strideQ,
                     R, strideR, work);
  QTT_HIP(hipGetLastError());
}

void eig_launch(int count, const int* dims, const int* keep, const double* G, int64_t strideG,
                int ldg, double* P, int64_t strideP, int ldp, double* lam, int64_t strideL,
                double* work, int max_n, hipStream_t s) {
  if (count <= 0) return;
  QTT_REQUIRE(max_n <= 1024 && max_n <= ldg, "eig: n <= 1024 and n <= ldg");
  rt::check_range(dims, 0, count - 1, sizeof(int), "eig dims");
  rt::check_range(keep, 0, count - 1, sizeof(int), "eig keep");
  rt::check_range(G, 0, (int64_t)(count - 1) * strideG + (int64_t)(max_n - 1) * ldg + max_n - 1,
                  sizeof(double), "eig input");
  rt::check_range(P, 0, (int64_t)(count - 1) * strideP + (int64_t)(max_n - 1) * ldp + ldp - 1,
                  sizeof(double), "eig vectors");
  rt::check_range(lam, 0, (int64_t)(count - 1) * strideL + max_n - 1, sizeof(double), "eig values");
  rt::check_range(work, 0, (int64_t)count * 2 * ldg * ldg - 1, sizeof(double), "eig workspace");
  if (rt::dry()) return;
  hipLaunchKernelGGL(eig_kernel, dim3(count), dim3(FT), 0, s, dims, keep, G, strideG, ldg, P,
                     strideP, ldp, lam, strideL, work);
  QTT_HIP(hipGetLastError());
}

}  // namespace qtt
