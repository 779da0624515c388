// FP64 factorisation kernels: Householder QR (thin explicit Q, optional R)
// and the symmetric eigen-decomposition used by the bond truncation.
//
// One workgroup per matrix; the matrix is staged column-major in a global
// workspace (L2 resident for the sizes used here) so that each Householder
// reflector or Jacobi rotation touches contiguous columns.  Reductions over
// a column use wavefront shuffles, then one LDS slot per wavefront.
#include <cstdio>
#include <cstdlib>
#include <string>

#include "common.h"

namespace qtt {

namespace {

constexpr int FT = 256;  // threads per factorisation workgroup
constexpr int FW = FT / 64;

// Wavefront reductions of doubles without LDS traffic: four DPP steps sum
// the 16 lanes of every row (quad xor 1, quad xor 2, half-row mirror, row
// mirror; each leaves the partial sum in every lane of its group), then
// row_bcast:15 adds row 0 into row 1 and row 2 into row 3, row_bcast:31 adds
// rows 0+1 into rows 2 and 3, and lane 63, which now holds the total, is read
// into scalar registers, so every lane gets the same value.
template <int CTRL, int ROWS>
__device__ inline double dpp_move(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffull), CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROWS, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// a DPP move within rows whose every lane has a valid source: no old value
template <int CTRL>
__device__ inline double dpp_row(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)(b & 0xffffffffull), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

__device__ inline double read_lane(double x, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffull), l);
  const int hi = __builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

struct OpAdd {
  __device__ static double f(double a, double b) { return a + b; }
};
struct OpMax {
  __device__ static double f(double a, double b) { return fmax(a, b); }
};

template <class Op, int K>
__device__ inline void wave_reduce_n(double (&v)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = Op::f(v[k], dpp_row<0xB1>(v[k]));  // quad_perm [1,0,3,2]
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = Op::f(v[k], dpp_row<0x4E>(v[k]));  // quad_perm [2,3,0,1]
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = Op::f(v[k], dpp_row<0x141>(v[k]));  // row_half_mirror
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = Op::f(v[k], dpp_row<0x140>(v[k]));  // row_mirror
  // rows outside the row mask receive 0, the identity of both operations here
  // (the max is only taken over non-negative values)
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = Op::f(v[k], dpp_move<0x142, 0xA>(v[k]));  // row_bcast:15 into rows 1, 3
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = Op::f(v[k], dpp_move<0x143, 0xC>(v[k]));  // row_bcast:31 into rows 2, 3
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = read_lane(v[k], 63);
}

template <int K>
__device__ inline void wave_sum_n(double (&v)[K]) {
  wave_reduce_n<OpAdd, K>(v);
}

__device__ inline double wave_sum(double v) {
  double a[1] = {v};
  wave_sum_n<1>(a);
  return a[0];
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
// General sizes, matrix in global memory (L2): 16 wavefronts, each applying
// a reflector to QCB columns at a time (one pass over v for all of them, one
// wavefront reduction for their QCB dot products).
// ---------------------------------------------------------------------------
constexpr int QFT = 1024, QFW = QFT / 64, QCB = 4;

__device__ inline double block_sum_q(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < QFW; ++w) s += red[w];
  return s;
}

// columns c0 .. c0+QCB-1 (those < n) of the column-major W (ld m):
// a -= tau (v^T a) v with v = column j of W below row j and v_j = 1.
// Called by a whole wavefront (c0 wave-uniform).
__device__ inline void qr_apply_cols(double* W, int m, int n, int j, double tau, int c0, int lane) {
  const double* cj = W + (int64_t)j * m;
  double p[QCB];
#pragma unroll
  for (int b = 0; b < QCB; ++b) p[b] = (lane == 0 && c0 + b < n) ? W[(int64_t)(c0 + b) * m + j] : 0.0;
  for (int r = j + 1 + lane; r < m; r += 64) {
    const double vr = cj[r];
#pragma unroll
    for (int b = 0; b < QCB; ++b)
      if (c0 + b < n) p[b] = fma(vr, W[(int64_t)(c0 + b) * m + r], p[b]);
  }
  wave_sum_n<QCB>(p);
#pragma unroll
  for (int b = 0; b < QCB; ++b) {
    if (c0 + b >= n) continue;
    double* cc = W + (int64_t)(c0 + b) * m;
    const double wgt = p[b] * tau;
    if (lane == 0) cc[j] -= wgt;
    for (int r = j + 1 + lane; r < m; r += 64) cc[r] = fma(-wgt, cj[r], cc[r]);
  }
}

__global__ __launch_bounds__(QFT) void qr_kernel(int m, int n, const double* __restrict__ A0,
                                                 int64_t strideA, int64_t rs, int64_t cs,
                                                 double* __restrict__ Q0, int64_t strideQ,
                                                 double* __restrict__ R0, int64_t strideR,
                                                 double* __restrict__ work, const int* __restrict__ sq,
                                                 int ldq, int64_t istride) {
  __shared__ double red[QFW];
  __shared__ double taus[1024];
  __shared__ double betas[1024];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t b = blockIdx.x;
  {  // instance of a fused launch (grid y): shift the data, not the size table
    const int64_t io = (int64_t)blockIdx.y * istride;
    A0 = ishift(A0, io);
    Q0 = ishift(Q0, io);
    R0 = ishift(R0, io);
    work = ishift(work, io);
  }
  const double* A = A0 + b * strideA;
  double* W = work + b * (int64_t)m * n;  // column-major, W[c*m + r]
  const int ldo = ldq > 0 ? ldq : n;  // leading dimension of Q and R (launch n by default)
  if (sq != nullptr) {  // per-matrix square size
    m = n = sq[b];
    if (n <= 0) return;
  }
  for (int64_t e = tid; e < (int64_t)m * n; e += QFT) {
    int r = (int)(e % m), c = (int)(e / m);
    W[e] = A[r * rs + c * cs];
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    double* cj = W + (int64_t)j * m;
    double part = 0.0;
    for (int r = j + 1 + tid; r < m; r += QFT) part += cj[r] * cj[r];
    double sig = block_sum_q(part, red);  // sum of squares below the diagonal
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
    for (int r = j + 1 + tid; r < m; r += QFT) cj[r] *= scale;
    if (tid == 0) {
      taus[j] = tau;
      betas[j] = beta;
    }
    __syncthreads();
    if (tau != 0.0)
      for (int c0 = j + 1 + wave * QCB; c0 < n; c0 += QFW * QCB) qr_apply_cols(W, m, n, j, tau, c0, lane);
    __syncthreads();
  }
  if (R0 != nullptr) {
    double* R = R0 + b * strideR;
    for (int e = tid; e < n * n; e += QFT) {
      int r = e / n, c = e % n;
      double v = 0.0;
      if (r == c) v = betas[r];
      else if (r < c) v = W[(int64_t)c * m + r];
      R[(int64_t)r * ldo + c] = v;
    }
  }
  __syncthreads();
  for (int j = n - 1; j >= 0; --j) {
    const double tau = taus[j];
    double* cj = W + (int64_t)j * m;
    if (tau != 0.0)
      for (int c0 = j + 1 + wave * QCB; c0 < n; c0 += QFW * QCB) qr_apply_cols(W, m, n, j, tau, c0, lane);
    __syncthreads();
    for (int r = tid; r < m; r += QFT) {
      double v;
      if (r < j) v = 0.0;
      else if (r == j) v = 1.0 - tau;
      else v = -tau * cj[r];
      cj[r] = v;
    }
    __syncthreads();
  }
  double* Q = Q0 + b * strideQ;
  for (int64_t e = tid; e < (int64_t)m * n; e += QFT) {
    int r = (int)(e / n), c = (int)(e % n);
    Q[(int64_t)r * ldo + c] = W[(int64_t)c * m + r];
  }
}

// ---------------------------------------------------------------------------
// Register-resident Householder QR for m <= 64*RS, n <= QW*CPW: QW wavefronts,
// column c lives in wavefront c % QW (slot c / QW), row r in lane r % 64
// (slot r / 64).  Step k: the owner of column k builds the reflector with one
// wavefront reduction and publishes v (double-buffered LDS); one barrier;
// every wavefront applies it to its columns c > k, CH column reductions at a
// time, skipping the row slots above k where v vanishes.  Q is formed in
// place by backward accumulation.
// ---------------------------------------------------------------------------
template <int RS, int CPW, int QW, int CH>
__device__ __forceinline__ void apply_reflector(double (&a)[RS][CPW], const double (&v)[RS], double t, int k,
                                       int n, int wave, int i0) {
#pragma unroll
  for (int j0 = 0; j0 < CPW; j0 += CH) {
    const int jl = (j0 + CH - 1 < CPW) ? j0 + CH - 1 : CPW - 1;
    if (wave + QW * jl <= k) continue;  // every column of the chunk is done
    if (wave + QW * j0 >= n) break;     // past the last column
    double d[CH];
#pragma unroll
    for (int jj = 0; jj < CH; ++jj) {
      const int j = (j0 + jj < CPW) ? j0 + jj : CPW - 1;
      double p = 0.0;
#pragma unroll
      for (int i = 0; i < RS; ++i)
        if (i >= i0) p += v[i] * a[i][j];
      d[jj] = p;
    }
    wave_sum_n<CH>(d);
#pragma unroll
    for (int jj = 0; jj < CH; ++jj) {
      if (j0 + jj >= CPW) continue;
      const int j = (j0 + jj < CPW) ? j0 + jj : CPW - 1;
      const int c = wave + QW * j;
      if (c > k && c < n) {
        const double w = t * d[jj];
#pragma unroll
        for (int i = 0; i < RS; ++i)
          if (i >= i0) a[i][j] -= w * v[i];
      }
    }
  }
}

template <int RS, int CPW, int QW, int CH>
__global__ __launch_bounds__(QW * 64) void qr_reg_kernel(int m, int n, const double* __restrict__ A0,
                                                      int64_t strideA, int64_t rs, int64_t cs,
                                                      double* __restrict__ Q0, int64_t strideQ,
                                                      double* __restrict__ R0, int64_t strideR,
                                                      const int* __restrict__ sq, int ldq, int64_t istride) {
  __shared__ double vbuf[2][64 * RS];
  __shared__ double taus[QW * CPW];
  __shared__ double betas[QW * CPW];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t bi = blockIdx.x;
  {  // instance of a fused launch (grid y): shift the data, not the size table
    const int64_t io = (int64_t)blockIdx.y * istride;
    A0 = ishift(A0, io);
    Q0 = ishift(Q0, io);
    R0 = ishift(R0, io);
  }
  const double* A = A0 + bi * strideA;
  const int ldo = ldq > 0 ? ldq : n;  // leading dimension of Q and R (launch n by default)
  if (sq != nullptr) {  // per-matrix square size
    m = n = sq[bi];
    if (n <= 0) return;
  }
  double a[RS][CPW];
#pragma unroll
  for (int j = 0; j < CPW; ++j) {
    const int c = wave + QW * j;
#pragma unroll
    for (int i = 0; i < RS; ++i) {
      const int r = lane + 64 * i;
      a[i][j] = (r < m && c < n) ? A[r * rs + c * cs] : 0.0;
    }
  }
  for (int k = 0; k < n; ++k) {
    const int owner = k % QW, jk = k / QW, buf = k & 1, i0 = k >> 6;
    if (wave == owner) {
      double col[RS];
#pragma unroll
      for (int i = 0; i < RS; ++i) {
        double v = 0.0;
#pragma unroll
        for (int j = 0; j < CPW; ++j) v = (j == jk) ? a[i][j] : v;
        col[i] = v;
      }
      double part = 0.0, xk = 0.0;
#pragma unroll
      for (int i = 0; i < RS; ++i) {
        const int r = lane + 64 * i;
        if (r > k) part += col[i] * col[i];
        if (i == i0) xk = col[i];
      }
      const double sig = wave_sum(part);
      const double x0 = read_lane(xk, k & 63);
      double tau = 0.0, beta = x0, scale = 0.0;
      if (sig != 0.0) {
        const double nrm = sqrt(x0 * x0 + sig);
        beta = x0 >= 0.0 ? -nrm : nrm;
        tau = (beta - x0) / beta;
        scale = 1.0 / (x0 - beta);
      }
#pragma unroll
      for (int i = 0; i < RS; ++i) {
        const int r = lane + 64 * i;
        const double v = (r > k) ? col[i] * scale : (r == k ? 1.0 : 0.0);
        vbuf[buf][r] = v;
        if (r > k) {
#pragma unroll
          for (int j = 0; j < CPW; ++j)
            if (j == jk) a[i][j] = v;
        }
      }
      if (lane == 0) {
        taus[k] = tau;
        betas[k] = beta;
      }
    }
    __syncthreads();
    const double t = taus[k];
    if (t != 0.0) {
      double v[RS];
#pragma unroll
      for (int i = 0; i < RS; ++i) v[i] = (i >= i0) ? vbuf[buf][lane + 64 * i] : 0.0;
      apply_reflector<RS, CPW, QW, CH>(a, v, t, k, n, wave, i0);
    }
  }
  __syncthreads();
  if (R0 != nullptr) {
    double* R = R0 + bi * strideR;
#pragma unroll
    for (int j = 0; j < CPW; ++j) {
      const int c = wave + QW * j;
      if (c >= n) continue;
#pragma unroll
      for (int i = 0; i < RS; ++i) {
        const int r = lane + 64 * i;
        if (r >= n) continue;
        R[(int64_t)r * ldo + c] = (r < c) ? a[i][j] : (r == c ? betas[c] : 0.0);
      }
    }
  }
  for (int k = n - 1; k >= 0; --k) {
    const int owner = k % QW, jk = k / QW, buf = k & 1, i0 = k >> 6;
    if (wave == owner) {
#pragma unroll
      for (int i = 0; i < RS; ++i) {
        const int r = lane + 64 * i;
        double v = 0.0;
#pragma unroll
        for (int j = 0; j < CPW; ++j) v = (j == jk) ? a[i][j] : v;
        vbuf[buf][r] = (r > k) ? v : (r == k ? 1.0 : 0.0);
      }
    }
    __syncthreads();
    const double t = taus[k];
    double v[RS];
#pragma unroll
    for (int i = 0; i < RS; ++i) v[i] = (i >= i0) ? vbuf[buf][lane + 64 * i] : 0.0;
    if (t != 0.0) apply_reflector<RS, CPW, QW, CH>(a, v, t, k, n, wave, i0);
    if (wave == owner) {
#pragma unroll
      for (int i = 0; i < RS; ++i) {
        const int r = lane + 64 * i;
        const double q = (r < k) ? 0.0 : (r == k ? 1.0 - t : -t * v[i]);
#pragma unroll
        for (int j = 0; j < CPW; ++j)
          if (j == jk) a[i][j] = q;
      }
    }
  }
  double* Q = Q0 + bi * strideQ;
#pragma unroll
  for (int j = 0; j < CPW; ++j) {
    const int c = wave + QW * j;
    if (c >= n) continue;
#pragma unroll
    for (int i = 0; i < RS; ++i) {
      const int r = lane + 64 * i;
      if (r < m) Q[(int64_t)r * ldo + c] = a[i][j];
    }
  }
}

// ---------------------------------------------------------------------------
// Householder QR with one column per 16-lane group (a DPP row): for
// m <= 16*RPL, n <= 4*NW*CS.  Lane li of group g of wavefront w holds rows
// li + 16 r (r < RPL) of the columns c = (4 NW) j + 4 w + g, slots j < CS.  A
// column dot product is a sum over the 16 lanes of a group: four row-local
// DPP steps reduce the four columns of a wavefront at once and leave each
// sum in every lane of its group.  The columns of slot j form phase j; the
// slot index is a compile-time constant inside each phase, and the row
// chunks above the phase's first column (where every reflector vanishes)
// are skipped.  Factorisation, step k: one barrier, every group applies H_k
// to its columns c > k, the owner of column k+1 first to that column, then
// builds and publishes v_(k+1) before its other columns (look-ahead).  Thin
// Q by backward accumulation, phase by phase: the phase's stored reflectors
// are published at once and applied with no barrier in between.
// ---------------------------------------------------------------------------

// sum over the 16 lanes of every row, left in every lane of the row
__device__ inline double row_sum(double v) {
  v += dpp_row<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_row<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_row<0x141>(v);  // row_half_mirror
  v += dpp_row<0x140>(v);  // row_mirror
  return v;
}

// a[:, c] -= t (v^T a[:, c]) v for this lane's columns c with k < c < n, in
// the slots J0 <= j < CS with (ONLY < 0 || j == ONLY) && j != SKIP.  Slots
// below J0 hold only columns <= k; v vanishes in the row chunks r < R0.
template <int RPL, int CS, int NW, int R0, int J0, int ONLY = -1, int SKIP = -1>
__device__ __forceinline__ void grp_apply(double (&a)[CS][RPL], const double (&v)[RPL], double t, int k,
                                          int n, int w, int g) {
  constexpr int CL = 4 * NW;
#pragma unroll
  for (int j = J0; j < CS; ++j) {
    if ((ONLY >= 0 && j != ONLY) || j == SKIP) continue;
    if (CL * j + 4 * w + 3 <= k) continue;  // no column of this slot is past k
    if (CL * j + 4 * w >= n) break;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};  // four short chains instead of one long one
#pragma unroll
    for (int r = R0; r < RPL; ++r) acc[r & 3] = fma(v[r], a[j][r], acc[r & 3]);
    const double d = row_sum((acc[0] + acc[1]) + (acc[2] + acc[3]));
    const int c = CL * j + 4 * w + g;
    const double wgt = (c > k && c < n) ? t * d : 0.0;
#pragma unroll
    for (int r = R0; r < RPL; ++r) a[j][r] = fma(-wgt, v[r], a[j][r]);
  }
}

// first row chunk (16 rows) in which a reflector v_k with k >= CL*JO can be
// nonzero: every row of the chunks below lies above the diagonal
template <int CL, int JO, int RPL>
constexpr int grp_r0() {
  return (CL * JO) / 16 < RPL ? (CL * JO) / 16 : RPL;
}

// Owner wavefront of column k (slot JO, group go): builds the reflector
// H_k = I - tau v v^T from the column in place, stores v below the diagonal,
// publishes v (vb) and tau / beta.  Called by the whole wavefront.
template <int RPL, int CS, int JO, int R0>
__device__ __forceinline__ void grp_reflector(double (&a)[CS][RPL], int k, int go, int g, int li, double* vb,
                                              double* taus, double* betas) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0}, xk = 0.0;
#pragma unroll
  for (int r = R0; r < RPL; ++r) {
    const int row = li + 16 * r;
    const double x = row > k ? a[JO][r] : 0.0;
    acc[r & 3] = fma(x, x, acc[r & 3]);
    if (r == (k >> 4)) xk = a[JO][r];
  }
  const double part = row_sum((acc[0] + acc[1]) + (acc[2] + acc[3]));
  const double sig = read_lane(part, 16 * go);
  const double x0 = read_lane(xk, 16 * go + (k & 15));
  double tau = 0.0, beta = x0, scale = 0.0;
  if (sig != 0.0) {
    // beta = -sign(x0) ||x||, u = x0 - beta (no cancellation), v = x / u with
    // v_k = 1, tau = -u / beta (two divisions: a product u * beta would
    // leave the range of doubles for columns of norm below ~1e-154)
    const double nrm = sqrt(x0 * x0 + sig);
    beta = x0 >= 0.0 ? -nrm : nrm;
    const double u = x0 - beta;
    scale = 1.0 / u;
    tau = -u / beta;
  }
  if (g == go) {
#pragma unroll
    for (int r = R0; r < RPL; ++r) {
      const int row = li + 16 * r;
      const double vv = (row > k) ? a[JO][r] * scale : (row == k ? 1.0 : 0.0);
      vb[row] = vv;
      if (row > k) a[JO][r] = vv;
    }
    if (li == 0) {
      taus[k] = tau;
      betas[k] = beta;
    }
  }
}

// Calls f(std::integral_constant<int, I>) for I = B, B+1, ..., E-1 (or, with
// DOWN, for I = E-1, ..., B): the slot index becomes a compile-time constant,
// so the register array is never indexed at run time.
template <int B, int E, bool DOWN = false, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    if constexpr (DOWN) {
      f(std::integral_constant<int, E - 1>{});
      static_for<B, E - 1, true>(f);
    } else {
      f(std::integral_constant<int, B>{});
      static_for<B + 1, E, false>(f);
    }
  }
}

// QF: the workgroup may form Q itself (needs the phase buffer vall, CL x 16
// RPL doubles of LDS); launches that leave reflectors (Vout) or write R only
// take QF = false and keep their LDS to the factorisation's few kilobytes,
// so the workgroup finds room on a CU that other launches keep busy.
template <int RPL, int CS, int NW, bool QF>
__global__ __launch_bounds__(NW * 64) void qr_grp_kernel(int m, int n, const double* __restrict__ A0,
                                                       int64_t strideA, int64_t rs, int64_t cs,
                                                       double* __restrict__ Q0, int64_t strideQ,
                                                       double* __restrict__ R0, int64_t strideR,
                                                       const int* __restrict__ sq, int ldq,
                                                       double* __restrict__ Vout, double* __restrict__ tout,
                                                       int64_t istride) {
  constexpr int CL = 4 * NW;
  __shared__ double vbuf[2][16 * RPL];
  __shared__ double vall[QF ? CL : 1][QF ? 16 * RPL : 1];
  __shared__ double taus[CL * CS];
  __shared__ double betas[CL * CS];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = lane >> 4, li = lane & 15;
  const int64_t bi = blockIdx.x;
  {  // instance of a fused launch (grid y): shift the data, not the size table
    const int64_t io = (int64_t)blockIdx.y * istride;
    A0 = ishift(A0, io);
    Q0 = ishift(Q0, io);
    R0 = ishift(R0, io);
    Vout = ishift(Vout, io);
    tout = ishift(tout, io);
  }
  const double* A = A0 + bi * strideA;
  const int ldo = ldq > 0 ? ldq : n;  // leading dimension of Q and R (launch n by default)
  if (sq != nullptr) {  // per-matrix square size
    m = n = sq[bi];
    if (n <= 0) return;
  }
  double a[CS][RPL];
#pragma unroll
  for (int j = 0; j < CS; ++j) {
    const int c = CL * j + 4 * w + g;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int row = li + 16 * r;
      a[j][r] = (row < m && c < n) ? A[row * rs + c * cs] : 0.0;
    }
  }
  auto wo_of = [](int k) { return (k % CL) >> 2; };
  double v[RPL];
  // ---- factorisation, one phase per slot (columns JO*CL .. JO*CL+CL-1), with
  // look-ahead: the owner of column k+1 applies H_k to that column first and
  // publishes v_(k+1) before updating its other columns
  if (w == 0) grp_reflector<RPL, CS, 0, 0>(a, 0, 0, g, li, vbuf[0], taus, betas);
#pragma unroll
  for (int r = 0; r < RPL; ++r) v[r] = 0.0;
  static_for<0, CS>([&](auto J) {
    constexpr int JO = decltype(J)::value;
    constexpr int R0 = grp_r0<CL, JO, RPL>();
    constexpr int R1 = grp_r0<CL, JO + 1, RPL>();
    const int kend = min(n, CL * (JO + 1));
    for (int k = CL * JO; k < kend; ++k) {
      __syncthreads();  // v_k, tau_k visible
      const double t = taus[k];
#pragma unroll
      for (int r = R0; r < RPL; ++r) v[r] = vbuf[k & 1][li + 16 * r];
      const int k1 = k + 1;
      const bool own = k1 < n && w == wo_of(k1);  // wave-uniform
      // the owner's chain up to publishing v_(k+1) gates the next step: it
      // runs at raised wave priority
      if (own) __builtin_amdgcn_s_setprio(2);
      if (t != 0.0) grp_apply<RPL, CS, NW, R0, JO, JO>(a, v, t, k, n, w, g);
      if (own && k1 < CL * (JO + 1)) {
        grp_reflector<RPL, CS, JO, R0>(a, k1, k1 & 3, g, li, vbuf[k1 & 1], taus, betas);
        __builtin_amdgcn_s_setprio(0);
      }
      if constexpr (JO + 1 < CS) {
        if (t != 0.0) grp_apply<RPL, CS, NW, R0, JO + 1, JO + 1>(a, v, t, k, n, w, g);
        if (own && k1 == CL * (JO + 1)) {
          grp_reflector<RPL, CS, JO + 1, R1>(a, k1, k1 & 3, g, li, vbuf[k1 & 1], taus, betas);
          __builtin_amdgcn_s_setprio(0);
        }
        if (t != 0.0) grp_apply<RPL, CS, NW, R0, JO + 2>(a, v, t, k, n, w, g);
      }
    }
  });
  __syncthreads();
  if (R0 != nullptr) {
    double* R = R0 + bi * strideR;
#pragma unroll
    for (int j = 0; j < CS; ++j) {
      const int c = CL * j + 4 * w + g;
      if (c >= n) continue;
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        const int row = li + 16 * r;
        if (row >= n) continue;
        R[(int64_t)row * ldo + c] = (row < c) ? a[j][r] : (row == c ? betas[c] : 0.0);
      }
    }
  }
  if (Vout != nullptr) {  // panel of a blocked QR: reflectors (m x n, unit diagonal) and taus, no Q
#pragma unroll
    for (int j = 0; j < CS; ++j) {
      const int c = CL * j + 4 * w + g;
      if (c >= n) continue;
#pragma unroll
      for (int r = 0; r < RPL; ++r) {
        const int row = li + 16 * r;
        if (row < m) Vout[(int64_t)row * n + c] = (row > c) ? a[j][r] : (row == c ? 1.0 : 0.0);
      }
    }
    for (int c = threadIdx.x; c < n; c += NW * 64) tout[c] = taus[c];
    return;
  }
  if (Q0 == nullptr) return;  // R only: no Q wanted
  if constexpr (!QF) {
    return;  // never reached: launches without Q space always pass Vout or no Q
  } else {
  // ---- thin Q by backward accumulation, one slot phase at a time (in
  // reverse): the reflectors of the phase's CL columns are published together,
  // then every wavefront applies them, last to first, to its own columns with
  // no barrier in between (the owner of column k resets it to H_k e_k when its
  // turn comes; nothing else touches it)
  static_for<0, CS, true>([&](auto J) {
    constexpr int JO = decltype(J)::value;
    constexpr int R0 = grp_r0<CL, JO, RPL>();
    const int kb = CL * JO, ke = min(n, CL * (JO + 1));
    if (kb >= ke) return;  // block-uniform
    __syncthreads();  // the previous phase has finished reading vall
    {
      const int k = kb + 4 * w + g;  // this lane's column in slot JO
      if (k < ke) {
#pragma unroll
        for (int r = R0; r < RPL; ++r) {
          const int row = li + 16 * r;
          vall[k - kb][row] = (row > k) ? a[JO][r] : (row == k ? 1.0 : 0.0);
        }
      }
    }
    __syncthreads();
    for (int k = ke - 1; k >= kb; --k) {
      const double t = taus[k];
#pragma unroll
      for (int r = R0; r < RPL; ++r) v[r] = vall[k - kb][li + 16 * r];
      if (t != 0.0) grp_apply<RPL, CS, NW, R0, JO>(a, v, t, k, n, w, g);
      if (w == wo_of(k) && g == (k & 3)) {
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
          const int row = li + 16 * r;
          a[JO][r] = (r < R0 || row < k) ? 0.0 : (row == k ? 1.0 - t : -t * v[r]);
        }
      }
    }
  });
  double* Q = Q0 + bi * strideQ;
#pragma unroll
  for (int j = 0; j < CS; ++j) {
    const int c = CL * j + 4 * w + g;
    if (c >= n) continue;
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
      const int row = li + 16 * r;
      if (row < m) Q[(int64_t)row * ldo + c] = a[j][r];
    }
  }
  }
}

// ---------------------------------------------------------------------------
// Thin Q of a factorisation left as reflectors (V: m x n, row-major, unit
// diagonal, zeros above; tau: n), Q = H_0 H_1 ... H_(n-1) [I; 0], one column
// per wavefront: column c = QQ_NW blockIdx.x + w, rows lane + 64 r (r < RW).
// Column c starts as e_c and takes the reflectors from the last to the first
// (those past c leave it unchanged: v_k vanishes above row k).  Reflectors
// pass through LDS in double-buffered chunks of KC.  A column takes them in
// pairs: with a = v_k, b = v_(k-1) and q the column, the dot products a.q
// and b.q and the product a.b go through one wavefront sum, and then
//   d_a = a.q,  d_b = b.q - tau_k d_a (a.b),  q -= tau_k d_a a + tau_(k-1) d_b b,
// which is H_(k-1) H_k q.  That halves the chain of sums a column waits on;
// the next pair's vectors are read from LDS while the current sums run.
// ---------------------------------------------------------------------------
constexpr int QQ_NW = 4;  // columns (wavefronts) per workgroup

// sums of K values over the wavefront at once (the K chains interleave), in
// every lane: the four in-row steps take no old value (every lane of a row is
// valid), the two row broadcasts add into the masked rows only, and lane 63,
// which then holds the total, is read into scalar registers
template <int K>
__device__ inline void wave_sum_k(double (&x)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) x[k] += dpp_row<0xB1>(x[k]);   // quad_perm [1,0,3,2]
#pragma unroll
  for (int k = 0; k < K; ++k) x[k] += dpp_row<0x4E>(x[k]);   // quad_perm [2,3,0,1]
#pragma unroll
  for (int k = 0; k < K; ++k) x[k] += dpp_row<0x141>(x[k]);  // row_half_mirror
#pragma unroll
  for (int k = 0; k < K; ++k) x[k] += dpp_row<0x140>(x[k]);  // row_mirror
#pragma unroll
  for (int k = 0; k < K; ++k) x[k] += dpp_move<0x142, 0xA>(x[k]);  // row_bcast:15 into rows 1, 3
#pragma unroll
  for (int k = 0; k < K; ++k) x[k] += dpp_move<0x143, 0xC>(x[k]);  // row_bcast:31 into rows 2, 3
#pragma unroll
  for (int k = 0; k < K; ++k) x[k] = read_lane(x[k], 63);
}

template <int RW>
__global__ __launch_bounds__(QQ_NW * 64) void qr_q_kernel(int m, int n, const double* __restrict__ V,
                                                        const double* __restrict__ tau, double* __restrict__ Q,
                                                        int ldq, int64_t istride) {
  constexpr int NWQ = QQ_NW;
  constexpr int NT = NWQ * 64;
  constexpr int KC = RW > 5 ? 8 : 16;
  constexpr int MR = 64 * RW;
  constexpr int NPRE = KC * MR / NT;
  static_assert(NPRE * NT == KC * MR, "chunk must split evenly over the workgroup");
  __shared__ double Vs[2][KC][MR + 1];  // odd row stride: a row's KC stores land on distinct banks
  __shared__ double ts[2][KC];
  {  // instance of a fused launch (grid y)
    const int64_t io = (int64_t)blockIdx.y * istride;
    V = ishift(V, io);
    tau = ishift(tau, io);
    Q = ishift(Q, io);
  }
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int c = (int)blockIdx.x * NWQ + w;  // wave-uniform
  double q[RW];
#pragma unroll
  for (int r = 0; r < RW; ++r) q[r] = (lane + 64 * r == c) ? 1.0 : 0.0;
  // chunk with top reflector khi: element e is reflector khi - e % KC, row e / KC
  // (every element of a chunk is written: zero past row m and below k = 0)
  double pre[NPRE];
  auto load = [&](int khi) {
#pragma unroll
    for (int i = 0; i < NPRE; ++i) {
      const int e = tid + NT * i;
      const int k = khi - e % KC, row = e / KC;
      pre[i] = (k >= 0 && row < m) ? V[(int64_t)row * n + k] : 0.0;
    }
  };
  auto store = [&](int buf, int khi) {
#pragma unroll
    for (int i = 0; i < NPRE; ++i) {
      const int e = tid + NT * i;
      Vs[buf][e % KC][e / KC] = pre[i];
    }
    if (tid < KC) ts[buf][tid] = (khi - tid >= 0) ? tau[khi - tid] : 0.0;
  };
  auto vec = [&](double (&x)[RW], int buf, int kk) {
#pragma unroll
    for (int r = 0; r < RW; ++r) x[r] = Vs[buf][kk][lane + 64 * r];
  };
  int khi = min(n - 1, (int)blockIdx.x * NWQ + NWQ - 1);
  load(khi);
  store(0, khi);
  __syncthreads();
  int buf = 0;
  while (khi >= 0) {  // block-uniform
    const int knext = khi - KC;
    if (knext >= 0) load(knext);
    const int kn = min(KC, khi + 1);
    int kk = max(0, khi - c);  // H_k with k > c leaves column c unchanged
    // pair step on (a, b) = (v_k, v_(k-1)) of this chunk, reading the next
    // pair into (na, nb) meanwhile (indices clamped into the chunk)
    auto pair = [&](const double (&a)[RW], const double (&b)[RW], double (&na)[RW], double (&nb)[RW])
        __attribute__((always_inline)) {
      const double ta = ts[buf][kk], tb = ts[buf][kk + 1];
      double x[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int r = 0; r < RW; ++r) {
        x[0] = fma(a[r], q[r], x[0]);
        x[1] = fma(b[r], q[r], x[1]);
        x[2] = fma(a[r], b[r], x[2]);
      }
      vec(na, buf, min(kk + 2, KC - 1));
      vec(nb, buf, min(kk + 3, KC - 1));
      wave_sum_k<3>(x);
      const double wa = ta * x[0];
      const double wb = tb * (x[1] - wa * x[2]);
#pragma unroll
      for (int r = 0; r < RW; ++r) q[r] = fma(-wb, b[r], fma(-wa, a[r], q[r]));
      kk += 2;
    };
    auto single = [&](const double (&a)[RW]) __attribute__((always_inline)) {
      double x[1] = {0.0};
#pragma unroll
      for (int r = 0; r < RW; ++r) x[0] = fma(a[r], q[r], x[0]);
      wave_sum_k<1>(x);
      const double wa = ts[buf][kk] * x[0];
#pragma unroll
      for (int r = 0; r < RW; ++r) q[r] = fma(-wa, a[r], q[r]);
    };
    if (kk < kn) {  // wave-uniform
      double a[RW], b[RW], na[RW], nb[RW];
      vec(a, buf, kk);
      vec(b, buf, min(kk + 1, KC - 1));
      for (;;) {  // pairs, alternating between the two register sets
        if (kk + 1 >= kn) {
          if (kk < kn) single(a);
          break;
        }
        pair(a, b, na, nb);
        if (kk + 1 >= kn) {
          if (kk < kn) single(na);
          break;
        }
        pair(na, nb, a, b);
      }
    }
    if (knext >= 0) store(buf ^ 1, knext);
    __syncthreads();
    buf ^= 1;
    khi = knext;
  }
  if (c < n) {
#pragma unroll
    for (int r = 0; r < RW; ++r) {
      const int row = lane + 64 * r;
      if (row < m) Q[(int64_t)row * ldq + c] = q[r];
    }
  }
}

// ---------------------------------------------------------------------------
// Symmetric PSD eigen-decomposition by one-sided (Hestenes) Jacobi, general
// sizes, columns in global memory (L2), 16 wavefronts.  Either from W = G,
// V = I, or (preconditioned) from W = R^T, V = Q where G = Q1 R^T Q^T comes
// from two QR factorisations (Q, R1, R2 as eig_precondition_launch leaves
// them): W is then R2 itself (its row c is column c of W) and V is written
// into R1's space, which the second factorisation no longer needs.  Round-
// robin pair ordering; a pair is left alone when its cross product is below
// 1e-15 |w_p| |w_q| or below the noise of the columns, u * lambda_max *
// max(|w_p|, |w_q|) (compared in squares); sweeps until no pair rotates.  For
// PSD G the columns of V J are eigenvectors and the column norms of W J the
// eigenvalues.
// ---------------------------------------------------------------------------
constexpr int EFT = 1024, EFW = EFT / 64;

__global__ __launch_bounds__(EFT) void eig_kernel(const int* dims, const int* keep,
                                                  const double* __restrict__ G0, int64_t strideG,
                                                  int ldg, double* __restrict__ P0, int64_t strideP,
                                                  int ldp, double* __restrict__ L0, int64_t strideL,
                                                  double* __restrict__ work, double unoise,
                                                  const double* __restrict__ Qp, double* __restrict__ R1p,
                                                  double* __restrict__ R2p, int64_t strideQR, int ldqr,
                                                  int64_t istride) {
  __shared__ int changed;
  __shared__ double gmax;
  __shared__ double nrm[1024];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t b = blockIdx.x;
  {  // instance of a fused launch (grid y): shift the data, not the size tables
    const int64_t io = (int64_t)blockIdx.y * istride;
    G0 = ishift(G0, io);
    P0 = ishift(P0, io);
    L0 = ishift(L0, io);
    work = ishift(work, io);
    Qp = ishift(Qp, io);
    R1p = ishift(R1p, io);
    R2p = ishift(R2p, io);
  }
  const int n = dims[b];
  const int k = keep[b];
  if (n <= 0) return;
  const double* G = G0 + b * strideG;
  double* P = P0 + b * strideP;
  double* L = L0 + b * strideL;
  double *Wm, *V;
  int ld;
  if (Qp != nullptr) {
    const double* Q = Qp + b * strideQR;
    Wm = R2p + b * strideQR;
    V = R1p + b * strideQR;
    ld = ldqr;
    for (int e = tid; e < n * n; e += EFT) {
      const int r = e % n, c = e / n;
      V[(int64_t)c * ld + r] = Q[(int64_t)r * ldqr + c];
    }
  } else {
    Wm = work + b * (int64_t)ldg * ldg * 2;  // G J, column-major
    V = Wm + (int64_t)ldg * ldg;             // J, column-major
    ld = n;
    for (int e = tid; e < n * n; e += EFT) {
      const int r = e % n, c = e / n;
      Wm[(int64_t)c * ld + r] = G[(int64_t)r * ldg + c];
      V[(int64_t)c * ld + r] = (r == c) ? 1.0 : 0.0;
    }
  }
  __syncthreads();
  const int np = n + (n & 1);  // even number of players (a dummy when n is odd)
  const int K = np - 1;
  for (int sweep = 0; sweep < 40 && np > 1; ++sweep) {
    // largest squared column norm: the noise level of this sweep
    for (int c = wave; c < n; c += EFW) {
      double sq = 0.0;
      for (int r = lane; r < n; r += 64) sq += Wm[(int64_t)c * ld + r] * Wm[(int64_t)c * ld + r];
      sq = wave_sum(sq);
      if (lane == 0) nrm[c] = sq;
    }
    if (tid == 0) changed = 0;
    __syncthreads();
    if (tid == 0) {
      double mx = 0.0;
      for (int c = 0; c < n; ++c) mx = fmax(mx, nrm[c]);
      gmax = mx;
    }
    __syncthreads();
    const double gf2 = unoise * unoise * gmax;
    for (int rnd = 0; rnd < K; ++rnd) {
      for (int i = wave; i < np / 2; i += EFW) {
        int p, q;
        if (i == 0) { p = rnd % K; q = K; }
        else { p = (rnd + i) % K; q = (rnd + K - i) % K; }
        if (p >= n || q >= n) continue;
        double* wp = Wm + (int64_t)p * ld;
        double* wq = Wm + (int64_t)q * ld;
        double s3[3] = {0.0, 0.0, 0.0};
#pragma unroll 4
        for (int r = lane; r < n; r += 64) {
          const double x = wp[r], y = wq[r];
          s3[0] = fma(x, x, s3[0]);
          s3[1] = fma(y, y, s3[1]);
          s3[2] = fma(x, y, s3[2]);
        }
        wave_sum_n<3>(s3);
        const double a = s3[0], bb = s3[1], g = s3[2];
        const double g2 = g * g;
        if (!(g2 > 1e-30 * a * bb && g2 > gf2 * fmax(a, bb))) continue;
        const double zeta = (bb - a) / (2.0 * g);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
#pragma unroll 4
        for (int r = lane; r < n; r += 64) {
          const double x = wp[r], y = wq[r];
          wp[r] = c * x - s * y;
          wq[r] = s * x + c * y;
        }
        double* vp = V + (int64_t)p * ld;
        double* vq = V + (int64_t)q * ld;
#pragma unroll 4
        for (int r = lane; r < n; r += 64) {
          const double x = vp[r], y = vq[r];
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
  // eigenvalues = column norms of W J
  for (int c = wave; c < n; c += EFW) {
    double sq = 0.0;
    for (int r = lane; r < n; r += 64) sq += Wm[(int64_t)c * ld + r] * Wm[(int64_t)c * ld + r];
    sq = wave_sum(sq);
    if (lane == 0) nrm[c] = sqrt(sq);
  }
  __syncthreads();
  // rank of each column by descending eigenvalue (ties by index)
  for (int c = tid; c < n; c += EFT) {
    const double v = nrm[c];
    int rank = 0;
    for (int o = 0; o < n; ++o) rank += (nrm[o] > v) || (nrm[o] == v && o < c);
    L[rank] = v;
    if (rank < k)
      for (int r = 0; r < n; ++r) P[(int64_t)r * ldp + rank] = V[(int64_t)c * ld + r];
  }
}

// ---------------------------------------------------------------------------
// Register-resident one-sided Jacobi for PSD G (n <= 2*NW*PPW, n <= 64*RS):
// the n columns of W = G J and of V = J are held as NP = ceil(n/2) column
// pairs ("slots"), PPW slots per wavefront, rows across lanes.  Each round
// rotates every pair: one wavefront reduction per pair for the cross product
// g = w_p . w_q (all PPW of a wavefront reduced together); the squared column
// norms are kept in LDS by column id, measured at the start of every sweep
// and updated exactly by each rotation (a' = a - t g, b' = b + t g).  Then
// the columns move one slot around the round-robin circle (slot 0 top fixed):
// within a wavefront by register moves, across wavefronts through a
// double-buffered LDS hand-off, one barrier per round.  2 NP - 1 rounds make
// a sweep in which every pair of columns meets once; sweeps repeat until no
// pair needs a rotation.
// ---------------------------------------------------------------------------
// Sums over the wavefront of 8 values at once, in transposed form.  Each
// step exchanges half of the values still in flight with the partner lanes
// and adds, so the count halves: the permlane swaps of gfx950 trade the
// upper half (S = 32) or the odd rows (S = 16) of one register for the lower
// half or even rows of another (one instruction per 32 bits for two
// values), then a rotation by 8 within each row; the one value left is
// summed over its 8-lane group by three in-row DPP steps.  On return lane l
// holds the total of value j = l5 + 2 l4 + 4 l3 (bits of l), identical in
// the 8 lanes of its group.
template <int S>
__device__ inline double swap_sum(double a, double b) {  // lanes of the lower half / even rows: a, others: b
  const unsigned long long ua = (unsigned long long)__double_as_longlong(a);
  const unsigned long long ub = (unsigned long long)__double_as_longlong(b);
  const unsigned alo = (unsigned)(ua & 0xffffffffull), ahi = (unsigned)(ua >> 32);
  const unsigned blo = (unsigned)(ub & 0xffffffffull), bhi = (unsigned)(ub >> 32);
  auto sw = [](unsigned u, unsigned v) {
    if constexpr (S == 32) return __builtin_amdgcn_permlane32_swap(u, v, false, false);
    else return __builtin_amdgcn_permlane16_swap(u, v, false, false);
  };
  const auto l = sw(alo, blo), h = sw(ahi, bhi);
  const double p = __longlong_as_double((long long)(((unsigned long long)h[0] << 32) | l[0]));
  const double q = __longlong_as_double((long long)(((unsigned long long)h[1] << 32) | l[1]));
  return p + q;
}

__device__ inline double transposed_sum8(const double (&x)[8]) {
  const double y0 = swap_sum<32>(x[0], x[1]), y1 = swap_sum<32>(x[2], x[3]);
  const double y2 = swap_sum<32>(x[4], x[5]), y3 = swap_sum<32>(x[6], x[7]);
  const double z0 = swap_sum<16>(y0, y1), z1 = swap_sum<16>(y2, y3);
  // lanes with bit 3 set keep z1 and send z0, the others the reverse; row_ror:8
  // reads the register of the lane 8 apart in the row
  const bool hi8 = (threadIdx.x & 8) != 0;
  double w = (hi8 ? z1 : z0) + dpp_row<0x128>(hi8 ? z0 : z1);
  w += dpp_row<0xB1>(w);                      // quad_perm [1,0,3,2]
  w += dpp_row<0x4E>(w);                      // quad_perm [2,3,0,1]
  w += dpp_row<0x141>(w);                     // row_half_mirror
  return w;
}

// first lane of the group holding value j after transposed_sum8
constexpr int eig_lane_of(int j) { return 32 * (j & 1) + 16 * ((j >> 1) & 1) + 8 * ((j >> 2) & 1); }

template <int RS, int PPW, int NW, int CH>
__global__ __launch_bounds__(NW * 64) void eig_reg_kernel(const int* dims, const int* keep,
                                                          const double* __restrict__ G0,
                                                          int64_t strideG, int ldg,
                                                          double* __restrict__ P0, int64_t strideP,
                                                          int ldp, double* __restrict__ L0,
                                                          int64_t strideL, double unoise,
                                                          const double* __restrict__ Q0,
                                                          const double* __restrict__ R0,
                                                          int64_t strideQR, int ldqr, int64_t istride) {
  __shared__ double xT[2][NW][2][64 * RS];  // outgoing last top column (W, V) per wave
  __shared__ double xB[2][NW][2][64 * RS];  // outgoing first bottom column (W, V) per wave
  __shared__ int xTid[2][NW], xBid[2][NW];
  __shared__ int rot_any;
  __shared__ double cn[2 * NW * PPW + 2];  // squared column norms (later eigenvalues) by id
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t bi = blockIdx.x;
  {  // instance of a fused launch (grid y): shift the data, not the size tables
    const int64_t io = (int64_t)blockIdx.y * istride;
    G0 = ishift(G0, io);
    P0 = ishift(P0, io);
    L0 = ishift(L0, io);
    Q0 = ishift(Q0, io);
    R0 = ishift(R0, io);
  }
  const int n = dims[bi];
  const int kk = keep[bi];
  if (n <= 0) return;
  const double* G = G0 + bi * strideG;
  double* P = P0 + bi * strideP;
  double* L = L0 + bi * strideL;
  const int NP = (n + 1) / 2;
  const int p0 = w * PPW;
  double wt[PPW][RS], wb[PPW][RS], vt[PPW][RS], vb[PPW][RS];
  int it[PPW], ib[PPW];
  // Starting point: W = G, V = I; or, given G = Q1 R^T Q^T with Q1, Q
  // orthogonal and R upper triangular (Q and R passed, n x n, row-major, ld
  // ldqr), W = R^T and V = Q.  Then W J = U S makes G = (Q1 U) S (Q J)^T an
  // SVD of G; G being symmetric PSD, the columns of V J = Q J are its
  // eigenvectors and the column norms of W J its eigenvalues.  The columns
  // of R^T are graded and far closer to orthogonal than those of G, which
  // cuts the number of sweeps.
  const double* Qb = Q0 ? Q0 + bi * strideQR : nullptr;
  const double* Rb = Q0 ? R0 + bi * strideQR : nullptr;
  auto w_at = [&](int r, int c) -> double {
    return Qb ? Rb[(int64_t)c * ldqr + r] : G[(int64_t)r * ldg + c];
  };
  auto v_at = [&](int r, int c) -> double {
    return Qb ? Qb[(int64_t)r * ldqr + c] : (r == c ? 1.0 : 0.0);
  };
  // initial circle: pair p = (p, 2NP - 1 - p); id n (odd n) is a zero column
#pragma unroll
  for (int j = 0; j < PPW; ++j) {
    const int p = p0 + j;
    it[j] = p;
    ib[j] = 2 * NP - 1 - p;
#pragma unroll
    for (int i = 0; i < RS; ++i) {
      const int r = lane + 64 * i;
      const bool okr = r < n;
      wt[j][i] = (okr && p < NP && it[j] < n) ? w_at(r, it[j]) : 0.0;
      wb[j][i] = (okr && p < NP && ib[j] < n) ? w_at(r, ib[j]) : 0.0;
      vt[j][i] = (okr && p < NP && it[j] < n) ? v_at(r, it[j]) : (r == it[j] ? 1.0 : 0.0);
      vb[j][i] = (okr && p < NP && ib[j] < n) ? v_at(r, ib[j]) : (r == ib[j] ? 1.0 : 0.0);
    }
  }
  const int rounds = 2 * NP - 1;
  int parity = 0;
  for (int sweep = 0; sweep < 40; ++sweep) {
    // exact squared norms of every column
#pragma unroll
    for (int j0 = 0; j0 < PPW; j0 += CH) {
      double nn[2 * CH];
#pragma unroll
      for (int jj = 0; jj < CH; ++jj) {
        const int j = (j0 + jj < PPW) ? j0 + jj : PPW - 1;
        double a = 0.0, b = 0.0;
#pragma unroll
        for (int i = 0; i < RS; ++i) {
          a += wt[j][i] * wt[j][i];
          b += wb[j][i] * wb[j][i];
        }
        nn[2 * jj] = a;
        nn[2 * jj + 1] = b;
      }
      wave_sum_n<2 * CH>(nn);
      if (lane == 0) {
#pragma unroll
        for (int jj = 0; jj < CH; ++jj) {
          const int j = (j0 + jj < PPW) ? j0 + jj : PPW - 1;
          if (j0 + jj >= PPW || p0 + j >= NP) continue;
          cn[it[j]] = nn[2 * jj];
          cn[ib[j]] = nn[2 * jj + 1];
        }
      }
    }
    if (threadIdx.x == 0) rot_any = 0;
    __syncthreads();
    // a rotation is skipped when the cross product is below the noise of the
    // columns, u * lambda_max * max(|w_p|, |w_q|) with u the relative noise of
    // G (its precision), or below 1e-15 |w_p| |w_q|; compared in squares
    double gf2;
    {
      double mx[1] = {0.0};
      for (int o = lane; o < 2 * NP; o += 64) mx[0] = fmax(mx[0], cn[o]);
      wave_reduce_n<OpMax, 1>(mx);
      gf2 = unoise * unoise * mx[0];
    }
    int rotated = 0;
    for (int rd = 0; rd < rounds; ++rd) {
      // ---- cross products of every pair of this wavefront, and the rotation
      // of pair j (t = tan of the angle that makes the pair orthogonal, the
      // root of smaller modulus) computed by one lane holding its sum
      double rc = 1.0, rs = 0.0;
      int jl = 0;     // pair whose rotation this lane computes
      bool rl = false;
      double gg = 0.0;
      if constexpr (PPW >= 4) {
        // sums in transposed form: value j ends in the 8 lanes whose bits
        // 5, 4, 3 spell j (eig_lane_of), each sum through fewer steps
        double x[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          double d = 0.0;
          if (j < PPW) {
#pragma unroll
            for (int i = 0; i < RS; ++i) d += wt[j][i] * wb[j][i];
          }
          x[j] = d;
        }
        gg = transposed_sum8(x);
        jl = ((lane >> 5) & 1) | (((lane >> 4) & 1) << 1) | (((lane >> 3) & 1) << 2);
        rl = (lane & 7) == 0 && jl < PPW;
      } else {
        double g[PPW];
#pragma unroll
        for (int j0 = 0; j0 < PPW; j0 += CH) {
          double gc[CH];
#pragma unroll
          for (int jj = 0; jj < CH; ++jj) {
            const int j = (j0 + jj < PPW) ? j0 + jj : PPW - 1;
            double x = 0.0;
#pragma unroll
            for (int i = 0; i < RS; ++i) x += wt[j][i] * wb[j][i];
            gc[jj] = x;
          }
          wave_sum_n<CH>(gc);
#pragma unroll
          for (int jj = 0; jj < CH; ++jj)
            if (j0 + jj < PPW) g[j0 + jj] = gc[jj];
        }
#pragma unroll
        for (int j = 0; j < PPW; ++j)
          if (lane == j) gg = g[j];
        jl = lane;
        rl = lane < PPW;
      }
      {
        int idt = 0, idb = 0;
#pragma unroll
        for (int j = 0; j < PPW; ++j)
          if (jl == j) {
            idt = it[j];
            idb = ib[j];
          }
        if (rl && p0 + jl < NP) {
          const double a = cn[idt], b = cn[idb];
          const double g2 = gg * gg;
          if (g2 > 1e-30 * a * b && g2 > gf2 * fmax(a, b)) {
            const double dd = b - a;
            const double r = sqrt(dd * dd + 4.0 * g2);
            const double t = (dd >= 0.0 ? 2.0 * gg : -2.0 * gg) / (fabs(dd) + r);
            rc = 1.0 / sqrt(1.0 + t * t);
            rs = rc * t;
            cn[idt] = fmax(a - t * gg, 0.0);
            cn[idb] = fmax(b + t * gg, 0.0);
          }
        }
      }
#pragma unroll
      for (int j = 0; j < PPW; ++j) {
        const int lj = PPW >= 4 ? eig_lane_of(j) : j;
        const double c = read_lane(rc, lj), s = read_lane(rs, lj);
        if (s == 0.0) continue;
#pragma unroll
        for (int i = 0; i < RS; ++i) {
          const double x = wt[j][i], y = wb[j][i];
          wt[j][i] = c * x - s * y;
          wb[j][i] = s * x + c * y;
          const double u = vt[j][i], z = vb[j][i];
          vt[j][i] = c * u - s * z;
          vb[j][i] = s * u + c * z;
        }
        rotated = 1;
      }
      if (NP == 1) continue;  // a single pair never moves
      // ---- move one slot around the circle
#pragma unroll
      for (int i = 0; i < RS; ++i) {
        xT[parity][w][0][lane + 64 * i] = wt[PPW - 1][i];
        xT[parity][w][1][lane + 64 * i] = vt[PPW - 1][i];
        xB[parity][w][0][lane + 64 * i] = wb[0][i];
        xB[parity][w][1][lane + 64 * i] = vb[0][i];
      }
      if (lane == 0) {
        xTid[parity][w] = it[PPW - 1];
        xBid[parity][w] = ib[0];
      }
      __syncthreads();
      const int wl = (w > 0) ? w - 1 : 0, wr = (w < NW - 1) ? w + 1 : w;
      // bottoms move left: slot p takes the bottom of p+1; the last slot its own top
#pragma unroll
      for (int j = 0; j < PPW; ++j) {
        const int p = p0 + j;
        if (p >= NP) continue;
        if (p == NP - 1) {
#pragma unroll
          for (int i = 0; i < RS; ++i) {
            wb[j][i] = wt[j][i];
            vb[j][i] = vt[j][i];
          }
          ib[j] = it[j];
        } else if (j + 1 < PPW) {
          const int jn = (j + 1 < PPW) ? j + 1 : j;
#pragma unroll
          for (int i = 0; i < RS; ++i) {
            wb[j][i] = wb[jn][i];
            vb[j][i] = vb[jn][i];
          }
          ib[j] = ib[jn];
        } else {
#pragma unroll
          for (int i = 0; i < RS; ++i) {
            wb[j][i] = xB[parity][wr][0][lane + 64 * i];
            vb[j][i] = xB[parity][wr][1][lane + 64 * i];
          }
          ib[j] = __builtin_amdgcn_readfirstlane(xBid[parity][wr]);
        }
      }
      // tops move right: slot 0 fixed, slot 1 takes the old bottom of slot 0
#pragma unroll
      for (int j = PPW - 1; j >= 0; --j) {
        const int p = p0 + j;
        if (p >= NP || p == 0) continue;
        if (p == 1) {
#pragma unroll
          for (int i = 0; i < RS; ++i) {
            wt[j][i] = xB[parity][0][0][lane + 64 * i];
            vt[j][i] = xB[parity][0][1][lane + 64 * i];
          }
          it[j] = __builtin_amdgcn_readfirstlane(xBid[parity][0]);
        } else if (j >= 1) {
          const int jp = (j >= 1) ? j - 1 : 0;
#pragma unroll
          for (int i = 0; i < RS; ++i) {
            wt[j][i] = wt[jp][i];
            vt[j][i] = vt[jp][i];
          }
          it[j] = it[jp];
        } else {
#pragma unroll
          for (int i = 0; i < RS; ++i) {
            wt[j][i] = xT[parity][wl][0][lane + 64 * i];
            vt[j][i] = xT[parity][wl][1][lane + 64 * i];
          }
          it[j] = __builtin_amdgcn_readfirstlane(xTid[parity][wl]);
        }
      }
      parity ^= 1;
    }
    if (rotated && lane == 0) rot_any = 1;
    __syncthreads();
    const int any = rot_any;
    __syncthreads();
    if (!any) break;
  }
  // eigenvalues: column norms of W (PSD: |G v| = lambda)
#pragma unroll
  for (int j0 = 0; j0 < PPW; j0 += CH) {
    double nn[2 * CH];
#pragma unroll
    for (int jj = 0; jj < CH; ++jj) {
      const int j = (j0 + jj < PPW) ? j0 + jj : PPW - 1;
      double a = 0.0, b = 0.0;
#pragma unroll
      for (int i = 0; i < RS; ++i) {
        a += wt[j][i] * wt[j][i];
        b += wb[j][i] * wb[j][i];
      }
      nn[2 * jj] = a;
      nn[2 * jj + 1] = b;
    }
    wave_sum_n<2 * CH>(nn);
    if (lane == 0) {
#pragma unroll
      for (int jj = 0; jj < CH; ++jj) {
        const int j = (j0 + jj < PPW) ? j0 + jj : PPW - 1;
        if (j0 + jj >= PPW || p0 + j >= NP) continue;
        cn[it[j]] = sqrt(nn[2 * jj]);
        cn[ib[j]] = sqrt(nn[2 * jj + 1]);
      }
    }
  }
  __syncthreads();
  // rank by descending eigenvalue (ties by index); dummy column n excluded
#pragma unroll
  for (int j = 0; j < PPW; ++j) {
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      if (p0 + j >= NP) continue;
      const int id = half ? ib[j] : it[j];
      if (id >= n) continue;
      const double v = cn[id];
      int cnt = 0;
      for (int o = lane; o < n; o += 64) cnt += (cn[o] > v) || (cn[o] == v && o < id);
      double cd[1] = {(double)cnt};
      wave_sum_n<1>(cd);
      cnt = (int)cd[0];
      if (lane == 0) L[cnt] = v;
      if (cnt < kk) {
#pragma unroll
        for (int i = 0; i < RS; ++i) {
          const int r = lane + 64 * i;
          if (r < n) P[(int64_t)r * ldp + cnt] = half ? vb[j][i] : vt[j][i];
        }
      }
    }
  }
}

}  // namespace

// register-resident configurations, tried in order: (rows per lane, columns
// per wave, waves, reduction chunk) and (rows per lane, pairs per wave,
// waves, reduction chunk); larger problems use the global-memory kernels
#define QTT_QR_CONFIGS(X) X(1, 1, 16, 1) X(2, 2, 16, 2)
// one column per 16-lane group: (rows per lane, column slots, waves)
#define QTT_QRG_CONFIGS(X) \
  X(2, 1, 8) X(4, 2, 8) X(8, 4, 8) X(9, 5, 8) X(12, 3, 8) X(16, 4, 8) X(16, 5, 8) X(18, 5, 8) X(36, 1, 8)
// larger than the group configurations
#define QTT_QR_CONFIGS_LARGE(X) X(5, 10, 16, 2)
#define QTT_EIG_CONFIGS(X) \
  X(1, 1, 4, 1) X(1, 2, 8, 2) X(1, 4, 8, 4) X(2, 4, 8, 4) X(2, 8, 8, 4) X(3, 6, 12, 2)

// the register kernels take matrices of at most this many columns; wider
// ones go to the group kernel, whose reflector and thin-Q launches are faster
// from 32 columns on (32 x 32: 25 against 40 us; 64 x 64: 53 against 142 us)
constexpr int QR_REG_MAXN = 16;

std::string qr_kernel_name(int m, int n) {
  char b[64];
#define QTT_QR_NAME(RS_, CPW_, NW_, CH_)                                              \
  if (m <= 64 * RS_ && n <= NW_ * CPW_ && n <= QR_REG_MAXN) {                        \
    snprintf(b, sizeof b, "qr_reg_kernel<%d, %d, %d, %d>", RS_, CPW_, NW_, CH_); \
    return b;                                                                         \
  }
  QTT_QR_CONFIGS(QTT_QR_NAME)
#undef QTT_QR_NAME
#define QTT_QRG_NAME(RPL_, CS_, NW_)                                                \
  if (m <= 16 * RPL_ && n <= 4 * NW_ * CS_) {                                       \
    snprintf(b, sizeof b, "qr_grp_kernel<%d, %d, %d>", RPL_, CS_, NW_);             \
    return b;                                                                       \
  }
  QTT_QRG_CONFIGS(QTT_QRG_NAME)
#undef QTT_QRG_NAME
#define QTT_QR_NAME(RS_, CPW_, NW_, CH_)                                              \
  if (m <= 64 * RS_ && n <= NW_ * CPW_) {                                             \
    snprintf(b, sizeof b, "qr_reg_kernel<%d, %d, %d, %d>", RS_, CPW_, NW_, CH_); \
    return b;                                                                         \
  }
  QTT_QR_CONFIGS_LARGE(QTT_QR_NAME)
#undef QTT_QR_NAME
  return "qr_kernel";
}

std::string eig_kernel_name(int max_n) {
  char b[64];
#define QTT_EIG_NAME(RS_, PPW_, NW_, CH_)                                               \
  if (max_n <= 64 * RS_ && max_n <= 2 * NW_ * PPW_) {                                   \
    snprintf(b, sizeof b, "eig_reg_kernel<%d, %d, %d, %d>", RS_, PPW_, NW_, CH_); \
    return b;                                                                           \
  }
  QTT_EIG_CONFIGS(QTT_EIG_NAME)
#undef QTT_EIG_NAME
  return "eig_kernel";
}

namespace {

// ---------------------------------------------------------------------------
// Blocked Householder QR of one m x n matrix (m <= 576) too wide for the
// register kernels: 32-column panels factorised in registers (reflectors
// and taus written out), the compact WY form Q_p = I - V T V^T of each
// panel (T upper triangular from V^T V and the taus), the trailing columns
// updated by Q_p^T with three FP64 contractions across the chip, and the thin
// Q accumulated backwards from [I; 0] by the same blocks.  R is the factored
// upper triangle.
// ---------------------------------------------------------------------------
constexpr int QB = 32;       // panel width
constexpr int QB_MAXM = 576; // rows of the register panel kernel (16 * 36)

// dst[r * ldd + c] = src[r * rs + c * cs], r < m, c < n
__global__ void qrb_copy_kernel(double* __restrict__ dst, int ldd, const double* __restrict__ src, int64_t rs,
                                int64_t cs, int m, int n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)m * n) return;
  const int r = (int)(e / n), c = (int)(e % n);
  dst[(int64_t)r * ldd + c] = src[r * rs + c * cs];
}

// Q (m x n, ld ldq) = [I; 0]
__global__ void qrb_eye_kernel(double* __restrict__ Q, int ldq, int m, int n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)m * n) return;
  const int r = (int)(e / n), c = (int)(e % n);
  Q[(int64_t)r * ldq + c] = (r == c) ? 1.0 : 0.0;
}

// R (n x n, ld ldr) = upper triangle of W (ld n)
__global__ void qrb_upper_kernel(double* __restrict__ R, int ldr, const double* __restrict__ W, int n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int r = (int)(e / n), c = (int)(e % n);
  R[(int64_t)r * ldr + c] = (r <= c) ? W[(int64_t)r * n + c] : 0.0;
}

// T (w x w, ld w, upper triangular) of the compact WY form of w reflectors
// with Gram matrix S = V^T V (w x w, ld w): T_ii = tau_i and, for j > i,
// T_ij = -tau_j sum_(i <= k < j) T_ik S_kj.  Row i needs only its own earlier
// entries, so thread i builds it alone (no barriers).
__global__ __launch_bounds__(64) void qrb_t_kernel(const double* __restrict__ S, int w,
                                                   const double* __restrict__ taus, double* __restrict__ T) {
  __shared__ double Ss[QB][QB + 1];
  for (int e = threadIdx.x; e < w * w; e += 64) Ss[e / w][e % w] = S[e];
  __syncthreads();
  const int i = threadIdx.x;
  if (i >= w) return;
  double t[QB];
#pragma unroll
  for (int j = 0; j < QB; ++j) t[j] = 0.0;
#pragma unroll
  for (int j = 0; j < QB; ++j) {
    if (j < i || j >= w) continue;
    if (j == i) {
      t[j] = taus[j];
      continue;
    }
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < QB; ++k)
      if (k >= i && k < j) acc = fma(t[k], Ss[k][j], acc);
    t[j] = -taus[j] * acc;
  }
#pragma unroll
  for (int j = 0; j < QB; ++j)
    if (j < w) T[(int64_t)i * w + j] = t[j];
}

// C = alpha op(A) op(B) + beta C in FP64, K split when that helps (partials in `part`)
void qrb_gemm(TcDesc d, double* part, hipStream_t s) {
  d.ksplit = tc_choose_ksplit(d, Prec::F64);
  if (tc_uses_part(d)) d.part = part;
  tc_launch(d, Prec::F64, s);
}

void qr_blocked(int m, int n, const double* A, int64_t rs, int64_t cs, double* Q, int ldq, double* R, double* work,
                hipStream_t s) {
  double* W = work;                          // m x n, ld n
  double* Vall = W + (int64_t)m * n;         // panels' reflectors, compact, (m - p0) x w each
  double* Tall = Vall + (int64_t)m * n;      // QB x QB per panel
  double* taus = Tall + (int64_t)n * QB;     // n
  double* W1 = taus + n;                     // QB x n
  double* W2 = W1 + (int64_t)QB * n;         // QB x n
  double* part = W2 + (int64_t)QB * n;       // K-split partials, <= 64 * QB * n
  auto grid = [](int64_t tot) { return dim3((unsigned)((tot + 255) / 256)); };
  const bool run = !rt::dry();  // dry runs validate the contractions' ranges only
  if (run) {
    hipLaunchKernelGGL(qrb_copy_kernel, grid((int64_t)m * n), dim3(256), 0, s, W, n, A, rs, cs, m, n);
    QTT_HIP(hipGetLastError());
  }
  std::vector<int64_t> voff;
  int64_t vo = 0;
  for (int p0 = 0; p0 < n; p0 += QB) {
    const int w = std::min(QB, n - p0), mr = m - p0;
    double* Vp = Vall + vo;
    double* Tp = Tall + (int64_t)p0 * QB;
    voff.push_back(vo);
    vo += (int64_t)mr * w;
    double* Wp = W + (int64_t)p0 * n + p0;
    // panel: reflectors to Vp, taus, its R block (w x w, ld n) to W2, then into W
    if (run) {
      hipLaunchKernelGGL((qr_grp_kernel<36, 1, 8, false>), dim3(1), dim3(512), 0, s, mr, w, (const double*)Wp, (int64_t)0,
                         (int64_t)n, (int64_t)1, (double*)nullptr, (int64_t)0, W2, (int64_t)0, (const int*)nullptr,
                         n, Vp, taus + p0, (int64_t)0);
      QTT_HIP(hipGetLastError());
      hipLaunchKernelGGL(qrb_copy_kernel, grid((int64_t)w * w), dim3(256), 0, s, Wp, n, (const double*)W2,
                         (int64_t)n, (int64_t)1, w, w);
      QTT_HIP(hipGetLastError());
    }
    qrb_gemm(gemm_desc(w, w, mr, Vp, w, true, Vp, w, false, W1, w), part, s);  // S = V^T V
    if (run) {
      hipLaunchKernelGGL(qrb_t_kernel, dim3(1), dim3(64), 0, s, (const double*)W1, w, (const double*)(taus + p0), Tp);
      QTT_HIP(hipGetLastError());
    }
    const int nt = n - p0 - w;
    if (nt > 0) {  // trailing columns: A_t <- (I - V T^T V^T) A_t
      double* At = Wp + w;
      qrb_gemm(gemm_desc(w, nt, mr, Vp, w, true, At, n, false, W1, nt), part, s);
      qrb_gemm(gemm_desc(w, nt, w, Tp, w, true, W1, nt, false, W2, nt), part, s);
      qrb_gemm(gemm_desc(mr, nt, w, Vp, w, false, W2, nt, false, At, n, -1.0, 1.0), part, s);
    }
  }
  if (run && R != nullptr) {
    hipLaunchKernelGGL(qrb_upper_kernel, grid((int64_t)n * n), dim3(256), 0, s, R, ldq, W, n);
    QTT_HIP(hipGetLastError());
  }
  if (run) {
    hipLaunchKernelGGL(qrb_eye_kernel, grid((int64_t)m * n), dim3(256), 0, s, Q, ldq, m, n);
    QTT_HIP(hipGetLastError());
  }
  int pi = (int)voff.size() - 1;
  for (int p0 = ((n - 1) / QB) * QB; p0 >= 0; p0 -= QB, --pi) {  // Q[p0:, p0:] <- (I - V T V^T) Q[p0:, p0:]
    const int w = std::min(QB, n - p0), mr = m - p0, nq = n - p0;
    const double* Vp = Vall + voff[pi];
    const double* Tp = Tall + (int64_t)p0 * QB;
    double* Qs = Q + (int64_t)p0 * ldq + p0;
    qrb_gemm(gemm_desc(w, nq, mr, Vp, w, true, Qs, ldq, false, W1, nq), part, s);
    qrb_gemm(gemm_desc(w, nq, w, Tp, w, false, W1, nq, false, W2, nq), part, s);
    qrb_gemm(gemm_desc(mr, nq, w, Vp, w, false, W2, nq, false, Qs, ldq, -1.0, 1.0), part, s);
  }
}

}  // namespace

namespace {
bool qr_split_on() {
  static const bool on = [] {
    const char* e = std::getenv("QTTPDF_QR_SPLIT");
    return !(e && e[0] == '0');
  }();
  return on;
}
// the group configuration a shape takes (RPL of it), or 0
int qr_grp_rpl(int m, int n) {
  if (qr_kernel_name(m, n).rfind("qr_grp_kernel", 0) != 0) return 0;
#define QTT_QRG_RPL(RPL_, CS_, NW_) \
  if (m <= 16 * RPL_ && n <= 4 * NW_ * CS_) return RPL_;
  QTT_QRG_CONFIGS(QTT_QRG_RPL)
#undef QTT_QRG_RPL
  return 0;
}
}  // namespace

bool qr_split(int m, int n, int64_t work_size) {
  return qr_split_on() && qr_grp_rpl(m, n) > 0 && work_size >= (int64_t)m * n + n;
}

// rows per lane of qr_q_kernel for the reflectors of an m x n factorisation
// (the row count the reflector kernel covers, over 64 lanes)
int qr_q_rows(int m, int n) { return (16 * qr_grp_rpl(m, n) + 63) / 64; }

std::string qr_q_kernel_name(int m, int n) { return "qr_q_kernel<" + std::to_string(qr_q_rows(m, n)) + ">"; }

void qr_reflectors_launch(int m, int n, const double* A, int64_t rs, int64_t cs, double* work, hipStream_t s) {
  QTT_REQUIRE(qr_grp_rpl(m, n) > 0, "qr: no reflector kernel for %d x %d", m, n);
  rt::check_range(A, 0, (int64_t)(m - 1) * rs + (int64_t)(n - 1) * cs, sizeof(double), "qr input");
  rt::check_range(work, 0, (int64_t)m * n + n - 1, sizeof(double), "qr reflectors");
  const rt::Fuse& fu = rt::fuse();
  if (fu.n > 1) {
    rt::fuse_check(A, 8 * ((int64_t)(m - 1) * rs + (int64_t)(n - 1) * cs + 1), "qr input");
    rt::fuse_check(work, 8 * ((int64_t)m * n + n), "qr reflectors");
  }
  if (rt::dry()) return;
  const dim3 grid(1, fu.n);
  const int64_t is = fu.stride;
#define QTT_QR_REFL(RPL_, CS_, NW_)                                                                   \
  if (m <= 16 * RPL_ && n <= 4 * NW_ * CS_) {                                                         \
    hipLaunchKernelGGL((qr_grp_kernel<RPL_, CS_, NW_, false>), grid, dim3(NW_ * 64), 0, s, m, n, A, (int64_t)0, rs, cs, \
                       (double*)nullptr, (int64_t)0, (double*)nullptr, (int64_t)0, (const int*)nullptr, n, work, \
                       work + (int64_t)m * n, is);                                                    \
    QTT_HIP(hipGetLastError());                                                                      \
    return;                                                                                          \
  }
  QTT_QRG_CONFIGS(QTT_QR_REFL)
#undef QTT_QR_REFL
}

void qr_form_q_launch(int m, int n, const double* work, double* Q, int ldq, hipStream_t s) {
  const int rpl = qr_grp_rpl(m, n);
  QTT_REQUIRE(rpl > 0 && ldq >= n, "qr: no Q kernel for %d x %d", m, n);
  rt::check_range(work, 0, (int64_t)m * n + n - 1, sizeof(double), "qr reflectors");
  rt::check_range(Q, 0, (int64_t)(m - 1) * ldq + n - 1, sizeof(double), "qr Q");
  const rt::Fuse& fu = rt::fuse();
  if (fu.n > 1) {
    rt::fuse_check(work, 8 * ((int64_t)m * n + n), "qr reflectors");
    rt::fuse_check(Q, 8 * ((int64_t)(m - 1) * ldq + n), "qr Q");
  }
  if (rt::dry()) return;
  const int64_t is = fu.stride;
  const double* tau = work + (int64_t)m * n;
  const dim3 grid((n + QQ_NW - 1) / QQ_NW, fu.n);
  const int rw = qr_q_rows(m, n);
#define QTT_QR_FORM(RW_)                                                                                 \
  if (rw == RW_) {                                                                                       \
    hipLaunchKernelGGL((qr_q_kernel<RW_>), grid, dim3(QQ_NW * 64), 0, s, m, n, work, tau, Q, ldq, is);   \
    QTT_HIP(hipGetLastError());                                                                          \
    return;                                                                                              \
  }
  QTT_QR_FORM(1) QTT_QR_FORM(2) QTT_QR_FORM(3) QTT_QR_FORM(4) QTT_QR_FORM(5) QTT_QR_FORM(9)
#undef QTT_QR_FORM
  QTT_REQUIRE(false, "qr: no Q kernel for %d rows per lane (%d x %d)", rw, m, n);
}

std::string qr_path_name(int m, int n) {
  const std::string k = qr_kernel_name(m, n);
  return (k == "qr_kernel" && m <= QB_MAXM) ? std::string("qr_blocked") : k;
}

void qr_launch(int count, int m, int n, const double* A, int64_t strideA, int64_t rs, int64_t cs,
               double* Q, int64_t strideQ, double* R, int64_t strideR, double* work,
               hipStream_t s, const int* sq, int ldq, int64_t work_size) {
  if (count <= 0) return;
  QTT_REQUIRE(m >= n && n >= 1 && n <= 1024, "qr: need m >= n, 1 <= n <= 1024 (m=%d n=%d)", m, n);
  QTT_REQUIRE(sq == nullptr || m == n, "qr: per-matrix sizes need square matrices");
  QTT_REQUIRE(ldq == 0 || ldq >= n, "qr: ld of Q below n");
  const int lq = ldq > 0 ? ldq : n;
  rt::check_range(A, 0, (int64_t)(count - 1) * strideA + (int64_t)(m - 1) * rs + (int64_t)(n - 1) * cs,
                  sizeof(double), "qr input");
  // Q may be left out (R only) where the group kernel factorises
  QTT_REQUIRE(Q != nullptr || (R != nullptr && qr_kernel_name(m, n).rfind("qr_grp_kernel", 0) == 0),
              "qr: R without Q needs the group kernel (m=%d n=%d)", m, n);
  if (Q) rt::check_range(Q, 0, (int64_t)(count - 1) * strideQ + (int64_t)(m - 1) * lq + n - 1, sizeof(double), "qr Q");
  if (R) rt::check_range(R, 0, (int64_t)(count - 1) * strideR + (int64_t)(n - 1) * lq + n - 1, sizeof(double),
                         "qr R");
  if (sq) rt::check_range(sq, 0, count - 1, sizeof(int), "qr sizes");
  const bool generic = qr_kernel_name(m, n) == "qr_kernel";
  if (generic) rt::check_range(work, 0, (int64_t)count * m * n - 1, sizeof(double), "qr workspace");
  if (generic && count == 1 && sq == nullptr && m <= QB_MAXM && work_size >= qr_work_size(1, m, n)) {
    rt::check_range(work, 0, qr_work_size(1, m, n) - 1, sizeof(double), "qr workspace");
    rt::fuse_refuse("the blocked QR");
    qr_blocked(m, n, A, rs, cs, Q, lq, R, work, s);
    return;
  }
  // One matrix, Q only, with a workspace for the reflectors: the group
  // kernels leave the reflectors and qr_q_kernel forms Q across workgroups
  // (QTTPDF_QR_SPLIT=0 keeps Q in the factorising workgroup).
  if (count == 1 && sq == nullptr && R == nullptr && work != nullptr && qr_split(m, n, work_size)) {
    qr_reflectors_launch(m, n, A, rs, cs, work, s);
    qr_form_q_launch(m, n, work, Q, lq, s);
    return;
  }
  const rt::Fuse& fu = rt::fuse();
  if (fu.n > 1) {
    rt::fuse_check(A, 8 * ((int64_t)(count - 1) * strideA + (int64_t)(m - 1) * rs + (int64_t)(n - 1) * cs + 1),
                   "qr input");
    if (Q) rt::fuse_check(Q, 8 * ((int64_t)(count - 1) * strideQ + (int64_t)(m - 1) * lq + n), "qr Q");
    if (R) rt::fuse_check(R, 8 * ((int64_t)(count - 1) * strideR + (int64_t)(n - 1) * lq + n), "qr R");
    if (generic) rt::fuse_check(work, 8 * ((int64_t)count * m * n), "qr workspace");
  }
  const dim3 grid(count, fu.n);
  const int64_t is = fu.stride;
  if (rt::dry()) return;
#define QTT_QR_REG(RS_, CPW_, NW_, CH_)                                                           \
  if (m <= 64 * RS_ && n <= NW_ * CPW_ && n <= QR_REG_MAXN) {                                    \
    hipLaunchKernelGGL((qr_reg_kernel<RS_, CPW_, NW_, CH_>), grid, dim3(NW_ * 64), 0, s, m, n, A,       \
                       strideA, rs, cs, Q, strideQ, R, strideR, sq, ldq, is);                         \
    QTT_HIP(hipGetLastError());                                                                  \
    return;                                                                                      \
  }
  QTT_QR_CONFIGS(QTT_QR_REG)
#undef QTT_QR_REG
#define QTT_QR_GRP(RPL_, CS_, NW_)                                                                \
  if (m <= 16 * RPL_ && n <= 4 * NW_ * CS_) {                                                     \
    if (Q != nullptr)                                                                             \
      hipLaunchKernelGGL((qr_grp_kernel<RPL_, CS_, NW_, true>), grid, dim3(NW_ * 64), 0, s, m, n, A,  \
                         strideA, rs, cs, Q, strideQ, R, strideR, sq, ldq, nullptr, nullptr, is);   \
    else                                                                                          \
      hipLaunchKernelGGL((qr_grp_kernel<RPL_, CS_, NW_, false>), grid, dim3(NW_ * 64), 0, s, m, n, A, \
                         strideA, rs, cs, Q, strideQ, R, strideR, sq, ldq, nullptr, nullptr, is);   \
    QTT_HIP(hipGetLastError());                                                                  \
    return;                                                                                      \
  }
  QTT_QRG_CONFIGS(QTT_QR_GRP)
#undef QTT_QR_GRP
#define QTT_QR_REG(RS_, CPW_, NW_, CH_)                                                           \
  if (m <= 64 * RS_ && n <= NW_ * CPW_) {                                                         \
    hipLaunchKernelGGL((qr_reg_kernel<RS_, CPW_, NW_, CH_>), grid, dim3(NW_ * 64), 0, s, m, n, A,       \
                       strideA, rs, cs, Q, strideQ, R, strideR, sq, ldq, is);                         \
    QTT_HIP(hipGetLastError());                                                                  \
    return;                                                                                      \
  }
  QTT_QR_CONFIGS_LARGE(QTT_QR_REG)
#undef QTT_QR_REG
  hipLaunchKernelGGL(qr_kernel, grid, dim3(QFT), 0, s, m, n, A, strideA, rs, cs, Q, strideQ,
                     R, strideR, work, sq, ldq, is);
  QTT_HIP(hipGetLastError());
}

bool eig_uses_precondition(int max_n) { return max_n >= 1 && max_n <= 1024; }

void eig_precondition_launch(int count, const int* dims, const double* G, int64_t strideG, int ldg,
                             double* work, int max_n, hipStream_t s) {
  if (count <= 0) return;
  QTT_REQUIRE(eig_uses_precondition(max_n), "eig: no preconditioned configuration for n = %d", max_n);
  QTT_REQUIRE(max_n <= ldg, "eig: n <= ldg");
  const int64_t st = (int64_t)ldg * ldg;
  rt::check_range(work, 0, eig_work_size(count, ldg) - 1, sizeof(double), "eig workspace");
  double* Q = work;
  double* R1 = work + count * st;
  double* R2 = work + 2 * count * st;
  double* qw = work + 3 * count * st;  // global-memory QR workspace (count * max_n^2 <= count * st)
  // G = Q1 R1 and R1^T = Q2 R2 give G = Q1 R2^T Q2^T: the sweeps run on
  // W = R2^T from V = Q2; Q1 is not needed (the group kernel skips forming
  // it).  Two factorisations leave the columns closer to orthogonal than one.
  const bool r_only = qr_kernel_name(max_n, max_n).rfind("qr_grp_kernel", 0) == 0;
  qr_launch(count, max_n, max_n, G, strideG, ldg, 1, r_only ? nullptr : Q, st, R1, st, qw, s, dims);
  qr_launch(count, max_n, max_n, R1, st, 1, max_n, Q, st, R2, st, qw, s, dims);
}

void eig_launch(int count, const int* dims, const int* keep, const double* G, int64_t strideG,
                int ldg, double* P, int64_t strideP, int ldp, double* lam, int64_t strideL,
                double* work, int max_n, double unoise, hipStream_t s, bool preconditioned) {
  if (count <= 0) return;
  QTT_REQUIRE(max_n <= 1024 && max_n <= ldg, "eig: n <= 1024 and n <= ldg");
  rt::check_range(dims, 0, count - 1, sizeof(int), "eig dims");
  rt::check_range(keep, 0, count - 1, sizeof(int), "eig keep");
  rt::check_range(G, 0, (int64_t)(count - 1) * strideG + (int64_t)(max_n - 1) * ldg + max_n - 1,
                  sizeof(double), "eig input");
  rt::check_range(P, 0, (int64_t)(count - 1) * strideP + (int64_t)(max_n - 1) * ldp + ldp - 1,
                  sizeof(double), "eig vectors");
  rt::check_range(lam, 0, (int64_t)(count - 1) * strideL + max_n - 1, sizeof(double), "eig values");
  rt::check_range(work, 0, eig_work_size(count, ldg) - 1, sizeof(double), "eig workspace");
  QTT_REQUIRE(!preconditioned || eig_uses_precondition(max_n), "eig: no preconditioned configuration");
  const rt::Fuse& fu = rt::fuse();
  if (fu.n > 1) {
    rt::fuse_check(G, 8 * ((int64_t)(count - 1) * strideG + (int64_t)(max_n - 1) * ldg + max_n), "eig input");
    rt::fuse_check(P, 8 * ((int64_t)(count - 1) * strideP + (int64_t)max_n * ldp), "eig vectors");
    rt::fuse_check(lam, 8 * ((int64_t)(count - 1) * strideL + max_n), "eig values");
    rt::fuse_check(work, 8 * eig_work_size(count, ldg), "eig workspace");
  }
  const dim3 grid(count, fu.n);
  const int64_t is = fu.stride;
  if (rt::dry()) return;
  const int64_t st = (int64_t)ldg * ldg;
  const double* Qf = preconditioned ? work : nullptr;
  const double* Rf = preconditioned ? work + 2 * count * st : nullptr;
#define QTT_EIG_REG(RS_, PPW_, NW_, CH_)                                                          \
  if (max_n <= 64 * RS_ && max_n <= 2 * NW_ * PPW_) {                                            \
    hipLaunchKernelGGL((eig_reg_kernel<RS_, PPW_, NW_, CH_>), grid, dim3(NW_ * 64), 0, s,        \
                       dims, keep, G, strideG, ldg, P, strideP, ldp, lam, strideL, unoise, Qf, Rf, \
                       st, max_n, is);                                                           \
    QTT_HIP(hipGetLastError());                                                                  \
    return;                                                                                      \
  }
  QTT_EIG_CONFIGS(QTT_EIG_REG)
#undef QTT_EIG_REG
  hipLaunchKernelGGL(eig_kernel, grid, dim3(EFT), 0, s, dims, keep, G, strideG, ldg, P,
                     strideP, ldp, lam, strideL, work, unoise, Qf, preconditioned ? work + count * st : nullptr,
                     preconditioned ? work + 2 * count * st : nullptr, st, max_n, is);
  QTT_HIP(hipGetLastError());
}

}  // namespace qtt
