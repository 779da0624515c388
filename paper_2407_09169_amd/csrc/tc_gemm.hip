// Batched 2-mode tensor contraction C[b](m,n) = alpha * sum_k A[b](m,k) B[b](k,n) + beta C.
//
// Every index (batch, m, n, k) may be the flattening of two tensor modes with
// their own strides (Mode2), so core contractions such as
// T[b,(alpha,s),z] = sum_{(beta,t)} W[alpha,t,s,beta] X[b,beta,t,z] map onto one
// launch without reshuffling copies.
//
// Three kernels:
//   * FP64: LDS-tiled SIMT FMA (64x64 or 32x32 tiles, 256 threads);
//   * FP32: v_mfma_f32_16x16x4f32, FP32 accumulation;
//   * BF16: v_mfma_f32_16x16x32_bf16 (CDNA4), FP32 accumulation.
// The MFMA kernels read the FP64 operands, round them to FP32 / BF16 while
// staging the tiles in LDS, and write FP64 results.
#include "common.h"

namespace qtt {

namespace {

constexpr int BK64 = 16;

template <int BM, int BN>
__global__ __launch_bounds__(256) void tc_f64_kernel(TcDesc d, int a_kfast, int b_nfast) {
  constexpr int TM = BM / 16, TN = BN / 16;
  __shared__ double As[BK64][BM + 1];
  __shared__ double Bs[BK64][BN + 1];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int z = blockIdx.z;
  const double* A = d.A + d.ab.off(z);
  const double* B = d.B + d.bb.off(z);
  double* C = d.C + d.cb.off(z);
  double acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = 0.0;

  for (int k0 = 0; k0 < d.K; k0 += BK64) {
    for (int e = tid; e < BM * BK64; e += 256) {
      int mm, kk;
      if (a_kfast) { kk = e % BK64; mm = e / BK64; } else { mm = e % BM; kk = e / BM; }
      int m = m0 + mm, k = k0 + kk;
      double v = 0.0;
      if (m < d.M && k < d.K) v = A[d.am.off(m) + d.ak.off(k)];
      As[kk][mm] = v;
    }
    for (int e = tid; e < BN * BK64; e += 256) {
      int nn, kk;
      if (b_nfast) { nn = e % BN; kk = e / BN; } else { kk = e % BK64; nn = e / BK64; }
      int n = n0 + nn, k = k0 + kk;
      double v = 0.0;
      if (n < d.N && k < d.K) v = B[d.bk.off(k) + d.bn.off(n)];
      Bs[kk][nn] = v;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < BK64; ++kk) {
      double a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < TN; ++j) b[j] = Bs[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    int m = m0 + ty + 16 * i;
    if (m >= d.M) continue;
    int64_t rowoff = d.cm.off(m);
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      int n = n0 + tx + 16 * j;
      if (n >= d.N) continue;
      double* p = C + rowoff + d.cn.off(n);
      double v = d.alpha * acc[i][j];
      if (d.beta != 0.0) v += d.beta * *p;
      *p = v;
    }
  }
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// 64x64 output tile per workgroup, 4 waves each owning a 32x32 quadrant made
// of 2x2 16x16 MFMA blocks.  LDS holds A as [m][k] and B as [n][k] so that a
// lane's MFMA operand is contiguous in k.
template <bool BF16>
__global__ __launch_bounds__(256) void tc_mfma_kernel(TcDesc d, int a_kfast, int b_nfast) {
  constexpr int BM = 64, BN = 64, BK = 32;
  using TIn = typename std::conditional<BF16, __bf16, float>::type;
  constexpr int PAD = BF16 ? 8 : 4;
  __shared__ TIn As[BM][BK + PAD];
  __shared__ TIn Bs[BN][BK + PAD];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int z = blockIdx.z;
  const double* A = d.A + d.ab.off(z);
  const double* B = d.B + d.bb.off(z);
  double* C = d.C + d.cb.off(z);
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int li = lane & 15, lq = lane >> 4;

  for (int k0 = 0; k0 < d.K; k0 += BK) {
    for (int e = tid; e < BM * BK; e += 256) {
      int mm, kk;
      if (a_kfast) { kk = e % BK; mm = e / BK; } else { mm = e % BM; kk = e / BM; }
      int m = m0 + mm, k = k0 + kk;
      double v = 0.0;
      if (m < d.M && k < d.K) v = A[d.am.off(m) + d.ak.off(k)];
      As[mm][kk] = (TIn)(float)v;
    }
    for (int e = tid; e < BN * BK; e += 256) {
      int nn, kk;
      if (b_nfast) { nn = e % BN; kk = e / BN; } else { kk = e % BK; nn = e / BK; }
      int n = n0 + nn, k = k0 + kk;
      double v = 0.0;
      if (n < d.N && k < d.K) v = B[d.bk.off(k) + d.bn.off(n)];
      Bs[nn][kk] = (TIn)(float)v;
    }
    __syncthreads();
    if constexpr (BF16) {
      bf16x8 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int t = 0; t < 8; ++t) a[i][t] = As[wm + 16 * i + li][8 * lq + t];
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int t = 0; t < 8; ++t) b[j][t] = Bs[wn + 16 * j + li][8 * lq + t];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    } else {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        float a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) a[i] = As[wm + 16 * i + li][kk + lq];
#pragma unroll
        for (int j = 0; j < 2; ++j) b[j] = Bs[wn + 16 * j + li][kk + lq];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // accumulator layout: lane holds rows 4*(lane/16)+r, column lane%16 of each block
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int m = m0 + wm + 16 * i + 4 * lq + r;
        int n = n0 + wn + 16 * j + li;
        if (m < d.M && n < d.N) {
          double* p = C + d.cm.off(m) + d.cn.off(n);
          double v = d.alpha * (double)acc[i][j][r];
          if (d.beta != 0.0) v += d.beta * *p;
          *p = v;
        }
      }
}

inline bool unit(const Mode2& m) { return m.n2 == 0 ? (m.s2 == 1) : (m.s2 == 1); }

}  // namespace

void tc_validate(const TcDesc& d) {
  if (d.M <= 0 || d.N <= 0 || d.batch <= 0) return;
  QTT_REQUIRE(d.M < (1 << 30) && d.N < (1 << 30) && d.K < (1 << 30), "contraction extent too large");
  if (d.K > 0) {
    rt::check_range(d.A, 0, mode_max(d.ab, d.batch) + mode_max(d.am, d.M) + mode_max(d.ak, d.K),
                    sizeof(double), "contraction operand A");
    rt::check_range(d.B, 0, mode_max(d.bb, d.batch) + mode_max(d.bk, d.K) + mode_max(d.bn, d.N),
                    sizeof(double), "contraction operand B");
  }
  rt::check_range(d.C, 0, mode_max(d.cb, d.batch) + mode_max(d.cm, d.M) + mode_max(d.cn, d.N),
                  sizeof(double), "contraction result C");
}

void tc_launch(const TcDesc& d, Prec p, hipStream_t s) {
  if (d.M <= 0 || d.N <= 0 || d.batch <= 0) return;
  tc_validate(d);
  if (rt::dry()) return;
  QTT_REQUIRE(d.batch <= 65535 && (d.M + 31) / 32 <= 65535, "contraction too large (M=%d batch=%d)",
              d.M, d.batch);
  int a_kfast = unit(d.ak) ? 1 : 0;
  int b_nfast = unit(d.bn) ? 1 : 0;
  if (p == Prec::F64) {
    if (d.M >= 48 && d.N >= 48) {
      dim3 grid((d.N + 63) / 64, (d.M + 63) / 64, d.batch);
      hipLaunchKernelGGL((tc_f64_kernel<64, 64>), grid, dim3(256), 0, s, d, a_kfast, b_nfast);
    } else if (d.M >= 48) {
      dim3 grid((d.N + 31) / 32, (d.M + 63) / 64, d.batch);
      hipLaunchKernelGGL((tc_f64_kernel<64, 32>), grid, dim3(256), 0, s, d, a_kfast, b_nfast);
    } else if (d.N >= 48) {
      dim3 grid((d.N + 63) / 64, (d.M + 31) / 32, d.batch);
      hipLaunchKernelGGL((tc_f64_kernel<32, 64>), grid, dim3(256), 0, s, d, a_kfast, b_nfast);
    } else {
      dim3 grid((d.N + 31) / 32, (d.M + 31) / 32, d.batch);
      hipLaunchKernelGGL((tc_f64_kernel<32, 32>), grid, dim3(256), 0, s, d, a_kfast, b_nfast);
    }
  } else {
    dim3 grid((d.N + 63) / 64, (d.M + 63) / 64, d.batch);
    if (p == Prec::BF16)
      hipLaunchKernelGGL((tc_mfma_kernel<true>), grid, dim3(256), 0, s, d, a_kfast, b_nfast);
    else
      hipLaunchKernelGGL((tc_mfma_kernel<false>), grid, dim3(256), 0, s, d, a_kfast, b_nfast);
  }
  QTT_HIP(hipGetLastError());
}

TcDesc gemm_desc(int M, int N, int K, const double* A, int64_t lda, bool transA, const double* B,
                 int64_t ldb, bool transB, double* C, int64_t ldc, double alpha, double beta) {
  TcDesc d;
  d.M = M;
  d.N = N;
  d.K = K;
  d.batch = 1;
  d.A = A;
  d.B = B;
  d.C = C;
  d.am = transA ? mode1(1) : mode1(lda);
  d.ak = transA ? mode1(lda) : mode1(1);
  d.bk = transB ? mode1(1) : mode1(ldb);
  d.bn = transB ? mode1(ldb) : mode1(1);
  d.cm = mode1(ldc);
  d.cn = mode1(1);
  d.ab = d.bb = d.cb = mode1(0);
  d.alpha = alpha;
  d.beta = beta;
  return d;
}

}  // namespace qtt
