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
//   * BF16: v_mfma_f32_16x16x32_bf16 (CDNA4), FP32 accumulation, each
//     operand split into a BF16 high and low part (three MFMAs per product).
// The MFMA kernels read the FP64 operands, round them to FP32 / split them
// into BF16 pairs while staging the tiles in LDS, and write FP64 results.  All kernels load the
// next K tile into registers while the current one is being multiplied; the
// MFMA kernels come with three pipelines (K tile 32 or 64, one or two LDS
// buffers), chosen per launch shape by measurement.
// Contractions with few output tiles and a long K are split along K
// (TcDesc::ksplit); their partial sums are added by tc_splitk_reduce.
#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <tuple>

#include "common.h"

namespace qtt {

namespace {

constexpr int BK64 = 16;

// blockIdx.z = ((instance * batch + batch index) * ng + group) * ksplit + K chunk
struct KRange {
  int z, g, beg, end;
  int zz;      // blockIdx.z within the instance
  int64_t io;  // byte offset of the instance's data
};

template <int BK>
__device__ inline KRange k_range(const TcDesc& d) {
  int zz = (int)blockIdx.z;
  int64_t io = 0;
  if (d.ninst > 1) {
    const int per = d.batch * d.ng * d.ksplit;
    const int inst = zz / per;
    zz -= inst * per;
    io = (int64_t)inst * d.istride;
  }
  if (d.ksplit == 1 && d.ng == 1) return {zz, 0, 0, d.K, zz, io};  // no split, no groups
  const int ks = zz % d.ksplit;
  const int zg = zz / d.ksplit;
  const int g = zg % d.ng;
  const int z = zg / d.ng;
  const int chunk = ((d.K + d.ksplit - 1) / d.ksplit + BK - 1) / BK * BK;
  const int beg = ks * chunk;
  const int end = min(d.K, beg + chunk);
  return {z, g, beg, end, zz, io};
}

// group base pointers from the device table (one scalar load each), shifted
// to the launch's instance
__device__ inline const gdouble* base_a(const TcDesc& d, const KRange& kr) {
  return as_global(ishift(d.ng > 1 ? d.gdev[kr.g] : d.A, kr.io) + d.ab.off(kr.z));
}
__device__ inline const gdouble* base_b(const TcDesc& d, const KRange& kr) {
  return as_global(ishift(d.ng > 1 ? d.gdev[d.ng + kr.g] : d.B, kr.io) + d.bb.off(kr.z));
}
__device__ inline gdouble* base_c(const TcDesc& d, const KRange& kr) {
  return as_global(ishift(d.ng > 1 ? const_cast<double*>(d.gdev[2 * d.ng + kr.g]) : d.C, kr.io) + d.cb.off(kr.z));
}
__device__ inline gdouble* base_part(const TcDesc& d, const KRange& kr) {
  return as_global(ishift(d.part, kr.io) + (int64_t)kr.zz * d.M * d.N);
}
__device__ inline bool to_part(const TcDesc& d) { return d.ksplit > 1 || (d.ng > 1 && d.gsum); }

template <int BM, int BN>
__global__ __launch_bounds__(256) void tc_f64_kernel(TcDesc d, int a_kfast, int b_nfast) {
  constexpr int TM = BM / 16, TN = BN / 16;
  constexpr int NA = BM * BK64 / 256, NB = BN * BK64 / 256;
  __shared__ double As[BK64][BM + 1];
  __shared__ double Bs[BK64][BN + 1];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const KRange kr = k_range<BK64>(d);
  const gdouble* A = base_a(d, kr);
  const gdouble* B = base_b(d, kr);
  double acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = 0.0;
  double ra[NA], rb[NB];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tid + 256 * q;
      const int mm = a_kfast ? e / BK64 : e % BM, kk = a_kfast ? e % BK64 : e / BM;
      const int m = m0 + mm, k = k0 + kk;
      ra[q] = (m < d.M && k < kr.end) ? A[d.am.off(m) + d.ak.off(k)] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = tid + 256 * q;
      const int nn = b_nfast ? e % BN : e / BK64, kk = b_nfast ? e / BN : e % BK64;
      const int n = n0 + nn, k = k0 + kk;
      rb[q] = (n < d.N && k < kr.end) ? B[d.bk.off(k) + d.bn.off(n)] : 0.0;
    }
  };
  if (kr.beg < kr.end) load(kr.beg);
  for (int k0 = kr.beg; k0 < kr.end; k0 += BK64) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tid + 256 * q;
      const int mm = a_kfast ? e / BK64 : e % BM, kk = a_kfast ? e % BK64 : e / BM;
      As[kk][mm] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = tid + 256 * q;
      const int nn = b_nfast ? e % BN : e / BK64, kk = b_nfast ? e / BN : e % BK64;
      Bs[kk][nn] = rb[q];
    }
    __syncthreads();
    if (k0 + BK64 < kr.end) load(k0 + BK64);
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
  if (to_part(d)) {
    gdouble* Pp = base_part(d, kr);
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      const int m = m0 + ty + 16 * i;
      if (m >= d.M) continue;
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int n = n0 + tx + 16 * j;
        if (n < d.N) Pp[(int64_t)m * d.N + n] = acc[i][j];
      }
    }
    return;
  }
  gdouble* C = base_c(d, kr);
  int64_t coff[TN];
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int n = n0 + tx + 16 * j;
    coff[j] = n < d.N ? d.cn.off(n) : 0;
  }
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    const int m = m0 + ty + 16 * i;
    if (m >= d.M) continue;
    const int64_t rowoff = d.cm.off(m);
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int n = n0 + tx + 16 * j;
      if (n >= d.N) continue;
      gdouble* p = C + rowoff + coff[j];
      double v = d.alpha * acc[i][j];
      if (d.beta != 0.0) v += d.beta * *p;
      *p = v;
    }
  }
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// BMN x BMN output tile per workgroup (64 or 32), 4 waves each owning a
// quadrant made of MI x MI 16x16 MFMA blocks (MI = BMN / 32): the 32-wide
// tile gives four times as many workgroups to shapes that a 64-wide tile
// leaves short of the chip's CUs, without splitting K.  LDS holds A as [m][k] and B as [n][k] so that a
// lane's MFMA operand is contiguous in k.  AKF / BNF: A is read along k
// (row-major operand) / B along n; each thread's tile elements keep their row
// (column) offsets for the whole K loop, so a K step costs one or NA mode
// offsets instead of two per element.
//
// BF16: every operand x is staged as two BF16 numbers, hi = bf16(x) and
// lo = bf16(x - hi), and each product is accumulated as hi*hi + hi*lo +
// lo*hi on v_mfma_f32_16x16x32_bf16 (the dropped lo*lo term and the rounding
// of lo leave a relative error of about 2^-16 per product instead of the
// 2^-8 of a single BF16 operand).
//
// Two pipelines: DB = false stages one K tile of BK in LDS (two barriers per
// step; the next tile is loaded into registers during the MFMAs); DB = true
// double-buffers the LDS tiles (one barrier per step: the MFMAs read one
// buffer while the next tile is stored into the other) and, for FP32, gives
// MFMA t of a 16-wide K block the k values 4 lq + t of lane group lq, so each
// lane reads its four operands of a block with one 16-byte LDS load.
template <bool BF16, bool AKF, bool BNF, int BK, bool DB, int BMN>
__global__ __launch_bounds__(256) void tc_mfma_kernel(TcDesc d) {
  constexpr int BM = BMN, BN = BMN;
  constexpr int MI = BMN / 32;  // 16x16 blocks per wave along m and along n
  constexpr int NA = BM * BK / 256, NB = BN * BK / 256;
  using TIn = typename std::conditional<BF16, __bf16, float>::type;
  constexpr int PAD = BF16 ? 8 : 4;
  constexpr int NH = BF16 ? 2 : 1;  // hi (and lo) parts of each staged operand
  constexpr int NBUF = DB ? 2 : 1;
  __shared__ __align__(16) TIn As[NBUF][NH][BM][BK + PAD];
  __shared__ __align__(16) TIn Bs[NBUF][NH][BN][BK + PAD];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * (BMN / 2), wn = (wave & 1) * (BMN / 2);
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const KRange kr = k_range<BK>(d);
  const gdouble* A = base_a(d, kr);
  const gdouble* B = base_b(d, kr);
  f32x4 acc[MI][MI];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < MI; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int li = lane & 15, lq = lane >> 4;
  // element q of this thread: A at (row am_q, column ak_q), B at (ak_q', bn_q)
  auto a_row = [&](int q) { return AKF ? tid / BK + q * (256 / BK) : tid % BM; };
  auto a_col = [&](int q) { return AKF ? tid % BK : tid / BM + q * (256 / BM); };
  auto b_col = [&](int q) { return BNF ? tid % BN : tid / BK + q * (256 / BK); };
  auto b_row = [&](int q) { return BNF ? tid / BN + q * (256 / BN) : tid % BK; };
  constexpr int NAR = AKF ? NA : 1, NBC = BNF ? 1 : NB;  // distinct rows of A / columns of B
  int64_t aoff[NAR], boff[NBC];
  bool aok[NAR], bok[NBC];
#pragma unroll
  for (int q = 0; q < NAR; ++q) {
    const int m = m0 + a_row(q);
    aok[q] = m < d.M;
    aoff[q] = aok[q] ? d.am.off(m) : 0;
  }
#pragma unroll
  for (int q = 0; q < NBC; ++q) {
    const int n = n0 + b_col(q);
    bok[q] = n < d.N;
    boff[q] = bok[q] ? d.bn.off(n) : 0;
  }
  double ra[NA], rb[NB];
  auto load = [&](int k0) {
    if (AKF) {
      const int k = k0 + a_col(0);
      const bool kok = k < kr.end;
      const int64_t ko = kok ? d.ak.off(k) : 0;
#pragma unroll
      for (int q = 0; q < NA; ++q) ra[q] = (aok[q] && kok) ? A[aoff[q] + ko] : 0.0;
    } else {
#pragma unroll
      for (int q = 0; q < NA; ++q) {
        const int k = k0 + a_col(q);
        ra[q] = (aok[0] && k < kr.end) ? A[aoff[0] + d.ak.off(k)] : 0.0;
      }
    }
    if (BNF) {
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const int k = k0 + b_row(q);
        rb[q] = (bok[0] && k < kr.end) ? B[d.bk.off(k) + boff[0]] : 0.0;
      }
    } else {
      const int k = k0 + b_row(0);
      const bool kok = k < kr.end;
      const int64_t ko = kok ? d.bk.off(k) : 0;
#pragma unroll
      for (int q = 0; q < NB; ++q) rb[q] = (bok[q] && kok) ? B[ko + boff[q]] : 0.0;
    }
  };
  // registers -> LDS buffer `buf` (rounded to FP32 or split into BF16 pairs)
  auto stage = [&](int buf) {
    if constexpr (BF16) {
#pragma unroll
      for (int q = 0; q < NA; ++q) {
        const float x = (float)ra[q];
        const __bf16 hi = (__bf16)x;
        As[buf][0][a_row(q)][a_col(q)] = hi;
        As[buf][1][a_row(q)][a_col(q)] = (__bf16)(x - (float)hi);
      }
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const float x = (float)rb[q];
        const __bf16 hi = (__bf16)x;
        Bs[buf][0][b_col(q)][b_row(q)] = hi;
        Bs[buf][1][b_col(q)][b_row(q)] = (__bf16)(x - (float)hi);
      }
    } else {
#pragma unroll
      for (int q = 0; q < NA; ++q) As[buf][0][a_row(q)][a_col(q)] = (float)ra[q];
#pragma unroll
      for (int q = 0; q < NB; ++q) Bs[buf][0][b_col(q)][b_row(q)] = (float)rb[q];
    }
  };
  // MFMAs over the tile in LDS buffer `buf`
  auto compute = [&](int buf) {
    if constexpr (BF16) {
#pragma unroll
      for (int kc = 0; kc < BK; kc += 32) {
        bf16x8 a[2][MI], b[2][MI];  // [hi/lo][block]
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int i = 0; i < MI; ++i)
#pragma unroll
            for (int t = 0; t < 8; ++t) {
              a[h][i][t] = As[buf][h][wm + 16 * i + li][kc + 8 * lq + t];
              b[h][i][t] = Bs[buf][h][wn + 16 * i + li][kc + 8 * lq + t];
            }
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
          for (int j = 0; j < MI; ++j) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1][i], b[0][j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[1][j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0][i], b[0][j], acc[i][j], 0, 0, 0);
          }
      }
    } else if constexpr (DB) {
#pragma unroll
      for (int kb = 0; kb < BK; kb += 16) {
        f32x4 a[MI], b[MI];
#pragma unroll
        for (int i = 0; i < MI; ++i) a[i] = *reinterpret_cast<const f32x4*>(&As[buf][0][wm + 16 * i + li][kb + 4 * lq]);
#pragma unroll
        for (int j = 0; j < MI; ++j) b[j] = *reinterpret_cast<const f32x4*>(&Bs[buf][0][wn + 16 * j + li][kb + 4 * lq]);
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int i = 0; i < MI; ++i)
#pragma unroll
            for (int j = 0; j < MI; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][t], b[j][t], acc[i][j], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        float a[MI], b[MI];
#pragma unroll
        for (int i = 0; i < MI; ++i) a[i] = As[buf][0][wm + 16 * i + li][kk + lq];
#pragma unroll
        for (int j = 0; j < MI; ++j) b[j] = Bs[buf][0][wn + 16 * j + li][kk + lq];
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
          for (int j = 0; j < MI; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
      }
    }
  };
  if constexpr (DB) {
    if (kr.beg < kr.end) {
      load(kr.beg);
      stage(0);
    }
    __syncthreads();
    int buf = 0;
    for (int k0 = kr.beg; k0 < kr.end; k0 += BK) {  // block-uniform trip count
      const bool more = k0 + BK < kr.end;
      if (more) load(k0 + BK);
      compute(buf);
      if (more) stage(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  } else {
    if (kr.beg < kr.end) load(kr.beg);
    for (int k0 = kr.beg; k0 < kr.end; k0 += BK) {
      stage(0);
      __syncthreads();
      if (k0 + BK < kr.end) load(k0 + BK);
      compute(0);
      __syncthreads();
    }
  }
  // accumulator layout: lane holds rows 4*(lane/16)+r, column lane%16 of each block
  if (to_part(d)) {
    gdouble* Pp = base_part(d, kr);
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < MI; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int m = m0 + wm + 16 * i + 4 * lq + r;
          const int n = n0 + wn + 16 * j + li;
          if (m < d.M && n < d.N) Pp[(int64_t)m * d.N + n] = (double)acc[i][j][r];
        }
    return;
  }
  gdouble* C = base_c(d, kr);
  // output offsets: 4 MI distinct rows and MI distinct columns per thread
  int64_t coff[MI];
  bool cok[MI];
#pragma unroll
  for (int j = 0; j < MI; ++j) {
    const int n = n0 + wn + 16 * j + li;
    cok[j] = n < d.N;
    coff[j] = cok[j] ? d.cn.off(n) : 0;
  }
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = m0 + wm + 16 * i + 4 * lq + r;
      if (m >= d.M) continue;
      const int64_t ro = d.cm.off(m);
#pragma unroll
      for (int j = 0; j < MI; ++j) {
        if (!cok[j]) continue;
        gdouble* p = C + ro + coff[j];
        double v = d.alpha * (double)acc[i][j][r];
        if (d.beta != 0.0) v += d.beta * *p;
        *p = v;
      }
    }
}

// C = alpha * sum part + beta * C, one thread per output element.  Outputs
// are (batch index, group) pairs, or batch indices alone when the groups are
// summed; the parts of an output (groups, then K chunks) are added in
// increasing order.
__global__ __launch_bounds__(256) void tc_splitk_reduce(TcDesc d) {
  const int64_t mn = (int64_t)d.M * d.N;
  const int gout = d.gsum ? 1 : d.ng;      // outputs per batch index
  const int nparts = (d.gsum ? d.ng : 1) * d.ksplit;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= mn * d.batch * gout) return;
  const int64_t io = (int64_t)blockIdx.y * d.istride;  // instance (grid y)
  const int zo = (int)(idx / mn);
  const int64_t rem = idx - (int64_t)zo * mn;
  const int m = (int)(rem / d.N), n = (int)(rem - (int64_t)m * d.N);
  const int z = zo / gout, g = zo - z * gout;
  const gdouble* Pp = as_global(ishift(d.part, io) + ((int64_t)z * d.ng + g) * d.ksplit * mn + rem);
  double s = 0.0;
  int k = 0;
  for (; k + 4 <= nparts; k += 4) {  // four loads in flight, added in order
    const double p0 = Pp[(int64_t)k * mn], p1 = Pp[(int64_t)(k + 1) * mn];
    const double p2 = Pp[(int64_t)(k + 2) * mn], p3 = Pp[(int64_t)(k + 3) * mn];
    s = (((s + p0) + p1) + p2) + p3;
  }
  for (; k < nparts; ++k) s += Pp[(int64_t)k * mn];
  gdouble* base = as_global(ishift((d.ng > 1 && !d.gsum) ? const_cast<double*>(d.gdev[2 * d.ng + g]) : d.C, io));
  gdouble* p = base + d.cb.off(z) + d.cm.off(m) + d.cn.off(n);
  double v = d.alpha * s;
  if (d.beta != 0.0) v += d.beta * *p;
  *p = v;
}

inline bool unit(const Mode2& m) { return m.s2 == 1; }

struct Tile {
  int bm, bn;
};
inline Tile tile_of(const TcDesc& d, Prec p) {
  if (p != Prec::F64) return d.tile >= 3 ? Tile{32, 32} : Tile{64, 64};
  switch (d.tile) {
    case 1: return {64, 64};
    case 2: return {64, 32};
    case 3: return {32, 64};
    case 4: return {32, 32};
    case 5: return {16, 16};  // the 16-wide tiles for shapes with M or N of at most 16
    case 6: return {16, 64};
    case 7: return {64, 16};
  }
  return {d.M >= 48 ? 64 : 32, d.N >= 48 ? 64 : 32};
}

}  // namespace

std::string tc_kernel_name(const TcDesc& d, Prec p) {
  if (p != Prec::F64) {
    const char* ak = unit(d.ak) ? "true" : "false";
    const char* bn = unit(d.bn) ? "true" : "false";
    const int pl = d.tile % 3;
    const char* var = pl == 2 ? ", 64, true" : pl == 1 ? ", 32, true" : ", 32, false";
    const char* tsz = d.tile >= 3 ? ", 32>" : ", 64>";
    return std::string("tc_mfma_kernel<") + (p == Prec::BF16 ? "true" : "false") + ", " + ak + ", " + bn + var + tsz;
  }
  const Tile t = tile_of(d, p);
  return "tc_f64_kernel<" + std::to_string(t.bm) + ", " + std::to_string(t.bn) + ">";
}

int tc_choose_ksplit(const TcDesc& d, Prec p) {
  if (d.M <= 0 || d.N <= 0 || d.batch <= 0) return 1;
  const Tile t = tile_of(d, p);
  const int64_t tiles = (int64_t)((d.M + t.bm - 1) / t.bm) * ((d.N + t.bn - 1) / t.bn) * d.batch * d.ng;
  if (tiles >= 128) return 1;
  // aim at ~256 workgroups.  The FP64 kernel is slow per K step, so it splits
  // down to one LDS tile (16) per chunk; the MFMA kernels keep >= 128 per chunk.
  const int minchunk = (p == Prec::F64) ? 16 : 128;
  if (d.K < 4 * minchunk) return 1;
  int ks = (int)std::min<int64_t>(d.K / minchunk, (256 + tiles - 1) / tiles);
  ks = std::min(ks, 64);
  return ks >= 2 ? ks : 1;
}

void tc_validate(const TcDesc& d) {
  if (d.M <= 0 || d.N <= 0 || d.batch <= 0) return;
  QTT_REQUIRE(d.M < (1 << 30) && d.N < (1 << 30) && d.K < (1 << 30), "contraction extent too large");
  QTT_REQUIRE(d.ksplit >= 1, "bad K split");
  QTT_REQUIRE(d.ng >= 1 && d.ng <= TC_MAXG, "contraction pointer groups %d outside 1..%d", d.ng, TC_MAXG);
  if (d.ng > 1) rt::check_range(d.gdev, 0, 3 * d.ng - 1, sizeof(double*), "contraction pointer table");
  // every pointer group is checked against its own allocation
  for (int g = 0; g < d.ng; ++g) {
    const double* A = d.ng > 1 ? d.gA[g] : d.A;
    const double* B = d.ng > 1 ? d.gB[g] : d.B;
    double* C = (d.ng > 1 && !d.gsum) ? d.gC[g] : d.C;
    if (d.K > 0) {
      rt::check_range(A, 0, mode_max(d.ab, d.batch) + mode_max(d.am, d.M) + mode_max(d.ak, d.K),
                      sizeof(double), "contraction operand A");
      rt::check_range(B, 0, mode_max(d.bb, d.batch) + mode_max(d.bk, d.K) + mode_max(d.bn, d.N),
                      sizeof(double), "contraction operand B");
    }
    const int64_t ce = mode_max(d.cb, d.batch) + mode_max(d.cm, d.M) + mode_max(d.cn, d.N);
    rt::check_range(C, 0, ce, sizeof(double), "contraction result C");
    if (rt::fuse().n > 1) {
      if (d.K > 0) {
        rt::fuse_check(A, 8 * (mode_max(d.ab, d.batch) + mode_max(d.am, d.M) + mode_max(d.ak, d.K) + 1),
                       "contraction operand A");
        rt::fuse_check(B, 8 * (mode_max(d.bb, d.batch) + mode_max(d.bk, d.K) + mode_max(d.bn, d.N) + 1),
                       "contraction operand B");
      }
      rt::fuse_check(C, 8 * (ce + 1), "contraction result C");
    }
  }
  if (tc_uses_part(d)) {
    rt::check_range(d.part, 0, tc_part_size(d) - 1, sizeof(double), "contraction partial sums");
    rt::fuse_check(d.part, 8 * tc_part_size(d), "contraction partial sums");
  }
}

void tc_launch(const TcDesc& d0, Prec p, hipStream_t s) {
  if (d0.M <= 0 || d0.N <= 0 || d0.batch <= 0) return;
  TcDesc d = d0;
  d.ninst = rt::fuse().n;
  d.istride = rt::fuse().stride;
  tc_validate(d);
  if (rt::dry()) return;
  const Tile t = tile_of(d, p);
  QTT_REQUIRE((int64_t)d.batch * d.ng * d.ksplit * d.ninst <= 65535 && (d.M + t.bm - 1) / t.bm <= 65535,
              "contraction too large (M=%d batch=%d groups=%d split=%d instances=%d)", d.M, d.batch, d.ng,
              d.ksplit, d.ninst);
  const int a_kfast = unit(d.ak) ? 1 : 0;
  const int b_nfast = unit(d.bn) ? 1 : 0;
  const dim3 grid((d.N + t.bn - 1) / t.bn, (d.M + t.bm - 1) / t.bm, d.batch * d.ng * d.ksplit * d.ninst);
  if (p == Prec::F64) {
    if (t.bm == 64 && t.bn == 64)
      hipLaunchKernelGGL((tc_f64_kernel<64, 64>), grid, dim3(256), 0, s, d, a_kfast, b_nfast);
    else if (t.bm == 64 && t.bn == 32)
      hipLaunchKernelGGL((tc_f64_kernel<64, 32>), grid, dim3(256), 0, s, d, a_kfast, b_nfast);
    else if (t.bm == 32 && t.bn == 64)
      hipLaunchKernelGGL((tc_f64_kernel<32, 64>), grid, dim3(256), 0, s, d, a_kfast, b_nfast);
    else if (t.bm == 32 && t.bn == 32)
      hipLaunchKernelGGL((tc_f64_kernel<32, 32>), grid, dim3(256), 0, s, d, a_kfast, b_nfast);
    else if (t.bm == 16 && t.bn == 16)
      hipLaunchKernelGGL((tc_f64_kernel<16, 16>), grid, dim3(256), 0, s, d, a_kfast, b_nfast);
    else if (t.bm == 16)
      hipLaunchKernelGGL((tc_f64_kernel<16, 64>), grid, dim3(256), 0, s, d, a_kfast, b_nfast);
    else
      hipLaunchKernelGGL((tc_f64_kernel<64, 16>), grid, dim3(256), 0, s, d, a_kfast, b_nfast);
  } else {
    // MFMA pipeline v % 3: 0 one LDS tile of 32, 1 double-buffered 32, 2
    // double-buffered 64; tile 64 x 64 for v < 3, 32 x 32 from 3 on
    const int v = d.tile;
#define QTT_TC_MFMA_T(BF, AK, BN, T)                                                              \
  if (v == (T == 64 ? 2 : 5))                                                                     \
    hipLaunchKernelGGL((tc_mfma_kernel<BF, AK, BN, 64, true, T>), grid, dim3(256), 0, s, d);      \
  else if (v == (T == 64 ? 1 : 4))                                                                \
    hipLaunchKernelGGL((tc_mfma_kernel<BF, AK, BN, 32, true, T>), grid, dim3(256), 0, s, d);      \
  else if (v == (T == 64 ? 0 : 3))                                                                \
    hipLaunchKernelGGL((tc_mfma_kernel<BF, AK, BN, 32, false, T>), grid, dim3(256), 0, s, d);
#define QTT_TC_MFMA(BF, AK, BN)                                                          \
  if ((p == Prec::BF16) == BF && (a_kfast != 0) == AK && (b_nfast != 0) == BN) {          \
    QTT_TC_MFMA_T(BF, AK, BN, 64)                                                         \
    QTT_TC_MFMA_T(BF, AK, BN, 32)                                                         \
  }
    QTT_TC_MFMA(true, true, true)
    QTT_TC_MFMA(true, true, false)
    QTT_TC_MFMA(true, false, true)
    QTT_TC_MFMA(true, false, false)
    QTT_TC_MFMA(false, true, true)
    QTT_TC_MFMA(false, true, false)
    QTT_TC_MFMA(false, false, true)
    QTT_TC_MFMA(false, false, false)
#undef QTT_TC_MFMA
#undef QTT_TC_MFMA_T
  }
  QTT_HIP(hipGetLastError());
  if (tc_uses_part(d)) {
    const int64_t tot = (int64_t)d.M * d.N * d.batch * (d.gsum ? 1 : d.ng);
    hipLaunchKernelGGL(tc_splitk_reduce, dim3((unsigned)((tot + 255) / 256), d.ninst), dim3(256), 0, s, d);
    QTT_HIP(hipGetLastError());
  }
}

// ---------------------------------------------------------------------------
// Autotuning of the FP64 tile and the K split, per launch shape
// ---------------------------------------------------------------------------
namespace {

struct TuneKey {
  int p, M, N, K, batch, ng, gsum, beta, akf, bnf;
  bool operator<(const TuneKey& o) const {
    return std::tie(p, M, N, K, batch, ng, gsum, beta, akf, bnf) <
           std::tie(o.p, o.M, o.N, o.K, o.batch, o.ng, o.gsum, o.beta, o.akf, o.bnf);
  }
};

std::mutex g_tune_mu;
std::map<TuneKey, std::pair<int, int>> g_tuned;  // (tile, ksplit)
hipStream_t g_tune_stream = nullptr;
int g_tune_shapes = 0;
double g_tune_seconds = 0.0;

bool autotune_on() {
  static int v = -1;
  if (v < 0) {
    const char* e = std::getenv("QTTPDF_AUTOTUNE");
    v = (e && e[0] == '0') ? 0 : 1;
  }
  return v == 1 && !rt::dry();
}

TuneKey key_of(const TcDesc& d, Prec p) {
  return {(int)p, d.M, d.N, d.K, d.batch, d.ng, d.gsum, d.beta != 0.0 ? 1 : 0, unit(d.ak) ? 1 : 0,
          unit(d.bn) ? 1 : 0};
}

// times the launch shape of d with every candidate (scratch outputs); returns (tile, ksplit)
std::pair<int, int> measure(const TcDesc& d, Prec p) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!g_tune_stream) QTT_HIP(hipStreamCreateWithFlags(&g_tune_stream, hipStreamNonBlocking));
  hipStream_t s = g_tune_stream;
  std::vector<int> tiles{0, 1, 2};  // MFMA pipelines with 64 x 64 tiles
  if (p != Prec::F64) {
    // the 32 x 32 tiles where 64 x 64 ones leave the chip short of workgroups
    const int64_t t64 = (int64_t)((d.M + 63) / 64) * ((d.N + 63) / 64) * d.batch * d.ng;
    if (t64 < 512) tiles.insert(tiles.end(), {3, 4, 5});
  }
  if (p == Prec::F64) {
    tiles = {4};
    if (d.N > 32) tiles.push_back(3);
    if (d.M > 32) tiles.push_back(2);
    if (d.M > 32 && d.N > 32) tiles.push_back(1);
    if (d.M <= 16 || d.N <= 16) tiles.push_back(5);
    if (d.M <= 16 && d.N > 32) tiles.push_back(6);
    if (d.N <= 16 && d.M > 32) tiles.push_back(7);
  }
  const int minchunk = (p == Prec::F64) ? 16 : 32;
  std::vector<int> splits;
  for (int ks = 1; ks <= 64; ks *= 2)
    if ((ks == 1 || d.K >= 2 * minchunk * ks / 2) && (int64_t)d.batch * d.ng * ks <= 65535) splits.push_back(ks);
  const int rule = tc_choose_ksplit(d, p);
  if (std::find(splits.begin(), splits.end(), rule) == splits.end()) splits.push_back(rule);
  // scratch output (every group writes into it), partial sums for the largest split, group table
  const int64_t cext = mode_max(d.cb, d.batch) + mode_max(d.cm, d.M) + mode_max(d.cn, d.N) + 1;
  DevBuf C(sizeof(double) * (size_t)cext);
  const int kmax = *std::max_element(splits.begin(), splits.end());
  TcDesc probe = d;
  probe.ksplit = kmax;
  DevBuf part(sizeof(double) * (size_t)std::max<int64_t>(1, tc_part_size(probe)));
  DevBuf table;
  if (d.ng > 1) {
    std::vector<const double*> t;
    for (int g = 0; g < d.ng; ++g) t.push_back(d.gA[g]);
    for (int g = 0; g < d.ng; ++g) t.push_back(d.gB[g]);
    for (int g = 0; g < d.ng; ++g) t.push_back(C.d());
    table.alloc(t.size() * sizeof(double*));
    rt::copy(table.p, t.data(), t.size() * sizeof(double*));
  }
  hipEvent_t e0, e1;
  QTT_HIP(hipEventCreate(&e0));
  QTT_HIP(hipEventCreate(&e1));
  std::pair<int, int> best{tiles[0], 1};
  float best_ms = 1e30f;
  for (int t : tiles)
    for (int ks : splits) {
      TcDesc e = d;
      e.tile = t;
      e.ksplit = ks;
      e.C = C.d();
      e.part = part.d();
      if (d.ng > 1) {
        for (int g = 0; g < d.ng; ++g) e.gC[g] = C.d();
        e.gdev = table.as<const double*>();
      }
      tc_launch(e, p, s);  // warm-up
      QTT_HIP(hipEventRecord(e0, s));
      for (int r = 0; r < 3; ++r) tc_launch(e, p, s);
      QTT_HIP(hipEventRecord(e1, s));
      QTT_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      QTT_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (ms < best_ms) {
        best_ms = ms;
        best = {t, ks};
      }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  QTT_HIP(hipStreamSynchronize(s));
  g_tune_seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  ++g_tune_shapes;
  return best;
}

}  // namespace

namespace {
// QTTPDF_MFMA_PIPELINE=0..5 forces one MFMA variant (pipeline v % 3, tile
// 64 x 64 below 3, 32 x 32 from 3 on) for every launch recorded from then on,
// QTTPDF_F64_TILE=1..7 one tile of the FP64 kernel (read at each call, so
// tests can cover each one)
int forced_pipeline() {
  const char* e = std::getenv("QTTPDF_MFMA_PIPELINE");
  if (!e || e[0] < '0' || e[0] > '5' || e[1] != 0) return -1;
  return e[0] - '0';
}
int forced_f64_tile() {
  const char* e = std::getenv("QTTPDF_F64_TILE");
  if (!e || e[0] < '1' || e[0] > '7' || e[1] != 0) return -1;
  return e[0] - '0';
}
}  // namespace

bool tc_configure(TcDesc& d, Prec p, bool measure_ok) {
  d.tile = 0;
  d.ksplit = tc_choose_ksplit(d, p);
  const int fp = p == Prec::F64 ? forced_f64_tile() : forced_pipeline();
  bool measured = false;
  if (autotune_on() && d.M > 0 && d.N > 0 && d.batch > 0 && d.K > 0) {
    const TuneKey k = key_of(d, p);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(k);
    if (it == g_tuned.end() && measure_ok) it = g_tuned.emplace(k, measure(d, p)).first;
    if (it != g_tuned.end()) {
      d.tile = it->second.first;
      d.ksplit = it->second.second;
      measured = true;
    }
  }
  if (fp >= 0) d.tile = fp;
  return measured;
}

void tc_autotune_stats(int* shapes, double* seconds) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (shapes) *shapes = g_tune_shapes;
  if (seconds) *seconds = g_tune_seconds;
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
