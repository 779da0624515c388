// Stencil kernels of the flow case on dense periodic M^3 grids: the
// Smagorinsky diffusivity (paragraph after eq. FP0), one Runge-Kutta stage of
// the moment equation (eq. FPMoms with S = 0, CFD2 in space), and a
// deterministic squared-difference reduction for the error measures (eq.
// RMSE0 / RMSE1).
//
// One thread per grid point, 256 points per workgroup along x3 and x2.  The
// six stencil neighbours of a point are read from the caches: the x3
// neighbours share the point's cache lines, the x2 neighbours lie in the
// adjacent rows of the same workgroup, the x1 neighbours in the adjacent
// planes.  Workgroups are dealt round-robin over the eight dies, so the
// kernels map the workgroup index to a tile such that every die works on one
// contiguous range of planes, whose x1 neighbours then sit in that die's L2.
#include "moments.h"

namespace qtt {

namespace {

constexpr int MT = 256;
constexpr int NXCD = 8;
constexpr int SQ_BLOCKS = 1024;

__device__ inline int64_t tile_of(int64_t bid, int64_t nb) {
  if (nb % NXCD) return bid;
  return (bid % NXCD) * (nb / NXCD) + bid / NXCD;
}

struct Pt {
  int64_t p;
  int64_t nb[3][2];  // [axis][0: +1, 1: -1], periodic
};

__device__ inline Pt point(int64_t p, int bits) {
  const int64_t M = 1ll << bits, mask = M - 1;
  const int64_t i3 = p & mask, i2 = (p >> bits) & mask, i1 = p >> (2 * bits);
  const int64_t b1 = i1 << (2 * bits), b2 = i2 << bits;
  Pt q;
  q.p = p;
  q.nb[0][0] = (((i1 + 1) & mask) << (2 * bits)) | b2 | i3;
  q.nb[0][1] = (((i1 - 1) & mask) << (2 * bits)) | b2 | i3;
  q.nb[1][0] = b1 | (((i2 + 1) & mask) << bits) | i3;
  q.nb[1][1] = b1 | (((i2 - 1) & mask) << bits) | i3;
  q.nb[2][0] = b1 | b2 | ((i3 + 1) & mask);
  q.nb[2][1] = b1 | b2 | ((i3 - 1) & mask);
  return q;
}

__global__ __launch_bounds__(MT) void smagorinsky_kernel(int bits, const double* __restrict__ U,
                                                         double c_sgs, double gamma,
                                                         double* __restrict__ G) {
  const int64_t n = 1ll << (3 * bits);
  const int64_t p = tile_of(blockIdx.x, gridDim.x) * MT + threadIdx.x;
  if (p >= n) return;
  const Pt q = point(p, bits);
  const double inv2h = 0.5 * (double)(1ll << bits);
  double g[3][3];  // g[i][j] = dU_i / dx_j
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      g[i][j] = (U[i * n + q.nb[j][0]] - U[i * n + q.nb[j][1]]) * inv2h;
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double t = g[i][j] + g[j][i];
      s += t * t;
    }
  G[p] = gamma + c_sgs * sqrt(s);
}

template <int COUNT>
__global__ __launch_bounds__(MT) void moment_stage_kernel(int bits, const double* __restrict__ U,
                                                          const double* __restrict__ G,
                                                          const double* __restrict__ src,
                                                          const double* base, double a_base,
                                                          double a_src, double c_rhs, double* dst) {
  const int64_t n = 1ll << (3 * bits);
  const int64_t p = tile_of(blockIdx.x, gridDim.x) * MT + threadIdx.x;
  if (p >= n) return;
  const Pt q = point(p, bits);
  const double M = (double)(1ll << bits);
  const double inv2h = 0.5 * M, invh2 = M * M;
  const double g0 = G[p];
  double u[3], dg[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    u[i] = U[i * n + p];
    dg[i] = (G[q.nb[i][0]] - G[q.nb[i][1]]) * inv2h;
  }
#pragma unroll
  for (int f = 0; f < COUNT; ++f) {
    const double* s = src + f * n;
    const double c0 = s[p];
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double sp = s[q.nb[i][0]], sm = s[q.nb[i][1]];
      const double d1 = (sp - sm) * inv2h;
      const double d2 = (sp - 2.0 * c0 + sm) * invh2;
      acc += (dg[i] - u[i]) * d1 + g0 * d2;
    }
    double v = a_src * c0 + c_rhs * acc;
    if (base) v += a_base * base[f * n + p];
    dst[f * n + p] = v;
  }
}

__device__ inline double block_sum(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < MT / 64; ++i) t += sh[i];
  return t;
}

__global__ __launch_bounds__(MT) void sq_diff_kernel(int64_t n, const double* __restrict__ a,
                                                     const double* __restrict__ b, double c,
                                                     double* __restrict__ partial) {
  __shared__ double sh[MT / 64];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * MT + threadIdx.x; i < n; i += (int64_t)gridDim.x * MT) {
    const double d = a[i] - (b ? b[i] : 0.0) - c;
    acc += d * d;
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ __launch_bounds__(MT) void sum_partials_kernel(int np, const double* __restrict__ partial,
                                                          double* __restrict__ out) {
  __shared__ double sh[MT / 64];
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += MT) acc += partial[i];
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) out[0] = t;
}

int64_t blocks_for(int bits) {
  QTT_REQUIRE(bits >= 3 && bits <= 10, "grid bits %d outside [3, 10]", bits);
  return ((1ll << (3 * bits)) + MT - 1) / MT;
}

}  // namespace

void smagorinsky(int bits, const double* U, double c_sgs, double gamma, double* G, hipStream_t s) {
  const int64_t nb = blocks_for(bits);
  if (rt::dry()) return;
  smagorinsky_kernel<<<dim3((unsigned)nb), dim3(MT), 0, s>>>(bits, U, c_sgs, gamma, G);
  QTT_HIP(hipGetLastError());
}

void moment_stage(int bits, int count, const double* U, const double* G, const double* src,
                  const double* base, double a_base, double a_src, double c_rhs, double* dst,
                  hipStream_t s) {
  const int64_t nb = blocks_for(bits);
  const int64_t n = 1ll << (3 * bits);
  QTT_REQUIRE(count >= 1 && count <= 2, "moment fields per launch %d outside [1, 2]", count);
  QTT_REQUIRE(src + count * n <= dst || dst + count * n <= src, "src overlaps dst");
  if (rt::dry()) return;
  if (count == 1)
    moment_stage_kernel<1><<<dim3((unsigned)nb), dim3(MT), 0, s>>>(bits, U, G, src, base, a_base,
                                                                   a_src, c_rhs, dst);
  else
    moment_stage_kernel<2><<<dim3((unsigned)nb), dim3(MT), 0, s>>>(bits, U, G, src, base, a_base,
                                                                   a_src, c_rhs, dst);
  QTT_HIP(hipGetLastError());
}

int sq_diff_partials() { return SQ_BLOCKS; }

void sq_diff_sum(int64_t n, const double* a, const double* b, double c, double* partial,
                 double* out, hipStream_t s) {
  QTT_REQUIRE(n >= 1, "empty reduction");
  if (rt::dry()) return;
  const int64_t need = (n + MT - 1) / MT;
  const int nb = (int)(need < SQ_BLOCKS ? need : SQ_BLOCKS);
  sq_diff_kernel<<<dim3(nb), dim3(MT), 0, s>>>(n, a, b, c, partial);
  QTT_HIP(hipGetLastError());
  sum_partials_kernel<<<dim3(1), dim3(MT), 0, s>>>(nb, partial, out);
  QTT_HIP(hipGetLastError());
}

}  // namespace qtt
