// Stencil kernels of the flow case on dense periodic M^3 grids: the
// Smagorinsky diffusivity (paragraph after eq. FP0), one Runge-Kutta stage of
// the moment equation (eq. FPMoms with S = 0, CFD2 in space), and a
// deterministic squared-difference reduction for the error measures (eq.
// RMSE0 / RMSE1).
//
// The Smagorinsky kernel and the moment stage on grids below 256^3 use one
// thread per grid point, 256 points per workgroup along x3 and x2, and read
// the six stencil neighbours of a point from the caches.  The moment stage on
// larger grids walks columns along x1 (below).  Workgroups are dealt
// round-robin over the eight dies, so the kernels map the workgroup index to
// a tile such that every die works on one contiguous range of tiles, whose
// neighbouring planes and rows then sit in that die's L2.
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

// Column form for M >= 256: a workgroup covers 128 (x3) x 4 (x2) columns,
// two adjacent x3 points per lane (16-byte loads and stores), and walks CH
// consecutive x1 planes.  The x1 neighbours of the fields and of G stay in
// registers from one plane to the next, the x3 neighbours come from the
// adjacent lanes of the wavefront (a load only at the two ends), and the x2
// neighbours are loads of the adjacent rows (cache hits: the rows belong to
// the same or a neighbouring workgroup on the same die).  U and the base
// fields are read one plane ahead and bypass the caches, as do the results.
constexpr int CH = 16;
typedef double v2d __attribute__((ext_vector_type(2)));

__device__ inline double lane_shift(double v, int src_lane) {
  return __shfl(v, src_lane, 64);
}

__device__ inline v2d ld2(const double* p) { return *reinterpret_cast<const v2d*>(p); }

__device__ inline v2d ld2_stream(const double* p) {
  return __builtin_nontemporal_load(reinterpret_cast<const v2d*>(p));
}

template <int COUNT>
__global__ __launch_bounds__(MT) void moment_stage_col_kernel(int bits, const double* __restrict__ U,
                                                              const double* __restrict__ G,
                                                              const double* __restrict__ src,
                                                              const double* base, double a_base,
                                                              double a_src, double c_rhs,
                                                              double* dst) {
  const int64_t M = 1ll << bits, mask = M - 1, n = 1ll << (3 * bits), plane = M * M;
  const int64_t nt3 = M >> 7, nt2 = M >> 2;
  int64_t t = tile_of(blockIdx.x, gridDim.x);
  const int64_t t3 = t % nt3;
  t /= nt3;
  const int64_t t2 = t % nt2;
  const int64_t chunk = t / nt2;
  const int lane = threadIdx.x & 63;
  const int64_t i3 = t3 * 128 + 2 * lane, i2 = t2 * 4 + (threadIdx.x >> 6);
  const int64_t col = (i2 << bits) | i3;  // even: 16-byte aligned
  const int64_t o2p = (((i2 + 1) & mask) << bits) | i3, o2m = (((i2 - 1) & mask) << bits) | i3;
  const int64_t o3p = (i2 << bits) | ((i3 + 2) & mask), o3m = (i2 << bits) | ((i3 - 1) & mask);
  const int lp = (lane + 1) & 63, lm = (lane - 1) & 63;
  const double Md = (double)M;
  const double inv2h = 0.5 * Md, invh2 = Md * Md;
  const int64_t i10 = chunk * CH;
  auto pl = [&](int64_t i1) { return (i1 & mask) * plane; };
  // register queues: the fields and G at planes i1 - 1, i1, i1 + 1; U and
  // the base fields of the current plane, loaded one plane ahead
  v2d sq[COUNT][3], gq[3], uq[3], bq[COUNT];
#pragma unroll
  for (int f = 0; f < COUNT; ++f) {
    sq[f][0] = ld2(src + f * n + pl(i10 - 1) + col);
    sq[f][1] = ld2(src + f * n + pl(i10) + col);
    bq[f] = base ? ld2_stream(base + f * n + pl(i10) + col) : v2d{0.0, 0.0};
  }
  gq[0] = ld2(G + pl(i10 - 1) + col);
  gq[1] = ld2(G + pl(i10) + col);
#pragma unroll
  for (int i = 0; i < 3; ++i) uq[i] = ld2_stream(U + i * n + pl(i10) + col);
  for (int k = 0; k < CH; ++k) {
    const int64_t P0 = pl(i10 + k), Pn = pl(i10 + k + 1);
#pragma unroll
    for (int f = 0; f < COUNT; ++f) sq[f][2] = ld2(src + f * n + Pn + col);
    gq[2] = ld2(G + Pn + col);
    const v2d u[3] = {uq[0], uq[1], uq[2]};
    v2d bcur[COUNT];
#pragma unroll
    for (int f = 0; f < COUNT; ++f) bcur[f] = bq[f];
    if (k + 1 < CH) {
#pragma unroll
      for (int i = 0; i < 3; ++i) uq[i] = ld2_stream(U + i * n + Pn + col);
      if (base) {
#pragma unroll
        for (int f = 0; f < COUNT; ++f) bq[f] = ld2_stream(base + f * n + Pn + col);
      }
    }
    // G: x3 neighbours of the pair (x, y) are the left lane's y and the right lane's x
    const v2d g0 = gq[1];
    double gr = lane_shift(g0.x, lp), gl = lane_shift(g0.y, lm);
    if (lane == 63) gr = G[P0 + o3p];
    if (lane == 0) gl = G[P0 + o3m];
    const v2d g2p = ld2(G + P0 + o2p), g2m = ld2(G + P0 + o2m);
    const double dgx[3] = {(gq[2].x - gq[0].x) * inv2h, (g2p.x - g2m.x) * inv2h, (g0.y - gl) * inv2h};
    const double dgy[3] = {(gq[2].y - gq[0].y) * inv2h, (g2p.y - g2m.y) * inv2h, (gr - g0.x) * inv2h};
#pragma unroll
    for (int f = 0; f < COUNT; ++f) {
      const double* s = src + f * n + P0;
      const v2d c0 = sq[f][1];
      double sr = lane_shift(c0.x, lp), sl = lane_shift(c0.y, lm);
      if (lane == 63) sr = s[o3p];
      if (lane == 0) sl = s[o3m];
      const v2d s2p = ld2(s + o2p), s2m = ld2(s + o2m);
      const double spx[3] = {sq[f][2].x, s2p.x, c0.y}, smx[3] = {sq[f][0].x, s2m.x, sl};
      const double spy[3] = {sq[f][2].y, s2p.y, sr}, smy[3] = {sq[f][0].y, s2m.y, c0.x};
      const double ux[3] = {u[0].x, u[1].x, u[2].x}, uy[3] = {u[0].y, u[1].y, u[2].y};
      double ax = 0.0, ay = 0.0;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double d1x = (spx[i] - smx[i]) * inv2h, d1y = (spy[i] - smy[i]) * inv2h;
        const double d2x = (spx[i] - 2.0 * c0.x + smx[i]) * invh2;
        const double d2y = (spy[i] - 2.0 * c0.y + smy[i]) * invh2;
        ax += (dgx[i] - ux[i]) * d1x + g0.x * d2x;
        ay += (dgy[i] - uy[i]) * d1y + g0.y * d2y;
      }
      v2d v{a_src * c0.x + c_rhs * ax, a_src * c0.y + c_rhs * ay};
      if (base) {
        v.x += a_base * bcur[f].x;
        v.y += a_base * bcur[f].y;
      }
      __builtin_nontemporal_store(v, reinterpret_cast<v2d*>(dst + f * n + P0 + col));
      sq[f][0] = sq[f][1];
      sq[f][1] = sq[f][2];
    }
    gq[0] = gq[1];
    gq[1] = gq[2];
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
  if (bits >= 8) {
    // 128 x 4 columns per workgroup, CH planes each: (M/128) (M/4) (M/CH) workgroups
    const int64_t ncol =
        (int64_t(1) << (bits - 7)) * (int64_t(1) << (bits - 2)) * ((int64_t(1) << bits) / CH);
    const dim3 g((unsigned)ncol), b(MT);
    if (count == 1)
      moment_stage_col_kernel<1><<<g, b, 0, s>>>(bits, U, G, src, base, a_base, a_src, c_rhs, dst);
    else
      moment_stage_col_kernel<2><<<g, b, 0, s>>>(bits, U, G, src, base, a_base, a_src, c_rhs, dst);
  } else if (count == 1) {
    moment_stage_kernel<1><<<dim3((unsigned)nb), dim3(MT), 0, s>>>(bits, U, G, src, base, a_base,
                                                                   a_src, c_rhs, dst);
  } else {
    moment_stage_kernel<2><<<dim3((unsigned)nb), dim3(MT), 0, s>>>(bits, U, G, src, base, a_base,
                                                                   a_src, c_rhs, dst);
  }
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
