// Dense 3-D fields of the flow case: the Smagorinsky diffusivity, the moment
// equation of the mean compositions (eq. FPMoms at Da = 0) and squared-error
// reductions.  Fields live on the periodic M^3 grid (M = 2^bits, h = 1/M),
// row-major [x1][x2][x3] with x3 fastest; a set of `count` fields is stored
// back to back, field f at offset f * M^3.
#pragma once
#include "common.h"

namespace qtt {

// G = gamma + c_sgs * sqrt(sum_ij (dU_i/dx_j + dU_j/dx_i)^2), CFD2 periodic
// differences; U holds the three velocity components (3 fields).
void smagorinsky(int bits, const double* U, double c_sgs, double gamma, double* G, hipStream_t s);

// dst_f = a_base * base_f + a_src * src_f + c_rhs * L(src_f) for f < count,
// with L(m) = sum_i [-U_i D1_i m + G D2_i m + (D1_i G)(D1_i m)] (CFD2,
// periodic).  base may be null or equal dst (read and written at the same
// point only); src must not overlap dst.
void moment_stage(int bits, int count, const double* U, const double* G, const double* src,
                  const double* base, double a_base, double a_src, double c_rhs, double* dst,
                  hipStream_t s);

// out[0] = sum_i (a_i - b_i - c)^2 over n values (b may be null), summed in a
// fixed order (per-workgroup partials, then one workgroup); `partial` holds
// sq_diff_partials() doubles.
int sq_diff_partials();
void sq_diff_sum(int64_t n, const double* a, const double* b, double c, double* partial,
                 double* out, hipStream_t s);

}  // namespace qtt
