#pragma once
#include "common.h"

namespace qtt {

// dst[((ro + a) * dp + s') * drr + co + b] = scale * (*dscale) * src[(a * sp + s) * rr + b]
// with s' = s, or s' = 2s + s (diag: an MPS core written as a diagonal MPO block)
struct CopyJob {
  const double* src;
  double* dst;
  int rl, sp, rr;   // source block [rl][sp][rr]
  int dp, drr;      // destination physical size and right-bond capacity
  int ro, co;       // block offsets in the destination core
  int diag;
  double scale;
  const double* dscale;  // optional device scalar multiplier
};

// out[(a*Dl + alpha), t, (b*Dr + beta)] = sum_s W[alpha,t,s,beta] x[a,s,b]
struct ApplyJob {
  const double* W;
  const double* x;
  double* out;
  int xl, xr, Dl, Dr;
};

void fill(double* p, int64_t n, double v, hipStream_t s);
// dst (cols x rows) = src^T, both row-major
void transpose(const double* src, int rows, int cols, double* dst, hipStream_t s);
// dst (m x m) = identity
void eye(double* dst, int m, hipStream_t s);
// out[i] = scale * (a[i] + cb * b[i]) for i < n <= 64 (b may be null)
void scalar_comb(double* out, const double* a, const double* b, double cb, double scale, int n,
                 hipStream_t s);
// host-side bounds checks of a job (call before uploading the job table)
void validate(const CopyJob& j);
void validate(const ApplyJob& j);
void copy_jobs(const CopyJob* d_jobs, int njobs, int64_t max_elems, hipStream_t s);
// with fused launches on: throws unless every block of the jobs (host copy of
// the table) lies in the instance slab
void fuse_check(const std::vector<CopyJob>& jobs);
// the products of the explicit MPO x MPS application in precision prec
// (FP64; FP32 inputs; BF16 high + low parts), summed in FP64
void apply_jobs(const ApplyJob* d_jobs, int njobs, int64_t max_elems, hipStream_t s, Prec prec = Prec::F64);
// zeroes the eigenvector columns of a batch of truncations (matrix i: dims[i]
// rows, keep[i] kept columns, eigenvalues descending) whose eigenvalue is at
// most tol2 times the largest; device and host copies of dims and keep
void rank_cut(double* P, int64_t strideP, int ldp, const double* lam, int64_t strideL, const int* d_dims,
              const int* d_keep, const std::vector<int>& dims, const std::vector<int>& keep, double tol2,
              hipStream_t s);
// *flag = 1 if any of the n values at p is NaN or infinite (flag untouched otherwise)
void check_finite(const double* p, int64_t n, int* flag, hipStream_t s);

}  // namespace qtt
