// Host-side FP64 tensor-train construction used at set-up time: quantics
// vectors and 1-D CFD2 operators, Kronecker products over dimensions, sums,
// operator products and compression.  Nothing here runs inside the time step.
#pragma once

#include <cstdint>
#include <vector>

namespace qtt {
namespace host {

// core [rl][p][rr] row-major; p = 2 for an MPS, 4 (= t*2 + s) for an MPO
struct Core {
  int rl = 1, p = 2, rr = 1;
  std::vector<double> v;
  Core() = default;
  Core(int a, int pp, int b) : rl(a), p(pp), rr(b), v((size_t)a * pp * b, 0.0) {}
  double& at(int a, int s, int b) { return v[((size_t)a * p + s) * rr + b]; }
  double at(int a, int s, int b) const { return v[((size_t)a * p + s) * rr + b]; }
};
using TT = std::vector<Core>;

// dense linear algebra (row-major)
void qr_thin(int m, int n, const double* A, std::vector<double>& Q, std::vector<double>& R, int& k);
// one-sided Jacobi SVD, descending singular values; U (m x k), S (k), Vt (k x n), k = min(m, n)
void svd_thin(int m, int n, const double* A, std::vector<double>& U, std::vector<double>& S,
              std::vector<double>& Vt);

// quantics vector (TT-SVD, relative tolerance on singular values)
TT vector_qtt(const double* v, int bits, double rel_tol = 1e-15);
TT ones_qtt(int bits);

// 1-D CFD2 operators on M = 2^bits points (op codes of tt_op1d), compressed
TT op1d(int op, int bits);

// (dimension, bit) of every site for a grid of ndims dimensions
std::vector<std::pair<int, int>> site_order(int ndims, int bits, int ordering);

// Kronecker product over dimensions in the given site order; per_dim[d] may
// be empty (all-ones vector for p == 2, identity for p == 4)
TT kron_dims(const std::vector<const TT*>& per_dim, const std::vector<std::pair<int, int>>& order,
             int ndims, int p);

// block-diagonal sum of several chains (coefficient on the first core)
TT tt_sum(const std::vector<std::pair<double, const TT*>>& terms);
// MPO product A * B
TT mpo_compose(const TT& A, const TT& B);
// diag(x) for an MPS x
TT mpo_diag(const TT& x);
// exact MPO x MPS product W x (bonds multiply)
TT mpo_apply(const TT& W, const TT& x);
// identity MPO over n sites
TT mpo_identity(int n);
// Periodic linear interpolation onto the grid of twice the resolution, on the
// bits sites of one dimension followed by a new least significant site that
// holds a copy of the coarse value (an identity core on the bond): the MPO
// I + (S+ - I) (x) diag(0, 1/2), so that a lifted value f(j) at digit b
// becomes f(j) + b (f(j+1 mod M) - f(j)) / 2 (bits + 1 sites, compressed)
TT prolong_block(int bits);

// textbook rounding (QR sweep + right-to-left truncated SVDs) with a
// relative tolerance per bond -- used to compress operators
TT round_svd(const TT& x, double rel_tol, int max_bond);
// LQ sweep + QR sweep + simultaneous truncation of every bond to
// min(chi, 2^n, 2^(N-n)) leading left singular vectors (Gram eigenvectors)
TT round_gram(const TT& x, int chi);

}  // namespace host
}  // namespace qtt
