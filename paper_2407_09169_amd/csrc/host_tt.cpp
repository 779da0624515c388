// Host FP64 tensor-train construction (set-up only).  See host_tt.h.
#include "host_tt.h"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <stdexcept>

#include "../../include/qttpdf.h"

namespace qtt {
namespace host {

// ---------------------------------------------------------------------------
// dense linear algebra
// ---------------------------------------------------------------------------
void qr_thin(int m, int n, const double* A, std::vector<double>& Q, std::vector<double>& R, int& k) {
  k = std::min(m, n);
  std::vector<double> W((size_t)m * n);  // column-major
  for (int r = 0; r < m; ++r)
    for (int c = 0; c < n; ++c) W[(size_t)c * m + r] = A[(size_t)r * n + c];
  std::vector<double> tau(k, 0.0), beta(k, 0.0);
  for (int j = 0; j < k; ++j) {
    double* cj = &W[(size_t)j * m];
    double sig = 0.0;
    for (int r = j + 1; r < m; ++r) sig += cj[r] * cj[r];
    double x0 = cj[j];
    if (sig == 0.0) {
      tau[j] = 0.0;
      beta[j] = x0;
      continue;
    }
    double nrm = std::sqrt(x0 * x0 + sig);
    double b = x0 >= 0.0 ? -nrm : nrm;
    tau[j] = (b - x0) / b;
    beta[j] = b;
    double sc = 1.0 / (x0 - b);
    for (int r = j + 1; r < m; ++r) cj[r] *= sc;
    for (int c = j + 1; c < n; ++c) {
      double* cc = &W[(size_t)c * m];
      double w = cc[j];
      for (int r = j + 1; r < m; ++r) w += cj[r] * cc[r];
      w *= tau[j];
      cc[j] -= w;
      for (int r = j + 1; r < m; ++r) cc[r] -= w * cj[r];
    }
  }
  R.assign((size_t)k * n, 0.0);
  for (int r = 0; r < k; ++r)
    for (int c = r; c < n; ++c) R[(size_t)r * n + c] = (r == c) ? beta[r] : W[(size_t)c * m + r];
  // Q = H_0 ... H_{k-1} [I_k; 0]
  std::vector<double> Qc((size_t)m * k, 0.0);  // column-major
  for (int c = 0; c < k; ++c) Qc[(size_t)c * m + c] = 1.0;
  for (int j = k - 1; j >= 0; --j) {
    if (tau[j] == 0.0) continue;
    const double* v = &W[(size_t)j * m];
    for (int c = 0; c < k; ++c) {
      double* qc = &Qc[(size_t)c * m];
      double w = qc[j];
      for (int r = j + 1; r < m; ++r) w += v[r] * qc[r];
      w *= tau[j];
      qc[j] -= w;
      for (int r = j + 1; r < m; ++r) qc[r] -= w * v[r];
    }
  }
  Q.assign((size_t)m * k, 0.0);
  for (int r = 0; r < m; ++r)
    for (int c = 0; c < k; ++c) Q[(size_t)r * k + c] = Qc[(size_t)c * m + r];
}

static void jacobi_cols(int m, int n, std::vector<double>& B, std::vector<double>& V) {
  // one-sided Jacobi on the columns of B (column-major m x n); V accumulates rotations
  V.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    bool rot = false;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double* bp = &B[(size_t)p * m];
        double* bq = &B[(size_t)q * m];
        double a = 0, b = 0, g = 0;
        for (int r = 0; r < m; ++r) {
          a += bp[r] * bp[r];
          b += bq[r] * bq[r];
          g += bp[r] * bq[r];
        }
        if (g == 0.0 || std::fabs(g) <= 1e-15 * std::sqrt(a * b)) continue;
        rot = true;
        double zeta = (b - a) / (2 * g);
        double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1 + zeta * zeta));
        double c = 1 / std::sqrt(1 + t * t), s = c * t;
        for (int r = 0; r < m; ++r) {
          double x = bp[r], y = bq[r];
          bp[r] = c * x - s * y;
          bq[r] = s * x + c * y;
        }
        double* vp = &V[(size_t)p * n];
        double* vq = &V[(size_t)q * n];
        for (int r = 0; r < n; ++r) {
          double x = vp[r], y = vq[r];
          vp[r] = c * x - s * y;
          vq[r] = s * x + c * y;
        }
      }
    if (!rot) break;
  }
}

void svd_thin(int m, int n, const double* A, std::vector<double>& U, std::vector<double>& S,
              std::vector<double>& Vt) {
  bool tr = m < n;
  int mm = tr ? n : m, nn = tr ? m : n;  // work on a tall matrix mm x nn
  std::vector<double> B((size_t)mm * nn), V;
  for (int r = 0; r < mm; ++r)
    for (int c = 0; c < nn; ++c)
      B[(size_t)c * mm + r] = tr ? A[(size_t)c * n + r] : A[(size_t)r * n + c];
  jacobi_cols(mm, nn, B, V);
  int k = nn;
  std::vector<double> sig(k);
  for (int c = 0; c < k; ++c) {
    double s = 0;
    for (int r = 0; r < mm; ++r) s += B[(size_t)c * mm + r] * B[(size_t)c * mm + r];
    sig[c] = std::sqrt(s);
  }
  std::vector<int> idx(k);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return sig[a] > sig[b]; });
  // tall: A' = Ut S Vt', with Ut = B/sig (mm x k), V' = V (nn x k)
  std::vector<double> Ut((size_t)mm * k), Vp((size_t)nn * k);
  S.assign(k, 0.0);
  for (int j = 0; j < k; ++j) {
    int c = idx[j];
    S[j] = sig[c];
    for (int r = 0; r < mm; ++r) Ut[(size_t)r * k + j] = sig[c] > 0 ? B[(size_t)c * mm + r] / sig[c] : 0.0;
    for (int r = 0; r < nn; ++r) Vp[(size_t)r * k + j] = V[(size_t)c * nn + r];
  }
  if (!tr) {
    U = Ut;  // m x k
    Vt.assign((size_t)k * n, 0.0);
    for (int j = 0; j < k; ++j)
      for (int c = 0; c < n; ++c) Vt[(size_t)j * n + c] = Vp[(size_t)c * k + j];
  } else {
    // A^T = Ut S Vp^T  =>  A = Vp S Ut^T
    U = Vp;  // m x k (m == nn)
    Vt.assign((size_t)k * n, 0.0);
    for (int j = 0; j < k; ++j)
      for (int c = 0; c < n; ++c) Vt[(size_t)j * n + c] = Ut[(size_t)c * k + j];
  }
}

// ---------------------------------------------------------------------------
// chains
// ---------------------------------------------------------------------------
TT vector_qtt(const double* v, int bits, double rel_tol) {
  TT out;
  int M = 1 << bits;
  std::vector<double> C(v, v + M);
  int r = 1;
  for (int n = 0; n < bits - 1; ++n) {
    int rows = r * 2, cols = (int)(C.size() / rows);
    std::vector<double> U, S, Vt;
    svd_thin(rows, cols, C.data(), U, S, Vt);
    int kmax = (int)S.size();
    int k = 1;
    if (S[0] > 0)
      for (k = 0; k < kmax && S[k] > rel_tol * S[0]; ++k) {
      }
    k = std::max(1, k);
    Core G(r, 2, k);
    for (int a = 0; a < r; ++a)
      for (int s = 0; s < 2; ++s)
        for (int b = 0; b < k; ++b) G.at(a, s, b) = U[(size_t)(a * 2 + s) * kmax + b];
    out.push_back(G);
    std::vector<double> Cn((size_t)k * cols);
    for (int b = 0; b < k; ++b)
      for (int c = 0; c < cols; ++c) Cn[(size_t)b * cols + c] = S[b] * Vt[(size_t)b * cols + c];
    C.swap(Cn);
    r = k;
  }
  Core G(r, 2, 1);
  for (int a = 0; a < r; ++a)
    for (int s = 0; s < 2; ++s) G.at(a, s, 0) = C[(size_t)a * 2 + s];
  out.push_back(G);
  return out;
}

TT ones_qtt(int bits) {
  TT out;
  for (int n = 0; n < bits; ++n) {
    Core G(1, 2, 1);
    G.v[0] = G.v[1] = 1.0;
    out.push_back(G);
  }
  return out;
}

TT mpo_identity(int n) {
  TT out;
  for (int i = 0; i < n; ++i) {
    Core G(1, 4, 1);
    G.v[0] = 1.0;  // t=0,s=0
    G.v[3] = 1.0;  // t=1,s=1
    out.push_back(G);
  }
  return out;
}

// shift by +1 (y_i = x_{i+1}) in MSB-first quantics form: the bond carries the
// carry of i + 1 from the less significant digits; open boundary: no carry
// out of the most significant digit; periodic: carry out allowed (wrap).
static TT shift_plus(int bits, bool periodic) {
  TT out;
  for (int n = 0; n < bits; ++n) {
    int rl = (n == 0) ? 1 : 2, rr = (n == bits - 1) ? 1 : 2;
    Core G(rl, 4, rr);
    for (int t = 0; t < 2; ++t)
      for (int beta = 0; beta < 2; ++beta) {
        if (n == bits - 1 && beta != 1) continue;  // carry into the LSB is 1
        int s = t ^ beta, alpha = t & beta;
        int bi = (n == bits - 1) ? 0 : beta;
        if (n == 0) {
          if (!periodic && alpha != 0) continue;
          G.at(0, t * 2 + s, bi) += 1.0;
        } else {
          G.at(alpha, t * 2 + s, bi) += 1.0;
        }
      }
    out.push_back(G);
  }
  return out;
}

static TT transpose_mpo(const TT& A) {
  TT out = A;
  for (auto& G : out)
    for (int a = 0; a < G.rl; ++a)
      for (int b = 0; b < G.rr; ++b) std::swap(G.at(a, 1, b), G.at(a, 2, b));
  return out;
}

static TT corner(int bits, int bit) {
  TT out;
  for (int n = 0; n < bits; ++n) {
    Core G(1, 4, 1);
    G.v[bit * 2 + bit] = 1.0;
    out.push_back(G);
  }
  return out;
}

// diag(phi_i), phi_i = h (i + 1/2) = h/2 + sum_n h 2^(bits-1-n) i_n (rank 2)
static TT phi_diag(int bits) {
  double h = 1.0 / (double)(1 << bits);
  TT out;
  for (int n = 0; n < bits; ++n) {
    double c = h * (double)(1 << (bits - 1 - n));
    int rl = (n == 0) ? 1 : 2, rr = (n == bits - 1) ? 1 : 2;
    Core G(rl, 4, rr);
    for (int t = 0; t < 2; ++t) {
      int ts = t * 2 + t;
      if (bits == 1) {
        G.at(0, ts, 0) = 0.5 * h + c * t;
      } else if (n == 0) {
        G.at(0, ts, 0) = 1.0;
        G.at(0, ts, 1) = 0.5 * h + c * t;
      } else if (n == bits - 1) {
        G.at(0, ts, 0) = c * t;
        G.at(1, ts, 0) = 1.0;
      } else {
        G.at(0, ts, 0) = 1.0;
        G.at(0, ts, 1) = c * t;
        G.at(1, ts, 1) = 1.0;
      }
    }
    out.push_back(G);
  }
  return out;
}

TT op1d(int op, int bits) {
  double h = 1.0 / (double)(1 << bits);
  if (op == TT_OP_ID) return mpo_identity(bits);
  if (op == TT_OP_PHI) return round_svd(phi_diag(bits), 1e-15, 1 << 30);
  TT I = mpo_identity(bits);
  TT E0 = corner(bits, 0), E1 = corner(bits, 1);
  bool periodic = (op == TT_OP_D1P || op == TT_OP_D2P);
  TT Sp = shift_plus(bits, periodic), Sm = transpose_mpo(Sp);
  TT out;
  switch (op) {
    case TT_OP_D1G:
      out = tt_sum({{0.5 / h, &Sp}, {-0.5 / h, &Sm}, {0.5 / h, &E0}, {-0.5 / h, &E1}});
      break;
    case TT_OP_D2G:
      out = tt_sum({{1 / (h * h), &Sp}, {1 / (h * h), &Sm}, {-2 / (h * h), &I},
                    {1 / (h * h), &E0}, {1 / (h * h), &E1}});
      break;
    case TT_OP_D1P:
      out = tt_sum({{0.5 / h, &Sp}, {-0.5 / h, &Sm}});
      break;
    case TT_OP_D2P:
      out = tt_sum({{1 / (h * h), &Sp}, {1 / (h * h), &Sm}, {-2 / (h * h), &I}});
      break;
    case TT_OP_D1G_PHI: {
      TT d1 = op1d(TT_OP_D1G, bits), ph = phi_diag(bits);
      out = mpo_compose(d1, ph);
      break;
    }
    default:
      throw std::invalid_argument("unknown 1-D operator");
  }
  return round_svd(out, 1e-15, 1 << 30);
}

TT prolong_block(int bits) {
  Core E11(1, 4, 1);
  E11.at(0, 3, 0) = 1.0;  // t = s = 1
  TT I = mpo_identity(bits + 1);
  TT S = shift_plus(bits, true);
  S.push_back(E11);
  TT D = mpo_identity(bits);
  D.push_back(E11);
  return round_svd(tt_sum({{1.0, &I}, {0.5, &S}, {-0.5, &D}}), 1e-15, 1 << 30);
}

std::vector<std::pair<int, int>> site_order(int ndims, int bits, int ordering) {
  std::vector<std::pair<int, int>> o;
  if (ordering == TT_SERIAL) {
    for (int d = 0; d < ndims; ++d)
      for (int b = 0; b < bits; ++b) o.emplace_back(d, b);
  } else {
    for (int b = 0; b < bits; ++b)
      for (int d = 0; d < ndims; ++d) o.emplace_back(d, b);
  }
  return o;
}

TT kron_dims(const std::vector<const TT*>& per_dim, const std::vector<std::pair<int, int>>& order,
             int ndims, int p) {
  int bits = (int)order.size() / ndims;
  TT ones = (p == 2) ? ones_qtt(bits) : mpo_identity(bits);
  std::vector<const TT*> pd(ndims);
  for (int d = 0; d < ndims; ++d) pd[d] = (per_dim[d] && !per_dim[d]->empty()) ? per_dim[d] : &ones;
  std::vector<int> pos(ndims, 0);
  auto bond = [&](int d, int q) { return q < bits ? (*pd[d])[q].rl : 1; };
  TT out;
  for (auto [d, b] : order) {
    const Core& G = (*pd[d])[b];
    int pre = 1, post = 1;
    for (int e = 0; e < d; ++e) pre *= bond(e, pos[e]);
    for (int e = d + 1; e < ndims; ++e) post *= bond(e, pos[e]);
    Core K(pre * G.rl * post, p, pre * G.rr * post);
    for (int P = 0; P < pre; ++P)
      for (int Q = 0; Q < post; ++Q)
        for (int a = 0; a < G.rl; ++a)
          for (int s = 0; s < p; ++s)
            for (int bb = 0; bb < G.rr; ++bb)
              K.at((P * G.rl + a) * post + Q, s, (P * G.rr + bb) * post + Q) = G.at(a, s, bb);
    out.push_back(std::move(K));
    pos[d] += 1;
  }
  return out;
}

TT tt_sum(const std::vector<std::pair<double, const TT*>>& terms) {
  size_t N = terms[0].second->size();
  int p = (*terms[0].second)[0].p;
  TT out;
  if (N == 1) {
    Core G(1, p, 1);
    for (auto& [c, x] : terms)
      for (int s = 0; s < p; ++s) G.v[s] += c * (*x)[0].v[s];
    out.push_back(G);
    return out;
  }
  for (size_t n = 0; n < N; ++n) {
    int rl = 0, rr = 0;
    for (auto& [c, x] : terms) {
      rl += (*x)[n].rl;
      rr += (*x)[n].rr;
    }
    if (n == 0) rl = 1;
    if (n == N - 1) rr = 1;
    Core G(rl, p, rr);
    int io = 0, jo = 0;
    for (auto& [c, x] : terms) {
      const Core& B = (*x)[n];
      double f = (n == 0) ? c : 1.0;
      for (int a = 0; a < B.rl; ++a)
        for (int s = 0; s < p; ++s)
          for (int b = 0; b < B.rr; ++b)
            G.at((n == 0 ? 0 : io) + a, s, (n == N - 1 ? 0 : jo) + b) += f * B.at(a, s, b);
      io += B.rl;
      jo += B.rr;
    }
    out.push_back(std::move(G));
  }
  return out;
}

TT mpo_compose(const TT& A, const TT& B) {
  TT out;
  for (size_t n = 0; n < A.size(); ++n) {
    const Core &a = A[n], &b = B[n];
    Core G(a.rl * b.rl, 4, a.rr * b.rr);
    for (int al = 0; al < a.rl; ++al)
      for (int bl = 0; bl < b.rl; ++bl)
        for (int t = 0; t < 2; ++t)
          for (int s = 0; s < 2; ++s)
            for (int ar = 0; ar < a.rr; ++ar)
              for (int br = 0; br < b.rr; ++br) {
                double v = 0;
                for (int u = 0; u < 2; ++u) v += a.at(al, t * 2 + u, ar) * b.at(bl, u * 2 + s, br);
                G.at(al * b.rl + bl, t * 2 + s, ar * b.rr + br) = v;
              }
    out.push_back(std::move(G));
  }
  return out;
}

TT mpo_apply(const TT& W, const TT& x) {
  TT out;
  for (size_t n = 0; n < x.size(); ++n) {
    const Core &A = W[n], &B = x[n];
    // out[(b, alpha), t, (c, beta)] = sum_s A[alpha, t, s, beta] B[b, s, c]
    Core G(B.rl * A.rl, 2, B.rr * A.rr);
    for (int b = 0; b < B.rl; ++b)
      for (int al = 0; al < A.rl; ++al)
        for (int t = 0; t < 2; ++t)
          for (int c = 0; c < B.rr; ++c)
            for (int be = 0; be < A.rr; ++be) {
              double v = 0.0;
              for (int s2 = 0; s2 < 2; ++s2) v += A.at(al, t * 2 + s2, be) * B.at(b, s2, c);
              G.at(b * A.rl + al, t, c * A.rr + be) = v;
            }
    out.push_back(std::move(G));
  }
  return out;
}

TT mpo_diag(const TT& x) {
  TT out;
  for (const Core& G : x) {
    Core W(G.rl, 4, G.rr);
    for (int a = 0; a < G.rl; ++a)
      for (int b = 0; b < G.rr; ++b) {
        W.at(a, 0, b) = G.at(a, 0, b);
        W.at(a, 3, b) = G.at(a, 1, b);
      }
    out.push_back(std::move(W));
  }
  return out;
}

// ---------------------------------------------------------------------------
// rounding
// ---------------------------------------------------------------------------
static void left_orth(TT& x) {
  for (size_t n = 0; n + 1 < x.size(); ++n) {
    Core& G = x[n];
    int m = G.rl * G.p, nn = G.rr, k;
    std::vector<double> Q, R;
    qr_thin(m, nn, G.v.data(), Q, R, k);
    Core Gn(G.rl, G.p, k);
    Gn.v = Q;
    Core& H = x[n + 1];
    Core Hn(k, H.p, H.rr);
    for (int a = 0; a < k; ++a)
      for (int c = 0; c < H.p * H.rr; ++c) {
        double v = 0;
        for (int b = 0; b < nn; ++b) v += R[(size_t)a * nn + b] * H.v[(size_t)b * H.p * H.rr + c];
        Hn.v[(size_t)a * H.p * H.rr + c] = v;
      }
    x[n] = std::move(Gn);
    x[n + 1] = std::move(Hn);
  }
}

static void right_orth(TT& x) {
  for (size_t n = x.size() - 1; n >= 1; --n) {
    Core& G = x[n];
    int rows = G.rl, cols = G.p * G.rr;
    // A = L Q from the QR of A^T
    std::vector<double> At((size_t)cols * rows);
    for (int r = 0; r < rows; ++r)
      for (int c = 0; c < cols; ++c) At[(size_t)c * rows + r] = G.v[(size_t)r * cols + c];
    std::vector<double> Q, R;
    int k;
    qr_thin(cols, rows, At.data(), Q, R, k);  // Q: cols x k, R: k x rows
    Core Gn(k, G.p, G.rr);
    for (int a = 0; a < k; ++a)
      for (int c = 0; c < cols; ++c) Gn.v[(size_t)a * cols + c] = Q[(size_t)c * k + a];
    Core& H = x[n - 1];
    int hm = H.rl * H.p;
    Core Hn(H.rl, H.p, k);
    for (int r = 0; r < hm; ++r)
      for (int a = 0; a < k; ++a) {
        double v = 0;
        for (int b = 0; b < rows; ++b) v += H.v[(size_t)r * H.rr + b] * R[(size_t)a * rows + b];
        Hn.v[(size_t)r * k + a] = v;
      }
    x[n] = std::move(Gn);
    x[n - 1] = std::move(Hn);
  }
}

TT round_svd(const TT& x0, double rel_tol, int max_bond) {
  TT x = x0;
  if (x.size() == 1) return x;
  left_orth(x);
  for (size_t n = x.size() - 1; n >= 1; --n) {
    Core& G = x[n];
    int rows = G.rl, cols = G.p * G.rr;
    std::vector<double> U, S, Vt;
    svd_thin(rows, cols, G.v.data(), U, S, Vt);
    int kk = (int)S.size(), k = 0;
    if (S[0] > 0)
      while (k < kk && S[k] > rel_tol * S[0]) ++k;
    k = std::max(1, std::min(k, max_bond));
    Core Gn(k, G.p, G.rr);
    for (int a = 0; a < k; ++a)
      for (int c = 0; c < cols; ++c) Gn.v[(size_t)a * cols + c] = Vt[(size_t)a * cols + c];
    Core& H = x[n - 1];
    int hm = H.rl * H.p;
    Core Hn(H.rl, H.p, k);
    for (int r = 0; r < hm; ++r)
      for (int a = 0; a < k; ++a) {
        double v = 0;
        for (int b = 0; b < rows; ++b) v += H.v[(size_t)r * H.rr + b] * U[(size_t)b * kk + a] * S[a];
        Hn.v[(size_t)r * k + a] = v;
      }
    x[n] = std::move(Gn);
    x[n - 1] = std::move(Hn);
  }
  return x;
}

TT round_gram(const TT& x0, int chi) {
  TT X = x0;
  size_t N = X.size();
  if (N == 1) return X;
  right_orth(X);
  left_orth(X);
  // right Gram matrices Gam[n] (bond left of site n), n = 1..N-1
  std::vector<std::vector<double>> Gam(N);
  {
    const Core& L = X[N - 1];
    int l = L.rl;
    Gam[N - 1].assign((size_t)l * l, 0.0);
    for (int a = 0; a < l; ++a)
      for (int b = 0; b < l; ++b) {
        double v = 0;
        for (int s = 0; s < 2; ++s) v += L.at(a, s, 0) * L.at(b, s, 0);
        Gam[N - 1][(size_t)a * l + b] = v;
      }
  }
  for (size_t n = N - 2; n >= 1; --n) {
    const Core& A = X[n];
    const std::vector<double>& Gn = Gam[n + 1];
    int l = A.rl, r = A.rr;
    std::vector<double> T((size_t)l * 2 * r, 0.0);
    for (int a = 0; a < l; ++a)
      for (int s = 0; s < 2; ++s)
        for (int c = 0; c < r; ++c) {
          double v = 0;
          for (int b = 0; b < r; ++b) v += A.at(a, s, b) * Gn[(size_t)b * r + c];
          T[((size_t)a * 2 + s) * r + c] = v;
        }
    Gam[n].assign((size_t)l * l, 0.0);
    for (int a = 0; a < l; ++a)
      for (int d = 0; d < l; ++d) {
        double v = 0;
        for (int s = 0; s < 2; ++s)
          for (int c = 0; c < r; ++c) v += T[((size_t)a * 2 + s) * r + c] * A.at(d, s, c);
        Gam[n][(size_t)a * l + d] = v;
      }
    if (n == 1) break;
  }
  std::vector<std::vector<double>> P(N);
  std::vector<int> kk(N + 1, 1);
  for (size_t n = 1; n < N; ++n) {
    int l = X[n].rl;
    std::vector<double> U, S, Vt;
    svd_thin(l, l, Gam[n].data(), U, S, Vt);  // PSD: Vt rows are eigenvectors
    long cap = std::min<long>(chi, std::min<long>(1L << std::min<size_t>(n, 40), 1L << std::min<size_t>(N - n, 40)));
    int k = (int)std::max<long>(1, std::min<long>(cap, l));
    P[n].assign((size_t)l * k, 0.0);
    for (int a = 0; a < l; ++a)
      for (int c = 0; c < k; ++c) P[n][(size_t)a * k + c] = Vt[(size_t)c * l + a];
    kk[n] = k;
  }
  TT out;
  for (size_t n = 0; n < N; ++n) {
    const Core& A = X[n];
    int kl = (n == 0) ? A.rl : kk[n];
    int kr = (n == N - 1) ? A.rr : kk[n + 1];
    Core G(kl, 2, kr);
    for (int c = 0; c < kl; ++c)
      for (int s = 0; s < 2; ++s)
        for (int e = 0; e < kr; ++e) {
          double v = 0;
          for (int a = 0; a < A.rl; ++a) {
            double pa = (n == 0) ? (a == c ? 1.0 : 0.0) : P[n][(size_t)a * kl + c];
            if (pa == 0.0) continue;
            for (int b = 0; b < A.rr; ++b) {
              double pb = (n == N - 1) ? (b == e ? 1.0 : 0.0) : P[n + 1][(size_t)b * kr + e];
              v += pa * A.at(a, s, b) * pb;
            }
          }
          G.at(c, s, e) = v;
        }
    out.push_back(std::move(G));
  }
  return out;
}

}  // namespace host
}  // namespace qtt
