// Two-sided randomized rounding of Y = sum_j c_j W_j x_j.
//
// The chain is orthogonalised from both ends towards its middle site c:
//   * sites 0..c-1 by the left-to-right sweep of the one-sided range finder
//     (sketched unfoldings S_n = [X_(<n)^T Y]_n Right_(n+1)(Y) Right_(n+1)(Zr)^T,
//     X_n = Householder Q of S_n), giving left-orthogonal cores;
//   * sites N-1..c+1 by the mirrored right-to-left sweep with the left
//     sketches Left_n(Zl)^T Left_n(Y) (V_n = Q of the transposed sketched
//     unfolding), giving right-orthogonal cores;
//   * the centre core X_(<c)^T Y V_(>c)^T.
// The two sweeps and, before them, the two families of partial sketches are
// independent and run on separate lanes, so the sequential chain of QR
// factorisations is half as long as in the one-sided sweep.
//
// Truncation of the mixed canonical form: at a bond n <= c the left part is
// orthonormal and the right Gram matrix decides (Gamma_c = G G^T from the
// centre core G, then the chain through X_(c-1)..X_1); at a bond n > c the
// right part is orthonormal and the left Gram matrix decides (Lambda_(c+1) =
// G^T G, then the chain through V_(c+1)..).  One batched eigen-decomposition
// over all bonds, then the cores P_n^T A_n P_(n+1).
//
// Layouts: an MPS core is [r][2][r'] row-major, an MPO core [D][2 out][2 in][D'].
// Right sketches R[(a,A), z] (r_n D_n x ell_n), left sketches Lk[y, (a,A)]
// (ell_n x r_n D_n), left-sweep cores C[(k,t), (b,B)], right-sweep cores
// Cr[(a,A), (t,z)], right-orthogonal cores kept as Vt[(t,z), y] = V[y,t,z]
// (the Q factor of the transposed sketch, as the QR kernel returns it).
#include <algorithm>

#include "library.h"

namespace qtt {

namespace {

Mode2 M1(int64_t s) { return mode1(s); }
Mode2 M2(int n2, int64_t s1, int64_t s2) { return mode2(n2, s1, s2); }

struct Shape {
  std::vector<int> r, D;  // bonds of the term's MPS and MPO (D = 1: identity)
};

// R_out[(a,A), z] = sum x[a,s,b] W[A,t,s,B] R_in[(b,B), z'] Z[z,t,z']  (site n): the
// launches of one term, in order
std::vector<TcDesc> rsketch_descs(const SketchTerm& t, const Shape& sh, const ChainView& Z, int n,
                                  const double* Rin, double* Rout, double* T1, double* T2) {
  std::vector<TcDesc> out;
  const int l = Z.caps[n], lp = Z.caps[n + 1];
  const int rn = sh.r[n], rp = sh.r[n + 1], Dn = sh.D[n], Dp = sh.D[n + 1];
  {  // T1[(b,B),(t,z)] = sum_z' R_in[(b,B),z'] Z[z,t,z']
    TcDesc d;
    d.M = rp * Dp;
    d.N = 2 * l;
    d.K = lp;
    d.A = Rin;
    d.am = M1(lp);
    d.ak = M1(1);
    d.B = Z.core[n];
    d.bk = M1(1);
    d.bn = M2(l, lp, 2 * lp);
    d.C = T1;
    d.cm = M1(2 * l);
    d.cn = M1(1);
    d.ab = d.bb = d.cb = M1(0);
    out.push_back(d);
  }
  if (t.diag_at(n)) {
    {  // T2[(A,s), b, z] = sum_B W[A,s,s,B] T1[(b,B),(s,z)], batch (b, s)
      TcDesc d;
      d.batch = 2 * rp;
      d.M = Dn;
      d.K = Dp;
      d.N = l;
      d.A = t.mpo->core[n];
      d.am = M1(4 * Dp);
      d.ak = M1(1);
      d.ab = M2(2, 0, 3 * Dp);
      d.B = T1;
      d.bk = M1(2 * l);
      d.bn = M1(1);
      d.bb = M2(2, (int64_t)Dp * 2 * l, l);
      d.C = T2;
      d.cm = M1((int64_t)2 * rp * l);
      d.cn = M1(1);
      d.cb = M2(2, l, (int64_t)rp * l);
      out.push_back(d);
    }
  }
  if (t.mpo && !t.diag_at(n)) {
    {  // T2[(A,s), b, z] = sum_(B,t) W[A,t,s,B] T1[(b,B),(t,z)], batch b
      TcDesc d;
      d.batch = rp;
      d.M = 2 * Dn;
      d.K = 2 * Dp;
      d.N = l;
      d.A = t.mpo->core[n];
      d.am = M2(2, 4 * Dp, Dp);
      d.ak = M2(2, 1, 2 * Dp);
      d.ab = M1(0);
      d.B = T1;
      d.bk = M2(2, 2 * l, l);
      d.bn = M1(1);
      d.bb = M1((int64_t)Dp * 2 * l);
      d.C = T2;
      d.cm = M1((int64_t)rp * l);
      d.cn = M1(1);
      d.cb = M1(l);
      out.push_back(d);
    }
  }
  if (t.mpo) {
    {  // R_out[(a,A),z] = sum_(s,b) x[a,s,b] T2[A,s,b,z], batch A
      TcDesc d;
      d.batch = Dn;
      d.M = rn;
      d.K = 2 * rp;
      d.N = l;
      d.A = t.x.core[n];
      d.am = M1(2 * rp);
      d.ak = M1(1);
      d.ab = M1(0);
      d.B = T2;
      d.bk = M1(l);
      d.bn = M1(1);
      d.bb = M1((int64_t)2 * rp * l);
      d.C = Rout;
      d.cm = M1((int64_t)Dn * l);
      d.cn = M1(1);
      d.cb = M1(l);
      out.push_back(d);
    }
  } else {  // R_out[a,z] = sum_(s,b) x[a,s,b] T1[b,(s,z)]
    TcDesc d;
    d.M = rn;
    d.K = 2 * rp;
    d.N = l;
    d.A = t.x.core[n];
    d.am = M1(2 * rp);
    d.ak = M1(1);
    d.B = T1;
    d.bk = M2(rp, l, 2 * l);
    d.bn = M1(1);
    d.C = Rout;
    d.cm = M1(l);
    d.cn = M1(1);
    d.ab = d.bb = d.cb = M1(0);
    out.push_back(d);
  }
  return out;
}

// L_out[z, (b,B)] = sum Zl[y,t,z] L_in[y,(a,A)] x[a,s,b] W[A,t,s,B]  (site n): the
// launches of one term, in order
std::vector<TcDesc> lsketch_descs(const SketchTerm& t, const Shape& sh, const ChainView& Zl, int n,
                                  const double* Lin, double* Lout, double* T1, double* T2) {
  std::vector<TcDesc> out;
  const int l = Zl.caps[n], lp = Zl.caps[n + 1];
  const int rn = sh.r[n], rp = sh.r[n + 1], Dn = sh.D[n], Dp = sh.D[n + 1];
  {  // T1[(a,A),(t,z)] = sum_y L_in[y,(a,A)] Zl[y,(t,z)]
    TcDesc d;
    d.M = rn * Dn;
    d.N = 2 * lp;
    d.K = l;
    d.A = Lin;
    d.am = M1(1);
    d.ak = M1((int64_t)rn * Dn);
    d.B = Zl.core[n];
    d.bk = M1(2 * lp);
    d.bn = M1(1);
    d.C = T1;
    d.cm = M1(2 * lp);
    d.cn = M1(1);
    d.ab = d.bb = d.cb = M1(0);
    out.push_back(d);
  }
  if (t.diag_at(n)) {
    {  // T2[a,(s,B),z] = sum_A W[A,s,s,B] T1[(a,A),(s,z)], batch (a, s)
      TcDesc d;
      d.batch = 2 * rn;
      d.M = Dp;
      d.K = Dn;
      d.N = lp;
      d.A = t.mpo->core[n];
      d.am = M1(1);
      d.ak = M1(4 * Dp);
      d.ab = M2(2, 0, 3 * Dp);
      d.B = T1;
      d.bk = M1(2 * lp);
      d.bn = M1(1);
      d.bb = M2(2, (int64_t)Dn * 2 * lp, lp);
      d.C = T2;
      d.cm = M1(lp);
      d.cn = M1(1);
      d.cb = M2(2, (int64_t)2 * Dp * lp, (int64_t)Dp * lp);
      out.push_back(d);
    }
  }
  if (t.mpo && !t.diag_at(n)) {
    {  // T2[a,(s,B),z] = sum_(A,t) W[A,t,s,B] T1[(a,A),(t,z)], batch a
      TcDesc d;
      d.batch = rn;
      d.M = 2 * Dp;
      d.K = 2 * Dn;
      d.N = lp;
      d.A = t.mpo->core[n];
      d.am = M1(1);
      d.ak = M1(2 * Dp);
      d.ab = M1(0);
      d.B = T1;
      d.bk = M1(lp);
      d.bn = M1(1);
      d.bb = M1((int64_t)Dn * 2 * lp);
      d.C = T2;
      d.cm = M1(lp);
      d.cn = M1(1);
      d.cb = M1((int64_t)2 * Dp * lp);
      out.push_back(d);
    }
  }
  if (t.mpo) {
    {  // L_out[z,(b,B)] = sum_(a,s) T2[a,(s,B),z] x[a,s,b], batch B
      TcDesc d;
      d.batch = Dp;
      d.M = lp;
      d.N = rp;
      d.K = 2 * rn;
      d.A = T2;
      d.am = M1(1);
      d.ak = M1((int64_t)Dp * lp);
      d.ab = M1(lp);
      d.B = t.x.core[n];
      d.bk = M1(rp);
      d.bn = M1(1);
      d.bb = M1(0);
      d.C = Lout;
      d.cm = M1((int64_t)rp * Dp);
      d.cn = M1(Dp);
      d.cb = M1(1);
      out.push_back(d);
    }
  } else {  // L_out[z,b] = sum_(a,s) T1[a,(s,z)] x[a,s,b]
    TcDesc d;
    d.M = lp;
    d.N = rp;
    d.K = 2 * rn;
    d.A = T1;
    d.am = M1(1);
    d.ak = M1(lp);
    d.B = t.x.core[n];
    d.bk = M1(rp);
    d.bn = M1(1);
    d.C = Lout;
    d.cm = M1(rp);
    d.cn = M1(1);
    d.ab = d.bb = d.cb = M1(0);
    out.push_back(d);
  }
  return out;
}

// C[(k,t),(b,B)] = alpha * sum M[k,(a,A)] x[a,s,b] W[A,t,s,B] + beta * C  (site n, l rows):
// the launches of one term, in order
std::vector<TcDesc> lcore_descs(const SketchTerm& t, const Shape& sh, int n, int l, const double* M, double* U1,
                                double* Cdst, double alpha, double beta) {
  const int rn = sh.r[n], rp = sh.r[n + 1], Dn = sh.D[n], Dp = sh.D[n + 1];
  if (!t.mpo)
    return {gemm_desc(l, 2 * rp, rn, M, rn, false, t.x.core[n], 2 * rp, false, Cdst, 2 * rp, alpha, beta)};
  std::vector<TcDesc> out(2);
  {  // U1[k,A,s,b] = sum_a M[k,(a,A)] x[a,s,b], batch A
    TcDesc& d = out[0];
    d.batch = Dn;
    d.M = l;
    d.K = rn;
    d.N = 2 * rp;
    d.A = M;
    d.am = M1((int64_t)rn * Dn);
    d.ak = M1(Dn);
    d.ab = M1(1);
    d.B = t.x.core[n];
    d.bk = M1(2 * rp);
    d.bn = M1(1);
    d.bb = M1(0);
    d.C = U1;
    d.cm = M1((int64_t)2 * Dn * rp);
    d.cn = M1(1);
    d.cb = M1(2 * rp);
  }
  if (t.diag_at(n)) {  // C[k,s,b,B] = sum_A U1[k,A,s,b] W[A,s,s,B], batch s
    TcDesc& d = out[1];
    d.batch = 2;
    d.M = l * rp;
    d.K = Dn;
    d.N = Dp;
    d.A = U1;
    d.am = M2(rp, (int64_t)2 * Dn * rp, 1);
    d.ak = M1(2 * rp);
    d.ab = M1(rp);
    d.B = t.mpo->core[n];
    d.bk = M1(4 * Dp);
    d.bn = M1(1);
    d.bb = M1(3 * Dp);
    d.C = Cdst;
    d.cm = M2(rp, (int64_t)2 * rp * Dp, Dp);
    d.cn = M1(1);
    d.cb = M1((int64_t)rp * Dp);
    d.alpha = alpha;
    d.beta = beta;
    return out;
  }
  {  // C[k,t,b,B] = sum_(A,s) U1[k,A,s,b] W[A,t,s,B]
    TcDesc& d = out[1];
    d.M = l * rp;
    d.K = 2 * Dn;
    d.N = 2 * Dp;
    d.A = U1;
    d.am = M2(rp, (int64_t)2 * Dn * rp, 1);
    d.ak = M1(rp);
    d.B = t.mpo->core[n];
    d.bk = M2(2, 4 * Dp, Dp);
    d.bn = M2(Dp, 2 * Dp, 1);
    d.C = Cdst;
    d.cm = M2(rp, (int64_t)2 * rp * Dp, Dp);
    d.cn = M2(Dp, (int64_t)rp * Dp, 1);
    d.ab = d.bb = d.cb = M1(0);
    d.alpha = alpha;
    d.beta = beta;
  }
  return out;
}

// Cr[(a,A),(t,z)] = sum x[a,s,b] W[A,t,s,B] Mr[(b,B),z]  (site n, lp columns of Mr):
// the launches of one term, in order
std::vector<TcDesc> rcore_descs(const SketchTerm& t, const Shape& sh, int n, int lp, const double* Mr, double* U1,
                                double* Cdst) {
  const int rn = sh.r[n], rp = sh.r[n + 1], Dn = sh.D[n], Dp = sh.D[n + 1];
  if (!t.mpo)  // Cr[(a,s),z] = sum_b x[a,s,b] Mr[b,z]
    return {gemm_desc(2 * rn, lp, rp, t.x.core[n], rp, false, Mr, lp, false, Cdst, lp, 1.0, 0.0)};
  std::vector<TcDesc> out(2);
  {  // U1[(a,s),B,z] = sum_b x[a,s,b] Mr[(b,B),z], batch B
    TcDesc& d = out[0];
    d.batch = Dp;
    d.M = 2 * rn;
    d.K = rp;
    d.N = lp;
    d.A = t.x.core[n];
    d.am = M1(rp);
    d.ak = M1(1);
    d.ab = M1(0);
    d.B = Mr;
    d.bk = M1((int64_t)Dp * lp);
    d.bn = M1(1);
    d.bb = M1(lp);
    d.C = U1;
    d.cm = M1((int64_t)Dp * lp);
    d.cn = M1(1);
    d.cb = M1(lp);
  }
  if (t.diag_at(n)) {  // Cr[(a,A),(s,z)] = sum_B W[A,s,s,B] U1[(a,s),B,z], batch s
    TcDesc& d = out[1];
    d.batch = 2;
    d.M = Dn;
    d.N = rn * lp;
    d.K = Dp;
    d.A = t.mpo->core[n];
    d.am = M1(4 * Dp);
    d.ak = M1(1);
    d.ab = M1(3 * Dp);
    d.B = U1;
    d.bk = M1(lp);
    d.bn = M2(lp, (int64_t)2 * Dp * lp, 1);
    d.bb = M1((int64_t)Dp * lp);
    d.C = Cdst;
    d.cm = M1(2 * lp);
    d.cn = M2(lp, (int64_t)Dn * 2 * lp, 1);
    d.cb = M1(lp);
    return out;
  }
  {  // Cr[(a,A),(t,z)] = sum_(s,B) W[(A,t),(s,B)] U1[(a,s),B,z]: rows (A,t), columns (a,z)
    TcDesc& d = out[1];
    d.M = 2 * Dn;
    d.N = rn * lp;
    d.K = 2 * Dp;
    d.A = t.mpo->core[n];
    d.am = M1(2 * Dp);
    d.ak = M1(1);
    d.B = U1;
    d.bk = M2(Dp, (int64_t)Dp * lp, lp);
    d.bn = M2(lp, (int64_t)2 * Dp * lp, 1);
    d.C = Cdst;
    d.cm = M1(lp);
    d.cn = M2(lp, (int64_t)Dn * 2 * lp, 1);
    d.ab = d.bb = d.cb = M1(0);
  }
  return out;
}

// one launch for the same contraction of several terms (same shapes and
// strides, own operands): pointer groups, summed into one result with gsum
void add_grouped(Plan& plan, const std::vector<TcDesc>& ds, bool gsum, Prec prec) {
  QTT_REQUIRE(!ds.empty() && (int)ds.size() <= TC_MAXG, "bad contraction group");
  if (ds.size() == 1) {
    add_tc(plan, ds[0], prec);
    return;
  }
  TcDesc d = ds[0];
  d.ng = (int)ds.size();
  d.gsum = gsum ? 1 : 0;
  for (int g = 0; g < d.ng; ++g) {
    const TcDesc& e = ds[g];
    QTT_REQUIRE(e.M == d.M && e.N == d.N && e.K == d.K && e.batch == d.batch && e.alpha == d.alpha &&
                    e.beta == d.beta && (!gsum || e.C == d.C),
                "grouped contractions differ in shape");
    d.gA[g] = e.A;
    d.gB[g] = e.B;
    d.gC[g] = e.C;
  }
  add_tc(plan, d, prec);
}

// ---------------------------------------------------------------------------
// One rounding while its phases are recorded.  Several independent roundings
// (same sketches, e.g. the two mean compositions) are recorded phase by phase
// side by side, their work items spread over the lanes; every phase forks
// from lane 0 and joins back to it.
// ---------------------------------------------------------------------------
struct TwoSided {
  const std::vector<SketchTerm>* terms = nullptr;
  RoundTarget* tg = nullptr;
  int J = 0, N = 0, c = 0;
  std::vector<Shape> sh;
  std::vector<std::vector<double*>> R, Lk;  // partial sketches per term and bond
  std::vector<double*> Ma, Mb, Cb, Mra, Mrb, Crb, U1L, U1R;
  std::vector<double*> T1, T2, L1, L2;  // sketch-chain scratch per term (right, left)
  double *SL = nullptr, *SR = nullptr, *qwL = nullptr, *qwR = nullptr;
  int64_t qwsz = 0;  // doubles in qwL, qwR
  // terms with the same operator and bonds, recorded as one launch per
  // contraction (pointer groups)
  std::vector<std::vector<int>> groups;
  std::vector<double*> X, Vt;  // left- / right-orthogonal cores
  double* Gc = nullptr;        // centre core
  std::vector<double*> Mcur, Mrcur;  // projections after the sweeps
  // truncation
  double *Gam = nullptr, *P = nullptr, *lam = nullptr, *ework = nullptr, *TgL = nullptr, *TgR = nullptr;
  int ldg = 1, ldp = 1, lmax = 1;
  int *d_dims = nullptr, *d_keep = nullptr;
  std::vector<int> dims_h, keep_h;
  size_t vsz = 1;
  double* G(int n) const { return Gam + (size_t)n * ldg * ldg; }
  double* Pn(int n) const { return P + (size_t)n * ldg * ldp; }
};

// shapes and buffers of one rounding; t1 / t2 / u1 grow to its scratch sizes
void ts_setup(Plan& plan, TwoSided& r, const std::vector<SketchTerm>& terms, RoundTarget& tg,
              const std::vector<int>& ell) {
  const int N = (int)ell.size() - 1;
  r.terms = &terms;
  r.tg = &tg;
  r.J = (int)terms.size();
  r.N = N;
  r.c = N / 2;
  const int J = r.J;
  QTT_REQUIRE(J >= 1, "rounding needs at least one term");
  QTT_REQUIRE((int)tg.caps.size() == N + 1 && (int)tg.core.size() == N, "truncation target shape");
  r.sh.resize(J);
  for (int j = 0; j < J; ++j) {
    QTT_REQUIRE(terms[j].x.N == N, "term length differs from the sketch");
    r.sh[j].r = terms[j].x.caps;
    if (terms[j].mpo) {
      QTT_REQUIRE(terms[j].mpo->N == N, "operator length differs from the sketch");
      r.sh[j].D = terms[j].mpo->caps;
    } else {
      r.sh[j].D.assign(N + 1, 1);
    }
  }
  size_t t1 = 1, t2 = 1, msz = 1, u1 = 1, csz = 1, crsz = 1, ssz = 1, qsz = 1;
  for (int j = 0; j < J; ++j)
    for (int n = 0; n < N; ++n) {
      const auto& rr = r.sh[j].r;
      const auto& D = r.sh[j].D;
      const size_t rn = rr[n], rp = rr[n + 1], Dn = D[n], Dp = D[n + 1], l = ell[n], lp = ell[n + 1];
      t1 = std::max({t1, rp * Dp * 2 * l, rn * Dn * 2 * lp});
      t2 = std::max({t2, 2 * Dn * rp * l, rn * 2 * Dp * lp});
      msz = std::max({msz, l * rn * Dn, rp * Dp * lp});
      u1 = std::max({u1, l * Dn * 2 * rp, 2 * rn * Dp * lp});
      csz = std::max(csz, l * 2 * rp * Dp);
      crsz = std::max(crsz, rn * Dn * 2 * lp);
      ssz = std::max(ssz, 2 * l * lp);
      qsz = std::max({qsz, (size_t)qr_work_size(1, (int)(2 * l), (int)lp), (size_t)qr_work_size(1, (int)(2 * lp), (int)l)});
    }
  r.R.assign(J, std::vector<double*>(N + 1, nullptr));
  r.Lk.assign(J, std::vector<double*>(N + 1, nullptr));
  r.Ma.resize(J);
  r.Mb.resize(J);
  r.Cb.resize(J);
  r.Mra.resize(J);
  r.Mrb.resize(J);
  r.Crb.resize(J);
  r.U1L.resize(J);
  r.U1R.resize(J);
  for (int j = 0; j < J; ++j) {
    for (int n = 1; n < N; ++n) {
      r.R[j][n] = plan.alloc((size_t)r.sh[j].r[n] * r.sh[j].D[n] * ell[n]);
      r.Lk[j][n] = plan.alloc((size_t)ell[n] * r.sh[j].r[n] * r.sh[j].D[n]);
    }
    // the sketch chains start from the term's coefficient instead of 1, so
    // every partial sketch carries c_j and the sums over terms need none
    double* cj = plan.upload(std::vector<double>{terms[j].coef});
    r.R[j][N] = cj;
    r.Lk[j][0] = cj;
    r.Ma[j] = plan.alloc(msz);
    r.Mb[j] = plan.alloc(msz);
    r.Cb[j] = plan.alloc(csz);
    r.Mra[j] = plan.alloc(msz);
    r.Mrb[j] = plan.alloc(msz);
    r.Crb[j] = plan.alloc(crsz);
    r.U1L[j] = plan.alloc(u1);
    r.U1R[j] = plan.alloc(u1);
    r.T1.push_back(plan.alloc(t1));
    r.T2.push_back(plan.alloc(t2));
    r.L1.push_back(plan.alloc(t1));
    r.L2.push_back(plan.alloc(t2));
  }
  for (int j = 0; j < J; ++j) {  // group terms of the same operator and bonds
    bool placed = false;
    for (auto& g : r.groups) {
      const int f = g[0];
      if ((int)g.size() < TC_MAXG && terms[f].mpo == terms[j].mpo && r.sh[f].r == r.sh[j].r &&
          r.sh[f].D == r.sh[j].D) {
        g.push_back(j);
        placed = true;
        break;
      }
    }
    if (!placed) r.groups.push_back({j});
  }
  r.SL = plan.alloc(ssz);
  r.SR = plan.alloc(ssz);
  r.qwL = plan.alloc(qsz);
  r.qwR = plan.alloc(qsz);
  r.qwsz = (int64_t)qsz;
  r.X.assign(N, nullptr);
  r.Vt.assign(N, nullptr);
  for (int n = 0; n < r.c; ++n) r.X[n] = plan.alloc((size_t)ell[n] * 2 * ell[n + 1]);
  for (int n = r.c + 1; n < N; ++n) r.Vt[n] = plan.alloc((size_t)2 * ell[n + 1] * ell[n]);
  r.Gc = plan.alloc((size_t)ell[r.c] * 2 * ell[r.c + 1]);
  // truncation buffers
  int lmax = 1, cmax = 1;
  for (int n = 0; n <= N; ++n) {
    lmax = std::max(lmax, ell[n]);
    cmax = std::max(cmax, tg.caps[n]);
  }
  r.lmax = lmax;
  r.ldg = lmax;
  r.ldp = cmax;
  r.Gam = plan.alloc((size_t)(N + 1) * r.ldg * r.ldg);
  r.P = plan.alloc((size_t)(N + 1) * r.ldg * r.ldp);
  r.lam = plan.alloc((size_t)(N + 1) * r.ldg);
  r.ework = plan.alloc((size_t)eig_work_size(std::max(1, N - 1), r.ldg));
  size_t tsz = 1;
  for (int n = 0; n < N; ++n) {
    tsz = std::max(tsz, (size_t)2 * ell[n] * ell[n + 1]);
    r.vsz = std::max(r.vsz, (size_t)tg.caps[n] * 2 * ell[n + 1]);
  }
  r.TgL = plan.alloc(tsz);
  r.TgR = plan.alloc(tsz);
  std::vector<int> dims, keep;
  for (int n = 1; n < N; ++n) {
    dims.push_back(ell[n]);
    keep.push_back(std::min(ell[n], tg.caps[n]));
  }
  r.d_dims = plan.upload(dims);
  r.d_keep = plan.upload(keep);
  r.dims_h = dims;
  r.keep_h = keep;
  tg.lam = r.lam;
  tg.ldl = r.ldg;
  tg.in_caps = ell;
}

// partial sketch chain q of a rounding: right sketches of term group q/2
// (q even), left sketches (q odd); one launch per contraction for the group
void ts_sketch(Plan& plan, TwoSided& r, int q, const ChainView& Zr, const ChainView& Zl, Prec prec) {
  const std::vector<int>& g = r.groups[q / 2];
  const int N = r.N;
  const auto& terms = *r.terms;
  auto record = [&](std::vector<std::vector<TcDesc>>& per) {
    for (size_t i = 0; i < per[0].size(); ++i) {
      std::vector<TcDesc> ds;
      for (auto& v : per) ds.push_back(v[i]);
      add_grouped(plan, ds, false, prec);
    }
  };
  if (q % 2 == 0) {
    for (int n = N - 1; n >= 1; --n) {
      std::vector<std::vector<TcDesc>> per;
      for (int j : g)
        per.push_back(rsketch_descs(terms[j], r.sh[j], Zr, n, r.R[j][n + 1], r.R[j][n], r.T1[j], r.T2[j]));
      record(per);
    }
  } else {
    for (int n = 0; n <= N - 2; ++n) {
      std::vector<std::vector<TcDesc>> per;
      for (int j : g)
        per.push_back(lsketch_descs(terms[j], r.sh[j], Zl, n, r.Lk[j][n], r.Lk[j][n + 1], r.L1[j], r.L2[j]));
      record(per);
    }
  }
}

// left-to-right sweep, sites 0..c-1
void ts_left_sweep(Plan& plan, TwoSided& r, const std::vector<int>& ell, double* one, Prec prec) {
  const int J = r.J;
  const auto& terms = *r.terms;
  const Prec dprec = data_prec(prec);
  std::vector<double*> Mcur(J, one), Mnext = r.Mb;
  for (int n = 0; n < r.c; ++n) {
    const int l = ell[n], lp = ell[n + 1];
    for (const auto& g : r.groups) {  // C_j = M_j x_j W
      std::vector<std::vector<TcDesc>> per;
      for (int j : g) per.push_back(lcore_descs(terms[j], r.sh[j], n, l, Mcur[j], r.U1L[j], r.Cb[j], 1.0, 0.0));
      for (size_t q = 0; q < per[0].size(); ++q) {
        std::vector<TcDesc> ds;
        for (auto& v : per) ds.push_back(v[q]);
        add_grouped(plan, ds, false, dprec);
      }
    }
    for (size_t gi = 0; gi < r.groups.size(); ++gi) {  // S = sum_j C_j R_j (c_j is in R_j)
      std::vector<TcDesc> ds;
      for (int j : r.groups[gi]) {
        const int rp = r.sh[j].r[n + 1], Dp = r.sh[j].D[n + 1];
        ds.push_back(gemm_desc(2 * l, lp, rp * Dp, r.Cb[j], (int64_t)rp * Dp, false, r.R[j][n + 1], lp, false,
                               r.SL, lp, 1.0, gi > 0 ? 1.0 : 0.0));
      }
      add_grouped(plan, ds, true, prec);
    }
    {
      double* Xn = r.X[n];
      double* SL = r.SL;
      double* qw = r.qwL;
      const int64_t qws = r.qwsz;
      const int m = 2 * l, nc = lp;
      add_qr_q(plan, m, nc, SL, nc, 1, Xn, qw, qws);
    }
    for (const auto& g : r.groups) {  // M'_j = X_n^T C_j
      std::vector<TcDesc> ds;
      for (int j : g) {
        const int rp = r.sh[j].r[n + 1], Dp = r.sh[j].D[n + 1];
        ds.push_back(gemm_desc(lp, rp * Dp, 2 * l, r.X[n], lp, true, r.Cb[j], (int64_t)rp * Dp, false, Mnext[j],
                               (int64_t)rp * Dp, 1.0, 0.0));
      }
      add_grouped(plan, ds, false, dprec);
    }
    for (int j = 0; j < J; ++j) {
      double* old = Mcur[j];
      Mcur[j] = Mnext[j];
      Mnext[j] = (old == one) ? r.Ma[j] : old;
    }
  }
  r.Mcur = Mcur;
}

// right-to-left sweep, sites N-1..c+1
void ts_right_sweep(Plan& plan, TwoSided& r, const std::vector<int>& ell, double* one, Prec prec) {
  const int J = r.J;
  const auto& terms = *r.terms;
  const Prec dprec = data_prec(prec);
  std::vector<double*> Mrcur(J, one), Mrnext = r.Mrb;
  for (int n = r.N - 1; n > r.c; --n) {
    const int l = ell[n], lp = ell[n + 1];
    for (const auto& g : r.groups) {  // Cr_j = x_j W Mr_j
      std::vector<std::vector<TcDesc>> per;
      for (int j : g) per.push_back(rcore_descs(terms[j], r.sh[j], n, lp, Mrcur[j], r.U1R[j], r.Crb[j]));
      for (size_t q = 0; q < per[0].size(); ++q) {
        std::vector<TcDesc> ds;
        for (auto& v : per) ds.push_back(v[q]);
        add_grouped(plan, ds, false, dprec);
      }
    }
    for (size_t gi = 0; gi < r.groups.size(); ++gi) {
      // SR[y,(t,z)] = sum_j Lk_j[y,(a,A)] Cr_j[(a,A),(t,z)] (c_j is in Lk_j)
      std::vector<TcDesc> ds;
      for (int j : r.groups[gi]) {
        const int rD = r.sh[j].r[n] * r.sh[j].D[n];
        ds.push_back(gemm_desc(l, 2 * lp, rD, r.Lk[j][n], rD, false, r.Crb[j], 2 * lp, false, r.SR, 2 * lp, 1.0,
                               gi > 0 ? 1.0 : 0.0));
      }
      add_grouped(plan, ds, true, prec);
    }
    {  // Q of SR^T (2 lp x l): the rows of V_n = Q^T are orthonormal
      double* Vn = r.Vt[n];
      double* SR = r.SR;
      double* qw = r.qwR;
      const int64_t qws = r.qwsz;
      const int m = 2 * lp, nc = l;
      add_qr_q(plan, m, nc, SR, 1, m, Vn, qw, qws);
    }
    for (const auto& g : r.groups) {  // Mr_j[(a,A),y] = sum_(t,z) Cr_j[(a,A),(t,z)] Vt[(t,z),y]
      std::vector<TcDesc> ds;
      for (int j : g) {
        const int rD = r.sh[j].r[n] * r.sh[j].D[n];
        ds.push_back(gemm_desc(rD, l, 2 * lp, r.Crb[j], 2 * lp, false, r.Vt[n], l, false, Mrnext[j], l, 1.0, 0.0));
      }
      add_grouped(plan, ds, false, dprec);
    }
    for (int j = 0; j < J; ++j) {
      double* old = Mrcur[j];
      Mrcur[j] = Mrnext[j];
      Mrnext[j] = (old == one) ? r.Mra[j] : old;
    }
  }
  r.Mrcur = Mrcur;
}

// centre core G = sum_j c_j [X_(<c)^T Y_j V_(>c)^T]_c
void ts_centre(Plan& plan, TwoSided& r, const std::vector<int>& ell, Prec prec) {
  const int c = r.c, l = ell[c], lp = ell[c + 1];
  const auto& terms = *r.terms;
  const Prec dprec = data_prec(prec);
  for (const auto& g : r.groups) {
    std::vector<std::vector<TcDesc>> per;
    for (int j : g) per.push_back(lcore_descs(terms[j], r.sh[j], c, l, r.Mcur[j], r.U1L[j], r.Cb[j], 1.0, 0.0));
    for (size_t q = 0; q < per[0].size(); ++q) {
      std::vector<TcDesc> ds;
      for (auto& v : per) ds.push_back(v[q]);
      add_grouped(plan, ds, false, dprec);
    }
  }
  for (int j = 0; j < r.J; ++j) {
    const int rD = r.sh[j].r[c + 1] * r.sh[j].D[c + 1];
    add_gemm(plan, 2 * l, lp, rD, r.Cb[j], rD, false, r.Mrcur[j], lp, false, r.Gc, lp, terms[j].coef,
             j > 0 ? 1.0 : 0.0, dprec);
  }
}

// Truncation of the mixed canonical chain (left-orthogonal X_n for n < c,
// centre G, right-orthogonal V_n for n > c, kept as Vt[(t,z),y]): at a bond
// n <= c the right Gram matrix decides (Gamma_c = G G^T, then the chain
// through X_(c-1)..X_1), at n > c the left one (Lambda_(c+1) = G^T G, then
// the chain through V_(c+1)..)
void ts_gram_right(Plan& plan, TwoSided& r, const std::vector<int>& ell) {
  const int c = r.c;
  if (c < 1) return;
  const int a = ell[c], b = ell[c + 1];
  add_gemm(plan, a, a, 2 * b, r.Gc, 2 * b, false, r.Gc, 2 * b, true, r.G(c), r.ldg, 1.0, 0.0, Prec::F64);
  for (int n = c - 1; n >= 1; --n) {
    const int an = ell[n], bn = ell[n + 1];
    add_gemm(plan, 2 * an, bn, bn, r.X[n], bn, false, r.G(n + 1), r.ldg, false, r.TgL, bn, 1.0, 0.0, Prec::F64);
    add_gemm(plan, an, an, 2 * bn, r.TgL, 2 * bn, false, r.X[n], 2 * bn, true, r.G(n), r.ldg, 1.0, 0.0, Prec::F64);
  }
}

void ts_gram_left(Plan& plan, TwoSided& r, const std::vector<int>& ell) {
  const int c = r.c, N = r.N;
  if (c + 1 > N - 1) return;
  const int a = ell[c], b = ell[c + 1];
  add_gemm(plan, b, b, 2 * a, r.Gc, b, true, r.Gc, b, false, r.G(c + 1), r.ldg, 1.0, 0.0, Prec::F64);
  for (int n = c + 1; n <= N - 2; ++n) {
    const int l = ell[n], lp = ell[n + 1];
    // H[(t,z),y'] = sum_y Vt[(t,z),y] Lambda_n[y,y']
    add_gemm(plan, 2 * lp, l, l, r.Vt[n], l, false, r.G(n), r.ldg, false, r.TgR, l, 1.0, 0.0, Prec::F64);
    // Lambda_(n+1)[z,z'] = sum_(t,y') H[(t,z),y'] Vt[(t,z'),y']
    TcDesc d;
    d.M = lp;
    d.N = lp;
    d.K = 2 * l;
    d.A = r.TgR;
    d.am = M1(l);
    d.ak = M2(l, (int64_t)lp * l, 1);
    d.B = r.Vt[n];
    d.bk = M2(l, (int64_t)lp * l, 1);
    d.bn = M1(l);
    d.C = r.G(n + 1);
    d.cm = M1(r.ldg);
    d.cn = M1(1);
    d.ab = d.bb = d.cb = M1(0);
    add_tc(plan, d, Prec::F64);
  }
}

// one batched eigen-decomposition over all bonds (after the Gram chains)
void ts_eig(Plan& plan, TwoSided& r, const std::vector<int>& ell, Prec prec) {
  const int N = r.N, ldg = r.ldg, ldp = r.ldp, lmax = r.lmax;
  {
    double* P = r.P;
    double* lam = r.lam;
    const size_t psz = (size_t)(N + 1) * ldg * ldp;
    plan.add([P, psz, lam, N, ldg](hipStream_t s) {
      fill(P, (int64_t)psz, 0.0, s);
      fill(lam, (int64_t)(N + 1) * ldg, 0.0, s);
    });
  }
  if (N < 2) return;
  // eigenvectors resolved down to the noise the contractions left in the
  // Gram matrices (see the one-sided truncation)
  const double u = machine_eps(data_prec(prec));
  const double unoise = std::max(machine_eps(Prec::F64), u * u);
  const double* g1 = r.G(1);
  double* p1 = r.Pn(1);
  double* l1 = r.lam + ldg;
  double* ework = r.ework;
  const int* d_dims = r.d_dims;
  const int* d_keep = r.d_keep;
  const int cnt = N - 1;
  const bool pre = eig_uses_precondition(lmax);
  if (pre) {
    // QR factors of every Gram matrix: the Jacobi sweeps start from R^T
    OpInfo qi;
    qi.kind = OP_QR;
    qi.what = qr_kernel_name(lmax, lmax) + "|eig precondition count" + std::to_string(cnt) + " n" +
              std::to_string(lmax);
    for (int n = 1; n < N; ++n) {
      const OpInfo one = qr_info(ell[n], ell[n]);
      qi.flops += one.flops;
      qi.bytes += one.bytes + 8.0 * (double)ell[n] * ell[n];  // G in, Q and R out
    }
    plan.add([=](hipStream_t s) {
      eig_precondition_launch(cnt, d_dims, g1, (int64_t)ldg * ldg, ldg, ework, lmax, s);
    }, qi);
  }
  OpInfo oi;
  oi.kind = OP_EIG;
  oi.what = eig_kernel_name(lmax) + "|count" + std::to_string(cnt) + " nmax" + std::to_string(lmax);
  for (int n = 1; n < N; ++n) {
    oi.bytes += 8.0 * ((double)ell[n] * ell[n] + (double)ell[n] * r.tg->caps[n]);
    oi.flops += 9.0 * (double)ell[n] * ell[n] * ell[n];
  }
  plan.add([=](hipStream_t s) {
    eig_launch(cnt, d_dims, d_keep, g1, (int64_t)ldg * ldg, ldg, p1, (int64_t)ldg * ldp, ldp, l1, ldg, ework,
               lmax, unoise, s, pre);
  }, oi);
  if (r.tg->rel_tol > 0.0) {
    const double tol2 = r.tg->rel_tol * r.tg->rel_tol;
    const std::vector<int> dims = r.dims_h, keep = r.keep_h;
    plan.add([=](hipStream_t s) { rank_cut(p1, (int64_t)ldg * ldp, ldp, l1, ldg, d_dims, d_keep, dims, keep, tol2, s); });
  }
}

// new core n: P_n^T A_n P_(n+1) (V1: scratch of r.vsz doubles)
void ts_core(Plan& plan, TwoSided& r, int n, const std::vector<int>& ell, double* V1) {
  const int N = r.N, c = r.c, ldp = r.ldp;
  RoundTarget& tg = *r.tg;
  const int l = ell[n], lp = ell[n + 1], cl = tg.caps[n], cr = tg.caps[n + 1];
  if (n <= c) {
    const double* A = (n == c) ? r.Gc : r.X[n];  // [l][2][lp]
    if (n == 0 && N == 1) {
      double* dst = tg.core[0];
      plan.add([=](hipStream_t s) { rt::copy_async(dst, A, 2 * sizeof(double), s); });
    } else if (n == 0) {
      add_gemm(plan, 2, cr, lp, A, lp, false, r.Pn(1), ldp, false, tg.core[0], cr, 1.0, 0.0, Prec::F64);
    } else if (n == N - 1) {
      add_gemm(plan, cl, 2, l, r.Pn(n), ldp, true, A, 2, false, tg.core[n], 2, 1.0, 0.0, Prec::F64);
    } else {
      add_gemm(plan, cl, 2 * lp, l, r.Pn(n), ldp, true, A, 2 * lp, false, V1, 2 * lp, 1.0, 0.0, Prec::F64);
      add_gemm(plan, 2 * cl, cr, lp, V1, lp, false, r.Pn(n + 1), ldp, false, tg.core[n], cr, 1.0, 0.0,
               Prec::F64);
    }
  } else {
    // V1[k,(t,z)] = sum_y P_n[y,k] V[y,t,z] = sum_y P_n[y,k] Vt[(t,z),y]
    const bool lastsite = (n == N - 1);
    TcDesc d;
    d.M = cl;
    d.N = 2 * lp;
    d.K = l;
    d.A = r.Pn(n);
    d.am = M1(1);
    d.ak = M1(ldp);
    d.B = r.Vt[n];
    d.bk = M1(1);
    d.bn = M1(l);
    d.C = lastsite ? tg.core[n] : V1;
    d.cm = M1(2 * lp);
    d.cn = M1(1);
    d.ab = d.bb = d.cb = M1(0);
    add_tc(plan, d, Prec::F64);
    if (!lastsite)
      add_gemm(plan, 2 * cl, cr, lp, V1, lp, false, r.Pn(n + 1), ldp, false, tg.core[n], cr, 1.0, 0.0,
               Prec::F64);
  }
}

}  // namespace

void plan_round_two_sided_multi(Plan& plan, const std::vector<RoundJob>& jobs, const ChainView& Zr,
                                const ChainView& Zl, Prec prec, int lanes) {
  const int N = Zr.N;
  const int K = (int)jobs.size();
  QTT_REQUIRE(K >= 1, "no rounding to record");
  QTT_REQUIRE(Zl.N == N && Zl.caps == Zr.caps, "the two sketches must have the same ranks");
  if (N < 2) {
    for (const RoundJob& jb : jobs) plan_round_sketch(plan, *jb.terms, Zr, *jb.tg, prec, lanes);
    return;
  }
  const std::vector<int>& ell = Zr.caps;
  for (int n = 0; n < N; ++n)
    QTT_REQUIRE(ell[n + 1] <= 2 * ell[n] && ell[n] <= 2 * ell[n + 1],
                "sketch ranks must satisfy ell_(n+1) <= 2 ell_n and ell_n <= 2 ell_(n+1)");
  const int L = lane_budget(plan, lanes);
  double* one = plan.upload(std::vector<double>{1.0});
  std::vector<TwoSided> rs(K);
  for (int k = 0; k < K; ++k) ts_setup(plan, rs[k], *jobs[k].terms, *jobs[k].tg, ell);

  // ---- partial sketches: right (sites N-1..1) and left (sites 0..N-2) of
  // every term group of every rounding, chain i on lane i % Ls
  {
    int Q = 0;
    for (const TwoSided& r : rs) Q += 2 * (int)r.groups.size();
    const int Ls = std::min(L, Q);
    plan.fork(Ls);
    int i = 0;
    for (TwoSided& r : rs)
      for (int q = 0; q < 2 * (int)r.groups.size(); ++q, ++i) {
        if (Ls > 1) plan.on(i % Ls);
        ts_sketch(plan, r, q, Zr, Zl, prec);
      }
    plan.join(Ls);
  }
  // ---- the sweeps (two per rounding), sweep i on lane i % Lw
  {
    const int Lw = std::min(L, 2 * K);
    plan.fork(Lw);
    for (int k = 0; k < K; ++k) {
      if (Lw > 1) plan.on((2 * k) % Lw);
      ts_left_sweep(plan, rs[k], ell, one, prec);
      if (Lw > 1) plan.on((2 * k + 1) % Lw);
      ts_right_sweep(plan, rs[k], ell, one, prec);
    }
    plan.join(Lw);
  }
  // ---- centre cores
  {
    const int Lk = std::min(L, K);
    plan.fork(Lk);
    for (int k = 0; k < K; ++k) {
      if (Lk > 1) plan.on(k % Lk);
      ts_centre(plan, rs[k], ell, prec);
    }
    plan.join(Lk);
  }
  // ---- Gram chains (two per rounding)
  {
    const int Lg = std::min(L, 2 * K);
    plan.fork(Lg);
    for (int k = 0; k < K; ++k) {
      if (Lg > 1) plan.on((2 * k) % Lg);
      ts_gram_right(plan, rs[k], ell);
      if (Lg > 1) plan.on((2 * k + 1) % Lg);
      ts_gram_left(plan, rs[k], ell);
    }
    plan.join(Lg);
  }
  // ---- eigen-decompositions (one batched launch per rounding)
  {
    const int Le = std::min(L, K);
    plan.fork(Le);
    for (int k = 0; k < K; ++k) {
      if (Le > 1) plan.on(k % Le);
      ts_eig(plan, rs[k], ell, prec);
    }
    plan.join(Le);
  }
  // ---- new cores, independent: item i on lane i % Lc with its own V1
  {
    const int Lc = std::min(L, std::max(1, std::min(4, K * N)));
    size_t vsz = 1;
    for (const TwoSided& r : rs) vsz = std::max(vsz, r.vsz);
    std::vector<double*> V1s(Lc);
    for (int l = 0; l < Lc; ++l) V1s[l] = plan.alloc(vsz);
    plan.fork(Lc);
    int i = 0;
    for (int k = 0; k < K; ++k)
      for (int n = 0; n < N; ++n, ++i) {
        if (Lc > 1) plan.on(i % Lc);
        ts_core(plan, rs[k], n, ell, V1s[i % Lc]);
      }
    plan.join(Lc);
  }
}

void plan_round_sketch_two_sided(Plan& plan, const std::vector<SketchTerm>& terms, const ChainView& Zr,
                                 const ChainView& Zl, RoundTarget& tg, Prec prec, int lanes) {
  plan_round_two_sided_multi(plan, {RoundJob{&terms, &tg}}, Zr, Zl, prec, lanes);
}

}  // namespace qtt
