// Launch planners of the MPS arithmetic: randomized range finding with right
// partial sketches, Householder QR sweeps, simultaneous SVD truncation of all
// bonds from their Gram matrices, block-diagonal sums, environment chains.
//
// Every planner appends enqueue operations to a Plan and allocates the
// workspaces it needs at planning time, so that a plan can be replayed many
// times (eagerly or captured as a HIP graph) without allocations.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <string>

#include "library.h"

namespace qtt {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
std::vector<int> chain_caps(int N, long cap) {
  std::vector<int> c(N + 1);
  for (int n = 0; n <= N; ++n) {
    long a = (n < 40) ? (1L << n) : (1L << 40);
    long b = (N - n < 40) ? (1L << (N - n)) : (1L << 40);
    c[n] = (int)std::min(cap, std::min(a, b));
  }
  return c;
}

std::unique_ptr<tt_tt> make_tt(tt_ctx* ctx, int kind, int N, const std::vector<int>& caps) {
  QTT_REQUIRE(N >= 1 && (int)caps.size() == N + 1, "bad chain length");
  QTT_REQUIRE(caps[0] == 1 && caps[N] == 1, "boundary bonds must be 1");
  auto t = std::make_unique<tt_tt>();
  t->ctx = ctx;
  t->kind = kind;
  t->N = N;
  t->p = (kind == TT_MPO) ? 4 : 2;
  t->caps = caps;
  t->off.assign(N + 1, 0);
  for (int n = 0; n < N; ++n) {
    QTT_REQUIRE(caps[n] >= 1 && caps[n + 1] >= 1, "bond capacities must be >= 1");
    t->off[n + 1] = t->off[n] + (int64_t)caps[n] * t->p * caps[n + 1];
  }
  t->buf.alloc((size_t)t->off[N] * sizeof(double));
  return t;
}

ChainView view(const tt_tt* t) {
  ChainView v;
  v.N = t->N;
  v.p = t->p;
  v.caps = t->caps;
  for (int n = 0; n < t->N; ++n) v.core.push_back(t->core(n));
  return v;
}

ChainView view_sites(const tt_tt* t, int first, int count) {
  ChainView v;
  v.N = count;
  v.p = t->p;
  for (int n = 0; n < count; ++n) v.core.push_back(t->core(first + n));
  for (int n = 0; n <= count; ++n) v.caps.push_back(t->caps[first + n]);
  return v;
}

static Mode2 M1(int64_t s) { return mode1(s); }
static Mode2 M2(int n2, int64_t s1, int64_t s2) { return mode2(n2, s1, s2); }

void add_tc(Plan& plan, TcDesc d, Prec p) {
  // measured tile and K split (no measurement into a fixed scratch buffer:
  // it would allocate; a cached choice or the rule then)
  tc_configure(d, p, plan.arena == nullptr);
  if (tc_uses_part(d)) d.part = plan.alloc_transient((size_t)tc_part_size(d));
  if (d.ng > 1) {
    std::vector<const double*> table;
    for (int g = 0; g < d.ng; ++g) table.push_back(d.gA[g]);
    for (int g = 0; g < d.ng; ++g) table.push_back(d.gB[g]);
    for (int g = 0; g < d.ng; ++g) table.push_back(d.gsum ? d.C : d.gC[g]);
    d.gdev = plan.upload(table);
  }
  tc_validate(d);
  OpInfo oi;
  oi.kind = OP_CONTRACT;
  const double ng = d.ng, nc = d.gsum ? 1.0 : ng;
  oi.flops = 2.0 * d.M * (double)d.N * d.K * d.batch * ng;
  double na = (mode_max(d.ab, d.batch) == 0) ? 1.0 : d.batch;
  double nb = (mode_max(d.bb, d.batch) == 0) ? 1.0 : d.batch;
  oi.bytes = 8.0 * (ng * na * d.M * (double)d.K + ng * nb * d.K * (double)d.N +
                    nc * (d.beta != 0.0 ? 2.0 : 1.0) * d.batch * d.M * (double)d.N);
  char w[112];
  if (d.ng > 1)
    snprintf(w, sizeof w, "|b%d m%d n%d k%d s%d g%d%s", d.batch, d.M, d.N, d.K, d.ksplit, d.ng,
             d.gsum ? "+" : "");
  else
    snprintf(w, sizeof w, "|b%d m%d n%d k%d s%d", d.batch, d.M, d.N, d.K, d.ksplit);
  oi.what = tc_kernel_name(d, p) + w;
  plan.add([d, p](hipStream_t s) { tc_launch(d, p, s); }, oi);
}

OpInfo qr_info(int m, int n) {
  OpInfo oi;
  oi.kind = OP_QR;
  oi.flops = 2.0 * (2.0 * m * (double)n * n - 2.0 * n * (double)n * n / 3.0);
  oi.bytes = 8.0 * 2.0 * m * (double)n;
  oi.what = qr_path_name(m, n) + "|m" + std::to_string(m) + " n" + std::to_string(n);
  return oi;
}

void add_qr_q(Plan& plan, int m, int n, const double* A, int64_t rs, int64_t cs, double* Q, double* work,
              int64_t work_size) {
  if (!qr_split(m, n, work_size)) {
    plan.add([=](hipStream_t s) { qr_launch(1, m, n, A, 0, rs, cs, Q, 0, nullptr, 0, work, s, nullptr, 0, work_size); },
             qr_info(m, n));
    return;
  }
  const std::string shape = "|m" + std::to_string(m) + " n" + std::to_string(n);
  OpInfo f;  // the factorisation: read A, write the reflectors
  f.kind = OP_QR;
  f.flops = 2.0 * m * (double)n * n - 2.0 * n * (double)n * n / 3.0;
  f.bytes = 8.0 * (2.0 * m * (double)n + n);
  f.what = qr_kernel_name(m, n) + shape;
  plan.add([=](hipStream_t s) { qr_reflectors_launch(m, n, A, rs, cs, work, s); }, f);
  OpInfo q = f;  // thin Q from the reflectors: as many flops, read the reflectors, write Q
  q.what = qr_q_kernel_name(m, n) + shape;
  plan.add([=](hipStream_t s) { qr_form_q_launch(m, n, work, Q, n, s); }, q);
}

Plan::~Plan() {
  for (auto e : events)
    if (e) (void)hipEventDestroy(e);
  for (auto st : streams)
    if (st) (void)hipStreamDestroy(st);
}

hipEvent_t Plan::new_event() {
  hipEvent_t e = nullptr;
  if (!rt::dry()) QTT_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  events.push_back(e);
  return e;
}

void Plan::ensure_lanes(int n) {
  while ((int)streams.size() < n - 1) {
    hipStream_t st = nullptr;
    if (!rt::dry()) QTT_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    streams.push_back(st);
  }
}

void Plan::fork(int n) {
  if (n <= 1) return;  // single lane: nothing to order
  QTT_REQUIRE(cur == 0, "fork from lane 0 only");
  QTT_REQUIRE(arena == nullptr, "a plan on a fixed scratch buffer runs on one lane");
  ensure_lanes(n);
  OpInfo rec, wait;
  rec.kind = wait.kind = OP_SYNC;
  rec.what = "lane fork record";
  wait.what = "lane fork wait";
  hipEvent_t e = new_event();
  add([e](hipStream_t s) {
    if (!rt::dry()) QTT_HIP(hipEventRecord(e, s));
  }, rec);
  for (int l = 1; l < n; ++l) {
    cur = l;
    add([e](hipStream_t s) {
      if (!rt::dry()) QTT_HIP(hipStreamWaitEvent(s, e, 0));
    }, wait);
  }
  cur = 0;
}

void Plan::join(int n) {
  if (n <= 1) return;
  QTT_REQUIRE(cur < n, "join of lanes that were not forked");
  OpInfo rec, wait;
  rec.kind = wait.kind = OP_SYNC;
  rec.what = "lane join record";
  wait.what = "lane join wait";
  for (int l = 1; l < n; ++l) {
    hipEvent_t e = new_event();
    cur = l;
    add([e](hipStream_t s) {
      if (!rt::dry()) QTT_HIP(hipEventRecord(e, s));
    }, rec);
    cur = 0;
    add([e](hipStream_t s) {
      if (!rt::dry()) QTT_HIP(hipStreamWaitEvent(s, e, 0));
    }, wait);
  }
  cur = 0;
}

void Plan::run_profiled(hipStream_t s, int kind, double& ms, int64_t& count, double& flops,
                        double& bytes) const {
  std::vector<size_t> idx;
  for (size_t i = 0; i < ops.size(); ++i)
    if ((kind == OP_ALL && info[i].kind != OP_SYNC) || info[i].kind == kind) idx.push_back(i);
  std::vector<hipEvent_t> ev(2 * idx.size(), nullptr);
  if (!rt::dry())
    for (auto& e : ev) QTT_HIP(hipEventCreate(&e));
  size_t j = 0;
  for (size_t i = 0; i < ops.size(); ++i) {
    bool tim = (j < idx.size() && idx[j] == i);
    hipStream_t si = stream_of(lane[i], s);
    if (tim && !rt::dry()) QTT_HIP(hipEventRecord(ev[2 * j], si));
    ops[i](si);
    if (tim) {
      if (!rt::dry()) QTT_HIP(hipEventRecord(ev[2 * j + 1], si));
      flops += info[i].flops;
      bytes += info[i].bytes;
      ++count;
      ++j;
    }
  }
  rt::sync(s);
  // log: one line per operation in plan order (index, class, ms, flops,
  // bytes, description, lane); lane fork / join events appear with class
  // OP_SYNC so that the lanes' ordering can be reconstructed
  const char* logp = std::getenv("QTTPDF_PROFILE_LOG");
  FILE* log = logp ? std::fopen(logp, "a") : nullptr;
  size_t k = 0;
  for (size_t i = 0; i < ops.size(); ++i) {
    const OpInfo& oi = info[i];
    const bool tim = (k < idx.size() && idx[k] == i);
    float t = 0.f;
    if (tim) {
      if (!rt::dry()) QTT_HIP(hipEventElapsedTime(&t, ev[2 * k], ev[2 * k + 1]));
      ms += t;
      ++k;
    }
    if (log && (tim || oi.kind == OP_SYNC))
      std::fprintf(log, "%zu\t%d\t%.6f\t%.6g\t%.6g\t%s\t%d\n", i, oi.kind, (double)t, oi.flops,
                   oi.bytes, oi.what.empty() ? "-" : oi.what.c_str(), lane[i]);
  }
  if (log) std::fclose(log);
  if (!rt::dry())
    for (auto& e : ev) (void)hipEventDestroy(e);
}

void add_gemm(Plan& plan, int M, int N, int K, const double* A, int64_t lda, bool ta,
              const double* B, int64_t ldb, bool tb, double* C, int64_t ldc, double alpha,
              double beta, Prec p) {
  add_tc(plan, gemm_desc(M, N, K, A, lda, ta, B, ldb, tb, C, ldc, alpha, beta), p);
}

// ---------------------------------------------------------------------------
// simultaneous truncation of a left-orthogonal chain X (caps ell) to the
// target caps: right Gram chain, batched eigen-decompositions, P^T X P
// ---------------------------------------------------------------------------
static void plan_trunc_gram(Plan& plan, const std::vector<double*>& X, const std::vector<int>& ell,
                            RoundTarget& tg, Prec prec) {
  // The Gram matrices are FP64, but X carries the relative noise u of the
  // contractions that produced it.  An eigen-residual r turns the direction
  // of singular value sigma_i by ~ r / sigma_i^2 and moves the tensor by
  // ~ r / sigma_i; keeping that below the u * sigma_1 the contractions already
  // cause, for every sigma_i >= u * sigma_1, needs r <= u^2 lambda_1.
  const double u = machine_eps(prec);
  const double unoise = std::max(machine_eps(Prec::F64), u * u);
  const int N = (int)X.size();
  QTT_REQUIRE((int)tg.caps.size() == N + 1 && (int)tg.core.size() == N, "truncation target shape");
  int lmax = 1, cmax = 1;
  for (int n = 0; n <= N; ++n) {
    lmax = std::max(lmax, ell[n]);
    cmax = std::max(cmax, tg.caps[n]);
  }
  const int ldg = lmax, ldp = cmax;
  double* Gam = plan.alloc((size_t)(N + 1) * ldg * ldg);
  double* P = plan.alloc((size_t)(N + 1) * ldg * ldp);
  double* lam = plan.alloc((size_t)(N + 1) * ldg);
  double* ework = plan.alloc((size_t)eig_work_size(std::max(1, N - 1), ldg));
  size_t tsz = 1, vsz = 1;
  for (int n = 0; n < N; ++n) {
    tsz = std::max(tsz, (size_t)2 * ell[n] * ell[n + 1]);
    vsz = std::max(vsz, (size_t)tg.caps[n] * 2 * ell[n + 1]);
  }
  double* Tg = plan.alloc(tsz);
  double* V1 = plan.alloc(vsz);
  std::vector<int> dims, keep;
  for (int n = 1; n < N; ++n) {
    dims.push_back(ell[n]);
    keep.push_back(std::min(ell[n], tg.caps[n]));
  }
  int* d_dims = plan.upload(dims);
  int* d_keep = plan.upload(keep);
  tg.lam = lam;
  tg.ldl = ldg;
  tg.in_caps = ell;
  const size_t psz = (size_t)(N + 1) * ldg * ldp;
  plan.add([P, psz, lam, N, ldg](hipStream_t s) {
    fill(P, (int64_t)psz, 0.0, s);
    fill(lam, (int64_t)(N + 1) * ldg, 0.0, s);
  });
  auto G = [&](int n) { return Gam + (size_t)n * ldg * ldg; };
  auto Pn = [&](int n) { return P + (size_t)n * ldg * ldp; };
  if (N >= 2) {
    int l = ell[N - 1];
    add_gemm(plan, l, l, 2, X[N - 1], 2, false, X[N - 1], 2, true, G(N - 1), ldg, 1.0, 0.0, Prec::F64);
    for (int n = N - 2; n >= 1; --n) {
      int a = ell[n], b = ell[n + 1];
      add_gemm(plan, 2 * a, b, b, X[n], b, false, G(n + 1), ldg, false, Tg, b, 1.0, 0.0, Prec::F64);
      add_gemm(plan, a, a, 2 * b, Tg, 2 * b, false, X[n], 2 * b, true, G(n), ldg, 1.0, 0.0, Prec::F64);
    }
    double* g1 = G(1);
    double* p1 = Pn(1);
    double* l1 = lam + ldg;
    int cnt = N - 1;
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
    // algorithmic flops: 9 n^3 per matrix, the count of a dense symmetric
    // eigen-decomposition with vectors (tridiagonal reduction + implicit QL)
    for (int n = 1; n < N; ++n) {
      oi.bytes += 8.0 * ((double)ell[n] * ell[n] + (double)ell[n] * tg.caps[n]);
      oi.flops += 9.0 * (double)ell[n] * ell[n] * ell[n];
    }
    plan.add([=](hipStream_t s) {
      eig_launch(cnt, d_dims, d_keep, g1, (int64_t)ldg * ldg, ldg, p1, (int64_t)ldg * ldp, ldp, l1,
                 ldg, ework, lmax, unoise, s, pre);
    }, oi);
    if (tg.rel_tol > 0.0) {
      const double tol2 = tg.rel_tol * tg.rel_tol;
      plan.add([=](hipStream_t s) {
        rank_cut(p1, (int64_t)ldg * ldp, ldp, l1, ldg, d_dims, d_keep, dims, keep, tol2, s);
      });
    }
  }
  // new cores P_n^T X_n P_{n+1}
  for (int n = 0; n < N; ++n) {
    int l = ell[n], lr = ell[n + 1], c = tg.caps[n], cr = tg.caps[n + 1];
    if (N == 1) {
      double* dst = tg.core[0];
      const double* src = X[0];
      plan.add([=](hipStream_t s) {
        rt::copy_async(dst, src, 2 * sizeof(double), s);
      });
    } else if (n == 0) {
      add_gemm(plan, 2, cr, lr, X[0], lr, false, Pn(1), ldp, false, tg.core[0], cr, 1.0, 0.0, Prec::F64);
    } else if (n == N - 1) {
      add_gemm(plan, c, 2, l, Pn(n), ldp, true, X[n], 2, false, tg.core[n], 2, 1.0, 0.0, Prec::F64);
    } else {
      add_gemm(plan, c, 2 * lr, l, Pn(n), ldp, true, X[n], 2 * lr, false, V1, 2 * lr, 1.0, 0.0, Prec::F64);
      add_gemm(plan, 2 * c, cr, lr, V1, lr, false, Pn(n + 1), ldp, false, tg.core[n], cr, 1.0, 0.0,
               Prec::F64);
    }
  }
}

// ---------------------------------------------------------------------------
// randomized range finding of Y = sum_j c_j W_j x_j (right sketches with the
// Gaussian TT Z, left-to-right QR sweep of the sketched unfoldings), then
// simultaneous truncation.
// ---------------------------------------------------------------------------
void plan_round_sketch(Plan& plan, const std::vector<SketchTerm>& terms, const ChainView& Z,
                       RoundTarget& tg, Prec prec, int lanes) {
  const int N = Z.N;
  const int J = (int)terms.size();
  // the terms' independent contraction chains are spread over L lanes
  const int L = lane_budget(plan, std::min(lanes, J));
  QTT_REQUIRE(J >= 1, "rounding needs at least one term");
  const std::vector<int>& ell = Z.caps;
  for (int n = 0; n < N; ++n)
    QTT_REQUIRE(ell[n + 1] <= 2 * ell[n], "sketch ranks must satisfy ell_{n+1} <= 2 ell_n");
  struct TermShape {
    std::vector<int> r, D;
  };
  std::vector<TermShape> sh(J);
  for (int j = 0; j < J; ++j) {
    QTT_REQUIRE(terms[j].x.N == N, "term length differs from the sketch");
    sh[j].r = terms[j].x.caps;
    if (terms[j].mpo) {
      QTT_REQUIRE(terms[j].mpo->N == N, "operator length differs from the sketch");
      sh[j].D = terms[j].mpo->caps;
    } else {
      sh[j].D.assign(N + 1, 1);
    }
  }
  // workspaces
  size_t t1 = 1, t2 = 1, msz = 1, u1 = 1, csz = 1, ssz = 1, qsz = 1;
  for (int j = 0; j < J; ++j)
    for (int n = 0; n < N; ++n) {
      const auto& r = sh[j].r;
      const auto& D = sh[j].D;
      t1 = std::max(t1, (size_t)r[n + 1] * D[n + 1] * 2 * ell[n]);
      t2 = std::max(t2, (size_t)2 * D[n] * r[n + 1] * ell[n]);
      msz = std::max(msz, (size_t)ell[n] * r[n] * D[n]);
      u1 = std::max(u1, (size_t)ell[n] * D[n] * 2 * r[n + 1]);
      csz = std::max(csz, (size_t)ell[n] * 2 * r[n + 1] * D[n + 1]);
      ssz = std::max(ssz, (size_t)2 * ell[n] * ell[n + 1]);
      qsz = std::max(qsz, (size_t)qr_work_size(1, 2 * ell[n], ell[n + 1]));
    }
  std::vector<double*> T1s(L), T2s(L), U1s(L);
  for (int l = 0; l < L; ++l) {
    T1s[l] = plan.alloc(t1);
    T2s[l] = plan.alloc(t2);
    U1s[l] = plan.alloc(u1);
  }
  double* S = plan.alloc(ssz);
  double* qrw = plan.alloc(qsz);
  const int64_t qrws = (int64_t)qsz;
  double* one = plan.upload(std::vector<double>{1.0});
  std::vector<std::vector<double*>> R(J, std::vector<double*>(N + 1, nullptr));
  std::vector<double*> Ma(J), Mb(J), Cb(J);
  for (int j = 0; j < J; ++j) {
    for (int n = 1; n < N; ++n) R[j][n] = plan.alloc((size_t)sh[j].r[n] * sh[j].D[n] * ell[n]);
    R[j][N] = one;
    Ma[j] = plan.alloc(msz);
    Mb[j] = plan.alloc(msz);
    Cb[j] = plan.alloc(csz);
  }
  std::vector<double*> X(N);
  for (int n = 0; n < N; ++n) X[n] = plan.alloc((size_t)ell[n] * 2 * ell[n + 1]);

  // ---- right partial sketches R_j[n] = Right_n(Y_j) Right_n(Z)^T, term j on lane j % L
  plan.fork(L);
  for (int j = 0; j < J; ++j) {
    const auto& r = sh[j].r;
    const auto& D = sh[j].D;
    const ChainView* W = terms[j].mpo;
    if (L > 1) plan.on(j % L);
    double* T1 = T1s[j % L];
    double* T2 = T2s[j % L];
    for (int n = N - 1; n >= 1; --n) {
      const int l = ell[n], lp = ell[n + 1], rn = r[n], rp = r[n + 1], Dn = D[n], Dp = D[n + 1];
      {  // T1[(b,beta),(t,z)] = sum_z' R[(b,beta),z'] Z_n[z,t,z']
        TcDesc d;
        d.M = rp * Dp;
        d.N = 2 * l;
        d.K = lp;
        d.A = R[j][n + 1];
        d.am = M1(lp);
        d.ak = M1(1);
        d.B = Z.core[n];
        d.bk = M1(1);
        d.bn = M2(l, lp, 2 * lp);
        d.C = T1;
        d.cm = M1(2 * l);
        d.cn = M1(1);
        d.ab = d.bb = d.cb = M1(0);
        add_tc(plan, d, prec);
      }
      if (W) {
        {  // T2[(alpha,s), b, z] = sum_(beta,t) W[alpha,t,s,beta] T1[(b,beta),(t,z)], batch b
          TcDesc d;
          d.batch = rp;
          d.M = 2 * Dn;
          d.K = 2 * Dp;
          d.N = l;
          d.A = W->core[n];
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
          add_tc(plan, d, prec);
        }
        {  // R[(a,alpha),z] = sum_(s,b) x[a,s,b] T2[alpha,s,b,z], batch alpha
          TcDesc d;
          d.batch = Dn;
          d.M = rn;
          d.K = 2 * rp;
          d.N = l;
          d.A = terms[j].x.core[n];
          d.am = M1(2 * rp);
          d.ak = M1(1);
          d.ab = M1(0);
          d.B = T2;
          d.bk = M1(l);
          d.bn = M1(1);
          d.bb = M1((int64_t)2 * rp * l);
          d.C = R[j][n];
          d.cm = M1((int64_t)Dn * l);
          d.cn = M1(1);
          d.cb = M1(l);
          add_tc(plan, d, prec);
        }
      } else {
        // R[a,z] = sum_(s,b) x[a,s,b] T1[b,(s,z)]
        TcDesc d;
        d.M = rn;
        d.K = 2 * rp;
        d.N = l;
        d.A = terms[j].x.core[n];
        d.am = M1(2 * rp);
        d.ak = M1(1);
        d.B = T1;
        d.bk = M2(rp, l, 2 * l);
        d.bn = M1(1);
        d.C = R[j][n];
        d.cm = M1(l);
        d.cn = M1(1);
        d.ab = d.bb = d.cb = M1(0);
        add_tc(plan, d, prec);
      }
    }
  }

  plan.join(L);

  const Prec dprec = data_prec(prec);
  // ---- left-to-right sweep; per bond the terms' contractions run on lanes
  // (the last bond accumulates all terms into one core, in order, on lane 0)
  std::vector<double*> Mcur(J, one), Mnext = Mb;
  for (int n = 0; n < N; ++n) {
    const bool last = (n == N - 1);
    const int l = ell[n], lp = ell[n + 1];
    const int Lb = last ? 1 : L;
    plan.fork(Lb);
    for (int j = 0; j < J; ++j) {
      const auto& r = sh[j].r;
      const auto& D = sh[j].D;
      const int rn = r[n], rp = r[n + 1], Dn = D[n], Dp = D[n + 1];
      const ChainView* W = terms[j].mpo;
      if (Lb > 1) plan.on(j % Lb);
      double* U1 = U1s[j % L];
      double* Cdst = last ? X[N - 1] : Cb[j];
      const double alpha = last ? terms[j].coef : 1.0;
      const double beta = (last && j > 0) ? 1.0 : 0.0;
      if (W) {
        {  // U1[k,alpha,s,b] = sum_a M[k,(a,alpha)] x[a,s,b], batch alpha
          TcDesc d;
          d.batch = Dn;
          d.M = l;
          d.K = rn;
          d.N = 2 * rp;
          d.A = Mcur[j];
          d.am = M1((int64_t)rn * Dn);
          d.ak = M1(Dn);
          d.ab = M1(1);
          d.B = terms[j].x.core[n];
          d.bk = M1(2 * rp);
          d.bn = M1(1);
          d.bb = M1(0);
          d.C = U1;
          d.cm = M1((int64_t)2 * Dn * rp);
          d.cn = M1(1);
          d.cb = M1(2 * rp);
          add_tc(plan, d, dprec);
        }
        {  // C[k,t,b,beta] = sum_(alpha,s) U1[k,alpha,s,b] W[alpha,t,s,beta]
          TcDesc d;
          d.M = l * rp;
          d.K = 2 * Dn;
          d.N = 2 * Dp;
          d.A = U1;
          d.am = M2(rp, (int64_t)2 * Dn * rp, 1);
          d.ak = M1(rp);
          d.B = W->core[n];
          d.bk = M2(2, 4 * Dp, Dp);
          d.bn = M2(Dp, 2 * Dp, 1);
          d.C = Cdst;
          d.cm = M2(rp, (int64_t)2 * rp * Dp, Dp);
          d.cn = M2(Dp, (int64_t)rp * Dp, 1);
          d.ab = d.bb = d.cb = M1(0);
          d.alpha = alpha;
          d.beta = beta;
          add_tc(plan, d, dprec);
        }
      } else {
        add_gemm(plan, l, 2 * rp, rn, Mcur[j], rn, false, terms[j].x.core[n], 2 * rp, false, Cdst,
                 2 * rp, alpha, beta, dprec);
      }
    }
    plan.join(Lb);
    if (last) break;
    // S = sum_j c_j C_j R_j[n+1]
    for (int j = 0; j < J; ++j) {
      const int rp = sh[j].r[n + 1], Dp = sh[j].D[n + 1];
      add_gemm(plan, 2 * l, lp, rp * Dp, Cb[j], (int64_t)rp * Dp, false, R[j][n + 1], lp, false, S,
               lp, terms[j].coef, j > 0 ? 1.0 : 0.0, prec);
    }
    {
      double* Xn = X[n];
      const int m = 2 * l, nc = lp;
      add_qr_q(plan, m, nc, S, nc, 1, Xn, qrw, qrws);
    }
    plan.fork(L);
    for (int j = 0; j < J; ++j) {
      const int rp = sh[j].r[n + 1], Dp = sh[j].D[n + 1];
      if (L > 1) plan.on(j % L);
      add_gemm(plan, lp, rp * Dp, 2 * l, X[n], lp, true, Cb[j], (int64_t)rp * Dp, false, Mnext[j],
               (int64_t)rp * Dp, 1.0, 0.0, dprec);
    }
    plan.join(L);
    for (int j = 0; j < J; ++j) {
      double* old = Mcur[j];
      Mcur[j] = Mnext[j];
      Mnext[j] = (old == one) ? Ma[j] : old;
    }
  }
  plan_trunc_gram(plan, X, ell, tg, dprec);
}

// ---------------------------------------------------------------------------
// deterministic sweeps
// ---------------------------------------------------------------------------
LeftOrth plan_left_orth(Plan& plan, const ChainView& x) {
  const int N = x.N;
  LeftOrth out;
  out.caps.assign(N + 1, 1);
  out.core.assign(N, nullptr);
  // cur: the core at site n after absorbing the factor from the left
  const double* cur = x.core[0];
  int cl = 1;  // left cap of cur
  size_t wsz = 1;
  for (int n = 0; n < N; ++n) wsz = std::max(wsz, (size_t)2 * 2 * x.caps[n] * std::max(x.caps[n + 1], 1));
  for (int n = 0; n < N; ++n) {
    const int cr = x.caps[n + 1];
    if (n == N - 1) {
      double* dst = plan.alloc((size_t)cl * 2 * cr);
      const double* src = cur;
      size_t bytes = (size_t)cl * 2 * cr * sizeof(double);
      plan.add([=](hipStream_t s) {
        rt::copy_async(dst, src, bytes, s);
      });
      out.core[n] = dst;
      out.caps[n] = cl;
      break;
    }
    const int m = 2 * cl;
    const int cnr = x.caps[n + 2];
    int knew;
    double* Q;
    double* next;
    if (m >= cr) {
      knew = cr;
      Q = plan.alloc((size_t)m * cr);
      double* Rm = plan.alloc((size_t)cr * cr);
      const int64_t ws = qr_work_size(1, m, cr);
      double* work = plan.alloc((size_t)ws);
      plan.add([=](hipStream_t s) { qr_launch(1, m, cr, cur, 0, cr, 1, Q, 0, Rm, 0, work, s, nullptr, 0, ws); },
               qr_info(m, cr));
      next = plan.alloc((size_t)knew * 2 * cnr);
      add_gemm(plan, knew, 2 * cnr, cr, Rm, cr, false, x.core[n + 1], 2 * cnr, false, next, 2 * cnr,
               1.0, 0.0, Prec::F64);
    } else {
      knew = m;
      Q = plan.alloc((size_t)m * m);
      plan.add([=](hipStream_t s) { eye(Q, m, s); });
      next = plan.alloc((size_t)knew * 2 * cnr);
      add_gemm(plan, m, 2 * cnr, cr, cur, cr, false, x.core[n + 1], 2 * cnr, false, next, 2 * cnr,
               1.0, 0.0, Prec::F64);
    }
    out.core[n] = Q;
    out.caps[n] = cl;
    out.caps[n + 1] = knew;
    cur = next;
    cl = knew;
  }
  out.caps[N] = 1;
  (void)wsz;
  return out;
}

void plan_round_det(Plan& plan, const ChainView& x, RoundTarget& tg) {
  const int N = x.N;
  // LQ sweep right to left -> right-orthogonal chain with caps c'
  std::vector<double*> rc(N, nullptr);
  std::vector<int> caps(N + 1, 1);
  const double* cur = x.core[N - 1];
  int cr = 1;  // right cap of cur
  for (int n = N - 1; n >= 1; --n) {
    const int cl = x.caps[n];
    const int cols = 2 * cr;
    const int cll = x.caps[n - 1];
    double* next = plan.alloc((size_t)cll * 2 * std::min(cl, cols));
    if (cl <= cols) {
      // A (cl x cols) = L Q from the QR of A^T (cols x cl)
      double* Qt = plan.alloc((size_t)cols * cl);
      double* Rm = plan.alloc((size_t)cl * cl);
      const int64_t ws = qr_work_size(1, cols, cl);
      double* work = plan.alloc((size_t)ws);
      double* core = plan.alloc((size_t)cl * cols);
      const double* A = cur;
      plan.add([=](hipStream_t s) {
        qr_launch(1, cols, cl, A, 0, 1, cols, Qt, 0, Rm, 0, work, s, nullptr, 0, ws);
        transpose(Qt, cols, cl, core, s);
      });
      // left neighbour absorbs L = R^T
      add_gemm(plan, 2 * cll, cl, cl, x.core[n - 1], cl, false, Rm, cl, true, next, cl, 1.0, 0.0,
               Prec::F64);
      rc[n] = core;
      caps[n] = cl;
    } else {
      double* core = plan.alloc((size_t)cols * cols);
      plan.add([=](hipStream_t s) { eye(core, cols, s); });
      add_gemm(plan, 2 * cll, cols, cl, x.core[n - 1], cl, false, cur, cols, false, next, cols, 1.0,
               0.0, Prec::F64);
      rc[n] = core;
      caps[n] = cols;
    }
    cur = next;
    cr = caps[n];
  }
  rc[0] = const_cast<double*>(cur);
  caps[0] = 1;
  ChainView rv;
  rv.N = N;
  rv.p = 2;
  rv.caps = caps;
  for (int n = 0; n < N; ++n) rv.core.push_back(rc[n]);
  LeftOrth lo = plan_left_orth(plan, rv);
  plan_trunc_gram(plan, lo.core, lo.caps, tg, Prec::F64);
}

RoundOutcome round_outcome(const RoundTarget& tg, hipStream_t s) {
  const int N = (int)tg.core.size();
  RoundOutcome o;
  o.discarded.assign(N + 1, 0.0);
  o.kept.assign(N + 1, 1);
  rt::sync(s);
  if (N < 2 || !tg.lam) {
    if (N == 1) {
      double v[2];
      rt::copy(v, tg.core[0], sizeof(v));
      o.norm2 = v[0] * v[0] + v[1] * v[1];
    }
    return o;
  }
  QTT_REQUIRE((int)tg.in_caps.size() == N + 1, "rounding outcome: bonds of the input unknown");
  std::vector<double> lam((size_t)(N + 1) * tg.ldl);
  rt::copy(lam.data(), tg.lam, lam.size() * sizeof(double));
  const double tol2 = tg.rel_tol * tg.rel_tol;
  for (int n = 1; n < N; ++n) {
    const double* l = &lam[(size_t)n * tg.ldl];
    const int e = tg.in_caps[n], keep = std::min(e, tg.caps[n]);
    int k = keep;
    if (tol2 > 0.0) {
      k = 1;
      while (k < keep && l[k] > tol2 * l[0]) ++k;
    }
    double d = 0.0;
    for (int i = k; i < e; ++i) d += std::max(0.0, l[i]);
    o.discarded[n] = d;
    o.kept[n] = k;
  }
  for (int i = 0; i < tg.in_caps[1]; ++i) o.norm2 += std::max(0.0, lam[(size_t)tg.ldl + i]);
  return o;
}

// ---------------------------------------------------------------------------
// block-diagonal sums and environment chains
// ---------------------------------------------------------------------------
void plan_axpby(Plan& plan, const std::vector<std::pair<double, ChainView>>& terms, tt_tt* dst) {
  const int N = dst->N;
  std::vector<CopyJob> jobs;
  std::vector<int> ro(N + 1, 0);
  int64_t maxe = 1;
  for (auto& [c, x] : terms) {
    QTT_REQUIRE(x.N == N, "axpby: chains differ in length");
    for (int n = 0; n < N; ++n) {
      CopyJob j{};
      j.src = x.core[n];
      j.dst = dst->core(n);
      j.rl = x.caps[n];
      j.sp = x.p;
      j.rr = x.caps[n + 1];
      j.dp = dst->p;
      j.drr = dst->caps[n + 1];
      j.ro = (n == 0) ? 0 : ro[n];
      j.co = (n == N - 1) ? 0 : ro[n + 1];
      j.diag = 0;
      j.scale = (n == 0) ? c : 1.0;
      j.dscale = nullptr;
      jobs.push_back(j);
      maxe = std::max<int64_t>(maxe, (int64_t)j.rl * j.sp * j.rr);
    }
    for (int n = 1; n < N; ++n) ro[n] += x.caps[n];
  }
  for (int n = 1; n < N; ++n)
    QTT_REQUIRE(ro[n] <= dst->caps[n], "axpby: destination bond %d too small", n);
  for (const CopyJob& j : jobs) validate(j);
  CopyJob* dj = plan.upload(jobs);
  double* base = dst->buf.d();
  int64_t tot = dst->total();
  int nj = (int)jobs.size();
  OpInfo oi;
  oi.kind = OP_STREAM;
  for (const CopyJob& j : jobs) oi.bytes += 16.0 * j.rl * j.sp * j.rr;
  oi.bytes += 8.0 * tot;
  plan.add([=](hipStream_t s) {
    fuse_check(jobs);
    fill(base, tot, 0.0, s);
    copy_jobs(dj, nj, maxe, s);
  }, oi);
}

void plan_partial(Plan& plan, const ChainView& w, const ChainView& x, double* out_dev) {
  const int Nw = w.N;
  QTT_REQUIRE(x.N >= Nw, "partial contraction longer than the chain");
  size_t esz = 1, tsz = 1;
  for (int n = 0; n <= Nw; ++n) esz = std::max(esz, (size_t)w.caps[n] * x.caps[n]);
  for (int n = 0; n < Nw; ++n) tsz = std::max(tsz, (size_t)w.caps[n] * 2 * x.caps[n + 1]);
  double* Ea = plan.alloc(esz);
  double* Eb = plan.alloc(esz);
  double* T = plan.alloc(tsz);
  double* one;
  if (plan.arena) {  // no uploads into a fixed scratch buffer: write the 1 when the plan runs
    one = plan.alloc(1);
    plan.add([one](hipStream_t s) { fill(one, 1, 1.0, s); });
  } else {
    one = plan.upload(std::vector<double>{1.0});
  }
  const double* E = one;
  for (int n = 0; n < Nw; ++n) {
    const int wl = w.caps[n], wr = w.caps[n + 1], xl = x.caps[n], xr = x.caps[n + 1];
    // T[w, (s, R)] = sum_r E[w, r] x[r, s, R]
    add_gemm(plan, wl, 2 * xr, xl, E, xl, false, x.core[n], 2 * xr, false, T, 2 * xr, 1.0, 0.0, Prec::F64);
    double* En = (n == Nw - 1) ? out_dev : ((E == Ea) ? Eb : Ea);
    // E'[W, R] = sum_(w,s) w[(w,s), W] T[(w,s), R]
    add_gemm(plan, wr, xr, 2 * wl, w.core[n], wr, true, T, xr, false, En, xr, 1.0, 0.0, Prec::F64);
    E = En;
  }
}

void plan_inner(Plan& plan, const ChainView& a, const ChainView& b, double* out_dev) {
  QTT_REQUIRE(a.N == b.N, "inner: chains differ in length");
  plan_partial(plan, a, b, out_dev);
}

}  // namespace qtt
