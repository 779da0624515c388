// extern "C" entry points of the qttpdf library (declared in include/qttpdf.h).
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <thread>

#include "library.h"
#include "moments.h"

namespace qtt {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
const char* get_error() { return g_err.c_str(); }

StreamScope::StreamScope(tt_ctx* ctx) : c(ctx) {
  if (rt::dry()) return;
  QTT_HIP(hipSetDevice(c->device));
  if (c->user_stream != c->stream) {
    QTT_HIP(hipEventRecord(c->ev_in, c->user_stream));
    QTT_HIP(hipStreamWaitEvent(c->stream, c->ev_in, 0));
  }
}
StreamScope::~StreamScope() {
  if (!rt::dry() && c->user_stream != c->stream) {
    (void)hipEventRecord(c->ev_out, c->stream);
    (void)hipStreamWaitEvent(c->user_stream, c->ev_out, 0);
  }
}

static Prec prec_of(int dtype) {
  switch (dtype) {
    case TT_F64: return Prec::F64;
    case TT_F32: return Prec::F32;
    case TT_BF16: return Prec::BF16;
  }
  QTT_THROW(TT_ERR_INVALID_ARG, "unknown dtype %d", dtype);
}

static host::TT download(const tt_tt* t) {
  std::vector<double> h(t->total());
  rt::sync(t->ctx->stream);
  rt::copy(h.data(), t->buf.p, h.size() * sizeof(double));
  host::TT out;
  for (int n = 0; n < t->N; ++n) {
    host::Core G(t->caps[n], t->p, t->caps[n + 1]);
    std::copy(h.begin() + t->off[n], h.begin() + t->off[n + 1], G.v.begin());
    out.push_back(std::move(G));
  }
  return out;
}

// host chain -> device chain with the given capacities (zero padded)
static std::unique_ptr<tt_tt> upload(tt_ctx* ctx, int kind, const host::TT& x,
                                     const std::vector<int>& caps) {
  const int N = (int)x.size();
  auto t = make_tt(ctx, kind, N, caps);
  std::vector<double> h(t->total(), 0.0);
  for (int n = 0; n < N; ++n) {
    const host::Core& G = x[n];
    QTT_REQUIRE(G.rl <= caps[n] && G.rr <= caps[n + 1], "bond %d exceeds its capacity", n);
    for (int a = 0; a < G.rl; ++a)
      for (int s = 0; s < G.p; ++s)
        for (int b = 0; b < G.rr; ++b)
          h[t->off[n] + ((int64_t)a * t->p + s) * caps[n + 1] + b] = G.at(a, s, b);
  }
  rt::copy(t->buf.p, h.data(), h.size() * sizeof(double));
  return t;
}

static std::vector<int> exact_caps(const host::TT& x) {
  std::vector<int> c(x.size() + 1, 1);
  for (size_t n = 0; n < x.size(); ++n) c[n + 1] = x[n].rr;
  c[0] = 1;
  return c;
}

static void check_tt(const tt_tt* t, tt_ctx* ctx = nullptr) {
  QTT_REQUIRE(t != nullptr, "null tensor-train handle");
  if (ctx) QTT_REQUIRE(t->ctx == ctx, "handle belongs to another context");
}

// ---------------------------------------------------------------------------
// operator assembly
// ---------------------------------------------------------------------------
static host::TT build_mpo_host(int ndims, int bits, int ordering, const tt_term* terms, int n_terms,
                               const std::vector<host::TT>& fields, int field_ndims, double rel_tol) {
  auto order = host::site_order(ndims, bits, ordering);
  const int N = ndims * bits;
  std::vector<host::TT> parts;
  std::vector<host::TT> ops1d(8);
  std::vector<bool> have(8, false);
  parts.reserve(n_terms);
  for (int t = 0; t < n_terms; ++t) {
    std::vector<host::TT> per(ndims);
    std::vector<const host::TT*> pp(ndims, nullptr);
    for (int d = 0; d < ndims; ++d) {
      int op = terms[t].op[d];
      QTT_REQUIRE(op >= TT_OP_ID && op <= TT_OP_D1G_PHI, "term %d: bad operator code %d", t, op);
      if (op == TT_OP_ID) continue;
      if (!have[op]) {
        ops1d[op] = host::op1d(op, bits);
        have[op] = true;
      }
      pp[d] = &ops1d[op];
    }
    host::TT W = host::kron_dims(pp, order, ndims, 4);
    if (terms[t].field >= 0) {
      QTT_REQUIRE(terms[t].field < (int)fields.size(), "term %d: bad field index", t);
      QTT_REQUIRE(ordering == TT_SERIAL, "fields need the serial ordering");
      const host::TT& f = fields[terms[t].field];
      const int nf = field_ndims * bits;
      QTT_REQUIRE((int)f.size() == nf, "field length %zu != %d", f.size(), nf);
      host::TT diag = host::mpo_identity(N - nf);
      host::TT dg = host::mpo_diag(f);
      diag.insert(diag.end(), dg.begin(), dg.end());
      W = host::mpo_compose(diag, W);
    }
    parts.push_back(std::move(W));
  }
  std::vector<std::pair<double, const host::TT*>> sum;
  for (int t = 0; t < n_terms; ++t) sum.emplace_back(terms[t].coeff, &parts[t]);
  host::TT A = host::tt_sum(sum);
  if (rel_tol > 0) A = host::round_svd(A, rel_tol, 1 << 30);
  return A;
}

// ---------------------------------------------------------------------------
// Static scratch of the entry points that allocate nothing (tt_inner_noalloc).
// Every GPU the library runs on holds its own copy of `scratch` until the
// process ends.  Host code never passes the array's name to a kernel: the
// device address of each GPU's copy is looked up once per device, with that
// device current, when the first context on it is created (tt_ctx_create),
// and kept in g_scratch_dev.  Dry runs use a host buffer in its place.
// ---------------------------------------------------------------------------
constexpr size_t kScratchDoubles = size_t(4) << 20;  // 32 MiB
constexpr int kMaxDevices = 64;
__device__ __align__(256) double scratch[kScratchDoubles];
static std::mutex g_scratch_mu;
static double* g_scratch_dev[kMaxDevices] = {};

static void scratch_init(int device) {
  QTT_REQUIRE(device >= 0 && device < kMaxDevices, "device %d beyond the scratch table", device);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_dev[device]) return;
  void* p = nullptr;
  if (rt::dry()) {
    p = std::calloc(kScratchDoubles, sizeof(double));
    if (!p) QTT_THROW(TT_ERR_OOM, "host stand-in of the static scratch");
  } else {
    QTT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  }
  rt::register_range(p, kScratchDoubles * sizeof(double));
  g_scratch_dev[device] = static_cast<double*>(p);
}

static double* scratch_of(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return (device >= 0 && device < kMaxDevices) ? g_scratch_dev[device] : nullptr;
}

// Enters a caller-owned device range into the bounds-check registry for the
// lifetime of the scope, unless an allocation of the library already covers it.
struct CallerRange {
  const void* p = nullptr;
  CallerRange(const void* ptr, size_t bytes, const char* what) {
    try {
      rt::check_range(ptr, 0, (int64_t)bytes - 1, 1, what);
    } catch (const Error&) {
      rt::register_range(ptr, bytes);
      p = ptr;
    }
  }
  ~CallerRange() {
    if (p) rt::unregister_range(p);
  }
};

}  // namespace qtt

using namespace qtt;

// ===========================================================================
// problem
// ===========================================================================
struct tt_problem {
  tt_ctx* ctx = nullptr;
  tt_params p{};
  int N = 0, nphi = 0, nx = 0;
  std::vector<int> fcaps, mcaps;
  std::unique_ptr<tt_tt> Z, Zm;    // sketches read from the right end
  std::unique_ptr<tt_tt> Zl, Zml;  // sketches read from the left end (two-sided rounding)
  std::unique_ptr<tt_tt> A;   // combined stage operator: fixed (+) mean-field part
  std::vector<int> Dfix;      // bonds of the fixed operator
  std::unique_ptr<tt_tt> Wm;  // mean-field weights over the phi sites (2 output channels)
  // flow-case x-fields: total diffusivity G(x) and LMSE frequency Omega(x);
  // Wom = diag(Omega) over the x sites (weights the mean-field rounding)
  bool has_G = false, has_Om = false;
  std::unique_ptr<tt_tt> Wom;
  ChainView Womv;
  DevBuf mf_first;                  // 2-D: unscaled first-core blocks [1][4][cols_a] of the two
  std::vector<int> mf_first_off;    //      mean-field terms, block a at a * 4 * mf_first_ld
  std::vector<int> mf_first_cols;
  int mf_first_ld = 1;
  std::unique_ptr<tt_tt> k[4];
  std::unique_ptr<tt_tt> mt[2];
  // Hadamard form of the mean-field term (5-D): the fixed operator F and, per
  // composition a, the term -Omega D1g^(phi_a) diag(<Phi_a>) as an MPO of its
  // own whose x-site cores are diagonal (written every stage), rounded as
  // separate terms instead of the block sum A when that is cheaper
  bool split_mf = false;
  std::unique_ptr<tt_tt> F, MF[2];
  ChainView Fv, MFv[2];
  DevBuf Ef, Ek, mff, mfk, scal;
  int cphi = 1, cphi1 = 1;  // caps of f at the phi|x cut and after the first x site
  // recorded step
  std::unique_ptr<Plan> plan;
  const tt_tt* plan_f = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  RoundTarget last;              // final rounding of the recording that ran last
  RoundTarget last_plain, last_tan;  // ... of the plain and of the tangent recording
  std::unique_ptr<Plan> obs_plan;
  DevBuf nonfinite;  // device int: set when a rounding of a step produced a NaN or Inf
  // host copy of the mean-field chain over the phi sites (unscaled) and the
  // mean-field bonds, for assembling further stage-shaped operators
  host::TT MFh;
  std::vector<int> Dmf;
  // forward-mode derivatives with respect to parameter q (0 Omega, 1 k):
  // operator B_q = dA_fix/dq - sum_a D1g^(phi_a) diag(.), its fixed bonds,
  // tangent stage slopes, rounded tangent mean fields, raw partial sums
  std::unique_ptr<tt_tt> Bt[2];
  std::vector<int> Dfix_t[2];
  std::unique_ptr<tt_tt> dk[2][4];
  std::unique_ptr<tt_tt> mtt[2][2];
  DevBuf Edf[2], Edk[2], mfdf[2], mfdk[2];
  std::unique_ptr<Plan> tplan;
  std::vector<const void*> tplan_key;
  hipGraph_t tgraph = nullptr;
  hipGraphExec_t texec = nullptr;
  ~tt_problem() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (texec) (void)hipGraphExecDestroy(texec);
    if (tgraph) (void)hipGraphDestroy(tgraph);
  }
};

namespace qtt {

// A stage-shaped MPO: the fixed part F stacked with the mean-field chain over
// the phi sites (its first core scaled by mf_scale) whose x-site blocks,
// diag(<Phi_a>) of a rounded mean field, are written when a step runs.  The
// time step dt is folded into the first core: the recorded step computes the
// stage increments dt k_i, so no launch of it depends on dt (problems that
// differ only in their coefficients record the same launches).
static std::unique_ptr<tt_tt> assemble_stage_mpo(tt_problem* P, const host::TT& F, double mf_scale,
                                                 std::vector<int>& Dfix) {
  const int N = P->N;
  Dfix = exact_caps(F);
  std::vector<int> Dc(N + 1, 1);
  for (int n = 1; n < N; ++n) Dc[n] = Dfix[n] + P->Dmf[n];
  auto A = make_tt(P->ctx, TT_MPO, N, Dc);
  std::vector<double> h(A->total(), 0.0);
  auto put = [&](int n, const host::Core& B, int ro, int co, double sc) {
    for (int i = 0; i < B.rl; ++i)
      for (int s = 0; s < 4; ++s)
        for (int j = 0; j < B.rr; ++j)
          h[A->off[n] + ((int64_t)(ro + i) * 4 + s) * Dc[n + 1] + co + j] = sc * B.at(i, s, j);
  };
  const double dt = P->p.dt;
  for (int n = 0; n < N; ++n) {
    put(n, F[n], 0, 0, n == 0 ? dt : 1.0);
    if (n < P->nphi) {
      const int ro = (n == 0) ? 0 : Dfix[n];
      const int co = (n == N - 1) ? 0 : Dfix[n + 1];
      put(n, P->MFh[n], ro, co, n == 0 ? mf_scale * dt : 1.0);
    }
  }
  rt::copy(A->buf.p, h.data(), h.size() * sizeof(double));
  return A;
}

// mean-field partial contraction of x over the phi sites: E (2 x cphi), and
// for 5-D the first x-core of each raw mean field, first[a] = E[a,:] x_{nphi}
static void plan_mean_raw(Plan& plan, tt_problem* P, const tt_tt* x, double* E, double* first) {
  ChainView w = view(P->Wm.get());
  ChainView xs = view_sites(x, 0, P->nphi);
  plan_partial(plan, w, xs, E);
  if (P->nx > 0) {
    const int c = x->caps[P->nphi], c1 = x->caps[P->nphi + 1];
    TcDesc d = gemm_desc(2, 2 * c1, c, E, c, false, x->core(P->nphi), 2 * c1, false, first, 2 * c1);
    plan.add([d](hipStream_t s) { tc_launch(d, Prec::F64, s); });
  }
}

// raw mean field a of x as an x-chain: first core from `first`, the rest from x
static ChainView mean_view(tt_problem* P, const tt_tt* x, const double* first, int a) {
  ChainView v;
  v.N = P->nx;
  v.p = 2;
  v.caps.push_back(1);
  for (int j = 1; j <= P->nx; ++j) v.caps.push_back(x->caps[P->nphi + j]);
  v.core.push_back(first + (size_t)a * 2 * x->caps[P->nphi + 1]);
  for (int j = 1; j < P->nx; ++j) v.core.push_back(x->core(P->nphi + j));
  return v;
}

// one term c * <Phi_a>(x) of a raw mean field (first x-core in `first`)
struct MeanTerm {
  double c;
  const tt_tt* x;
  const double* first;
};

// 5-D: rounds sum_j c_j <Phi_a>(x_j) to chi_mean into mt[a], a = 0, 1 (the
// two roundings recorded side by side, sharing the lanes)
static void plan_mean_round(Plan& plan, tt_problem* P, const std::vector<MeanTerm>& terms,
                            tt_tt* const mt[2]) {
  ChainView Zm = view(P->Zm.get());
  ChainView Zml = view(P->Zml.get());
  std::vector<SketchTerm> st[2];
  RoundTarget tg[2];
  std::vector<RoundJob> jobs;
  for (int a = 0; a < 2; ++a) {
    for (const MeanTerm& m : terms) {
      SketchTerm t;
      t.coef = m.c;
      t.mpo = P->has_Om ? &P->Womv : nullptr;
      t.x = mean_view(P, m.x, m.first, a);
      st[a].push_back(t);
    }
    for (int j = 0; j < P->nx; ++j) tg[a].core.push_back(mt[a]->core(j));
    tg[a].caps = mt[a]->caps;
    jobs.push_back({&st[a], &tg[a]});
  }
  plan_round_two_sided_multi(plan, jobs, Zm, Zml, Prec::F64, 4);
}

// 5-D: writes diag(mt[a]) into the x-site mean-field blocks of a stage-shaped
// MPO whose fixed part has bonds Dfix
static void plan_mf_blocks(Plan& plan, tt_problem* P, tt_tt* mpo, const std::vector<int>& Dfix,
                           tt_tt* const mt[2]) {
  std::vector<CopyJob> jobs;
  int64_t maxe = 1;
  const int N = P->N, nphi = P->nphi, nx = P->nx;
  for (int j = 0; j < nx; ++j) {
    const int n = nphi + j;
    for (int a = 0; a < 2; ++a) {
      const tt_tt* m = mt[a];
      CopyJob c{};
      c.src = m->core(j);
      c.dst = mpo->core(n);
      c.rl = m->caps[j];
      c.sp = 2;
      c.rr = m->caps[j + 1];
      c.dp = 4;
      c.drr = mpo->caps[n + 1];
      const int row0 = (n == 0) ? 0 : Dfix[n];
      const int col0 = (n == N - 1) ? 0 : Dfix[n + 1];
      c.ro = row0 + ((j == 0) ? a : a * P->mcaps[j]);
      c.co = col0 + ((j == nx - 1) ? 0 : a * P->mcaps[j + 1]);
      c.diag = 1;
      c.scale = 1.0;
      c.dscale = nullptr;
      jobs.push_back(c);
      maxe = std::max<int64_t>(maxe, (int64_t)c.rl * 2 * c.rr);
    }
  }
  for (const CopyJob& j : jobs) validate(j);
  CopyJob* dj = plan.upload(jobs);
  const int nj = (int)jobs.size();
  plan.add([=](hipStream_t s) {
    fuse_check(jobs);
    copy_jobs(dj, nj, maxe, s);
  });
}

// writes diag(mt[a]) into the x-site cores of the Hadamard-form term MF[a]
static void plan_mf_diag(Plan& plan, tt_problem* P, tt_tt* const mt[2]) {
  std::vector<CopyJob> jobs;
  int64_t maxe = 1;
  for (int a = 0; a < 2; ++a)
    for (int j = 0; j < P->nx; ++j) {
      const int n = P->nphi + j;
      CopyJob c{};
      c.src = mt[a]->core(j);
      c.dst = P->MF[a]->core(n);
      c.rl = mt[a]->caps[j];
      c.sp = 2;
      c.rr = mt[a]->caps[j + 1];
      c.dp = 4;
      c.drr = P->MF[a]->caps[n + 1];
      c.ro = 0;
      c.co = 0;
      c.diag = 1;
      c.scale = 1.0;
      c.dscale = nullptr;
      jobs.push_back(c);
      maxe = std::max<int64_t>(maxe, (int64_t)c.rl * 2 * c.rr);
    }
  for (const CopyJob& j : jobs) validate(j);
  CopyJob* dj = plan.upload(jobs);
  const int nj = (int)jobs.size();
  plan.add([=](hipStream_t s) {
    fuse_check(jobs);
    copy_jobs(dj, nj, maxe, s);
  });
}

// writes the mean-field part of the stage operator for the state
// g = f + cg * kprev (kprev may be null): the blocks of A, or with split the
// diagonal cores of MF[0], MF[1]
static void plan_stage_operator(Plan& plan, tt_problem* P, const tt_tt* f, const tt_tt* kprev,
                                double cg, bool split = false) {
  const tt_params& p = P->p;
  if (P->nx == 0) {
    // 2-D: scalars s_a = -Omega dt (m_a(f) + cg m_a(k)); first-core blocks scaled
    double* sc = P->scal.d();
    const double* ef = P->Ef.d();
    const double* ek = kprev ? P->Ek.d() : nullptr;
    const double om = p.omega * p.dt;
    plan.add([=](hipStream_t s) { scalar_comb(sc, ef, ek, cg, -om, 2, s); });
    std::vector<CopyJob> jobs;
    int64_t maxe = 1;
    for (int a = 0; a < 2; ++a) {
      CopyJob j{};
      j.src = P->mf_first.d() + (size_t)a * 4 * P->mf_first_ld;
      j.dst = P->A->core(0);
      j.rl = 1;
      j.sp = 4;
      j.rr = P->mf_first_cols[a];
      j.dp = 4;
      j.drr = P->A->caps[1];
      j.ro = 0;
      j.co = P->Dfix[1] + P->mf_first_off[a];
      j.diag = 0;
      j.scale = 1.0;
      j.dscale = sc + a;
      jobs.push_back(j);
      maxe = std::max<int64_t>(maxe, 4 * j.rr);
    }
    for (const CopyJob& j : jobs) validate(j);
    CopyJob* dj = plan.upload(jobs);
    plan.add([=](hipStream_t s) {
      fuse_check(jobs);
      copy_jobs(dj, 2, maxe, s);
    });
    return;
  }
  // 5-D: round the raw mean fields of g over the x sites, write diag blocks
  std::vector<MeanTerm> terms{{1.0, f, P->mff.d()}};
  if (kprev) terms.push_back({cg, kprev, P->mfk.d()});
  tt_tt* mt[2] = {P->mt[0].get(), P->mt[1].get()};
  plan_mean_round(plan, P, terms, mt);
  if (split) plan_mf_diag(plan, P, mt);
  else plan_mf_blocks(plan, P, P->A.get(), P->Dfix, mt);
}

// flags a NaN or Inf in the cores of x (after a rounding wrote them)
static void plan_check_finite(Plan& plan, const tt_tt* x, int* flag) {
  const double* p = x->buf.d();
  const int64_t n = x->total();
  plan.add([=](hipStream_t s) { check_finite(p, n, flag, s); });
}

// forward-mode derivative carried along a step: parameter q and its tangent df
struct Tangent {
  int q;
  tt_tt* df;
};

// Records one step of f; with tangents, also the derivative of the step
// with respect to each parameter (forward mode, stage by stage): with
// g_i = f + c_i k_(i-1) and dg_i = df + c_i dk_(i-1),
//   dk_i = Round( A(g_i) dg_i + B_q(g_i, dg_i) g_i ),
//   B_q = dA_fix/dq - sum_a D1g^(phi_a) diag(alpha_q <Phi_a>(g_i) + Omega <Phi_a>(dg_i)),
// alpha_Omega = 1, alpha_k = 0 (the mean field enters A through -Omega m_a(g)),
// and df+ = Round(df + sum_i b_i dk_i) beside f+ = Round(f + sum_i b_i k_i),
// where the last stage's k_S = A(g_S) g_S (and dk_S) enters the final
// rounding unrounded, as its MPO x MPS terms.  A and B_q carry dt, so k_i
// and dk_i are increments (dt times the slopes) and c_i, b_i are the
// tableau's plain numbers.
static std::unique_ptr<Plan> record_step(tt_problem* P, tt_tt* f, const std::vector<Tangent>& tan) {
  auto plan = std::make_unique<Plan>();
  const tt_params& p = P->p;
  const Prec prec = prec_of(p.dtype);
  ChainView Z = view(P->Z.get());
  ChainView Zl = view(P->Zl.get());
  ChainView Av = view(P->A.get());
  const bool rk4 = (p.integrator == TT_RK4);
  const int S = rk4 ? 4 : 2;
  // the stage operators carry dt (assemble_stage_mpo): k_i below is the stage
  // increment dt times the slope, g_i = f + c_i k_(i-1), f+ = f + sum_i b_i k_i
  const double cst[4] = {0.0, rk4 ? 0.5 : 1.0, 0.5, 1.0};
  std::vector<ChainView> Bv;
  for (const Tangent& t : tan) Bv.push_back(view(P->Bt[t.q].get()));
  auto sterm = [](double c, const ChainView* W, const tt_tt* x) {
    SketchTerm t;
    t.coef = c;
    t.mpo = W;
    t.x = view(x);
    return t;
  };
  auto target = [&](const tt_tt* x) {
    RoundTarget tg;
    for (int n = 0; n < P->N; ++n) tg.core.push_back(x->core(n));
    tg.caps = P->fcaps;
    return tg;
  };
  const double b4[4] = {1.0 / 6, 1.0 / 3, 1.0 / 3, 1.0 / 6}, b2[2] = {0.5, 0.5};
  const double* b = rk4 ? b4 : b2;
  // The last stage's product is never rounded by itself: its terms, weighted
  // by b_S, join the final combination's rounding (f is rounded once per
  // step, the slopes k_1 .. k_(S-1) once each).
  std::vector<SketchTerm> last;
  std::vector<std::vector<SketchTerm>> last_t(tan.size());
  plan_mean_raw(*plan, P, f, P->Ef.d(), P->mff.d());
  for (const Tangent& t : tan) plan_mean_raw(*plan, P, t.df, P->Edf[t.q].d(), P->mfdf[t.q].d());
  for (int i = 0; i < S; ++i) {
    const tt_tt* kp = (i == 0) ? nullptr : P->k[i - 1].get();
    const double cg = cst[i];
    const bool final_stage = (i == S - 1);
    const double w = final_stage ? b[i] : 1.0;
    if (kp) plan_mean_raw(*plan, P, kp, P->Ek.d(), P->mfk.d());
    const bool split = P->split_mf && tan.empty();
    plan_stage_operator(*plan, P, f, kp, cg, split);
    {
      std::vector<SketchTerm> terms;
      if (split) {
        // F g + sum_a MF_a g, g = f + cg kp: the mean-field terms' x sites are diagonal
        for (const ChainView* W : {&P->Fv, &P->MFv[0], &P->MFv[1]}) {
          const int df = (W == &P->Fv) ? -1 : P->nphi;
          terms.push_back(sterm(w, W, f));
          terms.back().diag_from = df;
          if (kp) {
            terms.push_back(sterm(w * cg, W, kp));
            terms.back().diag_from = df;
          }
        }
      } else {
        terms.push_back(sterm(w, &Av, f));
        if (kp) terms.push_back(sterm(w * cg, &Av, kp));
      }
      if (final_stage) {
        last = terms;
      } else {
        RoundTarget tg = target(P->k[i].get());
        plan_round_sketch_two_sided(*plan, terms, Z, Zl, tg, prec);
        plan_check_finite(*plan, P->k[i].get(), P->nonfinite.as<int>());
      }
    }
    for (size_t j = 0; j < tan.size(); ++j) {
      const int q = tan[j].q;
      const tt_tt* df = tan[j].df;
      const tt_tt* dkp = (i == 0) ? nullptr : P->dk[q][i - 1].get();
      if (dkp) plan_mean_raw(*plan, P, dkp, P->Edk[q].d(), P->mfdk[q].d());
      std::vector<MeanTerm> mterms;
      if (q == 0) {
        mterms.push_back({1.0, f, P->mff.d()});
        if (kp) mterms.push_back({cg, kp, P->mfk.d()});
      }
      mterms.push_back({p.omega, df, P->mfdf[q].d()});
      if (dkp) mterms.push_back({p.omega * cg, dkp, P->mfdk[q].d()});
      tt_tt* mt[2] = {P->mtt[q][0].get(), P->mtt[q][1].get()};
      plan_mean_round(*plan, P, mterms, mt);
      plan_mf_blocks(*plan, P, P->Bt[q].get(), P->Dfix_t[q], mt);
      std::vector<SketchTerm> terms{sterm(w, &Av, df), sterm(w, &Bv[j], f)};
      if (kp) {
        terms.push_back(sterm(w * cg, &Av, dkp));
        terms.push_back(sterm(w * cg, &Bv[j], kp));
      }
      if (final_stage) {
        last_t[j] = terms;
      } else {
        RoundTarget tg = target(P->dk[q][i].get());
        plan_round_sketch_two_sided(*plan, terms, Z, Zl, tg, prec);
        plan_check_finite(*plan, P->dk[q][i].get(), P->nonfinite.as<int>());
      }
    }
  }
  // The final combination is dominated by f itself, whose every digit the
  // next step inherits: its sketches run in the data precision (FP32 when
  // BF16 is requested), while BF16 serves the sketches of the stage slopes,
  // whose errors enter f+ weighted by dt.
  auto combine = [&](tt_tt* x, std::unique_ptr<tt_tt>* ks, const std::vector<SketchTerm>& tail) {
    std::vector<SketchTerm> comb{sterm(1.0, nullptr, x)};
    for (int i = 0; i + 1 < S; ++i) comb.push_back(sterm(b[i], nullptr, ks[i].get()));
    comb.insert(comb.end(), tail.begin(), tail.end());
    RoundTarget tg = target(x);
    plan_round_sketch_two_sided(*plan, comb, Z, Zl, tg, data_prec(prec));
    plan_check_finite(*plan, x, P->nonfinite.as<int>());
    return tg;
  };
  // the tangents' final terms read f (B_q f): their roundings go before f's own
  for (size_t j = 0; j < tan.size(); ++j) combine(tan[j].df, P->dk[tan[j].q], last_t[j]);
  P->last = combine(f, P->k, last);
  return plan;
}

static void build_step_plan(tt_problem* P, tt_tt* f) {
  auto plan = record_step(P, f, {});
  if (P->exec) {
    (void)hipGraphExecDestroy(P->exec);
    P->exec = nullptr;
  }
  if (P->graph) {
    (void)hipGraphDestroy(P->graph);
    P->graph = nullptr;
  }
  P->plan = std::move(plan);
  P->plan_f = f;
  P->last_plain = P->last;
}

// operator and buffers of the derivative with respect to parameter q
static void ensure_tangent(tt_problem* P, int q) {
  if (P->Bt[q]) return;
  QTT_REQUIRE(P->nx > 0, "parameter derivatives are available for 5-D problems");
  const tt_params& p = P->p;
  std::vector<tt_term> terms;
  for (int a = 0; a < 2; ++a) {
    tt_term t{};
    t.coeff = 1.0;
    for (int d = 0; d < 8; ++d) t.op[d] = TT_OP_ID;
    t.op[a] = TT_OP_D1G_PHI;  // d/dOmega of Omega D1g diag(phi_a)
    if (q == 1) t.op[1 - a] = TT_OP_PHI;  // d/dk of k D1g diag(phi1 phi2)
    t.field = -1;
    terms.push_back(t);
  }
  host::TT F = build_mpo_host(p.ndims, p.bits, p.ordering, terms.data(), (int)terms.size(), {}, 3, 1e-13);
  P->Bt[q] = assemble_stage_mpo(P, F, -1.0, P->Dfix_t[q]);
  const int S = (p.integrator == TT_RK4) ? 4 : 2;
  for (int i = 0; i < S; ++i) {
    P->dk[q][i] = make_tt(P->ctx, TT_MPS, P->N, P->fcaps);
    fill(P->dk[q][i]->buf.d(), P->dk[q][i]->total(), 0.0, P->ctx->stream);
  }
  for (int a = 0; a < 2; ++a) P->mtt[q][a] = make_tt(P->ctx, TT_MPS, P->nx, P->mcaps);
  P->Edf[q].alloc(sizeof(double) * 2 * P->cphi);
  P->Edk[q].alloc(sizeof(double) * 2 * P->cphi);
  P->mfdf[q].alloc(sizeof(double) * 2 * 2 * P->cphi1);
  P->mfdk[q].alloc(sizeof(double) * 2 * 2 * P->cphi1);
}

static bool use_graph() {
  const char* e = std::getenv("QTTPDF_NO_GRAPH");
  return !(e && e[0] == '1');
}

}  // namespace qtt

// ===========================================================================
// extern "C"
// ===========================================================================
extern "C" {

const char* tt_last_error(void) { return get_error(); }

tt_status tt_autotune_info(int* shapes, double* seconds) {
  return guard([&] { tc_autotune_stats(shapes, seconds); });
}

tt_status tt_set_allocator(tt_alloc_fn alloc, tt_free_fn free, void* user) {
  return guard([&] {
    QTT_REQUIRE((alloc == nullptr) == (free == nullptr), "give both allocator functions or neither");
    rt::set_allocator(alloc, free, user);
  });
}

tt_status tt_ctx_create(int device, void* hip_stream, tt_ctx** out) {
  return guard([&] {
    QTT_REQUIRE(out != nullptr, "out is null");
    auto c = std::make_unique<tt_ctx>();
    c->device = device;
    if (rt::dry()) {
      scratch_init(device);
      *out = c.release();
      return;
    }
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0) QTT_THROW(TT_ERR_STATE, "no HIP device available");
    QTT_REQUIRE(device >= 0 && device < n, "device %d out of range (%d devices)", device, n);
    QTT_HIP(hipSetDevice(device));
    scratch_init(device);
    QTT_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    QTT_HIP(hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming));
    QTT_HIP(hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming));
    c->user_stream = static_cast<hipStream_t>(hip_stream);
    *out = c.release();
  });
}

tt_status tt_ctx_destroy(tt_ctx* ctx) {
  return guard([&] {
    if (!ctx) return;
    if (!rt::dry()) {
      (void)hipStreamSynchronize(ctx->stream);
      (void)hipEventDestroy(ctx->ev_in);
      (void)hipEventDestroy(ctx->ev_out);
      (void)hipStreamDestroy(ctx->stream);
    }
    delete ctx;
  });
}

tt_status tt_ctx_set_stream(tt_ctx* ctx, void* hip_stream) {
  return guard([&] {
    QTT_REQUIRE(ctx, "null context");
    ctx->user_stream = static_cast<hipStream_t>(hip_stream);
  });
}

tt_status tt_ctx_synchronize(tt_ctx* ctx) {
  return guard([&] {
    QTT_REQUIRE(ctx, "null context");
    rt::sync(ctx->stream);
  });
}

tt_status tt_alloc(tt_ctx* ctx, tt_kind kind, int n_sites, const int32_t* bond_caps, tt_tt** out) {
  return guard([&] {
    QTT_REQUIRE(ctx && out && bond_caps, "null argument");
    QTT_REQUIRE(kind == TT_MPS || kind == TT_MPO, "bad kind");
    std::vector<int> caps(bond_caps, bond_caps + n_sites + 1);
    auto t = make_tt(ctx, kind, n_sites, caps);
    StreamScope sc(ctx);
    fill(t->buf.d(), t->total(), 0.0, ctx->stream);
    *out = t.release();
  });
}

tt_status tt_free(tt_tt* t) {
  return guard([&] {
    if (!t) return;
    if (!rt::dry()) (void)hipDeviceSynchronize();
    delete t;
  });
}

tt_status tt_info(const tt_tt* t, int* kind, int* n_sites, int32_t* bond_caps, int64_t* n_elems) {
  return guard([&] {
    check_tt(t);
    if (kind) *kind = t->kind;
    if (n_sites) *n_sites = t->N;
    if (bond_caps)
      for (int n = 0; n <= t->N; ++n) bond_caps[n] = t->caps[n];
    if (n_elems) *n_elems = t->total();
  });
}

tt_status tt_set_cores(tt_tt* t, const double* host_packed) {
  return guard([&] {
    check_tt(t);
    QTT_REQUIRE(host_packed, "null host pointer");
    StreamScope sc(t->ctx);
    rt::copy_async(t->buf.p, host_packed, t->total() * sizeof(double), t->ctx->stream);
    rt::sync(t->ctx->stream);
  });
}

tt_status tt_get_cores(const tt_tt* t, double* host_packed) {
  return guard([&] {
    check_tt(t);
    QTT_REQUIRE(host_packed, "null host pointer");
    StreamScope sc(t->ctx);
    rt::copy_async(host_packed, t->buf.p, t->total() * sizeof(double), t->ctx->stream);
    rt::sync(t->ctx->stream);
  });
}

tt_status tt_from_separable(tt_ctx* ctx, int ndims, int bits, int ordering, int n_terms,
                            const double* coeffs, const double* const* v, int chi, tt_tt** out) {
  return guard([&] {
    QTT_REQUIRE(ctx && out && coeffs && v, "null argument");
    QTT_REQUIRE(ndims >= 1 && ndims <= 8 && bits >= 1 && bits <= 20 && n_terms >= 1 && chi >= 1,
                "bad sizes");
    QTT_REQUIRE(ordering == TT_SERIAL || ordering == TT_INTERLEAVED, "bad ordering");
    auto order = host::site_order(ndims, bits, ordering);
    std::vector<host::TT> parts(n_terms);
    std::vector<std::pair<double, const host::TT*>> sum;
    for (int t = 0; t < n_terms; ++t) {
      std::vector<host::TT> per(ndims);
      std::vector<const host::TT*> pp(ndims, nullptr);
      for (int d = 0; d < ndims; ++d) {
        const double* vec = v[(size_t)t * ndims + d];
        if (vec) {
          per[d] = host::vector_qtt(vec, bits);
          pp[d] = &per[d];
        }
      }
      parts[t] = host::kron_dims(pp, order, ndims, 2);
      sum.emplace_back(coeffs[t], &parts[t]);
    }
    host::TT x = host::round_gram(host::tt_sum(sum), chi);
    const int N = ndims * bits;
    auto t = upload(ctx, TT_MPS, x, chain_caps(N, chi));
    *out = t.release();
  });
}

tt_status mpo_build(tt_ctx* ctx, int ndims, int bits, int ordering, const tt_term* terms,
                    int n_terms, const tt_tt* const* fields, int n_fields, int field_ndims,
                    double rel_tol, tt_tt** out, int* max_bond) {
  return guard([&] {
    QTT_REQUIRE(ctx && out && terms && n_terms >= 1, "null argument");
    QTT_REQUIRE(ndims >= 1 && ndims <= 8 && bits >= 1 && bits <= 20, "bad grid");
    std::vector<host::TT> fh;
    for (int i = 0; i < n_fields; ++i) {
      check_tt(fields[i], ctx);
      fh.push_back(download(fields[i]));
    }
    host::TT A = build_mpo_host(ndims, bits, ordering, terms, n_terms, fh, field_ndims, rel_tol);
    auto caps = exact_caps(A);
    if (max_bond) *max_bond = *std::max_element(caps.begin(), caps.end());
    *out = upload(ctx, TT_MPO, A, caps).release();
  });
}

tt_status mps_apply_mpo(tt_ctx* ctx, const tt_tt* mpo, const tt_tt* x, int dtype, tt_tt** out) {
  return guard([&] {
    const Prec prec = prec_of(dtype);
    check_tt(mpo, ctx);
    check_tt(x, ctx);
    QTT_REQUIRE(out, "out is null");
    QTT_REQUIRE(mpo->kind == TT_MPO && x->kind == TT_MPS && mpo->N == x->N, "shape mismatch");
    const int N = x->N;
    std::vector<int> caps(N + 1);
    for (int n = 0; n <= N; ++n) caps[n] = x->caps[n] * mpo->caps[n];
    auto y = make_tt(ctx, TT_MPS, N, caps);
    std::vector<ApplyJob> jobs;
    int64_t maxe = 1;
    for (int n = 0; n < N; ++n) {
      ApplyJob j{mpo->core(n), x->core(n), y->core(n), x->caps[n], x->caps[n + 1], mpo->caps[n],
                 mpo->caps[n + 1]};
      jobs.push_back(j);
      maxe = std::max<int64_t>(maxe, (int64_t)caps[n] * 2 * caps[n + 1]);
    }
    StreamScope sc(ctx);
    for (const ApplyJob& j : jobs) validate(j);
    DevBuf dj(jobs.size() * sizeof(ApplyJob));
    rt::copy(dj.p, jobs.data(), jobs.size() * sizeof(ApplyJob));
    apply_jobs(dj.as<ApplyJob>(), N, maxe, ctx->stream, prec);
    rt::sync(ctx->stream);
    *out = y.release();
  });
}

tt_status mps_axpby(tt_ctx* ctx, int n_terms, const double* coeffs, const tt_tt* const* xs,
                    tt_tt** out) {
  return guard([&] {
    QTT_REQUIRE(ctx && coeffs && xs && out && n_terms >= 1, "null argument");
    const int N = xs[0]->N;
    std::vector<int> caps(N + 1, 0);
    std::vector<std::pair<double, ChainView>> terms;
    for (int j = 0; j < n_terms; ++j) {
      check_tt(xs[j], ctx);
      QTT_REQUIRE(xs[j]->kind == TT_MPS && xs[j]->N == N, "axpby: operands differ");
      for (int n = 0; n <= N; ++n) caps[n] += xs[j]->caps[n];
      terms.emplace_back(coeffs[j], view(xs[j]));
    }
    caps[0] = caps[N] = 1;
    auto y = make_tt(ctx, TT_MPS, N, caps);
    Plan plan;
    plan_axpby(plan, terms, y.get());
    StreamScope sc(ctx);
    plan.run(ctx->stream);
    rt::sync(ctx->stream);
    *out = y.release();
  });
}

tt_status mps_round(tt_ctx* ctx, const tt_tt* x, int chi, double rel_tol, tt_round_info* info, tt_tt** out) {
  return guard([&] {
    check_tt(x, ctx);
    QTT_REQUIRE(out && chi >= 1 && x->kind == TT_MPS, "bad argument");
    QTT_REQUIRE(rel_tol >= 0.0 && rel_tol < 1.0, "rel_tol %g outside [0, 1)", rel_tol);
    auto y = make_tt(ctx, TT_MPS, x->N, chain_caps(x->N, chi));
    Plan plan;
    RoundTarget tg;
    for (int n = 0; n < x->N; ++n) tg.core.push_back(y->core(n));
    tg.caps = y->caps;
    tg.rel_tol = rel_tol;
    plan_round_det(plan, view(x), tg);
    StreamScope sc(ctx);
    plan.run(ctx->stream);
    rt::sync(ctx->stream);
    if (info) {
      const RoundOutcome o = round_outcome(tg, ctx->stream);
      info->max_bond = *std::max_element(o.kept.begin(), o.kept.end());
      info->discarded_weight = 0.0;
      for (double d : o.discarded) info->discarded_weight += d;
      info->norm2 = o.norm2;
      if (info->per_bond)
        for (int n = 0; n <= x->N; ++n) info->per_bond[n] = o.discarded[n];
    }
    *out = y.release();
  });
}

}  // extern "C"

// Rounding of sum_j coeffs[j] W_j x_j by the one-sided (no left sketch) or
// two-sided randomized range finder, then the bond truncation.
static void round_sketch_common(tt_ctx* ctx, int n_terms, const double* coeffs,
                                const tt_tt* const* mpos, const tt_tt* const* xs,
                                const tt_tt* sketch, const tt_tt* sketch_left, int chi, int dtype,
                                tt_tt** out) {
  QTT_REQUIRE(ctx && coeffs && xs && out && n_terms >= 1 && chi >= 1, "null argument");
  check_tt(sketch, ctx);
  const int N = sketch->N;
  QTT_REQUIRE(sketch->kind == TT_MPS, "sketch must be an MPS");
  if (sketch_left) {
    check_tt(sketch_left, ctx);
    QTT_REQUIRE(sketch_left->N == N && sketch_left->kind == TT_MPS && sketch_left->caps == sketch->caps,
                "left sketch must have the sketch's length and ranks");
  }
  std::vector<ChainView> mv(n_terms);
  std::vector<SketchTerm> terms;
  for (int j = 0; j < n_terms; ++j) {
    check_tt(xs[j], ctx);
    QTT_REQUIRE(xs[j]->N == N && xs[j]->kind == TT_MPS, "term %d shape", j);
    SketchTerm t;
    t.coef = coeffs[j];
    t.x = view(xs[j]);
    if (mpos && mpos[j]) {
      check_tt(mpos[j], ctx);
      QTT_REQUIRE(mpos[j]->N == N && mpos[j]->kind == TT_MPO, "operator %d shape", j);
      mv[j] = view(mpos[j]);
      t.mpo = &mv[j];
    }
    terms.push_back(t);
  }
  auto y = make_tt(ctx, TT_MPS, N, chain_caps(N, chi));
  Plan plan;
  RoundTarget tg;
  for (int n = 0; n < N; ++n) tg.core.push_back(y->core(n));
  tg.caps = y->caps;
  if (sketch_left)
    plan_round_sketch_two_sided(plan, terms, view(sketch), view(sketch_left), tg, prec_of(dtype));
  else
    plan_round_sketch(plan, terms, view(sketch), tg, prec_of(dtype));
  StreamScope sc(ctx);
  plan.run(ctx->stream);
  rt::sync(ctx->stream);
  *out = y.release();
}

extern "C" {

tt_status mps_round_sketch(tt_ctx* ctx, int n_terms, const double* coeffs,
                           const tt_tt* const* mpos, const tt_tt* const* xs, const tt_tt* sketch,
                           int chi, int dtype, tt_tt** out) {
  return guard([&] {
    round_sketch_common(ctx, n_terms, coeffs, mpos, xs, sketch, nullptr, chi, dtype, out);
  });
}

tt_status mps_round_sketch_two_sided(tt_ctx* ctx, int n_terms, const double* coeffs,
                                     const tt_tt* const* mpos, const tt_tt* const* xs,
                                     const tt_tt* sketch, const tt_tt* sketch_left, int chi,
                                     int dtype, tt_tt** out) {
  return guard([&] {
    QTT_REQUIRE(sketch_left, "null left sketch");
    round_sketch_common(ctx, n_terms, coeffs, mpos, xs, sketch, sketch_left, chi, dtype, out);
  });
}

tt_status tt_l2_diff(tt_ctx* ctx, const tt_tt* a, const tt_tt* b, double* rel_err) {
  return guard([&] {
    check_tt(a, ctx);
    check_tt(b, ctx);
    QTT_REQUIRE(rel_err && a->N == b->N, "bad argument");
    const int N = a->N;
    std::vector<int> caps(N + 1);
    for (int n = 0; n <= N; ++n) caps[n] = a->caps[n] + b->caps[n];
    caps[0] = caps[N] = 1;
    auto d = make_tt(ctx, TT_MPS, N, caps);
    Plan plan;
    plan_axpby(plan, {{1.0, view(a)}, {-1.0, view(b)}}, d.get());
    LeftOrth ld = plan_left_orth(plan, view(d.get()));
    LeftOrth lb = plan_left_orth(plan, view(b));
    StreamScope sc(ctx);
    plan.run(ctx->stream);
    rt::sync(ctx->stream);
    auto nrm = [&](const LeftOrth& lo) {
      int n = lo.caps[N - 1] * 2;
      std::vector<double> h(n);
      rt::copy(h.data(), lo.core[N - 1], n * sizeof(double));
      double s = 0;
      for (double v : h) s += v * v;
      return std::sqrt(s);
    };
    double nd = nrm(ld), nb = nrm(lb);
    *rel_err = (nb > 0) ? nd / nb : nd;
  });
}

tt_status tt_inner(tt_ctx* ctx, const tt_tt* a, const tt_tt* b, double* out) {
  return guard([&] {
    check_tt(a, ctx);
    check_tt(b, ctx);
    QTT_REQUIRE(out && a->N == b->N, "bad argument");
    Plan plan;
    double* r = plan.alloc(1);
    plan_inner(plan, view(a), view(b), r);
    StreamScope sc(ctx);
    plan.run(ctx->stream);
    rt::copy_async(out, r, sizeof(double), ctx->stream);
    rt::sync(ctx->stream);
  });
}

tt_status tt_inner_noalloc(tt_ctx* ctx, const tt_tt* a, const tt_tt* b, double* out_dev) {
  return guard([&] {
    check_tt(a, ctx);
    check_tt(b, ctx);
    QTT_REQUIRE(out_dev, "out_dev is null");
    QTT_REQUIRE(a->N == b->N && a->kind == TT_MPS && b->kind == TT_MPS, "inner of MPSs of equal length");
    double* base = scratch_of(ctx->device);
    QTT_REQUIRE(base, "no static scratch on device %d", ctx->device);
    CallerRange out(out_dev, sizeof(double), "tt_inner_noalloc output");
    Plan plan;
    plan.arena = base;
    plan.arena_cap = kScratchDoubles;
    plan_inner(plan, view(a), view(b), out_dev);
    StreamScope sc(ctx);
    plan.run(ctx->stream);
  });
}

// ---------------------------------------------------------------------------
// problem
// ---------------------------------------------------------------------------
tt_status tt_problem_create(tt_ctx* ctx, const tt_params* pp, const tt_tt* const* velocity,
                            const tt_tt* sketch, const tt_tt* sketch_left, const tt_tt* sketch_mean,
                            const tt_tt* sketch_mean_left, tt_problem** out) {
  return tt_problem_create_flow(ctx, pp, velocity, nullptr, nullptr, sketch, sketch_left,
                                sketch_mean, sketch_mean_left, out);
}

tt_status tt_problem_create_flow(tt_ctx* ctx, const tt_params* pp, const tt_tt* const* velocity,
                                 const tt_tt* diffusivity, const tt_tt* mixing,
                                 const tt_tt* sketch, const tt_tt* sketch_left,
                                 const tt_tt* sketch_mean, const tt_tt* sketch_mean_left,
                                 tt_problem** out) {
  return guard([&] {
    QTT_REQUIRE(ctx && pp && out, "null argument");
    const tt_params& p = *pp;
    QTT_REQUIRE(p.ndims == 2 || p.ndims == 5, "ndims must be 2 or 5");
    QTT_REQUIRE(p.bits >= 1 && p.bits <= 16, "bits out of range");
    QTT_REQUIRE(p.ordering == TT_SERIAL || (p.ordering == TT_INTERLEAVED && p.ndims == 2),
                "interleaved ordering is supported for 2-D problems only");
    QTT_REQUIRE(p.chi >= 1 && p.ell >= p.chi, "need ell >= chi >= 1");
    QTT_REQUIRE(p.integrator == TT_RK4 || p.integrator == TT_RK2_HEUN, "bad integrator");
    (void)prec_of(p.dtype);
    auto P = std::make_unique<tt_problem>();
    P->ctx = ctx;
    P->p = p;
    const int N = p.ndims * p.bits;
    P->N = N;
    P->nphi = 2 * p.bits;
    P->nx = N - P->nphi;
    if (P->nx > 0) {
      QTT_REQUIRE(velocity && velocity[0] && velocity[1] && velocity[2], "5-D problem needs velocity");
      QTT_REQUIRE(sketch_mean && sketch_mean_left, "5-D problem needs the two mean-field sketches");
      QTT_REQUIRE(p.chi_mean >= 1 && p.ell_mean >= p.chi_mean, "need ell_mean >= chi_mean >= 1");
    }
    check_tt(sketch, ctx);
    QTT_REQUIRE(sketch->N == N && sketch->kind == TT_MPS, "sketch length");
    auto ell = chain_caps(N, p.ell);
    QTT_REQUIRE(sketch->caps == ell, "sketch ranks must be min(ell, 2^n, 2^(N-n))");
    P->fcaps = chain_caps(N, p.chi);
    check_tt(sketch_left, ctx);
    QTT_REQUIRE(sketch_left->N == N && sketch_left->kind == TT_MPS && sketch_left->caps == ell,
                "the left sketch must have the ranks of the sketch");
    // copies of the sketches
    {
      P->Z = make_tt(ctx, TT_MPS, N, ell);
      rt::copy(P->Z->buf.p, sketch->buf.p, sketch->total() * sizeof(double));
      P->Zl = make_tt(ctx, TT_MPS, N, ell);
      rt::copy(P->Zl->buf.p, sketch_left->buf.p, sketch_left->total() * sizeof(double));
    }
    if (P->nx > 0) {
      check_tt(sketch_mean, ctx);
      auto ellm = chain_caps(P->nx, p.ell_mean);
      QTT_REQUIRE(sketch_mean->N == P->nx && sketch_mean->caps == ellm, "mean-field sketch shape");
      P->Zm = make_tt(ctx, TT_MPS, P->nx, ellm);
      rt::copy(P->Zm->buf.p, sketch_mean->buf.p, sketch_mean->total() * sizeof(double));
      check_tt(sketch_mean_left, ctx);
      QTT_REQUIRE(sketch_mean_left->N == P->nx && sketch_mean_left->caps == ellm, "left mean-field sketch shape");
      P->Zml = make_tt(ctx, TT_MPS, P->nx, ellm);
      rt::copy(P->Zml->buf.p, sketch_mean_left->buf.p, sketch_mean_left->total() * sizeof(double));
      P->mcaps = chain_caps(P->nx, p.chi_mean);
    }
    // ---- fixed operator (eq. FP2): drift, dissipation, reaction, convection, diffusion
    std::vector<tt_term> terms;
    auto term = [&](double c, std::vector<std::pair<int, int>> ops, int field) {
      tt_term t{};
      t.coeff = c;
      for (int d = 0; d < 8; ++d) t.op[d] = TT_OP_ID;
      for (auto [d, op] : ops) t.op[d] = op;
      t.field = field;
      terms.push_back(t);
    };
    // flow-case x-fields (fields 3: G, 4..6: D1p_i G, 7: Omega)
    std::vector<host::TT> fields;
    if (diffusivity || mixing) QTT_REQUIRE(P->nx > 0, "x-fields need a 5-D problem");
    if (P->nx > 0) {
      for (int i = 0; i < 3; ++i) {
        check_tt(velocity[i], ctx);
        QTT_REQUIRE(velocity[i]->N == P->nx, "velocity component %d length", i);
        fields.push_back(download(velocity[i]));
      }
      auto x_order = host::site_order(3, p.bits, TT_SERIAL);
      host::TT Gh, Omh;
      if (diffusivity) {
        check_tt(diffusivity, ctx);
        QTT_REQUIRE(diffusivity->N == P->nx && diffusivity->kind == TT_MPS, "diffusivity field shape");
        Gh = host::round_svd(download(diffusivity), 1e-14, 1 << 30);  // drops the zero padding
      }
      if (mixing) {
        check_tt(mixing, ctx);
        QTT_REQUIRE(mixing->N == P->nx && mixing->kind == TT_MPS, "mixing field shape");
        Omh = host::round_svd(download(mixing), 1e-14, 1 << 30);
      }
      fields.push_back(Gh);
      host::TT d1p = host::op1d(TT_OP_D1P, p.bits);
      for (int i = 0; i < 3; ++i) {
        host::TT dG;
        if (diffusivity) {
          std::vector<const host::TT*> per(3, nullptr);
          per[i] = &d1p;
          dG = host::mpo_apply(host::kron_dims(per, x_order, 3, 4), Gh);
        }
        fields.push_back(dG);
      }
      fields.push_back(Omh);
      P->has_G = diffusivity != nullptr;
      P->has_Om = mixing != nullptr;
      if (P->has_Om) {
        host::TT W = host::mpo_diag(Omh);
        P->Wom = upload(ctx, TT_MPO, W, exact_caps(W));
        P->Womv = view(P->Wom.get());
      }
    }
    for (int a = 0; a < 2; ++a) {
      if (P->has_Om) term(1.0, {{a, TT_OP_D1G_PHI}}, 7);
      else term(p.omega, {{a, TT_OP_D1G_PHI}}, -1);
      term(p.nu_phi, {{a, TT_OP_D2G}}, -1);
      if (p.k_react != 0.0) term(p.k_react, {{a, TT_OP_D1G_PHI}, {1 - a, TT_OP_PHI}}, -1);
    }
    if (P->nx > 0) {
      for (int i = 0; i < 3; ++i) {
        if (P->has_G) {
          term(1.0, {{2 + i, TT_OP_D2P}}, 3);
          term(1.0, {{2 + i, TT_OP_D1P}}, 4 + i);
        } else if (p.gamma != 0.0) {
          term(p.gamma, {{2 + i, TT_OP_D2P}}, -1);
        }
        term(-1.0, {{2 + i, TT_OP_D1P}}, i);
      }
    }
    host::TT Fx = build_mpo_host(p.ndims, p.bits, p.ordering, terms.data(), (int)terms.size(),
                                 fields, 3, 1e-13);
    // ---- mean-field part  -Omega sum_a D1g^(a) diag(<Phi_a>)
    auto order = host::site_order(p.ndims, p.bits, p.ordering);
    std::vector<std::pair<int, int>> phi_order(order.begin(), order.begin() + P->nphi);
    host::TT d1g = host::op1d(TT_OP_D1G, p.bits);
    host::TT T[2];
    for (int a = 0; a < 2; ++a) {
      std::vector<const host::TT*> pp2(2, nullptr);
      pp2[a] = &d1g;
      T[a] = host::kron_dims(pp2, phi_order, 2, 4);
    }
    // stacked mean-field chain over the phi sites (right bond 2 = channel a for 5-D)
    host::TT MF;
    std::vector<int> Dmf(N + 1, 1);
    {
      const int nphi = P->nphi;
      for (int n = 0; n < nphi; ++n) {
        const host::Core &A0 = T[0][n], &A1 = T[1][n];
        int rl = (n == 0) ? 1 : A0.rl + A1.rl;
        int rr = (n == nphi - 1) ? ((P->nx > 0) ? 2 : 1) : A0.rr + A1.rr;
        host::Core G(rl, 4, rr);
        for (int a = 0; a < 2; ++a) {
          const host::Core& B = T[a][n];
          int ro = (n == 0) ? 0 : (a == 0 ? 0 : A0.rl);
          int co;
          if (n == nphi - 1) co = (P->nx > 0) ? a : 0;
          else co = (a == 0) ? 0 : A0.rr;
          for (int i = 0; i < B.rl; ++i)
            for (int s = 0; s < 4; ++s)
              for (int j = 0; j < B.rr; ++j) G.at(ro + i, s, co + j) += B.at(i, s, j);
        }
        MF.push_back(std::move(G));
      }
      for (int n = 0; n < nphi; ++n) Dmf[n + 1] = MF[n].rr;
      Dmf[0] = 1;
      for (int j = 1; j < P->nx; ++j) Dmf[nphi + j] = 2 * P->mcaps[j];
      Dmf[N] = 1;
    }
    P->MFh = MF;
    P->Dmf = Dmf;
    // 5-D: the mean-field block carries -Omega in its first core; 2-D: the
    // first-core blocks are rescaled by -Omega <Phi_a> at every stage
    P->A = assemble_stage_mpo(P.get(), Fx, P->nx > 0 ? (P->has_Om ? -1.0 : -p.omega) : 1.0, P->Dfix);
    if (P->nx > 0) {
      // Hadamard form when the time its sketch contractions save over those
      // of the block sum (flops per x site of a sketch chain: dense MPO of
      // bond D, or diagonal cores of bond chi_mean; at the ~20 TFLOP/s these
      // launches reach) exceeds what its six extra launches per x site cost
      // (~10 us each).  Measured: the 1024^5 chi = 128 step with chi_mean =
      // 128 gains 1.4x; the 128^5 chi = 64 step with chi_mean <= 64 loses.
      const double r = p.chi, l = p.ell;
      auto dense = [&](double D) { return D * 2 * r * l * l + 4 * D * D * r * l + 2 * D * r * r * l; };
      auto diag = [&](double D) { return D * 2 * r * l * l + 2 * D * D * r * l + 2 * D * r * r * l; };
      int dfx = 1;
      for (int n = P->nphi; n <= N; ++n) dfx = std::max(dfx, P->Dfix[n]);
      const double cm = p.chi_mean;
      const char* e = std::getenv("QTTPDF_MEAN_FORM");
      if (e && std::strcmp(e, "split") == 0) P->split_mf = true;
      else if (e && std::strcmp(e, "block") == 0) P->split_mf = false;
      else P->split_mf = (dense(dfx + 2 * cm) - dense(dfx) - 2 * diag(cm)) / 2e13 > 6 * 1e-5;
      if (P->split_mf) {
        host::TT Fdt = Fx;
        for (double& v : Fdt[0].v) v *= p.dt;
        P->F = upload(ctx, TT_MPO, Fdt, exact_caps(Fdt));
        P->Fv = view(P->F.get());
        const double sc = (P->has_Om ? -1.0 : -p.omega) * p.dt;
        for (int a = 0; a < 2; ++a) {
          host::TT W = T[a];
          for (double& v : W[0].v) v *= sc;
          std::vector<int> caps(N + 1, 1);
          for (int n = 0; n < P->nphi; ++n) caps[n + 1] = W[n].rr;
          for (int j = 1; j < P->nx; ++j) caps[P->nphi + j] = P->mcaps[j];
          for (int j = 0; j < P->nx; ++j) W.push_back(host::Core(caps[P->nphi + j], 4, caps[P->nphi + j + 1]));
          P->MF[a] = upload(ctx, TT_MPO, W, caps);
          P->MFv[a] = view(P->MF[a].get());
        }
      }
    }
    if (P->nx == 0) {
      // first-core blocks of the two mean-field terms, kept unscaled
      P->mf_first_cols = {T[0][0].rr, T[1][0].rr};
      P->mf_first_off = {0, T[0][0].rr};
      P->mf_first_ld = std::max(T[0][0].rr, T[1][0].rr);
      std::vector<double> h((size_t)2 * 4 * P->mf_first_ld, 0.0);
      for (int a = 0; a < 2; ++a)
        for (int s = 0; s < 4; ++s)
          for (int j = 0; j < T[a][0].rr; ++j)
            h[(size_t)a * 4 * P->mf_first_ld + (size_t)s * T[a][0].rr + j] = T[a][0].at(0, s, j);
      P->mf_first.alloc(h.size() * sizeof(double));
      rt::copy(P->mf_first.p, h.data(), h.size() * sizeof(double));
    }
    // ---- mean-field weights: h phi_a on dimension a, h on the other (two channels)
    {
      const int M = 1 << p.bits;
      const double h = 1.0 / M;
      std::vector<double> wphi(M), wone(M, h);
      for (int i = 0; i < M; ++i) wphi[i] = h * (i + 0.5) * h;
      host::TT Wa[2];
      for (int a = 0; a < 2; ++a) {
        host::TT q0 = host::vector_qtt(a == 0 ? wphi.data() : wone.data(), p.bits);
        host::TT q1 = host::vector_qtt(a == 1 ? wphi.data() : wone.data(), p.bits);
        Wa[a] = host::kron_dims({&q0, &q1}, phi_order, 2, 2);
      }
      const int nphi = P->nphi;
      host::TT W;
      for (int n = 0; n < nphi; ++n) {
        const host::Core &A0 = Wa[0][n], &A1 = Wa[1][n];
        int rl = (n == 0) ? 1 : A0.rl + A1.rl;
        int rr = (n == nphi - 1) ? 2 : A0.rr + A1.rr;
        host::Core G(rl, 2, rr);
        for (int a = 0; a < 2; ++a) {
          const host::Core& B = Wa[a][n];
          int ro = (n == 0) ? 0 : (a == 0 ? 0 : A0.rl);
          int co = (n == nphi - 1) ? a : (a == 0 ? 0 : A0.rr);
          for (int i = 0; i < B.rl; ++i)
            for (int s = 0; s < 2; ++s)
              for (int j = 0; j < B.rr; ++j) G.at(ro + i, s, co + j) += B.at(i, s, j);
        }
        W.push_back(std::move(G));
      }
      std::vector<int> wc(nphi + 1, 1);
      for (int n = 0; n < nphi; ++n) wc[n + 1] = W[n].rr;
      // a chain container needs boundary bonds 1: store the channel bond as the
      // last capacity through a raw view (planner reads caps from the view)
      auto t = std::make_unique<tt_tt>();
      t->ctx = ctx;
      t->kind = TT_MPS;
      t->N = nphi;
      t->p = 2;
      t->caps = wc;
      t->off.assign(nphi + 1, 0);
      for (int n = 0; n < nphi; ++n) t->off[n + 1] = t->off[n] + (int64_t)wc[n] * 2 * wc[n + 1];
      t->buf.alloc((size_t)t->off[nphi] * sizeof(double));
      std::vector<double> hv(t->off[nphi], 0.0);
      for (int n = 0; n < nphi; ++n) std::copy(W[n].v.begin(), W[n].v.end(), hv.begin() + t->off[n]);
      rt::copy(t->buf.p, hv.data(), hv.size() * sizeof(double));
      P->Wm = std::move(t);
    }
    // ---- per-step buffers
    const int S = (p.integrator == TT_RK4) ? 4 : 2;
    for (int i = 0; i < S; ++i) P->k[i] = make_tt(ctx, TT_MPS, N, P->fcaps);
    P->cphi = P->fcaps[P->nphi];
    P->cphi1 = (P->nx > 0) ? P->fcaps[P->nphi + 1] : 1;
    P->Ef.alloc(sizeof(double) * 2 * P->cphi);
    P->Ek.alloc(sizeof(double) * 2 * P->cphi);
    P->mff.alloc(sizeof(double) * 2 * 2 * P->cphi1);
    P->mfk.alloc(sizeof(double) * 2 * 2 * P->cphi1);
    P->scal.alloc(sizeof(double) * 4);
    P->nonfinite.alloc(sizeof(int));
    {
      const int zero = 0;
      rt::copy(P->nonfinite.p, &zero, sizeof(int));
    }
    if (P->nx > 0)
      for (int a = 0; a < 2; ++a) P->mt[a] = make_tt(ctx, TT_MPS, P->nx, P->mcaps);
    rt::sync(ctx->stream);
    *out = P.release();
  });
}

tt_status tt_problem_destroy(tt_problem* prob) {
  return guard([&] {
    if (!prob) return;
    if (!rt::dry()) (void)hipDeviceSynchronize();
    delete prob;
  });
}

tt_status tt_problem_info(const tt_problem* prob, int* n_sites, int32_t* mpo_bonds, int* max_mpo_bond) {
  return guard([&] {
    QTT_REQUIRE(prob, "null problem");
    if (n_sites) *n_sites = prob->N;
    if (mpo_bonds)
      for (int n = 0; n <= prob->N; ++n) mpo_bonds[n] = prob->Dfix[n];
    if (max_mpo_bond) *max_mpo_bond = *std::max_element(prob->Dfix.begin(), prob->Dfix.end());
  });
}

tt_status tt_problem_state(tt_problem* prob, tt_tt** f) {
  return guard([&] {
    QTT_REQUIRE(prob && f, "null argument");
    auto t = make_tt(prob->ctx, TT_MPS, prob->N, prob->fcaps);
    StreamScope sc(prob->ctx);
    fill(t->buf.d(), t->total(), 0.0, prob->ctx->stream);
    *f = t.release();
  });
}

}  // extern "C"

// The step plan of (problem, state), recorded on first use, and with graphs
// enabled captured once from the context's stream as a HIP graph.
static void ensure_step_graph(tt_problem* prob, tt_tt* f) {
  if (!prob->plan || prob->plan_f != f) build_step_plan(prob, f);
  if (rt::dry() || !use_graph() || prob->exec) return;
  StreamScope sc(prob->ctx);
  hipStream_t s = prob->ctx->stream;
  QTT_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  try {
    prob->plan->run(s);
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(s, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  QTT_HIP(hipStreamEndCapture(s, &prob->graph));
  QTT_HIP(hipGraphInstantiate(&prob->exec, prob->graph, nullptr, nullptr, 0));
}

// reads and clears the problem's non-finite flag (synchronous); throws
// TT_ERR_NONFINITE if it was set
static void take_nonfinite(tt_problem* P, const char* where) {
  int h = 0;
  rt::sync(P->ctx->stream);
  rt::copy(&h, P->nonfinite.p, sizeof(int));
  if (h) {
    const int zero = 0;
    rt::copy(P->nonfinite.p, &zero, sizeof(int));
    QTT_THROW(TT_ERR_NONFINITE, "NaN or Inf in the result of %s", where);
  }
}

// weight chain of h^d sum_x,phi w1(phi1) w2(phi2) f (NULL: all ones)
static host::TT weight_chain(const tt_params& p, const std::vector<double>* w1, const std::vector<double>* w2) {
  const int M = 1 << p.bits;
  const double h = 1.0 / M;
  auto order = host::site_order(p.ndims, p.bits, p.ordering);
  std::vector<double> one(M, h);
  std::vector<host::TT> q(p.ndims);
  std::vector<const host::TT*> pp(p.ndims);
  for (int d = 0; d < p.ndims; ++d) {
    const std::vector<double>* v = (d == 0 && w1) ? w1 : (d == 1 && w2) ? w2 : &one;
    q[d] = host::vector_qtt(v->data(), p.bits);
    pp[d] = &q[d];
  }
  return host::kron_dims(pp, order, p.ndims, 2);
}

// one step of a problem whose plan (and graph) exist, on stream s
static void launch_step(tt_problem* prob, hipStream_t s) {
  prob->last = prob->last_plain;
  if (rt::dry() || !use_graph()) prob->plan->run(s);
  else QTT_HIP(hipGraphLaunch(prob->exec, s));
}

extern "C" {

tt_status tt_step(tt_ctx* ctx, tt_problem* prob, tt_tt* f, int n_steps) {
  return guard([&] {
    QTT_REQUIRE(prob && f && n_steps >= 0, "bad argument");
    check_tt(f, ctx);
    QTT_REQUIRE(prob->ctx == ctx, "problem belongs to another context");
    QTT_REQUIRE(f->caps == prob->fcaps, "state caps differ from the problem's");
    if (n_steps == 0) return;
    ensure_step_graph(prob, f);
    StreamScope sc(ctx);
    for (int i = 0; i < n_steps; ++i) launch_step(prob, ctx->stream);
  });
}

tt_status tt_step_ex(tt_ctx* ctx, tt_problem* prob, tt_tt* f, int n_steps, tt_step_record* records) {
  return guard([&] {
    QTT_REQUIRE(prob && f && n_steps >= 0, "bad argument");
    check_tt(f, ctx);
    QTT_REQUIRE(prob->ctx == ctx, "problem belongs to another context");
    QTT_REQUIRE(f->caps == prob->fcaps, "state caps differ from the problem's");
    if (n_steps == 0) return;
    ensure_step_graph(prob, f);
    host::TT w = weight_chain(prob->p, nullptr, nullptr);
    auto wt = upload(ctx, TT_MPS, w, exact_caps(w));
    Plan mp;
    double* mass = mp.alloc(1);
    plan_inner(mp, view(wt.get()), view(f), mass);
    StreamScope sc(ctx);
    for (int i = 0; i < n_steps; ++i) {
      launch_step(prob, ctx->stream);
      mp.run(ctx->stream);
      const RoundOutcome o = round_outcome(prob->last, ctx->stream);
      double m = 0.0;
      int bad = 0;
      rt::copy(&m, mass, sizeof(double));
      rt::copy(&bad, prob->nonfinite.p, sizeof(int));
      if (records) {
        tt_step_record& r = records[i];
        r.mass_dev = m - 1.0;
        r.discarded_weight = 0.0;
        for (double d : o.discarded) r.discarded_weight += d;
        r.max_bond = *std::max_element(o.kept.begin(), o.kept.end());
        r.nonfinite = bad ? 1 : 0;
      }
      if (bad) take_nonfinite(prob, "a rounding of this step");
    }
  });
}

// ---------------------------------------------------------------------------
// batching
// ---------------------------------------------------------------------------
}  // extern "C"

// parallel branches of a batched step: QTTPDF_BATCH_BRANCHES, default 8
static int batch_branches() {
  const char* e = std::getenv("QTTPDF_BATCH_BRANCHES");
  const int v = e ? std::atoi(e) : 0;
  return v >= 1 ? v : 8;
}

// fusing instances of the same structure into shared launches:
// QTTPDF_BATCH_FUSE=0 turns it off
static bool batch_fuse() {
  const char* e = std::getenv("QTTPDF_BATCH_FUSE");
  return !(e && e[0] == '0');
}

namespace qtt {

// device buffers of a problem that its plain step reads or writes, in a
// fixed order: (pointer, bytes); absent members are (null, 0)
static std::vector<std::pair<void*, size_t>> step_buffers(const tt_problem* P) {
  std::vector<std::pair<void*, size_t>> v;
  auto t = [&](const std::unique_ptr<tt_tt>& x) {
    v.push_back(x ? std::make_pair(x->buf.p, x->buf.bytes) : std::make_pair((void*)nullptr, (size_t)0));
  };
  auto d = [&](const DevBuf& b) { v.push_back({b.p, b.bytes}); };
  t(P->Z), t(P->Zl), t(P->Zm), t(P->Zml), t(P->A), t(P->Wm), t(P->Wom), t(P->F), t(P->MF[0]), t(P->MF[1]);
  for (int i = 0; i < 4; ++i) t(P->k[i]);
  t(P->mt[0]), t(P->mt[1]);
  d(P->mf_first), d(P->Ef), d(P->Ek), d(P->mff), d(P->mfk), d(P->scal), d(P->nonfinite);
  return v;
}

// a chain with the shape of t and fresh (uninitialised) storage
static std::unique_ptr<tt_tt> clone_shape(const tt_tt* t) {
  if (!t) return nullptr;
  auto c = std::make_unique<tt_tt>();
  c->ctx = t->ctx;
  c->kind = t->kind;
  c->N = t->N;
  c->p = t->p;
  c->caps = t->caps;
  c->off = t->off;
  c->buf.alloc(t->buf.bytes);
  return c;
}

// a problem with P's structure and fresh buffers for its plain step (the
// contents are copied in afterwards), allocated in a fixed order
static std::unique_ptr<tt_problem> clone_problem(const tt_problem* P) {
  auto C = std::make_unique<tt_problem>();
  C->ctx = P->ctx;
  C->p = P->p;
  C->N = P->N;
  C->nphi = P->nphi;
  C->nx = P->nx;
  C->fcaps = P->fcaps;
  C->mcaps = P->mcaps;
  C->Dfix = P->Dfix;
  C->has_G = P->has_G;
  C->has_Om = P->has_Om;
  C->mf_first_off = P->mf_first_off;
  C->mf_first_cols = P->mf_first_cols;
  C->mf_first_ld = P->mf_first_ld;
  C->split_mf = P->split_mf;
  C->cphi = P->cphi;
  C->cphi1 = P->cphi1;
  C->MFh = P->MFh;
  C->Dmf = P->Dmf;
  C->Z = clone_shape(P->Z.get());
  C->Zl = clone_shape(P->Zl.get());
  C->Zm = clone_shape(P->Zm.get());
  C->Zml = clone_shape(P->Zml.get());
  C->A = clone_shape(P->A.get());
  C->Wm = clone_shape(P->Wm.get());
  C->Wom = clone_shape(P->Wom.get());
  C->F = clone_shape(P->F.get());
  for (int a = 0; a < 2; ++a) C->MF[a] = clone_shape(P->MF[a].get());
  for (int i = 0; i < 4; ++i) C->k[i] = clone_shape(P->k[i].get());
  for (int a = 0; a < 2; ++a) C->mt[a] = clone_shape(P->mt[a].get());
  auto cl = [](DevBuf& dst, const DevBuf& src) {
    if (src.p) dst.alloc(src.bytes);
  };
  cl(C->mf_first, P->mf_first), cl(C->Ef, P->Ef), cl(C->Ek, P->Ek), cl(C->mff, P->mff), cl(C->mfk, P->mfk);
  cl(C->scal, P->scal), cl(C->nonfinite, P->nonfinite);
  if (C->Wom) C->Womv = view(C->Wom.get());
  if (C->F) C->Fv = view(C->F.get());
  for (int a = 0; a < 2; ++a)
    if (C->MF[a]) C->MFv[a] = view(C->MF[a].get());
  return C;
}

// Instances whose recorded steps are the same launches on different data:
// equal structure (grid, caps, operator bonds, forms, precision, scheme).
// The coefficients live in the data (the stage operators carry dt), so
// problems that differ in them share a key.
static std::string structure_key(const tt_problem* P) {
  std::string k;
  auto add = [&](long v) { k += std::to_string(v) + ","; };
  auto vec = [&](const std::vector<int>& v) {
    add((long)v.size());
    for (int x : v) add(x);
    k += ";";
  };
  const tt_params& p = P->p;
  add(p.ndims), add(p.bits), add(p.ordering), add(p.chi), add(p.ell), add(p.chi_mean), add(p.ell_mean);
  add(p.integrator), add(p.dtype), add(P->split_mf), add(P->has_G), add(P->has_Om);
  vec(P->fcaps), vec(P->mcaps), vec(P->Dfix);
  for (const auto& [ptr, bytes] : step_buffers(P)) add(ptr ? (long)bytes : -1L);
  for (const tt_tt* t : {P->A.get(), P->F.get(), P->MF[0].get(), P->MF[1].get(), P->Wom.get(), P->Wm.get()})
    if (t) vec(t->caps);
  return k;
}

}  // namespace qtt

// Instances of one structure stepped by shared launches: every instance's
// buffers lie at the same offsets in its slab (slab i at slab + i * stride);
// the step is recorded once, for slab 0, and every launch of it runs for all
// the instances (rt::Fuse).
struct FusedClass {
  std::vector<int> members;  // instance indices
  DevBuf slab;
  char* base = nullptr;      // slab 0, 256-byte aligned
  int64_t stride = 0;        // bytes
  std::unique_ptr<tt_problem> P0;
  std::unique_ptr<tt_tt> f0;
  std::unique_ptr<Plan> plan;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  FusedClass() = default;
  FusedClass(const FusedClass&) = delete;
  FusedClass& operator=(const FusedClass&) = delete;
  ~FusedClass() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    plan.reset();  // before the slab they live in
    f0.reset();
    P0.reset();
  }
  rt::Fuse fuse() const {
    rt::Fuse f;
    f.n = (int)members.size();
    f.stride = stride;
    f.lo = (uintptr_t)base;
    f.hi = (uintptr_t)base + (uintptr_t)stride;
    return f;
  }
};

// sets this thread's fused-launch setting for a scope
struct FuseScope {
  explicit FuseScope(const rt::Fuse& f) { rt::fuse() = f; }
  ~FuseScope() { rt::fuse() = rt::Fuse{}; }
};

struct tt_batch {
  tt_ctx* ctx = nullptr;
  std::vector<tt_problem*> probs;
  std::vector<tt_tt*> states;
  // units of work: a single instance (its own step graph) or a fused class
  struct Unit {
    int inst = -1;
    int cls = -1;
  };
  std::vector<Unit> units;
  std::vector<std::unique_ptr<FusedClass>> classes;
  std::vector<std::vector<int>> chain;  // units of each branch, in order
  std::vector<hipStream_t> streams;     // one per branch
  std::vector<hipEvent_t> events;       // fork + one join per branch
  ~tt_batch() {
    for (auto e : events) (void)hipEventDestroy(e);
    for (auto st : streams) (void)hipStreamDestroy(st);
  }
};

namespace qtt {

// Records and captures the fused step of the instances `members` (equal
// structure keys): the slab stride is measured by recording once with
// ordinary allocations, then the clone of the first instance is built in
// slab 0 and recorded again (the contraction shapes are tuned by then, so
// the second recording allocates the same sequence), and every instance's
// inputs are copied to its slab.
static std::unique_ptr<FusedClass> build_fused_class(tt_batch* b, const std::vector<int>& members) {
  auto C = std::make_unique<FusedClass>();
  C->members = members;
  const tt_problem* P = b->probs[members[0]];
  const tt_tt* f = b->states[members[0]];
  size_t bytes = 0;
  {
    rt::alloc_count_reset();
    auto Pc = clone_problem(P);
    auto fc = clone_shape(f);
    auto plan = record_step(Pc.get(), fc.get(), {});
    bytes = rt::alloc_count();
  }
  const size_t align = size_t(1) << 16;
  C->stride = (int64_t)((bytes + align - 1) / align * align);
  C->slab.alloc((size_t)C->stride * members.size() + 256);
  C->base = reinterpret_cast<char*>(((uintptr_t)C->slab.p + 255) & ~uintptr_t(255));
  {
    rt::SlabScope scope(C->base, (size_t)C->stride);
    C->P0 = clone_problem(P);
    C->f0 = clone_shape(f);
    C->plan = record_step(C->P0.get(), C->f0.get(), {});
  }
  // what the recording wrote into slab 0 (tables, and constants such as the
  // ones of the mean-field chains, which fused launches read per instance)
  for (const auto& [ptr, n] : C->plan->uploads)
    for (size_t i = 1; i < members.size(); ++i) rt::copy(ishift(ptr, (int64_t)i * C->stride), ptr, n);
  const auto dst0 = step_buffers(C->P0.get());
  for (size_t i = 0; i < members.size(); ++i) {
    const auto src = step_buffers(b->probs[members[i]]);
    QTT_REQUIRE(src.size() == dst0.size(), "fused batch: buffer lists differ");
    for (size_t j = 0; j < src.size(); ++j) {
      QTT_REQUIRE(src[j].second == dst0[j].second, "fused batch: instance %d buffer %zu differs in size",
                  members[i], j);
      if (src[j].first) rt::copy(ishift(dst0[j].first, (int64_t)i * C->stride), src[j].first, src[j].second);
    }
  }
  if (rt::dry() || !use_graph()) return C;
  StreamScope sc(b->ctx);
  hipStream_t s = b->ctx->stream;
  FuseScope fs(C->fuse());
  QTT_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  try {
    C->plan->run(s);
  } catch (...) {
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(s, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  QTT_HIP(hipStreamEndCapture(s, &C->graph));
  QTT_HIP(hipGraphInstantiate(&C->exec, C->graph, nullptr, nullptr, 0));
  return C;
}

// drops a problem's recorded plain step (plan, graph and their buffers)
static void release_step_plan(tt_problem* P) {
  if (P->exec) (void)hipGraphExecDestroy(P->exec);
  if (P->graph) (void)hipGraphDestroy(P->graph);
  P->exec = nullptr;
  P->graph = nullptr;
  if (P->plan) rt::sync(P->ctx->stream);
  P->plan.reset();
  P->plan_f = nullptr;
  P->last_plain = RoundTarget{};
  P->last = P->tplan ? P->last_tan : RoundTarget{};
}

// one step of a fused class on stream s
static void launch_fused(FusedClass& C, hipStream_t s) {
  if (C.exec) {
    QTT_HIP(hipGraphLaunch(C.exec, s));
  } else {
    FuseScope fs(C.fuse());
    C.plan->run(s);
  }
}

// the instances' states into (in) or out of their slabs
static void fused_states(tt_batch* b, bool in, hipStream_t s) {
  for (auto& C : b->classes) {
    const size_t bytes = (size_t)C->f0->total() * sizeof(double);
    for (size_t i = 0; i < C->members.size(); ++i) {
      double* slab_f = ishift(C->f0->buf.d(), (int64_t)i * C->stride);
      double* user_f = b->states[C->members[i]]->buf.d();
      if (in) rt::copy_async(slab_f, user_f, bytes, s);
      else rt::copy_async(user_f, slab_f, bytes, s);
    }
  }
}

}  // namespace qtt

extern "C" {

tt_status tt_batch_create(tt_ctx* ctx, int count, tt_problem* const* probs, tt_tt* const* states,
                          tt_batch** out) {
  return guard([&] {
    QTT_REQUIRE(ctx && out && probs && states && count >= 1, "bad argument");
    auto b = std::make_unique<tt_batch>();
    b->ctx = ctx;
    for (int i = 0; i < count; ++i) {
      tt_problem* P = probs[i];
      tt_tt* f = states[i];
      QTT_REQUIRE(P && f, "instance %d: null handle", i);
      QTT_REQUIRE(P->ctx == ctx, "instance %d: problem belongs to another context", i);
      check_tt(f, ctx);
      QTT_REQUIRE(f->caps == P->fcaps, "instance %d: state caps differ from the problem's", i);
      for (int j = 0; j < i; ++j)
        QTT_REQUIRE(probs[j] != P && states[j] != f, "instance %d repeats a problem or a state", i);
      b->probs.push_back(P);
      b->states.push_back(f);
    }
    // 5-D instances of equal structure form fused classes; the rest (and
    // classes of one) step with their own graphs, as tt_step records them
    std::map<std::string, std::vector<int>> groups;
    std::vector<std::string> key_order;
    for (int i = 0; i < count; ++i) {
      const bool fusable = batch_fuse() && b->probs[i]->nx > 0;
      const std::string k = fusable ? structure_key(b->probs[i]) : "single" + std::to_string(i);
      if (!groups.count(k)) key_order.push_back(k);
      groups[k].push_back(i);
    }
    std::vector<double> cost;
    auto inst_cost = [&](int i) {
      double c = 0.0;
      for (int x : b->probs[i]->fcaps) c += (double)x * x * x;
      return c;
    };
    for (const std::string& k : key_order) {
      const std::vector<int>& m = groups[k];
      tt_batch::Unit u;
      if (m.size() == 1) {
        u.inst = m[0];
        ensure_step_graph(b->probs[m[0]], b->states[m[0]]);
        cost.push_back(inst_cost(m[0]));
      } else {
        u.cls = (int)b->classes.size();
        b->classes.push_back(build_fused_class(b.get(), m));
        // the members' own step plans are not needed by the batch: their
        // memory goes back (tt_step records them again when called)
        for (int i : m) release_step_plan(b->probs[i]);
        // a fused launch runs the instances side by side: about one instance's time
        cost.push_back(inst_cost(m[0]) * (1.0 + 0.25 * (m.size() - 1)));
      }
      b->units.push_back(u);
    }
    // Units run on a few parallel branches (streams), each a chain of whole
    // steps; a unit joins the branch with the least estimated work so far,
    // largest first (work ~ sum of cap^3 over the bonds).
    const int nu = (int)b->units.size();
    const int nb = std::min(nu, batch_branches());
    std::vector<int> order(nu);
    for (int i = 0; i < nu; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    b->chain.assign(nb, {});
    std::vector<double> load(nb, 0.0);
    for (int i : order) {
      const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      b->chain[k].push_back(i);
      load[k] += cost[i];
    }
    if (!rt::dry()) {
      b->streams.resize(nb, nullptr);
      for (auto& st : b->streams) QTT_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
      b->events.resize(nb + 1, nullptr);
      for (auto& e : b->events) QTT_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    *out = b.release();
  });
}

tt_status tt_batch_info(const tt_batch* b, int* n_units, int* n_fused_classes, int* n_fused_instances,
                        int64_t* slab_bytes) {
  return guard([&] {
    QTT_REQUIRE(b, "null batch");
    int fi = 0;
    int64_t sb = 0;
    for (const auto& C : b->classes) {
      fi += (int)C->members.size();
      sb += C->stride * (int64_t)C->members.size();
    }
    if (n_units) *n_units = (int)b->units.size();
    if (n_fused_classes) *n_fused_classes = (int)b->classes.size();
    if (n_fused_instances) *n_fused_instances = fi;
    if (slab_bytes) *slab_bytes = sb;
  });
}

tt_status tt_step_batched(tt_batch* b, int n_steps) {
  return guard([&] {
    QTT_REQUIRE(b && n_steps >= 0, "bad argument");
    StreamScope sc(b->ctx);
    hipStream_t s0 = b->ctx->stream;
    // Submitting a recorded step graph costs host time per node; with
    // QTTPDF_BATCH_THREADS=1 every branch is submitted by a host thread of
    // its own, so the branches' submissions overlap.
    static const bool threaded = [] {
      const char* e = std::getenv("QTTPDF_BATCH_THREADS");
      return e && e[0] == '1';
    }();
    auto run_unit = [&](int u, hipStream_t s) {
      const tt_batch::Unit& un = b->units[u];
      if (un.cls >= 0) launch_fused(*b->classes[un.cls], s);
      else launch_step(b->probs[un.inst], s);
    };
    if (n_steps > 0) fused_states(b, true, s0);
    for (int step = 0; step < n_steps; ++step) {
      if (rt::dry()) {
        for (auto& ch : b->chain)
          for (int u : ch) run_unit(u, s0);
        continue;
      }
      // fork from the context's stream, one chain per branch, join back
      QTT_HIP(hipEventRecord(b->events[0], s0));
      const int nb = (int)b->chain.size();
      auto branch = [&](int k) {
        QTT_HIP(hipStreamWaitEvent(b->streams[k], b->events[0], 0));
        for (int u : b->chain[k]) run_unit(u, b->streams[k]);
        QTT_HIP(hipEventRecord(b->events[k + 1], b->streams[k]));
      };
      if (threaded && nb > 1) {
        std::vector<std::thread> th;
        std::vector<std::string> errs(nb);
        const int dev = b->ctx->device;
        for (int k = 0; k < nb; ++k)
          th.emplace_back([&, k] {
            try {
              QTT_HIP(hipSetDevice(dev));
              branch(k);
            } catch (const Error& e) {
              errs[k] = e.msg;
            }
          });
        for (auto& t : th) t.join();
        for (const auto& e : errs)
          if (!e.empty()) QTT_THROW(TT_ERR_HIP, "%s", e.c_str());
      } else {
        for (int k = 0; k < nb; ++k) branch(k);
      }
      for (int k = 0; k < nb; ++k) QTT_HIP(hipStreamWaitEvent(s0, b->events[k + 1], 0));
    }
    if (n_steps > 0) fused_states(b, false, s0);
  });
}

tt_status tt_batch_destroy(tt_batch* b) {
  return guard([&] {
    if (!b) return;
    if (!rt::dry()) (void)hipStreamSynchronize(b->ctx->stream);
    delete b;
  });
}

tt_status tt_step_tangent(tt_ctx* ctx, tt_problem* prob, tt_tt* f, int n_params, const int* params,
                          tt_tt* const* dfs, int n_steps) {
  return guard([&] {
    QTT_REQUIRE(prob && f && n_steps >= 0 && n_params >= 1 && n_params <= 2 && params && dfs,
                "bad argument");
    check_tt(f, ctx);
    QTT_REQUIRE(prob->ctx == ctx, "problem belongs to another context");
    if (prob->has_G || prob->has_Om)
      QTT_THROW(TT_ERR_UNSUPPORTED, "parameter derivatives need constant coefficients (no x-fields)");
    QTT_REQUIRE(f->caps == prob->fcaps, "state caps differ from the problem's");
    std::vector<Tangent> tan;
    std::vector<const void*> key{f};
    for (int j = 0; j < n_params; ++j) {
      QTT_REQUIRE(params[j] == TT_PARAM_OMEGA || params[j] == TT_PARAM_K, "unknown parameter %d", params[j]);
      for (int i = 0; i < j; ++i) QTT_REQUIRE(params[i] != params[j], "parameter listed twice");
      check_tt(dfs[j], ctx);
      QTT_REQUIRE(dfs[j]->caps == prob->fcaps, "tangent caps differ from the problem's");
      QTT_REQUIRE(dfs[j] != f, "tangent aliases the state");
      for (int i = 0; i < j; ++i) QTT_REQUIRE(dfs[i] != dfs[j], "two parameters share a tangent");
      ensure_tangent(prob, params[j]);
      tan.push_back({params[j], dfs[j]});
      key.push_back(dfs[j]);
      key.push_back(reinterpret_cast<const void*>((intptr_t)params[j]));
    }
    if (n_steps == 0) return;
    if (!prob->tplan || prob->tplan_key != key) {
      prob->tplan = record_step(prob, f, tan);
      prob->tplan_key = key;
      if (prob->texec) (void)hipGraphExecDestroy(prob->texec);
      if (prob->tgraph) (void)hipGraphDestroy(prob->tgraph);
      prob->texec = nullptr;
      prob->tgraph = nullptr;
      prob->last_tan = prob->last;
      prob->last = prob->last_plain;
    }
    prob->last = prob->last_tan;
    StreamScope sc(ctx);
    if (rt::dry() || !use_graph()) {
      for (int i = 0; i < n_steps; ++i) prob->tplan->run(ctx->stream);
      return;
    }
    if (!prob->texec) {
      QTT_HIP(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
      try {
        prob->tplan->run(ctx->stream);
      } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(ctx->stream, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      QTT_HIP(hipStreamEndCapture(ctx->stream, &prob->tgraph));
      QTT_HIP(hipGraphInstantiate(&prob->texec, prob->tgraph, nullptr, nullptr, 0));
    }
    for (int i = 0; i < n_steps; ++i) QTT_HIP(hipGraphLaunch(prob->texec, ctx->stream));
  });
}

tt_status tt_profile(tt_ctx* ctx, tt_problem* prob, tt_tt* f, int n_steps, int kernel, double* ms,
                     int64_t* launches, double* flops, double* bytes) {
  return guard([&] {
    QTT_REQUIRE(prob && f && n_steps >= 1, "bad argument");
    check_tt(f, ctx);
    QTT_REQUIRE(f->caps == prob->fcaps, "state caps differ from the problem's");
    QTT_REQUIRE(kernel >= 0 && kernel <= 4, "unknown kernel class %d", kernel);
    if (!prob->plan || prob->plan_f != f) build_step_plan(prob, f);
    StreamScope sc(ctx);
    double t = 0, fl = 0, by = 0;
    int64_t n = 0;
    for (int i = 0; i < n_steps; ++i) prob->plan->run_profiled(ctx->stream, kernel, t, n, fl, by);
    if (ms) *ms = t;
    if (launches) *launches = n;
    if (flops) *flops = fl;
    if (bytes) *bytes = by;
  });
}

tt_status tt_step_info(tt_problem* prob, double* discarded, double* norm2) {
  return guard([&] {
    QTT_REQUIRE(prob && prob->plan, "no step recorded yet");
    rt::sync(prob->ctx->stream);
    const int N = prob->N, ld = prob->last.ldl;
    std::vector<double> lam((size_t)(N + 1) * ld);
    rt::copy(lam.data(), prob->last.lam, lam.size() * sizeof(double));
    auto ell = chain_caps(N, prob->p.ell);
    for (int n = 0; n <= N; ++n) {
      double d = 0.0;
      if (n >= 1 && n < N)
        for (int i = std::min(ell[n], prob->fcaps[n]); i < ell[n]; ++i) d += std::max(0.0, lam[(size_t)n * ld + i]);
      if (discarded) discarded[n] = d;
    }
    if (norm2) {
      double s = 0.0;
      if (N >= 2)
        for (int i = 0; i < ell[1]; ++i) s += std::max(0.0, lam[(size_t)ld + i]);
      *norm2 = s;
    }
    take_nonfinite(prob, "a rounding of a step");
  });
}

tt_status tt_mean_field(tt_ctx* ctx, tt_problem* prob, const tt_tt* f, int a, tt_tt** out,
                        double* scalar) {
  return guard([&] {
    QTT_REQUIRE(prob && (a == 0 || a == 1), "bad argument");
    check_tt(f, ctx);
    QTT_REQUIRE(f->caps == prob->fcaps, "state caps differ from the problem's");
    Plan plan;
    double* E = plan.alloc(2 * f->caps[prob->nphi]);
    double* first = plan.alloc(2 * 2 * std::max(1, prob->nx > 0 ? f->caps[prob->nphi + 1] : 1));
    plan_mean_raw(plan, prob, f, E, first);
    StreamScope sc(ctx);
    plan.run(ctx->stream);
    rt::sync(ctx->stream);
    if (prob->nx == 0) {
      double h[2];
      rt::copy(h, E, sizeof(h));
      if (scalar) *scalar = h[a];
      if (out) *out = nullptr;
      return;
    }
    QTT_REQUIRE(out, "out is null");
    std::vector<int> caps(prob->nx + 1);
    caps[0] = 1;
    for (int j = 1; j <= prob->nx; ++j) caps[j] = f->caps[prob->nphi + j];
    auto m = make_tt(ctx, TT_MPS, prob->nx, caps);
    const int c1 = f->caps[prob->nphi + 1];
    rt::copy(m->core(0), first + (size_t)a * 2 * c1, 2 * c1 * sizeof(double));
    for (int j = 1; j < prob->nx; ++j)
      rt::copy(m->core(j), f->core(prob->nphi + j),
                        (m->off[j + 1] - m->off[j]) * sizeof(double));
    *out = m.release();
  });
}

tt_status tt_observable(tt_ctx* ctx, tt_problem* prob, const tt_tt* f, int which, double* out) {
  return guard([&] {
    QTT_REQUIRE(prob && out, "bad argument");
    check_tt(f, ctx);
    QTT_REQUIRE(f->caps == prob->fcaps, "state caps differ from the problem's");
    QTT_REQUIRE(which >= TT_OBS_MASS && which <= TT_OBS_PRODUCT, "unknown observable %d", which);
    const tt_params& p = prob->p;
    const int M = 1 << p.bits;
    const double h = 1.0 / M;
    auto order = host::site_order(p.ndims, p.bits, p.ordering);
    std::vector<double> one(M, h), phi(M);
    for (int i = 0; i < M; ++i) phi[i] = h * (i + 0.5) * h;
    // weight chain for sum_x,phi w(phi) f h^d
    auto weight = [&](const std::vector<const std::vector<double>*>& per_phi) {
      std::vector<host::TT> q(p.ndims);
      std::vector<const host::TT*> pp(p.ndims);
      for (int d = 0; d < p.ndims; ++d) {
        const std::vector<double>* v = (d < 2) ? per_phi[d] : &one;
        q[d] = host::vector_qtt(v->data(), p.bits);
        pp[d] = &q[d];
      }
      return host::kron_dims(pp, order, p.ndims, 2);
    };
    auto contract = [&](const host::TT& w) {
      auto wt = upload(ctx, TT_MPS, w, exact_caps(w));
      Plan plan;
      double* r = plan.alloc(1);
      plan_inner(plan, view(wt.get()), view(f), r);
      StreamScope sc(ctx);
      plan.run(ctx->stream);
      double v;
      rt::copy_async(&v, r, sizeof(double), ctx->stream);
      rt::sync(ctx->stream);
      return v;
    };
    auto mass = [&] { return contract(weight({&one, &one})); };
    auto mean = [&](int a) { return contract(weight({a == 0 ? &phi : &one, a == 1 ? &phi : &one})); };
    auto mean12 = [&] { return contract(weight({&phi, &phi})); };
    auto avg_m1m2 = [&]() -> double {
      if (prob->nx == 0) return mean(0) * mean(1);
      tt_tt *m0 = nullptr, *m1 = nullptr;
      tt_status st = tt_mean_field(ctx, prob, f, 0, &m0, nullptr);
      if (st != TT_OK) QTT_THROW(st, "%s", get_error());
      st = tt_mean_field(ctx, prob, f, 1, &m1, nullptr);
      if (st != TT_OK) QTT_THROW(st, "%s", get_error());
      std::unique_ptr<tt_tt> u0(m0), u1(m1);
      double v;
      st = tt_inner(ctx, m0, m1, &v);
      if (st != TT_OK) QTT_THROW(st, "%s", get_error());
      return std::pow(h, prob->nx / p.bits) * v;
    };
    double v = 0.0;
    switch (which) {
      case TT_OBS_MASS: v = mass(); break;
      case TT_OBS_MEAN1: v = mean(0); break;
      case TT_OBS_MEAN2: v = mean(1); break;
      case TT_OBS_MEAN12: v = mean12(); break;
      case TT_OBS_PRODUCT: v = mass() - mean(0) - mean(1); break;
      case TT_OBS_R12: v = avg_m1m2() - mean(0) * mean(1); break;
      case TT_OBS_Y12: v = mean12() - avg_m1m2(); break;
    }
    *out = v;
  });
}

tt_status tt_linalg_qr(tt_ctx* ctx, int count, int m, int n, const double* A, double* Q, double* R) {
  return guard([&] {
    QTT_REQUIRE(ctx && A && Q && count >= 1 && n >= 1 && m >= n && n <= 1024, "bad argument");
    const size_t mn = (size_t)m * n, nn = (size_t)n * n;
    const int64_t ws = qr_work_size(count, m, n);
    DevBuf dA(count * mn * 8), dQ(count * mn * 8), dR(count * nn * 8), dW((size_t)ws * 8);
    StreamScope sc(ctx);
    rt::copy(dA.p, A, count * mn * 8);
    qr_launch(count, m, n, dA.d(), (int64_t)mn, n, 1, dQ.d(), (int64_t)mn, R ? dR.d() : nullptr,
              (int64_t)nn, dW.d(), ctx->stream, nullptr, 0, ws);
    rt::sync(ctx->stream);
    rt::copy(Q, dQ.p, count * mn * 8);
    if (R) rt::copy(R, dR.p, count * nn * 8);
  });
}

tt_status tt_linalg_eigh(tt_ctx* ctx, int count, int n, int keep, const double* G, double* P,
                         double* lam) {
  return guard([&] {
    QTT_REQUIRE(ctx && G && P && lam && count >= 1 && n >= 1 && n <= 1024 && keep >= 1 && keep <= n,
                "bad argument");
    const size_t nn = (size_t)n * n;
    DevBuf dG(count * nn * 8), dP(count * (size_t)n * keep * 8), dL(count * (size_t)n * 8),
        dW(eig_work_size(count, n) * 8), dd(count * sizeof(int)), dk(count * sizeof(int));
    std::vector<int> dims(count, n), kp(count, keep);
    StreamScope sc(ctx);
    rt::copy(dG.p, G, count * nn * 8);
    rt::copy(dd.p, dims.data(), count * sizeof(int));
    rt::copy(dk.p, kp.data(), count * sizeof(int));
    fill(dP.d(), (int64_t)count * n * keep, 0.0, ctx->stream);
    const bool pre = eig_uses_precondition(n);
    if (pre) eig_precondition_launch(count, dd.as<int>(), dG.d(), (int64_t)nn, n, dW.d(), n, ctx->stream);
    eig_launch(count, dd.as<int>(), dk.as<int>(), dG.d(), (int64_t)nn, n, dP.d(), (int64_t)n * keep,
               keep, dL.d(), n, dW.d(), n, machine_eps(Prec::F64), ctx->stream, pre);
    rt::sync(ctx->stream);
    rt::copy(P, dP.p, count * (size_t)n * keep * 8);
    rt::copy(lam, dL.p, count * (size_t)n * 8);
  });
}

}  // extern "C"

// ===========================================================================
// flow case: composition moments as x-fields, dense evaluation, the
// Smagorinsky field, the moment equation and the error measures
// ===========================================================================
tt_status tt_moment_field(tt_ctx* ctx, tt_problem* prob, const tt_tt* f, const double* w1,
                          const double* w2, tt_tt** out) {
  return guard([&] {
    QTT_REQUIRE(prob && out, "bad argument");
    check_tt(f, ctx);
    QTT_REQUIRE(prob->nx > 0, "moment fields need a problem with x dimensions");
    QTT_REQUIRE(f->caps == prob->fcaps, "state caps differ from the problem's");
    const tt_params& p = prob->p;
    const int M = 1 << p.bits;
    const double h = 1.0 / M;
    std::vector<double> v1(M, h), v2(M, h);
    for (int i = 0; i < M; ++i) {
      if (w1) v1[i] = h * w1[i];
      if (w2) v2[i] = h * w2[i];
    }
    auto order = host::site_order(p.ndims, p.bits, p.ordering);
    std::vector<std::pair<int, int>> phi_order(order.begin(), order.begin() + prob->nphi);
    host::TT q1 = host::vector_qtt(v1.data(), p.bits), q2 = host::vector_qtt(v2.data(), p.bits);
    host::TT w = host::kron_dims({&q1, &q2}, phi_order, 2, 2);
    auto wt = upload(ctx, TT_MPS, w, exact_caps(w));
    const int c = f->caps[prob->nphi], c1 = f->caps[prob->nphi + 1];
    std::vector<int> caps(prob->nx + 1);
    caps[0] = 1;
    for (int j = 1; j <= prob->nx; ++j) caps[j] = f->caps[prob->nphi + j];
    auto m = make_tt(ctx, TT_MPS, prob->nx, caps);
    Plan plan;
    double* E = plan.alloc(c);
    plan_partial(plan, view(wt.get()), view_sites(f, 0, prob->nphi), E);
    TcDesc d = gemm_desc(1, 2 * c1, c, E, c, false, f->core(prob->nphi), 2 * c1, false, m->core(0),
                         2 * c1);
    plan.add([d](hipStream_t s) { tc_launch(d, Prec::F64, s); });
    StreamScope sc(ctx);
    plan.run(ctx->stream);
    for (int j = 1; j < prob->nx; ++j)
      rt::copy_async(m->core(j), f->core(prob->nphi + j),
                     (m->off[j + 1] - m->off[j]) * sizeof(double), ctx->stream);
    rt::sync(ctx->stream);
    *out = m.release();
  });
}

tt_status tt_to_dense(tt_ctx* ctx, const tt_tt* x, double* out) {
  return guard([&] {
    check_tt(x, ctx);
    QTT_REQUIRE(out, "out is null");
    QTT_REQUIRE(x->kind == TT_MPS, "tt_to_dense needs an MPS");
    const int N = x->N;
    QTT_REQUIRE(N >= 1 && N <= 30, "tt_to_dense: %d sites outside [1, 30]", N);
    // T_n (2^n x c_n, row-major) = T_{n-1} (2^(n-1) x c_{n-1}) * core (c_{n-1} x 2 c_n)
    int64_t maxsz = 2 * (int64_t)x->caps[1];
    for (int n = 1; n < N; ++n) maxsz = std::max(maxsz, (int64_t(1) << n) * 2 * x->caps[n + 1]);
    DevBuf A((size_t)maxsz * sizeof(double)), B((size_t)maxsz * sizeof(double));
    StreamScope sc(ctx);
    rt::copy_async(A.p, x->core(0), 2 * (size_t)x->caps[1] * sizeof(double), ctx->stream);
    int64_t rows = 2;
    constexpr int64_t CHUNK = int64_t(1) << 20;
    for (int n = 1; n < N; ++n) {
      const int K = x->caps[n], NC = 2 * x->caps[n + 1];
      for (int64_t r0 = 0; r0 < rows; r0 += CHUNK) {
        const int rr = (int)std::min(CHUNK, rows - r0);
        TcDesc d = gemm_desc(rr, NC, K, A.d() + r0 * K, K, false, x->core(n), NC, false,
                             B.d() + r0 * NC, NC);
        tc_launch(d, Prec::F64, ctx->stream);
      }
      std::swap(A, B);
      rows *= 2;
    }
    rt::copy_async(out, A.p, (size_t)rows * sizeof(double), ctx->stream);
    rt::sync(ctx->stream);
  });
}

tt_status fd_smagorinsky(tt_ctx* ctx, int bits, const double* U, double c_s, double delta,
                         double gamma, double* G) {
  return guard([&] {
    QTT_REQUIRE(ctx && U && G, "bad argument");
    QTT_REQUIRE(delta > 0 && c_s >= 0 && gamma >= 0, "bad closure constants");
    const int64_t n = int64_t(1) << (3 * bits);
    QTT_REQUIRE(G + n <= U || U + 3 * n <= G, "G overlaps U");
    StreamScope sc(ctx);
    smagorinsky(bits, U, c_s * delta * delta / 2.0, gamma, G, ctx->stream);
  });
}

tt_status fd_moment_steps(tt_ctx* ctx, int bits, int count, const double* U, const double* G,
                          double* m, double* work, double dt, int n_steps) {
  return guard([&] {
    QTT_REQUIRE(ctx && U && G && m && work, "bad argument");
    QTT_REQUIRE(count >= 1 && count <= 2, "count %d outside [1, 2]", count);
    QTT_REQUIRE(n_steps >= 0, "negative step count");
    const int64_t n = int64_t(1) << (3 * bits);
    QTT_REQUIRE(m + count * n <= work || work + count * n <= m, "work overlaps m");
    StreamScope sc(ctx);
    for (int k = 0; k < n_steps; ++k) {
      // Heun: m1 = m + dt L(m); m+ = (m + m1) / 2 + dt / 2 L(m1)
      moment_stage(bits, count, U, G, m, nullptr, 0.0, 1.0, dt, work, ctx->stream);
      moment_stage(bits, count, U, G, work, m, 0.5, 0.5, 0.5 * dt, m, ctx->stream);
    }
  });
}

tt_status fd_sq_diff_sum(tt_ctx* ctx, int64_t n, const double* a, const double* b, double c,
                         double* out) {
  return guard([&] {
    QTT_REQUIRE(ctx && a && out && n >= 1, "bad argument");
    DevBuf part((size_t)(sq_diff_partials() + 1) * sizeof(double));
    StreamScope sc(ctx);
    sq_diff_sum(n, a, b, c, part.d(), part.d() + sq_diff_partials(), ctx->stream);
    rt::copy_async(out, part.d() + sq_diff_partials(), sizeof(double), ctx->stream);
    rt::sync(ctx->stream);
  });
}

tt_status flow_error_measures(int n_samples, const double* mean_bar, const double* sq_mean_x,
                              const double* sq_norm_x, double* out) {
  return guard([&] {
    QTT_REQUIRE(n_samples >= 1 && mean_bar && sq_norm_x && out, "bad argument");
    const int T = n_samples;
    double up = 0.0, dn = 0.0, cu = 0.0, cd = 0.0;
    for (int t = 0; t < T; ++t) {
      for (int a = 0; a < 2; ++a) {
        const double e = mean_bar[a * T + t] - 0.5;
        up += e * e;
        if (sq_mean_x) dn += sq_mean_x[a * T + t];
      }
      const double d = mean_bar[t] - mean_bar[T + t];
      cu += d * d;
      cd += sq_norm_x[t];
    }
    out[0] = std::sqrt(0.5 * up / T);
    out[1] = sq_mean_x ? std::sqrt(0.5 * dn / T) : std::nan("");
    out[2] = std::sqrt(cu / T);
    out[3] = std::sqrt(cd / T);
  });
}

extern "C" {

tt_status tt_prolong(tt_ctx* ctx, const tt_tt* x, int ndims, int bits, int chi, tt_tt** out,
                     double* discarded) {
  return guard([&] {
    check_tt(x, ctx);
    QTT_REQUIRE(out && x->kind == TT_MPS, "bad argument");
    QTT_REQUIRE(ndims >= 1 && ndims <= 8 && bits >= 1 && bits <= 20 && x->N == ndims * bits,
                "tt_prolong: %d sites are not %d dimensions of %d bits", x->N, ndims, bits);
    QTT_REQUIRE(chi >= 1, "bad chi");
    StreamScope sc(ctx);
    hipStream_t s = ctx->stream;
    const host::TT Q = host::prolong_block(bits);
    std::unique_ptr<tt_tt> cur;  // the chain after the dimensions refined so far
    const tt_tt* y = x;
    double disc = 0.0;
    for (int d = 0; d < ndims; ++d) {
      // lift: a new site after the last digit of dimension d whose core is the
      // identity on its bond, so the lifted value does not depend on the new digit
      const int N = y->N, p = (d + 1) * bits + d;  // index of the new site
      std::vector<int> lc(N + 2);
      for (int n = 0; n <= p; ++n) lc[n] = y->caps[n];
      lc[p + 1] = y->caps[p];
      for (int n = p + 1; n <= N; ++n) lc[n + 1] = y->caps[n];
      auto z = make_tt(ctx, TT_MPS, N + 1, lc);
      for (int n = 0; n < N; ++n) {
        const int m = n < p ? n : n + 1;
        rt::copy_async(z->core(m), y->core(n), (size_t)(y->off[n + 1] - y->off[n]) * sizeof(double), s);
      }
      {
        const int r = y->caps[p];
        std::vector<double> id((size_t)r * 2 * r, 0.0);
        for (int a = 0; a < r; ++a) id[(size_t)a * 2 * r + a] = id[((size_t)a * 2 + 1) * r + a] = 1.0;
        rt::copy(z->core(p), id.data(), id.size() * sizeof(double));
      }
      // interpolation MPO on the lifted chain: identity outside dimension d's block
      host::TT W;
      for (int n = 0; n < d * bits + d; ++n) W.push_back(host::mpo_identity(1)[0]);
      W.insert(W.end(), Q.begin(), Q.end());
      while ((int)W.size() < N + 1) W.push_back(host::mpo_identity(1)[0]);
      auto Wd = upload(ctx, TT_MPO, W, exact_caps(W));
      // exact product, then deterministic rounding to chi
      std::vector<int> pc(N + 2);
      for (int n = 0; n <= N + 1; ++n) pc[n] = z->caps[n] * Wd->caps[n];
      auto yz = make_tt(ctx, TT_MPS, N + 1, pc);
      std::vector<ApplyJob> jobs;
      int64_t maxe = 1;
      for (int n = 0; n <= N; ++n) {
        jobs.push_back({Wd->core(n), z->core(n), yz->core(n), z->caps[n], z->caps[n + 1], Wd->caps[n],
                        Wd->caps[n + 1]});
        maxe = std::max<int64_t>(maxe, (int64_t)pc[n] * 2 * pc[n + 1]);
      }
      for (const ApplyJob& j : jobs) validate(j);
      DevBuf dj(jobs.size() * sizeof(ApplyJob));
      rt::copy(dj.p, jobs.data(), jobs.size() * sizeof(ApplyJob));
      apply_jobs(dj.as<ApplyJob>(), N + 1, maxe, s);
      auto r = make_tt(ctx, TT_MPS, N + 1, chain_caps(N + 1, chi));
      Plan plan;
      RoundTarget tg;
      for (int n = 0; n <= N; ++n) tg.core.push_back(r->core(n));
      tg.caps = r->caps;
      plan_round_det(plan, view(yz.get()), tg);
      plan.run(s);
      const RoundOutcome o = round_outcome(tg, s);  // synchronises before the temporaries go
      for (double v : o.discarded) disc += v;
      cur = std::move(r);
      y = cur.get();
    }
    if (discarded) *discarded = disc;
    *out = cur.release();
  });
}

tt_status tt_from_dense(tt_ctx* ctx, int n_sites, const double* values, int chi, tt_tt** out,
                        double* discarded) {
  return guard([&] {
    QTT_REQUIRE(ctx && values && out, "bad argument");
    const int N = n_sites;
    QTT_REQUIRE(N >= 2 && N <= 30, "tt_from_dense: %d sites outside [2, 30]", N);
    QTT_REQUIRE(chi >= 1 && chi <= 512, "tt_from_dense: chi %d outside [1, 512]", chi);
    const int64_t total = int64_t(1) << N;
    auto caps = chain_caps(N, chi);
    auto x = make_tt(ctx, TT_MPS, N, caps);
    DevBuf A((size_t)total * 8), B((size_t)total * 8);
    int gm = 2;
    for (int n = 0; n < N; ++n) gm = std::max(gm, 2 * caps[n]);
    DevBuf Gd((size_t)gm * gm * 8), Pd((size_t)gm * gm * 8), Ld((size_t)gm * 8),
        Wd((size_t)eig_work_size(1, gm) * 8), dd(sizeof(int)), dk(sizeof(int));
    StreamScope sc(ctx);
    hipStream_t s = ctx->stream;
    rt::copy_async(A.p, values, (size_t)total * 8, s);
    double disc = 0.0;
    std::vector<double> lam(gm);
    for (int n = 0; n + 1 < N; ++n) {
      // C (rows = 2 r, K = 2^(N-n-1) columns) -> Gram C C^T -> leading eigenvectors P
      const int r = caps[n], rows = 2 * r, k = caps[n + 1];
      const int64_t K = total >> (n + 1);
      TcDesc g = gemm_desc(rows, rows, (int)K, A.d(), K, false, A.d(), K, true, Gd.d(), rows);
      g.ksplit = tc_choose_ksplit(g, Prec::F64);
      DevBuf part;
      if (tc_uses_part(g)) {
        part.alloc((size_t)tc_part_size(g) * 8);
        g.part = part.d();
      }
      tc_launch(g, Prec::F64, s);
      rt::copy_async(dd.p, &rows, sizeof(int), s);
      rt::copy_async(dk.p, &k, sizeof(int), s);
      const bool pre = eig_uses_precondition(rows);
      if (pre) eig_precondition_launch(1, dd.as<int>(), Gd.d(), (int64_t)rows * rows, rows, Wd.d(), rows, s);
      eig_launch(1, dd.as<int>(), dk.as<int>(), Gd.d(), (int64_t)rows * rows, rows, Pd.d(),
                 (int64_t)rows * k, k, Ld.d(), rows, Wd.d(), rows, machine_eps(Prec::F64), s, pre);
      // core n = P (r x 2 x k, the caps of this chain exactly); next C = P^T C
      rt::copy_async(x->core(n), Pd.d(), (size_t)rows * k * 8, s);
      TcDesc c = gemm_desc(k, (int)K, rows, Pd.d(), k, true, A.d(), K, false, B.d(), K);
      tc_launch(c, Prec::F64, s);
      rt::copy_async(lam.data(), Ld.d(), (size_t)rows * 8, s);
      rt::sync(s);  // the part buffer and the host copies of dims, keep and lam
      for (int i = k; i < rows; ++i) disc += std::max(0.0, lam[i]);
      std::swap(A, B);
    }
    rt::copy_async(x->core(N - 1), A.p, 2 * (size_t)caps[N - 1] * 8, s);
    rt::sync(s);
    if (discarded) *discarded = disc;
    *out = x.release();
  });
}

}  // extern "C"
