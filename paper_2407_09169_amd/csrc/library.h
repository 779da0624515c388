// Internal structures of the qttpdf library: contexts, device tensor trains,
// launch plans (recorded once, replayed eagerly or as a HIP graph) and the
// rounding planners.
#pragma once

#include <functional>
#include <string>
#include <memory>
#include <unordered_map>

#include "common.h"
#include "elementwise.h"
#include "host_tt.h"

struct tt_ctx {
  int device = 0;
  hipStream_t stream = nullptr;       // the library's own stream (non-blocking)
  hipStream_t user_stream = nullptr;  // caller's stream (ordering is kept with events)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
};

struct tt_tt {
  tt_ctx* ctx = nullptr;
  int kind = TT_MPS;  // TT_MPS or TT_MPO
  int N = 0;
  int p = 2;  // physical size of a core (2 MPS, 4 MPO)
  std::vector<int> caps;
  std::vector<int64_t> off;  // element offset of every core, off[N] = total
  qtt::DevBuf buf;
  double* core(int n) const { return buf.d() + off[n]; }
  int64_t total() const { return off[N]; }
};

namespace qtt {

// enqueue-on-own-stream scope: orders the library stream after the user's
// stream on entry and the user's stream after the library stream on exit
struct StreamScope {
  tt_ctx* c;
  explicit StreamScope(tt_ctx* ctx);
  ~StreamScope();
};

std::unique_ptr<tt_tt> make_tt(tt_ctx* ctx, int kind, int N, const std::vector<int>& caps);
std::vector<int> chain_caps(int N, long cap);

// per-site core pointers and bond capacities of a chain
struct ChainView {
  int N = 0;
  int p = 2;
  std::vector<const double*> core;
  std::vector<int> caps;  // N + 1
};
ChainView view(const tt_tt* t);
ChainView view_sites(const tt_tt* t, int first, int count);  // sub-chain (bond caps as stored)

// kernel classes of a plan (for per-class timing)
enum OpKind { OP_SYNC = -2, OP_OTHER = -1, OP_CONTRACT = 0, OP_QR = 1, OP_EIG = 2, OP_STREAM = 3, OP_ALL = 4 };
struct OpInfo {
  int kind = OP_OTHER;
  double flops = 0.0;  // algorithmic flops of the launch
  double bytes = 0.0;  // algorithmic bytes (operands read once, results written once)
  std::string what;    // shape description for per-op timing logs
};

// List of enqueue operations with the workspaces they use.  Operations go to
// lanes: lane 0 is the stream the plan runs on, lanes 1.. are streams the
// plan owns (default priority).  fork(n) makes lanes 1..n-1 wait for what
// lane 0 has enqueued so far; join(n) makes lane 0 wait for lanes 1..n-1.
// A plan ends joined, so a replay (eager or captured into a HIP graph) is
// ordered with the caller's stream at both ends.
//
// Every fork starts from lane 0 and every join ends on it: under HIP graph
// capture, a lane other than the capturing stream may neither record an
// event that another such lane waits for nor wait for one recorded there
// (this host runtime fails at capture time on that pattern).
struct Plan {
  std::vector<std::function<void(hipStream_t)>> ops;
  std::vector<OpInfo> info;
  std::vector<int> lane;  // lane of every op
  std::vector<std::unique_ptr<DevBuf>> bufs;
  std::vector<hipStream_t> streams;  // lanes 1..
  std::vector<hipEvent_t> events;
  int cur = 0;  // lane of the next op
  Plan() = default;
  Plan(const Plan&) = delete;
  Plan& operator=(const Plan&) = delete;
  ~Plan();
  // With an arena (a device buffer owned by the caller), alloc() carves
  // 256-byte aligned pieces from its bottom instead of allocating, and
  // upload() and lanes are refused: recording such a plan allocates no device
  // memory.  alloc_transient() serves buffers that live for one launch only
  // (split-K partial sums): with an arena they all share its top, which is
  // safe because the plan's launches run one after another on one stream.
  double* arena = nullptr;
  size_t arena_cap = 0, arena_used = 0, arena_top = 0;  // in doubles
  double* alloc(size_t n_doubles) {
    if (arena) {
      const size_t n = (std::max<size_t>(n_doubles, 1) + 31) & ~size_t(31);
      arena_fits(arena_used + n, arena_top);
      double* p = arena + arena_used;
      arena_used += n;
      return p;
    }
    bufs.emplace_back(new DevBuf(std::max<size_t>(n_doubles, 1) * sizeof(double)));
    return bufs.back()->d();
  }
  double* alloc_transient(size_t n_doubles) {
    if (!arena) return alloc(n_doubles);
    const size_t n = (std::max<size_t>(n_doubles, 1) + 31) & ~size_t(31);
    arena_fits(arena_used, std::max(arena_top, n));
    arena_top = std::max(arena_top, n);
    return arena + (arena_cap - n);
  }
  template <class T>
  T* upload(const std::vector<T>& host) {
    QTT_REQUIRE(arena == nullptr, "a plan on a fixed scratch buffer cannot upload tables");
    bufs.emplace_back(new DevBuf(std::max<size_t>(host.size(), 1) * sizeof(T)));
    if (!host.empty()) rt::copy(bufs.back()->p, host.data(), host.size() * sizeof(T));
    uploads.push_back({bufs.back()->p, host.size() * sizeof(T)});
    return static_cast<T*>(bufs.back()->p);
  }
  // device memory written when the plan was recorded (uploaded tables and
  // constants): (pointer, bytes)
  std::vector<std::pair<void*, size_t>> uploads;
  void add(std::function<void(hipStream_t)> f, OpInfo oi = OpInfo{}) {
    ops.push_back(std::move(f));
    info.push_back(oi);
    lane.push_back(cur);
  }
  void fork(int n);
  void arena_fits(size_t bottom, size_t top) const {
    if (bottom + top > arena_cap)
      QTT_THROW(TT_ERR_INVALID_ARG,
                "the operation needs %zu bytes of scratch, more than the %zu bytes of the static scratch buffer",
                (bottom + top) * sizeof(double), arena_cap * sizeof(double));
  }
  void on(int l) { cur = l; }
  void join(int n);
  hipStream_t stream_of(int l, hipStream_t s0) const {
    if (l == 0) return s0;
    QTT_REQUIRE(l >= 1 && l - 1 < (int)streams.size(), "plan lane %d has no stream", l);
    return streams[l - 1];
  }
  void run(hipStream_t s) const {
    for (size_t i = 0; i < ops.size(); ++i) ops[i](stream_of(lane[i], s));
  }

  // eager run with a pair of events around every op of class `kind` (OP_ALL:
  // every op); adds the event time (ms), the number of such ops and their
  // flops / bytes.  With QTTPDF_PROFILE_LOG=<file> set, one line per timed op
  // (index, class, ms, flops, bytes, kernel|shape) is appended to that
  // file.
  void run_profiled(hipStream_t s, int kind, double& ms, int64_t& count, double& flops,
                    double& bytes) const;

 private:
  hipEvent_t new_event();
  void ensure_lanes(int n);
};

// lanes a planner may fork into (at most `want`): 1 unless it records on
// lane 0 of a plan with lanes
inline int lane_budget(const Plan& plan, int want) {
  if (plan.cur != 0) return 1;
  return std::max(1, want);
}

// Precision by role in a sketched rounding.  The sketch chains and the
// sketched unfoldings only choose the bases that the QR sweeps
// orthogonalise, so they run in the requested contraction precision; the
// contractions that carry the data into the result (the projections of the
// terms onto the bases, the centre core) run in FP32 when BF16 is requested,
// so the operator's cores (whose column sums vanish, keeping the mass) and
// the state keep FP32 accuracy.  FP32 and FP64 use one precision throughout.
inline Prec data_prec(Prec p) { return p == Prec::BF16 ? Prec::F32 : p; }

struct SketchTerm {
  double coef = 1.0;
  const ChainView* mpo = nullptr;  // nullptr: identity
  ChainView x;
  // sites >= diag_from (if >= 0) have MPO cores that are diagonal in the
  // physical index (W[A,t,s,B] = 0 for t != s), such as diag(field) on the x
  // sites of a Hadamard-product term: their contractions skip the zeros
  // (two-sided rounding only)
  int diag_from = -1;
  bool diag_at(int n) const { return mpo != nullptr && diag_from >= 0 && n >= diag_from; }
};

// Output of a rounding: destination cores (caps chi_n) and, for reporting,
// the eigenvalues of every bond's Gram matrix.
struct RoundTarget {
  std::vector<double*> core;
  std::vector<int> caps;
  double* lam = nullptr;  // (N+1) x ldl eigenvalues (optional, filled by the planner)
  int ldl = 0;
  // > 0: at every bond also drop the singular values at most rel_tol sigma_1
  double rel_tol = 0.0;
  std::vector<int> in_caps;  // bonds of the chain that is truncated (filled by the planner)
};

// Outcome of a recorded rounding, read back on the host after it ran:
// per-bond discarded weight (sum of the dropped squared singular values),
// kept directions per bond, and the squared norm of the result.
struct RoundOutcome {
  std::vector<double> discarded;  // N + 1
  std::vector<int> kept;          // N + 1
  double norm2 = 0.0;
};
// synchronises `s` and reads the eigenvalues the rounding left in tg.lam
RoundOutcome round_outcome(const RoundTarget& tg, hipStream_t s);

// randomized range finding (right sketches + QR sweep) into an ell-rank
// left-orthogonal chain, then simultaneous SVD truncation to target.caps
// (the terms' independent chains use up to `lanes` lanes when called on lane 0)
void plan_round_sketch(Plan& plan, const std::vector<SketchTerm>& terms, const ChainView& Z,
                       RoundTarget& target, Prec prec, int lanes = 4);
// randomized range finding from both ends towards the middle site (right
// sketches with Zr for the left sweep, left sketches with Zl for the right
// sweep), then simultaneous truncation of the mixed canonical form
void plan_round_sketch_two_sided(Plan& plan, const std::vector<SketchTerm>& terms, const ChainView& Zr,
                                 const ChainView& Zl, RoundTarget& target, Prec prec, int lanes = 4);

// Several independent two-sided roundings with the same sketches, recorded
// phase by phase side by side so that their work shares the lanes.
struct RoundJob {
  const std::vector<SketchTerm>* terms;
  RoundTarget* tg;
};
void plan_round_two_sided_multi(Plan& plan, const std::vector<RoundJob>& jobs, const ChainView& Zr,
                                const ChainView& Zl, Prec prec, int lanes = 4);
// planner building blocks shared by the rounding planners
void add_tc(Plan& plan, TcDesc d, Prec p);
void add_gemm(Plan& plan, int M, int N, int K, const double* A, int64_t lda, bool ta, const double* B,
              int64_t ldb, bool tb, double* C, int64_t ldc, double alpha, double beta, Prec p);
OpInfo qr_info(int m, int n);
// thin Q of one m x n matrix (A at rows rs, columns cs apart; Q with ld n):
// one launch, or the reflector and Q launches of qr_split as two ops
void add_qr_q(Plan& plan, int m, int n, const double* A, int64_t rs, int64_t cs, double* Q, double* work,
              int64_t work_size);
// LQ sweep + QR sweep + simultaneous truncation of an explicit chain
void plan_round_det(Plan& plan, const ChainView& x, RoundTarget& target);
// QR sweep only: left-orthogonal copy (returns caps of the result); used for norms
struct LeftOrth {
  std::vector<double*> core;
  std::vector<int> caps;
};
LeftOrth plan_left_orth(Plan& plan, const ChainView& x);
// block-diagonal sum into dst (dst caps must equal the sums of the term caps)
void plan_axpby(Plan& plan, const std::vector<std::pair<double, ChainView>>& terms, tt_tt* dst);
// <a, b> environment chain; result in *out_dev (device scalar)
void plan_inner(Plan& plan, const ChainView& a, const ChainView& b, double* out_dev);
// contraction of the first sites of x with a weight chain w (right bond = channels);
// result E (channels x cap of x after the last contracted site) in out_dev
void plan_partial(Plan& plan, const ChainView& w, const ChainView& x, double* out_dev);

}  // namespace qtt
