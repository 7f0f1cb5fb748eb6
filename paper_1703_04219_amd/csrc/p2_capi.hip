// Host runtime and C ABI of the PARAFAC2-ALS hot path (see include/parafac2.h).
//
// A context owns no device memory: every buffer is carved out of the caller's
// workspace by a fixed plan (Plan below).  Init validates the input on the
// device, relabels columns by decreasing frequency (hot columns get the
// smallest ids, so the mode-2 kernel can keep their partial sums in LDS with a
// single range test), re-encodes the slices compactly (16-bit columns, 16-bit
// subject-relative row starts) and copies V into the internal column order.
//
// Iterations are driven by a Runner: launch groups of equal-rank problems,
// each with a device array of problem descriptors and tile lists.  A context
// has its own runner (a batch of one, arrays in its workspace); a batch has a
// runner over many contexts (arrays in the batch workspace).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "../../include/parafac2.h"
#include "p2_batch.h"
#include "p2_device.h"
#include "p2_host.h"
#include "p2_kernels.h"

namespace p2host {

std::string& last_error() {
  static thread_local std::string s;
  return s;
}

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  last_error() = buf;
  return code;
}

}  // namespace p2host

namespace {

using p2::kBins;
using p2::kFitRing;

using p2host::fail;

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }
inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }
inline int ldv_of(int R) { return (R + 3) & ~3; }

constexpr int kDefaultRounds = 4;
// subjects per window of the per-subject pass order (sorted by row count within)
constexpr int64_t kOrderWindow = 256;
constexpr int kDefaultM2Capacity = 512;
constexpr int kMaxM2Capacity = 4096;

int m2_capacity(const parafac2_opts* o) {
  if (o && o->m2_capacity > 0) return std::min(o->m2_capacity, kMaxM2Capacity);
  return kDefaultM2Capacity;
}

int hot_columns(const parafac2_opts* o, int R, int64_t J) {
  const int maxhot = p2::mode2_max_hot(R);
  if (o && o->hot_cols < 0) return 0;
  if (o && o->hot_cols > 0) return (int)std::min<int64_t>({(int64_t)o->hot_cols, (int64_t)maxhot, J});
  return (int)std::min<int64_t>(maxhot, J);
}

// Mode-2 partial-sum slots (tiles) of a problem of K subjects under a cap.
int64_t mode2_parts(int64_t K, int R, int cap) {
  const int64_t unit = std::max(1, p2::mode2_tile_unit(R));
  return std::max<int64_t>(1, std::min<int64_t>(cap, ceil_div(K, unit)));
}

// Offsets of every piece of the context workspace.
struct Plan {
  size_t zbase, rbase, rstart, nzrow, col16, val, rank, perm, hist, order, econ, V[2], F, M2, M3, E,
      small, err, part, desc, tiles, m2tiles, tickets, iter, erow, eval, runs, runbase, Q, yr, yj,
      yk, yv, acc, total;
  bool baseline = false;  // explicit-Y comparison method: runs, Q and Y are planned
  bool warm = false;
  bool nonneg = false;  // V and W by NNLS: a float64 copy of M3 feeds the W rows
  int64_t cap_tiles = 0, cap_m2 = 0;  // tile capacities of the context's own runner
  int m2cap = 0;                      // mode-2 partial-sum slots
  int hot = 0;
};

Plan make_plan(int64_t K, int64_t J, int64_t n_rows, int64_t nnz, int R, const parafac2_opts* o) {
  Plan p{};
  const int64_t LDV = ldv_of(R);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + std::max<size_t>(bytes, 1));
    return at;
  };
  p.hot = hot_columns(o, R, J);
  p.m2cap = m2_capacity(o);
  const int64_t nparts = mode2_parts(K, R, p.m2cap);
  p.cap_tiles = round_up(ceil_div(K, std::max(1, p2::polar_tile_unit(R))), kBins);
  p.cap_m2 = round_up(nparts, kBins);
  p.zbase = take(sizeof(int64_t) * (K + 1));
  p.rbase = take(sizeof(int64_t) * (K + 1));
  p.rstart = take(sizeof(uint16_t) * (size_t)n_rows);
  p.nzrow = take(sizeof(uint16_t) * (size_t)nnz);
  p.col16 = take(sizeof(uint16_t) * (size_t)nnz);
  p.val = take(sizeof(float) * (size_t)nnz);
  p.rank = take(sizeof(int32_t) * J);
  p.perm = take(sizeof(int32_t) * J);
  p.hist = take(sizeof(uint32_t) * J);
  p.order = take(sizeof(int32_t) * K);
  p.econ = take(sizeof(int32_t) * K);
  p.V[0] = take(sizeof(float) * J * LDV);
  p.V[1] = take(sizeof(float) * J * LDV);
  p.F = take(sizeof(double) * (size_t)K * R * R);
  p.M2 = take(sizeof(float) * J * LDV);
  p.M3 = take(sizeof(float) * (size_t)K * R);
  p.nonneg = o && o->nonneg;
  p.warm = (o && o->keep_bases) && p2::warm_supported(R);
  const int64_t NC = (R & 1) ? R + 1 : R;
  p.E = p.warm ? take(sizeof(float) * (size_t)K * NC * R) : 0;
  p.part = take(sizeof(float) * (size_t)nparts * p.hot * R);
  p.small = take(sizeof(double) * p2::small_layout(R).total);
  p.err = take(sizeof(int) * 4);
  p.desc = take(sizeof(p2::ProbDesc));
  p.tiles = take(sizeof(p2::Tile) * (size_t)p.cap_tiles);
  p.m2tiles = take(sizeof(p2::Tile) * (size_t)p.cap_m2);
  p.tickets = take(sizeof(int) * p2::kTicketKinds * kBins);
  p.iter = take(sizeof(int64_t));
  p.baseline = o && o->baseline;
  if (p.baseline) {
    const size_t ny = (size_t)R * (size_t)nnz;  // at most one run per nonzero
    p.erow = take(sizeof(uint16_t) * (size_t)nnz);
    p.eval = take(sizeof(float) * (size_t)nnz);
    p.runs = take(sizeof(uint32_t) * (size_t)nnz);
    p.runbase = take(sizeof(int64_t) * (K + 1));
    p.Q = take(sizeof(float) * (size_t)n_rows * R);
    p.yr = take(sizeof(int32_t) * ny);
    p.yj = take(sizeof(int32_t) * ny);
    p.yk = take(sizeof(int32_t) * ny);
    p.yv = take(sizeof(float) * ny);
    // FP64 sums of the mode-2 and mode-3 outputs (J x LDV, then K x R)
    p.acc = take(sizeof(double) * std::max<size_t>((size_t)J * LDV, (size_t)K * R));
  }
  p.total = off;
  return p;
}

p2::PolarParams polar_params(const parafac2_opts* o, int R) {
  p2::PolarParams pp;
  const int NC = (R & 1) ? R + 1 : R;
  // eigenvalues of G that should be zero (exact rank deficiency of X_k)
  // come out below ~1e-15 lambda_max from FP32-accumulated A_k, while genuine
  // ones reach ~1e-11 lambda_max on the Zipf workloads: cut in between
  pp.tau_polar = (o && o->tau_polar > 0) ? o->tau_polar : 1e-13;
  pp.tau_pinv = (o && o->tau_pinv > 0) ? o->tau_pinv : R * 2.220446049250313e-16;
  pp.tol = 8.0 * 2.220446049250313e-16 * std::sqrt((double)NC);
  pp.tau_c = 1e-12;
  pp.tau_s = 1e-12;
  pp.stop2 = 1e-10;
  pp.max_sweeps = (o && o->max_sweeps > 0) ? o->max_sweeps : 30;
  return pp;
}

bool same_params(const p2::PolarParams& a, const p2::PolarParams& b) {
  return a.tau_polar == b.tau_polar && a.tau_pinv == b.tau_pinv && a.max_sweeps == b.max_sweeps;
}

parafac2_sched normalized(const parafac2_sched* s) {
  parafac2_sched r{};
  if (s) r = *s;
  if (r.tile_rounds <= 0) r.tile_rounds = kDefaultRounds;
  r.tile_rounds = std::min(r.tile_rounds, 1 << 16);
  r.dynamic = r.dynamic ? 1 : 0;
  if (r.m2_tiles < 0) r.m2_tiles = 0;
  r.graph = r.graph ? 1 : 0;
  r.warm_polar = r.warm_polar ? 1 : 0;
  r.m2_threads = std::max(0, std::min(r.m2_threads, 1024)) / 64 * 64;
  r.m2_blocks = std::max(0, std::min(r.m2_blocks, 8));
  return r;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return fail(P2_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define P2_TRY(expr)            \
  do {                          \
    const int rc_ = (expr);     \
    if (rc_ != P2_OK) return rc_; \
  } while (0)

struct Runner;

}  // namespace

struct parafac2_ctx {
  int64_t K = 0, J = 0, n_rows = 0, nnz = 0;
  int R = 0, LDV = 0, hot = 0;
  hipStream_t stream = nullptr;
  double* H = nullptr;
  float* Vuser = nullptr;
  float* W = nullptr;
  unsigned char* ws = nullptr;
  Plan plan{};
  p2::PolarParams pp{};
  p2::XEnc X{};
  int cur = 0;          // index of V_t in V[2]
  int qv = -1;          // index of the V used by the last Q-step (for get_q)
  bool have_F = false;  // F/M1 hold the Procrustes step of the next iteration
  bool failed = false;
  int64_t iters_done = 0;
  int64_t n_econ = 0;  // subjects with I_k < R (economy Procrustes factor)
  p2::BaselineView base{};  // the explicit-Y comparison method (plan.baseline)
  std::vector<int64_t> subj_host;
  Runner* own = nullptr;  // batch of one over this context

  template <class T>
  T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
  double* small() const { return at<double>(plan.small); }
  float* V(int i) const { return at<float>(plan.V[i]); }
  p2::ProbDesc desc() const {
    p2::ProbDesc d{};
    d.X = X;
    d.K = K;
    d.J = J;
    d.V[0] = V(0);
    d.V[1] = V(1);
    d.W = W;
    d.H = H;
    d.F = at<double>(plan.F);
    d.M2 = at<float>(plan.M2);
    d.M3 = at<float>(plan.M3);
    d.E = plan.warm ? at<float>(plan.E) : nullptr;
    d.small = small();
    d.iter = at<int64_t>(plan.iter);
    d.part = at<float>(plan.part);
    d.nparts = 0;  // set by the runner from its schedule
    d.hot = hot;
    d.order = at<int32_t>(plan.order);
    d.nonneg = plan.nonneg ? 1 : 0;
    d.econ = at<int32_t>(plan.econ);
    d.n_econ = n_econ;
    return d;
  }
};

namespace {

// ---------------------------------------------------------------------------
// Runner: launch groups (one per rank) over a set of contexts
// ---------------------------------------------------------------------------

struct Group {
  int R = 0;
  bool nonneg = false;  // some member updates V and W by NNLS
  bool econ = false;    // some member has subjects with I_k < R
  std::vector<int> members;  // indices into Runner::ctxs
  p2::PolarParams pp{};
  p2::BatchView bv{};
  p2::ProbDesc* desc = nullptr;  // device arrays (in the owner's workspace)
  p2::Tile* tiles = nullptr;
  p2::Tile* m2tiles = nullptr;
  int* tickets = nullptr;
  int64_t cap_tiles = 0, cap_m2 = 0;
};

struct Runner {
  std::vector<parafac2_ctx*> ctxs;
  std::vector<Group> groups;
  parafac2_sched sched{};
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;  // capture stream of the graphs
  hipGraphExec_t exec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  bool planned = false;
  bool any_econ = false;
  bool baseline = false;  // a context of one running the explicit-Y method
  // profiling: event pairs per phase, resolved lazily
  bool profiling = false;
  struct EvPair {
    int phase;
    hipEvent_t a, b;
  };
  std::vector<EvPair> events;
  double prof_ms[P2_NPHASES] = {0};
  int64_t prof_n[P2_NPHASES] = {0};

  ~Runner() {
    drop_graphs();
    for (auto& e : events) {
      (void)hipEventDestroy(e.a);
      (void)hipEventDestroy(e.b);
    }
    if (cap) (void)hipStreamDestroy(cap);
  }
  void drop_graphs() {
    for (auto& row : exec)
      for (auto& g : row) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
      }
  }
};

// Workspace bytes of a runner's arrays for these contexts, and the offsets.
struct RunnerLayout {
  struct G {
    int R;
    std::vector<int> members;
    size_t desc, tiles, m2tiles, tickets;
    int64_t cap_tiles, cap_m2;
  };
  std::vector<G> groups;
  size_t total = 0;
};

RunnerLayout runner_layout(parafac2_ctx* const* ctxs, int n) {
  RunnerLayout L;
  std::map<int, std::vector<int>> by_rank;
  for (int i = 0; i < n; ++i) by_rank[ctxs[i]->R].push_back(i);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + std::max<size_t>(bytes, 1));
    return at;
  };
  for (auto& kv : by_rank) {
    RunnerLayout::G g;
    g.R = kv.first;
    g.members = kv.second;
    const int unit = std::max(1, p2::polar_tile_unit(g.R));
    int64_t nt = 0, nm = 0;
    for (int i : g.members) {
      nt += ceil_div(ctxs[i]->K, unit);
      nm += mode2_parts(ctxs[i]->K, g.R, ctxs[i]->plan.m2cap);
    }
    g.cap_tiles = round_up(nt, kBins);
    g.cap_m2 = round_up(nm, kBins);
    g.desc = take(sizeof(p2::ProbDesc) * g.members.size());
    g.tiles = take(sizeof(p2::Tile) * (size_t)g.cap_tiles);
    g.m2tiles = take(sizeof(p2::Tile) * (size_t)g.cap_m2);
    g.tickets = take(sizeof(int) * p2::kTicketKinds * kBins);
    L.groups.push_back(g);
  }
  L.total = off;
  return L;
}

// Spread a (problem, subject)-ordered tile sequence over kBins contiguous
// bins of equal length (the last ones padded with empty tiles) and store them
// bin-interleaved: position u * kBins + x holds tile u of bin x.
std::vector<p2::Tile> bin_interleave(const std::vector<p2::Tile>& seq) {
  const size_t n = seq.size();
  const size_t per = std::max<size_t>(1, (n + kBins - 1) / kBins);
  std::vector<p2::Tile> out(per * kBins, p2::Tile{0, 0, 0, 0});
  for (size_t i = 0; i < n; ++i) out[(i % per) * kBins + i / per] = seq[i];
  return out;
}

// Build descriptors and tile lists for the runner's schedule, upload them and
// plan the launches.  Synchronises the stream.
int runner_plan(Runner& r) {
  r.drop_graphs();
  r.planned = false;
  for (Group& g : r.groups) {
    const int unit = std::max(1, p2::polar_tile_unit(g.R));
    const int64_t tile = (int64_t)unit * r.sched.tile_rounds;
    std::vector<p2::ProbDesc> descs;
    std::vector<p2::Tile> seq, m2seq;
    int max_hot = 0;
    int64_t maxK = 0, maxJ = 0, maxEcon = 0;
    bool warm = r.sched.warm_polar != 0;
    for (size_t q = 0; q < g.members.size(); ++q) {
      parafac2_ctx* c = r.ctxs[g.members[q]];
      p2::ProbDesc d = c->desc();
      int cap = c->plan.m2cap;
      if (r.sched.m2_tiles > 0) cap = std::min(cap, r.sched.m2_tiles);
      const int64_t nparts = mode2_parts(c->K, g.R, cap);
      const int64_t per = ceil_div(c->K, nparts);
      d.nparts = (int32_t)ceil_div(c->K, per);
      descs.push_back(d);
      for (int64_t k0 = 0; k0 < c->K; k0 += tile)
        seq.push_back(p2::Tile{(int32_t)q, 0, k0, std::min(c->K, k0 + tile)});
      for (int32_t sidx = 0; sidx < d.nparts; ++sidx) {
        const int64_t k0 = (int64_t)sidx * per;
        m2seq.push_back(p2::Tile{(int32_t)q, sidx, k0, std::min(c->K, k0 + per)});
      }
      max_hot = std::max(max_hot, c->hot);
      warm = warm && c->plan.warm;
      maxK = std::max(maxK, c->K);
      maxJ = std::max(maxJ, c->J);
      maxEcon = std::max(maxEcon, c->n_econ);
    }
    const std::vector<p2::Tile> tiles = bin_interleave(seq);
    const std::vector<p2::Tile> m2tiles = bin_interleave(m2seq);
    if ((int64_t)tiles.size() > g.cap_tiles || (int64_t)m2tiles.size() > g.cap_m2 ||
        tiles.size() > (size_t)INT_MAX / 2)
      return fail(P2_EINVAL, "tile lists exceed the planned capacity");
    HIP_TRY(hipMemcpyAsync(g.desc, descs.data(), sizeof(p2::ProbDesc) * descs.size(),
                           hipMemcpyHostToDevice, r.stream));
    HIP_TRY(hipMemcpyAsync(g.tiles, tiles.data(), sizeof(p2::Tile) * tiles.size(),
                           hipMemcpyHostToDevice, r.stream));
    HIP_TRY(hipMemcpyAsync(g.m2tiles, m2tiles.data(), sizeof(p2::Tile) * m2tiles.size(),
                           hipMemcpyHostToDevice, r.stream));
    HIP_TRY(hipStreamSynchronize(r.stream));  // the host vectors go out of scope
    p2::BatchView& b = g.bv;
    b = p2::BatchView{};
    b.R = g.R;
    b.np = (int)g.members.size();
    b.desc = g.desc;
    b.tiles = g.tiles;
    b.ntiles = (int)tiles.size();
    b.m2tiles = g.m2tiles;
    b.nm2 = (int)m2tiles.size();
    b.tickets = g.tickets;
    b.dynamic = r.sched.dynamic;
    b.warm = warm ? 1 : 0;
    b.nonneg = g.nonneg ? 1 : 0;
    b.max_hot = max_hot;
    b.m2_threads = r.sched.m2_threads;
    b.m2_blocks = r.sched.m2_blocks;
    b.maxK = maxK;
    b.maxJ = maxJ;
    b.maxEcon = maxEcon;
    HIP_TRY(p2::plan_launch(b));
  }
  r.planned = true;
  return P2_OK;
}

int runner_capture(Runner& r, int parity, int do_next);

// Plan, then capture every graph the schedule will replay, so that no
// capture happens inside a timed run.
int runner_prepare(Runner& r) {
  P2_TRY(runner_plan(r));
  if (r.sched.graph)
    for (int parity = 0; parity < 2; ++parity)
      for (int dn = 0; dn < 2; ++dn) P2_TRY(runner_capture(r, parity, dn));
  return P2_OK;
}

// Runs stmt (HIP_TRY'd launches) bracketed by events when profiling is on.
#define PHASE(ph, stmt)                                                   \
  do {                                                                    \
    hipEvent_t ea_ = nullptr, eb_ = nullptr;                              \
    if (prof) {                                                           \
      HIP_TRY(hipEventCreate(&ea_));                                      \
      HIP_TRY(hipEventCreate(&eb_));                                      \
      HIP_TRY(hipEventRecord(ea_, s));                                    \
    }                                                                     \
    stmt;                                                                 \
    if (prof) {                                                           \
      HIP_TRY(hipEventRecord(eb_, s));                                    \
      r.events.push_back({ph, ea_, eb_});                                 \
    }                                                                     \
  } while (0)

// The Procrustes step and mode-1 partial sums of the first iteration of a run.
int runner_alpha(Runner& r, int parity, hipStream_t s, bool prof) {
  for (Group& g : r.groups) {
    HIP_TRY(p2::run_reset_tickets(g.bv, s));
    HIP_TRY(p2::run_zero(g.bv, 1, s));
    PHASE(P2_PHASE_ALPHA, HIP_TRY(p2::run_alpha(g.bv, parity, g.pp, s)));
  }
  return P2_OK;
}

// One iteration after its Procrustes step: H, V and W updates, the fit and,
// if do_next, the next Procrustes step.  Launches only (may be captured).
int runner_body(Runner& r, int parity, int do_next, hipStream_t s, bool prof) {
  for (Group& g : r.groups) {
    const p2::BatchView& b = g.bv;
    HIP_TRY(p2::run_reset_tickets(b, s));
    HIP_TRY(p2::run_zero(b, 2 | 4 | 8 | 16, s));
    // mode 1 -> H
    PHASE(P2_PHASE_SOLVE_H, HIP_TRY(p2::run_gram(b, 0, parity, s));
          HIP_TRY(p2::run_solve_h(b, g.pp, s)));
    // mode 2 -> V
    PHASE(P2_PHASE_MODE2, HIP_TRY(p2::run_mode2(b, parity, s)));
    PHASE(P2_PHASE_VUPDATE, HIP_TRY(p2::run_vupdate(b, parity, s));
          if (g.nonneg) HIP_TRY(p2::run_nnls(b, parity, s));
          HIP_TRY(p2::run_gram(b, 1, parity, s)); HIP_TRY(p2::run_solve_n3(b, g.pp, s));
          HIP_TRY(p2::run_vscale(b, parity, s)));
    // mode 3 -> W, fit (+ next Procrustes step)
    if (do_next) HIP_TRY(p2::run_zero(b, 1, s));
    PHASE(P2_PHASE_GAMMA, HIP_TRY(p2::run_gamma(b, parity, do_next, g.pp, s));
          if (g.econ) HIP_TRY(p2::run_econ_fit(b, parity, s)));
    PHASE(P2_PHASE_FIT, HIP_TRY(p2::run_fit(b, s)));
  }
  return P2_OK;
}

// One iteration of the explicit-Y comparison method after its Procrustes
// step (F_k from runner_alpha): Q, Y, the three coordinate-format MTTKRPs
// with the H, V and W updates, the fit.  A runner of one context.
int runner_body_baseline(Runner& r, int parity, hipStream_t s, bool prof) {
  Group& g = r.groups[0];
  const p2::BatchView& b = g.bv;
  parafac2_ctx* c = r.ctxs[0];
  const int R = c->R;
  const p2::SmallLayout SL = p2::small_layout(R);
  double* sm = c->small();
  PHASE(P2_PHASE_ALPHA,
        HIP_TRY(p2::run_getq(R, c->X, 0, c->K, c->V(parity), c->at<double>(c->plan.F),
                             c->at<float>(c->plan.Q), 0, nullptr, s));
        HIP_TRY(p2::run_form_y(R, c->base, s)));
  HIP_TRY(p2::run_zero(b, 1 | 2 | 4 | 8 | 16, s));
  double* acc = c->at<double>(c->plan.acc);
  const int64_t nacc = std::max<int64_t>(c->J * c->LDV, c->K * R);
  PHASE(P2_PHASE_SOLVE_H, HIP_TRY(p2::run_gram(b, 0, parity, s));
        HIP_TRY(p2::run_coo_mttkrp(R, c->base, 1, c->H, c->V(parity), c->LDV, c->W, sm + SL.M1,
                                   nullptr, 0, s));
        HIP_TRY(p2::run_solve_h(b, g.pp, s)));
  PHASE(P2_PHASE_MODE2, HIP_TRY(p2::run_fill_f64(acc, nacc, 0.0, s));
        HIP_TRY(p2::run_coo_mttkrp(R, c->base, 2, c->H, nullptr, 0, c->W, nullptr, acc, c->LDV,
                                   s));
        HIP_TRY(p2::run_round_rows(acc, c->at<float>(c->plan.M2), c->J, R, c->LDV, s)));
  PHASE(P2_PHASE_VUPDATE, HIP_TRY(p2::run_vupdate(b, parity, s));
        HIP_TRY(p2::run_gram(b, 1, parity, s)); HIP_TRY(p2::run_solve_n3(b, g.pp, s));
        HIP_TRY(p2::run_vscale(b, parity, s)));
  PHASE(P2_PHASE_GAMMA, HIP_TRY(p2::run_fill_f64(acc, nacc, 0.0, s));
        HIP_TRY(p2::run_coo_mttkrp(R, c->base, 3, c->H, c->V(parity ^ 1), c->LDV, nullptr,
                                   nullptr, acc, R, s));
        HIP_TRY(p2::run_round_rows(acc, c->at<float>(c->plan.M3), c->K, R, R, s));
        HIP_TRY(p2::run_wupdate(R, b.desc, c->K, s)));
  PHASE(P2_PHASE_FIT, HIP_TRY(p2::run_fit(b, s)));
  return P2_OK;
}

int runner_capture(Runner& r, int parity, int do_next) {
  if (!r.cap) HIP_TRY(hipStreamCreateWithFlags(&r.cap, hipStreamNonBlocking));
  HIP_TRY(hipStreamBeginCapture(r.cap, hipStreamCaptureModeRelaxed));
  const int rc = runner_body(r, parity, do_next, r.cap, false);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(r.cap, &graph);
  if (rc != P2_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  HIP_TRY(e);
  const hipError_t ei = hipGraphInstantiate(&r.exec[parity][do_next], graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  HIP_TRY(ei);
  return P2_OK;
}

int runner_check(Runner& r) {
  parafac2_ctx* c0 = r.ctxs[0];
  for (parafac2_ctx* c : r.ctxs) {
    if (c->failed) return fail(P2_ESTATE, "a context is in a failed state");
    if (c->cur != c0->cur || c->have_F != c0->have_F)
      return fail(P2_ESTATE, "the contexts of the batch are not at the same point");
  }
  return P2_OK;
}

// n (<= kFitRing) iterations of every context of the runner.
int runner_iterate_n(Runner& r, int32_t n, double* fit_host, double* loss_host) {
  if (!r.planned) P2_TRY(runner_prepare(r));
  hipStream_t s = r.stream;
  const bool prof = r.profiling;
  const bool graph = r.sched.graph && !prof;
  int parity = r.ctxs[0]->cur;
  bool have_F = r.ctxs[0]->have_F;
  int qv = -1;
  for (int32_t it = 0; it < n; ++it) {
    if (!have_F) P2_TRY(runner_alpha(r, parity, s, prof));
    // the non-negative W rows are solved after the mode-3 pass, and the loss
    // terms of subjects with I_k < R need this iteration's F_k after it, so
    // in either case the next Procrustes step cannot be fused into that pass
    const int do_next = (it + 1 < n && !r.any_econ && !r.baseline) ? 1 : 0;
    if (r.baseline) {
      P2_TRY(runner_body_baseline(r, parity, s, prof));
    } else if (graph) {
      if (!r.exec[parity][do_next]) P2_TRY(runner_capture(r, parity, do_next));
      HIP_TRY(hipGraphLaunch(r.exec[parity][do_next], s));
    } else {
      P2_TRY(runner_body(r, parity, do_next, s, prof));
    }
    qv = parity;
    parity ^= 1;
    have_F = do_next != 0;
  }
  for (parafac2_ctx* c : r.ctxs) {
    c->cur = parity;
    c->qv = qv;
    c->have_F = have_F;
    c->iters_done += n;
    // publish V in the caller's column order
    HIP_TRY(p2::run_permute_rows(c->V(c->cur), c->Vuser, c->J, c->R, c->LDV, c->R,
                                 c->at<int32_t>(c->plan.perm), s));
  }
  // the last n entries of the fit and loss rings, one copy each per context
  const int nc = (int)r.ctxs.size();
  double* outs[2] = {fit_host, loss_host};
  std::vector<double> tmp[2];
  for (int which = 0; which < 2; ++which) {
    if (!outs[which]) continue;
    tmp[which].resize((size_t)n * nc);
    for (int b = 0; b < nc; ++b) {
      parafac2_ctx* c = r.ctxs[b];
      const p2::SmallLayout SL = p2::small_layout(c->R);
      const double* ring = c->small() + (which == 0 ? SL.fits : SL.losses);
      const int64_t first = (c->iters_done - n) % kFitRing;
      const int64_t n1 = std::min<int64_t>(n, kFitRing - first);
      double* dst = tmp[which].data() + (size_t)b * n;
      HIP_TRY(hipMemcpyAsync(dst, ring + first, sizeof(double) * n1, hipMemcpyDeviceToHost, s));
      if (n1 < n)
        HIP_TRY(hipMemcpyAsync(dst + n1, ring, sizeof(double) * (n - n1), hipMemcpyDeviceToHost,
                               s));
    }
  }
  if (fit_host || loss_host) {
    HIP_TRY(hipStreamSynchronize(s));
    for (int which = 0; which < 2; ++which)
      if (outs[which])
        for (int b = 0; b < nc; ++b)
          for (int32_t i = 0; i < n; ++i)
            outs[which][(size_t)i * nc + b] = tmp[which][(size_t)b * n + i];
  }
  return P2_OK;
}

int runner_iterate(Runner& r, int32_t n_iters, double* fit_host, double* loss_host = nullptr) {
  if (n_iters < 0) return fail(P2_EINVAL, "n_iters < 0");
  if (n_iters == 0) return P2_OK;
  P2_TRY(runner_check(r));
  const int nc = (int)r.ctxs.size();
  int32_t done = 0;
  while (done < n_iters) {
    const int32_t n = std::min<int32_t>(n_iters - done, kFitRing);
    const int rc = runner_iterate_n(r, n, fit_host ? fit_host + (size_t)done * nc : nullptr,
                                    loss_host ? loss_host + (size_t)done * nc : nullptr);
    if (rc != P2_OK) {
      for (parafac2_ctx* c : r.ctxs) c->failed = true;
      return rc;
    }
    done += n;
  }
  return P2_OK;
}

int runner_set_sched(Runner& r, const parafac2_sched* sched) {
  HIP_TRY(hipStreamSynchronize(r.stream));
  r.sched = normalized(sched);
  return runner_prepare(r);
}

// Coordinate search over the schedule, timed with events on real iterations.
int runner_autotune(Runner& r, int32_t iters, parafac2_sched* chosen, double* best_ms) {
  if (iters < 1) return fail(P2_EINVAL, "iters_per_trial must be >= 1");
  P2_TRY(runner_check(r));
  const bool prof = r.profiling;
  r.profiling = false;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  auto trial = [&](const parafac2_sched& sc, double* ms) -> int {
    P2_TRY(runner_set_sched(r, &sc));
    P2_TRY(runner_iterate(r, 1, nullptr));  // warm: graphs captured, caches filled
    HIP_TRY(hipEventRecord(e0, r.stream));
    P2_TRY(runner_iterate(r, iters, nullptr));
    HIP_TRY(hipEventRecord(e1, r.stream));
    HIP_TRY(hipEventSynchronize(e1));
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, e0, e1));
    *ms = (double)t / iters;
    return P2_OK;
  };
  int rc = P2_OK;
  parafac2_sched best = r.sched;
  double best_t = 1e300;
  // tile schedules: each once, then the three fastest again, interleaved and
  // twice each.  The trials run successive ALS iterations, whose cost drifts
  // as ALS converges (the eigen-solves' sweeps change), and one trial's
  // timing varies by a few per cent; interleaving the finalists puts the
  // drift on all of them alike.
  const int rounds[] = {1, 2, 4, 8, 16};
  std::vector<std::pair<double, parafac2_sched>> tiles;
  for (int dyn = 0; dyn < 2 && rc == P2_OK; ++dyn)
    for (int rd : rounds) {
      parafac2_sched sc = best;
      sc.tile_rounds = rd;
      sc.dynamic = dyn;
      double t = 0;
      rc = trial(sc, &t);
      if (rc != P2_OK) break;
      tiles.emplace_back(t, normalized(&sc));
    }
  if (rc == P2_OK) {
    std::stable_sort(tiles.begin(), tiles.end(),
                     [](const auto& a, const auto& b) { return a.first < b.first; });
    const size_t nf = std::min<size_t>(3, tiles.size());
    std::vector<double> sum(nf, 0.0);
    for (int rep = 0; rep < 2 && rc == P2_OK; ++rep)
      for (size_t i = 0; i < nf; ++i) {
        double t = 0;
        rc = trial(tiles[i].second, &t);
        if (rc != P2_OK) break;
        sum[i] += t;
      }
    if (rc == P2_OK && nf > 0) {
      size_t bi = 0;
      for (size_t i = 1; i < nf; ++i)
        if (sum[i] < sum[bi]) bi = i;
      best = tiles[bi].second;
      best_t = sum[bi] / 2;
    }
  }
  // every later candidate is timed right after the schedule it challenges,
  // which is timed again, so that both see the same state of the iteration
  auto challenge = [&](const parafac2_sched& sc) -> int {
    double tb = 0, tc = 0;
    P2_TRY(trial(best, &tb));
    P2_TRY(trial(sc, &tc));
    if (tc < tb) {
      best_t = tc;
      best = normalized(&sc);
    } else {
      best_t = tb;
    }
    return P2_OK;
  };
  int maxcap = 0;
  for (parafac2_ctx* c : r.ctxs) maxcap = std::max(maxcap, c->plan.m2cap);
  // mode-2 tiles per problem; fewer than the device's 256 CUs leave CUs idle
  const int m2s[] = {128, 256, 512};
  for (int m2 : m2s) {
    if (rc != P2_OK) break;
    if (m2 > maxcap || m2 == best.m2_tiles) continue;
    parafac2_sched sc = best;
    sc.m2_tiles = m2;
    rc = challenge(sc);
  }
  // (threads per block, blocks per CU): fewer or smaller blocks leave more of
  // the LDS for hot columns (fewer global atomics, each of which is a memory
  // transaction) at the price of occupancy
  const int m2shapes[][2] = {{0, 1}, {768, 1}, {512, 1}, {512, 2}, {768, 2}, {512, 3}, {256, 4}};
  for (const auto& sh : m2shapes) {
    if (rc != P2_OK) break;
    parafac2_sched sc = best;
    if (sc.m2_threads == sh[0] && std::max(sc.m2_blocks, 1) == sh[1]) continue;
    sc.m2_threads = sh[0];
    sc.m2_blocks = sh[1];
    rc = challenge(sc);
  }
  bool any_warm = false;
  for (parafac2_ctx* c : r.ctxs) any_warm = any_warm || c->plan.warm;
  for (int wp = 0; wp < 2 && any_warm; ++wp) {
    if (rc != P2_OK) break;
    parafac2_sched sc = best;
    if (sc.warm_polar == wp) continue;
    sc.warm_polar = wp;
    rc = challenge(sc);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  r.profiling = prof;
  if (rc != P2_OK) return rc;
  P2_TRY(runner_set_sched(r, &best));
  if (chosen) *chosen = best;
  if (best_ms) *best_ms = best_t;
  return P2_OK;
}

int resolve_profile(Runner& r) {
  if (r.events.empty()) return P2_OK;
  HIP_TRY(hipStreamSynchronize(r.stream));
  for (auto& e : r.events) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e.a, e.b));
    r.prof_ms[e.phase] += ms;
    r.prof_n[e.phase] += 1;
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  r.events.clear();
  return P2_OK;
}

int runner_set_profiling(Runner& r, int32_t on) {
  P2_TRY(resolve_profile(r));
  r.profiling = on != 0;
  for (int i = 0; i < P2_NPHASES; ++i) {
    r.prof_ms[i] = 0.0;
    r.prof_n[i] = 0;
  }
  return P2_OK;
}

int runner_get_profile(Runner& r, double* ms, int64_t* launches) {
  P2_TRY(resolve_profile(r));
  for (int i = 0; i < P2_NPHASES; ++i) {
    if (ms) ms[i] = r.prof_ms[i];
    if (launches) launches[i] = r.prof_n[i];
  }
  return P2_OK;
}

// Attach the layout's arrays (at base) to a new runner over ctxs.
int runner_make(Runner** out, parafac2_ctx* const* ctxs, int n, const RunnerLayout& L,
                unsigned char* base, hipStream_t s, const parafac2_sched* sched) {
  auto* r = new Runner();
  r->ctxs.assign(ctxs, ctxs + n);
  r->stream = s;
  r->sched = normalized(sched);
  for (const auto& lg : L.groups) {
    Group g;
    g.R = lg.R;
    g.members = lg.members;
    g.pp = ctxs[lg.members[0]]->pp;
    for (int i : lg.members)
      if (!same_params(ctxs[i]->pp, g.pp)) {
        delete r;
        return fail(P2_EINVAL, "contexts of rank %d have different tau_polar/tau_pinv/max_sweeps",
                    lg.R);
      }
    g.desc = reinterpret_cast<p2::ProbDesc*>(base + lg.desc);
    g.tiles = reinterpret_cast<p2::Tile*>(base + lg.tiles);
    g.m2tiles = reinterpret_cast<p2::Tile*>(base + lg.m2tiles);
    g.tickets = reinterpret_cast<int*>(base + lg.tickets);
    g.cap_tiles = lg.cap_tiles;
    g.cap_m2 = lg.cap_m2;
    for (int i : lg.members) {
      g.nonneg = g.nonneg || ctxs[i]->plan.nonneg;
      g.econ = g.econ || ctxs[i]->n_econ > 0;
    }
    r->any_econ = r->any_econ || g.econ;
    for (int i : lg.members) r->baseline = r->baseline || ctxs[i]->plan.baseline;
    r->groups.push_back(g);
  }
  *out = r;
  return P2_OK;
}

}  // namespace

struct parafac2_batch {
  Runner* r = nullptr;
  ~parafac2_batch() { delete r; }
};

// ---------------------------------------------------------------------------
// The explicit-Y comparison method's static structure, from the encoded
// slices: each subject's nonzeros sorted by (column, row) -- row within the
// subject and value, at the subject's nonzero positions -- and one run per
// distinct column, (start within the subject) | column << 16, at
// [runbase[k], runbase[k+1]); then the coordinate indices of Y on the device.
// Sorted on the host, one thread per range of subjects; synchronises s.
// ---------------------------------------------------------------------------
static int build_baseline(parafac2_ctx* c, hipStream_t s) {
  const Plan& P = c->plan;
  const int64_t K = c->K, nnz = c->nnz, n_rows = c->n_rows;
  std::vector<uint16_t> col(nnz), rst(n_rows), erow(nnz), ecol(nnz);
  std::vector<float> val(nnz), eval(nnz);
  std::vector<int64_t> zb(K + 1), nruns(K), runbase(K + 1);
  HIP_TRY(hipMemcpyAsync(col.data(), c->at<uint16_t>(P.col16), sizeof(uint16_t) * nnz,
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(rst.data(), c->at<uint16_t>(P.rstart), sizeof(uint16_t) * n_rows,
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(val.data(), c->at<float>(P.val), sizeof(float) * nnz,
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(zb.data(), c->at<int64_t>(P.zbase), sizeof(int64_t) * (K + 1),
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const std::vector<int64_t>& rb = c->subj_host;
  auto sort_range = [&](int64_t k0, int64_t k1) {
    std::vector<uint32_t> key, idx;
    for (int64_t k = k0; k < k1; ++k) {
      const int64_t z0 = zb[k];
      const int n = (int)(zb[k + 1] - z0);
      const int64_t r0 = rb[k];
      const int nr = (int)(rb[k + 1] - r0);
      key.resize(n);
      idx.resize(n);
      for (int i = 0; i < nr; ++i) {
        const int e1 = i + 1 < nr ? (int)rst[r0 + i + 1] : n;
        for (int z = rst[r0 + i]; z < e1; ++z) key[z] = ((uint32_t)col[z0 + z] << 16) | (uint32_t)i;
      }
      std::iota(idx.begin(), idx.end(), 0u);
      std::sort(idx.begin(), idx.end(), [&](uint32_t a, uint32_t b) { return key[a] < key[b]; });
      int64_t runs = 0;
      for (int e = 0; e < n; ++e) {
        const uint32_t kk = key[idx[e]];
        erow[z0 + e] = (uint16_t)(kk & 0xffffu);
        ecol[z0 + e] = (uint16_t)(kk >> 16);
        eval[z0 + e] = val[z0 + idx[e]];
        if (e == 0 || ecol[z0 + e] != ecol[z0 + e - 1]) ++runs;
      }
      nruns[k] = runs;
    }
  };
  const int nth =
      (int)std::max<unsigned>(1, std::min<unsigned>(16, std::thread::hardware_concurrency()));
  {
    std::vector<std::thread> th;
    for (int t = 0; t < nth; ++t) th.emplace_back(sort_range, K * t / nth, K * (t + 1) / nth);
    for (auto& x : th) x.join();
  }
  runbase[0] = 0;
  for (int64_t k = 0; k < K; ++k) runbase[k + 1] = runbase[k] + nruns[k];
  std::vector<uint32_t> runs(std::max<int64_t>(runbase[K], 1));
  auto run_range = [&](int64_t k0, int64_t k1) {
    for (int64_t k = k0; k < k1; ++k) {
      const int64_t z0 = zb[k];
      const int n = (int)(zb[k + 1] - z0);
      int64_t u = runbase[k];
      for (int e = 0; e < n; ++e)
        if (e == 0 || ecol[z0 + e] != ecol[z0 + e - 1])
          runs[u++] = (uint32_t)e | ((uint32_t)ecol[z0 + e] << 16);
    }
  };
  {
    std::vector<std::thread> th;
    for (int t = 0; t < nth; ++t) th.emplace_back(run_range, K * t / nth, K * (t + 1) / nth);
    for (auto& x : th) x.join();
  }
  HIP_TRY(hipMemcpyAsync(c->at<uint16_t>(P.erow), erow.data(), sizeof(uint16_t) * nnz,
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(c->at<float>(P.eval), eval.data(), sizeof(float) * nnz,
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(c->at<uint32_t>(P.runs), runs.data(), sizeof(uint32_t) * runbase[K],
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(c->at<int64_t>(P.runbase), runbase.data(), sizeof(int64_t) * (K + 1),
                         hipMemcpyHostToDevice, s));
  p2::BaselineView& v = c->base;
  v.zbase = c->at<int64_t>(P.zbase);
  v.rbase = c->at<int64_t>(P.rbase);
  v.erow = c->at<uint16_t>(P.erow);
  v.eval = c->at<float>(P.eval);
  v.runs = c->at<uint32_t>(P.runs);
  v.runbase = c->at<int64_t>(P.runbase);
  v.nruns = runbase[K];
  v.yr = c->at<int32_t>(P.yr);
  v.yj = c->at<int32_t>(P.yj);
  v.yk = c->at<int32_t>(P.yk);
  v.yv = c->at<float>(P.yv);
  v.ny = (int64_t)c->R * runbase[K];
  v.Q = c->at<float>(P.Q);
  HIP_TRY(p2::run_y_index(c->R, v, K, s));
  HIP_TRY(hipStreamSynchronize(s));  // the host vectors go out of scope
  return P2_OK;
}

// ---------------------------------------------------------------------------
// host-side validation
// ---------------------------------------------------------------------------

static int validate_host_impl(const parafac2_csr* X, int32_t R, std::string& msg) {
  char buf[256];
  if (!X) { msg = "X is NULL"; return P2_EINVAL; }
  if (R < 1) { msg = "R must be >= 1"; return P2_EINVAL; }
  if (X->K < 1 || X->J < 1 || X->n_rows < 0 || X->nnz < 0) {
    msg = "K and J must be >= 1, n_rows and nnz >= 0";
    return P2_EINVAL;
  }
  if (!p2::rank_supported(R)) {
    snprintf(buf, sizeof(buf), "R=%d is not built (supported: 1-6, 8, 10, 12, 16, 20, 32, 40)", R);
    msg = buf;
    return P2_ENOTSUP;
  }
  if (X->J > 65536) { msg = "J > 65536 is not supported"; return P2_ENOTSUP; }
  if (X->K > INT32_MAX) { msg = "K > 2^31 - 1 is not supported"; return P2_ENOTSUP; }
  if (!X->subj_ptr || !X->row_ptr || (X->nnz > 0 && (!X->col || !X->val))) {
    msg = "NULL array";
    return P2_EINVAL;
  }
  if (X->subj_ptr[0] != 0 || X->subj_ptr[X->K] != X->n_rows) {
    msg = "subj_ptr must start at 0 and end at n_rows";
    return P2_EINVAL;
  }
  if (X->row_ptr[0] != 0 || X->row_ptr[X->n_rows] != X->nnz) {
    msg = "row_ptr must start at 0 and end at nnz";
    return P2_EINVAL;
  }
  for (int64_t k = 0; k < X->K; ++k) {
    const int64_t a = X->subj_ptr[k], b = X->subj_ptr[k + 1];
    if (b < a) { snprintf(buf, sizeof(buf), "subj_ptr decreases at subject %lld", (long long)k); msg = buf; return P2_EINVAL; }
    if (b - a < 1) {
      snprintf(buf, sizeof(buf), "subject %lld has no rows", (long long)k);
      msg = buf;
      return P2_EINVAL;
    }
    if (b - a > 65535) { msg = "I_k > 65535 is not supported"; return P2_ENOTSUP; }
    if (X->row_ptr[b] - X->row_ptr[a] > 65535) {
      msg = "more than 65535 nonzeros in one subject is not supported";
      return P2_ENOTSUP;
    }
  }
  for (int64_t i = 0; i < X->n_rows; ++i) {
    const int64_t a = X->row_ptr[i], b = X->row_ptr[i + 1];
    if (b < a) { snprintf(buf, sizeof(buf), "row_ptr decreases at row %lld", (long long)i); msg = buf; return P2_EINVAL; }
    int prev = -1;
    for (int64_t z = a; z < b; ++z) {
      const int c = X->col[z];
      if (c < 0 || c >= X->J) {
        snprintf(buf, sizeof(buf), "column %d out of range at nonzero %lld", c, (long long)z);
        msg = buf;
        return P2_EINVAL;
      }
      if (c <= prev) {
        snprintf(buf, sizeof(buf), "columns not strictly increasing in row %lld", (long long)i);
        msg = buf;
        return P2_EINVAL;
      }
      prev = c;
      if (!std::isfinite(X->val[z])) {
        snprintf(buf, sizeof(buf), "non-finite value at nonzero %lld", (long long)z);
        msg = buf;
        return P2_EINVAL;
      }
    }
  }
  msg.clear();
  return P2_OK;
}

// ---------------------------------------------------------------------------
// Device scratch of parafac2_project_noalloc: the model state of one call
// (padded V, H, V^T V, H^T H, N3, N3^+, row map), at most kNoAllocScratchBytes.
// Each device holds its own copy for the life of the process.  Host code
// never uses the array's name as an address: the device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocScratchBytes = size_t(8) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;

static int noalloc_scratch(void** out) {
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};  // device -> address of its scratch copy
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(P2_ENOTSUP, "device %d: at most %d devices", dev,
                                                 kMaxDevices);
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(P2_EDEVICE, "no device address for the scratch array");
    addr[dev] = p;
  }
  *out = addr[dev];
  return P2_OK;
}

extern "C" {

int parafac2_abi_version(void) { return PARAFAC2_ABI_VERSION; }

const char* parafac2_last_error(void) { return p2host::last_error().c_str(); }

int parafac2_validate_host(const parafac2_csr* host_X, int32_t R, char* msg, size_t msg_len) {
  std::string m;
  const int rc = validate_host_impl(host_X, R, m);
  if (msg && msg_len) {
    std::strncpy(msg, m.c_str(), msg_len - 1);
    msg[msg_len - 1] = 0;
  }
  if (rc != P2_OK) p2host::last_error() = m;
  return rc;
}

int parafac2_workspace_size(const parafac2_csr* X, int32_t R, const parafac2_opts* opts,
                            size_t* bytes) {
  if (!X || !bytes) return fail(P2_EINVAL, "NULL argument");
  if (R < 1 || X->K < 1 || X->J < 1 || X->n_rows < 0 || X->nnz < 0)
    return fail(P2_EINVAL, "bad sizes");
  *bytes = make_plan(X->K, X->J, X->n_rows, X->nnz, R, opts).total;
  return P2_OK;
}

int parafac2_init(parafac2_ctx** out, const parafac2_csr* X, int32_t R, double* H, float* V,
                  float* W, void* workspace, size_t ws_bytes, void* stream,
                  const parafac2_opts* opts) {
  if (!out) return fail(P2_EINVAL, "out is NULL");
  *out = nullptr;
  if (!X || !H || !V || !W || !workspace) return fail(P2_EINVAL, "NULL argument");
  if (R < 1 || X->K < 1 || X->J < 1 || X->n_rows < 0 || X->nnz < 0)
    return fail(P2_EINVAL, "K, J, R must be >= 1");
  if (!p2::rank_supported(R)) return fail(P2_ENOTSUP, "R=%d is not built", R);
  if (X->J > 65536) return fail(P2_ENOTSUP, "J > 65536 is not supported");
  if (X->K > INT32_MAX) return fail(P2_ENOTSUP, "K > 2^31 - 1 is not supported");
  if (X->n_rows < X->K) return fail(P2_EINVAL, "n_rows < K: some subject has no rows");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return fail(P2_EINVAL, "workspace must be 256-byte aligned");
  const Plan plan = make_plan(X->K, X->J, X->n_rows, X->nnz, R, opts);
  if (ws_bytes < plan.total)
    return fail(P2_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, plan.total);

  auto* c = new parafac2_ctx();
  c->K = X->K;
  c->J = X->J;
  c->n_rows = X->n_rows;
  c->nnz = X->nnz;
  c->R = R;
  c->LDV = ldv_of(R);
  c->stream = reinterpret_cast<hipStream_t>(stream);
  c->H = H;
  c->Vuser = V;
  c->W = W;
  c->ws = reinterpret_cast<unsigned char*>(workspace);
  c->plan = plan;
  c->pp = polar_params(opts, R);
  c->hot = plan.hot;

  auto cleanup = [&](int rc) {
    delete c->own;
    delete c;
    return rc;
  };
  hipStream_t s = c->stream;
  int* err = c->at<int>(plan.err);
  int64_t* zbase = c->at<int64_t>(plan.zbase);
  int64_t* rbase = c->at<int64_t>(plan.rbase);
#define INIT_TRY(expr)                                                               \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return cleanup(fail(P2_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)));     \
  } while (0)
  INIT_TRY(hipMemsetAsync(err, 0, sizeof(int) * 4, s));
  INIT_TRY(p2::run_validate(X->subj_ptr, X->row_ptr, X->col, X->val, X->K, X->n_rows, X->nnz,
                            X->J, 1, err, zbase, rbase, s));
  int herr = 0;
  INIT_TRY(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s));
  INIT_TRY(hipStreamSynchronize(s));
  if (herr) {
    if (herr & (1 | 16)) return cleanup(fail(P2_EINVAL, "row_ptr/subj_ptr are not monotone offsets"));
    if (herr & 2) return cleanup(fail(P2_EINVAL, "column index out of [0, J)"));
    if (herr & 4) return cleanup(fail(P2_EINVAL, "columns not strictly increasing within a row"));
    if (herr & 8) return cleanup(fail(P2_EINVAL, "non-finite value"));
    if (herr & 32) return cleanup(fail(P2_EINVAL, "a subject has no rows"));
    if (herr & 64) return cleanup(fail(P2_ENOTSUP, "a subject has more than 65535 rows"));
    if (herr & 128) return cleanup(fail(P2_ENOTSUP, "a subject has more than 65535 nonzeros"));
    return cleanup(fail(P2_EINVAL, "invalid input (code %d)", herr));
  }
  // subject offsets on the host (for get_q)
  c->subj_host.resize(X->K + 1);
  INIT_TRY(hipMemcpyAsync(c->subj_host.data(), X->subj_ptr, sizeof(int64_t) * (X->K + 1),
                          hipMemcpyDeviceToHost, s));
  // column frequencies -> relabelling (most frequent first, ties by id)
  uint32_t* hist = c->at<uint32_t>(plan.hist);
  INIT_TRY(hipMemsetAsync(hist, 0, sizeof(uint32_t) * X->J, s));
  INIT_TRY(p2::run_col_hist(X->col, X->nnz, X->J, hist, s));
  std::vector<uint32_t> hh(X->J);
  INIT_TRY(hipMemcpyAsync(hh.data(), hist, sizeof(uint32_t) * X->J, hipMemcpyDeviceToHost, s));
  INIT_TRY(hipStreamSynchronize(s));
  std::vector<int32_t> perm(X->J), rank(X->J);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(),
                   [&](int32_t a, int32_t b) { return hh[a] > hh[b]; });
  for (int64_t i = 0; i < X->J; ++i) rank[perm[i]] = (int32_t)i;
  INIT_TRY(hipMemcpyAsync(c->at<int32_t>(plan.perm), perm.data(), sizeof(int32_t) * X->J,
                          hipMemcpyHostToDevice, s));
  INIT_TRY(hipMemcpyAsync(c->at<int32_t>(plan.rank), rank.data(), sizeof(int32_t) * X->J,
                          hipMemcpyHostToDevice, s));
  // Subject order of the per-subject passes.  The groups of a wave take
  // consecutive positions and the wave runs until its largest subject is
  // done, so within each window of kOrderWindow subjects the subjects go by
  // decreasing row count (stable).  Windows are short against an XCD bin and
  // a mode-2 tile, which keep their mix of sizes; the Procrustes tiles (about
  // a hundred subjects) get runs of similar sizes, which the ticket schedule
  // balances.
  std::vector<int32_t> order(X->K);
  std::iota(order.begin(), order.end(), 0);
  for (int64_t w0 = 0; w0 < X->K; w0 += kOrderWindow) {
    const int64_t w1 = std::min<int64_t>(X->K, w0 + kOrderWindow);
    std::stable_sort(order.begin() + w0, order.begin() + w1, [&](int32_t a, int32_t b) {
      return c->subj_host[a + 1] - c->subj_host[a] > c->subj_host[b + 1] - c->subj_host[b];
    });
  }
  INIT_TRY(hipMemcpyAsync(c->at<int32_t>(plan.order), order.data(), sizeof(int32_t) * X->K,
                          hipMemcpyHostToDevice, s));
  // subjects with fewer rows than R get the economy Procrustes factor, whose
  // loss terms need their own pass
  std::vector<int32_t> econ;
  for (int64_t k = 0; k < X->K; ++k)
    if (c->subj_host[k + 1] - c->subj_host[k] < R) econ.push_back((int32_t)k);
  c->n_econ = (int64_t)econ.size();
  if (!econ.empty())
    INIT_TRY(hipMemcpyAsync(c->at<int32_t>(plan.econ), econ.data(), sizeof(int32_t) * econ.size(),
                            hipMemcpyHostToDevice, s));
  double* sm = c->small();
  const p2::SmallLayout SL = p2::small_layout(R);
  INIT_TRY(p2::run_fill_f64(sm, SL.total, 0.0, s));
  INIT_TRY(p2::run_fill_f64(reinterpret_cast<double*>(c->at<int64_t>(plan.iter)), 1, 0.0, s));
  INIT_TRY(p2::run_encode(X->subj_ptr, X->row_ptr, X->col, X->val, X->K, X->nnz,
                          c->at<int32_t>(plan.rank), c->at<uint16_t>(plan.rstart),
                          c->at<uint16_t>(plan.nzrow), c->at<uint16_t>(plan.col16), c->at<float>(plan.val), sm + SL.nx2, s));
  if (plan.warm) INIT_TRY(p2::run_eye_basis(c->at<float>(plan.E), X->K, R, s));
  INIT_TRY(p2::run_fill_f32(c->V(0), X->J * c->LDV, 0.f, s));
  INIT_TRY(p2::run_fill_f32(c->V(1), X->J * c->LDV, 0.f, s));
  INIT_TRY(p2::run_permute_rows(V, c->V(0), X->J, R, R, c->LDV, c->at<int32_t>(plan.rank), s));
  INIT_TRY(p2::run_gram_rows(R, c->V(0), X->J, c->LDV, sm + SL.VtV, s));
  INIT_TRY(hipStreamSynchronize(s));  // host vectors above go out of scope
  if (plan.baseline) {
    if (c->n_econ > 0 || plan.nonneg)
      return cleanup(fail(P2_ENOTSUP, "the explicit-Y comparison method needs I_k >= R and no "
                                      "constraints"));
    const int rb = build_baseline(c, s);
    if (rb != P2_OK) return cleanup(rb);
  }
  c->X.zbase = zbase;
  c->X.rbase = rbase;
  c->X.rstart = c->at<uint16_t>(plan.rstart);
  c->X.nzrow = c->at<uint16_t>(plan.nzrow);
  c->X.col = c->at<uint16_t>(plan.col16);
  c->X.val = c->at<float>(plan.val);
  c->cur = 0;
  c->have_F = false;
  {
    RunnerLayout L;
    RunnerLayout::G g;
    g.R = R;
    g.members = {0};
    g.desc = plan.desc;
    g.tiles = plan.tiles;
    g.m2tiles = plan.m2tiles;
    g.tickets = plan.tickets;
    g.cap_tiles = plan.cap_tiles;
    g.cap_m2 = plan.cap_m2;
    L.groups.push_back(g);
    parafac2_ctx* self = c;
    const int rc = runner_make(&c->own, &self, 1, L, c->ws, s, opts ? &opts->sched : nullptr);
    if (rc != P2_OK) return cleanup(rc);
    const int rp = runner_prepare(*c->own);
    if (rp != P2_OK) return cleanup(rp);
  }
  *out = c;
  p2host::last_error().clear();
  return P2_OK;
#undef INIT_TRY
}

int parafac2_iterate(parafac2_ctx* c, int32_t n_iters, double* fit_host, double* loss_host) {
  if (!c) return fail(P2_EINVAL, "ctx is NULL");
  if (c->failed) return fail(P2_ESTATE, "context is in a failed state");
  return runner_iterate(*c->own, n_iters, fit_host, loss_host);
}

int parafac2_iterate_until(parafac2_ctx* c, int32_t max_iters, double tol, int32_t* n_done,
                           double* fit_host, double* loss_host) {
  if (!c || !n_done) return fail(P2_EINVAL, "NULL argument");
  if (c->failed) return fail(P2_ESTATE, "context is in a failed state");
  if (max_iters < 0 || !(tol >= 0.0)) return fail(P2_EINVAL, "max_iters < 0 or tol not >= 0");
  *n_done = 0;
  double prev = 0.0;
  for (int32_t it = 0; it < max_iters; ++it) {
    double fit = 0.0, loss = 0.0;
    P2_TRY(runner_iterate(*c->own, 1, &fit, &loss));
    if (fit_host) fit_host[it] = fit;
    if (loss_host) loss_host[it] = loss;
    *n_done = it + 1;
    // relative decrease of the loss between consecutive iterations; a loss
    // that reaches zero has converged as well
    if (it > 0 && (loss <= 0.0 || std::fabs(prev - loss) <= tol * std::fabs(prev))) break;
    prev = loss;
  }
  return P2_OK;
}

int parafac2_get_mttkrp(parafac2_ctx* c, double* M1, float* M2, float* M3) {
  if (!c) return fail(P2_EINVAL, "ctx is NULL");
  if (c->failed) return fail(P2_ESTATE, "context is in a failed state");
  if (c->iters_done == 0) return fail(P2_ESTATE, "no iteration has run");
  const Plan& P = c->plan;
  hipStream_t s = c->stream;
  if (M1)
    HIP_TRY(hipMemcpyAsync(M1, c->small() + p2::small_layout(c->R).M1,
                           sizeof(double) * c->R * c->R, hipMemcpyDeviceToDevice, s));
  if (M2)
    HIP_TRY(p2::run_permute_rows(c->at<float>(P.M2), M2, c->J, c->R, c->LDV, c->R,
                                 c->at<int32_t>(P.perm), s));
  if (M3)
    HIP_TRY(hipMemcpyAsync(M3, c->at<float>(P.M3), sizeof(float) * c->K * c->R,
                           hipMemcpyDeviceToDevice, s));
  return P2_OK;
}

static int get_q_or_u(parafac2_ctx* c, int64_t k0, int64_t k1, float* Q, bool u) {
  if (!c || !Q) return fail(P2_EINVAL, "NULL argument");
  if (c->failed) return fail(P2_ESTATE, "context is in a failed state");
  if (k0 < 0 || k1 > c->K || k0 > k1) return fail(P2_EINVAL, "bad subject range");
  if (c->have_F || c->qv < 0)
    return fail(P2_ESTATE, "no completed Procrustes step to report");
  if (k0 == k1) return P2_OK;
  HIP_TRY(p2::run_getq(c->R, c->X, k0, k1, c->V(c->qv), c->at<double>(c->plan.F), Q,
                       c->subj_host[k0], u ? c->H : nullptr, c->stream));
  return P2_OK;
}

int parafac2_get_q(parafac2_ctx* c, int64_t k0, int64_t k1, float* Q) {
  return get_q_or_u(c, k0, k1, Q, false);
}

int parafac2_get_u(parafac2_ctx* c, int64_t k0, int64_t k1, float* U) {
  return get_q_or_u(c, k0, k1, U, true);
}

int parafac2_set_profiling(parafac2_ctx* c, int32_t on) {
  if (!c) return fail(P2_EINVAL, "ctx is NULL");
  return runner_set_profiling(*c->own, on);
}

int parafac2_get_profile(parafac2_ctx* c, double* ms, int64_t* launches) {
  if (!c) return fail(P2_EINVAL, "ctx is NULL");
  return runner_get_profile(*c->own, ms, launches);
}

int parafac2_set_sched(parafac2_ctx* c, const parafac2_sched* sched) {
  if (!c) return fail(P2_EINVAL, "ctx is NULL");
  if (c->failed) return fail(P2_ESTATE, "context is in a failed state");
  return runner_set_sched(*c->own, sched);
}

int parafac2_autotune(parafac2_ctx* c, int32_t iters_per_trial, parafac2_sched* chosen,
                      double* best_ms) {
  if (!c) return fail(P2_EINVAL, "ctx is NULL");
  if (c->failed) return fail(P2_ESTATE, "context is in a failed state");
  return runner_autotune(*c->own, iters_per_trial, chosen, best_ms);
}

int parafac2_launch_config(int32_t R, int32_t kernel, int32_t* threads, int64_t* lds_bytes,
                           int32_t* max_hot) {
  if (!p2::rank_supported(R)) return fail(P2_ENOTSUP, "R=%d is not built", R);
  if (kernel < 0 || kernel > 4) return fail(P2_EINVAL, "kernel id %d", kernel);
  if (threads) *threads = p2::launch_threads(R, kernel);
  if (lds_bytes) *lds_bytes = (int64_t)p2::launch_lds(R, kernel);
  if (max_hot) *max_hot = p2::mode2_max_hot(R);
  return P2_OK;
}

void parafac2_destroy(parafac2_ctx* c) {
  if (!c) return;
  delete c->own;
  delete c;
}

// ---------------------------------------------------------------------------
// batches
// ---------------------------------------------------------------------------

static int check_ctx_list(parafac2_ctx* const* ctxs, int32_t n) {
  if (!ctxs || n < 1) return fail(P2_EINVAL, "need at least one context");
  for (int32_t i = 0; i < n; ++i) {
    if (!ctxs[i]) return fail(P2_EINVAL, "context %d is NULL", i);
    for (int32_t j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return fail(P2_EINVAL, "context %d appears twice", i);
  }
  return P2_OK;
}

int parafac2_batch_workspace_size(parafac2_ctx* const* ctxs, int32_t n, size_t* bytes) {
  if (!bytes) return fail(P2_EINVAL, "NULL argument");
  P2_TRY(check_ctx_list(ctxs, n));
  *bytes = runner_layout(ctxs, n).total;
  return P2_OK;
}

int parafac2_batch_create(parafac2_batch** out, parafac2_ctx* const* ctxs, int32_t n,
                          void* workspace, size_t ws_bytes, void* stream,
                          const parafac2_sched* sched) {
  if (!out) return fail(P2_EINVAL, "out is NULL");
  *out = nullptr;
  P2_TRY(check_ctx_list(ctxs, n));
  if (!workspace) return fail(P2_EINVAL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return fail(P2_EINVAL, "workspace must be 256-byte aligned");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  for (int32_t i = 0; i < n; ++i)
    if (ctxs[i]->stream != s) return fail(P2_EINVAL, "context %d has another stream", i);
  for (int32_t i = 0; i < n; ++i)
    if (ctxs[i]->plan.baseline)
      return fail(P2_ENOTSUP, "context %d runs the explicit-Y comparison method", i);
  const RunnerLayout L = runner_layout(ctxs, n);
  if (ws_bytes < L.total)
    return fail(P2_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, L.total);
  auto* b = new parafac2_batch();
  int rc = runner_make(&b->r, ctxs, n, L, reinterpret_cast<unsigned char*>(workspace), s, sched);
  if (rc == P2_OK) rc = runner_prepare(*b->r);
  if (rc != P2_OK) {
    delete b;
    return rc;
  }
  *out = b;
  return P2_OK;
}

int parafac2_batch_iterate(parafac2_batch* b, int32_t n_iters, double* fit_host,
                           double* loss_host) {
  if (!b) return fail(P2_EINVAL, "batch is NULL");
  return runner_iterate(*b->r, n_iters, fit_host, loss_host);
}

int parafac2_batch_set_sched(parafac2_batch* b, const parafac2_sched* sched) {
  if (!b) return fail(P2_EINVAL, "batch is NULL");
  return runner_set_sched(*b->r, sched);
}

int parafac2_batch_autotune(parafac2_batch* b, int32_t iters_per_trial, parafac2_sched* chosen,
                            double* best_ms) {
  if (!b) return fail(P2_EINVAL, "batch is NULL");
  return runner_autotune(*b->r, iters_per_trial, chosen, best_ms);
}

int parafac2_batch_set_profiling(parafac2_batch* b, int32_t on) {
  if (!b) return fail(P2_EINVAL, "batch is NULL");
  return runner_set_profiling(*b->r, on);
}

int parafac2_batch_get_profile(parafac2_batch* b, double* ms, int64_t* launches) {
  if (!b) return fail(P2_EINVAL, "batch is NULL");
  return runner_get_profile(*b->r, ms, launches);
}

void parafac2_batch_destroy(parafac2_batch* b) { delete b; }

// ---------------------------------------------------------------------------
// projection model
// ---------------------------------------------------------------------------

static void model_layout(parafac2_model* m) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  const size_t RR = (size_t)m->R * m->R;
  m->oV = take(sizeof(float) * m->J * m->LDV);
  m->oH = take(sizeof(double) * RR);
  m->oN3 = take(sizeof(double) * RR);
  m->oN3p = take(sizeof(double) * RR);
  m->oVtV = take(sizeof(double) * RR);
  m->oHtH = take(sizeof(double) * RR);
  m->oMap = take(sizeof(int32_t) * m->J);
  m->total = off;
}

int parafac2_model_workspace_size(int64_t J, int32_t R, size_t* bytes) {
  if (!bytes || J < 1 || R < 1) return fail(P2_EINVAL, "bad arguments");
  parafac2_model m;
  m.J = J;
  m.R = R;
  m.LDV = ldv_of(R);
  model_layout(&m);
  *bytes = m.total;
  return P2_OK;
}

// Enqueue the model state into m->ws on stream s: V (J x R) copied into rows
// of LDV floats, H, V^T V, H^T H, N3 = (V^T V) * (H^T H) and N3^+.  No
// allocation and no synchronisation.
static hipError_t model_fill(parafac2_model* m, const float* V, const double* H, hipStream_t s) {
  const int64_t J = m->J;
  const int R = m->R;
  float* Vm = reinterpret_cast<float*>(m->ws + m->oV);
  double* Hm = reinterpret_cast<double*>(m->ws + m->oH);
  double* VtV = reinterpret_cast<double*>(m->ws + m->oVtV);
  int32_t* map = reinterpret_cast<int32_t*>(m->ws + m->oMap);
  hipError_t e;
  if ((e = p2::run_fill_f32(Vm, J * m->LDV, 0.f, s)) != hipSuccess) return e;
  if ((e = p2::run_iota(map, J, s)) != hipSuccess) return e;
  if ((e = p2::run_permute_rows(V, Vm, J, R, R, m->LDV, map, s)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(Hm, H, sizeof(double) * R * R, hipMemcpyDeviceToDevice, s)) != hipSuccess)
    return e;
  if ((e = p2::run_fill_f64(VtV, (int64_t)R * R, 0.0, s)) != hipSuccess) return e;
  if ((e = p2::run_gram_rows(R, Vm, J, m->LDV, VtV, s)) != hipSuccess) return e;
  return p2::run_model_prep(R, VtV, Hm, reinterpret_cast<double*>(m->ws + m->oHtH),
                            reinterpret_cast<double*>(m->ws + m->oN3),
                            reinterpret_cast<double*>(m->ws + m->oN3p), m->pp, s);
}

// Checks of a projection request against model m (shapes and pointers).
static int check_request(const parafac2_model* m, const parafac2_csr* req, int32_t n_steps,
                         const float* w_out) {
  if (!req || !w_out) return fail(P2_EINVAL, "NULL argument");
  if (req->J != m->J) return fail(P2_EINVAL, "request J=%lld != model J=%lld",
                                  (long long)req->J, (long long)m->J);
  if (req->K < 0 || n_steps < 0) return fail(P2_EINVAL, "bad sizes");
  if (req->K > 0 && (!req->subj_ptr || !req->row_ptr || (req->nnz > 0 && (!req->col || !req->val))))
    return fail(P2_EINVAL, "NULL array");
  return P2_OK;
}

static int project_launch(const parafac2_model* m, const parafac2_csr* req, int32_t n_steps,
                          const float* w0, float* Q_out, float* w_out, double* loss_out,
                          hipStream_t s) {
  p2::XRaw X{req->subj_ptr, req->row_ptr, req->col, req->val};
  HIP_TRY(p2::run_project(m->R, X, req->K, reinterpret_cast<const float*>(m->ws + m->oV),
                          reinterpret_cast<const double*>(m->ws + m->oH),
                          reinterpret_cast<const double*>(m->ws + m->oN3),
                          reinterpret_cast<const double*>(m->ws + m->oN3p), n_steps, w0, Q_out,
                          w_out, loss_out, m->pp, s));
  return P2_OK;
}

int parafac2_model_create(parafac2_model** out, int64_t J, int32_t R, const float* V,
                          const double* H, void* workspace, size_t ws_bytes, void* stream) {
  if (!out) return fail(P2_EINVAL, "out is NULL");
  *out = nullptr;
  if (!V || !H || !workspace || J < 1 || R < 1) return fail(P2_EINVAL, "bad arguments");
  if (!p2::rank_supported(R)) return fail(P2_ENOTSUP, "R=%d is not built", R);
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return fail(P2_EINVAL, "workspace must be 256-byte aligned");
  auto* m = new parafac2_model();
  m->J = J;
  m->R = R;
  m->LDV = ldv_of(R);
  m->stream = reinterpret_cast<hipStream_t>(stream);
  m->ws = reinterpret_cast<unsigned char*>(workspace);
  m->pp = polar_params(nullptr, R);
  model_layout(m);
  if (ws_bytes < m->total) {
    const size_t need = m->total;
    delete m;
    return fail(P2_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, need);
  }
  hipError_t e = model_fill(m, V, H, m->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(m->stream);
  if (e != hipSuccess) {
    delete m;
    return fail(P2_EDEVICE, "model state: %s", hipGetErrorString(e));
  }
  *out = m;
  return P2_OK;
}

int parafac2_project(parafac2_model* m, const parafac2_csr* req, int32_t n_steps, const float* w0,
                     float* Q_out, float* w_out, double* loss_out, void* stream) {
  if (!m) return fail(P2_EINVAL, "NULL argument");
  P2_TRY(check_request(m, req, n_steps, w_out));
  if (req->K == 0) return P2_OK;
  hipStream_t s = stream ? reinterpret_cast<hipStream_t>(stream) : m->stream;
  return project_launch(m, req, n_steps, w0, Q_out, w_out, loss_out, s);
}

void parafac2_model_destroy(parafac2_model* m) { delete m; }

int parafac2_project_noalloc(int64_t J, int32_t R, const float* V, const double* H,
                             const parafac2_csr* req, int32_t n_steps, const float* w0,
                             float* Q_out, float* w_out, double* loss_out, void* stream) {
  if (!V || !H || J < 1 || R < 1) return fail(P2_EINVAL, "bad arguments");
  if (!p2::rank_supported(R)) return fail(P2_ENOTSUP, "R=%d is not built", R);
  parafac2_model m;  // on the stack: its state lives in the device scratch array
  m.J = J;
  m.R = R;
  m.LDV = ldv_of(R);
  m.pp = polar_params(nullptr, R);
  model_layout(&m);
  if (m.total > kNoAllocScratchBytes)
    return fail(P2_EINVAL, "J=%lld, R=%d need %zu bytes of model state, more than the %zu bytes "
                "of the no-allocation scratch", (long long)J, R, m.total, kNoAllocScratchBytes);
  P2_TRY(check_request(&m, req, n_steps, w_out));
  void* base = nullptr;
  P2_TRY(noalloc_scratch(&base));
  m.ws = reinterpret_cast<unsigned char*>(base);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const hipError_t e = model_fill(&m, V, H, s);
  if (e != hipSuccess) return fail(P2_EDEVICE, "model state: %s", hipGetErrorString(e));
  if (req->K == 0) return P2_OK;
  return project_launch(&m, req, n_steps, w0, Q_out, w_out, loss_out, s);
}

}  // extern "C"
