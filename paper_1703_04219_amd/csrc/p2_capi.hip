// Host runtime and C ABI of the PARAFAC2-ALS hot path (see include/parafac2.h).
//
// The context owns no device memory: every buffer is carved out of the
// caller's workspace by a fixed plan (Plan below).  Init validates the input
// on the device, relabels columns by decreasing frequency (hot columns get the
// smallest ids, so the mode-2 kernel can keep their partial sums in LDS with a
// single range test), re-encodes the slices compactly (16-bit columns, 16-bit
// subject-relative row starts) and copies V into the internal column order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/parafac2.h"
#include "p2_device.h"
#include "p2_kernels.h"

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

inline int ldv_of(int R) { return (R + 3) & ~3; }

constexpr int kFitRing = 1024;

// Offsets of every piece of the context workspace.
struct Plan {
  size_t zbase, rbase, rstart, col16, val, rank, perm, hist, V[2], F, M2, M2part, M3, small, err,
      total;
  // small block (doubles)
  size_t oM1, oWtW, oVtV, oVtVraw, oHtH, oN2p, oN3, oN3p, oInv, oFitAcc, oNx2, oFits, nsmall;
};

Plan make_plan(int64_t K, int64_t J, int64_t n_rows, int64_t nnz, int R) {
  Plan p{};
  const int64_t LDV = ldv_of(R);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  p.zbase = take(sizeof(int64_t) * (K + 1));
  p.rbase = take(sizeof(int64_t) * (K + 1));
  p.rstart = take(sizeof(uint16_t) * (size_t)std::max<int64_t>(n_rows, 1));
  p.col16 = take(sizeof(uint16_t) * (size_t)std::max<int64_t>(nnz, 1));
  p.val = take(sizeof(float) * (size_t)std::max<int64_t>(nnz, 1));
  p.rank = take(sizeof(int32_t) * J);
  p.perm = take(sizeof(int32_t) * J);
  p.hist = take(sizeof(uint32_t) * J);
  p.V[0] = take(sizeof(float) * J * LDV);
  p.V[1] = take(sizeof(float) * J * LDV);
  p.F = take(sizeof(float) * (size_t)K * R * R);
  p.M2 = take(sizeof(float) * J * LDV);
  p.M2part = take(p2::mode2_part_bytes(R, K, (int)std::min<int64_t>(p2::mode2_max_hot(R), J)));
  p.M3 = take(sizeof(float) * (size_t)K * R);
  const size_t RR = (size_t)R * R;
  size_t s = 0;
  p.oM1 = s; s += RR;
  p.oWtW = s; s += RR;
  p.oVtV = s; s += RR;
  p.oVtVraw = s; s += RR;
  p.oHtH = s; s += RR;
  p.oN2p = s; s += RR;
  p.oN3 = s; s += RR;
  p.oN3p = s; s += RR;
  p.oInv = s; s += R;
  p.oFitAcc = s; s += 2;
  p.oNx2 = s; s += 1;
  p.oFits = s; s += kFitRing;
  p.nsmall = s;
  p.small = take(sizeof(double) * s);
  p.err = take(sizeof(int) * 4);
  p.total = off;
  return p;
}

p2::PolarParams polar_params(const parafac2_opts* o, int R) {
  p2::PolarParams pp;
  const int NC = (R & 1) ? R + 1 : R;
  pp.tau_polar = (o && o->tau_polar > 0) ? o->tau_polar : 1e-10;
  pp.tau_pinv = (o && o->tau_pinv > 0) ? o->tau_pinv : R * 2.220446049250313e-16;
  pp.tol = 8.0 * 2.220446049250313e-16 * std::sqrt((double)NC);
  pp.tau_c = 1e-12;
  pp.tau_s = 1e-12;
  pp.max_sweeps = (o && o->max_sweeps > 0) ? o->max_sweeps : 30;
  return pp;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return fail(P2_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

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
  std::vector<int64_t> subj_host;
  // profiling: event pairs per phase, resolved lazily
  bool profiling = false;
  struct EvPair {
    int phase;
    hipEvent_t a, b;
  };
  std::vector<EvPair> events;
  double prof_ms[P2_NPHASES] = {0};
  int64_t prof_n[P2_NPHASES] = {0};

  template <class T>
  T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
  double* small() const { return at<double>(plan.small); }
  float* V(int i) const { return at<float>(plan.V[i]); }
};

struct parafac2_model {
  int64_t J = 0;
  int R = 0, LDV = 0;
  hipStream_t stream = nullptr;
  unsigned char* ws = nullptr;
  size_t oV = 0, oH = 0, oN3 = 0, oN3p = 0, oVtV = 0, oHtH = 0, oMap = 0, total = 0;
  p2::PolarParams pp{};
};

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
    if (b - a < R) {
      snprintf(buf, sizeof(buf), "subject %lld has I_k=%lld < R=%d", (long long)k, (long long)(b - a), R);
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

extern "C" {

int parafac2_abi_version(void) { return PARAFAC2_ABI_VERSION; }

const char* parafac2_last_error(void) { return g_last_error.c_str(); }

int parafac2_validate_host(const parafac2_csr* host_X, int32_t R, char* msg, size_t msg_len) {
  std::string m;
  const int rc = validate_host_impl(host_X, R, m);
  if (msg && msg_len) {
    std::strncpy(msg, m.c_str(), msg_len - 1);
    msg[msg_len - 1] = 0;
  }
  if (rc != P2_OK) g_last_error = m;
  return rc;
}

int parafac2_workspace_size(const parafac2_csr* X, int32_t R, const parafac2_opts* /*opts*/,
                            size_t* bytes) {
  if (!X || !bytes) return fail(P2_EINVAL, "NULL argument");
  if (R < 1 || X->K < 1 || X->J < 1 || X->n_rows < 0 || X->nnz < 0)
    return fail(P2_EINVAL, "bad sizes");
  *bytes = make_plan(X->K, X->J, X->n_rows, X->nnz, R).total;
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
  if (X->n_rows < X->K * (int64_t)R) return fail(P2_EINVAL, "n_rows < K*R: some I_k < R");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return fail(P2_EINVAL, "workspace must be 256-byte aligned");
  const Plan plan = make_plan(X->K, X->J, X->n_rows, X->nnz, R);
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
  const int maxhot = p2::mode2_max_hot(R);
  if (opts && opts->hot_cols < 0)
    c->hot = 0;
  else if (opts && opts->hot_cols > 0)
    c->hot = (int)std::min<int64_t>({(int64_t)opts->hot_cols, (int64_t)maxhot, X->J});
  else
    c->hot = (int)std::min<int64_t>(maxhot, X->J);

  auto cleanup = [&](int rc) {
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
                            X->J, R, err, zbase, rbase, s));
  int herr = 0;
  INIT_TRY(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, s));
  INIT_TRY(hipStreamSynchronize(s));
  if (herr) {
    if (herr & (1 | 16)) return cleanup(fail(P2_EINVAL, "row_ptr/subj_ptr are not monotone offsets"));
    if (herr & 2) return cleanup(fail(P2_EINVAL, "column index out of [0, J)"));
    if (herr & 4) return cleanup(fail(P2_EINVAL, "columns not strictly increasing within a row"));
    if (herr & 8) return cleanup(fail(P2_EINVAL, "non-finite value"));
    if (herr & 32) return cleanup(fail(P2_EINVAL, "a subject has I_k < R=%d", R));
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
  double* sm = c->small();
  INIT_TRY(p2::run_fill_f64(sm, (int64_t)plan.nsmall, 0.0, s));
  INIT_TRY(p2::run_encode(X->subj_ptr, X->row_ptr, X->col, X->val, X->K, X->nnz,
                          c->at<int32_t>(plan.rank), c->at<uint16_t>(plan.rstart),
                          c->at<uint16_t>(plan.col16), c->at<float>(plan.val), sm + plan.oNx2, s));
  INIT_TRY(p2::run_fill_f32(c->V(0), X->J * c->LDV, 0.f, s));
  INIT_TRY(p2::run_fill_f32(c->V(1), X->J * c->LDV, 0.f, s));
  INIT_TRY(p2::run_permute_rows(V, c->V(0), X->J, R, R, c->LDV, c->at<int32_t>(plan.rank), s));
  INIT_TRY(p2::run_gram_tall(R, c->V(0), X->J, c->LDV, sm + plan.oVtV, s));
  INIT_TRY(hipStreamSynchronize(s));  // host vectors above go out of scope
  c->X.zbase = zbase;
  c->X.rbase = rbase;
  c->X.rstart = c->at<uint16_t>(plan.rstart);
  c->X.col = c->at<uint16_t>(plan.col16);
  c->X.val = c->at<float>(plan.val);
  c->cur = 0;
  c->have_F = false;
  *out = c;
  g_last_error.clear();
  return P2_OK;
#undef INIT_TRY
}

// Runs stmt (a HIP_TRY'd launch) bracketed by events when profiling is on.
#define PHASE(ph, stmt)                                                   \
  do {                                                                    \
    hipEvent_t ea_ = nullptr, eb_ = nullptr;                              \
    if (c->profiling) {                                                   \
      HIP_TRY(hipEventCreate(&ea_));                                      \
      HIP_TRY(hipEventCreate(&eb_));                                      \
      HIP_TRY(hipEventRecord(ea_, s));                                    \
    }                                                                     \
    stmt;                                                                 \
    if (c->profiling) {                                                   \
      HIP_TRY(hipEventRecord(eb_, s));                                    \
      c->events.push_back({ph, ea_, eb_});                                \
    }                                                                     \
  } while (0)

static int iterate_impl(parafac2_ctx* c, int32_t n_iters, double* fit_host) {
  const Plan& P = c->plan;
  hipStream_t s = c->stream;
  const int R = c->R;
  double* sm = c->small();
  double* M1 = sm + P.oM1;
  double* WtW = sm + P.oWtW;
  double* VtV = sm + P.oVtV;
  double* VtVraw = sm + P.oVtVraw;
  double* HtH = sm + P.oHtH;
  double* N2p = sm + P.oN2p;
  double* N3 = sm + P.oN3;
  double* N3p = sm + P.oN3p;
  double* inv = sm + P.oInv;
  double* fitacc = sm + P.oFitAcc;
  double* nx2 = sm + P.oNx2;
  double* fits = sm + P.oFits;
  float* F = c->at<float>(P.F);
  float* M2 = c->at<float>(P.M2);
  float* M3 = c->at<float>(P.M3);
  const int64_t RR = (int64_t)R * R;
  for (int32_t it = 0; it < n_iters; ++it) {
    float* Vc = c->V(c->cur);
    float* Vn = c->V(1 - c->cur);
    if (!c->have_F) {
      HIP_TRY(p2::run_fill_f64(M1, RR, 0.0, s));
      PHASE(P2_PHASE_ALPHA, HIP_TRY(p2::run_alpha(R, c->X, c->K, Vc, c->W, c->H, F, M1, c->pp, s)));
    }
    // mode 1 -> H
    HIP_TRY(p2::run_fill_f64(WtW, RR, 0.0, s));
    PHASE(P2_PHASE_SOLVE_H, HIP_TRY(p2::run_gram_tall(R, c->W, c->K, R, WtW, s));
          HIP_TRY(p2::run_solve_h(R, M1, WtW, VtV, c->H, HtH, N2p, c->pp, s)));
    // mode 2 -> V
    HIP_TRY(p2::run_fill_f32(M2, c->J * c->LDV, 0.f, s));
    PHASE(P2_PHASE_MODE2, HIP_TRY(p2::run_mode2(R, c->X, c->K, Vc, c->W, c->H, F, M2,
                                                 c->at<float>(P.M2part), c->hot, s)));
    PHASE(P2_PHASE_VUPDATE, HIP_TRY(p2::run_vupdate(R, M2, N2p, c->J, Vn, s));
          HIP_TRY(p2::run_fill_f64(VtVraw, RR, 0.0, s));
          HIP_TRY(p2::run_gram_tall(R, Vn, c->J, c->LDV, VtVraw, s));
          HIP_TRY(p2::run_solve_n3(R, VtVraw, HtH, VtV, inv, N3, N3p, c->pp, s));
          HIP_TRY(p2::run_vscale(R, Vn, c->J, inv, s)));
    // mode 3 -> W, fit (+ next Procrustes step)
    const int do_next = (it + 1 < n_iters) ? 1 : 0;
    if (do_next) HIP_TRY(p2::run_fill_f64(M1, RR, 0.0, s));
    HIP_TRY(p2::run_fill_f64(fitacc, 2, 0.0, s));
    PHASE(P2_PHASE_GAMMA,
          HIP_TRY(p2::run_gamma(R, c->X, c->K, Vc, Vn, c->W, c->H, N3, N3p, F, M3, M1, fitacc,
                                do_next, c->pp, s)));
    PHASE(P2_PHASE_FIT, HIP_TRY(p2::run_fit(fitacc, nx2, fits + (c->iters_done % kFitRing), s)));
    c->qv = c->cur;
    c->cur = 1 - c->cur;
    c->have_F = do_next != 0;
    c->iters_done++;
  }
  // publish V in the caller's column order
  HIP_TRY(p2::run_permute_rows(c->V(c->cur), c->Vuser, c->J, R, c->LDV, R,
                               c->at<int32_t>(P.perm), s));
  if (fit_host) {
    const int64_t first = c->iters_done - n_iters;
    for (int32_t i = 0; i < n_iters; ++i) {
      HIP_TRY(hipMemcpyAsync(fit_host + i, fits + ((first + i) % kFitRing), sizeof(double),
                             hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
  }
  return P2_OK;
}

int parafac2_iterate(parafac2_ctx* c, int32_t n_iters, double* fit_host) {
  if (!c) return fail(P2_EINVAL, "ctx is NULL");
  if (c->failed) return fail(P2_ESTATE, "context is in a failed state");
  if (n_iters < 0) return fail(P2_EINVAL, "n_iters < 0");
  if (n_iters == 0) return P2_OK;
  int32_t done = 0;
  while (done < n_iters) {
    const int32_t n = std::min<int32_t>(n_iters - done, kFitRing);
    const int rc = iterate_impl(c, n, fit_host ? fit_host + done : nullptr);
    if (rc != P2_OK) {
      c->failed = true;
      return rc;
    }
    done += n;
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
    HIP_TRY(hipMemcpyAsync(M1, c->small() + P.oM1, sizeof(double) * c->R * c->R,
                           hipMemcpyDeviceToDevice, s));
  if (M2)
    HIP_TRY(p2::run_permute_rows(c->at<float>(P.M2), M2, c->J, c->R, c->LDV, c->R,
                                 c->at<int32_t>(P.perm), s));
  if (M3)
    HIP_TRY(hipMemcpyAsync(M3, c->at<float>(P.M3), sizeof(float) * c->K * c->R,
                           hipMemcpyDeviceToDevice, s));
  return P2_OK;
}

int parafac2_get_q(parafac2_ctx* c, int64_t k0, int64_t k1, float* Q) {
  if (!c || !Q) return fail(P2_EINVAL, "NULL argument");
  if (c->failed) return fail(P2_ESTATE, "context is in a failed state");
  if (k0 < 0 || k1 > c->K || k0 > k1) return fail(P2_EINVAL, "bad subject range");
  if (c->have_F || c->qv < 0)
    return fail(P2_ESTATE, "no completed Procrustes step to report");
  if (k0 == k1) return P2_OK;
  HIP_TRY(p2::run_getq(c->R, c->X, k0, k1, c->V(c->qv), c->at<float>(c->plan.F), Q,
                       c->subj_host[k0], c->stream));
  return P2_OK;
}

static int resolve_profile(parafac2_ctx* c) {
  if (c->events.empty()) return P2_OK;
  HIP_TRY(hipStreamSynchronize(c->stream));
  for (auto& e : c->events) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e.a, e.b));
    c->prof_ms[e.phase] += ms;
    c->prof_n[e.phase] += 1;
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  c->events.clear();
  return P2_OK;
}

int parafac2_set_profiling(parafac2_ctx* c, int32_t on) {
  if (!c) return fail(P2_EINVAL, "ctx is NULL");
  const int rc = resolve_profile(c);
  if (rc != P2_OK) return rc;
  c->profiling = on != 0;
  for (int i = 0; i < P2_NPHASES; ++i) {
    c->prof_ms[i] = 0.0;
    c->prof_n[i] = 0;
  }
  return P2_OK;
}

int parafac2_get_profile(parafac2_ctx* c, double* ms, int64_t* launches) {
  if (!c) return fail(P2_EINVAL, "ctx is NULL");
  const int rc = resolve_profile(c);
  if (rc != P2_OK) return rc;
  for (int i = 0; i < P2_NPHASES; ++i) {
    if (ms) ms[i] = c->prof_ms[i];
    if (launches) launches[i] = c->prof_n[i];
  }
  return P2_OK;
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
  for (auto& e : c->events) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  delete c;
}

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
  hipStream_t s = m->stream;
  float* Vm = reinterpret_cast<float*>(m->ws + m->oV);
  double* Hm = reinterpret_cast<double*>(m->ws + m->oH);
  double* VtV = reinterpret_cast<double*>(m->ws + m->oVtV);
  int32_t* map = reinterpret_cast<int32_t*>(m->ws + m->oMap);
  auto bad = [&](hipError_t e, const char* what) {
    delete m;
    return fail(P2_EDEVICE, "%s: %s", what, hipGetErrorString(e));
  };
  hipError_t e;
  if ((e = p2::run_fill_f32(Vm, J * m->LDV, 0.f, s)) != hipSuccess) return bad(e, "fill");
  if ((e = p2::run_iota(map, J, s)) != hipSuccess) return bad(e, "iota");
  if ((e = p2::run_permute_rows(V, Vm, J, R, R, m->LDV, map, s)) != hipSuccess) return bad(e, "copy V");
  if ((e = hipMemcpyAsync(Hm, H, sizeof(double) * R * R, hipMemcpyDeviceToDevice, s)) != hipSuccess)
    return bad(e, "copy H");
  if ((e = p2::run_fill_f64(VtV, (int64_t)R * R, 0.0, s)) != hipSuccess) return bad(e, "fill");
  if ((e = p2::run_gram_tall(R, Vm, J, m->LDV, VtV, s)) != hipSuccess) return bad(e, "VtV");
  if ((e = p2::run_model_prep(R, VtV, Hm, reinterpret_cast<double*>(m->ws + m->oHtH),
                              reinterpret_cast<double*>(m->ws + m->oN3),
                              reinterpret_cast<double*>(m->ws + m->oN3p), m->pp, s)) != hipSuccess)
    return bad(e, "N3");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return bad(e, "sync");
  *out = m;
  return P2_OK;
}

int parafac2_project(parafac2_model* m, const parafac2_csr* req, int32_t n_steps, const float* w0,
                     float* Q_out, float* w_out, double* loss_out, void* stream) {
  if (!m || !req || !w_out) return fail(P2_EINVAL, "NULL argument");
  if (req->J != m->J) return fail(P2_EINVAL, "request J=%lld != model J=%lld",
                                  (long long)req->J, (long long)m->J);
  if (req->K < 0 || n_steps < 0) return fail(P2_EINVAL, "bad sizes");
  if (req->K == 0) return P2_OK;
  if (!req->subj_ptr || !req->row_ptr || (req->nnz > 0 && (!req->col || !req->val)))
    return fail(P2_EINVAL, "NULL array");
  hipStream_t s = stream ? reinterpret_cast<hipStream_t>(stream) : m->stream;
  p2::XRaw X{req->subj_ptr, req->row_ptr, req->col, req->val};
  HIP_TRY(p2::run_project(m->R, X, req->K, reinterpret_cast<const float*>(m->ws + m->oV),
                          reinterpret_cast<const double*>(m->ws + m->oH),
                          reinterpret_cast<const double*>(m->ws + m->oN3),
                          reinterpret_cast<const double*>(m->ws + m->oN3p), n_steps, w0, Q_out,
                          w_out, loss_out, m->pp, s));
  return P2_OK;
}

void parafac2_model_destroy(parafac2_model* m) { delete m; }

}  // extern "C"
