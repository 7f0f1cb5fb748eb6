// Serving: continuous batching of projection requests (see parafac2_server_*
// in include/parafac2.h).
//
// A request is one new subject X (I x J, host CSR).  Requests wait in a host
// queue; each batch slot owns a fixed share of the workspace (capacity in
// requests, rows and nonzeros), pinned host staging buffers, a stream and a
// completion event.  poll() harvests slots whose event has completed and
// refills every free slot with the requests at the front of the queue that
// fit it, so new arrivals join the device as soon as capacity frees up and
// batches on different slots overlap (copies of one with compute of another).
// The projection of each request is the per-subject kernel that
// parafac2_project runs; its result depends on the request's own slice only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <vector>

#include "../../include/parafac2.h"
#include "p2_device.h"
#include "p2_host.h"
#include "p2_kernels.h"

using p2host::fail;

namespace {

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

struct ServerCaps {
  int slots, max_requests, max_queue, n_steps, want_q;
  int64_t max_rows, max_nnz;
};

ServerCaps caps_of(const parafac2_server_opts* o) {
  ServerCaps c{};
  c.slots = (o && o->slots > 0) ? std::min(o->slots, 64) : 4;
  c.max_requests = (o && o->max_requests > 0) ? o->max_requests : 512;
  c.max_rows = (o && o->max_rows > 0) ? o->max_rows : 65536;
  c.max_nnz = (o && o->max_nnz > 0) ? o->max_nnz : (int64_t)1 << 21;
  c.max_queue = (o && o->max_queue > 0) ? o->max_queue : 1 << 16;
  c.n_steps = (o && o->n_steps > 0) ? o->n_steps : 10;
  c.want_q = (o && o->want_q) ? 1 : 0;
  return c;
}

// Device bytes of one slot, and the offsets of its arrays.
struct SlotLayout {
  size_t subj, row, col, val, w, loss, q, total;
};

SlotLayout slot_layout(const ServerCaps& c, int R) {
  SlotLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + std::max<size_t>(bytes, 1));
    return at;
  };
  L.subj = take(sizeof(int64_t) * (size_t)(c.max_requests + 1));
  L.row = take(sizeof(int64_t) * (size_t)(c.max_rows + 1));
  L.col = take(sizeof(int32_t) * (size_t)c.max_nnz);
  L.val = take(sizeof(float) * (size_t)c.max_nnz);
  L.w = take(sizeof(float) * (size_t)c.max_requests * R);
  L.loss = take(sizeof(double) * (size_t)c.max_requests);
  L.q = c.want_q ? take(sizeof(float) * (size_t)c.max_rows * R) : 0;
  L.total = off;
  return L;
}

struct Request {
  int64_t id = 0;
  int32_t I = 0;
  std::vector<int64_t> row_ptr;
  std::vector<int32_t> col;
  std::vector<float> val;
  int64_t nnz() const { return (int64_t)col.size(); }
};

struct Result {
  int64_t id = 0;
  std::vector<float> w, q;
  double loss = 0.0;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  // device (in the workspace)
  int64_t* d_subj = nullptr;
  int64_t* d_row = nullptr;
  int32_t* d_col = nullptr;
  float* d_val = nullptr;
  float* d_w = nullptr;
  double* d_loss = nullptr;
  float* d_q = nullptr;
  // pinned host staging (one block)
  void* h_block = nullptr;
  int64_t* h_subj = nullptr;
  int64_t* h_row = nullptr;
  int32_t* h_col = nullptr;
  float* h_val = nullptr;
  float* h_w = nullptr;
  double* h_loss = nullptr;
  float* h_q = nullptr;
  // the batch in flight
  bool busy = false;
  std::vector<int64_t> ids;
  std::vector<int32_t> rows_of;
  int64_t rows = 0, nnz = 0;
};

}  // namespace

struct parafac2_server {
  parafac2_model* m = nullptr;
  ServerCaps caps{};
  std::vector<Slot> slots;
  std::deque<Request> queue;
  std::deque<Result> finished;

  ~parafac2_server() {
    for (Slot& s : slots) {
      if (s.stream) (void)hipStreamSynchronize(s.stream);
      if (s.done) (void)hipEventDestroy(s.done);
      if (s.stream) (void)hipStreamDestroy(s.stream);
      if (s.h_block) (void)hipHostFree(s.h_block);
    }
  }
};

namespace {

// Pack the requests at the front of the queue that fit into slot s and start
// its batch.  Returns P2_OK with nothing started if the queue is empty.
int start_batch(parafac2_server* sv, Slot& s) {
  const ServerCaps& c = sv->caps;
  const int R = sv->m->R;
  s.ids.clear();
  s.rows_of.clear();
  s.rows = 0;
  s.nnz = 0;
  s.h_subj[0] = 0;
  while (!sv->queue.empty() && (int)s.ids.size() < c.max_requests) {
    const Request& q = sv->queue.front();
    if (s.rows + q.I > c.max_rows || s.nnz + q.nnz() > c.max_nnz) break;
    for (int32_t i = 0; i < q.I; ++i) s.h_row[s.rows + i] = s.nnz + q.row_ptr[i];
    std::memcpy(s.h_col + s.nnz, q.col.data(), sizeof(int32_t) * q.col.size());
    std::memcpy(s.h_val + s.nnz, q.val.data(), sizeof(float) * q.val.size());
    s.rows += q.I;
    s.nnz += q.nnz();
    s.ids.push_back(q.id);
    s.rows_of.push_back(q.I);
    s.h_subj[s.ids.size()] = s.rows;
    sv->queue.pop_front();
  }
  const int64_t n = (int64_t)s.ids.size();
  if (n == 0) return P2_OK;
  s.h_row[s.rows] = s.nnz;
  hipStream_t st = s.stream;
  P2_HIP_TRY(hipMemcpyAsync(s.d_subj, s.h_subj, sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, st));
  P2_HIP_TRY(hipMemcpyAsync(s.d_row, s.h_row, sizeof(int64_t) * (s.rows + 1), hipMemcpyHostToDevice, st));
  if (s.nnz > 0) {
    P2_HIP_TRY(hipMemcpyAsync(s.d_col, s.h_col, sizeof(int32_t) * s.nnz, hipMemcpyHostToDevice, st));
    P2_HIP_TRY(hipMemcpyAsync(s.d_val, s.h_val, sizeof(float) * s.nnz, hipMemcpyHostToDevice, st));
  }
  const p2::XRaw X{s.d_subj, s.d_row, s.d_col, s.d_val};
  const parafac2_model* m = sv->m;
  P2_HIP_TRY(p2::run_project(R, X, n, m->V(), m->H(), m->N3(), m->N3p(), c.n_steps, nullptr,
                             c.want_q ? s.d_q : nullptr, s.d_w, s.d_loss, m->pp, st));
  P2_HIP_TRY(hipMemcpyAsync(s.h_w, s.d_w, sizeof(float) * n * R, hipMemcpyDeviceToHost, st));
  P2_HIP_TRY(hipMemcpyAsync(s.h_loss, s.d_loss, sizeof(double) * n, hipMemcpyDeviceToHost, st));
  if (c.want_q)
    P2_HIP_TRY(hipMemcpyAsync(s.h_q, s.d_q, sizeof(float) * s.rows * R, hipMemcpyDeviceToHost, st));
  P2_HIP_TRY(hipEventRecord(s.done, st));
  s.busy = true;
  return P2_OK;
}

void harvest(parafac2_server* sv, Slot& s) {
  const int R = sv->m->R;
  int64_t r0 = 0;
  for (size_t i = 0; i < s.ids.size(); ++i) {
    Result res;
    res.id = s.ids[i];
    res.w.assign(s.h_w + i * R, s.h_w + (i + 1) * R);
    res.loss = s.h_loss[i];
    if (sv->caps.want_q) res.q.assign(s.h_q + r0 * R, s.h_q + (r0 + s.rows_of[i]) * R);
    r0 += s.rows_of[i];
    sv->finished.push_back(std::move(res));
  }
  s.busy = false;
  s.ids.clear();
  s.rows_of.clear();
}

// Harvest finished slots, then refill free slots from the queue.
int pump(parafac2_server* sv) {
  for (Slot& s : sv->slots) {
    if (!s.busy) continue;
    const hipError_t e = hipEventQuery(s.done);
    if (e == hipErrorNotReady) continue;
    P2_HIP_TRY(e);
    harvest(sv, s);
  }
  for (Slot& s : sv->slots) {
    if (sv->queue.empty()) break;
    if (s.busy) continue;
    const int rc = start_batch(sv, s);
    if (rc != P2_OK) return rc;
  }
  return P2_OK;
}

}  // namespace

extern "C" {

int parafac2_server_workspace_size(const parafac2_model* m, const parafac2_server_opts* o,
                                   size_t* bytes) {
  if (!m || !bytes) return fail(P2_EINVAL, "NULL argument");
  const ServerCaps c = caps_of(o);
  *bytes = slot_layout(c, m->R).total * (size_t)c.slots;
  return P2_OK;
}

int parafac2_server_create(parafac2_server** out, parafac2_model* m,
                           const parafac2_server_opts* o, void* workspace, size_t ws_bytes) {
  if (!out) return fail(P2_EINVAL, "out is NULL");
  *out = nullptr;
  if (!m || !workspace) return fail(P2_EINVAL, "NULL argument");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return fail(P2_EINVAL, "workspace must be 256-byte aligned");
  const ServerCaps c = caps_of(o);
  if (c.max_rows < m->R || c.max_rows > ((int64_t)1 << 40) || c.max_nnz > ((int64_t)1 << 40))
    return fail(P2_EINVAL, "bad batch capacity");
  const SlotLayout L = slot_layout(c, m->R);
  if (ws_bytes < L.total * (size_t)c.slots)
    return fail(P2_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes,
                L.total * (size_t)c.slots);
  auto* sv = new parafac2_server();
  sv->m = m;
  sv->caps = c;
  sv->slots.resize(c.slots);
  unsigned char* base = reinterpret_cast<unsigned char*>(workspace);
  const size_t hbytes = sizeof(int64_t) * (c.max_requests + 1) + sizeof(int64_t) * (c.max_rows + 1) +
                        (sizeof(int32_t) + sizeof(float)) * c.max_nnz +
                        sizeof(float) * (size_t)c.max_requests * m->R +
                        sizeof(double) * c.max_requests +
                        (c.want_q ? sizeof(float) * (size_t)c.max_rows * m->R : 0) + 64;
  for (int i = 0; i < c.slots; ++i) {
    Slot& s = sv->slots[i];
    unsigned char* b = base + L.total * i;
    s.d_subj = reinterpret_cast<int64_t*>(b + L.subj);
    s.d_row = reinterpret_cast<int64_t*>(b + L.row);
    s.d_col = reinterpret_cast<int32_t*>(b + L.col);
    s.d_val = reinterpret_cast<float*>(b + L.val);
    s.d_w = reinterpret_cast<float*>(b + L.w);
    s.d_loss = reinterpret_cast<double*>(b + L.loss);
    s.d_q = c.want_q ? reinterpret_cast<float*>(b + L.q) : nullptr;
    hipError_t e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipHostMalloc(&s.h_block, hbytes, hipHostMallocDefault);
    if (e != hipSuccess) {
      delete sv;
      return fail(P2_EDEVICE, "server slot setup: %s", hipGetErrorString(e));
    }
    // host staging, 8-byte fields first
    unsigned char* h = reinterpret_cast<unsigned char*>(s.h_block);
    s.h_subj = reinterpret_cast<int64_t*>(h);
    h += sizeof(int64_t) * (c.max_requests + 1);
    s.h_row = reinterpret_cast<int64_t*>(h);
    h += sizeof(int64_t) * (c.max_rows + 1);
    s.h_loss = reinterpret_cast<double*>(h);
    h += sizeof(double) * c.max_requests;
    s.h_col = reinterpret_cast<int32_t*>(h);
    h += sizeof(int32_t) * c.max_nnz;
    s.h_val = reinterpret_cast<float*>(h);
    h += sizeof(float) * c.max_nnz;
    s.h_w = reinterpret_cast<float*>(h);
    h += sizeof(float) * (size_t)c.max_requests * m->R;
    s.h_q = c.want_q ? reinterpret_cast<float*>(h) : nullptr;
  }
  *out = sv;
  return P2_OK;
}

int parafac2_server_submit(parafac2_server* sv, int64_t id, int32_t I, const int64_t* row_ptr,
                           const int32_t* col, const float* val) {
  if (!sv || !row_ptr) return fail(P2_EINVAL, "NULL argument");
  const int R = sv->m->R;
  const ServerCaps& c = sv->caps;
  if (I < R) return fail(P2_EINVAL, "request %lld has I=%d < R=%d", (long long)id, I, R);
  if (row_ptr[0] != 0) return fail(P2_EINVAL, "row_ptr must start at 0");
  for (int32_t i = 0; i < I; ++i)
    if (row_ptr[i + 1] < row_ptr[i]) return fail(P2_EINVAL, "row_ptr decreases at row %d", i);
  const int64_t nnz = row_ptr[I];
  if (I > c.max_rows || nnz > c.max_nnz)
    return fail(P2_EINVAL, "request %lld (I=%d, nnz=%lld) exceeds a batch slot", (long long)id, I,
                (long long)nnz);
  if (nnz > 0 && (!col || !val)) return fail(P2_EINVAL, "NULL col/val");
  for (int64_t z = 0; z < nnz; ++z) {
    if (col[z] < 0 || col[z] >= sv->m->J)
      return fail(P2_EINVAL, "column %d out of range in request %lld", col[z], (long long)id);
    if (!std::isfinite(val[z]))
      return fail(P2_EINVAL, "non-finite value in request %lld", (long long)id);
  }
  if ((int64_t)sv->queue.size() >= c.max_queue) return fail(P2_EBUSY, "request queue is full");
  Request q;
  q.id = id;
  q.I = I;
  q.row_ptr.assign(row_ptr, row_ptr + I + 1);
  q.col.assign(col, col + nnz);
  q.val.assign(val, val + nnz);
  sv->queue.push_back(std::move(q));
  return P2_OK;
}

int parafac2_server_poll(parafac2_server* sv, int32_t max_out, int64_t* ids, float* w,
                         double* loss, float* q, int64_t q_cap, int32_t* q_rows, int32_t* n_out) {
  if (!sv || !n_out) return fail(P2_EINVAL, "NULL argument");
  *n_out = 0;
  if (max_out > 0 && (!ids || !w)) return fail(P2_EINVAL, "NULL ids/w");
  const int rc = pump(sv);
  if (rc != P2_OK) return rc;
  const int R = sv->m->R;
  int32_t n = 0;
  int64_t qused = 0;
  while (n < max_out && !sv->finished.empty()) {
    Result& r = sv->finished.front();
    const int64_t rows = (int64_t)r.q.size() / R;
    if (sv->caps.want_q && q) {
      if (qused + rows > q_cap) break;
      std::memcpy(q + qused * R, r.q.data(), sizeof(float) * r.q.size());
      if (q_rows) q_rows[n] = (int32_t)rows;
      qused += rows;
    }
    ids[n] = r.id;
    std::memcpy(w + (size_t)n * R, r.w.data(), sizeof(float) * R);
    if (loss) loss[n] = r.loss;
    sv->finished.pop_front();
    ++n;
  }
  *n_out = n;
  return P2_OK;
}

int parafac2_server_pending(parafac2_server* sv, int64_t* queued, int64_t* in_flight,
                            int64_t* finished) {
  if (!sv) return fail(P2_EINVAL, "NULL argument");
  int64_t f = 0;
  for (const Slot& s : sv->slots) f += s.busy ? (int64_t)s.ids.size() : 0;
  if (queued) *queued = (int64_t)sv->queue.size();
  if (in_flight) *in_flight = f;
  if (finished) *finished = (int64_t)sv->finished.size();
  return P2_OK;
}

int parafac2_server_drain(parafac2_server* sv) {
  if (!sv) return fail(P2_EINVAL, "NULL argument");
  for (;;) {
    const int rc = pump(sv);
    if (rc != P2_OK) return rc;
    bool busy = false;
    for (Slot& s : sv->slots)
      if (s.busy) {
        busy = true;
        P2_HIP_TRY(hipEventSynchronize(s.done));
      }
    if (!busy && sv->queue.empty()) break;
  }
  return P2_OK;
}

void parafac2_server_destroy(parafac2_server* sv) { delete sv; }

}  // extern "C"
