/*
 * parafac2.h -- C ABI of the MI355X (gfx950) PARAFAC2-ALS hot path.
 *
 * The method is SPARTan (Perros et al., "SPARTan: Scalable PARAFAC2 for Large
 * & Sparse Data", KDD'17).  Given K sparse slices X_k (I_k x J) and a target
 * rank R, PARAFAC2 fits X_k ~ Q_k H S_k V^T with Q_k^T Q_k = I, S_k diagonal
 * (Sec. "Model", equation (paratwo_basic)).  One ALS iteration (Algorithm
 * "PARAFAC2-ALS") is:
 *   1. the orthogonal Procrustes step, Q_k = polar(X_k V S_k H^T) for every
 *      subject (objective (procrustes_obj));
 *   2. one CP-ALS iteration (Algorithm "CP-ALS") on the tensor Y with frontal
 *      slices Y_k = Q_k^T X_k, whose three MTTKRPs are computed slice by slice
 *      over the nonzero columns of X_k only (Sec. "Methodology", Algorithm
 *      "MTTKRP for SPARTan", equations (mttkrp1_3), (mttkrp2_3),
 *      (mttkrp3_row_wise));
 *   3. S_k <- diag(W(k,:)).
 * The library never forms Y or Q_k during an iteration: every MTTKRP is
 * rewritten in terms of per-subject R x R matrices and per-row R-vectors.
 *
 * Conventions for every call:
 *   - return value: 0 (P2_OK) or a negative status; nothing aborts and nothing
 *     throws across the ABI; parafac2_last_error() gives the text of the last
 *     failure on the calling thread;
 *   - matrices are row-major and 0-based;
 *   - "device" pointers are HIP device allocations on the current device;
 *     "host" pointers are ordinary CPU memory;
 *   - stream is a hipStream_t passed as void* (NULL = default stream); all
 *     device work of a context or model is enqueued on its stream;
 *   - the caller owns every buffer it passes, including the workspace; the
 *     library allocates no device memory.
 */
#ifndef PARAFAC2_H
#define PARAFAC2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  P2_OK = 0,
  P2_EINVAL = -1,  /* bad argument or input data (message says which)          */
  P2_ENOMEM = -2,  /* reserved: no call returns it (a workspace smaller than
                      parafac2_workspace_size() asked for is P2_EINVAL)      */
  P2_EDEVICE = -3, /* a HIP call failed; the context is then unusable           */
  P2_ESTATE = -4,  /* context or model is in a failed state                    */
  P2_ENOTSUP = -5, /* valid input outside what the library supports (e.g. R)  */
  P2_EBUSY = -6    /* a server's request queue is full; poll and submit again   */
};

#define PARAFAC2_ABI_VERSION 1

/* Opaque handles.  A context holds one decomposition, a model holds fixed
 * (V, H) for projecting new subjects.  Neither is thread-safe; calls that
 * overlap on one handle race. */
typedef struct parafac2_ctx parafac2_ctx;
typedef struct parafac2_model parafac2_model;

/* The input collection {X_k} (Algorithm "PARAFAC2-ALS", REQUIRE) as one
 * concatenated CSR.  Subject k owns rows [subj_ptr[k], subj_ptr[k+1]); row i
 * owns nonzeros [row_ptr[i], row_ptr[i+1]).  Columns are in [0, J) and
 * strictly increasing within a row; values are finite.  Empty rows are
 * accepted (they contribute nothing; the paper filters them, Sec.
 * "Challenges of PARAFAC2 on sparse data").  Limits of the library:
 * 1 <= I_k <= 65535, nnz of one subject <= 65535, J <= 65536,
 * K <= 2^31 - 1; every rank 1 <= R <= 40 is built.  A subject with
 * I_k < R (the paper runs such data at ranks above its largest I_k, Table
 * "table:data_stats") gets the economy
 * Procrustes factor Q_k = Z P^T from the thin SVD H S_k V^T X_k^T = P S Z^T:
 * an I_k x R matrix with orthonormal rows (Q_k Q_k^T = I), and the loss
 * counts ||Q_k H S_k V^T||_F with that Q_k.  A context with such subjects
 * does not fuse the next Procrustes step into the mode-3 pass. */
typedef struct {
  int64_t K, J, n_rows, nnz;
  const int64_t* subj_ptr; /* [K+1]      */
  const int64_t* row_ptr;  /* [n_rows+1] */
  const int32_t* col;      /* [nnz]      */
  const float* val;        /* [nnz]      */
} parafac2_csr;

/* Launch schedule of the per-subject passes (the Procrustes step fused with
 * mode 3, and the mode-2 scatter).  Subjects are independent within an
 * iteration (Sec. "Methodology": the slice-wise MTTKRPs may be computed in any
 * order), so the passes run over tiles -- ranges of subjects of one problem --
 * in any order.  Tile lists are split into 8 contiguous bins, one per XCD.
 * A zero-initialised struct selects the defaults. */
typedef struct {
  int32_t tile_rounds; /* subjects per Procrustes/mode-3 tile, in units of the
                          subject groups that one workgroup holds; 0 -> 4      */
  int32_t dynamic;     /* 0: static, workgroup b takes tiles b, b + grid, ...
                          (all in the bin of its XCD); 1: workgroups take tiles
                          from per-bin counters and move on to other bins when
                          their own is used up                                 */
  int32_t m2_tiles;    /* at most this many mode-2 tiles per problem (each
                          writes one slot of hot-column partial sums); 0 ->
                          the context's capacity                              */
  int32_t graph;       /* 1: every iteration after the first Procrustes step
                          replays a HIP graph captured once (per parity of the
                          V buffers and per whether the next Procrustes step is
                          fused in); 0: plain launches                        */
  int32_t m2_threads;  /* mode-2 workgroup size (multiple of 64, <= 1024);
                          0 -> the rank's default                             */
  int32_t m2_blocks;   /* mode-2 workgroups meant to share a CU: each keeps
                          the hot-column partial sums that fit its 1/m2_blocks
                          share of the LDS (fewer hot columns, more waves in
                          flight); 0 -> 1                                    */
  int32_t warm_polar;  /* 1: where the context keeps each subject's last
                          eigenvector basis (parafac2_opts.keep_bases) and this
                          build has the warm-started kernels (R <= 20), the
                          Procrustes eigen-solves start from it; 0: they start
                          from scratch                                        */
} parafac2_sched;

/* Options; a zero-initialised struct selects the defaults. */
typedef struct {
  double tau_polar;  /* eigenvalues of G_k = B_k^T B_k (B_k = X_k V S_k H^T)
                        below tau_polar * lambda_max are dropped from the
                        inverse square root in the Procrustes step;
                        0 -> 1e-13                                           */
  double tau_pinv;   /* eigenvalue cut of the R x R pseudo-inverses of the
                        normal equations (Algorithm "CP-ALS"), relative to
                        lambda_max; 0 -> R * 2.22e-16                         */
  int32_t hot_cols;  /* columns whose mode-2 partial sums are kept in LDS;
                        0 -> as many as fit, -1 -> none                       */
  int32_t max_sweeps;/* cap on Jacobi sweeps per R x R eigenproblem; 0 -> 30 */
  parafac2_sched sched;  /* launch schedule of the context                    */
  int32_t m2_capacity;   /* mode-2 partial-sum slots planned in the workspace
                            (the largest m2_tiles a schedule may use); 0 -> 512 */
  int32_t keep_bases;    /* 1: each subject keeps the eigenvector basis of its
                            last Procrustes step in the workspace (K x R x R
                            floats, R rounded up to even; ranks <= 20) so that
                            a schedule with warm_polar can start the next
                            eigen-solve from it; 0: no bases are kept          */
  int32_t nonneg;        /* 1: V and W (the diagonals of S_k) are updated by
                            non-negative least squares on the same normal
                            equations (the constraints of the paper's
                            experiments, Sec. "Classical Algorithm for PARAFAC2"
                            and Sec. "Setup"); H stays unconstrained.  The W
                            rows are solved inside the mode-3 pass, which
                            still takes the next Procrustes step;
                            0: unconstrained                                  */
  int32_t baseline;      /* 1: run the paper's comparison method instead of
                            SPARTan's MTTKRPs ("Sparse PARAFAC2", Sec. "Setup"):
                            every iteration materialises Q_k, forms the sparse
                            tensor Y (Y_k = Q_k^T X_k over the nonzero columns
                            of X_k, R entries per nonzero column, coordinate
                            format) and runs the three MTTKRPs as generic
                            coordinate-format sums over its entries.  Same
                            results up to rounding; for comparison only.
                            The workspace then holds the runs of equal columns
                            of every subject, Q (n_rows x R floats) and Y
                            (16 bytes for each of at most R * nnz entries);
                            unconstrained and I_k >= R only (P2_ENOTSUP
                            otherwise); a context with it cannot join a batch */
} parafac2_opts;

/* ABI version of the loaded library (PARAFAC2_ABI_VERSION). */
int parafac2_abi_version(void);

/* Text of the last failing call on this thread ("" if none). */
const char* parafac2_last_error(void);

/* Host-only validation of a CSR whose pointers are HOST memory: shapes,
 * monotone offsets, column range and order, finiteness, I_k >= 1 and the
 * build limits above.  Writes a message to msg (if non-NULL).  Returns P2_OK,
 * P2_EINVAL or P2_ENOTSUP.  Touches no GPU. */
int parafac2_validate_host(const parafac2_csr* host_X, int32_t R, char* msg, size_t msg_len);

/* Bytes of device workspace that parafac2_init needs for X (only the sizes
 * K, J, n_rows, nnz of X are read) and rank R.  Touches no GPU. */
int parafac2_workspace_size(const parafac2_csr* X, int32_t R, const parafac2_opts* opts,
                            size_t* bytes);

/* Create a context for one decomposition (Algorithm "PARAFAC2-ALS").
 *   X          device CSR; read only during this call (it is validated on the
 *              device and re-encoded into the workspace).
 *   R          target rank.
 *   H, V, W    device, row-major: H is R x R float64, V is J x R float32, W is
 *              K x R float32 (S_k = diag(W(k,:))).  On entry the initial state
 *              (Algorithm "PARAFAC2-ALS", "Initialize"); the context borrows
 *              them until parafac2_destroy and updates them in place.
 *   workspace  device buffer of at least parafac2_workspace_size() bytes,
 *              256-byte aligned, borrowed until parafac2_destroy.
 * Synchronises the stream once (validation result and column statistics).
 * Errors: P2_EINVAL (shapes, data, small workspace), P2_ENOTSUP (R or sizes
 * outside the library's limits), P2_EDEVICE. */
int parafac2_init(parafac2_ctx** out, const parafac2_csr* X, int32_t R, double* H, float* V,
                  float* W, void* workspace, size_t ws_bytes, void* stream,
                  const parafac2_opts* opts);

/* Run n_iters PARAFAC2-ALS iterations.  Each iteration is the Procrustes
 * step, the mode-1 MTTKRP and H update, the mode-2 MTTKRP and V update, the
 * mode-3 MTTKRP and W update (Algorithm "CP-ALS" order; H and V columns
 * normalised, W keeps the scale).  On return H, V and W hold the new state.
 * loss_host (host, n_iters entries, or NULL) receives per iteration
 * loss = sum_k ||X_k - Q_k H S_k V^T||_F^2 (the objective of Sec. "Classical
 * Algorithm for PARAFAC2") evaluated after the W update, and fit_host (host,
 * n_iters entries, or NULL) fit = 1 - loss / sum_k ||X_k||_F^2.
 * Enqueues on the context's stream; synchronises only if fit_host or
 * loss_host is non-NULL (one device-to-host copy each). */
int parafac2_iterate(parafac2_ctx* c, int32_t n_iters, double* fit_host, double* loss_host);

/* Iterate until convergence (Algorithm "PARAFAC2-ALS", "while convergence
 * criterion is not met"; the paper leaves the criterion open): stop after
 * iteration t >= 2 when |loss_{t-1} - loss_t| <= tol * loss_{t-1} (or the
 * loss is 0), or after max_iters iterations.  *n_done (host) receives the
 * iterations run; fit_host and loss_host (host, max_iters entries, or NULL)
 * receive the first *n_done values as for parafac2_iterate.  Synchronises the
 * stream after every iteration to read its loss.  tol >= 0, max_iters >= 0,
 * else P2_EINVAL. */
int parafac2_iterate_until(parafac2_ctx* c, int32_t max_iters, double tol, int32_t* n_done,
                           double* fit_host, double* loss_host);

/* The three MTTKRPs of the last iteration (equations (mttkrp1), (mttkrp2),
 * (mttkrp3)), for parity checks.  Device pointers, any may be NULL:
 * M1 R x R float64, M2 J x R float32, M3 K x R float32.  Enqueued on the
 * context's stream. */
int parafac2_get_mttkrp(parafac2_ctx* c, double* M1, float* M2, float* M3);

/* Q_k of the last Procrustes step for subjects [k0, k1) (Algorithm
 * "PARAFAC2-ALS": U_k = Q_k H after the loop).  Q (device, float32) receives
 * the rows of those subjects, (subj_ptr[k1] - subj_ptr[k0]) x R, row-major.
 * P2_ESTATE if no iteration has run since init. */
int parafac2_get_q(parafac2_ctx* c, int64_t k0, int64_t k1, float* Q);

/* U_k = Q_k H (Algorithm "PARAFAC2-ALS", ENSURE: the factors {U_k} after
 * the loop; Sec. "Model": X_k ~ U_k S_k V^T) for subjects [k0, k1), with Q_k
 * from the last Procrustes step and the context's current H.  U (device,
 * float32) receives (subj_ptr[k1] - subj_ptr[k0]) x R rows, row-major.
 * P2_ESTATE if no iteration has run since init. */
int parafac2_get_u(parafac2_ctx* c, int64_t k0, int64_t k1, float* U);

/* Per-phase device timing (for benchmarks).  While profiling is on, every
 * kernel launch of parafac2_iterate is bracketed by HIP events recorded on the
 * context's stream; parafac2_get_profile synchronises the stream and returns,
 * per phase, the summed elapsed milliseconds and the number of launches since
 * profiling was switched on.  Phases (P2_PHASE_*): Procrustes step of the
 * first iteration, H solve (W^T W and the R x R solve), mode-2 MTTKRP, V
 * update (V = M2 N2^+, normalisation, N3), mode-3 MTTKRP with the W update and
 * the next Procrustes step, fit. */
enum {
  P2_PHASE_ALPHA = 0,
  P2_PHASE_SOLVE_H = 1,
  P2_PHASE_MODE2 = 2,
  P2_PHASE_VUPDATE = 3,
  P2_PHASE_GAMMA = 4,
  P2_PHASE_FIT = 5,
  P2_NPHASES = 6
};
int parafac2_set_profiling(parafac2_ctx* c, int32_t on);
int parafac2_get_profile(parafac2_ctx* c, double* ms, int64_t* launches);

/* Launch configuration of the compiled kernels (diagnostics for tests and tuning;
 * touches no GPU).  kernel: 0 Procrustes step of the first iteration,
 * 1 mode-3 / W update / next Procrustes step, 2 mode-2 scatter,
 * 3 projection, 4 Q assembly.  threads receives the workgroup size,
 * lds_bytes the dynamic LDS of one workgroup (for kernel 2 with the largest
 * hot-column set, whose size goes to max_hot).  P2_ENOTSUP for an R outside
 * 1..40. */
int parafac2_launch_config(int32_t R, int32_t kernel, int32_t* threads, int64_t* lds_bytes,
                           int32_t* max_hot);

/* Replace the context's launch schedule (takes effect at the next iterate;
 * captured graphs are dropped).  Synchronises the stream. */
int parafac2_set_sched(parafac2_ctx* c, const parafac2_sched* sched);

/* Time candidate schedules on real iterations of the context and keep the
 * fastest: tile_rounds in {1, 2, 4, 8, 16} x {static, dynamic}, then m2_tiles
 * in {128, 256, 512} (up to the capacity), then (m2_threads, m2_blocks) in
 * {(default, 1), (512, 2), (768, 2), (512, 3), (256, 4)}, then warm_polar in
 * {0, 1} where bases are kept; the graph setting is kept.  Every
 * trial runs iters_per_trial (>= 1) iterations, which advance the
 * decomposition like parafac2_iterate.  chosen (host, or NULL) receives the
 * schedule kept, best_ms (host, or NULL) its milliseconds per iteration. */
int parafac2_autotune(parafac2_ctx* c, int32_t iters_per_trial, parafac2_sched* chosen,
                      double* best_ms);

/* Release a context (the caller's buffers are not freed). */
void parafac2_destroy(parafac2_ctx* c);

/* ---- batches of independent decompositions --------------------------------
 * Not in the paper, which runs one problem at a time; it extends the paper's
 * per-subject independence (Sec. "Methodology") to independent problems.  A
 * batch drives n contexts (each made by parafac2_init, any mix of K, J and R)
 * in lock step: every kernel of an iteration runs once per rank present in
 * the batch, over the tiles of all its problems, instead of once per problem.
 * The contexts must share the batch's stream and must all be at the same
 * point: equal iteration parity and no context iterated on its own since the
 * last batch call (else P2_ESTATE).  Contexts of one rank must have equal
 * tau_polar, tau_pinv and max_sweeps.  A context may still be used on its own
 * between batch calls (get_mttkrp, get_q, iterate), which moves it out of
 * step until the others catch up. */
typedef struct parafac2_batch parafac2_batch;

/* Bytes of device workspace (descriptors, tile lists, counters) for a batch
 * of these n contexts.  Touches no GPU. */
int parafac2_batch_workspace_size(parafac2_ctx* const* ctxs, int32_t n, size_t* bytes);

/* Create a batch over ctxs[0..n) (host array of handles, borrowed until
 * parafac2_batch_destroy).  workspace: device, 256-byte aligned, at least
 * parafac2_batch_workspace_size bytes.  sched may be NULL (defaults).
 * Synchronises the stream once. */
int parafac2_batch_create(parafac2_batch** out, parafac2_ctx* const* ctxs, int32_t n,
                          void* workspace, size_t ws_bytes, void* stream,
                          const parafac2_sched* sched);

/* n_iters iterations of every context of the batch.  fit_host and
 * loss_host (host, or NULL) receive n_iters x n values, entry [i * n + b] for
 * iteration i of context b.  Each context's H, V, W are updated as by
 * parafac2_iterate. */
int parafac2_batch_iterate(parafac2_batch* b, int32_t n_iters, double* fit_host,
                           double* loss_host);

int parafac2_batch_set_sched(parafac2_batch* b, const parafac2_sched* sched);

/* As parafac2_autotune, over the whole batch. */
int parafac2_batch_autotune(parafac2_batch* b, int32_t iters_per_trial, parafac2_sched* chosen,
                            double* best_ms);

/* Per-phase timing of batch iterations, as for a context. */
int parafac2_batch_set_profiling(parafac2_batch* b, int32_t on);
int parafac2_batch_get_profile(parafac2_batch* b, double* ms, int64_t* launches);

void parafac2_batch_destroy(parafac2_batch* b);

/* ---- projection of new subjects onto fixed (V, H) --------------------------
 * Not in the paper: it applies the subject-wise half of Algorithm
 * "PARAFAC2-ALS" with V and H fixed.  For each request subject, starting from
 * w (R), repeat n_steps times: Q = polar(X V diag(w) H^T) (objective
 * (procrustes_obj)); w <- diag(H^T Q^T X V) ((V^T V) * (H^T H))^+
 * (equation (mttkrp3_row_wise) and the W update of Algorithm "CP-ALS").  */

/* Bytes of device workspace for a model of J x R. */
int parafac2_model_workspace_size(int64_t J, int32_t R, size_t* bytes);

/* Create a model.  V (device, J x R float32) and H (device, R x R float64)
 * are copied into the workspace (device, >= parafac2_model_workspace_size
 * bytes, borrowed until parafac2_model_destroy).  Synchronises once. */
int parafac2_model_create(parafac2_model** out, int64_t J, int32_t R, const float* V,
                          const double* H, void* workspace, size_t ws_bytes, void* stream);

/* Project req->K subjects (device CSR with req->J equal to the model's J,
 * I_k >= R).  Subject k's result depends only on its own slice.
 *   w0      device K x R float32 start values, or NULL for all ones;
 *   Q_out   device (sum_k I_k) x R float32 (rows in req's row order), or NULL;
 *   w_out   device K x R float32 (required);
 *   loss_out device K float64 ||X_k - Q_k H diag(w_k) V^T||_F^2, or NULL.
 * stream: NULL uses the model's stream.  Nothing is synchronised. */
int parafac2_project(parafac2_model* m, const parafac2_csr* req, int32_t n_steps, const float* w0,
                     float* Q_out, float* w_out, double* loss_out, void* stream);

void parafac2_model_destroy(parafac2_model* m);

/* parafac2_project for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same projection as parafac2_model_create + parafac2_project, with the
 * model state (V in rows of R rounded up to 4 floats, H, (V^T V) * (H^T H)
 * and its pseudo-inverse) built on the stream in a device scratch array of
 * the library instead of a caller workspace.  The scratch holds at most
 * 8 MiB of model state: J * ceil4(R) * 4 + 6 * R * R * 8 + 4 * J bytes (plus
 * 256-byte alignment of each part), e.g. J <= 50,000 at R = 40; larger J or R
 * gives P2_EINVAL.  Nothing is allocated and nothing is synchronised.  V, H,
 * req, w0, Q_out, w_out and loss_out are as for parafac2_model_create and
 * parafac2_project (device); stream as elsewhere (NULL = default stream).
 * Each device has one scratch array, shared by every call on it and left
 * holding the last call's model state: calls that overlap on one device
 * (other streams, other threads) race and give wrong results; serialise
 * them on one stream. */
int parafac2_project_noalloc(int64_t J, int32_t R, const float* V, const double* H,
                             const parafac2_csr* req, int32_t n_steps, const float* w0,
                             float* Q_out, float* w_out, double* loss_out, void* stream);

/* ---- serving: continuous batching of projection requests ------------------
 * A server projects requests (single new subjects, each an I x J slice in
 * host memory) onto a model as they arrive.  Requests wait in a bounded host
 * queue; whenever one of the server's batch slots is free, the queued
 * requests at the front that fit the slot's capacity (requests, rows,
 * nonzeros: the slot's share of the workspace) are packed into it, copied to
 * the device and projected on the slot's own stream, so batches run and copy
 * while others are in flight.  Every request is computed exactly as by
 * parafac2_project on its own (same kernel, results depend only on its own
 * slice), so a result is bitwise the same alone and in any mix.
 * The server allocates pinned host staging buffers and one stream per slot
 * (default priority) at create time; device memory comes from the workspace.
 * Not thread-safe: one thread submits and polls. */
typedef struct parafac2_server parafac2_server;

typedef struct {
  int32_t slots;        /* batches in flight; 0 -> 4                        */
  int32_t max_requests; /* requests per batch; 0 -> 512                     */
  int64_t max_rows;     /* rows per batch; 0 -> 65536                       */
  int64_t max_nnz;      /* nonzeros per batch; 0 -> 1 << 21                 */
  int32_t max_queue;    /* requests waiting on the host; 0 -> 1 << 16       */
  int32_t n_steps;      /* alternations per request; 0 -> 10                */
  int32_t want_q;       /* 1: also return each request's Q (I x R)          */
  int32_t reserved[5];
} parafac2_server_opts;

/* Device workspace bytes of a server over model m. */
int parafac2_server_workspace_size(const parafac2_model* m, const parafac2_server_opts* o,
                                   size_t* bytes);

/* Create a server (workspace: device, 256-byte aligned, borrowed until
 * destroy; the model must outlive the server). */
int parafac2_server_create(parafac2_server** out, parafac2_model* m,
                           const parafac2_server_opts* o, void* workspace, size_t ws_bytes);

/* Queue one request, copied from host memory: I rows, row_ptr (host, I+1
 * offsets from 0), col (host, nnz, in [0, J)), val (host, nnz, finite).
 * P2_EINVAL if the request is malformed, has I < R, or can never fit one
 * batch; P2_EBUSY if the queue is full.  Launches nothing by itself. */
int parafac2_server_submit(parafac2_server* s, int64_t id, int32_t I, const int64_t* row_ptr,
                           const int32_t* col, const float* val);

/* Collect finished batches and start queued requests on free slots, then
 * return up to max_out finished results in completion order: ids (host,
 * max_out), w (host, max_out x R float32), loss (host, max_out float64,
 * ||X - Q H diag(w) V^T||_F^2, or NULL); with want_q, q (host, q_cap rows x R
 * float32, concatenated in result order) and q_rows (host, max_out) -- a
 * result whose Q no longer fits q_cap stays for the next poll.  *n_out gets
 * the number returned.  Never blocks. */
int parafac2_server_poll(parafac2_server* s, int32_t max_out, int64_t* ids, float* w,
                         double* loss, float* q, int64_t q_cap, int32_t* q_rows, int32_t* n_out);

/* Requests queued on the host, in flight on the device, and finished but not
 * yet returned by poll. */
int parafac2_server_pending(parafac2_server* s, int64_t* queued, int64_t* in_flight,
                            int64_t* finished);

/* Wait for every request in flight to finish (queued ones are started as
 * slots free up), without returning results. */
int parafac2_server_drain(parafac2_server* s);

void parafac2_server_destroy(parafac2_server* s);

#ifdef __cplusplus
}
#endif

#endif /* PARAFAC2_H */
