// Host-side interface of the HIP kernels (launchers dispatch on R at run time).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace p2 {

struct XEnc;
struct XRaw;
struct ProbDesc;
struct Tile;

struct PolarParams {
  double tau_polar;  // relative eigenvalue cut in G^{-1/2}
  double tau_pinv;   // relative eigenvalue cut of the normal-equation pseudo-inverses
  double tol;        // Jacobi rotation threshold |g_p . g_q| > tol ||g_p|| ||g_q||
  double tau_c;      // relative eigenvalue cut of C = A^T A in the factored polar
  double tau_s;      // relative singular value cut of T in the factored polar
  double stop2;      // a Jacobi sweep with no pair above gamma^2 > stop2 alpha beta ends the solve
  int max_sweeps;
};

bool rank_supported(int R);
// Whether the warm-started Procrustes kernels are built for rank R.
bool warm_supported(int R);
int lds_bytes_per_cu();

// Largest number of hot columns whose mode-2 partial sums fit the LDS budget.
int mode2_max_hot(int R);

// One launch group: problems of one rank R whose per-iteration kernels run
// together.  Every pointer is device memory.
struct BatchView {
  int R = 0, np = 0;
  const ProbDesc* desc = nullptr;  // [np]
  const Tile* tiles = nullptr;     // Procrustes / mode-3 tiles, ntiles % kBins == 0
  int ntiles = 0;
  const Tile* m2tiles = nullptr;   // mode-2 tiles, nm2 % kBins == 0
  int nm2 = 0;
  int* tickets = nullptr;          // kTicketKinds * kBins counters (dynamic schedule)
  int dynamic = 0;
  int warm = 0;                    // warm-started polar (every problem has its basis E);
                                   // plan_launch clears it for ranks built without it
  int nonneg = 0;                  // some problem updates V and W by NNLS
  int max_hot = 0;                 // hot columns planned by the problems (max over them)
  int64_t maxK = 0, maxJ = 0;
  int64_t maxEcon = 0;             // most subjects with I_k < R in one problem
  int m2_blocks = 0;               // mode-2 blocks meant to share a CU (0 = 1)
  int m2_threads = 0;              // in: requested mode-2 block size (0 = default); out: used
  // filled by plan_launch (needs the current device; nothing but launches
  // happen afterwards, so the run_* calls below may be captured in a graph)
  int grid_alpha = 0, grid_gamma = 0, grid_mode2 = 0;
  int m2_hot = 0;                  // hot columns of the mode-2 launch (<= max_hot)
  size_t m2_lds = 0;               // dynamic LDS of one mode-2 block
};

// Subjects per Procrustes / mode-3 tile step (subject groups of one
// workgroup), and per mode-2 workgroup round.
int polar_tile_unit(int R);
int mode2_tile_unit(int R);
// Threads per block of a kernel (0 alpha, 1 gamma, 2 mode2, 3 project, 4 getq).
int launch_threads(int R, int kernel);
size_t launch_lds(int R, int kernel);

hipError_t plan_launch(BatchView& b);
hipError_t run_alpha(const BatchView& b, int parity, const PolarParams& pp, hipStream_t s);
hipError_t run_gamma(const BatchView& b, int parity, int do_next, const PolarParams& pp,
                     hipStream_t s);
hipError_t run_mode2(const BatchView& b, int parity, hipStream_t s);
hipError_t run_gram(const BatchView& b, int which, int parity, hipStream_t s);
hipError_t run_solve_h(const BatchView& b, const PolarParams& pp, hipStream_t s);
hipError_t run_vupdate(const BatchView& b, int parity, hipStream_t s);
// Non-negative V_{t+1} rows of the problems with the constraint (instead of
// run_vupdate); their W rows are solved in run_gamma.
hipError_t run_nnls(const BatchView& b, int parity, hipStream_t s);
// Loss terms of the subjects with I_k < R (after the W update).
hipError_t run_econ_fit(const BatchView& b, int parity, hipStream_t s);
hipError_t run_solve_n3(const BatchView& b, const PolarParams& pp, hipStream_t s);
hipError_t run_vscale(const BatchView& b, int parity, hipStream_t s);
// Zero per-problem accumulators: 1 M1, 2 W^T W, 4 V^T V raw, 8 fit terms, 16 M2.
hipError_t run_zero(const BatchView& b, int mask, hipStream_t s);
hipError_t run_fit(const BatchView& b, hipStream_t s);
hipError_t run_reset_tickets(const BatchView& b, hipStream_t s);
hipError_t run_gram_rows(int R, const float* A, int64_t n, int lda, double* out, hipStream_t s);
// Q_k (Hm == nullptr) or U_k = Q_k Hm of subjects [k0, k1)
hipError_t run_getq(int R, const XEnc& X, int64_t k0, int64_t k1, const float* V, const double* F,
                    float* Q, int64_t row0, const double* Hm, hipStream_t s);
hipError_t run_project(int R, const XRaw& X, int64_t K, const float* V, const double* H,
                       const double* N3, const double* N3p, int n_steps, const float* w0,
                       float* Qout, float* wout, double* lossout, const PolarParams& pp,
                       hipStream_t s);

// init-time helpers (R-independent)
hipError_t run_validate(const int64_t* subj_ptr, const int64_t* row_ptr, const int32_t* col,
                        const float* val, int64_t K, int64_t n_rows, int64_t nnz, int64_t J,
                        int min_rows, int* err, int64_t* zbase, int64_t* rbase, hipStream_t s);
hipError_t run_encode(const int64_t* subj_ptr, const int64_t* row_ptr, const int32_t* col,
                      const float* val, int64_t K, int64_t nnz, const int32_t* rank,
                      uint16_t* rstart, uint16_t* nzrow, uint16_t* col16, float* val_out,
                      double* nx2, hipStream_t s);
hipError_t run_col_hist(const int32_t* col, int64_t nnz, int64_t J, unsigned int* hist,
                        hipStream_t s);
hipError_t run_permute_rows(const float* src, float* dst, int64_t J, int R, int ld_src,
                            int ld_dst, const int32_t* map, hipStream_t s);
hipError_t run_fill_f64(double* p, int64_t n, double v, hipStream_t s);
hipError_t run_fill_f32(float* p, int64_t n, float v, hipStream_t s);
// K identity bases (NC x R floats each, NC = R rounded up to even)
hipError_t run_eye_basis(float* E, int64_t K, int R, hipStream_t s);
hipError_t run_model_prep(int R, const double* VtV, const double* H, double* HtH, double* N3,
                          double* N3p, const PolarParams& pp, hipStream_t s);
hipError_t run_iota(int32_t* p, int64_t n, hipStream_t s);

// The explicit-Y ("Sparse PARAFAC2") baseline of one problem (p2_baseline.hip).
struct BaselineView {
  const int64_t* zbase = nullptr;   // per-subject nonzero offsets (encoded slices)
  const int64_t* rbase = nullptr;   // per-subject row offsets
  const uint16_t* erow = nullptr;   // nonzeros sorted by (column, row) per subject: row
  const float* eval = nullptr;      //   and value
  const uint32_t* runs = nullptr;   // runs of equal columns: start | column << 16
  const int64_t* runbase = nullptr; // per-subject run offsets
  int64_t nruns = 0;                // sum_k c_k
  const int32_t* yr = nullptr;      // coordinate tensor Y: R * nruns entries
  const int32_t* yj = nullptr;
  const int32_t* yk = nullptr;
  float* yv = nullptr;
  int64_t ny = 0;
  const float* Q = nullptr;         // materialised Q (n_rows x R)
};
hipError_t run_y_index(int R, const BaselineView& v, int64_t K, hipStream_t s);
hipError_t run_form_y(int R, const BaselineView& v, hipStream_t s);
// mode 1: out1 (R x R FP64) += ...; modes 2, 3: out (rows x ldo) += ...
hipError_t run_coo_mttkrp(int R, const BaselineView& v, int mode, const double* H, const float* V,
                          int ldv, const float* W, double* out1, double* out, int ldo,
                          hipStream_t s);
// dst = (float) src over n rows, columns < R, row stride ld (both)
hipError_t run_round_rows(const double* src, float* dst, int64_t n, int R, int ld, hipStream_t s);
// W = M3 N3^+ and the fit terms of problem desc[0] (K rows)
hipError_t run_wupdate(int R, const ProbDesc* desc, int64_t K, hipStream_t s);

}  // namespace p2
