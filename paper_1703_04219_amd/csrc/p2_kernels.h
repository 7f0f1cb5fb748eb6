// Host-side interface of the HIP kernels (launchers dispatch on R at run time).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace p2 {

struct XEnc;
struct XRaw;

struct PolarParams {
  double tau_polar;  // relative eigenvalue cut in G^{-1/2}
  double tau_pinv;   // relative eigenvalue cut of the normal-equation pseudo-inverses
  double tol;        // Jacobi rotation threshold |g_p . g_q| > tol ||g_p|| ||g_q||
  double tau_c;      // relative eigenvalue cut of C = A^T A in the factored polar
  double tau_s;      // relative singular value cut of T in the factored polar
  int max_sweeps;
};

bool rank_supported(int R);
int lds_bytes_per_cu();

// Largest number of hot columns whose mode-2 partial sums fit the LDS budget.
int mode2_max_hot(int R);

hipError_t run_alpha(int R, const XEnc& X, int64_t K, const float* V, const float* W,
                     const double* H, float* F, double* M1, const PolarParams& pp,
                     hipStream_t s);
hipError_t run_gamma(int R, const XEnc& X, int64_t K, const float* V0, const float* V1, float* W,
                     const double* H, const double* N3, const double* N3p, float* F, float* M3,
                     double* M1next, double* fitacc, int do_next, const PolarParams& pp,
                     hipStream_t s);
hipError_t run_mode2(int R, const XEnc& X, int64_t K, const float* V, const float* W,
                     const double* H, const float* F, float* M2, float* part, int hot,
                     hipStream_t s);
// Bytes of the per-block partial sums that run_mode2 writes.
size_t mode2_part_bytes(int R, int64_t K, int hot);
// Threads per block of a kernel (0 alpha, 1 gamma, 2 mode2, 3 project, 4 getq).
int launch_threads(int R, int kernel);
size_t launch_lds(int R, int kernel);
hipError_t run_gram_tall(int R, const float* A, int64_t n, int lda, double* out, hipStream_t s);
hipError_t run_solve_h(int R, const double* M1, const double* WtW, const double* VtV, double* H,
                       double* HtH, double* N2p, const PolarParams& pp, hipStream_t s);
hipError_t run_vupdate(int R, const float* M2, const double* N2p, int64_t J, float* Vout,
                       hipStream_t s);
hipError_t run_solve_n3(int R, const double* VtVraw, const double* HtH, double* VtV,
                        double* invnorm, double* N3, double* N3p, const PolarParams& pp,
                        hipStream_t s);
hipError_t run_vscale(int R, float* V, int64_t J, const double* invnorm, hipStream_t s);
hipError_t run_getq(int R, const XEnc& X, int64_t k0, int64_t k1, const float* V, const float* F,
                    float* Q, int64_t row0, hipStream_t s);
hipError_t run_project(int R, const XRaw& X, int64_t K, const float* V, const double* H,
                       const double* N3, const double* N3p, int n_steps, const float* w0,
                       float* Qout, float* wout, double* lossout, const PolarParams& pp,
                       hipStream_t s);

// init-time helpers (R-independent)
hipError_t run_validate(const int64_t* subj_ptr, const int64_t* row_ptr, const int32_t* col,
                        const float* val, int64_t K, int64_t n_rows, int64_t nnz, int64_t J,
                        int R, int* err, int64_t* zbase, int64_t* rbase, hipStream_t s);
hipError_t run_encode(const int64_t* subj_ptr, const int64_t* row_ptr, const int32_t* col,
                      const float* val, int64_t K, int64_t nnz, const int32_t* rank,
                      uint16_t* rstart, uint16_t* col16, float* val_out, double* nx2,
                      hipStream_t s);
hipError_t run_col_hist(const int32_t* col, int64_t nnz, int64_t J, unsigned int* hist,
                        hipStream_t s);
hipError_t run_permute_rows(const float* src, float* dst, int64_t J, int R, int ld_src,
                            int ld_dst, const int32_t* map, hipStream_t s);
hipError_t run_fill_f64(double* p, int64_t n, double v, hipStream_t s);
hipError_t run_fill_f32(float* p, int64_t n, float v, hipStream_t s);
hipError_t run_model_prep(int R, const double* VtV, const double* H, double* HtH, double* N3,
                          double* N3p, const PolarParams& pp, hipStream_t s);
hipError_t run_iota(int32_t* p, int64_t n, hipStream_t s);
hipError_t run_fit(const double* fitacc, const double* nx2, double* fit_out, hipStream_t s);

}  // namespace p2
