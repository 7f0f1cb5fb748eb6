// Rank-independent kernels of the PARAFAC2-ALS hot path (init-time
// validation and encoding, fills) and the run-time dispatch on R: each run_*
// call goes through the rank's table of launchers (RankOps, built in
// p2_ranks.hip from the templates of p2_rank_impl.h).
#include "p2_rank_impl.h"

namespace p2 {

__global__ void k_fill_i32(int* __restrict__ p, int n, int v) {
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) p[q] = v;
}

__global__ void k_iota(int32_t* __restrict__ p, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    p[t] = (int32_t)t;
}

// ---------------------------------------------------------------------------
// init-time kernels (encoding, validation, statistics)
// ---------------------------------------------------------------------------

__global__ void k_validate_rows(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                const float* __restrict__ val, int64_t n_rows, int64_t nnz,
                                int64_t J, int* __restrict__ err) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_rows;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = row_ptr[i], b = row_ptr[i + 1];
    if (a < 0 || b < a || b > nnz) {
      atomicOr(err, 1);
      continue;
    }
    int prev = -1;
    for (int64_t z = a; z < b; ++z) {
      const int cz = col[z];
      if (cz < 0 || cz >= J) atomicOr(err, 2);
      if (cz <= prev) atomicOr(err, 4);
      prev = cz;
      if (!isfinite(val[z])) atomicOr(err, 8);
    }
  }
}

__global__ void k_validate_subj(const int64_t* __restrict__ subj_ptr,
                                const int64_t* __restrict__ row_ptr, int64_t K, int64_t n_rows,
                                int min_rows, int* __restrict__ err,
                                int64_t* __restrict__ zbase, int64_t* __restrict__ rbase) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k <= K;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = subj_ptr[k];
    if (r < 0 || r > n_rows) {
      atomicOr(err, 16);
      continue;
    }
    rbase[k] = r;
    zbase[k] = row_ptr[r];
    if (k < K) {
      const int64_t r1 = subj_ptr[k + 1];
      if (r1 < r || r1 > n_rows) {
        atomicOr(err, 16);
        continue;
      }
      const int64_t I = r1 - r;
      if (I < min_rows) atomicOr(err, 32);
      if (I > 65535) atomicOr(err, 64);
      if (r1 <= n_rows && row_ptr[r1] - row_ptr[r] > 65535) atomicOr(err, 128);
    }
  }
}

__global__ void k_encode_rows(const int64_t* __restrict__ subj_ptr,
                              const int64_t* __restrict__ row_ptr, int64_t K,
                              uint16_t* __restrict__ rstart, uint16_t* __restrict__ nzrow) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < K;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r0 = subj_ptr[k], r1 = subj_ptr[k + 1];
    const int64_t z0 = row_ptr[r0];
    for (int64_t i = r0; i < r1; ++i) {
      rstart[i] = (uint16_t)(row_ptr[i] - z0);
      for (int64_t z = row_ptr[i]; z < row_ptr[i + 1]; ++z) nzrow[z] = (uint16_t)(i - r0);
    }
  }
}

// Column histogram: block-private counts in LDS (J <= kHistLds), then one
// global atomic per touched column per block.  Zipf-skewed columns make
// direct global atomics on the hottest counters serialise.
constexpr int kHistLds = 16384;

__global__ void k_col_hist(const int32_t* __restrict__ col, int64_t nnz, int64_t J,
                           unsigned int* __restrict__ hist) {
  __shared__ unsigned int sh[kHistLds];
  const bool local = J <= kHistLds;
  if (local) {
    for (int i = threadIdx.x; i < J; i += blockDim.x) sh[i] = 0u;
    __syncthreads();
  }
  for (int64_t z = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; z < nnz;
       z += (int64_t)gridDim.x * blockDim.x) {
    if (local)
      atomicAdd(&sh[col[z]], 1u);
    else
      atomicAdd(&hist[col[z]], 1u);
  }
  if (local) {
    __syncthreads();
    for (int i = threadIdx.x; i < J; i += blockDim.x)
      if (sh[i]) atomicAdd(&hist[i], sh[i]);
  }
}

__global__ void k_encode_cols(const int32_t* __restrict__ col, const float* __restrict__ val,
                              int64_t nnz, const int32_t* __restrict__ rank,
                              uint16_t* __restrict__ col16, float* __restrict__ val_out,
                              double* __restrict__ nx2) {
  double acc = 0.0;
  for (int64_t z = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; z < nnz;
       z += (int64_t)gridDim.x * blockDim.x) {
    col16[z] = (uint16_t)rank[col[z]];
    const float v = val[z];
    val_out[z] = v;
    acc = fma((double)v, (double)v, acc);
  }
  // wave reduction, then one atomic per wave
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0 && acc != 0.0) atomicAdd(nx2, acc);
}

// Vint(rank[j], :) = V(j, :)  or the inverse when to_user != 0
__global__ void k_permute_rows(const float* __restrict__ src, float* __restrict__ dst, int64_t J,
                               int R, int ld_src, int ld_dst, const int32_t* __restrict__ map) {
  const int64_t n = J * R;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = t / R;
    const int c = (int)(t % R);
    dst[(int64_t)map[j] * ld_dst + c] = src[j * ld_src + c];
  }
}

__global__ void k_fill_f64(double* __restrict__ p, int64_t n, double v) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    p[t] = v;
}

// Per-subject start bases of the warm-started polar: column p of subject k is
// e_p (p < R) or zero (the padding column of odd R).
__global__ void k_eye_basis(float* __restrict__ E, int64_t K, int R, int NC) {
  const int64_t per = (int64_t)NC * R;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < K * per;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = t % per;
    const int p = (int)(q / R), i = (int)(q % R);
    E[t] = (p == i) ? 1.f : 0.f;
  }
}

__global__ void k_fill_f32(float* __restrict__ p, int64_t n, float v) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    p[t] = v;
}

namespace {

const RankOps* ops_for(int R) {
  switch (R) {
#define P2_CASE(r) \
  case r:          \
    return rank_ops_##r();
    P2_RANKS(P2_CASE)
#undef P2_CASE
    default:
      return nullptr;
  }
}

}  // namespace

// the launchers of rank R, or an error for a rank that is not built
#define P2_OPS(R)                           \
  const RankOps* o = ops_for(R);            \
  if (o == nullptr) return hipErrorInvalidValue

bool rank_supported(int R) { return ops_for(R) != nullptr; }

int lds_bytes_per_cu() { return (int)kLdsPerCu; }

int mode2_max_hot(int R) {
  const RankOps* o = ops_for(R);
  return o ? o->max_hot : 0;
}

size_t launch_lds(int R, int kernel) {
  const RankOps* o = ops_for(R);
  return (o && kernel >= 0 && kernel < 5) ? o->lds[kernel] : 0;
}

int launch_threads(int R, int kernel) {
  const RankOps* o = ops_for(R);
  return (o && kernel >= 0 && kernel < 5) ? o->threads[kernel] : 0;
}

hipError_t run_getq(int R, const XEnc& X, int64_t k0, int64_t k1, const float* V, const double* F,
                    float* Q, int64_t row0, const double* Hm, hipStream_t s) {
  P2_OPS(R);
  return o->getq(X, k0, k1, V, F, Q, row0, Hm, s);
}

hipError_t run_project(int R, const XRaw& X, int64_t K, const float* V, const double* H,
                       const double* N3, const double* N3p, int n_steps, const float* w0,
                       float* Qout, float* wout, double* lossout, const PolarParams& pp,
                       hipStream_t s) {
  P2_OPS(R);
  return o->project(X, K, V, H, N3, N3p, n_steps, w0, Qout, wout, lossout, pp, s);
}

hipError_t run_validate(const int64_t* subj_ptr, const int64_t* row_ptr, const int32_t* col,
                        const float* val, int64_t K, int64_t n_rows, int64_t nnz, int64_t J,
                        int min_rows, int* err, int64_t* zbase, int64_t* rbase, hipStream_t s) {
  hipLaunchKernelGGL(k_validate_subj, dim3(grid1(K + 1)), dim3(256), 0, s, subj_ptr, row_ptr, K,
                     n_rows, min_rows, err, zbase, rbase);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_validate_rows, dim3(grid1(n_rows)), dim3(256), 0, s, row_ptr, col, val,
                     n_rows, nnz, J, err);
  return hipGetLastError();
}

hipError_t run_encode(const int64_t* subj_ptr, const int64_t* row_ptr, const int32_t* col,
                      const float* val, int64_t K, int64_t nnz, const int32_t* rank,
                      uint16_t* rstart, uint16_t* nzrow, uint16_t* col16, float* val_out,
                      double* nx2, hipStream_t s) {
  hipLaunchKernelGGL(k_encode_rows, dim3(grid1(K)), dim3(256), 0, s, subj_ptr, row_ptr, K, rstart,
                     nzrow);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_encode_cols, dim3(grid1(nnz)), dim3(256), 0, s, col, val, nnz, rank, col16,
                     val_out, nx2);
  return hipGetLastError();
}

hipError_t run_col_hist(const int32_t* col, int64_t nnz, int64_t J, unsigned int* hist,
                        hipStream_t s) {
  int blocks = grid1(nnz);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_col_hist, dim3(blocks), dim3(256), 0, s, col, nnz, J, hist);
  return hipGetLastError();
}

hipError_t run_permute_rows(const float* src, float* dst, int64_t J, int R, int ld_src,
                            int ld_dst, const int32_t* map, hipStream_t s) {
  hipLaunchKernelGGL(k_permute_rows, dim3(grid1(J * R)), dim3(256), 0, s, src, dst, J, R, ld_src,
                     ld_dst, map);
  return hipGetLastError();
}

hipError_t run_fill_f64(double* p, int64_t n, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_f64, dim3(grid1(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t run_eye_basis(float* E, int64_t K, int R, hipStream_t s) {
  hipLaunchKernelGGL(k_eye_basis, dim3(grid1(K * R * R)), dim3(256), 0, s, E, K, R,
                     (R & 1) ? R + 1 : R);
  return hipGetLastError();
}

hipError_t run_fill_f32(float* p, int64_t n, float v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_f32, dim3(grid1(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t run_model_prep(int R, const double* VtV, const double* H, double* HtH, double* N3,
                          double* N3p, const PolarParams& pp, hipStream_t s) {
  P2_OPS(R);
  return o->model_prep(VtV, H, HtH, N3, N3p, pp, s);
}

hipError_t run_iota(int32_t* p, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_iota, dim3(grid1(n)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

bool warm_supported(int R) { return rank_supported(R) && R <= kWarmMaxR; }

int polar_tile_unit(int R) {
  const RankOps* o = ops_for(R);
  return o ? o->polar_unit : 0;
}

int mode2_tile_unit(int R) {
  const RankOps* o = ops_for(R);
  return o ? o->mode2_unit : 0;
}

hipError_t plan_launch(BatchView& b) {
  P2_OPS(b.R);
  return o->plan(b);
}

hipError_t run_alpha(const BatchView& b, int parity, const PolarParams& pp, hipStream_t s) {
  P2_OPS(b.R);
  return o->alpha(b, parity, pp, s);
}

hipError_t run_gamma(const BatchView& b, int parity, int do_next, const PolarParams& pp,
                     hipStream_t s) {
  P2_OPS(b.R);
  return o->gamma(b, parity, do_next, pp, s);
}

hipError_t run_mode2(const BatchView& b, int parity, hipStream_t s) {
  P2_OPS(b.R);
  return o->mode2(b, parity, s);
}

hipError_t run_gram(const BatchView& b, int which, int parity, hipStream_t s) {
  P2_OPS(b.R);
  return o->gram(b, which, parity, s);
}

hipError_t run_solve_h(const BatchView& b, const PolarParams& pp, hipStream_t s) {
  P2_OPS(b.R);
  return o->solve_h(b, pp, s);
}

hipError_t run_vupdate(const BatchView& b, int parity, hipStream_t s) {
  P2_OPS(b.R);
  return o->vupdate(b, parity, s);
}

hipError_t run_econ_fit(const BatchView& b, int parity, hipStream_t s) {
  P2_OPS(b.R);
  return o->econ_fit(b, parity, s);
}

hipError_t run_nnls(const BatchView& b, int parity, hipStream_t s) {
  P2_OPS(b.R);
  return o->nnls(b, parity, s);
}

hipError_t run_solve_n3(const BatchView& b, const PolarParams& pp, hipStream_t s) {
  P2_OPS(b.R);
  return o->solve_n3(b, pp, s);
}

hipError_t run_vscale(const BatchView& b, int parity, hipStream_t s) {
  P2_OPS(b.R);
  return o->vscale(b, parity, s);
}

hipError_t run_zero(const BatchView& b, int mask, hipStream_t s) {
  P2_OPS(b.R);
  return o->zero(b, mask, s);
}

hipError_t run_fit(const BatchView& b, hipStream_t s) {
  P2_OPS(b.R);
  return o->fit(b, s);
}

hipError_t run_reset_tickets(const BatchView& b, hipStream_t s) {
  if (!b.dynamic) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, s, b.tickets, kTicketKinds * kBins, 0);
  return hipGetLastError();
}

hipError_t run_gram_rows(int R, const float* A, int64_t n, int lda, double* out, hipStream_t s) {
  P2_OPS(R);
  return o->gram_rows(A, n, lda, out, s);
}

#undef P2_OPS

}  // namespace p2
