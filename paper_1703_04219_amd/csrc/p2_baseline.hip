// The "Sparse PARAFAC2" baseline of the paper's experiments (Sec. "Setup":
// the classical PARAFAC2-ALS of Sec. "Classical Algorithm for PARAFAC2"
// running the CP-ALS step on an explicitly formed sparse tensor Y with a
// generic sparse MTTKRP), on the GPU, for comparison with the SPARTan path
// on the same hardware.  Per iteration:
//   1. the Procrustes step (shared with the SPARTan path: F_k from k_alpha);
//   2. Q_k = A_k F_k^T for every subject, materialised (k_getq);
//   3. Y_k = Q_k^T X_k over the nonzero columns of X_k, stored as a
//      coordinate-format tensor with R entries (r, j, k, value) per nonzero
//      column of each subject: R sum_k c_k entries (k_form_y);
//   4. the three MTTKRPs of the CP-ALS step on that tensor by the plain
//      coordinate-format rule (equations (mttkrp1), (mttkrp2), (mttkrp3)):
//      every entry y = Y(r, j, k) adds y * (B(., :) * C(., :)) to row (r, j
//      or k) of the output, where B, C are the two other factors
//      (k_coo_mttkrp); the R x R mode-1 output is summed per block in LDS,
//      the others with FP64 global atomics (a hot column receives millions
//      of terms: FP32 atomics lose about 1e-4 of it), then rounded to FP32;
//   5. the W rows from M3 (k_wupdate), with the fit terms.
// The coordinate tensor's indices are built once at init from each subject's
// nonzeros sorted by column (the same per-subject runs of equal columns).
#include <hip/hip_runtime.h>

#include "p2_batch.h"
#include "p2_device.h"
#include "p2_kernels.h"

namespace p2 {

extern __shared__ __align__(16) unsigned char p2_base_smem[];

// Y values of subject runs: one thread per run u (a nonzero column j of
// subject k = yk[u * R]), R values y(r) = sum over the run's nonzeros x_ij
// Q_k(i, r), written at u * R + r.  Q is the materialised (n_rows x R) Q.
template <int R>
__global__ void __launch_bounds__(256) k_form_y(const int64_t* __restrict__ zbase,
                                                 const int64_t* __restrict__ rbase,
                                                 const uint16_t* __restrict__ erow,
                                                 const float* __restrict__ eval,
                                                 const uint32_t* __restrict__ runs,
                                                 const int64_t* __restrict__ runbase,
                                                 const int32_t* __restrict__ yk,
                                                 const float* __restrict__ Q, int64_t nruns,
                                                 float* __restrict__ yv) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < nruns;
       u += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = glob(yk)[u * R];
    const int64_t z0 = glob(zbase)[k];
    const int nnz_k = (int)(glob(zbase)[k + 1] - z0);
    const int64_t r0 = glob(rbase)[k];
    const int e0 = (int)(glob(runs)[u] & 0xffffu);
    const int e1 = (u + 1 < glob(runbase)[k + 1]) ? (int)(glob(runs)[u + 1] & 0xffffu) : nnz_k;
    float acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0.f;
    for (int e = e0; e < e1; ++e) {
      const float x = glob(eval)[z0 + e];
      const P2_GLOBAL float* q = glob(Q) + (r0 + glob(erow)[z0 + e]) * R;
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] = fmaf(x, q[r], acc[r]);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) glob(yv)[u * R + r] = acc[r];
  }
}

// Generic coordinate-format MTTKRP over n entries (yr, yj, yk, yv) of the
// R x J x K tensor Y.  mode 1: out1 (R x R, FP64) += y (W(k,:) * V(j,:)) at
// row r, summed per block in LDS; mode 2: out (J x ldo) += y (W(k,:) *
// H(r,:)) at row j; mode 3: out (K x ldo) += y (V(j,:) * H(r,:)) at row k.
// V rows have stride ldv, W rows stride R, H is R x R (FP64).
template <int R>
__global__ void __launch_bounds__(256) k_coo_mttkrp(int mode, const int32_t* __restrict__ yr,
                                                     const int32_t* __restrict__ yj,
                                                     const int32_t* __restrict__ yk,
                                                     const float* __restrict__ yv, int64_t n,
                                                     const double* __restrict__ H,
                                                     const float* __restrict__ V, int ldv,
                                                     const float* __restrict__ W,
                                                     double* __restrict__ out1,
                                                     double* __restrict__ out, int ldo) {
  double* sh = reinterpret_cast<double*>(p2_base_smem);  // mode 1: R x R
  float* hs = reinterpret_cast<float*>(sh + R * R);       // H as float, R x R
  for (int q = threadIdx.x; q < R * R; q += blockDim.x) {
    sh[q] = 0.0;
    hs[q] = (float)glob(H)[q];
  }
  __syncthreads();
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int r = glob(yr)[t];
    const int64_t j = glob(yj)[t];
    const int64_t k = glob(yk)[t];
    const float y = glob(yv)[t];
    if (y == 0.f) continue;
    if (mode == 1) {
#pragma unroll
      for (int c = 0; c < R; ++c)
        atomicAdd(sh + r * R + c, (double)(y * glob(W)[k * R + c] * glob(V)[j * ldv + c]));
    } else if (mode == 2) {
#pragma unroll
      for (int c = 0; c < R; ++c)
        gadd(out + j * ldo + c, (double)(y * glob(W)[k * R + c] * hs[r * R + c]));
    } else {
#pragma unroll
      for (int c = 0; c < R; ++c)
        gadd(out + k * ldo + c, (double)(y * glob(V)[j * ldv + c] * hs[r * R + c]));
    }
  }
  if (mode == 1) {
    __syncthreads();
    for (int q = threadIdx.x; q < R * R; q += blockDim.x)
      if (sh[q] != 0.0) gadd(out1 + q, sh[q]);
  }
}

// dst(i, c) = (float) src(i, c) for rows i < n, columns c < R of stride ld.
__global__ void __launch_bounds__(256) k_round_rows(const double* __restrict__ src,
                                                     float* __restrict__ dst, int64_t n, int R,
                                                     int ld) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n * ld;
       t += (int64_t)gridDim.x * blockDim.x)
    if ((int)(t % ld) < R) glob(dst)[t] = (float)glob(src)[t];
}

// W(k, :) = M3(k, :) N3^+ and the fit terms <W, M3>, W N3 W^T (from the stored
// float W); one thread per row.  grid = rows.
template <int R>
__global__ void __launch_bounds__(256) k_wupdate(const ProbDesc* __restrict__ P) {
  constexpr SmallLayout SL = small_layout(R);
  const ProbDesc& D = P[0];
  double* N3s = reinterpret_cast<double*>(p2_base_smem);
  double* N3ps = N3s + R * R;
  double* shf = N3ps + R * R;
  for (int q = threadIdx.x; q < R * R; q += blockDim.x) {
    N3s[q] = glob(D.small)[SL.N3 + q];
    N3ps[q] = glob(D.small)[SL.N3p + q];
  }
  if (threadIdx.x < 2) shf[threadIdx.x] = 0.0;
  __syncthreads();
  double fa = 0.0, fb = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < D.K;
       k += (int64_t)gridDim.x * blockDim.x) {
    double m[R], w[R];
#pragma unroll
    for (int l = 0; l < R; ++l) m[l] = (double)glob(D.M3)[k * R + l];
#pragma unroll
    for (int c = 0; c < R; ++c) {
      double t = 0.0;
#pragma unroll
      for (int l = 0; l < R; ++l) t = fma(m[l], N3ps[l * R + c], t);
      const float wf = (float)t;
      glob(D.W)[k * R + c] = wf;
      w[c] = (double)wf;
    }
#pragma unroll
    for (int c = 0; c < R; ++c) {
      double t = 0.0;
#pragma unroll
      for (int l = 0; l < R; ++l) t = fma(N3s[c * R + l], w[l], t);
      fa = fma(w[c], m[c], fa);
      fb = fma(w[c], t, fb);
    }
  }
  atomicAdd(&shf[0], fa);
  atomicAdd(&shf[1], fb);
  __syncthreads();
  if (threadIdx.x == 0) {
    gadd(D.small + SL.fitacc + 0, shf[0]);
    gadd(D.small + SL.fitacc + 1, shf[1]);
  }
}

// Coordinate indices of Y: entry u * R + r is (r, column of run u, subject k)
// for every run u of subject k.  One thread per subject.
__global__ void __launch_bounds__(256) k_y_index(const uint32_t* __restrict__ runs,
                                                  const int64_t* __restrict__ runbase, int64_t K,
                                                  int R, int32_t* __restrict__ yr,
                                                  int32_t* __restrict__ yj,
                                                  int32_t* __restrict__ yk) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < K;
       k += (int64_t)gridDim.x * blockDim.x) {
    for (int64_t u = glob(runbase)[k]; u < glob(runbase)[k + 1]; ++u) {
      const int32_t j = (int32_t)(glob(runs)[u] >> 16);
      for (int r = 0; r < R; ++r) {
        glob(yr)[u * R + r] = r;
        glob(yj)[u * R + r] = j;
        glob(yk)[u * R + r] = (int32_t)k;
      }
    }
  }
}

namespace {

inline int grid_of(int64_t n, int per) {
  int64_t b = (n + per - 1) / per;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return (int)b;
}

template <int R>
hipError_t form_y_t(const BaselineView& v, hipStream_t s) {
  hipLaunchKernelGGL(k_form_y<R>, dim3(grid_of(v.nruns, 256)), dim3(256), 0, s, v.zbase, v.rbase,
                     v.erow, v.eval, v.runs, v.runbase, v.yk, v.Q, v.nruns, v.yv);
  return hipGetLastError();
}

template <int R>
hipError_t coo_t(const BaselineView& v, int mode, const double* H, const float* V, int ldv,
                 const float* W, double* out1, double* out, int ldo, hipStream_t s) {
  const size_t lds = sizeof(double) * R * R + sizeof(float) * R * R;
  hipLaunchKernelGGL(k_coo_mttkrp<R>, dim3(grid_of(v.ny, 256 * 8)), dim3(256), lds, s, mode, v.yr,
                     v.yj, v.yk, v.yv, v.ny, H, V, ldv, W, out1, out, ldo);
  return hipGetLastError();
}

template <int R>
hipError_t wupdate_t(const ProbDesc* desc, int64_t K, hipStream_t s) {
  const size_t lds = sizeof(double) * (2 * R * R + 2);
  hipLaunchKernelGGL(k_wupdate<R>, dim3(grid_of(K, 256 * 4)), dim3(256), lds, s, desc);
  return hipGetLastError();
}

}  // namespace

#define P2_BDISPATCH(R, CALL)                 \
  switch (R) {                                \
    case 1: { constexpr int RR = 1; CALL; } \
    case 2: { constexpr int RR = 2; CALL; } \
    case 3: { constexpr int RR = 3; CALL; } \
    case 4: { constexpr int RR = 4; CALL; } \
    case 5: { constexpr int RR = 5; CALL; } \
    case 6: { constexpr int RR = 6; CALL; } \
    case 7: { constexpr int RR = 7; CALL; } \
    case 8: { constexpr int RR = 8; CALL; } \
    case 9: { constexpr int RR = 9; CALL; } \
    case 10: { constexpr int RR = 10; CALL; } \
    case 11: { constexpr int RR = 11; CALL; } \
    case 12: { constexpr int RR = 12; CALL; } \
    case 13: { constexpr int RR = 13; CALL; } \
    case 14: { constexpr int RR = 14; CALL; } \
    case 15: { constexpr int RR = 15; CALL; } \
    case 16: { constexpr int RR = 16; CALL; } \
    case 17: { constexpr int RR = 17; CALL; } \
    case 18: { constexpr int RR = 18; CALL; } \
    case 19: { constexpr int RR = 19; CALL; } \
    case 20: { constexpr int RR = 20; CALL; } \
    case 21: { constexpr int RR = 21; CALL; } \
    case 22: { constexpr int RR = 22; CALL; } \
    case 23: { constexpr int RR = 23; CALL; } \
    case 24: { constexpr int RR = 24; CALL; } \
    case 25: { constexpr int RR = 25; CALL; } \
    case 26: { constexpr int RR = 26; CALL; } \
    case 27: { constexpr int RR = 27; CALL; } \
    case 28: { constexpr int RR = 28; CALL; } \
    case 29: { constexpr int RR = 29; CALL; } \
    case 30: { constexpr int RR = 30; CALL; } \
    case 31: { constexpr int RR = 31; CALL; } \
    case 32: { constexpr int RR = 32; CALL; } \
    case 33: { constexpr int RR = 33; CALL; } \
    case 34: { constexpr int RR = 34; CALL; } \
    case 35: { constexpr int RR = 35; CALL; } \
    case 36: { constexpr int RR = 36; CALL; } \
    case 37: { constexpr int RR = 37; CALL; } \
    case 38: { constexpr int RR = 38; CALL; } \
    case 39: { constexpr int RR = 39; CALL; } \
    case 40: { constexpr int RR = 40; CALL; } \
    default: return hipErrorInvalidValue;     \
  }

hipError_t run_y_index(int R, const BaselineView& v, int64_t K, hipStream_t s) {
  hipLaunchKernelGGL(k_y_index, dim3(grid_of(K, 256)), dim3(256), 0, s, v.runs, v.runbase, K, R,
                     const_cast<int32_t*>(v.yr), const_cast<int32_t*>(v.yj),
                     const_cast<int32_t*>(v.yk));
  return hipGetLastError();
}

hipError_t run_form_y(int R, const BaselineView& v, hipStream_t s) {
  P2_BDISPATCH(R, return form_y_t<RR>(v, s))
}

hipError_t run_coo_mttkrp(int R, const BaselineView& v, int mode, const double* H, const float* V,
                          int ldv, const float* W, double* out1, double* out, int ldo,
                          hipStream_t s) {
  P2_BDISPATCH(R, return coo_t<RR>(v, mode, H, V, ldv, W, out1, out, ldo, s))
}

hipError_t run_round_rows(const double* src, float* dst, int64_t n, int R, int ld, hipStream_t s) {
  hipLaunchKernelGGL(k_round_rows, dim3(grid_of(n * ld, 256 * 8)), dim3(256), 0, s, src, dst, n, R,
                     ld);
  return hipGetLastError();
}

hipError_t run_wupdate(int R, const ProbDesc* desc, int64_t K, hipStream_t s) {
  P2_BDISPATCH(R, return wupdate_t<RR>(desc, K, s))
}

}  // namespace p2
