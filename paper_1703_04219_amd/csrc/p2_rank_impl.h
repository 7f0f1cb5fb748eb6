// Rank-templated kernels of the PARAFAC2-ALS hot path (gfx950), their launch
// plans and launchers, and the table of one rank's launchers (RankOps).
// p2_ranks.hip builds the tables, compiled once per subset of the ranks so
// that the subsets compile in parallel; p2_kernels.hip dispatches on R
// through them and holds the rank-independent kernels.
//
// Per-iteration kernel sequence (see p2_capi.hip for the driver):
//   k_alpha     (first iteration only) gather A_k = X_k V, C_k = A_k^T A_k,
//               Procrustes polar in FP64, F_k = G_k^{-1/2} H S_k, mode-1
//               partial (Y_k V) S_k accumulated into M1;
//   k_gram      W^T W;
//   k_solve_h   H <- M1 ((W^T W) * (V^T V))^+, normalise, prepare N2^+;
//   k_mode2_dpp (R <= 16) or k_mode2, then k_mode2_reduce: regather A_k,
//               D_k = A_k F_k^T H S_k, scatter X_k^T D_k into M2;
//   k_vupdate (or k_nnls_rows) / k_gram / k_solve_n3 / k_vscale
//               V <- M2 N2^+, normalise, N3 = (V^T V) * (H^T H) and its
//               pseudo-inverse;
//   k_gamma     regather A_k against V_t and V_{t+1}: mode-3 row
//               diag(H^T F_k A_k^T A'_k), W row update, fit terms, and the
//               next iteration's Procrustes step and mode-1 partial from
//               C'_k = A'_k^T A'_k;
//   k_fit       fit of the iteration.
#pragma once

#include "p2_batch.h"
#include "p2_device.h"
#include "p2_kernels.h"

#include <utility>

namespace p2 {

// ---------------------------------------------------------------------------
// shared helpers
// ---------------------------------------------------------------------------

struct Lane {
  int lane;    // lane in wavefront
  int grp;     // group index in wavefront
  int j;       // position in group
  int gbase;   // first lane of the group
  uint64_t gmask;
  bool live;   // lane belongs to a group
};

template <int R>
__device__ __forceinline__ Lane lane_info() {
  constexpr int NC = Geo<R>::NC;
  constexpr int GPW = Geo<R>::GPW;
  Lane L;
  L.lane = threadIdx.x & (kWave - 1);
  L.grp = L.lane / NC;
  L.live = L.grp < GPW;
  if (L.live) {
    L.j = L.lane - L.grp * NC;
    L.gbase = L.grp * NC;
    L.gmask = (NC == 64) ? ~0ull : (((1ull << NC) - 1ull) << L.gbase);
  } else {
    L.j = 0;
    L.gbase = L.lane;
    L.gmask = 0ull;
  }
  return L;
}

__device__ __forceinline__ void block_reduce_atomic(double* sh, int n, double* out) {
  // sh holds n partial values (already summed in LDS by atomics)
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double v = sh[i];
    if (v != 0.0) gadd(out + i, v);
  }
}

// per-group LDS regions are carved from one dynamic allocation
extern __shared__ __align__(16) unsigned char p2_smem[];

// Per-group LDS of the polar kernels (doubles): a region that holds the
// gather chunks in the first phase and C, F, P and the Jacobi scratch later,
// then w, a second R-vector and the eigenvalue slots.
// LDS layout of the per-subject kernels.  For even R every region below
// starts at an even number of doubles (16-byte aligned), which the vector
// reads of gram_accum rely on.
template <int R>
struct PolarLds {
  static constexpr int NC = Geo<R>::NC;
  static constexpr int LDV = Geo<R>::LDV;
  // rows per lane and gather chunk, and rows per chunk: at small ranks one
  // (a second row's accumulators would cost occupancy), two above
  static constexpr int kRowsPerLane = R <= 10 ? 1 : 2;
  static constexpr int CH = kRowsPerLane * NC;
  // the chunk's rows, in doubles: FP32 rows of A (stride R) and A' (stride
  // LDV) in gamma; FP64 rows (stride R) in alpha and the projection
  static constexpr int kAf = (CH * (R + LDV) + 1) / 2;
  static constexpr int kA = kAf > CH * R ? kAf : CH * R;
  static constexpr int kB = R * R + NC * R;
  // the non-negative W row solve in gamma uses the region once the mode-3 row
  // is formed (its factor, right-hand side and reductions)
  static constexpr int kNnls = R * R + R + 3 * NC;
  static constexpr int kRegion = kA > kB ? (kA > kNnls ? kA : kNnls) : (kB > kNnls ? kB : kNnls);
  // minimum waves per SIMD in k_gamma's launch bound: none asked for.  At
  // R = 10 the kernel fits three waves by itself (163 VGPRs without warm
  // starts; two waves cost about 0.6 ms per launch of the K = 1M pass), and a
  // bound asking for three changed its schedule and cost about 0.2 ms
  static constexpr int kMinWaves = 1;
  // with the W row's NNLS in the kernel (non-negative problems) R = 10 needs
  // about 200 VGPRs; bounded to three waves it spills 92 bytes per lane and
  // runs 10 % faster (5.53 against 6.16 ms per pass at K = 1M)
  static constexpr int kMinWavesNN = R == 10 ? 3 : 1;
  static constexpr int kPerGroup = kRegion + 2 * R + NC;
  static_assert(R % 2 == 1 || (kPerGroup % 2 == 0 && (CH * R) % 4 == 0),
                "even-R group regions and the FP32 A' rows must stay 16-byte aligned");
};

template <int R>
__device__ __forceinline__ void load_shared_rxr(double* dst, const double* __restrict__ src) {
  for (int i = threadIdx.x; i < R * R; i += blockDim.x) dst[i] = glob(src)[i];
}

// M1 partial of one subject, column c: (Y_k V)(:, c) w(c)  (equation (mttkrp1_3))
template <int R>
__device__ __forceinline__ void add_m1(double* shM1, const double (&y)[R], double wc, int c) {
  if (c < R) {
#pragma unroll
    for (int i = 0; i < R; ++i) atomicAdd(&shM1[i * R + c], y[i] * wc);
  }
}

// ---------------------------------------------------------------------------
// Batches.  Every per-iteration kernel below runs over an array of problem
// descriptors (ProbDesc, all of rank R) and, for the per-subject kernels, a
// list of tiles (problem, subject range).  Blocks take tiles either in a
// static order or from per-bin ticket counters in global memory (dynamic);
// per-problem state that a block shares in LDS (H, N3, the mode-1 and fit
// partial sums) is loaded and flushed per tile.  Empty (padding) tiles are
// skipped.
// ---------------------------------------------------------------------------

// Tile index of this block's i-th claim, or -1 when there is none left.
// Static (tickets == nullptr): tiles blockIdx.x, blockIdx.x + gridDim.x, ...;
// with gridDim.x a multiple of kBins, every tile of a block lies in the bin of
// the block's XCD.  Dynamic: the block takes the next tile of its own bin from
// that bin's counter and, once the bin is used up, moves on to the following
// bins.  sh[1] (bins used up so far) starts at 0.
__device__ __forceinline__ int claim_tile(int ntiles, int* tickets, int i, int* sh) {
  if (tickets == nullptr) {
    const int t = blockIdx.x + i * gridDim.x;
    return t < ntiles ? t : -1;
  }
  __syncthreads();  // every thread has read the previous claim
  if (threadIdx.x == 0) {
    int t = -1, b = sh[1];
    const int x0 = blockIdx.x % kBins;
    while (b < kBins) {
      const int x = (x0 + b) % kBins;
      const int tt = atomicAdd(&tickets[x], 1) * kBins + x;
      if (tt < ntiles) {
        t = tt;
        break;
      }
      ++b;
    }
    sh[0] = t;
    sh[1] = b;
  }
  __syncthreads();
  return sh[0];
}

// ---------------------------------------------------------------------------
// k_alpha: the Procrustes step that starts a run of iterations.  Per subject:
// A_k = X_k V (sparse gather, equation (mttkrp1_3)), C_k = A_k^T A_k (FP64),
// F_k and (Y_k V) from the polar factor (objective (procrustes_obj)), mode-1
// partial (Y_k V) S_k added into M1 (equation (mttkrp1_2)).
// ---------------------------------------------------------------------------
template <int R, bool WARM>
__global__ void __launch_bounds__(256) k_alpha(const ProbDesc* __restrict__ P,
                                                const Tile* __restrict__ T, int ntiles,
                                                int* tickets, int parity, PolarParams pp) {
  constexpr int GPW = Geo<R>::GPW;
  constexpr int CH = PolarLds<R>::CH;
  constexpr SmallLayout SL = small_layout(R);
  __shared__ int sh_t[2];
  if (threadIdx.x == 0) sh_t[1] = 0;
  const Lane L = lane_info<R>();
  const int wave = threadIdx.x / kWave;
  const int gpb = (blockDim.x / kWave) * GPW;
  const int gslot = wave * GPW + (L.live ? L.grp : 0);
  double* Hs = reinterpret_cast<double*>(p2_smem);
  double* shM1 = Hs + R * R;
  double* gbuf = shM1 + R * R + gslot * PolarLds<R>::kPerGroup;
  double* region = gbuf;
  double* Cs = region;
  double* S = region + R * R;
  double* wv = gbuf + PolarLds<R>::kRegion;
  double* dl = wv + 2 * R;
  const int c = L.j;
  for (int i = 0;; ++i) {
    const int t = claim_tile(ntiles, tickets, i, sh_t);
    if (t < 0) break;
    const Tile tile = T[t];
    if (tile.k0 >= tile.k1) continue;
    const ProbDesc& D = P[tile.p];
    const XEnc X = D.X;
    const float* __restrict__ V = D.V[parity];
    const float* __restrict__ W = D.W;
    double* __restrict__ F = D.F;
    __syncthreads();
    load_shared_rxr<R>(Hs, D.H);
    for (int q = threadIdx.x; q < R * R; q += blockDim.x) shM1[q] = 0.0;
    __syncthreads();
    if (L.live) {
      for (int64_t pos = tile.k0 + gslot; pos < tile.k1; pos += gpb) {
        const int64_t k = subject_at(D, pos);
        const Subj s = X.subj(k);
        {
          double crow[R];
#pragma unroll
          for (int l = 0; l < R; ++l) crow[l] = 0.0;
          for (int i0 = 0; i0 < s.nrows; i0 += CH) {
            const int n = min(CH, s.nrows - i0);
            gather_rows<R>(X, s, i0, n, V, region, c);
            wave_sync();
            gram_accum<R>(region, region, n, c, crow);
            wave_sync();
          }
          if (c < R) {
#pragma unroll
            for (int l = 0; l < R; ++l) Cs[c * R + l] = crow[l];
            wv[c] = (double)glob(W)[k * R + c];
          }
        }
        wave_sync();
        double f[R], y[R];
        float* Ek = WARM ? D.E + k * (Geo<R>::NC * R) : nullptr;
        polar_rxr<R, WARM>(Cs, wv, Hs, S, dl, Ek, c, L.gbase, L.gmask, true, pp.tau_polar, pp.tol,
                     pp.stop2,
                     pp.max_sweeps, f, y);
        if (c < R) {
          P2_GLOBAL double* Fk = glob(F) + (size_t)k * R * R + (size_t)c * R;
#pragma unroll
          for (int q = 0; q < R; ++q) Fk[q] = f[q];
          add_m1<R>(shM1, y, wv[c], c);
        }
        wave_sync();
      }
    }
    __syncthreads();
    double* M1 = D.small + SL.M1;
    for (int q = threadIdx.x; q < R * R; q += blockDim.x) {
      const double v = shM1[q];
      if (v != 0.0) gadd(M1 + q, v);
    }
  }
}

// ---------------------------------------------------------------------------
// Non-negative least squares per row: the non-negative V and S_k of the
// paper's experiments (Sec. "Classical Algorithm for PARAFAC2" and Sec.
// "Setup", where the fast NNLS of Bro and De Jong is used).  For one row m of
// an MTTKRP and the R x R normal matrix N of its update, x = argmin over
// x >= 0 of the least-squares problem whose normal equations are N x = m, by
// the active-set method on the cross products N, m:
//   x = 0; w = m - N x
//   while the largest w_j off the passive set P exceeds tol: j joins P;
//     s = solution of N[P,P] s_P = m_P (0 off P);
//     while some s_j <= 0 on P: step x towards s until the first such x_j
//       reaches 0, drop the variables at 0 from P, solve again;
//     x = s; w = m - N x.
// One group of NC lanes per row, lane c owns x_c and column c of N (N is
// symmetric).  Reductions over the group (largest gradient, smallest step,
// largest |x|) go through LDS and take the first index on ties.  The passive
// block is solved by a Cholesky factorisation of N with the rows and columns
// off P replaced by those of the identity, column c per lane, factor columns
// broadcast through LDS.
// ---------------------------------------------------------------------------
template <int R>
struct NnlsLds {
  static constexpr int NC = Geo<R>::NC;
  // L (R x R, factor column k at k * R), v (R), xs (NC), pf (NC), red (NC)
  static constexpr int kPerGroup = R * R + R + 3 * NC;
};

// Group reductions over lanes 0..R-1 of one value per lane: largest value
// (first index on ties) or smallest value (first index on ties).
template <int R>
__device__ __forceinline__ void group_argmax(double* red, double v, int c, double& best, int& at) {
  if (c < R) red[c] = v;
  wave_sync();
  best = red[0];
  at = 0;
  for (int i = 1; i < R; ++i) {
    const double t = red[i];
    if (t > best) {
      best = t;
      at = i;
    }
  }
  wave_sync();
}

template <int R>
__device__ __forceinline__ void group_argmin(double* red, double v, int c, double& best, int& at) {
  if (c < R) red[c] = v;
  wave_sync();
  best = red[0];
  at = 0;
  for (int i = 1; i < R; ++i) {
    const double t = red[i];
    if (t < best) {
      best = t;
      at = i;
    }
  }
  wave_sync();
}

// s_c of the solution of N[P,P] s_P = m_P (s = 0 off P) for the group.
template <int R>
__device__ double nnls_solve(const double (&ncol)[R], double m, bool p, int c, double* L,
                             double* v, double* pf) {
  const bool real = c < R;
  if (real) pf[c] = p ? 1.0 : 0.0;
  wave_sync();
  double g[R];
#pragma unroll
  for (int i = 0; i < R; ++i) g[i] = (p && pf[i] != 0.0) ? ncol[i] : (i == c ? 1.0 : 0.0);
#pragma nounroll
  for (int k = 0; k < R; ++k) {
    if (c == k) {
      const double piv = g[k];
      const double rs = piv > 0.0 ? 1.0 / sqrt(piv) : 0.0;
#pragma unroll
      for (int i = 0; i < R; ++i) {
        g[i] *= rs;
        L[k * R + i] = g[i];
      }
    }
    wave_sync();
    if (real && c > k) {
      const double lck = L[k * R + c];
#pragma unroll
      for (int i = 0; i < R; ++i) g[i] = fma(-lck, L[k * R + i], g[i]);
    }
    wave_sync();
  }
  if (real) v[c] = p ? m : 0.0;
  wave_sync();
#pragma nounroll
  for (int k = 0; k < R; ++k) {  // L y = m_P
    if (c == k) {
      const double d = L[k * R + k];
      v[k] = d > 0.0 ? v[k] / d : 0.0;
    }
    wave_sync();
    if (real && c > k) v[c] = fma(-L[k * R + c], v[k], v[c]);
    wave_sync();
  }
#pragma nounroll
  for (int k = R - 1; k >= 0; --k) {  // L^T s = y
    if (c == k) {
      const double d = L[k * R + k];
      v[k] = d > 0.0 ? v[k] / d : 0.0;
    }
    wave_sync();
    if (real && c < k) v[c] = fma(-L[c * R + k], v[k], v[c]);
    wave_sync();
  }
  const double sc = (real && p) ? v[c] : 0.0;
  wave_sync();
  return sc;
}

// x_c of the NNLS solution for the group's row (m = m_c of lane c).  warm:
// lane c's variable was positive in the previous iteration's row; if solving
// on that support gives a positive solution, the method starts from it (a
// feasible point with x > 0 exactly on P, from which the steps above apply
// unchanged), else from x = 0.  N is positive definite, so the solution is
// unique and does not depend on the starting point.
template <int R>
__device__ double nnls_group(const double (&ncol)[R], double m, int c, double* buf, bool warm) {
  constexpr int NC = Geo<R>::NC;
  constexpr double eps = 2.220446049250313e-16;
  const double inf = __builtin_huge_val();
  double* L = buf;
  double* v = L + R * R;
  double* xs = v + R;
  double* pf = xs + NC;
  double* red = pf + NC;
  const bool real = c < R;
  double x = 0.0;
  bool p = false, blocked = false;
  double scale, tmp;
  int at;
  group_argmax<R>(red, real ? fabs(m) : 0.0, c, scale, at);
  scale = fmax(scale, 2.2250738585072014e-308);
  double tol = 10.0 * R * eps * scale;
  double w = m;
  double any_warm;
  group_argmax<R>(red, (real && warm) ? 1.0 : 0.0, c, any_warm, at);
  if (any_warm > 0.0) {
    const bool pw = real && warm;
    const double s = nnls_solve<R>(ncol, m, pw, c, L, v, pf);
    double smin;
    group_argmin<R>(red, pw ? s : __builtin_huge_val(), c, smin, at);
    if (smin > 0.0) {
      p = pw;
      x = s;
      if (real) xs[c] = x;
      wave_sync();
      double nx = 0.0;
#pragma unroll
      for (int i = 0; i < R; ++i) nx = fma(ncol[i], xs[i], nx);
      wave_sync();
      w = m - nx;
      group_argmax<R>(red, real ? fabs(nx) : 0.0, c, tmp, at);
      scale = fmax(scale, tmp);
      tol = 10.0 * R * eps * scale;
    }
  }
  for (int outer = 0; outer < 3 * R; ++outer) {
    double best;
    int j;
    group_argmax<R>(red, (real && !p && !blocked) ? w : -inf, c, best, j);
    if (!(best > tol)) break;
    if (c == j) p = true;
    double s = nnls_solve<R>(ncol, m, p, c, L, v, pf);
    for (int inner = 0; inner <= R; ++inner) {
      const bool bad = p && s <= 0.0;
      const double d = x - s;
      double alpha;
      int q;
      group_argmin<R>(red, bad ? (d > 0.0 ? x / d : 0.0) : inf, c, alpha, q);
      if (alpha == inf) break;
      x = fma(alpha, s - x, x);
      if (c == q) x = 0.0;  // the variable that limits the step reaches zero
      double xm;
      group_argmax<R>(red, real ? fabs(x) : 0.0, c, xm, at);
      if (p && x <= 10.0 * eps * fmax(xm, 1e-300)) p = false;
      if (!p) x = 0.0;
      if (alpha > 0.0)
        blocked = false;
      else if (c == j && !p)
        blocked = true;  // rounding: w_j > tol but its solve was <= 0
      s = nnls_solve<R>(ncol, m, p, c, L, v, pf);
    }
    x = s;
    if (real) xs[c] = x;
    wave_sync();
    double nx = 0.0;
#pragma unroll
    for (int i = 0; i < R; ++i) nx = fma(ncol[i], xs[i], nx);
    wave_sync();
    w = m - nx;
    group_argmax<R>(red, real ? fabs(nx) : 0.0, c, tmp, at);
    scale = fmax(scale, tmp);
    tol = 10.0 * R * eps * scale;
  }
  return x;
}

// ---------------------------------------------------------------------------
// k_gamma: mode-3 MTTKRP row per subject (equation (mttkrp3_row_wise)) from
// A_k = X_k V_t and A'_k = X_k V_{t+1}: (Y_k V_{t+1}) = F_k A_k^T A'_k,
// m3(c) = H(:, c) . (Y_k V_{t+1})(:, c); the W row update
// w = m3 ((V^T V) * (H^T H))^+ (Algorithm "CP-ALS"); the loss terms; and, if
// do_next, the next iteration's Procrustes step and mode-1 partial from
// C'_k = A'_k^T A'_k.  With NN (a launch with problems under the
// non-negativity constraint) the W row of such problems is the NNLS solution
// of N3 w = m3 instead, formed in the group before the Procrustes step, so
// that the next step stays fused into this pass.
// ---------------------------------------------------------------------------
template <int R, bool WARM, bool NN>
__global__ void __launch_bounds__(256, NN ? PolarLds<R>::kMinWavesNN : PolarLds<R>::kMinWaves) k_gamma(const ProbDesc* __restrict__ P,
                                                const Tile* __restrict__ T, int ntiles,
                                                int* tickets, int parity, int do_next,
                                                PolarParams pp) {
  constexpr int GPW = Geo<R>::GPW;
  constexpr int CH = PolarLds<R>::CH;
  constexpr SmallLayout SL = small_layout(R);
  __shared__ int sh_t[2];
  if (threadIdx.x == 0) sh_t[1] = 0;
  const Lane L = lane_info<R>();
  const int wave = threadIdx.x / kWave;
  const int gpb = (blockDim.x / kWave) * GPW;
  const int gslot = wave * GPW + (L.live ? L.grp : 0);
  double* Hs = reinterpret_cast<double*>(p2_smem);
  double* N3s = Hs + R * R;
  double* N3ps = N3s + R * R;
  double* shM1 = N3ps + R * R;
  double* shFit = shM1 + R * R;
  double* gbuf = shFit + 2 + gslot * PolarLds<R>::kPerGroup;
  double* region = gbuf;
  float* A0 = reinterpret_cast<float*>(region);
  float* A1 = A0 + CH * R;
  double* SF = region;          // F column-major (SF[col * R + row]), later C'
  double* SP = region + R * R;  // P rows, later the Jacobi scratch
  double* wv = gbuf + PolarLds<R>::kRegion;
  double* mv = wv + R;
  double* dl = mv + R;
  const int c = L.j;
  const bool real = c < R;
  const int cc = real ? c : 0;
  for (int i = 0;; ++i) {
    const int t = claim_tile(ntiles, tickets, i, sh_t);
    if (t < 0) break;
    const Tile tile = T[t];
    if (tile.k0 >= tile.k1) continue;
    const ProbDesc& D = P[tile.p];
    const XEnc X = D.X;
    const float* __restrict__ V0 = D.V[parity];
    const float* __restrict__ V1 = D.V[parity ^ 1];
    float* __restrict__ W = D.W;
    double* __restrict__ F = D.F;
    float* __restrict__ M3 = D.M3;
    __syncthreads();
    load_shared_rxr<R>(Hs, D.H);
    load_shared_rxr<R>(N3s, D.small + SL.N3);
    load_shared_rxr<R>(N3ps, D.small + SL.N3p);
    for (int q = threadIdx.x; q < R * R + 2; q += blockDim.x) shM1[q] = 0.0;
    __syncthreads();
    double fa = 0.0, fb = 0.0;
    if (L.live) {
      for (int64_t pos = tile.k0 + gslot; pos < tile.k1; pos += gpb) {
        const int64_t k = subject_at(D, pos);
        const Subj s = X.subj(k);
        double crow[R];
        {
          double prow[R];
#pragma unroll
          for (int l = 0; l < R; ++l) prow[l] = crow[l] = 0.0;
          for (int i0 = 0; i0 < s.nrows; i0 += CH) {
            const int n = min(CH, s.nrows - i0);
            gather_rows2<R, PolarLds<R>::kRowsPerLane>(X, s, i0, n, V0, V1, A0, A1, c);
            wave_sync();
            gram_accum2<R>(A0, A1, n, c, prow, crow);  // rows c of P = A^T A', C' = A'^T A'
            wave_sync();
          }
          if (real) {
            const P2_GLOBAL double* Fk = glob(F) + (size_t)k * R * R + (size_t)c * R;
#pragma unroll
            for (int q = 0; q < R; ++q) SF[c * R + q] = Fk[q];
#pragma unroll
            for (int l = 0; l < R; ++l) SP[c * R + l] = prow[l];
          }
        }
        wave_sync();
        double m3 = 0.0;
        {
          double yv[R];
#pragma unroll
          for (int q = 0; q < R; ++q) yv[q] = 0.0;
#pragma nounroll
          for (int l = 0; l < R; ++l) {
            const double plc = SP[l * R + cc];
#pragma unroll
            for (int q = 0; q < R; ++q) yv[q] = fma(SF[l * R + q], plc, yv[q]);
          }
#pragma unroll
          for (int q = 0; q < R; ++q) m3 = fma(Hs[q * R + cc], yv[q], m3);
        }
        if (real) mv[c] = m3;
        wave_sync();
        double wn = 0.0;
        if (NN && D.nonneg) {
          // NNLS from the float64 row, started from the support of W_t's row;
          // the region (F and P above) is free again
          double ncol[R];
#pragma unroll
          for (int i = 0; i < R; ++i) ncol[i] = N3s[i * R + cc];
          const bool warm = real && glob(W)[k * R + c] > 0.f;
          wn = nnls_group<R>(ncol, m3, c, region, warm);
        } else {
#pragma unroll
          for (int l = 0; l < R; ++l) wn = fma(mv[l], N3ps[l * R + cc], wn);
        }
        if (real) {
          glob(W)[k * R + c] = (float)wn;
          glob(M3)[k * R + c] = (float)m3;
          wv[c] = (double)(float)wn;
        }
        wave_sync();
        if (real) {
          const double wf = wv[c];
          double tt = 0.0;
#pragma unroll
          for (int l = 0; l < R; ++l) tt = fma(N3s[c * R + l], wv[l], tt);
          fa = fma(wf, m3, fa);
          fb = fma(wf, tt, fb);
        }
        if (do_next) {
          if (real) {
#pragma unroll
            for (int l = 0; l < R; ++l) SF[c * R + l] = crow[l];
          }
          wave_sync();
          double f[R], y[R];
          float* Ek = WARM ? D.E + k * (Geo<R>::NC * R) : nullptr;
          // at ranks up to 16 the polar step runs at raised wave priority: a
          // wave in its chain of dependent FP64 steps issues ahead of waves
          // waiting on gathers (measured: the pass 1.6 % faster at R = 10,
          // unchanged at R = 12, 16 and 20, and 2 % slower at R = 40, which
          // runs one wave per SIMD)
          if constexpr (R <= 16) __builtin_amdgcn_s_setprio(1);
          polar_rxr<R, WARM>(SF, wv, Hs, SP, dl, Ek, c, L.gbase, L.gmask, true, pp.tau_polar, pp.tol,
                       pp.stop2,
                       pp.max_sweeps, f, y);
          if constexpr (R <= 16) __builtin_amdgcn_s_setprio(0);
          if (real) {
            P2_GLOBAL double* Fk = glob(F) + (size_t)k * R * R + (size_t)c * R;
#pragma unroll
            for (int q = 0; q < R; ++q) Fk[q] = f[q];
            add_m1<R>(shM1, y, wv[c], c);
          }
        }
        wave_sync();
      }
    }
    if (L.live && real) {
      atomicAdd(&shFit[0], fa);
      atomicAdd(&shFit[1], fb);
    }
    __syncthreads();
    if (do_next) {
      double* M1 = D.small + SL.M1;
      for (int q = threadIdx.x; q < R * R; q += blockDim.x) {
        const double v = shM1[q];
        if (v != 0.0) gadd(M1 + q, v);
      }
    }
    if (threadIdx.x == 0) {
      gadd(D.small + SL.fitacc + 0, shFit[0]);
      gadd(D.small + SL.fitacc + 1, shFit[1]);
    }
  }
}

// ---------------------------------------------------------------------------
// k_mode2: M2 += X_k^T (A_k E_k),  E_k = F_k^T H diag(w_k)  (equation
// (mttkrp2_3): for every nonzero column j of X_k, row j of Y_k^T H diag(w_k)).
// This kernel serves R > 16 (k_mode2_dpp below serves R <= 16).  One lane per
// row: it gathers A(i, :) into registers, forms D(i, :) = A(i, :) E_k with
// E_k staged in the group's LDS, and adds x_ij D(i, :) into M2(j, :):
//  * hot columns (ids < hot, the most frequent after relabelling) into the
//    block's FP64 partial sums in LDS; each tile writes them, without
//    atomics, to its own slot among its problem's partial sums, and
//    k_mode2_reduce adds the slots up per problem;
//  * cold columns through a per-wave LDS queue, added to M2 when the queue is
//    full and at the end of a tile, with the lanes of one atomic instruction
//    on consecutive (row, component) entries.  Device-wide float atomics are
//    carried out past the L2, one memory transaction per 32-byte sector an
//    instruction touches, and they retire in order with the wave's loads, so
//    an atomic issued per row would also hold up the next wait for a load.
// ---------------------------------------------------------------------------
constexpr int kMode2Threads = 1024;

#ifndef P2_M2D_QUEUE
#define P2_M2D_QUEUE 16
#endif
#ifndef P2_M2D_CHUNK
#define P2_M2D_CHUNK 4
#endif
#ifndef P2_M2_QUEUE
#define P2_M2_QUEUE 16
#endif
template <int R>
struct Mode2Lds {
  // E_k in FP64, rows of stride NC (R rounded up to even, so that rows are
  // 16-byte aligned), counted in floats: E_k = F^T H' diag(w') carries the
  // 1/sigma_min scale of ill-conditioned subjects, so D = A E_k cancels and
  // is formed in FP64
  static constexpr int kPerGroup = 2 * R * Geo<R>::NC;
  // largest workgroup; ranks above 16 use at most 512 threads so that a
  // lane may hold 256 VGPRs (the FP64 D row alone takes 2R of them)
  static constexpr int kMaxThreads = R <= 16 ? kMode2Threads : kMode2Threads / 2;
  // rows a lane gathers per step (register budget: T x LDV floats)
  static constexpr int kRowsPerStep = R <= 20 ? 2 : 1;
  // floats before the group buffers: the hot partial sums, in FP64 (LDS
  // float atomics are carried out one lane at a time, about 3 cycles per
  // lane, while FP64 ones take about 24 cycles per wave instruction), rounded
  // up so that E rows are 16-byte aligned
  static constexpr int hot_floats(int hot) { return (2 * hot * R + 3) & ~3; }
  // per wave after all group buffers: a count, then up to kQueue staged cold
  // updates (column ids, then R-float rows), added to M2 when the queue is
  // full and at the end of a tile
  static constexpr int kQueue = P2_M2_QUEUE;
  static constexpr int kQueueFloats = (4 + kQueue * (R + 1) + 3) & ~3;
};

// Adds the n staged rows of a wave's cold queue to M2 with the active lanes
// on consecutive (row, component) entries, so that the lanes of one atomic
// instruction touch a few rows of M2 (one memory transaction per 32-byte
// sector) rather than one row each.
template <int R>
__device__ __forceinline__ void cold_flush(float* M2, const int* qj, const float* qv, int n) {
  constexpr int LDV = Geo<R>::LDV;
  const uint64_t am = __ballot(true);
  const int nact = __popcll(am);
  const int me = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(am >> 32),
                                                __builtin_amdgcn_mbcnt_lo((uint32_t)am, 0u));
  for (int v = me; v < n * R; v += nact) {
    const int e = v / R;
    gadd(M2 + (size_t)qj[e] * LDV + (v - e * R), qv[v]);
  }
  wave_sync();
}

// Appends the active lanes' cold updates x d (those with `cold`) to the wave's
// queue, in passes of what the queue has room for; a full queue is added to
// M2 first.  The count lives in LDS (qcount[0]), where every group of the
// wave sees it on whichever path it is.  d may be padded past R (odd ranks
// keep NC entries); only its first R are staged.
template <int R, int QN, class DT, int N>
__device__ __forceinline__ void cold_stage(bool cold, int j, float x, const DT (&d)[N], float* M2,
                                           int* qcount, int* qj, float* qv) {
  static_assert(N >= R, "the D row holds at least R entries");
  const uint64_t cm = __ballot(cold);
  if (cm == 0ull) return;
  const int ncold = __popcll(cm);
  const int rank = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(cm >> 32),
                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)cm, 0u));
  int base = qcount[0];
  for (int done = 0; done < ncold;) {  // the same on every active lane
    if (base == QN) {
      // the flush's coalesced updates go out ahead of the SIMD's other waves
      __builtin_amdgcn_s_setprio(2);
      cold_flush<R>(M2, qj, qv, QN);
      __builtin_amdgcn_s_setprio(0);
      base = 0;
    }
    const int take = min(QN - base, ncold - done);
    if (cold && rank >= done && rank < done + take) {
      const int slot = base + rank - done;
      qj[slot] = j;
#pragma unroll
      for (int q = 0; q < R; ++q) qv[slot * R + q] = x * (float)d[q];
    }
    base += take;
    done += take;
  }
  if (cold && rank == 0) qcount[0] = base;
  wave_sync();
}

template <int R>
__global__ void __launch_bounds__(Mode2Lds<R>::kMaxThreads) k_mode2(const ProbDesc* __restrict__ P,
                                                          const Tile* __restrict__ T, int ntiles,
                                                          int* tickets, int parity,
                                                          int max_hot) {
  constexpr int NC = Geo<R>::NC;
  constexpr int GPW = Geo<R>::GPW;
  constexpr int LDV = Geo<R>::LDV;
  __shared__ int sh_t[2];
  if (threadIdx.x == 0) sh_t[1] = 0;
  const Lane L = lane_info<R>();
  const int wave = threadIdx.x / kWave;
  const int gpb = (blockDim.x / kWave) * GPW;
  const int gslot = wave * GPW + (L.live ? L.grp : 0);
  double* shM2 = reinterpret_cast<double*>(p2_smem);  // up to max_hot x R
  float* shM2f = reinterpret_cast<float*>(p2_smem);
  double* Es = reinterpret_cast<double*>(shM2f + Mode2Lds<R>::hot_floats(max_hot) +
                                         gslot * Mode2Lds<R>::kPerGroup);
  constexpr int QN = Mode2Lds<R>::kQueue;
  int* qcount = reinterpret_cast<int*>(shM2f + Mode2Lds<R>::hot_floats(max_hot) +
                                       gpb * Mode2Lds<R>::kPerGroup +
                                       wave * Mode2Lds<R>::kQueueFloats);
  int* qj = qcount + 4;
  float* qv = reinterpret_cast<float*>(qj + QN);
  if (L.lane == 0) qcount[0] = 0;
  const int c = L.j;
  const bool real = c < R;
  const int cc = real ? c : 0;
  for (int i = 0;; ++i) {
    const int t = claim_tile(ntiles, tickets, i, sh_t);
    if (t < 0) break;
    const Tile tile = T[t];
    if (tile.k0 >= tile.k1) continue;
    const ProbDesc& D = P[tile.p];
    const XEnc X = D.X;
    const float* __restrict__ V = D.V[parity];
    const float* __restrict__ W = D.W;
    const double* __restrict__ F = D.F;
    float* __restrict__ M2 = D.M2;
    const int hot = min(D.hot, max_hot);
    __syncthreads();
    for (int q = threadIdx.x; q < hot * R; q += blockDim.x) shM2[q] = 0.0;
    __syncthreads();
    if (L.live) {
      // H'(:, c) held as FP32: with E = F^T H' diag(w') formed in FP64, a
      // rounding dH of H' moves D = A E by Q_k dH diag(w'), and Q_k = A F^T
      // has orthonormal columns, so that change is not scaled by the
      // condition number of the subject as a rounding of E would be
      float hc[R];
#pragma unroll
      for (int q = 0; q < R; ++q) hc[q] = (float)glob(D.H)[q * R + cc];
      for (int64_t pos = tile.k0 + gslot; pos < tile.k1; pos += gpb) {
        const int64_t k = subject_at(D, pos);
        const Subj s = X.subj(k);
        {
          // F_k (R x R doubles, F(q, p) at p * R + q) staged in the group's E
          // buffer with coalesced loads, then E(:, c) = w(c) F^T H(:, c),
          // stored row-major E(p, c) = Es[p * NC + c]; the padding column of
          // an odd rank (c = R) holds zeros
          const P2_GLOBAL double* Fk = glob(F) + (size_t)k * R * R;
          for (int f = c; f < R * R; f += NC) Es[f] = Fk[f];
          const double wc = real ? (double)glob(W)[k * R + cc] : 0.0;
#pragma unroll
          for (int q = 0; q < R; ++q) settle(hc[q]);  // widened here, per subject
          wave_sync();
          // two rows of E at a time, each as two independent FMA chains; the
          // settle after each pair keeps the scheduler from holding all of
          // F_k in registers across the barrier below
          double e[R];
#pragma unroll
          for (int p0 = 0; p0 < R; p0 += 2) {
#pragma unroll
            for (int p = p0; p < p0 + 2 && p < R; ++p) {
              double t0 = 0.0, t1 = 0.0;
#pragma unroll
              for (int q = 0; q < R; ++q) {
                if (q & 1)
                  t1 = fma(Es[p * R + q], (double)hc[q], t1);
                else
                  t0 = fma(Es[p * R + q], (double)hc[q], t0);
              }
              e[p] = (t0 + t1) * wc;
            }
#pragma unroll
            for (int p = p0; p < p0 + 2 && p < R; ++p) settle(e[p]);
          }
          wave_sync();
#pragma unroll
          for (int p = 0; p < R; ++p) Es[p * NC + c] = e[p];
        }
        wave_sync();
        // T rows per lane and step: every row bound, first nonzero and V row
        // of the step is requested before any of them is used, so a lane has
        // T independent load chains in flight instead of one
        constexpr int T = Mode2Lds<R>::kRowsPerStep;
        const P2_GLOBAL uint16_t* __restrict__ rst = glob(X.rstart) + s.r0;
        const P2_GLOBAL uint16_t* __restrict__ cl = glob(X.col) + s.z0;
        const P2_GLOBAL float* __restrict__ vl = glob(X.val) + s.z0;
#pragma nounroll
        for (int ib = 0; ib < s.nrows; ib += T * NC) {
          // the step's loads at raised wave priority, its products and
          // updates at the normal one: a wave whose loads are ready issues the
          // next ones ahead of the SIMD's waves that are computing
          __builtin_amdgcn_s_setprio(1);
          int zs[T], ze[T];
#pragma unroll
          for (int t = 0; t < T; ++t) {
            const int ii = ib + c + t * NC;
            const bool ok = ii < s.nrows;
            zs[t] = ok ? (int)rst[ii] : 0;
            ze[t] = ok ? ((ii + 1 < s.nrows) ? (int)rst[ii + 1] : s.nnz) : 0;
          }
          int j0[T];
          float x0[T];
#pragma unroll
          for (int t = 0; t < T; ++t) {
            const bool any = zs[t] < ze[t];
            j0[t] = any ? (int)cl[zs[t]] : 0;
            x0[t] = any ? vl[zs[t]] : 0.f;
          }
          float a[T][LDV];
#pragma unroll
          for (int t = 0; t < T; ++t) {
            const float* vr = V + (size_t)j0[t] * LDV;
#pragma unroll
            for (int q = 0; q < LDV / 4; ++q) {
              const p2_f4 v4 = ldg4(vr + 4 * q);
              a[t][4 * q + 0] = x0[t] * v4.x;
              a[t][4 * q + 1] = x0[t] * v4.y;
              a[t][4 * q + 2] = x0[t] * v4.z;
              a[t][4 * q + 3] = x0[t] * v4.w;
            }
          }
#pragma unroll
          for (int t = 0; t < T; ++t) {
            for (int z = zs[t] + 1; z < ze[t]; ++z) {
              const float x = vl[z];
              const float* vr = V + (size_t)cl[z] * LDV;
#pragma unroll
              for (int q = 0; q < LDV / 4; ++q) {
                const p2_f4 v4 = ldg4(vr + 4 * q);
                a[t][4 * q + 0] = fmaf(x, v4.x, a[t][4 * q + 0]);
                a[t][4 * q + 1] = fmaf(x, v4.y, a[t][4 * q + 1]);
                a[t][4 * q + 2] = fmaf(x, v4.z, a[t][4 * q + 2]);
                a[t][4 * q + 3] = fmaf(x, v4.w, a[t][4 * q + 3]);
              }
            }
          }
          __builtin_amdgcn_s_setprio(0);
#pragma unroll
          for (int t = 0; t < T; ++t) {
            const int nz = ze[t] - zs[t];  // 0 for rows past the subject
            // D(i, :) = A(i, :) E in FP64, reading E rows as 16-byte LDS vectors
            // (NC columns: the padding of E beyond them is never read)
            double d[NC];
#pragma unroll
            for (int q = 0; q < NC; ++q) d[q] = 0.0;
            if (nz > 0) {
#pragma unroll
              for (int p = 0; p < R; ++p) {
                const double ap = (double)a[t][p];
                const double2* e2 = reinterpret_cast<const double2*>(Es + p * NC);
#pragma unroll
                for (int q = 0; q < NC / 2; ++q) {
                  const double2 e = e2[q];
                  d[2 * q + 0] = fma(ap, e.x, d[2 * q + 0]);
                  d[2 * q + 1] = fma(ap, e.y, d[2 * q + 1]);
                }
              }
            }
            // one nonzero of the row per lane and round; the rounds run while
            // any active lane of the wave has one left
            for (int r = 0; __ballot(r < nz) != 0ull; ++r) {
              const bool act = r < nz;
              int j = 0;
              float x = 0.f;
              if (act) {
                j = (r == 0) ? j0[t] : (int)cl[zs[t] + r];
                x = (r == 0) ? x0[t] : vl[zs[t] + r];
              }
              if (act && j < hot) {
                double* dst = shM2 + j * R;
#pragma unroll
                for (int q = 0; q < R; ++q) atomicAdd(dst + q, (double)x * d[q]);
              }
              // cold columns: staged in the wave's queue (count in LDS, so
              // that every group of the wave sees it on whichever path it is)
              cold_stage<R, QN>(act && j >= hot, j, x, d, M2, qcount, qj, qv);
            }
          }
        }
        wave_sync();
      }
    }
    cold_flush<R>(M2, qj, qv, qcount[0]);
    if (L.lane == 0) qcount[0] = 0;
    __syncthreads();
    P2_GLOBAL float* mine = glob(D.part) + (int64_t)tile.slot * hot * R;
    for (int q = threadIdx.x; q < hot * R; q += blockDim.x) mine[q] = (float)shM2[q];
  }
}

// ---------------------------------------------------------------------------
// k_mode2 for R <= 16.  A subject's group is one 16-lane DPP row.
//  * E_k in registers: lane p (p < R) forms row p of E_k = F_k^T H diag(w_k)
//    from its contiguous column of F_k, and every lane forms D(i, :) =
//    A(i, :) E_k with one v_fmac_f64 per product whose first source is read
//    from lane p of the row (row_newbcast:p); no LDS traffic per row.
//  * One nonzero per lane and step: lane c takes nonzero zb + c of the
//    subject, gathers the whole row of that nonzero and adds x_ij D(i, :) for
//    its own nonzero, so a step makes each update once (a lane per row would
//    need as many rounds as the longest row of the wave has nonzeros).
//  * Hot columns add into FP64 partial sums in LDS: LDS float atomics are
//    carried out one lane at a time (about 3 cycles per lane), FP64 ones take
//    about 24 cycles per wave instruction.
//  * Cold columns are staged in a per-wave LDS queue and added to M2 only when
//    the queue is full and at the end of a tile, with the lanes on
//    consecutive entries.  A device-wide atomic is acknowledged from memory,
//    and a wave's vector memory counter retires in order, so an atomic issued
//    in a step would hold up the wait for every later load of the wave.
// ---------------------------------------------------------------------------
template <int R>
struct Mode2Dpp {
  static constexpr int kLanes = 16;               // one DPP row per subject
  static constexpr int kGroups = kWave / kLanes;  // subjects per wave
  // steps whose nonzero indices a lane loads at once (one nonzero per step)
  static constexpr int kChunk = P2_M2D_CHUNK;
  // H' as floats after the hot partial sums
  static constexpr int kHFloats = (R * R + 3) & ~3;
  // per wave after H': a count, then up to kQueue staged cold updates (column
  // ids, then R-float rows); they are added to M2 only when the queue is full
  // and at the end of a tile
  static constexpr int kQueue = P2_M2D_QUEUE;
  static constexpr int kQueueFloats = (4 + kQueue * (R + 1) + 3) & ~3;
};
template <int R> constexpr bool kMode2UsesDpp = R <= 16;

// d += a * E(P, q), E(P, q) held by lane P of this lane's 16-lane row in e.
// A DPP read needs five wait states after EXEC was written and two after its
// source VGPR was written by the VALU; the caller issues s_nop 4 (dpp_guard)
// before the first product of each row and after forming e.
template <int P>
__device__ __forceinline__ void fmac_bcast(double& d, double e, double a) {
  asm volatile("v_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
               : "+v"(d)
               : "v"(e), "v"(a), "n"(P));
}
__device__ __forceinline__ void dpp_guard() { asm volatile("s_nop 4" ::: "memory"); }

// d(q) += sum_p a(p) E(p, q), a widened per p
template <int R, int P, int N>
__device__ __forceinline__ void dpp_row_products(double (&d)[R], const double (&e)[R],
                                                 const float (&a)[N]) {
  const double ap = (double)a[P];
#pragma unroll
  for (int q = 0; q < R; ++q) fmac_bcast<P>(d[q], e[q], ap);
}
template <int R, int N, int... P>
__device__ __forceinline__ void dpp_products(double (&d)[R], const double (&e)[R],
                                             const float (&a)[N],
                                             std::integer_sequence<int, P...>) {
  (dpp_row_products<R, P, N>(d, e, a), ...);
}

template <int R>
__global__ void __launch_bounds__(kMode2Threads) k_mode2_dpp(const ProbDesc* __restrict__ P,
                                                            const Tile* __restrict__ T,
                                                            int ntiles, int* tickets, int parity,
                                                            int max_hot) {
  using MD = Mode2Dpp<R>;
  constexpr int G = MD::kLanes;
  constexpr int LDV = Geo<R>::LDV;
  __shared__ int sh_t[2];
  if (threadIdx.x == 0) sh_t[1] = 0;
  const int c = threadIdx.x & (G - 1);  // lane in the group (and DPP row)
  const int wave = threadIdx.x / kWave;
  const int gpb = (blockDim.x / kWave) * MD::kGroups;
  const int gslot = wave * MD::kGroups + (threadIdx.x & (kWave - 1)) / G;
  double* shM2 = reinterpret_cast<double*>(p2_smem);  // up to max_hot x R
  float* shH = reinterpret_cast<float*>(p2_smem) + Mode2Lds<R>::hot_floats(max_hot);
  constexpr int QN = MD::kQueue;
  int* qcount = reinterpret_cast<int*>(shH + MD::kHFloats + wave * MD::kQueueFloats);
  int* qj = qcount + 4;
  float* qv = reinterpret_cast<float*>(qj + QN);
  if ((threadIdx.x & (kWave - 1)) == 0) qcount[0] = 0;
  const int pc = c < R ? c : 0;  // the row of E_k this lane forms
  for (int i = 0;; ++i) {
    const int t = claim_tile(ntiles, tickets, i, sh_t);
    if (t < 0) break;
    const Tile tile = T[t];
    if (tile.k0 >= tile.k1) continue;
    const ProbDesc& D = P[tile.p];
    const XEnc X = D.X;
    const float* __restrict__ V = D.V[parity];
    const float* __restrict__ W = D.W;
    const double* __restrict__ F = D.F;
    float* __restrict__ M2 = D.M2;
    const int hot = min(D.hot, max_hot);
    __syncthreads();
    for (int q = threadIdx.x; q < hot * R; q += blockDim.x) shM2[q] = 0.0;
    // H' in FP32 (as in k_mode2: Q_k = A F^T has orthonormal columns, so a
    // rounding of H' moves D by Q_k dH diag(w'), unscaled by the subject's
    // condition number)
    for (int q = threadIdx.x; q < R * R; q += blockDim.x) shH[q] = (float)glob(D.H)[q];
    __syncthreads();
    for (int64_t pos = tile.k0 + gslot; pos < tile.k1; pos += gpb) {
      const int64_t k = subject_at(D, pos);
      const Subj s = X.subj(k);
      // E(p, q) = w(q) sum_r F(r, p) H(r, q) for p = pc: F(:, p) is contiguous
      // (F(r, p) at p * R + r), so the group loads F_k coalesced
      double e[R];
      {
        // every load of the subject is issued before the first is used (the
        // scheduler would otherwise interleave them with the products and
        // wait for each in turn)
        const P2_GLOBAL double* Fp = glob(F) + (size_t)k * R * R + pc * R;
        double f[R];
        float wq[R];
#pragma unroll
        for (int r = 0; r < R; ++r) f[r] = Fp[r];
#pragma unroll
        for (int q = 0; q < R; ++q) wq[q] = glob(W)[k * R + q];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < R; ++q) {
          double acc = 0.0;
#pragma unroll
          for (int r = 0; r < R; ++r) acc = fma(f[r], (double)shH[r * R + q], acc);
          e[q] = acc * (double)wq[q];
        }
      }
#pragma unroll
      for (int q = 0; q < R; ++q) settle(e[q]);
      dpp_guard();
      // one nonzero per lane and step: lane c takes nonzero zb + c, gathers
      // the whole row of that nonzero (its own term first) and adds x_ij D(i, :)
      // for its nonzero only, so a step issues the R atomics of each of its 16
      // nonzeros once (a lane per row needs as many rounds as the longest row
      // of the wave has nonzeros)
      const P2_GLOBAL uint16_t* __restrict__ rst = glob(X.rstart) + s.r0;
      const P2_GLOBAL uint16_t* __restrict__ nzr = glob(X.nzrow) + s.z0;
      const P2_GLOBAL uint16_t* __restrict__ cl = glob(X.col) + s.z0;
      const P2_GLOBAL float* __restrict__ vl = glob(X.val) + s.z0;
      // nonzeros in chunks of kChunk per lane: the rows, columns and values of
      // a chunk are requested together (coalesced over the group) before the
      // chunk's first step, so a step waits only for its V rows and row bounds
      constexpr int NB = MD::kChunk;
#pragma nounroll
      for (int zc = 0; zc < s.nnz; zc += G * NB) {
        // loads at raised wave priority, products and updates at the normal
        // one (as in k_mode2)
        __builtin_amdgcn_s_setprio(1);
        uint32_t rjc[NB];  // row << 16 | column
        float xc[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const int zb = zc + c + b * G;
          const int zz = zb < s.nnz ? zb : 0;
          rjc[b] = ((uint32_t)nzr[zz] << 16) | (uint32_t)cl[zz];
          xc[b] = vl[zz];
        }
        // the chunk's steps in one loop body: each step takes entry 0 and
        // shifts the rest down (register arrays are not indexed at run time)
#pragma nounroll
        for (int b = 0; b < NB; ++b) {
        const int zb = zc + b * G;
        if (zb >= s.nnz) break;  // uniform over the group
        const int z = zb + c;
        const bool ok = z < s.nnz;
        const int ir = (int)(rjc[0] >> 16);
        const int j = (int)(rjc[0] & 0xffffu);
        const float x = ok ? xc[0] : 0.f;
#pragma unroll
        for (int u = 0; u + 1 < NB; ++u) {
          rjc[u] = rjc[u + 1];
          xc[u] = xc[u + 1];
        }
        // V(j, :) and the row's bounds, in flight together
        __builtin_amdgcn_s_setprio(1);
        p2_f4 v4[LDV / 4];
        const float* vr = V + (size_t)j * LDV;
#pragma unroll
        for (int q = 0; q < LDV / 4; ++q) v4[q] = ldg4(vr + 4 * q);
        const int rs0 = rst[ir];
        const int re0 = rst[ir + 1 < s.nrows ? ir + 1 : ir];
        float a[LDV];
#pragma unroll
        for (int q = 0; q < LDV / 4; ++q) {
          a[4 * q + 0] = x * v4[q].x;
          a[4 * q + 1] = x * v4[q].y;
          a[4 * q + 2] = x * v4[q].z;
          a[4 * q + 3] = x * v4[q].w;
        }
        const int rs = ok ? rs0 : 0;
        const int re = ok ? ((ir + 1 < s.nrows) ? re0 : s.nnz) : 0;
        for (int y = rs; y < re; ++y) {
          if (y == z) continue;
          const float xo = vl[y];
          const float* vr = V + (size_t)cl[y] * LDV;
#pragma unroll
          for (int q = 0; q < LDV / 4; ++q) {
            const p2_f4 v4 = ldg4(vr + 4 * q);
            a[4 * q + 0] = fmaf(xo, v4.x, a[4 * q + 0]);
            a[4 * q + 1] = fmaf(xo, v4.y, a[4 * q + 1]);
            a[4 * q + 2] = fmaf(xo, v4.z, a[4 * q + 2]);
            a[4 * q + 3] = fmaf(xo, v4.w, a[4 * q + 3]);
          }
        }
        // D(i, :) = A(i, :) E_k for every lane of the group (lanes past the
        // subject have A = 0)
        __builtin_amdgcn_s_setprio(0);
        double d[R];
#pragma unroll
        for (int q = 0; q < R; ++q) d[q] = 0.0;
        dpp_guard();
        dpp_products<R>(d, e, a, std::make_integer_sequence<int, R>{});
        if (ok && j < hot) {
          double* dst = shM2 + j * R;
#pragma unroll
          for (int q = 0; q < R; ++q) atomicAdd(dst + q, (double)x * d[q]);
        }
        // cold columns: staged in the wave's queue (the count is kept in LDS,
        // where every group of the wave sees it whichever path it is on)
        cold_stage<R, QN>(ok && j >= hot, j, x, d, M2, qcount, qj, qv);
        }
      }
    }
    cold_flush<R>(M2, qj, qv, qcount[0]);
    if ((threadIdx.x & (kWave - 1)) == 0) qcount[0] = 0;
    __syncthreads();
    P2_GLOBAL float* mine = glob(D.part) + (int64_t)tile.slot * hot * R;
    for (int q = threadIdx.x; q < hot * R; q += blockDim.x) mine[q] = (float)shM2[q];
  }
}

// M2_p(j, :) += sum of the hot partial sums of problem p's mode-2 tiles;
// grid.y = problem.
template <int R>
__global__ void __launch_bounds__(256) k_mode2_reduce(const ProbDesc* __restrict__ P,
                                                       int max_hot) {
  constexpr int LDV = Geo<R>::LDV;
  const ProbDesc& D = P[blockIdx.y];
  const int hot = min(D.hot, max_hot);
  const int n = hot * R;
  const float* __restrict__ src = D.part;
  float* __restrict__ M2 = D.M2;
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
    // four independent partial sums (fixed order, so the result does not
    // depend on the launch) keep several of the strided loads in flight
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    int t = 0;
    for (; t + 4 <= D.nparts; t += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] += glob(src)[(int64_t)(t + u) * n + q];
    }
    for (; t < D.nparts; ++t) acc[0] += glob(src)[(int64_t)t * n + q];
    const int j = q / R, r = q - j * R;
    glob(M2)[(size_t)j * LDV + r] += (acc[0] + acc[1]) + (acc[2] + acc[3]);
  }
}

// ---------------------------------------------------------------------------
// Tall-skinny Gram out += A^T A (FP64) of an n x R float matrix with row
// stride lda: a group of lanes per row, column c per lane, block partial sums
// in LDS, one atomic per entry and block.
// ---------------------------------------------------------------------------
template <int R>
__device__ void gram_rows(const float* __restrict__ A, int64_t n, int lda, double* out,
                          int block, int nblocks) {
  constexpr int GPW = Geo<R>::GPW;
  const Lane L = lane_info<R>();
  const int wave = threadIdx.x / kWave;
  const int gpb = (blockDim.x / kWave) * GPW;
  double* sh = reinterpret_cast<double*>(p2_smem);
  for (int i = threadIdx.x; i < R * R; i += blockDim.x) sh[i] = 0.0;
  __syncthreads();
  const int c = L.j;
  if (L.live && c < R) {
    double acc[R];
#pragma unroll
    for (int l = 0; l < R; ++l) acc[l] = 0.0;
    const int64_t gid = (int64_t)block * gpb + wave * GPW + L.grp;
    const int64_t stride = (int64_t)nblocks * gpb;
    for (int64_t r = gid; r < n; r += stride) {
      const P2_GLOBAL float* a = glob(A) + r * lda;
      const double ac = (double)a[c];
#pragma unroll
      for (int l = 0; l < R; ++l) acc[l] = fma(ac, (double)a[l], acc[l]);
    }
#pragma unroll
    for (int l = 0; l < R; ++l)
      if (acc[l] != 0.0) atomicAdd(&sh[c * R + l], acc[l]);
  }
  block_reduce_atomic(sh, R * R, out);
}

template <int R>
__global__ void __launch_bounds__(256) k_gram_rows(const float* __restrict__ A, int64_t n,
                                                    int lda, double* out) {
  gram_rows<R>(A, n, lda, out, blockIdx.x, gridDim.x);
}

// Per problem (grid.y): which = 0: W^T W; 1: V_{t+1}^T V_{t+1} before
// normalisation (into VtVraw); 2: V_t^T V_t (into VtV).
template <int R>
__global__ void __launch_bounds__(256) k_gram(const ProbDesc* __restrict__ P, int which,
                                               int parity) {
  constexpr SmallLayout SL = small_layout(R);
  const ProbDesc& D = P[blockIdx.y];
  if (which == 0)
    gram_rows<R>(D.W, D.K, R, D.small + SL.WtW, blockIdx.x, gridDim.x);
  else if (which == 1)
    gram_rows<R>(D.V[parity ^ 1], D.J, Geo<R>::LDV, D.small + SL.VtVraw, blockIdx.x, gridDim.x);
  else
    gram_rows<R>(D.V[parity], D.J, Geo<R>::LDV, D.small + SL.VtV, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// small FP64 solves (one group of NC lanes per problem; grid = problems)
// ---------------------------------------------------------------------------

// Column c of N^+ for symmetric PSD N given column-per-lane (n = N(:, c)).
template <int R>
__device__ void pinv_cols(const double (&ncol)[R], int c, double* S, double* dl, double tau,
                          double tol, int max_sweeps, double (&out)[R]) {
  constexpr int NC = Geo<R>::NC;
  double g[R], v[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    g[i] = (c < R) ? ncol[i] : 0.0;
    v[i] = (i == c) ? 1.0 : 0.0;
  }
  const uint64_t gmask = (NC == 64) ? ~0ull : ((1ull << NC) - 1ull);
  // the normal-equation solves are tiny: run them to full FP64 convergence
  jacobi_onesided<R, R, false>(g, v, c, 0, gmask, c < NC, tol, 1e-18, max_sweeps);
  double lam2 = 0.0;
#pragma unroll
  for (int i = 0; i < R; ++i) lam2 = fma(g[i], g[i], lam2);
  const double lam = sqrt(lam2);
  if (c < NC) dl[c] = lam;
  __syncthreads();
  double lmax = 0.0;
  for (int p = 0; p < NC; ++p) lmax = fmax(lmax, dl[p]);
  __syncthreads();
  const bool keep = lam > tau * lmax && lam > 0.0;
  const double inv = keep ? 1.0 / lam : 0.0;
  if (c < NC) {
#pragma unroll
    for (int i = 0; i < R; ++i) S[c * R + i] = g[i] * inv;
    dl[c] = inv;
  }
  __syncthreads();
  const int cc = c < R ? c : 0;
#pragma unroll
  for (int i = 0; i < R; ++i) out[i] = 0.0;
  for (int p = 0; p < NC; ++p) {
    const double z = S[p * R + cc] * dl[p];
#pragma unroll
    for (int i = 0; i < R; ++i) out[i] = fma(z, S[p * R + i], out[i]);
  }
  __syncthreads();
}

// H <- M1 ((W^T W) * (V^T V))^+ (Algorithm "CP-ALS"), unit columns; H^T H;
// N2^+ = ((W^T W) * (H^T H))^+.
template <int R>
__global__ void __launch_bounds__(64) k_solve_h(const ProbDesc* __restrict__ P, PolarParams pp) {
  constexpr int NC = Geo<R>::NC;
  constexpr SmallLayout SL = small_layout(R);
  __shared__ double S[NC * R];
  __shared__ double dl[NC];
  __shared__ double Hs[R * R];
  const ProbDesc& D = P[blockIdx.x];
  const P2_GLOBAL double* M1 = glob(D.small) + SL.M1;
  const P2_GLOBAL double* WtW = glob(D.small) + SL.WtW;
  const P2_GLOBAL double* VtV = glob(D.small) + SL.VtV;
  P2_GLOBAL double* HtH = glob(D.small) + SL.HtH;
  P2_GLOBAL double* N2p = glob(D.small) + SL.N2p;
  P2_GLOBAL double* H = glob(D.H);
  const int c = threadIdx.x;
  const int cc = c < R ? c : 0;
  double ncol[R], np[R];
#pragma unroll
  for (int i = 0; i < R; ++i) ncol[i] = WtW[i * R + cc] * VtV[i * R + cc];
  pinv_cols<R>(ncol, c, S, dl, pp.tau_pinv, pp.tol, pp.max_sweeps, np);
  double h[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    double t = 0.0;
#pragma unroll
    for (int l = 0; l < R; ++l) t = fma(M1[i * R + l], np[l], t);
    h[i] = t;
  }
  double nrm = 0.0;
#pragma unroll
  for (int i = 0; i < R; ++i) nrm = fma(h[i], h[i], nrm);
  nrm = sqrt(nrm);
  const double sc = nrm > 1e-300 ? 1.0 / nrm : 1.0;
  __syncthreads();  // every lane has read M1 and the old H is no longer needed
  if (c < R) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      h[i] *= sc;
      Hs[i * R + c] = h[i];
      H[i * R + c] = h[i];
    }
  }
  __syncthreads();
#pragma unroll
  for (int l = 0; l < R; ++l) {
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < R; ++i) t = fma(Hs[i * R + l], Hs[i * R + cc], t);
    if (c < R) HtH[l * R + c] = t;
    ncol[l] = WtW[l * R + cc] * t;
  }
  pinv_cols<R>(ncol, c, S, dl, pp.tau_pinv, pp.tol, pp.max_sweeps, np);
  if (c < R) {
#pragma unroll
    for (int i = 0; i < R; ++i) N2p[i * R + c] = np[i];
  }
}

// V_raw(j, :) = M2(j, :) N2^+ into V_{t+1} (padding stays zero); grid.y = problem
template <int R>
__global__ void __launch_bounds__(256) k_vupdate(const ProbDesc* __restrict__ P, int parity) {
  constexpr int LDV = Geo<R>::LDV;
  constexpr SmallLayout SL = small_layout(R);
  const ProbDesc& D = P[blockIdx.y];
  if (D.nonneg) return;  // k_nnls_rows updates V
  const P2_GLOBAL float* M2 = glob(D.M2);
  const P2_GLOBAL double* N2p = glob(D.small) + SL.N2p;
  P2_GLOBAL float* Vout = glob(D.V[parity ^ 1]);
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < D.J;
       j += (int64_t)gridDim.x * blockDim.x) {
    double m[R];
#pragma unroll
    for (int l = 0; l < R; ++l) m[l] = (double)M2[j * LDV + l];
#pragma unroll
    for (int c = 0; c < R; ++c) {
      double t = 0.0;
#pragma unroll
      for (int l = 0; l < R; ++l) t = fma(m[l], N2p[l * R + c], t);
      Vout[j * LDV + c] = (float)t;
    }
  }
}

// V_{t+1} rows = NNLS((W^T W) * (H^T H), M2 rows) (replaces k_vupdate for the
// problems under the non-negativity constraint; the others are skipped; the W
// rows are solved in k_gamma).  grid.y = problem.
template <int R>
__global__ void __launch_bounds__(256) k_nnls_rows(const ProbDesc* __restrict__ P, int parity) {
  constexpr int GPW = Geo<R>::GPW;
  constexpr int LDV = Geo<R>::LDV;
  constexpr SmallLayout SL = small_layout(R);
  const ProbDesc& D = P[blockIdx.y];
  if (!D.nonneg) return;
  double* Ns = reinterpret_cast<double*>(p2_smem);  // N (R x R)
  const Lane L = lane_info<R>();
  const int wave = threadIdx.x / kWave;
  const int gpb = (blockDim.x / kWave) * GPW;
  double* buf = Ns + R * R + (wave * GPW + (L.live ? L.grp : 0)) * NnlsLds<R>::kPerGroup;
  const P2_GLOBAL double* sm = glob(D.small);
  for (int q = threadIdx.x; q < R * R; q += blockDim.x) Ns[q] = sm[SL.WtW + q] * sm[SL.HtH + q];
  __syncthreads();
  const int c = L.j;
  const bool real = c < R;
  const int cc = real ? c : 0;
  double ncol[R];
#pragma unroll
  for (int i = 0; i < R; ++i) ncol[i] = Ns[i * R + cc];
  if (L.live) {
    const int64_t stride = (int64_t)gridDim.x * gpb;
    for (int64_t r = (int64_t)blockIdx.x * gpb + wave * GPW + L.grp; r < D.J; r += stride) {
      const double m = real ? (double)glob(D.M2)[r * LDV + c] : 0.0;
      // the previous iteration's row gives the starting support
      const bool warm = real && glob(D.V[parity])[r * LDV + c] > 0.f;
      const double x = nnls_group<R>(ncol, m, c, buf, warm);
      if (real) glob(D.V[parity ^ 1])[r * LDV + c] = (float)x;
    }
  }
}

// ---------------------------------------------------------------------------
// Loss of subjects with I_k < R.  Their Procrustes factor Q_k = A F^T has
// orthonormal rows (the economy polar factor), so Q_k^T Q_k is a projector P_k
// rather than I and ||Q_k H S_k V^T||_F^2 = sum_rs w_r w_s (V^T V)_rs
// (H^T P_k H)_rs instead of w^T ((V^T V) * (H^T H)) w, which the mode-3 pass
// adds for every subject.  For each such subject this kernel forms
// K = H^T P_k H = sum_i u_i^T u_i from the rows u_i = A(i, :) F^T H of U_k,
// and adds the difference to the fit terms.  It runs after the W update
// (w = the stored W_{t+1} row), with F_k still from this iteration's
// Procrustes step (the next step is not fused for such problems).
// grid.y = problem.
// ---------------------------------------------------------------------------
template <int R>
struct EconLds {
  static constexpr int NC = Geo<R>::NC;
  static constexpr int CH = Geo<R>::CH;
  // gathered rows (CH x R floats), U rows (CH x R doubles), w (R)
  static constexpr int kPerGroup = (CH * R + 1) / 2 + CH * R + R;
};

template <int R>
__global__ void __launch_bounds__(256) k_econ_fit(const ProbDesc* __restrict__ P, int parity) {
  constexpr int NC = Geo<R>::NC;
  constexpr int GPW = Geo<R>::GPW;
  constexpr int CH = Geo<R>::CH;
  constexpr SmallLayout SL = small_layout(R);
  const ProbDesc& D = P[blockIdx.y];
  if (D.n_econ == 0) return;
  double* VtVs = reinterpret_cast<double*>(p2_smem);
  double* HtHs = VtVs + R * R;
  double* Hs = HtHs + R * R;
  double* shd = Hs + R * R;
  const Lane L = lane_info<R>();
  const int wave = threadIdx.x / kWave;
  const int gpb = (blockDim.x / kWave) * GPW;
  double* gb = shd + 2 + (wave * GPW + (L.live ? L.grp : 0)) * EconLds<R>::kPerGroup;
  float* Ab = reinterpret_cast<float*>(gb);
  double* Ub = gb + (CH * R + 1) / 2;
  double* wv = Ub + CH * R;
  load_shared_rxr<R>(VtVs, D.small + SL.VtV);
  load_shared_rxr<R>(HtHs, D.small + SL.HtH);
  load_shared_rxr<R>(Hs, D.H);
  if (threadIdx.x == 0) shd[0] = 0.0;
  __syncthreads();
  const int c = L.j;
  const bool real = c < R;
  const int cc = real ? c : 0;
  const float* __restrict__ V = D.V[parity];
  double delta = 0.0;
  if (L.live) {
    for (int64_t e = (int64_t)blockIdx.x * gpb + wave * GPW + L.grp; e < D.n_econ;
         e += (int64_t)gridDim.x * gpb) {
      const int64_t k = glob(D.econ)[e];
      const Subj sj = D.X.subj(k);
      // T(:, c) = F^T H(:, c): T(q, c) = sum_p F(p, q) H(p, c), F(p, q) at q R + p
      const P2_GLOBAL double* Fk = glob(D.F) + (size_t)k * R * R;
      double fr[R], kc[R];
#pragma unroll
      for (int q = 0; q < R; ++q) {
        double t = 0.0;
#pragma unroll
        for (int p = 0; p < R; ++p) t = fma(Fk[q * R + p], Hs[p * R + cc], t);
        fr[q] = t;
        kc[q] = 0.0;
      }
      for (int i0 = 0; i0 < sj.nrows; i0 += CH) {
        const int n = min(CH, sj.nrows - i0);
        gather_rows<R>(D.X, sj, i0, n, V, Ab, c);
        wave_sync();
        if (real) {
          for (int ii = 0; ii < n; ++ii) {
            double u = 0.0;
#pragma unroll
            for (int q = 0; q < R; ++q) u = fma((double)Ab[ii * R + q], fr[q], u);
            Ub[ii * R + c] = u;
          }
        }
        wave_sync();
        if (real) {
          for (int ii = 0; ii < n; ++ii) {
            const double uc = Ub[ii * R + c];
#pragma unroll
            for (int l = 0; l < R; ++l) kc[l] = fma(Ub[ii * R + l], uc, kc[l]);
          }
        }
        wave_sync();
      }
      if (real) wv[c] = (double)glob(D.W)[k * R + c];
      wave_sync();
      if (real) {
        double t = 0.0;
#pragma unroll
        for (int l = 0; l < R; ++l)
          t = fma(wv[l] * VtVs[l * R + c], kc[l] - HtHs[l * R + c], t);
        delta = fma(wv[c], t, delta);
      }
      wave_sync();
    }
  }
  if (L.live && real && delta != 0.0) atomicAdd(&shd[0], delta);
  __syncthreads();
  if (threadIdx.x == 0 && shd[0] != 0.0) gadd(D.small + SL.fitacc + 1, shd[0]);
}

// Column norms of V_raw from its Gram, V^T V of the normalised V,
// N3 = (V^T V) * (H^T H) and N3^+; grid = problems.
template <int R>
__global__ void __launch_bounds__(64) k_solve_n3(const ProbDesc* __restrict__ P, PolarParams pp) {
  constexpr int NC = Geo<R>::NC;
  constexpr SmallLayout SL = small_layout(R);
  __shared__ double S[NC * R];
  __shared__ double dl[NC];
  __shared__ double inv[R];
  const ProbDesc& D = P[blockIdx.x];
  const P2_GLOBAL double* VtVraw = glob(D.small) + SL.VtVraw;
  const P2_GLOBAL double* HtH = glob(D.small) + SL.HtH;
  P2_GLOBAL double* VtV = glob(D.small) + SL.VtV;
  P2_GLOBAL double* invnorm = glob(D.small) + SL.inv;
  P2_GLOBAL double* N3 = glob(D.small) + SL.N3;
  P2_GLOBAL double* N3p = glob(D.small) + SL.N3p;
  const int c = threadIdx.x;
  const int cc = c < R ? c : 0;
  if (c < R) {
    const double nrm = sqrt(VtVraw[c * R + c]);
    inv[c] = nrm > 1e-300 ? 1.0 / nrm : 1.0;
    invnorm[c] = inv[c];
  }
  __syncthreads();
  double ncol[R], np[R];
#pragma unroll
  for (int l = 0; l < R; ++l) {
    const double vtv = VtVraw[l * R + cc] * inv[l] * inv[cc];
    if (c < R) {
      VtV[l * R + c] = vtv;
      N3[l * R + c] = vtv * HtH[l * R + c];
    }
    ncol[l] = vtv * HtH[l * R + cc];
  }
  pinv_cols<R>(ncol, c, S, dl, pp.tau_pinv, pp.tol, pp.max_sweeps, np);
  if (c < R) {
#pragma unroll
    for (int i = 0; i < R; ++i) N3p[i * R + c] = np[i];
  }
}

// V_{t+1}(:, c) *= 1 / ||column c||; grid.y = problem
template <int R>
__global__ void __launch_bounds__(256) k_vscale(const ProbDesc* __restrict__ P, int parity) {
  constexpr int LDV = Geo<R>::LDV;
  constexpr SmallLayout SL = small_layout(R);
  const ProbDesc& D = P[blockIdx.y];
  P2_GLOBAL float* Vv = glob(D.V[parity ^ 1]);
  const P2_GLOBAL double* invnorm = glob(D.small) + SL.inv;
  const int64_t n = D.J * LDV;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(t % LDV);
    if (c < R) Vv[t] = (float)((double)Vv[t] * invnorm[c]);
  }
}

// Zero the per-iteration accumulators selected by mask (1 M1, 2 W^T W,
// 4 V^T V raw, 8 fit terms, 16 M2); grid.y = problem.
template <int R>
__global__ void __launch_bounds__(256) k_zero(const ProbDesc* __restrict__ P, int mask) {
  constexpr int LDV = Geo<R>::LDV;
  constexpr SmallLayout SL = small_layout(R);
  const ProbDesc& D = P[blockIdx.y];
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int nth = gridDim.x * blockDim.x;
  if (mask & 1)
    for (int q = tid; q < R * R; q += nth) glob(D.small)[SL.M1 + q] = 0.0;
  if (mask & 2)
    for (int q = tid; q < R * R; q += nth) glob(D.small)[SL.WtW + q] = 0.0;
  if (mask & 4)
    for (int q = tid; q < R * R; q += nth) glob(D.small)[SL.VtVraw + q] = 0.0;
  if (mask & 8)
    for (int q = tid; q < 2; q += nth) glob(D.small)[SL.fitacc + q] = 0.0;
  if (mask & 16) {
    const int64_t n = D.J * LDV;
    for (int64_t q = tid; q < n; q += nth) glob(D.M2)[q] = 0.f;
  }
}

// loss and fit = 1 - loss / ||X||^2 into the ring slots of the iteration,
// which it then counts as done; grid = problems
template <int R>
__global__ void k_fit(const ProbDesc* __restrict__ P) {
  constexpr SmallLayout SL = small_layout(R);
  if (threadIdx.x == 0) {
    const ProbDesc& D = P[blockIdx.x];
    const P2_GLOBAL double* fa = glob(D.small) + SL.fitacc;
    const double nx2 = glob(D.small)[SL.nx2];
    const double loss = nx2 - 2.0 * fa[0] + fa[1];
    const int64_t it = glob(D.iter)[0];
    glob(D.small)[SL.fits + (int)(it % kFitRing)] = 1.0 - loss / nx2;
    glob(D.small)[SL.losses + (int)(it % kFitRing)] = loss;
    glob(D.iter)[0] = it + 1;
  }
}


// ---------------------------------------------------------------------------
// Q_k = A_k F_k^T for subjects [k0, k1), or U_k = Q_k Hm = A_k (F_k^T Hm)
// when Hm (R x R, row-major) is given: rows written contiguously from Q.
// ---------------------------------------------------------------------------
template <int R>
__global__ void __launch_bounds__(256) k_getq(XEnc X, int64_t k0, int64_t k1,
                                               const float* __restrict__ V,
                                               const double* __restrict__ F, float* __restrict__ Q,
                                               int64_t row0, const double* __restrict__ Hm) {
  constexpr int NC = Geo<R>::NC;
  constexpr int GPW = Geo<R>::GPW;
  constexpr int CH = NC;
  const Lane L = lane_info<R>();
  const int wave = threadIdx.x / kWave;
  const int groups_per_block = (blockDim.x / kWave) * GPW;
  float* gbuf = reinterpret_cast<float*>(p2_smem) + (wave * GPW + (L.live ? L.grp : 0)) * (CH * R);
  if (!L.live) return;
  const int c = L.j;
  const int64_t gid = (int64_t)blockIdx.x * groups_per_block + wave * GPW + L.grp;
  const int64_t stride = (int64_t)gridDim.x * groups_per_block;
  for (int64_t k = k0 + gid; k < k1; k += stride) {
    const Subj s = X.subj(k);
    double fr[R];  // Q(i, c) = sum_p A(i, p) F(c, p), F(c, p) at p R + c
    const P2_GLOBAL double* Fk = glob(F) + (size_t)k * R * R;
    const int cc = c < R ? c : 0;
    if (Hm) {
      // U(i, c) = sum_q A(i, q) T(q, c), T = F^T Hm: T(q, c) = sum_p F(p, q) Hm(p, c)
#pragma unroll
      for (int q = 0; q < R; ++q) {
        double t = 0.0;
#pragma unroll
        for (int p = 0; p < R; ++p) t = fma(Fk[q * R + p], glob(Hm)[p * R + cc], t);
        fr[q] = t;
      }
    } else {
#pragma unroll
      for (int p = 0; p < R; ++p) fr[p] = Fk[p * R + cc];
    }
    for (int i0 = 0; i0 < s.nrows; i0 += CH) {
      const int n = min(CH, s.nrows - i0);
      gather_rows<R>(X, s, i0, n, V, gbuf, c);
      wave_sync();
      if (c < R) {
        for (int ii = 0; ii < n; ++ii) {
          double t = 0.0;
#pragma unroll
          for (int p = 0; p < R; ++p) t = fma((double)gbuf[ii * R + p], fr[p], t);
          Q[(s.r0 - row0 + i0 + ii) * R + c] = (float)t;
        }
      }
      wave_sync();
    }
  }
}

// ---------------------------------------------------------------------------
// projection of new subjects onto fixed (V, H): n_steps alternations of the
// Procrustes step and the least-squares update of w (plain CSR input).  The
// Procrustes step uses the factored form (polar_factored), with C = A^T A
// eigen-decomposed once per subject.
// ---------------------------------------------------------------------------
template <int R>
struct ProjLds {
  static constexpr int NC = Geo<R>::NC;
  // C = A^T A until it is factored, then each lane's start basis for the
  // SVD steps (NC x R), then F
  static constexpr int oCs = 0;
  static constexpr int oEc = oCs + NC * R;
  static constexpr int oS = oEc + NC * R;   // also the gather chunk
  static constexpr int oS2 = oS + NC * R;
  static constexpr int oSv = oS2 + NC * R;
  static constexpr int oIsv = oSv + NC;
  static constexpr int oW = oIsv + NC;
  static constexpr int oM = oW + R;
  static constexpr int oDl = oM + R;
  static constexpr int kPerGroup = oDl + NC;
};

template <int R>
__global__ void __launch_bounds__(256) k_project(XRaw X, int64_t K, const float* __restrict__ V,
                                                  const double* __restrict__ H,
                                                  const double* __restrict__ N3,
                                                  const double* __restrict__ N3p, int n_steps,
                                                  const float* __restrict__ w0,
                                                  float* __restrict__ Qout,
                                                  float* __restrict__ wout,
                                                  double* __restrict__ lossout, PolarParams pp) {
  constexpr int NC = Geo<R>::NC;
  constexpr int GPW = Geo<R>::GPW;
  constexpr int CH = NC;
  using PL = ProjLds<R>;
  const Lane L = lane_info<R>();
  const int wave = threadIdx.x / kWave;
  const int groups_per_block = (blockDim.x / kWave) * GPW;
  double* Hs = reinterpret_cast<double*>(p2_smem);
  double* N3s = Hs + R * R;
  double* N3ps = N3s + R * R;
  double* gbuf = N3ps + R * R + (wave * GPW + (L.live ? L.grp : 0)) * PL::kPerGroup;
  double* Cs = gbuf + PL::oCs;
  double* Ec = gbuf + PL::oEc;
  double* S = gbuf + PL::oS;
  double* S2 = gbuf + PL::oS2;
  double* sv = gbuf + PL::oSv;
  double* isv = gbuf + PL::oIsv;
  double* wv = gbuf + PL::oW;
  double* mv = gbuf + PL::oM;
  double* dl = gbuf + PL::oDl;
  load_shared_rxr<R>(Hs, H);
  load_shared_rxr<R>(N3s, N3);
  load_shared_rxr<R>(N3ps, N3p);
  __syncthreads();
  if (!L.live) return;
  const int c = L.j;
  const bool real = c < R;
  const int cc = real ? c : 0;
  const int64_t gid = (int64_t)blockIdx.x * groups_per_block + wave * GPW + L.grp;
  const int64_t stride = (int64_t)gridDim.x * groups_per_block;
  for (int64_t k = gid; k < K; k += stride) {
    const Subj s = X.subj(k);
    {
      double crow[R];
#pragma unroll
      for (int l = 0; l < R; ++l) crow[l] = 0.0;
      for (int i0 = 0; i0 < s.nrows; i0 += CH) {
        const int n = min(CH, s.nrows - i0);
        gather_rows<R>(X, s, i0, n, V, S, c);
        wave_sync();
        gram_accum<R>(S, S, n, c, crow);
        wave_sync();
      }
      if (real) {
#pragma unroll
        for (int l = 0; l < R; ++l) Cs[c * R + l] = crow[l];
        wv[c] = w0 ? (double)w0[k * R + c] : 1.0;
      }
    }
    double xx = 0.0;  // ||X_k||^2, summed by lane 0 of the group
    if (c == 0) {
      for (int z = 0; z < s.nnz; ++z) {
        const double x = (double)X.val[s.z0 + z];
        xx = fma(x, x, xx);
      }
    }
    wave_sync();
    factor_c<R>(Cs, Ec, sv, isv, dl, c, L.gbase, L.gmask, pp.tau_c, pp.tol, pp.stop2,
                pp.max_sweeps);
    double yv[R], m3 = 0.0;
#pragma nounroll
    for (int step = 0; step < n_steps; ++step) {
      // steps after the first start the SVD from the previous step's basis
      polar_factored<R>(Ec, sv, isv, wv, Hs, S, S2, dl, c, L.gbase, L.gmask, pp.tau_s, pp.tol,
                        pp.stop2, pp.max_sweeps, step + 1 == n_steps, step > 0, Cs, yv, Cs);
      m3 = 0.0;
#pragma unroll
      for (int i = 0; i < R; ++i) m3 = fma(Hs[i * R + cc], yv[i], m3);
      if (real) mv[c] = m3;
      wave_sync();
      double wn = 0.0;
#pragma unroll
      for (int l = 0; l < R; ++l) wn = fma(mv[l], N3ps[l * R + cc], wn);
      wave_sync();
      if (real) wv[c] = wn;
      wave_sync();
    }
    // outputs: w, loss = ||X||^2 - 2 <w, m3> + w^T N3 w, Q = A F^T
    double t = 0.0;
#pragma unroll
    for (int l = 0; l < R; ++l) t = fma(N3s[cc * R + l], wv[l], t);
    const double part = real ? (-2.0 * wv[c] * m3 + wv[c] * t) : 0.0;
    if (real) wout[k * R + c] = (float)wv[c];
    wave_sync();
    if (real) mv[c] = part;
    wave_sync();
    if (c == 0 && lossout) {
      double loss = xx;
      for (int l = 0; l < R; ++l) loss += mv[l];
      lossout[k] = loss;
    }
    wave_sync();
    if (Qout && n_steps > 0) {
      // Q(i, c) = sum_p A(i, p) F(c, p)
      float* Ab = reinterpret_cast<float*>(S);
      for (int i0 = 0; i0 < s.nrows; i0 += CH) {
        const int n = min(CH, s.nrows - i0);
        gather_rows<R>(X, s, i0, n, V, Ab, c);
        wave_sync();
        if (real) {
          for (int ii = 0; ii < n; ++ii) {
            double q = 0.0;
#pragma unroll
            for (int p = 0; p < R; ++p) q = fma((double)Ab[ii * R + p], Cs[c * R + p], q);
            Qout[(s.r0 + i0 + ii) * R + c] = (float)q;
          }
        }
        wave_sync();
      }
    }
    wave_sync();
  }
}

// N3 = (V^T V) * (H^T H) and N3^+ for a projection model with fixed V and H.
template <int R>
__global__ void __launch_bounds__(64) k_model_prep(const double* __restrict__ VtV,
                                                    const double* __restrict__ H,
                                                    double* __restrict__ HtH,
                                                    double* __restrict__ N3,
                                                    double* __restrict__ N3p, PolarParams pp) {
  constexpr int NC = Geo<R>::NC;
  __shared__ double S[NC * R];
  __shared__ double dl[NC];
  const int c = threadIdx.x;
  const int cc = c < R ? c : 0;
  double ncol[R], np[R];
#pragma unroll
  for (int l = 0; l < R; ++l) {
    double t = 0.0;
    for (int i = 0; i < R; ++i) t = fma(H[i * R + l], H[i * R + cc], t);
    if (c < R) {
      HtH[l * R + c] = t;
      N3[l * R + c] = VtV[l * R + c] * t;
    }
    ncol[l] = VtV[l * R + cc] * t;
  }
  pinv_cols<R>(ncol, c, S, dl, pp.tau_pinv, pp.tol, pp.max_sweeps, np);
  if (c < R) {
#pragma unroll
    for (int i = 0; i < R; ++i) N3p[i * R + c] = np[i];
  }
}

}  // namespace p2

// ===========================================================================
// launchers
// ===========================================================================
namespace p2 {

namespace {

constexpr int kMaxBlocks = 2048;
constexpr size_t kLdsPerCu = 160 * 1024;  // bytes of LDS one workgroup may use on gfx950

inline int grid_for(int64_t units, int per_block) {
  int64_t b = (units + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > kMaxBlocks) b = kMaxBlocks;
  return (int)b;
}

// LDS a plan may hand out as dynamic LDS: the CU's LDS less room for the few
// words of static LDS some kernels declare (tile claims).
constexpr size_t kStaticLdsRoom = 256;
constexpr size_t kLdsBudget = kLdsPerCu - kStaticLdsRoom;

// Refuse an LDS request that does not fit next to the kernel's static LDS;
// above the default 64 KB, raise the kernel's dynamic-LDS cap to all that
// is left (a cap, not a reservation: launches of the same kernel with other
// sizes stay valid).
template <class Kern>
hipError_t allow_lds(Kern k, size_t bytes) {
  hipFuncAttributes fa{};
  hipError_t e = hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(k));
  if (e != hipSuccess) return e;
  const size_t stat = fa.sharedSizeBytes;
  if (stat > kStaticLdsRoom || bytes + stat > kLdsPerCu) return hipErrorInvalidConfiguration;
  if (bytes + stat <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(k),
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)(kLdsPerCu - stat));
}

// Largest block (from `cands`, in wavefronts of 64) whose LDS, `shared` bytes
// for the block plus `group` bytes per subject group, fits in `budget`; 0 if
// none does.
template <int R>
constexpr int pick_threads(size_t shared, size_t group, size_t budget, int max_threads) {
  for (int t = max_threads; t >= kWave; t /= 2) {
    if (shared + (size_t)(t / kWave) * Geo<R>::GPW * group <= budget) return t;
  }
  return 0;
}

// LDS layout of each kernel: bytes shared by the block and bytes per group.
template <int R> constexpr size_t alpha_shared() { return sizeof(double) * 2 * R * R; }
template <int R> constexpr size_t alpha_group() { return sizeof(double) * PolarLds<R>::kPerGroup; }
template <int R> constexpr size_t gamma_shared() { return sizeof(double) * (4 * R * R + 2); }
template <int R> constexpr size_t gamma_group() { return sizeof(double) * PolarLds<R>::kPerGroup; }
template <int R> constexpr size_t proj_shared() { return sizeof(double) * 3 * R * R; }
template <int R> constexpr size_t proj_group() { return sizeof(double) * ProjLds<R>::kPerGroup; }
template <int R> constexpr size_t getq_group() { return sizeof(float) * Geo<R>::NC * R; }
template <int R> constexpr size_t mode2_group() { return sizeof(float) * Mode2Lds<R>::kPerGroup; }

template <int R> constexpr int alpha_threads() {
  return pick_threads<R>(alpha_shared<R>(), alpha_group<R>(), kLdsBudget, 256);
}
template <int R> constexpr int gamma_threads() {
  return pick_threads<R>(gamma_shared<R>(), gamma_group<R>(), kLdsBudget, 256);
}
template <int R> constexpr int proj_threads() {
  return pick_threads<R>(proj_shared<R>(), proj_group<R>(), kLdsBudget, 256);
}
template <int R> constexpr int getq_threads() {
  return pick_threads<R>(0, getq_group<R>(), kLdsBudget, 256);
}
// mode 2: the per-group buffers may take at most half of the LDS, the waves'
// cold-update queues and the hot column partial sums take the rest; the DPP
// kernel (R <= 16) has no per-group buffers, only H' next to the hot sums
template <int R> constexpr size_t mode2_groups_bytes_at(int threads) {
  if constexpr (kMode2UsesDpp<R>)
    return sizeof(float) * (Mode2Dpp<R>::kHFloats + (size_t)(threads / kWave) * Mode2Dpp<R>::kQueueFloats);
  return (size_t)(threads / kWave) *
         (Geo<R>::GPW * mode2_group<R>() + sizeof(float) * Mode2Lds<R>::kQueueFloats);
}
template <int R> constexpr size_t mode2_ebytes_at(int threads) {
  if constexpr (kMode2UsesDpp<R>) return 0;
  return (size_t)(threads / kWave) * Geo<R>::GPW * mode2_group<R>();
}
// Share of a block's LDS budget that the groups' E_k buffers of the R > 16
// mode-2 kernel may take; the rest holds the hot-column sums.  The pass is
// bound by the latency of its loads, so waves in flight count for more than
// hot columns (on the K = 1M slices, R = 32: 29.0 ms with half of the LDS,
// 19.1 with 3/4, 17.2 with 7/8; R = 40: 38.5, 31.0, 31.0 ms).
constexpr size_t mode2_ebudget(size_t budget) { return budget * 7 / 8; }

// Default mode-2 block: for R > 16 the most waves whose E_k buffers fit in
// that share.
template <int R> constexpr int mode2_threads() {
  if constexpr (kMode2UsesDpp<R>) return kMode2Threads;
  for (int t = Mode2Lds<R>::kMaxThreads; t >= kWave; t -= kWave)
    if (mode2_ebytes_at<R>(t) <= mode2_ebudget(kLdsBudget) &&
        mode2_groups_bytes_at<R>(t) + 2048 <= kLdsBudget)
      return t;
  return 0;
}
// subject groups per wave of the rank's mode-2 kernel
template <int R> constexpr int mode2_gpw() {
  if constexpr (kMode2UsesDpp<R>) return Mode2Dpp<R>::kGroups;
  return Geo<R>::GPW;
}
template <int R> constexpr size_t mode2_groups_bytes() {
  return mode2_groups_bytes_at<R>(mode2_threads<R>());
}
template <int R> constexpr int max_hot_t() {
  return (int)((kLdsBudget - 2048 - mode2_groups_bytes<R>()) / (sizeof(double) * R));
}

// The ranks the library is built for: every R from 1 to 40.
#define P2_RANKS(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) X(18) X(19) X(20) X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) X(29) X(30) X(31) X(32) X(33) X(34) X(35) X(36) X(37) X(38) X(39) X(40)

// every built rank has a launch configuration that fits the LDS
#define P2_CHECK_PLAN(r)                                                         \
  static_assert(r % 2 == 1 || (alpha_shared<r>() % 16 == 0 &&                    \
                               gamma_shared<r>() % 16 == 0),                     \
                "block LDS prefix must keep group regions 16-byte aligned");    \
  static_assert(alpha_threads<r>() > 0 && gamma_threads<r>() > 0 &&              \
                    proj_threads<r>() > 0 && getq_threads<r>() > 0 &&            \
                    mode2_threads<r>() > 0 && max_hot_t<r>() >= 0,               \
                "LDS plan does not fit for R=" #r);

template <int R> constexpr int polar_gpb() { return (gamma_threads<R>() / kWave) * Geo<R>::GPW; }
template <int R> constexpr int mode2_gpb() { return (mode2_threads<R>() / kWave) * mode2_gpw<R>(); }
template <int R> constexpr size_t alpha_lds() {
  return alpha_shared<R>() + (size_t)(alpha_threads<R>() / kWave) * Geo<R>::GPW * alpha_group<R>();
}
template <int R> constexpr size_t gamma_lds() {
  return gamma_shared<R>() + (size_t)(gamma_threads<R>() / kWave) * Geo<R>::GPW * gamma_group<R>();
}
template <int R> size_t mode2_lds(int hot) {
  return sizeof(float) * (size_t)Mode2Lds<R>::hot_floats(hot) + mode2_groups_bytes<R>();
}

inline int device_cus() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return n;
}

// Workgroups of kernel k that fit on the device at once, rounded down to a
// multiple of kBins (so a static schedule keeps every block in its XCD's bin)
// and capped at `want` rounded up the same way.
template <class Kern>
hipError_t resident_grid(Kern k, int threads, size_t lds, int want, int* grid) {
  hipError_t e = allow_lds(k, lds);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k),
                                                   threads, lds);
  if (e != hipSuccess) return e;
  const int cus = device_cus();
  if (per_cu < 1 || cus < 1) return hipErrorInvalidConfiguration;
  int g = per_cu * cus / kBins * kBins;
  if (g < kBins) g = kBins;
  const int w = (want + kBins - 1) / kBins * kBins;
  if (w > 0 && g > w) g = w;
  *grid = g;
  return hipSuccess;
}

// Ranks whose warm-started polar kernels are built (the accumulated Jacobi
// basis must fit the register file next to the rest of the kernel).
constexpr int kWarmMaxR = 20;

template <int R>
hipError_t plan_t(BatchView& b) {
  if (b.ntiles % kBins != 0 || b.nm2 % kBins != 0) return hipErrorInvalidValue;
  if (b.max_hot < 0 || b.max_hot > max_hot_t<R>()) return hipErrorInvalidValue;
  if (R > kWarmMaxR) b.warm = 0;
  hipError_t e;
  if constexpr (R <= kWarmMaxR) {
    if (b.warm) {
      e = resident_grid(k_alpha<R, true>, alpha_threads<R>(), alpha_lds<R>(), b.ntiles,
                        &b.grid_alpha);
      if (e != hipSuccess) return e;
      e = b.nonneg ? resident_grid(k_gamma<R, true, true>, gamma_threads<R>(), gamma_lds<R>(),
                                   b.ntiles, &b.grid_gamma)
                   : resident_grid(k_gamma<R, true, false>, gamma_threads<R>(), gamma_lds<R>(),
                                   b.ntiles, &b.grid_gamma);
      if (e != hipSuccess) return e;
    }
  }
  if (!b.warm) {
    e = resident_grid(k_alpha<R, false>, alpha_threads<R>(), alpha_lds<R>(), b.ntiles,
                      &b.grid_alpha);
    if (e != hipSuccess) return e;
    e = b.nonneg ? resident_grid(k_gamma<R, false, true>, gamma_threads<R>(), gamma_lds<R>(),
                                 b.ntiles, &b.grid_gamma)
                 : resident_grid(k_gamma<R, false, false>, gamma_threads<R>(), gamma_lds<R>(),
                                 b.ntiles, &b.grid_gamma);
    if (e != hipSuccess) return e;
  }
  // mode 2: blocks of m2_threads (0 = the rank's default) with m2_blocks of
  // them sharing a CU; each block's hot-column partial sums get what its
  // share of the LDS leaves after the groups' E buffers
  const int bpc = b.m2_blocks > 0 ? b.m2_blocks : 1;
  const size_t budget = kLdsBudget / (size_t)bpc;
  int threads = b.m2_threads > 0 ? b.m2_threads : mode2_threads<R>();
  threads = threads / kWave * kWave;
  if (threads > Mode2Lds<R>::kMaxThreads) threads = Mode2Lds<R>::kMaxThreads;
  while (threads > kWave && (mode2_ebytes_at<R>(threads) > mode2_ebudget(budget) ||
                             mode2_groups_bytes_at<R>(threads) + 2048 > budget))
    threads -= kWave;
  if (threads < kWave || mode2_groups_bytes_at<R>(threads) + 2048 > budget)
    return hipErrorInvalidConfiguration;
  int hot = (int)((budget - 2048 - mode2_groups_bytes_at<R>(threads)) / (sizeof(double) * R));
  if (hot > b.max_hot) hot = b.max_hot;
  b.m2_threads = threads;
  b.m2_hot = hot;
  b.m2_lds = sizeof(float) * (size_t)Mode2Lds<R>::hot_floats(hot) +
             mode2_groups_bytes_at<R>(threads);
  if constexpr (kMode2UsesDpp<R>)
    return resident_grid(k_mode2_dpp<R>, threads, b.m2_lds, b.nm2, &b.grid_mode2);
  else
    return resident_grid(k_mode2<R>, threads, b.m2_lds, b.nm2, &b.grid_mode2);
}

inline int* tickets_of(const BatchView& b, int kind) {
  return b.dynamic ? b.tickets + kind * kBins : nullptr;
}

template <int R, bool WARM>
hipError_t alpha_w(const BatchView& b, int parity, const PolarParams& pp, hipStream_t s) {
  hipLaunchKernelGGL((k_alpha<R, WARM>), dim3(b.grid_alpha), dim3(alpha_threads<R>()),
                     alpha_lds<R>(), s, b.desc, b.tiles, b.ntiles, tickets_of(b, kTicketAlpha),
                     parity, pp);
  return hipGetLastError();
}

template <int R, bool WARM>
hipError_t gamma_w(const BatchView& b, int parity, int do_next, const PolarParams& pp,
                   hipStream_t s) {
  if (b.nonneg)
    hipLaunchKernelGGL((k_gamma<R, WARM, true>), dim3(b.grid_gamma), dim3(gamma_threads<R>()),
                       gamma_lds<R>(), s, b.desc, b.tiles, b.ntiles,
                       tickets_of(b, kTicketGamma), parity, do_next, pp);
  else
    hipLaunchKernelGGL((k_gamma<R, WARM, false>), dim3(b.grid_gamma), dim3(gamma_threads<R>()),
                       gamma_lds<R>(), s, b.desc, b.tiles, b.ntiles,
                       tickets_of(b, kTicketGamma), parity, do_next, pp);
  return hipGetLastError();
}

template <int R>
hipError_t alpha_t(const BatchView& b, int parity, const PolarParams& pp, hipStream_t s) {
  if constexpr (R <= kWarmMaxR) {
    if (b.warm) return alpha_w<R, true>(b, parity, pp, s);
  }
  return alpha_w<R, false>(b, parity, pp, s);
}

template <int R>
hipError_t gamma_t(const BatchView& b, int parity, int do_next, const PolarParams& pp,
                   hipStream_t s) {
  if constexpr (R <= kWarmMaxR) {
    if (b.warm) return gamma_w<R, true>(b, parity, do_next, pp, s);
  }
  return gamma_w<R, false>(b, parity, do_next, pp, s);
}

template <int R>
hipError_t mode2_t(const BatchView& b, int parity, hipStream_t s) {
  if constexpr (kMode2UsesDpp<R>)
    hipLaunchKernelGGL(k_mode2_dpp<R>, dim3(b.grid_mode2), dim3(b.m2_threads), b.m2_lds, s,
                       b.desc, b.m2tiles, b.nm2, tickets_of(b, kTicketMode2), parity, b.m2_hot);
  else
    hipLaunchKernelGGL(k_mode2<R>, dim3(b.grid_mode2), dim3(b.m2_threads), b.m2_lds, s, b.desc,
                       b.m2tiles, b.nm2, tickets_of(b, kTicketMode2), parity, b.m2_hot);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || b.m2_hot == 0) return e;
  int rb = (b.m2_hot * R + 255) / 256;
  if (rb > 1024) rb = 1024;
  hipLaunchKernelGGL(k_mode2_reduce<R>, dim3(rb, b.np), dim3(256), 0, s, b.desc, b.m2_hot);
  return hipGetLastError();
}

template <int R>
hipError_t gram_t(const BatchView& b, int which, int parity, hipStream_t s) {
  const int gpb = (256 / kWave) * Geo<R>::GPW;
  // about 64 rows per lane group: each block ends with R^2 FP64 global
  // atomics, which are memory transactions, so fewer and longer blocks
  const int gx = grid_for(which == 0 ? b.maxK : b.maxJ, gpb * 64);
  hipLaunchKernelGGL(k_gram<R>, dim3(gx, b.np), dim3(256), sizeof(double) * R * R, s, b.desc,
                     which, parity);
  return hipGetLastError();
}

template <int R>
hipError_t getq_t(const XEnc& X, int64_t k0, int64_t k1, const float* V, const double* F, float* Q,
                  int64_t row0, const double* Hm, hipStream_t s) {
  constexpr int T = getq_threads<R>();
  const int gpb = (T / kWave) * Geo<R>::GPW;
  const size_t lds = (size_t)gpb * getq_group<R>();
  hipError_t e = allow_lds(k_getq<R>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_getq<R>, dim3(grid_for(k1 - k0, gpb)), dim3(T), lds, s, X, k0, k1, V, F, Q,
                     row0, Hm);
  return hipGetLastError();
}

template <int R>
hipError_t project_t(const XRaw& X, int64_t K, const float* V, const double* H, const double* N3,
                     const double* N3p, int n_steps, const float* w0, float* Qout, float* wout,
                     double* lossout, const PolarParams& pp, hipStream_t s) {
  constexpr int T = proj_threads<R>();
  const int gpb = (T / kWave) * Geo<R>::GPW;
  const size_t lds = proj_shared<R>() + (size_t)gpb * proj_group<R>();
  hipError_t e = allow_lds(k_project<R>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_project<R>, dim3(grid_for(K, gpb)), dim3(T), lds, s, X, K, V, H, N3, N3p,
                     n_steps, w0, Qout, wout, lossout, pp);
  return hipGetLastError();
}

inline int grid1(int64_t n, int T = 256) {
  int64_t b = (n + T - 1) / T;
  if (b < 1) b = 1;
  if (b > 4096) b = 4096;
  return (int)b;
}


template <int R>
hipError_t nnls_t(const BatchView& b, int parity, hipStream_t s) {
  constexpr int T = 256;
  constexpr int gpb = (T / kWave) * Geo<R>::GPW;
  constexpr size_t lds = sizeof(double) * (R * R + gpb * NnlsLds<R>::kPerGroup);
  static_assert(lds <= kLdsBudget, "NNLS LDS plan");
  hipError_t e = allow_lds(k_nnls_rows<R>, lds);
  if (e != hipSuccess) return e;
  const int gx = (int)std::max<int64_t>(1, std::min<int64_t>((b.maxJ + gpb - 1) / gpb, 8192));
  hipLaunchKernelGGL(k_nnls_rows<R>, dim3(gx, b.np), dim3(T), lds, s, b.desc, parity);
  return hipGetLastError();
}

template <int R>
hipError_t econ_t(const BatchView& b, int parity, hipStream_t s) {
  constexpr int T = 256;
  constexpr int gpb = (T / kWave) * Geo<R>::GPW;
  constexpr size_t lds = sizeof(double) * (3 * R * R + 2 + gpb * EconLds<R>::kPerGroup);
  static_assert(lds <= kLdsBudget, "loss-correction LDS plan");
  hipError_t e = allow_lds(k_econ_fit<R>, lds);
  if (e != hipSuccess) return e;
  const int gx = (int)std::max<int64_t>(1, std::min<int64_t>((b.maxEcon + gpb - 1) / gpb, 4096));
  hipLaunchKernelGGL(k_econ_fit<R>, dim3(gx, b.np), dim3(T), lds, s, b.desc, parity);
  return hipGetLastError();
}

template <int R>
hipError_t solve_h_t(const BatchView& b, const PolarParams& pp, hipStream_t s) {
  hipLaunchKernelGGL(k_solve_h<R>, dim3(b.np), dim3(64), 0, s, b.desc, pp);
  return hipGetLastError();
}

template <int R>
hipError_t vupdate_t(const BatchView& b, int parity, hipStream_t s) {
  hipLaunchKernelGGL(k_vupdate<R>, dim3(grid1(b.maxJ), b.np), dim3(256), 0, s, b.desc, parity);
  return hipGetLastError();
}

template <int R>
hipError_t solve_n3_t(const BatchView& b, const PolarParams& pp, hipStream_t s) {
  hipLaunchKernelGGL(k_solve_n3<R>, dim3(b.np), dim3(64), 0, s, b.desc, pp);
  return hipGetLastError();
}

template <int R>
hipError_t vscale_t(const BatchView& b, int parity, hipStream_t s) {
  hipLaunchKernelGGL(k_vscale<R>, dim3(grid1(b.maxJ * Geo<R>::LDV), b.np), dim3(256), 0, s,
                     b.desc, parity);
  return hipGetLastError();
}

template <int R>
hipError_t zero_t(const BatchView& b, int mask, hipStream_t s) {
  const int gx = (mask & 16) ? grid1(b.maxJ * ((R + 3) & ~3)) : 1;
  hipLaunchKernelGGL(k_zero<R>, dim3(gx, b.np), dim3(256), 0, s, b.desc, mask);
  return hipGetLastError();
}

template <int R>
hipError_t fit_t(const BatchView& b, hipStream_t s) {
  hipLaunchKernelGGL(k_fit<R>, dim3(b.np), dim3(64), 0, s, b.desc);
  return hipGetLastError();
}

template <int R>
hipError_t gram_rows_t(const float* A, int64_t n, int lda, double* out, hipStream_t s) {
  const int gpb = (256 / kWave) * Geo<R>::GPW;
  hipLaunchKernelGGL(k_gram_rows<R>, dim3(grid_for(n, gpb * 16)), dim3(256),
                     sizeof(double) * R * R, s, A, n, lda, out);
  return hipGetLastError();
}

template <int R>
hipError_t model_prep_t(const double* VtV, const double* H, double* HtH, double* N3, double* N3p,
                        const PolarParams& pp, hipStream_t s) {
  hipLaunchKernelGGL(k_model_prep<R>, dim3(1), dim3(64), 0, s, VtV, H, HtH, N3, N3p, pp);
  return hipGetLastError();
}

}  // namespace

// One rank's launch geometry and launchers: all that the rank-independent
// code needs of it.  Kernel slots 0..4 of threads/lds are alpha, gamma,
// mode 2 (at the largest hot-column count), projection and Q export.
struct RankOps {
  int max_hot;
  int polar_unit, mode2_unit;
  int threads[5];
  size_t lds[5];
  hipError_t (*plan)(BatchView&);
  hipError_t (*alpha)(const BatchView&, int, const PolarParams&, hipStream_t);
  hipError_t (*gamma)(const BatchView&, int, int, const PolarParams&, hipStream_t);
  hipError_t (*mode2)(const BatchView&, int, hipStream_t);
  hipError_t (*gram)(const BatchView&, int, int, hipStream_t);
  hipError_t (*solve_h)(const BatchView&, const PolarParams&, hipStream_t);
  hipError_t (*vupdate)(const BatchView&, int, hipStream_t);
  hipError_t (*nnls)(const BatchView&, int, hipStream_t);
  hipError_t (*econ_fit)(const BatchView&, int, hipStream_t);
  hipError_t (*solve_n3)(const BatchView&, const PolarParams&, hipStream_t);
  hipError_t (*vscale)(const BatchView&, int, hipStream_t);
  hipError_t (*zero)(const BatchView&, int, hipStream_t);
  hipError_t (*fit)(const BatchView&, hipStream_t);
  hipError_t (*gram_rows)(const float*, int64_t, int, double*, hipStream_t);
  hipError_t (*getq)(const XEnc&, int64_t, int64_t, const float*, const double*, float*, int64_t,
                     const double*, hipStream_t);
  hipError_t (*project)(const XRaw&, int64_t, const float*, const double*, const double*,
                        const double*, int, const float*, float*, float*, double*,
                        const PolarParams&, hipStream_t);
  hipError_t (*model_prep)(const double*, const double*, double*, double*, double*,
                           const PolarParams&, hipStream_t);
};

namespace {

template <int R>
RankOps make_rank_ops() {
  RankOps o{};
  o.max_hot = max_hot_t<R>();
  o.polar_unit = polar_gpb<R>();
  o.mode2_unit = mode2_gpb<R>();
  o.threads[0] = alpha_threads<R>();
  o.threads[1] = gamma_threads<R>();
  o.threads[2] = mode2_threads<R>();
  o.threads[3] = proj_threads<R>();
  o.threads[4] = getq_threads<R>();
  o.lds[0] = alpha_lds<R>();
  o.lds[1] = gamma_lds<R>();
  o.lds[2] = mode2_lds<R>(max_hot_t<R>());
  o.lds[3] = proj_shared<R>() + (size_t)(proj_threads<R>() / kWave) * Geo<R>::GPW * proj_group<R>();
  o.lds[4] = (size_t)(getq_threads<R>() / kWave) * Geo<R>::GPW * getq_group<R>();
  o.plan = plan_t<R>;
  o.alpha = alpha_t<R>;
  o.gamma = gamma_t<R>;
  o.mode2 = mode2_t<R>;
  o.gram = gram_t<R>;
  o.solve_h = solve_h_t<R>;
  o.vupdate = vupdate_t<R>;
  o.nnls = nnls_t<R>;
  o.econ_fit = econ_t<R>;
  o.solve_n3 = solve_n3_t<R>;
  o.vscale = vscale_t<R>;
  o.zero = zero_t<R>;
  o.fit = fit_t<R>;
  o.gram_rows = gram_rows_t<R>;
  o.getq = getq_t<R>;
  o.project = project_t<R>;
  o.model_prep = model_prep_t<R>;
  return o;
}

constexpr bool rank_listed(int r) {
#define P2_OR(x) || r == x
  return false P2_RANKS(P2_OR);
#undef P2_OR
}

}  // namespace

// Each rank's table, defined in the object that p2_ranks.hip compiles for
// the rank's subset.
#define P2_DECLARE_RANK(r) const RankOps* rank_ops_##r();
P2_RANKS(P2_DECLARE_RANK)
#undef P2_DECLARE_RANK

#define P2_DEFINE_RANK(r)                                          \
  P2_CHECK_PLAN(r)                                                 \
  static_assert(rank_listed(r), "R=" #r " is not in P2_RANKS");    \
  const RankOps* rank_ops_##r() {                                  \
    static const RankOps ops = make_rank_ops<r>();                 \
    return &ops;                                                   \
  }

}  // namespace p2
