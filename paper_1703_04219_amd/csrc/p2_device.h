// Device building blocks of the PARAFAC2-ALS hot path on gfx950 (CDNA4).
//
// Work layout used by every per-subject kernel: a subject is owned by a
// "group" of NC consecutive lanes of one 64-wide wavefront (NC = R rounded up
// to even).  Lane c of the group owns column c of every R x R matrix of that
// subject, so R x R products are R-wide FMA loops per lane, and the Jacobi
// eigen-solver exchanges whole columns between lane pairs with shuffles.
// Several groups share a wavefront (6 at R = 10, 1 at R = 40); all data
// exchange inside a group goes through shuffles or the group's own LDS
// region, so no workgroup barrier is needed inside the subject loop.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace p2 {

constexpr int kWave = 64;

template <int R>
struct Geo {
  static constexpr int NC = (R & 1) ? R + 1 : R;  // lanes per subject group
  static constexpr int GPW = kWave / NC;           // groups per wavefront
  static constexpr int LDV = (R + 3) & ~3;         // padded row stride of V/M2
  // rows of one gather chunk: whole multiples of the group width, about 24
  static constexpr int CH = NC * ((24 + NC - 1) / NC);
};

// Global-memory views of pointers.  Buffers reached through descriptors in
// memory are generic pointers to the compiler, which then emits FLAT
// instructions; a FLAT access counts against the LDS wait counter as well, so
// every LDS wait would also wait for the global loads and atomics in flight.
// Casting to the global address space gives plain global instructions.
#define P2_GLOBAL __attribute__((address_space(1)))

template <class T>
__device__ __forceinline__ P2_GLOBAL T* glob(T* p) {
  return (P2_GLOBAL T*)p;
}

// 16-byte global load (p 16-byte aligned)
typedef float p2_f4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ p2_f4 ldg4(const float* p) {
  return *reinterpret_cast<const P2_GLOBAL p2_f4*>(glob(p));
}

__device__ __forceinline__ void gadd(float* p, float v) {
  __hip_atomic_fetch_add(glob(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void gadd(double* p, double v) {
  __hip_atomic_fetch_add(glob(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Orders LDS traffic between lanes of one wavefront (no workgroup barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Makes v count as computed (and redefined) at this point: the scheduler may
// otherwise sink the arithmetic that produces v past a following barrier, or
// hoist a conversion of v out of a loop, and keep the wider values live.
// Emits no instruction.
__device__ __forceinline__ void settle(double& v) { asm volatile("" : "+v"(v)); }
__device__ __forceinline__ void settle(float& v) { asm volatile("" : "+v"(v)); }

// ---------------------------------------------------------------------------
// Slice access.  XEnc is the re-encoded collection built at init (16-bit
// columns relabelled by frequency, 16-bit row starts relative to the subject),
// XRaw is the caller's plain CSR (used for projection requests).
// ---------------------------------------------------------------------------

struct Subj {
  int64_t z0;  // first nonzero
  int64_t r0;  // first row
  int nrows;
  int nnz;
};

struct XEnc {
  const int64_t* zbase;
  const int64_t* rbase;
  const uint16_t* rstart;
  const uint16_t* col;
  const float* val;
  const uint16_t* nzrow;  // row of each nonzero, relative to its subject
  __device__ __forceinline__ Subj subj(int64_t k) const {
    Subj s;
    s.z0 = glob(zbase)[k];
    s.r0 = glob(rbase)[k];
    s.nrows = (int)(glob(rbase)[k + 1] - s.r0);
    s.nnz = (int)(glob(zbase)[k + 1] - s.z0);
    return s;
  }
  __device__ __forceinline__ void row(const Subj& s, int i, int& zs, int& ze) const {
    zs = glob(rstart)[s.r0 + i];
    ze = (i + 1 < s.nrows) ? (int)glob(rstart)[s.r0 + i + 1] : s.nnz;
  }
  __device__ __forceinline__ int colat(const Subj& s, int z) const { return glob(col)[s.z0 + z]; }
  __device__ __forceinline__ float valat(const Subj& s, int z) const {
    return glob(val)[s.z0 + z];
  }
};

struct XRaw {
  const int64_t* subj_ptr;
  const int64_t* row_ptr;
  const int32_t* col;
  const float* val;
  __device__ __forceinline__ Subj subj(int64_t k) const {
    Subj s;
    s.r0 = glob(subj_ptr)[k];
    s.nrows = (int)(glob(subj_ptr)[k + 1] - s.r0);
    s.z0 = glob(row_ptr)[s.r0];
    s.nnz = (int)(glob(row_ptr)[s.r0 + s.nrows] - s.z0);
    return s;
  }
  __device__ __forceinline__ void row(const Subj& s, int i, int& zs, int& ze) const {
    zs = (int)(glob(row_ptr)[s.r0 + i] - s.z0);
    ze = (int)(glob(row_ptr)[s.r0 + i + 1] - s.z0);
  }
  __device__ __forceinline__ int colat(const Subj& s, int z) const { return glob(col)[s.z0 + z]; }
  __device__ __forceinline__ float valat(const Subj& s, int z) const {
    return glob(val)[s.z0 + z];
  }
};

// ---------------------------------------------------------------------------
// Sparse gather (equation (mttkrp1_3): only the rows of V of the nonzero
// columns of X_k are touched):  A(i,:) = sum_z x_z V(col_z, :) in FP32 for the
// chunk rows [i0, i0 + n) of subject s, written to LDS as T (float or double).
// V rows have stride LDV (16-byte aligned, zero padded).
// ---------------------------------------------------------------------------
template <int R, class XS, class T>
__device__ __forceinline__ void gather_rows(const XS& X, const Subj& s, int i0, int n,
                                            const float* __restrict__ V, T* A, int j) {
  constexpr int NC = Geo<R>::NC;
  constexpr int LDV = Geo<R>::LDV;
#pragma nounroll
  for (int ii = j; ii < n; ii += NC) {
    float acc[LDV];
#pragma unroll
    for (int c = 0; c < LDV; ++c) acc[c] = 0.f;
    int zs, ze;
    X.row(s, i0 + ii, zs, ze);
    for (int z = zs; z < ze; ++z) {
      const int col = X.colat(s, z);
      const float x = X.valat(s, z);
      const float* vr = V + (size_t)col * LDV;
#pragma unroll
      for (int q = 0; q < LDV / 4; ++q) {
        const p2_f4 t = ldg4(vr + 4 * q);
        acc[4 * q + 0] = fmaf(x, t.x, acc[4 * q + 0]);
        acc[4 * q + 1] = fmaf(x, t.y, acc[4 * q + 1]);
        acc[4 * q + 2] = fmaf(x, t.z, acc[4 * q + 2]);
        acc[4 * q + 3] = fmaf(x, t.w, acc[4 * q + 3]);
      }
    }
#pragma unroll
    for (int c = 0; c < R; ++c) A[ii * R + c] = (T)acc[c];
  }
}

// Two gathers of the same rows against two factor matrices (V_t and V_{t+1}),
// stored as FP32 (the gathered values are FP32 sums, so nothing is lost):
// row ii of X_k V0 at A0 + ii * R, row ii of X_k V1 at A1 + ii * LDV (16-byte
// rows for the Gram's vector reads; the padding columns are zero).
template <int R, int T, class XS>
__device__ __forceinline__ void gather_rows2(const XS& X, const Subj& s, int i0, int n,
                                             const float* __restrict__ V0,
                                             const float* __restrict__ V1, float* A0, float* A1,
                                             int j) {
  constexpr int NC = Geo<R>::NC;
  constexpr int LDV = Geo<R>::LDV;
#pragma nounroll
  for (int ib = 0; ib < n; ib += T * NC) {
    // T rows per lane, their nonzeros walked together so that the T load
    // chains (row bounds, column, V rows) are in flight at once
    int zs[T], len[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int ii = ib + j + t * NC;
      int a = 0, b = 0;
      if (ii < n) X.row(s, i0 + ii, a, b);
      zs[t] = a;
      len[t] = b - a;
    }
    float a0[T][LDV], a1[T][LDV];
#pragma unroll
    for (int t = 0; t < T; ++t) {
#pragma unroll
      for (int c = 0; c < LDV; ++c) a0[t][c] = a1[t][c] = 0.f;
    }
    int steps = len[0];
#pragma unroll
    for (int t = 1; t < T; ++t) steps = max(steps, len[t]);
    for (int u = 0; u < steps; ++u) {
#pragma unroll
      for (int t = 0; t < T; ++t) {
        if (u < len[t]) {
          const int col = X.colat(s, zs[t] + u);
          const float x = X.valat(s, zs[t] + u);
          const float* v0 = V0 + (size_t)col * LDV;
          const float* v1 = V1 + (size_t)col * LDV;
#pragma unroll
          for (int q = 0; q < LDV / 4; ++q) {
            const p2_f4 tv = ldg4(v0 + 4 * q);
            const p2_f4 uv = ldg4(v1 + 4 * q);
            a0[t][4 * q + 0] = fmaf(x, tv.x, a0[t][4 * q + 0]);
            a0[t][4 * q + 1] = fmaf(x, tv.y, a0[t][4 * q + 1]);
            a0[t][4 * q + 2] = fmaf(x, tv.z, a0[t][4 * q + 2]);
            a0[t][4 * q + 3] = fmaf(x, tv.w, a0[t][4 * q + 3]);
            a1[t][4 * q + 0] = fmaf(x, uv.x, a1[t][4 * q + 0]);
            a1[t][4 * q + 1] = fmaf(x, uv.y, a1[t][4 * q + 1]);
            a1[t][4 * q + 2] = fmaf(x, uv.z, a1[t][4 * q + 2]);
            a1[t][4 * q + 3] = fmaf(x, uv.w, a1[t][4 * q + 3]);
          }
        }
      }
    }
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int ii = ib + j + t * NC;
      if (ii < n) {
#pragma unroll
        for (int c = 0; c < R; ++c) A0[ii * R + c] = a0[t][c];
#pragma unroll
        for (int c = 0; c < LDV; ++c) A1[ii * LDV + c] = c < R ? a1[t][c] : 0.f;
      }
    }
  }
}

// Gram rows from an LDS chunk: lane c (< R) accumulates row c of A^T B in
// FP64 (products of the FP32 values are exact in FP64).  For even R the rows
// of B are read as 16-byte LDS vectors (rows start 16-byte aligned).
template <int R>
__device__ __forceinline__ void gram_accum(const double* A, const double* B, int n, int c,
                                           double (&row)[R]) {
  const int cc = c < R ? c : 0;
#pragma nounroll
  for (int ii = 0; ii < n; ++ii) {
    const double a = A[ii * R + cc];
    if constexpr (R % 2 == 0) {
      const double2* b = reinterpret_cast<const double2*>(B + ii * R);
#pragma unroll
      for (int l = 0; l < R / 2; ++l) {
        const double2 bb = b[l];
        row[2 * l] = fma(a, bb.x, row[2 * l]);
        row[2 * l + 1] = fma(a, bb.y, row[2 * l + 1]);
      }
    } else {
#pragma unroll
      for (int l = 0; l < R; ++l) row[l] = fma(a, B[ii * R + l], row[l]);
    }
  }
}

// Rows c of A0^T A1 and A1^T A1 together (one read of each A1 row), from the
// FP32 rows gather_rows2 leaves in LDS; products and sums in FP64 (products of
// FP32 values are exact in FP64).  FP32 rows halve the LDS bytes each lane
// reads, which bound this loop when the rows were held as FP64.
template <int R>
__device__ __forceinline__ void gram_accum2(const float* A0, const float* A1, int n, int c,
                                            double (&prow)[R], double (&crow)[R]) {
  constexpr int LDV = Geo<R>::LDV;
  const int cc = c < R ? c : 0;
#pragma nounroll
  for (int ii = 0; ii < n; ++ii) {
    const double a0 = (double)A0[ii * R + cc];
    const double a1 = (double)A1[ii * LDV + cc];
    if constexpr (R % 2 == 0) {
      const float4* b = reinterpret_cast<const float4*>(A1 + ii * LDV);
#pragma unroll
      for (int l = 0; l < LDV / 4; ++l) {
        const float4 bb = b[l];
        const float e[4] = {bb.x, bb.y, bb.z, bb.w};
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (4 * l + u < R) {
            const double be = (double)e[u];
            prow[4 * l + u] = fma(a0, be, prow[4 * l + u]);
            crow[4 * l + u] = fma(a1, be, crow[4 * l + u]);
          }
        }
      }
    } else {
#pragma unroll
      for (int l = 0; l < R; ++l) {
        const double b = (double)A1[ii * LDV + l];
        prow[l] = fma(a0, b, prow[l]);
        crow[l] = fma(a1, b, crow[l]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Cross-lane moves with DPP (no LDS traffic).  quad_perm [1,0,3,2] swaps
// lanes 2t and 2t+1; wave_shl:1 reads lane i+1, wave_shr:1 reads lane i-1.
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const int lo = __double2loint(x);
  const int hi = __double2hiint(x);
  // lanes without a valid source read 0; only in-group partners are used
  const int lo2 = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, true);
  const int hi2 = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi2, lo2);
}
constexpr int kDppSwapPairs = 0xB1;  // quad_perm:[1,0,3,2]
constexpr int kDppFromNext = 0x130;  // wave_shl:1
constexpr int kDppFromPrev = 0x138;  // wave_shr:1

// Value of the Jacobi partner.  Even steps pair lanes (2t, 2t+1); odd steps
// pair (2t+1, 2t+2): an odd lane reads lane+1, an even lane lane-1.  Groups
// start at even lanes, so lane parity equals position parity.
template <bool ODD>
__device__ __forceinline__ double partner_of(double x, bool lane_odd) {
  if constexpr (!ODD) {
    return dpp_f64<kDppSwapPairs>(x);
  } else {
    const double a = dpp_f64<kDppFromNext>(x);
    const double b = dpp_f64<kDppFromPrev>(x);
    return lane_odd ? a : b;
  }
}

// 1/sqrt(x) and 1/x in FP64 from the hardware approximations plus one Newton
// step each.  The rotation parameters only need c^2 + s^2 = 1 to far below
// FP32 precision: an error e per rotation scales a column by 1 + e, and a
// solve makes a few hundred rotations; the refined values are good to about
// the square of the hardware approximation's relative error.
__device__ __forceinline__ double rsq_nr(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  return y * fma(-0.5 * x * y, y, 1.5);
}
__device__ __forceinline__ double rcp_nr(double x) {
  const double y = __builtin_amdgcn_rcp(x);
  return fma(y, fma(-x, y, 1.0), y);
}

// ---------------------------------------------------------------------------
// One-sided (Hestenes) Jacobi on the columns of a matrix, one column per lane.
// On entry lane j of the group holds g = column j (length N) and v = e_j
// (zero columns on the padding lane).  Pairs of positions rotate and then
// swap ("caterpillar" odd-even ordering: positions (2t, 2t+1) on even steps,
// (2t+1, 2t+2) on odd steps; NC steps make every pair meet once).  At
// convergence the columns g_j = (input) v_j are mutually orthogonal and the
// v_j orthonormal: for a symmetric PSD input the v_j are its eigenvectors.
// For a symmetric PSD input the rotations need not be accumulated (ACCUM =
// false): G^2 = sum_j g_j g_j^T with orthogonal g_j, so g_j / ||g_j|| is an
// eigenvector of G with eigenvalue ||g_j||.
// A group stops (no rotation, no swap) after a sweep in which no pair had
// gamma^2 > stop2 * alpha * beta (gamma the pair's inner product, alpha and
// beta its squared norms; stop2 = 1e-10 by default, rotations below 1e-5).
// Jacobi converges quadratically, so the columns are then orthogonal to about
// stop2 relative, far below the FP32 precision of every output.  Stopping per
// group keeps its result independent of the other groups of the wavefront.
// ---------------------------------------------------------------------------
// own2 is this position's squared column norm, carried from step to step
// (updated from the rotation instead of recomputed; the sweep loop recomputes
// it at the start of every sweep).
template <int R, int N, bool ODD, bool ACCUM>
__device__ __forceinline__ void jacobi_step(double (&g)[N], double (&v)[R], double& own2, int j,
                                            bool lane_odd, bool done, double tol2, double stop2,
                                            bool& rot, bool& big) {
  constexpr int NC = Geo<R>::NC;
  // a copy of the partner column saves its second DPP exchange in the
  // rotation; it fits the register budget when no rotations are accumulated
  constexpr bool kKeepPartner = ACCUM ? N <= 20 : N <= 40;
  const int partner = ODD ? (lane_odd ? j + 1 : j - 1) : (j ^ 1);
  const bool act = !done && (!ODD || (j != 0 && j != NC - 1));
  const bool lower = j < partner;
  // the inner product with the partner's column, in two independent chains
  double gam0 = 0.0, gam1 = 0.0;
  double pg[kKeepPartner ? N : 1];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const double p = partner_of<ODD>(g[i], lane_odd);
    if constexpr (kKeepPartner) pg[i] = p;
    if (i & 1)
      gam1 = fma(g[i], p, gam1);
    else
      gam0 = fma(g[i], p, gam0);
  }
  const double gam = gam0 + gam1;
  const double par2 = partner_of<ODD>(own2, lane_odd);
  const double alpha = lower ? own2 : par2;
  const double beta = lower ? par2 : own2;
  // rotation (c, s) zeroing the pair's inner product, t = s / c
  double cs = 1.0, sn = 0.0;
  const double g2 = gam * gam;
  const double ab = alpha * beta;
  if (act && g2 > tol2 * ab) {
    const double d = beta - alpha;
    const double e = 2.0 * gam;
    const double h2 = fma(d, d, e * e);
    const double h = h2 * rsq_nr(h2);
    const double t = copysign(1.0, d) * e * rcp_nr(fabs(d) + h);
    cs = rsq_nr(fma(t, t, 1.0));
    sn = cs * t;
    rot = true;
    if (g2 > stop2 * ab) big = true;
  }
  // rotate and swap: the lower position receives s x + c y, the upper c x - s y;
  // a lane that does not take part keeps its column (coefficients 1, 0)
  const double a_own = act ? (lower ? sn : -sn) : 1.0;
  const double a_par = act ? cs : 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double p;
    if constexpr (kKeepPartner)
      p = pg[i];
    else
      p = partner_of<ODD>(g[i], lane_odd);
    g[i] = fma(a_own, g[i], a_par * p);
  }
  // ||a_own x + a_par y||^2 from the norms and the inner product
  own2 = fma(a_own * a_own, own2, fma(a_par * a_par, par2, 2.0 * a_own * a_par * gam));
  if constexpr (ACCUM) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const double pv = partner_of<ODD>(v[i], lane_odd);
      v[i] = fma(a_own, v[i], a_par * pv);
    }
  }
}

template <int R, int N = R, bool ACCUM = true>
__device__ __forceinline__ void jacobi_onesided(double (&g)[N], double (&v)[R], int j, int gbase,
                                                uint64_t gmask, bool live, double tol,
                                                double stop2, int max_sweeps) {
  constexpr int NC = Geo<R>::NC;
  static_assert(NC % 2 == 0, "groups have an even number of lanes");
  const bool lane_odd = (j & 1) != 0;
  const double tol2 = tol * tol;
  bool done = !live;
#pragma nounroll
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    if (__ballot(!done) == 0ull) break;
    bool rot = false, big = false;
    double own0 = 0.0, own1 = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
      if (i & 1)
        own1 = fma(g[i], g[i], own1);
      else
        own0 = fma(g[i], g[i], own0);
    }
    double own2 = own0 + own1;
#pragma nounroll
    for (int step = 0; step < NC; step += 2) {
      jacobi_step<R, N, false, ACCUM>(g, v, own2, j, lane_odd, done, tol2, stop2, rot, big);
      jacobi_step<R, N, true, ACCUM>(g, v, own2, j, lane_odd, done, tol2, stop2, rot, big);
    }
    (void)rot;
    if ((__ballot(big) & gmask) == 0ull) done = true;
  }
}

// ---------------------------------------------------------------------------
// Diagonally pivoted Cholesky factorisation G = (P L)(P L)^T of the group's
// symmetric positive semi-definite G, in place.  On entry lane c (< R) holds
// G(:, c) in g.  On exit every lane holds one column of P L with rows in the
// original order; the lane chosen as the j-th pivot holds column j.  Once the
// largest remaining Schur-complement diagonal is at or below floor_rel times
// the first pivot, the remaining columns are dropped (set to zero), as are the
// columns of padding lanes (c >= R) and of groups that are not live.
//
// One-sided Jacobi converges in far fewer sweeps on such a factor than on G
// itself: the factor has half of G's dynamic range, and pivoting orders its
// columns by size (the preconditioning of Drmac and Veselic, SIAM J. Matrix
// Anal. Appl. 29, 2008).
//
// The pivot is chosen with one LDS 64-bit atomic max per lane on a key made
// of the diagonal's bits (non-negative doubles order like their bit
// patterns) with the lane index in the low 6 bits.  Lc is R doubles of group
// LDS scratch (the pivot column), key one 64-bit word of group LDS.
// ---------------------------------------------------------------------------
template <int R>
__device__ __forceinline__ void pivoted_cholesky(double (&g)[R], int c, bool live, double* Lc,
                                                 unsigned long long* key, double floor_rel) {
  static_assert(Geo<R>::NC <= 64, "the lane index fits in the key's low 6 bits");
  const bool real = c < R;
  // this lane's current Schur-complement diagonal, G(c, c) to start with
  double d = 0.0;
#pragma unroll
  for (int i = 0; i < R; ++i) d = (i == c) ? g[i] : d;
  bool cand = real && live;  // column not yet factored
  bool stopped = !live;
  double first = 0.0;
  if (c == 0) *key = 0ull;
  wave_sync();
#pragma nounroll
  for (int j = 0; j < R; ++j) {
    if (cand && d > 0.0)
      atomicMax(key, ((unsigned long long)__double_as_longlong(d) & ~63ull) | (unsigned)c);
    wave_sync();
    const unsigned long long k = *key;
    wave_sync();
    if (c == 0) *key = 0ull;
    const int p = (int)(k & 63ull);
    const double best = __longlong_as_double((long long)(k & ~63ull));
    if (j == 0) first = best;
    stopped = stopped || k == 0ull || best <= floor_rel * first;
    const bool piv = !stopped && c == p;
    if (piv) {
      const double rs = 1.0 / sqrt(d);
#pragma unroll
      for (int i = 0; i < R; ++i) {
        g[i] *= rs;
        Lc[i] = g[i];
      }
      cand = false;
    }
    wave_sync();
    if (!stopped && cand) {
      // Schur-complement update of this column with the new factor column
      const double lc = Lc[c];
#pragma unroll
      for (int i = 0; i < R; ++i) g[i] = fma(-lc, Lc[i], g[i]);
      d = fma(-lc, lc, d);
    }
    wave_sync();
  }
  if (cand || !real || !live) {
#pragma unroll
    for (int i = 0; i < R; ++i) g[i] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// Per-subject R x R algebra of the Procrustes step (objective
// (procrustes_obj)) in FP64, column per lane.  With A = X_k V, C = A^T A,
// M = H diag(w), B = A M^T and G = B^T B = M C M^T, the polar factor is
// Q_k = B G^{-1/2} and
//     F    = G^{-1/2} M        (so that Q_k = A F^T)
//     Y V  = Q_k^T A = F C     (the R x R product Y_k V of equation (mttkrp1_3))
// G^{-1/2} is the pseudo-inverse square root: eigenvalues <= tau * lambda_max
// are dropped.  Cs is C (R x R, row-major, symmetric) and w the subject's row
// of W (R doubles), both in the group's LDS; Hs is H (R x R, row-major) in
// the block's LDS.  On exit lane c (< R) holds F(:, c) in f and (Y V)(:, c)
// in y.  S is the group's LDS scratch of NC x R doubles, dl of NC doubles.
//
// With WARM, E is the subject's eigenvector basis of G from its previous
// Procrustes step: NC columns of R floats, column p at E + p R (the identity,
// plus a zero column for odd R, before the first step).  With E the solve is
// warm-started: Jacobi (accumulating its rotations) starts from the columns
// G E, which are already close to orthogonal when G moved little since the
// last iteration.  The accumulated basis is orthonormal to the FP32 rounding
// of the stored E; one Newton-Schulz step V (3I - V^T V) / 2 restores FP64
// orthonormality before it is used and written back, so rounding does not
// build up over iterations.  Without WARM, Jacobi runs on the columns of G's
// pivoted Cholesky factor P L and does not accumulate: the converged columns
// are sigma_p u_p, where u_p are eigenvectors of G with eigenvalues
// lambda_p = sigma_p^2.
// ---------------------------------------------------------------------------
template <int R, bool WARM>
__device__ __forceinline__ void polar_rxr(const double* Cs, const double* w, const double* Hs,
                                          double* S, double* dl, float* __restrict__ E, int c,
                                          int gbase, uint64_t gmask, bool live, double tau,
                                          double tol, double stop2, int max_sweeps,
                                          double (&f)[R], double (&y)[R]) {
  constexpr int NC = Geo<R>::NC;
  const bool real = c < R;
  const int cc = real ? c : 0;
  constexpr bool warm = WARM;
  double g[R], v[R];
#pragma unroll
  for (int i = 0; i < R; ++i) v[i] = warm ? (double)glob(E)[c * R + i] : ((i == c) ? 1.0 : 0.0);
  // T(c, :) = C(c, :) M^T,   T(c, j) = sum_l C(c, l) w(l) H(j, l)
  {
    double cw[R];
#pragma unroll
    for (int l = 0; l < R; ++l) cw[l] = Cs[cc * R + l] * w[l];
#pragma nounroll
    for (int jj = 0; jj < R; ++jj) {
      double t = 0.0;
#pragma unroll
      for (int l = 0; l < R; ++l) t = fma(Hs[jj * R + l], cw[l], t);
      if (real) S[c * R + jj] = t;
    }
  }
  wave_sync();
  // g = G(:, c) = sum_l H(:, l) w(l) T(l, c)
#pragma unroll
  for (int i = 0; i < R; ++i) g[i] = 0.0;
#pragma nounroll
  for (int l = 0; l < R; ++l) {
    const double u = real ? w[l] * S[l * R + cc] : 0.0;
#pragma unroll
    for (int i = 0; i < R; ++i) g[i] = fma(Hs[i * R + l], u, g[i]);
  }
  wave_sync();
  if constexpr (warm) {
    // g = G v, with the columns of G staged in S
    if (real) {
#pragma unroll
      for (int i = 0; i < R; ++i) S[c * R + i] = g[i];
    }
    wave_sync();
#pragma unroll
    for (int i = 0; i < R; ++i) g[i] = 0.0;
#pragma nounroll
    for (int q = 0; q < R; ++q) {
      const double vq = v[q];
#pragma unroll
      for (int i = 0; i < R; ++i) g[i] = fma(S[q * R + i], vq, g[i]);
    }
    wave_sync();
    jacobi_onesided<R, R, true>(g, v, c, gbase, gmask, live, tol, stop2, max_sweeps);
  } else {
    // Jacobi on the columns of G's pivoted Cholesky factor P L: the
    // converged columns are sigma_p u_p with G = sum_p sigma_p^2 u_p u_p^T
    pivoted_cholesky<R>(g, c, live, S, reinterpret_cast<unsigned long long*>(dl), 1e-2 * tau);
    jacobi_onesided<R, R, false>(g, v, c, gbase, gmask, live, tol, stop2, max_sweeps);
  }
  // eigenvalue of G at this position and the group's largest eigenvalue:
  // ||g|| for the warm start's columns G E V, ||g||^2 for the factor's
  double nrm2 = 0.0;
#pragma unroll
  for (int i = 0; i < R; ++i) nrm2 = fma(g[i], g[i], nrm2);
  const double nrm = sqrt(nrm2);
  const double lam = warm ? nrm : nrm2;
  dl[c] = lam;
  wave_sync();
  double lmax = 0.0;
  for (int p = 0; p < NC; ++p) lmax = fmax(lmax, dl[p]);
  wave_sync();
  const bool keep = lam > tau * lmax && lam > 0.0;
  const double d = keep ? 1.0 / sqrt(lam) : 0.0;
  if constexpr (warm) {
    // eigenvectors v, made orthonormal in FP64 and kept for the next step
#pragma unroll
    for (int i = 0; i < R; ++i) S[c * R + i] = v[i];
    wave_sync();
    double acc[R];
#pragma unroll
    for (int i = 0; i < R; ++i) acc[i] = 0.0;
#pragma nounroll
    for (int q = 0; q < NC; ++q) {
      double t = 0.0;
#pragma unroll
      for (int i = 0; i < R; ++i) t = fma(S[q * R + i], v[i], t);
#pragma unroll
      for (int i = 0; i < R; ++i) acc[i] = fma(t, S[q * R + i], acc[i]);
    }
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = fma(1.5, v[i], -0.5 * acc[i]);
    wave_sync();
#pragma unroll
    for (int i = 0; i < R; ++i) {
      glob(E)[c * R + i] = (float)v[i];
      S[c * R + i] = keep ? v[i] : 0.0;
    }
  } else {
    const double inv_nrm = keep ? 1.0 / nrm : 0.0;
#pragma unroll
    for (int i = 0; i < R; ++i) S[c * R + i] = g[i] * inv_nrm;
  }
  dl[c] = d;
  wave_sync();
  // F(:, c) = sum_p d_p u_p (u_p . M(:, c)),   M(:, c) = H(:, c) w(c)
  {
    double m[R];
#pragma unroll
    for (int i = 0; i < R; ++i) m[i] = Hs[i * R + cc] * w[cc];
#pragma unroll
    for (int i = 0; i < R; ++i) f[i] = 0.0;
#pragma nounroll
    for (int p = 0; p < NC; ++p) {
      double z = 0.0;
#pragma unroll
      for (int i = 0; i < R; ++i) z = fma(S[p * R + i], m[i], z);
      z *= dl[p];
#pragma unroll
      for (int i = 0; i < R; ++i) f[i] = fma(z, S[p * R + i], f[i]);
    }
    if (!real) {
#pragma unroll
      for (int i = 0; i < R; ++i) f[i] = 0.0;
    }
  }
  wave_sync();
  // (Y V)(:, c) = sum_l F(:, l) C(l, c)
  if (real) {
#pragma unroll
    for (int i = 0; i < R; ++i) S[c * R + i] = f[i];
  }
  wave_sync();
#pragma unroll
  for (int i = 0; i < R; ++i) y[i] = 0.0;
#pragma nounroll
  for (int l = 0; l < R; ++l) {
    const double cl = Cs[l * R + cc];
#pragma unroll
    for (int i = 0; i < R; ++i) y[i] = fma(S[l * R + i], cl, y[i]);
  }
  if (!real) {
#pragma unroll
    for (int i = 0; i < R; ++i) y[i] = 0.0;
  }
  wave_sync();
}

// ---------------------------------------------------------------------------
// Factored Procrustes step, used where the conditioning of B_k must not be
// squared (projection of new subjects, where a weight passing near zero makes
// B_k nearly singular).  C = A^T A is eigen-decomposed once (factor_c), giving
// C = L L^T with L = E_C diag(s).  Each step then takes the one-sided Jacobi
// SVD of the R x R factor T = L^T M^T (T^T T = G), T V = U Sigma, and
//     Y V = V U^T L^T,     F = V U^T L^{-1}     (Q_k = A F^T),
// so small singular values of B_k enter only through T, never through G.
// ---------------------------------------------------------------------------

// Eigen-decomposition of C (Cs, row-major, group LDS).  Writes row p of Ec =
// eigenvector at position p, sv[p] = sqrt(lambda_p) and isv[p] = 1/sqrt(lambda_p)
// (all three 0 for lambda_p <= tau_c * lambda_max; such rows only ever enter
// multiplied by sv or isv).
template <int R>
__device__ __forceinline__ void factor_c(const double* Cs, double* Ec, double* sv, double* isv,
                                         double* dl, int c, int gbase, uint64_t gmask,
                                         double tau_c, double tol, double stop2, int max_sweeps) {
  constexpr int NC = Geo<R>::NC;
  double g[R], v[R];
#pragma unroll
  for (int i = 0; i < R; ++i) g[i] = (c < R) ? Cs[i * R + c] : 0.0;
  // Jacobi on the columns of C's pivoted Cholesky factor (Ec's first R
  // doubles and dl[0] are scratch until the results are written below): the
  // converged columns are sigma_p u_p, eigenvectors u_p of C with eigenvalues
  // sigma_p^2, found without accumulating the rotations
  pivoted_cholesky<R>(g, c, true, Ec, reinterpret_cast<unsigned long long*>(dl), 1e-2 * tau_c);
  jacobi_onesided<R, R, false>(g, v, c, gbase, gmask, true, tol, stop2, max_sweeps);
  double lam = 0.0;
#pragma unroll
  for (int i = 0; i < R; ++i) lam = fma(g[i], g[i], lam);
  dl[c] = lam;
  wave_sync();
  double lmax = 0.0;
  for (int p = 0; p < NC; ++p) lmax = fmax(lmax, dl[p]);
  wave_sync();
  const bool keep = lam > tau_c * lmax && lam > 0.0;
  const double s = sqrt(lam);
  const double inv_s = keep ? 1.0 / s : 0.0;
#pragma unroll
  for (int i = 0; i < R; ++i) Ec[c * R + i] = g[i] * inv_s;
  sv[c] = keep ? s : 0.0;
  isv[c] = inv_s;
  wave_sync();
}

// One factored Procrustes step.  On exit lane c (< R) holds (Y V)(:, c) in yv
// and, if want_f, row c of F at frs[c * R ..].  S and S2 are group LDS
// scratch of NC x R doubles each, dl of NC doubles.  vbs[c * R ..] (group
// LDS, NC x R doubles) is lane c's column of an orthonormal start basis for
// the right singular vectors (read only when warm; a cold start uses e_c); on
// exit it holds this step's right singular vector at position c, so that a
// following step with a nearby w (warm) starts from T V_prev, whose columns
// are already nearly orthogonal, and needs fewer sweeps.  The basis and F
// live in LDS rather than registers: the R = 40 solve with accumulated
// rotations already fills the register file.
template <int R>
__device__ __forceinline__ void polar_factored(const double* Ec, const double* sv,
                                               const double* isv, const double* w,
                                               const double* Hs, double* S, double* S2,
                                               double* dl, int c, int gbase, uint64_t gmask,
                                               double tau_s, double tol, double stop2,
                                               int max_sweeps, bool want_f, bool warm,
                                               double* vbs, double (&yv)[R], double* frs) {
  constexpr int NC = Geo<R>::NC;
  const bool real = c < R;
  const int cc = real ? c : 0;
  // column c of T:  T(p, c) = s_p  e_p . M(c, :),   M(c, l) = H(c, l) w(l)
  double g[NC], v[R];
  {
    double mrow[R];
#pragma unroll
    for (int l = 0; l < R; ++l) mrow[l] = real ? Hs[cc * R + l] * w[l] : 0.0;
#pragma unroll
    for (int p = 0; p < NC; ++p) {
      double t = 0.0;
#pragma unroll
      for (int l = 0; l < R; ++l) t = fma(Ec[p * R + l], mrow[l], t);
      g[p] = sv[p] * t;
    }
  }
  if (warm) {
    // g = T vb: column i of T (held by lane i) staged in S2[i * NC + p]
    if (real) {
#pragma unroll
      for (int p = 0; p < NC; ++p) S2[c * NC + p] = g[p];
    }
    wave_sync();
#pragma unroll
    for (int p = 0; p < NC; ++p) g[p] = 0.0;
#pragma nounroll
    for (int i = 0; i < R; ++i) {
      const double b = vbs[c * R + i];
#pragma unroll
      for (int p = 0; p < NC; ++p) g[p] = fma(S2[i * NC + p], b, g[p]);
    }
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = vbs[c * R + i];
    wave_sync();
  } else {
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = (i == c) ? 1.0 : 0.0;
  }
  jacobi_onesided<R, NC>(g, v, c, gbase, gmask, true, tol, stop2, max_sweeps);
#pragma unroll
  for (int i = 0; i < R; ++i) vbs[c * R + i] = v[i];
  double sig2 = 0.0;
#pragma unroll
  for (int p = 0; p < NC; ++p) sig2 = fma(g[p], g[p], sig2);
  const double sig = sqrt(sig2);
  dl[c] = sig;
  wave_sync();
  double smax = 0.0;
  for (int p = 0; p < NC; ++p) smax = fmax(smax, dl[p]);
  wave_sync();
  const double inv_sig = (sig > tau_s * smax && sig > 0.0) ? 1.0 / sig : 0.0;
  // y_c = L u_c = sum_p s_p u_c(p) e_p
  {
    double yl[R];
#pragma unroll
    for (int l = 0; l < R; ++l) yl[l] = 0.0;
    for (int p = 0; p < NC; ++p) {
      const double a = sv[p] * g[p] * inv_sig;
#pragma unroll
      for (int l = 0; l < R; ++l) yl[l] = fma(a, Ec[p * R + l], yl[l]);
    }
#pragma unroll
    for (int i = 0; i < R; ++i) {
      S[c * R + i] = v[i];
      S2[c * R + i] = yl[i];
    }
  }
  wave_sync();
  // (Y V)(:, c) = sum_q v_q y_q(c)
#pragma unroll
  for (int i = 0; i < R; ++i) yv[i] = 0.0;
  for (int q = 0; q < NC; ++q) {
    const double yqc = S2[q * R + cc];
#pragma unroll
    for (int i = 0; i < R; ++i) yv[i] = fma(S[q * R + i], yqc, yv[i]);
  }
  if (!real) {
#pragma unroll
    for (int i = 0; i < R; ++i) yv[i] = 0.0;
  }
  wave_sync();
  if (want_f) {
    // z_c = sum_p u_c(p) / s_p e_p;   F(c, :) = sum_q v_q(c) z_q
    double zl[R];
#pragma unroll
    for (int l = 0; l < R; ++l) zl[l] = 0.0;
    for (int p = 0; p < NC; ++p) {
      const double a = isv[p] * g[p] * inv_sig;
#pragma unroll
      for (int l = 0; l < R; ++l) zl[l] = fma(a, Ec[p * R + l], zl[l]);
    }
#pragma unroll
    for (int i = 0; i < R; ++i) S2[c * R + i] = zl[i];
    wave_sync();
    double fr[R];
#pragma unroll
    for (int i = 0; i < R; ++i) fr[i] = 0.0;
    for (int q = 0; q < NC; ++q) {
      const double vqc = S[q * R + cc];
#pragma unroll
      for (int i = 0; i < R; ++i) fr[i] = fma(vqc, S2[q * R + i], fr[i]);
    }
#pragma unroll
    for (int i = 0; i < R; ++i) frs[c * R + i] = fr[i];
    wave_sync();
  }
}

}  // namespace p2
