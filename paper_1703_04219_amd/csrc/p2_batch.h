// Device-visible descriptors of a batch of independent decompositions.
//
// Every per-iteration kernel runs over a batch: an array of ProbDesc (one per
// decomposition, all of the same rank R) and a list of tiles, each tile a
// range of subjects of one problem.  A single decomposition is a batch of one.
#pragma once

#include <stdint.h>

#include "p2_device.h"

namespace p2 {

constexpr int kFitRing = 1024;

// Offsets (in doubles) of the per-problem small FP64 block.
struct SmallLayout {
  int M1, WtW, VtV, VtVraw, HtH, N2p, N3, N3p, inv, fitacc, nx2, fits, losses, total;
};

__host__ __device__ constexpr SmallLayout small_layout(int R) {
  SmallLayout s{};
  const int RR = R * R;
  s.M1 = 0;
  s.WtW = s.M1 + RR;
  s.VtV = s.WtW + RR;
  s.VtVraw = s.VtV + RR;
  s.HtH = s.VtVraw + RR;
  s.N2p = s.HtH + RR;
  s.N3 = s.N2p + RR;
  s.N3p = s.N3 + RR;
  s.inv = s.N3p + RR;
  s.fitacc = s.inv + R;
  s.nx2 = s.fitacc + 2;
  s.fits = s.nx2 + 1;
  s.losses = s.fits + kFitRing;
  s.total = s.losses + kFitRing;
  return s;
}

struct ProbDesc {
  XEnc X;           // re-encoded slices
  int64_t K, J;
  float* V[2];      // V_t / V_{t+1} ping-pong, internal column order, row stride LDV
  float* W;         // K x R
  double* H;        // R x R (the caller's buffer)
  double* F;        // K x R x R, per subject F_k column-major (FP64: F carries the
                    // 1/sigma_min scale of ill-conditioned subjects)
  float* M2;        // J x LDV
  float* M3;        // K x R
  float* E;         // K x NC x R eigenvector bases of G_k (warm start), or nullptr
  double* small;    // small_layout(R)
  int64_t* iter;    // iterations completed (selects the fit ring slot)
  float* part;      // mode-2 hot partial sums: nparts slots of hot * R floats
  int32_t nparts;   // mode-2 tiles of this problem
  int32_t hot;      // mode-2 hot columns of this problem
  const int32_t* order;  // subject at each position of the per-subject passes, or
                         // nullptr for the natural order
  int32_t nonneg;   // 1: V and W (the diagonals of S_k) are updated by NNLS
  const int32_t* econ;  // the subjects with I_k < R (n_econ of them)
  int64_t n_econ;
};

// Subject handled at position pos of a tile.  The order only changes which
// subjects share a wave; every per-subject array stays indexed by subject.
__device__ __forceinline__ int64_t subject_at(const ProbDesc& D, int64_t pos) {
  return D.order != nullptr ? (int64_t)glob(D.order)[pos] : pos;
}

// A range of subjects of one problem.  Tile arrays are padded to a multiple
// of kBins with empty tiles (k0 == k1) and stored bin-interleaved: position t
// belongs to bin t % kBins.  Bins are contiguous, work-balanced runs of the
// (problem, subject)-ordered tile sequence, one per XCD, so that the blocks of
// one XCD keep to few problems and their factor rows stay in that XCD's L2.
struct Tile {
  int32_t p;        // problem
  int32_t slot;     // mode-2 tiles: index of this tile's partial-sum slot within its problem
  int64_t k0, k1;   // subjects [k0, k1)
};

constexpr int kBins = 8;  // XCDs of the device; workgroups are dispatched to them round-robin

// Per-launch ticket counters of the dynamic schedule (kBins each).
enum { kTicketAlpha = 0, kTicketMode2 = 1, kTicketGamma = 2, kTicketKinds = 3 };

}  // namespace p2
