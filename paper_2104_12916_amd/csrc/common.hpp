// Shared declarations of the qpgpu HIP library (gfx950 / CDNA4).
//
// Layout conventions used by every kernel: dense row-major storage, leading
// dimension = stride between rows (in elements).  Lower-triangular operands keep
// explicit zeros above the diagonal; kernels skip those regions by tile.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>

namespace qpg {

constexpr int kWave = 64;

// State of one PCG solve, resident in device memory.  Kernels read alpha/beta/
// rho from here and the host only polls `done` every few steps.
struct PcgScalars {
  double rho;      // r^T z of the current iterate
  double pq;       // p^T q of the current step
  double alpha;
  double beta;
  double rr;       // ||r||_2^2 after the last update
  double bb;       // ||b||_2^2 of the right-hand side
  double tol2;     // stop when rr <= tol2
  double wmax;     // max_i |w_i r_i| after the last update (w = nu)
  double wtol;     // stop when wmax <= wtol (negative: test disabled)
  int iter;        // completed CG steps
  int maxit;
  int done;        // 1 converged, 2 iteration cap, 3 breakdown (p^T q <= 0)
  int pad;
};

// Triangular shape of a matrix operand.
enum Shape : int { kDense = 0, kLower = 1 };

// ---- launch helpers (defined in the .hip files) ---------------------------
struct DevInfo {
  int cu_count = 256;
  int device = 0;
};
DevInfo& dev_info();

// Optional pair of events recorded around the main kernel of a launch (used to
// sample kernel durations during a solve).
struct EventPair {
  hipEvent_t begin;
  hipEvent_t end;
};

// Workspace of the two-pass column sweep: per-chunk partial sums.
template <typename T>
struct GemvWork {
  T* part;
  size_t part_elems;
};

}  // namespace qpg
