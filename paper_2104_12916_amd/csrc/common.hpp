// Shared declarations of the qpgpu HIP library (gfx950 / CDNA4).
//
// Layout conventions used by every kernel: dense row-major storage, leading
// dimension = stride between rows (in elements).  Lower-triangular operands keep
// explicit zeros above the diagonal; kernels skip those regions by tile.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
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
  int fresh;       // folded-update step (cg_fold): 1 until the first update of a solve
  double rho_next; // folded-update step: r^T z of the current z, the rho of the step's alpha
};

// Triangular shape of a matrix operand.
// kUpper: row i holds columns i..cols-1 (zeros before), read from the aligned chunk containing i.
enum Shape : int { kDense = 0, kLower = 1, kUpper = 2 };

// ---- launch helpers (defined in the .hip files) ---------------------------
struct DevInfo {
  int cu_count = 256;
  int device = 0;
};
DevInfo& dev_info();

// Launch shapes of the streaming sweeps.  Defaults were chosen by timing on
// gfx950 (qp_op_time); per size bucket they come from the autotuner's cache, and
// the environment variable QPGPU_TUNE ("rows_bpc=4,rows_unroll=8,ld_pad=0,...")
// overrides the base entry (tune.hip).
struct Tune {
  int rows_bpc = 4;     // gemv_rows / pcg_q: workgroups per CU (grid cap)
  int rows_unroll = 8;  // 16-byte loads in flight per lane: 4, 8 or 16
  int cols_bpc = 2;     // gemv_cols: target workgroups per CU
  int cols_unroll = 8;  // gemv_cols: rows in flight per wave: 4 or 8
  int ld_pad = 64;      // elements added to every matrix leading dimension (multiple of 64);
                        // breaks the power-of-two row stride of n = 4096 matrices
  int qe_stage = 0;     // explicit operator sweep: 1 stage p in LDS, 0 read it through the caches
  int rows_stage = 0;   // other row sweeps (gemv_rows, q = C w + D p): the same choice for their x
  int brows_stage = 1;  // batched row sweeps (many short rows per QP): stage x in LDS
  int brows_unroll = 4; // batched row sweeps: 16-byte loads in flight per lane
  int op_t = 1;         // keep transposed copies of C and M so every CG-step sweep is a row sweep
                        // (0: column sweeps with per-chunk partials, no extra memory)
  int k0_sym = 1;       // one pass over M for M^T Sigma M u (n small enough for register rows)
  int sym_wg = 2;       // one-pass sweep: workgroups per CU (each writes one partial of w)
  int bsym_wave = 1;    // batched one-pass sweep: 1 lets each wavefront take whole rows when every
                        // QP of the launch has rows of at most 4 x 64 lanes x 16 bytes
  int bsym_units = 16;  // batched one-pass sweep: row units per workgroup (buffer layout: the
                        // pooled partials are sized with it when a QP is admitted)
  int sym_units = 8;    // one-pass sweep: at least this many row units (about n entries
                        // each) per workgroup, so the partials stay small against M (but at
                        // least one workgroup per CU while there are units for it)
  int sym_teams = 2;    // one-pass sweep: teams of 256 threads per workgroup (1 or 2), each
                        // with its own rows and partial; a workgroup writes one partial of w
                        // (fewer partials to write and sum; used when every CU still gets a
                        // workgroup, never in the pipelined form)
  int sym_rows = 4;     // one-pass sweep: rows per block reduction (2 or 4)
  int sym_pipe = 0;     // one-pass sweep: 1 issues the next 2 rows' loads before the current rows'
                        // reduction (rounds of 2 rows; sym_rows is then ignored)
  int upd_threads = 512;  // threads of the single-workgroup PCG update (256, 512 or 1024; 512 measured
                          // 1 us faster per CG step than 1024 at m2 = 2048)
  int mv_rt = 1;         // multi-vector sweeps of the block PCG: rows per thread (1 or 2)
  int cg_fold = 6;       // single-QP implicit CG step with the vector update folded into the
                         // operator sweeps (C^T sweep, sum of the one-pass partials, q sweep, and
                         // for P_H the sum of the X_P apply's partials): bit 0 for P_L and
                         // unpreconditioned solves, bit 1 for P_H.  Two launches fewer per P_H
                         // step, one per P_L step, where the C^T sweep also reduces the previous
                         // step's partials.  Bit 2: the folded C^T sweep takes C^T p_old from the
                         // previous step's u instead of a second dot per row.  Measured whole
                         // solves: few-eq (P_H) 4.86 solves/s with bits 1 and 2, 4.79 with bit 1,
                         // 4.53 unfolded; low-dof (P_L, n = 4096) 67.2 us per CG step with bits 0
                         // and 2 (set in that size bucket of the autotune cache), 68.7 with bit 0,
                         // 69.9 unfolded; small P_L (n = 200) is faster unfolded (23.9 against 22.8
                         // solves/s)
  int ld_nt = 1;        // non-temporal matrix loads: bit 0 single-problem row sweeps (and q = C w + D p),
                        // bit 1 the one-pass sweep; a clear bit uses plain loads.  A CG step streams
                        // more than the 256 MB last-level cache holds; loading M plainly and C, C^T
                        // non-temporally keeps part of M cached from step to step (step time 77 -> 70
                        // us at n = 4096, m1 = 3072, m2 = 2048; the opposite split is equal)
};
Tune& tune();
// Selects the launch shapes of the size bucket of n (n <= 0: the base entry) for
// the enclosing scope on this thread.
class TuneScope {
 public:
  explicit TuneScope(int n);
  ~TuneScope();
  TuneScope(const TuneScope&) = delete;
  TuneScope& operator=(const TuneScope&) = delete;

 private:
  const Tune* prev_;
};
constexpr int kMaxRowsBpc = 8;
constexpr int kMaxColsBpc = 8;
constexpr int kMaxSymWg = 4;

// Optional pair of events recorded around the main kernel of a launch (used to
// sample kernel durations during a solve).
struct EventPair {
  hipEvent_t begin;
  hipEvent_t end;
};

// Launch a kernel; when ev is non-null the runtime stamps the kernel's own
// start and stop times into ev->begin / ev->end (no marker packets around it).
#define QPG_LAUNCH(kernel, grid, block, smem, st, ev, ...)                                              \
  do {                                                                                                   \
    if (ev)                                                                                              \
      hipExtLaunchKernelGGL(kernel, grid, block, smem, st, (ev)->begin, (ev)->end, 0u, __VA_ARGS__);     \
    else                                                                                                 \
      hipLaunchKernelGGL(kernel, grid, block, smem, st, __VA_ARGS__);                                    \
  } while (0)

// Workspace of the two-pass column sweep: per-chunk partial sums.
template <typename T>
struct GemvWork {
  T* part;
  size_t part_elems;
};

}  // namespace qpg
