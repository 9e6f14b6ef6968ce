// Streaming matrix-vector kernels for gfx950: the operator applications of the
// CG step (C^T p, the two triangular sweeps with the inverted K0 factor, C y)
// and the IPM residual products.
//
// Every kernel here is HBM-bound (one FMA per matrix element read), so the
// design goals are: 16-byte coalesced loads along rows, several loads in flight
// per lane, the vector operand staged once per workgroup in LDS, and
// deterministic reductions (fixed summation order, no floating-point atomics).
//
//   gemv_rows : y_i = sum_j A_ij x_j  -- one wavefront per row, x in LDS.
//   gemv_cols : y_j = sum_i A_ij x_i  -- two passes: workgroups own a column
//               tile and a chunk of rows and write per-chunk partial sums; a
//               second small kernel adds them in chunk order.  (A single
//               kernel whose last workgroup reduces needs a device-scope
//               release/acquire pair per workgroup, measured 4-6x slower than
//               the extra launch on gfx950.)
//
// Each sweep exists as a single-problem kernel and as a batched kernel that
// walks a list of descriptors (desc.hpp), one per QP, so one launch streams the
// matrices of many QPs of different sizes.  Both call the same device bodies.
// Lower-triangular operands (row i holds columns 0..i, zeros above) are read
// only up to the tile containing the diagonal.  Launch shapes come from tune().
#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "kernels.hpp"
#include "gemv_core.hpp"
#include "desc.hpp"

namespace qpg {

// ---------------------------------------------------------------------------
// device bodies

// Rows bid, bid + nb, ... (in units of 4 waves) of y = alpha A x (+ beta y0),
// rows >= nsplit negated.  xs: LDS of at least round_chunk(min(m,k) or k) elements.
// skip (nullable): stop flag of the solve, the same for the whole grid; it is
// tested after the first row's loads, so its latency overlaps theirs, and a
// set flag leaves y untouched.
template <typename T, int U>
__device__ __forceinline__ void rows_body(const T* __restrict__ A, int lda, int m, int k, int shape,
                                          const T* __restrict__ x, T* __restrict__ y, T alpha, T beta,
                                          const T* __restrict__ y0, int nsplit, int bid, int nb, T* xs,
                                          const int* __restrict__ skip, int nt = 1) {
  const int sk = skip ? *skip : 0;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int waves = blockDim.x / kWave;
  // rows are dealt round-robin over all waves, so every block sees rows up to the last one
  const int maxlen = (shape == kLower) ? min(m, k) : k;
  const int lenR_max = round_chunk<T>(maxlen, lda);
  if (xs) stage_x<T>(xs, x, k, lenR_max);  // xs null: x is read through the caches
  constexpr int CH = kWave * Vec16<T>::n;
  for (int i = bid * waves + wave; i < m; i += nb * waves) {
    int s0 = 0, len = k;
    if (shape == kLower) len = min(i + 1, k);
    if (shape == kUpper) {
      s0 = min(i, k) / CH * CH;  // aligned start of the chunk holding the diagonal
      len = k - s0;
    }
    const int lenR = round_chunk<T>(len, lda - s0);
    const T* arow = A + (size_t)i * lda + s0;
    T v;
    if (nt)
      v = xs ? row_dot<T, U>(arow, xs + s0, lenR, lane) : row_dot_gx<T, U>(arow, x + s0, lenR, k - s0, lane);
    else
      v = xs ? row_dot<T, U, false>(arow, xs + s0, lenR, lane)
             : row_dot_gx<T, U, false>(arow, x + s0, lenR, k - s0, lane);
    if (sk) return;
    if (lane == 0) {
      v *= alpha;
      if (i >= nsplit) v = -v;
      if (y0) v += beta * y0[i];
      y[i] = v;
    }
  }
}

// First pass of a column sweep for one (tile, chunk) block.
template <typename T, int U>
__device__ __forceinline__ void cols_part_body(const T* __restrict__ A, int lda, int m, int shape,
                                               const T* __restrict__ x, T* __restrict__ part, int rpc, int tile,
                                               int chunk, int ntiles) {
  constexpr int CW = kWave * Vec16<T>::n;
  const size_t ps = (size_t)ntiles * CW;
  const int c0 = tile * CW;
  const int first_chunk = (shape == kLower) ? (c0 / rpc) : 0;
  if (chunk < first_chunk) return;  // whole block above the diagonal (uniform exit, before any barrier)
  const int r0 = chunk * rpc;
  const int r1 = min(m, r0 + rpc);
  __shared__ T red[4][CW];
  cols_block_partial<T, U>(A, lda, r0, r1, c0, shape, x, red);
  if (threadIdx.x < CW) {
    const int jj = threadIdx.x;
    part[(size_t)chunk * ps + c0 + jj] = (red[0][jj] + red[1][jj]) + (red[2][jj] + red[3][jj]);
  }
}

// Second pass: y_j = alpha * sum over chunks + beta * y0_j for the 16 columns
// of group `grp`.  The 16 threads of a column load chunks t, t + 16, ...
// (coalesced across columns) and combine them with a fixed butterfly, so the
// summation order is the same on every run.
constexpr int kRedCols = 16;
template <typename T>
__device__ __forceinline__ void cols_reduce_body(int k, int ps, int shape, const T* __restrict__ part, int rpc,
                                                 int nchunks, T* __restrict__ y, T alpha, T beta,
                                                 const T* __restrict__ y0, int grp) {
  constexpr int CW = kWave * Vec16<T>::n;
  const int c = threadIdx.x % kRedCols, t = threadIdx.x / kRedCols;
  const int col = grp * kRedCols + c;
  T s = 0;
  if (col < k) {
    const int first_chunk = (shape == kLower) ? ((col / CW) * CW / rpc) : 0;
    for (int ch = first_chunk + t; ch < nchunks; ch += 256 / kRedCols) s += part[(size_t)ch * ps + col];
  }
  // lanes of one column are kRedCols apart inside the wave: reduce the wave's
  // 4 chunk lanes, then the 4 waves through LDS
#pragma unroll
  for (int off = 32; off >= kRedCols; off >>= 1) s += __shfl_xor(s, off, kWave);
  __shared__ T sh[4][kRedCols];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  if (lane < kRedCols) sh[wave][lane] = s;
  __syncthreads();
  if (threadIdx.x < kRedCols && col < k) {
    T v = alpha * ((sh[0][c] + sh[1][c]) + (sh[2][c] + sh[3][c]));
    if (y0) v += beta * y0[col];
    y[col] = v;
  }
}

// ---------------------------------------------------------------------------
// single-problem kernels.  TAG only separates launch sites in profiles (same
// code for every value): 0 generic, 1 C^T p, 2 Sigma M u, 3 M^T v (the CG-step
// operator sweeps; 1 and 3 as row sweeps over the stored transposes, or as
// column sweeps), 4 X_P r, 5 X_P^T t (the P_H apply).
template <typename T, int TAG, int U>
__global__ void __launch_bounds__(256) gemv_rows_kernel(
    const T* __restrict__ A, int lda, int m, int k, int shape, const T* __restrict__ x,
    T* __restrict__ y, T alpha, T beta, const T* __restrict__ y0, int nsplit, const int* __restrict__ skip,
    int stage, int nt) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  rows_body<T, U>(A, lda, m, k, shape, x, y, alpha, beta, y0, nsplit, blockIdx.x, gridDim.x,
                  stage ? reinterpret_cast<T*>(smem_raw) : nullptr, skip, nt);
}

template <typename T, int TAG, int U>
__global__ void __launch_bounds__(256) gemv_cols_part_kernel(
    const T* __restrict__ A, int lda, int m, int shape, const T* __restrict__ x, T* __restrict__ part, int rpc,
    const int* __restrict__ skip) {
  if (skip && *skip) return;
  cols_part_body<T, U>(A, lda, m, shape, x, part, rpc, blockIdx.x, blockIdx.y, gridDim.x);
}

template <typename T>
__global__ void __launch_bounds__(256) gemv_cols_reduce_kernel(int k, int ps, int shape, const T* __restrict__ part,
                                                               int rpc, int nchunks, T* __restrict__ y, T alpha,
                                                               T beta, const T* __restrict__ y0,
                                                               const int* __restrict__ skip) {
  if (skip && *skip) return;
  cols_reduce_body<T>(k, ps, shape, part, rpc, nchunks, y, alpha, beta, y0, blockIdx.x);
}

// ---------------------------------------------------------------------------
// batched kernels (one flattened grid over a descriptor list)
template <typename T, int TAG, int U>
__global__ void __launch_bounds__(256) bgemv_rows_kernel(const RowsDesc<T>* __restrict__ descs,
                                                         const int* __restrict__ prefix, int ndesc, int stage) {
  const DescBlock db = desc_of_block(prefix, ndesc, blockIdx.x);
  const RowsDesc<T> d = descs[db.j];
  extern __shared__ __align__(16) unsigned char smem_raw[];
  rows_body<T, U>(d.A, d.lda, d.m, d.k, d.shape, d.x, d.y, d.alpha, d.beta, d.y0, d.nsplit, db.local, d.nblocks,
                  stage ? reinterpret_cast<T*>(smem_raw) : nullptr, d.skip);
}

template <typename T, int TAG, int U>
__global__ void __launch_bounds__(256) bgemv_cols_part_kernel(const ColsDesc<T>* __restrict__ descs,
                                                              const int* __restrict__ prefix, int ndesc) {
  const DescBlock db = desc_of_block(prefix, ndesc, blockIdx.x);
  const ColsDesc<T> d = descs[db.j];
  if (d.skip && *d.skip) return;
  const int local = db.local;
  cols_part_body<T, U>(d.A, d.lda, d.m, d.shape, d.x, d.part, d.rpc, local % d.tiles, local / d.tiles, d.tiles);
}

template <typename T>
__global__ void __launch_bounds__(256) bgemv_cols_reduce_kernel(const ColsDesc<T>* __restrict__ descs,
                                                                const int* __restrict__ prefix, int ndesc) {
  constexpr int CW = kWave * Vec16<T>::n;
  const DescBlock db = desc_of_block(prefix, ndesc, blockIdx.x);
  const ColsDesc<T> d = descs[db.j];
  if (d.skip && *d.skip) return;
  cols_reduce_body<T>(d.k, d.tiles * CW, d.shape, d.part, d.rpc, d.nchunks, d.y, d.alpha, d.beta, d.y0, db.local);
}

// ---------------------------------------------------------------------------
// host launchers
template <typename T>
int gemv_rows_grid(int m) {
  int blocks = (m + 3) / 4;
  int cap = dev_info().cu_count * tune().rows_bpc;
  return blocks < cap ? blocks : cap;
}

template <typename T>
size_t rows_smem_bytes(int m, int k, int shape, int lda) {
  constexpr int CH = kWave * Vec16<T>::n;
  int maxlen = (shape == kLower) ? (m < k ? m : k) : k;
  int lenR = (maxlen + CH - 1) / CH * CH;
  if (lenR > lda) lenR = lda;
  return (size_t)lenR * sizeof(T);
}

template <typename T, int TAG>
static void launch_rows_tag(dim3 grid, size_t smem, hipStream_t st, const EventPair* ev, const T* A, int lda, int m,
                            int k, int shape, const T* x, T* y, T alpha, T beta, const T* y0, int nsplit,
                            const int* skip) {
  const int stage = tune().rows_stage;
  const int nt = tune().ld_nt & 1;
  if (!stage) smem = 0;
  if (tune().rows_unroll == 16)
    QPG_LAUNCH((gemv_rows_kernel<T, TAG, 16>), grid, dim3(256), (uint32_t)smem, st, ev, A, lda, m, k, shape, x, y,
               alpha, beta, y0, nsplit, skip, stage, nt);
  else if (tune().rows_unroll == 8)
    QPG_LAUNCH((gemv_rows_kernel<T, TAG, 8>), grid, dim3(256), (uint32_t)smem, st, ev, A, lda, m, k, shape, x, y,
               alpha, beta, y0, nsplit, skip, stage, nt);
  else
    QPG_LAUNCH((gemv_rows_kernel<T, TAG, 4>), grid, dim3(256), (uint32_t)smem, st, ev, A, lda, m, k, shape, x, y,
               alpha, beta, y0, nsplit, skip, stage, nt);
}

template <typename T>
hipError_t launch_gemv_rows(hipStream_t st, const T* A, int lda, int m, int k, int shape, const T* x, T* y,
                            T alpha, T beta, const T* y0, int nsplit, const int* skip, int tag, const EventPair* ev) {
  if (m <= 0) return hipSuccess;
  size_t smem = rows_smem_bytes<T>(m, k, shape, lda);
  if (smem > 150 * 1024) return hipErrorInvalidValue;
  if (nsplit < 0) nsplit = m;
  dim3 grid(gemv_rows_grid<T>(m));
  switch (tag) {
    case 1: launch_rows_tag<T, 1>(grid, smem, st, ev, A, lda, m, k, shape, x, y, alpha, beta, y0, nsplit, skip); break;
    case 2: launch_rows_tag<T, 2>(grid, smem, st, ev, A, lda, m, k, shape, x, y, alpha, beta, y0, nsplit, skip); break;
    case 3: launch_rows_tag<T, 3>(grid, smem, st, ev, A, lda, m, k, shape, x, y, alpha, beta, y0, nsplit, skip); break;
    case 4: launch_rows_tag<T, 4>(grid, smem, st, ev, A, lda, m, k, shape, x, y, alpha, beta, y0, nsplit, skip); break;
    default: launch_rows_tag<T, 0>(grid, smem, st, ev, A, lda, m, k, shape, x, y, alpha, beta, y0, nsplit, skip);
  }
  return hipGetLastError();
}

// Column tiling: 64-lane tiles of CW columns, chunks of rows_per_chunk rows,
// about target_blocks workgroups over the whole sweep.
template <typename T>
void gemv_cols_plan(int m, int k, int& rows_per_chunk, int& nchunks, int& tiles, int target_blocks) {
  constexpr int CW = kWave * Vec16<T>::n;
  tiles = (k + CW - 1) / CW;
  int nc = target_blocks / (tiles > 0 ? tiles : 1);
  int maxc = (m + 15) / 16;
  if (nc > maxc) nc = maxc;
  if (nc < 1) nc = 1;
  int rpc = (m + nc - 1) / nc;
  rpc = (rpc + 15) / 16 * 16;
  if (rpc < 16) rpc = 16;
  rows_per_chunk = rpc;
  nchunks = (m + rpc - 1) / rpc;
}

// Exact partial-buffer sizes (elements) of one column sweep over an m x k
// operand: in the single-problem launch shape and in the batched shape.
template <typename T>
size_t gemv_cols_need(int m, int k) {
  constexpr int CW = kWave * Vec16<T>::n;
  if (m <= 0 || k <= 0) return 0;
  int rpc, nch, tiles;
  gemv_cols_plan<T>(m, k, rpc, nch, tiles, dev_info().cu_count * tune().cols_bpc);
  return (size_t)nch * tiles * CW;
}

template <typename T>
static int bcols_target(int m, int k) {
  constexpr int CW = kWave * Vec16<T>::n;
  // about 64 rows per chunk: enough work per workgroup without a large reduction
  return ((k + CW - 1) / CW) * ((m + 63) / 64);
}

template <typename T>
size_t bgemv_cols_need(int m, int k) {
  constexpr int CW = kWave * Vec16<T>::n;
  if (m <= 0 || k <= 0) return 0;
  int rpc, nch, tiles;
  gemv_cols_plan<T>(m, k, rpc, nch, tiles, bcols_target<T>(m, k));
  return (size_t)nch * tiles * CW;
}

size_t gemv_cols_part_elems(int max_ld) {
  // chunks <= max(1, target / tiles), so chunks * tiles * CW <= target * CW + tiles * CW
  return (size_t)dev_info().cu_count * kMaxColsBpc * 256 + (size_t)max_ld + 4096;
}

template <typename T, int TAG>
static void launch_cols_tag(dim3 grid, hipStream_t st, const EventPair* ev, const T* A, int lda, int m, int shape,
                            const T* x, T* part, int rpc, const int* skip) {
  if (tune().cols_unroll == 8)
    QPG_LAUNCH((gemv_cols_part_kernel<T, TAG, 8>), grid, dim3(256), 0u, st, ev, A, lda, m, shape, x, part, rpc, skip);
  else
    QPG_LAUNCH((gemv_cols_part_kernel<T, TAG, 4>), grid, dim3(256), 0u, st, ev, A, lda, m, shape, x, part, rpc, skip);
}

template <typename T>
hipError_t launch_gemv_cols(hipStream_t st, const T* A, int lda, int m, int k, int shape, const T* x, T* y,
                            T alpha, T beta, const T* y0, const GemvWork<T>& w, const int* skip, int tag,
                            const EventPair* ev) {
  constexpr int CW = kWave * Vec16<T>::n;
  if (k <= 0) return hipSuccess;
  if (m <= 0) return hipErrorInvalidValue;
  if (shape == kLower && k > m) return hipErrorInvalidValue;  // every column tile must meet a row chunk
  int rpc, nch, tiles;
  gemv_cols_plan<T>(m, k, rpc, nch, tiles, dev_info().cu_count * tune().cols_bpc);
  if ((size_t)nch * tiles * CW > w.part_elems) return hipErrorInvalidValue;
  if (tiles * CW > lda) return hipErrorInvalidValue;  // the last tile reads inside the padded row
  dim3 grid(tiles, nch);
  switch (tag) {
    case 1: launch_cols_tag<T, 1>(grid, st, ev, A, lda, m, shape, x, w.part, rpc, skip); break;
    case 3: launch_cols_tag<T, 3>(grid, st, ev, A, lda, m, shape, x, w.part, rpc, skip); break;
    case 5: launch_cols_tag<T, 5>(grid, st, ev, A, lda, m, shape, x, w.part, rpc, skip); break;
    default: launch_cols_tag<T, 0>(grid, st, ev, A, lda, m, shape, x, w.part, rpc, skip);
  }
  hipLaunchKernelGGL(gemv_cols_reduce_kernel<T>, dim3((k + kRedCols - 1) / kRedCols), dim3(256), 0, st, k,
                     tiles * CW, shape, w.part, rpc, nch, y, alpha, beta, y0, skip);
  return hipGetLastError();
}

// ---- batched launchers ----------------------------------------------------
template <typename T>
void fill_rows_desc(RowsDesc<T>& d, const T* A, int lda, int m, int k, int shape, const T* x, T* y, T alpha, T beta,
                    const T* y0, int nsplit, const int* skip) {
  d.A = A;
  d.lda = lda;
  d.m = m;
  d.k = k;
  d.shape = shape;
  d.x = x;
  d.y = y;
  d.alpha = alpha;
  d.beta = beta;
  d.y0 = y0;
  d.nsplit = nsplit < 0 ? m : nsplit;
  d.skip = skip;
  // a batch has many problems in flight, so each gets about one row per wave
  int blocks = (m + 15) / 16;
  d.nblocks = blocks < 1 ? 1 : blocks;
}

template <typename T>
bool fill_cols_desc(ColsDesc<T>& d, const T* A, int lda, int m, int k, int shape, const T* x, T* y, T alpha, T beta,
                    const T* y0, T* part, size_t part_elems, const int* skip) {
  constexpr int CW = kWave * Vec16<T>::n;
  d.A = A;
  d.lda = lda;
  d.m = m;
  d.k = k;
  d.shape = shape;
  d.x = x;
  d.y = y;
  d.alpha = alpha;
  d.beta = beta;
  d.y0 = y0;
  d.part = part;
  d.skip = skip;
  gemv_cols_plan<T>(m, k, d.rpc, d.nchunks, d.tiles, bcols_target<T>(m, k));
  d.nblocks = d.tiles * d.nchunks;
  d.rblocks = (k + kRedCols - 1) / kRedCols;
  return (size_t)d.nchunks * d.tiles * CW <= part_elems && d.tiles * CW <= lda && !(shape == kLower && k > m);
}

template <typename T, int TAG>
static void launch_brows_tag(dim3 grid, size_t smem, hipStream_t st, const EventPair* ev, const RowsDesc<T>* ddesc,
                             const int* dprefix, int ndesc) {
  const int stage = tune().brows_stage;
  if (!stage) smem = 0;
  if (tune().brows_unroll == 8)
    QPG_LAUNCH((bgemv_rows_kernel<T, TAG, 8>), grid, dim3(256), (uint32_t)smem, st, ev, ddesc, dprefix, ndesc, stage);
  else
    QPG_LAUNCH((bgemv_rows_kernel<T, TAG, 4>), grid, dim3(256), (uint32_t)smem, st, ev, ddesc, dprefix, ndesc, stage);
}

template <typename T>
hipError_t launch_bgemv_rows(hipStream_t st, const RowsDesc<T>* ddesc, const int* dprefix, int ndesc, int total_blocks,
                             size_t smem, int tag, const EventPair* ev) {
  if (ndesc <= 0 || total_blocks <= 0) return hipSuccess;
  if (smem > 150 * 1024) return hipErrorInvalidValue;
  dim3 grid(total_blocks);
  switch (tag) {
    case 1: launch_brows_tag<T, 1>(grid, smem, st, ev, ddesc, dprefix, ndesc); break;
    case 2: launch_brows_tag<T, 2>(grid, smem, st, ev, ddesc, dprefix, ndesc); break;
    case 3: launch_brows_tag<T, 3>(grid, smem, st, ev, ddesc, dprefix, ndesc); break;
    case 4: launch_brows_tag<T, 4>(grid, smem, st, ev, ddesc, dprefix, ndesc); break;
    default: launch_brows_tag<T, 0>(grid, smem, st, ev, ddesc, dprefix, ndesc);
  }
  return hipGetLastError();
}

template <typename T, int TAG>
static void launch_bcols_tag(dim3 grid, hipStream_t st, const EventPair* ev, const ColsDesc<T>* ddesc,
                             const int* dprefix, int ndesc) {
  if (tune().cols_unroll == 8)
    QPG_LAUNCH((bgemv_cols_part_kernel<T, TAG, 8>), grid, dim3(256), 0u, st, ev, ddesc, dprefix, ndesc);
  else
    QPG_LAUNCH((bgemv_cols_part_kernel<T, TAG, 4>), grid, dim3(256), 0u, st, ev, ddesc, dprefix, ndesc);
}

template <typename T>
hipError_t launch_bgemv_cols(hipStream_t st, const ColsDesc<T>* ddesc, const int* dprefix_part, int total_part,
                             const int* dprefix_red, int total_red, int ndesc, int tag, const EventPair* ev) {
  if (ndesc <= 0 || total_part <= 0) return hipSuccess;
  dim3 grid(total_part);
  switch (tag) {
    case 1: launch_bcols_tag<T, 1>(grid, st, ev, ddesc, dprefix_part, ndesc); break;
    case 3: launch_bcols_tag<T, 3>(grid, st, ev, ddesc, dprefix_part, ndesc); break;
    case 5: launch_bcols_tag<T, 5>(grid, st, ev, ddesc, dprefix_part, ndesc); break;
    default: launch_bcols_tag<T, 0>(grid, st, ev, ddesc, dprefix_part, ndesc);
  }
  hipLaunchKernelGGL(bgemv_cols_reduce_kernel<T>, dim3(total_red), dim3(256), 0, st, ddesc, dprefix_red, ndesc);
  return hipGetLastError();
}

// ---- one-pass K0 block product ---------------------------------------------------
// w = M^T Sigma M u with M = L^{-1}[:, :n] (N x n, lower trapezoid: row i holds
// columns 0..min(i, n-1)) and Sigma = diag(I_n, -I_{N-n}) -- the K0^{-1}_{11}
// product of the implicit CG step, K0^{-1} = L^{-T} Sigma L^{-1}.  The step
// needs M u only to form this product, so every row of M is read once: the
// workgroup that owns row i forms v_i = sigma_i (M_i . u) and adds v_i M_i^T to
// its private partial of w.  A second kernel adds the partials in workgroup order.
//
// Rows are dealt in units of about n entries: a pair (i, n-1-i) of the
// triangular part or one row of the rectangular part; workgroup g takes units
// [g U / G, (g+1) U / G).  A team of BT threads spans the columns (thread t
// owns columns c*BT*VE + t*VE .. + VE-1 of every row), so u and the partial stay
// in registers, and R rows share one block reduction.  A workgroup of TM teams
// deals its rows to them in turn, R at a time, and adds the teams' partials in
// team order through LDS before writing its one partial: the same number of
// loads in flight per CU as TM workgroups of one team, with 1/TM of the partials
// to write and to sum.

// Row of local ordinal q in a workgroup's unit range [u0, u1): np pairs first,
// then the middle row of an odd n and the rectangular rows.
__device__ __forceinline__ int sym_row(int q, int u0, int np, int us, int n) {
  if (q < 2 * np) {
    const int uu = u0 + q / 2;
    return (q & 1) ? n - 1 - uu : uu;
  }
  const int uu = us + (q - 2 * np);
  const int tri = (n + 1) / 2;
  return uu < tri ? uu : n + (uu - tri);
}

// Workgroup g of G of one product (TM teams of BT threads).
template <typename T, int BT, int K, int R, bool NT, int TM = 1>
__device__ __forceinline__ void k0_sym_body(const T* __restrict__ M, int ldm, int N, int n, const T* __restrict__ u,
                                            T* __restrict__ part, int ldp, int G, int g,
                                            const int* __restrict__ skip) {
  const int sk = skip ? *skip : 0;  // tested after the first round's loads (uniform over the grid)
  using V = typename Vec16<T>::type;
  constexpr int VE = Vec16<T>::n;
  constexpr int CHB = BT * VE;
  constexpr int NW = BT / kWave;
  const int team = TM > 1 ? (int)threadIdx.x / BT : 0;  // uniform per wavefront
  const int tid = (int)threadIdx.x % BT, wave = tid / kWave, lane = tid % kWave;
  const int P = n / 2, U = (n + 1) / 2 + (N - n);
  const int u0 = (int)((long long)g * U / G), u1 = (int)((long long)(g + 1) * U / G);
  const int np = max(0, min(u1, P) - u0);
  const int us = max(u0, P);
  const int nrows = 2 * np + max(0, u1 - us);
  T xu[K][VE], acc[K][VE];
#pragma unroll
  for (int c = 0; c < K; ++c) {
    const int col = c * CHB + tid * VE;
#pragma unroll
    for (int e = 0; e < VE; ++e) {
      xu[c][e] = (col + e < n) ? u[col + e] : T(0);
      acc[c][e] = T(0);
    }
  }
  __shared__ T sh[2][TM][R][NW];
  int buf = 0;
  for (int qt = 0; qt < nrows; qt += TM * R) {  // the same trip count in every team
    const int q0 = qt + team * R;
    V a[R][K];
    int rowi[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int q = q0 + r;
      int i = -1, len = 0;
      if (q < nrows) {
        i = sym_row(q, u0, np, us, n);
        len = min(i + 1, n);
      }
      rowi[r] = i;
      const T* arow = M + (size_t)(i < 0 ? 0 : i) * ldm;
#pragma unroll
      for (int c = 0; c < K; ++c) {
        const int col = c * CHB + tid * VE;
        if (col < len) {
          a[r][c] = ld16<V, NT>(reinterpret_cast<const V*>(arow + col));
        } else {
#pragma unroll
          for (int e = 0; e < VE; ++e) a[r][c][e] = T(0);
        }
      }
    }
    T d[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      d[r] = T(0);
#pragma unroll
      for (int c = 0; c < K; ++c) d[r] += dot16<V, T>(a[r][c], xu[c]);
    }
    if (sk) return;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const T s = wave_sum<T>(d[r]);
      if (lane == 0) sh[buf][team][r][wave] = s;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      T v = sh[buf][team][r][0];
#pragma unroll
      for (int w2 = 1; w2 < NW; ++w2) v += sh[buf][team][r][w2];
      if (rowi[r] >= n) v = -v;
#pragma unroll
      for (int c = 0; c < K; ++c) {
#pragma unroll
        for (int e = 0; e < VE; ++e) acc[c][e] += a[r][c][e] * v;
      }
    }
    buf ^= 1;  // the next round writes the other buffer: one barrier per round suffices
  }
  if constexpr (TM > 1) {
    // teams 1 .. TM-1 hand their partials to team 0, which adds them in team order
    __shared__ T tp[TM - 1][K][VE][BT];
    if (team > 0) {
#pragma unroll
      for (int c = 0; c < K; ++c)
#pragma unroll
        for (int e = 0; e < VE; ++e) tp[team - 1][c][e][tid] = acc[c][e];
    }
    __syncthreads();
    if (team > 0) return;
#pragma unroll
    for (int t2 = 0; t2 < TM - 1; ++t2)
#pragma unroll
      for (int c = 0; c < K; ++c)
#pragma unroll
        for (int e = 0; e < VE; ++e) acc[c][e] += tp[t2][c][e][tid];
  }
  T* pg = part + (size_t)g * ldp;
#pragma unroll
  for (int c = 0; c < K; ++c) {
    const int col = c * CHB + tid * VE;
#pragma unroll
    for (int e = 0; e < VE; ++e)
      if (col + e < n) pg[col + e] = acc[c][e];
  }
}

// Pipelined form of the same sweep: the loads of the next R rows are issued
// before the current rows' dot, block reduction and accumulation, so the
// workgroup keeps HBM requests in flight across its barriers (two register
// buffers of R rows; R = 2 keeps them within 256 VGPRs at n = 4096).  Same
// rows, same order, same arithmetic as k0_sym_body.
template <typename T, int BT, int K, int R, bool NT>
__device__ __forceinline__ void k0_sym_body_pipe(const T* __restrict__ M, int ldm, int N, int n,
                                                 const T* __restrict__ u, T* __restrict__ part, int ldp, int G,
                                                 int g, const int* __restrict__ skip) {
  if (skip && *skip) return;  // before any matrix load is in flight
  using V = typename Vec16<T>::type;
  constexpr int VE = Vec16<T>::n;
  constexpr int CHB = BT * VE;
  constexpr int NW = BT / kWave;
  const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
  const int P = n / 2, U = (n + 1) / 2 + (N - n);
  const int u0 = (int)((long long)g * U / G), u1 = (int)((long long)(g + 1) * U / G);
  const int np = max(0, min(u1, P) - u0);
  const int us = max(u0, P);
  const int nrows = 2 * np + max(0, u1 - us);
  T xu[K][VE], acc[K][VE];
#pragma unroll
  for (int c = 0; c < K; ++c) {
    const int col = c * CHB + tid * VE;
#pragma unroll
    for (int e = 0; e < VE; ++e) {
      xu[c][e] = (col + e < n) ? u[col + e] : T(0);
      acc[c][e] = T(0);
    }
  }
  __shared__ T sh[2][R][NW];
  int buf = 0;
  // Issue the loads of rows q0 .. q0 + R - 1 into a; lens[r] = entries of row r
  // (0 past the workgroup's range).  Every lane issues every load (a lane past
  // its row's length loads column 0 of a valid row; consume() masks it), so
  // the loads form one unconditional group and the wait before a round's use
  // leaves the next round's group in flight.
  auto issue = [&](int q0, V (&a)[R][K], int (&rowi)[R], int (&lens)[R]) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int q = q0 + r;
      int i = -1, len = 0;
      if (q < nrows) {
        i = sym_row(q, u0, np, us, n);
        len = min(i + 1, n);
      }
      rowi[r] = i;
      lens[r] = len;
      const T* arow = M + (size_t)(i < 0 ? 0 : i) * ldm;
#pragma unroll
      for (int c = 0; c < K; ++c) {
        const int col = c * CHB + tid * VE;
        a[r][c] = ld16<V, NT>(reinterpret_cast<const V*>(arow + (col < len ? col : 0)));
      }
    }
  };
  // consume rows held in a (one block reduction for the R dots, then the rank-one updates)
  auto consume = [&](V (&a)[R][K], const int (&rowi)[R], const int (&lens)[R]) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
      for (int c = 0; c < K; ++c) {
        const bool in = c * CHB + tid * VE < lens[r];
#pragma unroll
        for (int e = 0; e < VE; ++e) a[r][c][e] = in ? a[r][c][e] : T(0);
      }
    }
    T d[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      d[r] = T(0);
#pragma unroll
      for (int c = 0; c < K; ++c) d[r] += dot16<V, T>(a[r][c], xu[c]);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const T s = wave_sum<T>(d[r]);
      if (lane == 0) sh[buf][r][wave] = s;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      T v = sh[buf][r][0];
#pragma unroll
      for (int w2 = 1; w2 < NW; ++w2) v += sh[buf][r][w2];
      if (rowi[r] >= n) v = -v;
#pragma unroll
      for (int c = 0; c < K; ++c) {
#pragma unroll
        for (int e = 0; e < VE; ++e) acc[c][e] += a[r][c][e] * v;
      }
    }
    buf ^= 1;
  };
  V a0[R][K], a1[R][K];
  int r0[R], r1[R], l0[R], l1[R];
  issue(0, a0, r0, l0);
  for (int q0 = 0; q0 < nrows; q0 += 2 * R) {
    issue(q0 + R, a1, r1, l1);  // past the end: masked (one cached line per wave)
    consume(a0, r0, l0);
    if (q0 + R >= nrows) break;
    issue(q0 + 2 * R, a0, r0, l0);
    consume(a1, r1, l1);
  }
  T* pg = part + (size_t)g * ldp;
#pragma unroll
  for (int c = 0; c < K; ++c) {
    const int col = c * CHB + tid * VE;
#pragma unroll
    for (int e = 0; e < VE; ++e)
      if (col + e < n) pg[col + e] = acc[c][e];
  }
}

// Batched one-pass sweep of a QP with short rows (at most 4 x 64 lanes x 16 bytes:
// n <= 512 in float64, 1024 in float32).  There a row spread over the 256 threads
// of a workgroup leaves most lanes idle and every round waits at a barrier for a
// few hundred bytes.  Here each wavefront takes whole rows: lane l
// owns columns c*64*VE + l*VE .. + VE-1 (c < KW) of every row, the row's dot is a
// wavefront sum (no barrier), and a wavefront keeps R rows' loads in flight; the
// workgroup's rows (units [g U / G, (g+1) U / G) as above) are dealt to its four
// wavefronts R at a time in turn.  At the end the four wavefronts' register partials
// are added in wavefront order through LDS into the workgroup's one partial.  A
// stopped QP's workgroups return before any matrix load.  KW is the QP's own
// width, so its arithmetic does not depend on the other QPs of the launch.
template <typename T, int KW, int R, bool NT>
__device__ __forceinline__ void k0_sym_body_wave(const T* __restrict__ M, int ldm, int N, int n,
                                                 const T* __restrict__ u, T* __restrict__ part, int ldp, int G,
                                                 int g, const int* __restrict__ skip) {
  if (skip && *skip) return;
  using V = typename Vec16<T>::type;
  constexpr int VE = Vec16<T>::n;
  constexpr int CW = kWave * VE;
  constexpr int NW = 4;  // wavefronts of the 256-thread workgroup
  const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x / kWave), lane = (int)threadIdx.x % kWave;
  const int P = n / 2, U = (n + 1) / 2 + (N - n);
  const int u0 = (int)((long long)g * U / G), u1 = (int)((long long)(g + 1) * U / G);
  const int np = max(0, min(u1, P) - u0);
  const int us = max(u0, P);
  const int nrows = 2 * np + max(0, u1 - us);
  T xu[KW][VE], acc[KW][VE];
#pragma unroll
  for (int c = 0; c < KW; ++c) {
    const int col = c * CW + lane * VE;
#pragma unroll
    for (int e = 0; e < VE; ++e) {
      xu[c][e] = (col + e < n) ? u[col + e] : T(0);
      acc[c][e] = T(0);
    }
  }
  for (int q0 = wave * R; q0 < nrows; q0 += NW * R) {
    V a[R][KW];
    int rowi[R], lens[R];
    // every lane issues every load (past a row's end it loads column 0 of a valid
    // row and masks the value below), so the R rows' loads are one group
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int q = q0 + r;
      int i = -1, len = 0;
      if (q < nrows) {
        i = sym_row(q, u0, np, us, n);
        len = min(i + 1, n);
      }
      rowi[r] = i;
      lens[r] = len;
      const T* arow = M + (size_t)(i < 0 ? 0 : i) * ldm;
#pragma unroll
      for (int c = 0; c < KW; ++c) {
        const int col = c * CW + lane * VE;
        a[r][c] = ld16<V, NT>(reinterpret_cast<const V*>(arow + (col < len ? col : 0)));
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      T d = T(0);
#pragma unroll
      for (int c = 0; c < KW; ++c) {
        const bool in = c * CW + lane * VE < lens[r];
#pragma unroll
        for (int e = 0; e < VE; ++e) a[r][c][e] = in ? a[r][c][e] : T(0);
        d += dot16<V, T>(a[r][c], xu[c]);
      }
      T v = wave_sum<T>(d);
      if (rowi[r] >= n) v = -v;
#pragma unroll
      for (int c = 0; c < KW; ++c)
#pragma unroll
        for (int e = 0; e < VE; ++e) acc[c][e] += a[r][c][e] * v;
    }
  }
  __shared__ T red[NW - 1][KW][VE][kWave];
  if (wave > 0) {
#pragma unroll
    for (int c = 0; c < KW; ++c)
#pragma unroll
      for (int e = 0; e < VE; ++e) red[wave - 1][c][e][lane] = acc[c][e];
  }
  __syncthreads();
  if (wave > 0) return;
#pragma unroll
  for (int w2 = 0; w2 < NW - 1; ++w2)
#pragma unroll
    for (int c = 0; c < KW; ++c)
#pragma unroll
      for (int e = 0; e < VE; ++e) acc[c][e] += red[w2][c][e][lane];
  T* pg = part + (size_t)g * ldp;
#pragma unroll
  for (int c = 0; c < KW; ++c) {
    const int col = c * CW + lane * VE;
#pragma unroll
    for (int e = 0; e < VE; ++e)
      if (col + e < n) pg[col + e] = acc[c][e];
  }
}

// w_j = sum over g of part[g][j]: 16 columns per workgroup, 16 lanes per column
// take g = t, t + 16, ... with four loads in flight, then a fixed butterfly.
template <typename T, int BT, int K, int R, bool NT, bool PIPE = false, int TM = 1>
__global__ void __launch_bounds__(BT * TM) k0_sym_kernel(const T* __restrict__ M, int ldm, int N, int n,
                                                         const T* __restrict__ u, T* __restrict__ part, int ldp,
                                                         int G, const int* __restrict__ skip) {
  if constexpr (PIPE)
    k0_sym_body_pipe<T, BT, K, R, NT>(M, ldm, N, n, u, part, ldp, G, blockIdx.x, skip);
  else
    k0_sym_body<T, BT, K, R, NT, TM>(M, ldm, N, n, u, part, ldp, G, blockIdx.x, skip);
}

// wave_rows: QPs with short rows take the wavefront-row form (k0_sym_body_wave)
template <typename T, int BT, int K, int R, bool NT, bool PIPE = false>
__global__ void __launch_bounds__(BT) bk0_sym_kernel(const SymDesc<T>* __restrict__ descs,
                                                     const int* __restrict__ prefix, int ndesc, int wave_rows) {
  const DescBlock db = desc_of_block(prefix, ndesc, blockIdx.x);
  const SymDesc<T> d = descs[db.j];
  if (wave_rows) {
    static_assert(BT == 4 * kWave, "the wavefront-row form runs four wavefronts per workgroup");
    constexpr int CW = kWave * Vec16<T>::n;
    const int kc = (d.n + CW - 1) / CW;
    if (kc <= 1) return k0_sym_body_wave<T, 1, 2, NT>(d.M, d.ldm, d.N, d.n, d.u, d.part, d.ldp, d.G, db.local, d.skip);
    if (kc <= 2) return k0_sym_body_wave<T, 2, 2, NT>(d.M, d.ldm, d.N, d.n, d.u, d.part, d.ldp, d.G, db.local, d.skip);
    if (kc <= 4) return k0_sym_body_wave<T, 4, 2, NT>(d.M, d.ldm, d.N, d.n, d.u, d.part, d.ldp, d.G, db.local, d.skip);
  }
  if constexpr (PIPE)
    k0_sym_body_pipe<T, BT, K, R, NT>(d.M, d.ldm, d.N, d.n, d.u, d.part, d.ldp, d.G, db.local, d.skip);
  else
    k0_sym_body<T, BT, K, R, NT>(d.M, d.ldm, d.N, d.n, d.u, d.part, d.ldp, d.G, db.local, d.skip);
}

// Columns grp*16 .. +15 of w = sum over g of part[g].  Thread t adds column
// pair t % 8 of the partials g = t / 8 + 32 j; its 16 loads of a round are in
// flight together (16-byte pairs; rows are 64-element aligned), and the 32 row
// groups are then combined by a fixed butterfly and a fixed sum over the four
// wavefronts, so the order of the additions never depends on timing.
template <typename T>
struct Pair2 {
  typedef T type __attribute__((ext_vector_type(2)));
};

// Returns, in the threads that wrote them (t < 8), the two columns written
// (zeros elsewhere); false when the skip flag was set (nothing written).
template <typename T>
__device__ __forceinline__ bool k0_sym_reduce_body(const T* __restrict__ part, int ldp, int G, int n,
                                                   T* __restrict__ w, const int* __restrict__ skip, int grp,
                                                   typename Pair2<T>::type* out = nullptr) {
  using P2 = typename Pair2<T>::type;
  constexpr int kPairs = kRedCols / 2, kGroups = 256 / kPairs, kInFlight = 16;
  const int sk = skip ? *skip : 0;  // tested once the partial loads are in flight
  const int c = threadIdx.x % kPairs, q = threadIdx.x / kPairs;
  const int col = grp * kRedCols + 2 * c;
  P2 acc[kInFlight];
#pragma unroll
  for (int j = 0; j < kInFlight; ++j) acc[j] = P2{T(0), T(0)};
  if (col < n) {
    const T* base = part + col;
    for (int g0 = q; g0 < G; g0 += kGroups * kInFlight) {
      P2 v[kInFlight];
#pragma unroll
      for (int j = 0; j < kInFlight; ++j) {
        const int g = g0 + kGroups * j;
        v[j] = g < G ? *reinterpret_cast<const P2*>(base + (size_t)g * ldp) : P2{T(0), T(0)};
      }
#pragma unroll
      for (int j = 0; j < kInFlight; ++j) acc[j] += v[j];
    }
  }
  if (sk) return false;
#pragma unroll
  for (int h = kInFlight / 2; h >= 1; h >>= 1)
#pragma unroll
    for (int j = 0; j < h; ++j) acc[j] += acc[j + h];
  P2 s = acc[0];
  // lanes of one column pair are kPairs apart inside the wavefront
#pragma unroll
  for (int off = 32; off >= kPairs; off >>= 1) {
    s.x += __shfl_xor(s.x, off, kWave);
    s.y += __shfl_xor(s.y, off, kWave);
  }
  __shared__ P2 sh[4][kPairs];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  if (lane < kPairs) sh[wave][lane] = s;
  __syncthreads();
  P2 res = P2{T(0), T(0)};
  if (threadIdx.x < kPairs && col < n) {
    const P2 t = (sh[0][c] + sh[1][c]) + (sh[2][c] + sh[3][c]);
    w[col] = t.x;
    res.x = t.x;
    if (col + 1 < n) {
      w[col + 1] = t.y;
      res.y = t.y;
    }
  }
  if (out) *out = res;
  return true;
}

// The sum of the one-pass partials inside the folded CG step, with one more
// per-workgroup partial: the K0 sum adds u^T w over its 16 columns and
// p_new^T D p_new over its share of the m2 entries (p_new = z + beta p_old), so
// the q sweep gets p^T q = u^T w + p^T D p from these partials; the P_H sum adds
// r^T z over its columns.
template <typename T>
__global__ void __launch_bounds__(256) k0_sym_reduce_fold_kernel(const T* __restrict__ part, int ldp, int G, int n,
                                                                 T* __restrict__ w, const PcgScalars* __restrict__ sc,
                                                                 const T* __restrict__ u, const T* __restrict__ z,
                                                                 const T* __restrict__ p,
                                                                 const T* __restrict__ dvec, int m2,
                                                                 double* __restrict__ al) {
  __shared__ double sh[16];
  if (sc->done) return;
  // the vector entries this workgroup's two dot products need are loaded before
  // the partial sums, so their latency hides behind the partials' (loads at
  // indices clamped into the vectors, n, m2 >= 1, masked afterwards: a load under
  // a branch is waited for at the branch's end)
  const T bt = (T)sc->beta;
  const int col = blockIdx.x * kRedCols + 2 * (int)threadIdx.x;
  const bool own = threadIdx.x < kRedCols / 2 && col < n;
  const T ua = u[min(col, n - 1)], ub = u[min(col + 1, n - 1)];
  const T u0 = own ? ua : T(0), u1 = (own && col + 1 < n) ? ub : T(0);
  const int share = (m2 + gridDim.x - 1) / gridDim.x;
  const int j0 = blockIdx.x * share + threadIdx.x, j1 = min(m2, (int)(blockIdx.x + 1) * share);
  double s = 0;
  if (share <= (int)blockDim.x) {  // one entry per thread at most: its loads go first
    const int jc = min(j0, m2 - 1);
    const T zj = z[jc], pj0 = p[jc], dj = dvec[jc];
    typename Pair2<T>::type t;
    k0_sym_reduce_body<T>(part, ldp, G, n, w, nullptr, blockIdx.x, &t);
    if (own) s = (double)u0 * t.x + (double)u1 * t.y;
    if (j0 < j1) {
      const T pj = zj + bt * pj0;
      s += (double)dj * pj * pj;
    }
  } else {
    typename Pair2<T>::type t;
    k0_sym_reduce_body<T>(part, ldp, G, n, w, nullptr, blockIdx.x, &t);
    if (own) s = (double)u0 * t.x + (double)u1 * t.y;
    for (int j = j0; j < j1; j += blockDim.x) {
      const T pj = z[j] + bt * p[j];
      s += (double)dvec[j] * pj * pj;
    }
  }
  s = block_sum<double>(s, sh);
  if (threadIdx.x == 0) al[blockIdx.x] = s;
}

template <typename T>
__global__ void __launch_bounds__(256) ph_reduce_fold_kernel(const T* __restrict__ part, int ldp, int G, int m2,
                                                             T* __restrict__ z, const PcgScalars* __restrict__ sc,
                                                             const T* __restrict__ r, double* __restrict__ rz) {
  __shared__ double sh[16];
  if (sc->done) return;
  // r is loaded before the partial sums
  const int col = blockIdx.x * kRedCols + 2 * (int)threadIdx.x;
  const bool own = threadIdx.x < kRedCols / 2 && col < m2;
  const T r0 = r[min(col, m2 - 1)], r1 = r[min(col + 1, m2 - 1)];  // clamped, used only where own
  typename Pair2<T>::type t;
  k0_sym_reduce_body<T>(part, ldp, G, m2, z, nullptr, blockIdx.x, &t);
  double s = 0;
  if (own) {
    s = (double)r0 * t.x;
    if (col + 1 < m2) s += (double)r1 * t.y;
  }
  s = block_sum<double>(s, sh);
  if (threadIdx.x == 0) rz[blockIdx.x] = s;
}

template <typename T>
__global__ void __launch_bounds__(256) k0_sym_reduce_kernel(const T* __restrict__ part, int ldp, int G, int n,
                                                            T* __restrict__ w, const int* __restrict__ skip) {
  k0_sym_reduce_body<T>(part, ldp, G, n, w, skip, blockIdx.x);
}

template <typename T>
__global__ void __launch_bounds__(256) bk0_sym_reduce_kernel(const SymDesc<T>* __restrict__ descs,
                                                             const int* __restrict__ prefix, int ndesc) {
  const DescBlock db = desc_of_block(prefix, ndesc, blockIdx.x);
  const SymDesc<T> d = descs[db.j];
  k0_sym_reduce_body<T>(d.part, d.ldp, d.G, d.n, d.w, d.skip, db.local);
}

constexpr int kSymBT = 256;  // threads of one team of the one-pass sweep (512 spanning the columns measured slower)
int k0_sym_ldp(int n) { return (n + 63) / 64 * 64; }

template <typename T>
int k0_sym_max_n() {
  return 8 * kSymBT * Vec16<T>::n;
}

// Teams of the one-pass sweep's workgroups and their number.  Teams are counted
// as workgroups were: at least sym_units row units per team, but never fewer
// teams than CUs while there are units for them (small problems are
// latency-bound), at most sym_wg per CU.  They are grouped sym_teams to a
// workgroup when that still leaves every CU a workgroup (not in the pipelined form).
template <typename T>
static void k0_sym_shape(int N, int n, int& G, int& TM) {
  const int U = (n + 1) / 2 + (N - n);
  const int cus = dev_info().cu_count;
  const int cap = cus * tune().sym_wg;
  const int su = tune().sym_units;
  const int teams = std::max(1, std::min(std::max((U + su - 1) / su, std::min(U, cus)), cap));
  TM = tune().sym_pipe ? 1 : tune().sym_teams;
  if (TM > 1 && teams < cus * TM) TM = 1;
  G = (teams + TM - 1) / TM;
}

template <typename T>
int k0_sym_grid(int N, int n) {
  int G, TM;
  k0_sym_shape<T>(N, n, G, TM);
  return G;
}

size_t k0_sym_part_elems(int n) { return (size_t)dev_info().cu_count * kMaxSymWg * k0_sym_ldp(n); }

template <typename T, int BT, int R, bool NT, bool PIPE = false, int TM = 1>
static void launch_sym_r(int K, dim3 grid, hipStream_t st, const EventPair* ev, const T* M, int ldm, int N, int n,
                         const T* u, T* part, int ldp, int G, const int* skip) {
  const dim3 blk(BT * TM);
  switch (K) {
    case 1: QPG_LAUNCH((k0_sym_kernel<T, BT, 1, R, NT, PIPE, TM>), grid, blk, 0u, st, ev, M, ldm, N, n, u, part, ldp, G, skip); break;
    case 2: QPG_LAUNCH((k0_sym_kernel<T, BT, 2, R, NT, PIPE, TM>), grid, blk, 0u, st, ev, M, ldm, N, n, u, part, ldp, G, skip); break;
    case 4: QPG_LAUNCH((k0_sym_kernel<T, BT, 4, R, NT, PIPE, TM>), grid, blk, 0u, st, ev, M, ldm, N, n, u, part, ldp, G, skip); break;
    default: QPG_LAUNCH((k0_sym_kernel<T, BT, 8, R, NT, PIPE, TM>), grid, blk, 0u, st, ev, M, ldm, N, n, u, part, ldp, G, skip);
  }
}

template <typename T>
hipError_t launch_k0_sym_sweep(hipStream_t st, const T* M, int ldm, int N, int n, const T* u, T* part,
                               size_t part_elems, const int* skip, const EventPair* ev) {
  constexpr int VE = Vec16<T>::n;
  if (n <= 0) return hipSuccess;
  if (N < n || n > k0_sym_max_n<T>() || ldm < N || ldm % 64 != 0) return hipErrorInvalidValue;
  int G, TM;
  k0_sym_shape<T>(N, n, G, TM);
  const int ldp = k0_sym_ldp(n);
  if ((size_t)G * ldp > part_elems) return hipErrorInvalidValue;
  const int K = k0_sym_width<T>(n);
  const dim3 grid(G);
  const bool nt = tune().ld_nt & 2;
  if (TM == 2) {  // two teams per workgroup (rounds of sym_rows rows)
    if (tune().sym_rows == 2) {
      if (nt)
        launch_sym_r<T, kSymBT, 2, true, false, 2>(K, grid, st, ev, M, ldm, N, n, u, part, ldp, G, skip);
      else
        launch_sym_r<T, kSymBT, 2, false, false, 2>(K, grid, st, ev, M, ldm, N, n, u, part, ldp, G, skip);
    } else {
      if (nt)
        launch_sym_r<T, kSymBT, 4, true, false, 2>(K, grid, st, ev, M, ldm, N, n, u, part, ldp, G, skip);
      else
        launch_sym_r<T, kSymBT, 4, false, false, 2>(K, grid, st, ev, M, ldm, N, n, u, part, ldp, G, skip);
    }
  } else if (tune().sym_pipe) {  // pipelined rounds of 2 rows
    if (nt)
      launch_sym_r<T, kSymBT, 2, true, true>(K, grid, st, ev, M, ldm, N, n, u, part, ldp, G, skip);
    else
      launch_sym_r<T, kSymBT, 2, false, true>(K, grid, st, ev, M, ldm, N, n, u, part, ldp, G, skip);
  } else if (tune().sym_rows == 2) {
    if (nt)
      launch_sym_r<T, kSymBT, 2, true>(K, grid, st, ev, M, ldm, N, n, u, part, ldp, G, skip);
    else
      launch_sym_r<T, kSymBT, 2, false>(K, grid, st, ev, M, ldm, N, n, u, part, ldp, G, skip);
  } else {
    if (nt)
      launch_sym_r<T, kSymBT, 4, true>(K, grid, st, ev, M, ldm, N, n, u, part, ldp, G, skip);
    else
      launch_sym_r<T, kSymBT, 4, false>(K, grid, st, ev, M, ldm, N, n, u, part, ldp, G, skip);
  }
  return hipGetLastError();
}

// Batched forms: each QP gets about one workgroup per bsym_units row units (many
// QPs share the launch), which keeps its partials near 1/bsym_units of M.
template <typename T>
int bk0_sym_grid(int N, int n) {
  const int U = (n + 1) / 2 + (N - n);
  const int su = tune().bsym_units;
  return std::max(1, (U + su - 1) / su);
}

template <typename T>
int k0_sym_width(int n) {
  constexpr int CHB = kSymBT * Vec16<T>::n;
  const int kc = (n + CHB - 1) / CHB;
  return kc <= 1 ? 1 : kc <= 2 ? 2 : kc <= 4 ? 4 : 8;
}

template <typename T>
bool fill_sym_desc(SymDesc<T>& d, const T* M, int ldm, int N, int n, const T* u, T* w, T* part, size_t part_elems,
                   const int* skip) {
  d.M = M;
  d.ldm = ldm;
  d.N = N;
  d.n = n;
  d.u = u;
  d.w = w;
  d.part = part;
  d.ldp = k0_sym_ldp(n);
  d.G = bk0_sym_grid<T>(N, n);
  d.skip = skip;
  d.rblocks = (n + kRedCols - 1) / kRedCols;
  return n > 0 && N >= n && n <= k0_sym_max_n<T>() && ldm >= N && ldm % 64 == 0 &&
         (size_t)d.G * d.ldp <= part_elems;
}

template <typename T, int R, bool NT, bool PIPE = false>
static void launch_bsym_r(int K, dim3 grid, hipStream_t st, const EventPair* ev, const SymDesc<T>* d,
                          const int* prefix, int ndesc) {
  const dim3 blk(kSymBT);
  const int wv = tune().bsym_wave;
  switch (K) {
    case 1: QPG_LAUNCH((bk0_sym_kernel<T, kSymBT, 1, R, NT, PIPE>), grid, blk, 0u, st, ev, d, prefix, ndesc, wv); break;
    case 2: QPG_LAUNCH((bk0_sym_kernel<T, kSymBT, 2, R, NT, PIPE>), grid, blk, 0u, st, ev, d, prefix, ndesc, wv); break;
    case 4: QPG_LAUNCH((bk0_sym_kernel<T, kSymBT, 4, R, NT, PIPE>), grid, blk, 0u, st, ev, d, prefix, ndesc, wv); break;
    default: QPG_LAUNCH((bk0_sym_kernel<T, kSymBT, 8, R, NT, PIPE>), grid, blk, 0u, st, ev, d, prefix, ndesc, wv);
  }
}

template <typename T>
hipError_t launch_bk0_sym(hipStream_t st, const SymDesc<T>* d, const int* prefix_sweep, int total_sweep,
                          const int* prefix_red, int total_red, int ndesc, int K, const EventPair* ev_sweep,
                          const EventPair* ev_red) {
  if (ndesc <= 0 || total_sweep <= 0) return hipSuccess;
  if (K != 1 && K != 2 && K != 4 && K != 8) return hipErrorInvalidValue;
  const dim3 grid(total_sweep);
  if (tune().sym_pipe) {
    if (tune().ld_nt & 2) launch_bsym_r<T, 2, true, true>(K, grid, st, ev_sweep, d, prefix_sweep, ndesc);
    else launch_bsym_r<T, 2, false, true>(K, grid, st, ev_sweep, d, prefix_sweep, ndesc);
  } else if (tune().ld_nt & 2) {
    if (tune().sym_rows == 2) launch_bsym_r<T, 2, true>(K, grid, st, ev_sweep, d, prefix_sweep, ndesc);
    else launch_bsym_r<T, 4, true>(K, grid, st, ev_sweep, d, prefix_sweep, ndesc);
  } else {
    if (tune().sym_rows == 2) launch_bsym_r<T, 2, false>(K, grid, st, ev_sweep, d, prefix_sweep, ndesc);
    else launch_bsym_r<T, 4, false>(K, grid, st, ev_sweep, d, prefix_sweep, ndesc);
  }
  QPG_LAUNCH(bk0_sym_reduce_kernel<T>, dim3(total_red), dim3(256), 0u, st, ev_red, d, prefix_red, ndesc);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_k0_sym_reduce(hipStream_t st, int N, int n, const T* part, T* w, const int* skip,
                                const EventPair* ev) {
  if (n <= 0) return hipSuccess;
  const int G = k0_sym_grid<T>(N, n), ldp = k0_sym_ldp(n);
  QPG_LAUNCH(k0_sym_reduce_kernel<T>, dim3((n + kRedCols - 1) / kRedCols), dim3(256), 0u, st, ev, part, ldp, G, n,
             w, skip);
  return hipGetLastError();
}

int k0_sym_reduce_grid(int n) { return (n + kRedCols - 1) / kRedCols; }

template <typename T>
hipError_t launch_k0_sym_reduce_fold(hipStream_t st, int N, int n, const T* part, T* w, const PcgScalars* sc,
                                     const T* u, const T* z, const T* p, const T* dvec, int m2, double* al, int nal,
                                     const EventPair* ev) {
  if (n <= 0) return hipSuccess;
  const int grid = k0_sym_reduce_grid(n);
  if (grid > nal) return hipErrorInvalidValue;
  QPG_LAUNCH(k0_sym_reduce_fold_kernel<T>, dim3(grid), dim3(256), 0u, st, ev, part, k0_sym_ldp(n),
             k0_sym_grid<T>(N, n), n, w, sc, u, z, p, dvec, m2, al);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ph_reduce_fold(hipStream_t st, int m2, const T* part, T* z, const PcgScalars* sc, const T* r,
                                 double* rz, int nrz, const EventPair* ev) {
  if (m2 <= 0) return hipSuccess;
  const int grid = k0_sym_reduce_grid(m2);
  if (grid > nrz) return hipErrorInvalidValue;
  QPG_LAUNCH(ph_reduce_fold_kernel<T>, dim3(grid), dim3(256), 0u, st, ev, part, k0_sym_ldp(m2),
             k0_sym_grid<T>(m2, m2), m2, z, sc, r, rz);
  return hipGetLastError();
}

// ---- transposes ---------------------------------------------------------------
// dst = src^T (src rows x cols, row-major), optionally rounded to float32;
// 32 x 32 tiles through LDS so both sides are coalesced.
__device__ __forceinline__ void transpose_body(const double* __restrict__ src, int lds, int rows, int cols,
                                               void* __restrict__ dst, int ldd, int to_float, int bx, int by) {
  __shared__ double tile[32][33];
  const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;  // 32 x 8 threads
  const int c0 = bx * 32, r0 = by * 32;
  for (int r = ty; r < 32; r += 8) {
    const int i = r0 + r, j = c0 + tx;
    tile[r][tx] = (i < rows && j < cols) ? src[(size_t)i * lds + j] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int j = c0 + r, i = r0 + tx;
    if (j < cols && i < rows) {
      const double v = tile[tx][r];
      if (to_float)
        static_cast<float*>(dst)[(size_t)j * ldd + i] = (float)v;
      else
        static_cast<double*>(dst)[(size_t)j * ldd + i] = v;
    }
  }
}

__global__ void __launch_bounds__(256) transpose_kernel(const double* __restrict__ src, int lds, int rows, int cols,
                                                        void* __restrict__ dst, int ldd, int to_float) {
  transpose_body(src, lds, rows, cols, dst, ldd, to_float, blockIdx.x, blockIdx.y);
}

__global__ void __launch_bounds__(256) btranspose_kernel(const TransDesc* __restrict__ descs) {
  const TransDesc t = descs[blockIdx.z];
  if ((int)blockIdx.x * 32 >= t.cols || (int)blockIdx.y * 32 >= t.rows) return;
  transpose_body(t.src, t.lds, t.rows, t.cols, t.dst, t.ldd, t.to_float, blockIdx.x, blockIdx.y);
}

hipError_t transpose_2d(hipStream_t st, const double* src, int lds, int rows, int cols, void* dst, int ldd,
                        int to_float) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  if ((rows + 31) / 32 > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(transpose_kernel, dim3((cols + 31) / 32, (rows + 31) / 32), dim3(256), 0, st, src, lds, rows,
                     cols, dst, ldd, to_float);
  return hipGetLastError();
}

hipError_t btranspose_2d(hipStream_t st, const TransDesc* d, int count, int max_rows, int max_cols) {
  if (count <= 0 || max_rows <= 0 || max_cols <= 0) return hipSuccess;
  if ((max_rows + 31) / 32 > 65535 || count > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(btranspose_kernel, dim3((max_cols + 31) / 32, (max_rows + 31) / 32, count), dim3(256), 0, st, d);
  return hipGetLastError();
}

#define QPG_GEMV_INST(T)                                                                                          \
  template int gemv_rows_grid<T>(int);                                                                            \
  template size_t rows_smem_bytes<T>(int, int, int, int);                                                         \
  template hipError_t launch_gemv_rows<T>(hipStream_t, const T*, int, int, int, int, const T*, T*, T, T,          \
                                          const T*, int, const int*, int, const EventPair*);                     \
  template hipError_t launch_gemv_cols<T>(hipStream_t, const T*, int, int, int, int, const T*, T*, T, T,          \
                                          const T*, const GemvWork<T>&, const int*, int, const EventPair*);      \
  template void gemv_cols_plan<T>(int, int, int&, int&, int&, int);                                               \
  template size_t gemv_cols_need<T>(int, int);                                                                    \
  template size_t bgemv_cols_need<T>(int, int);                                                                   \
  template void fill_rows_desc<T>(RowsDesc<T>&, const T*, int, int, int, int, const T*, T*, T, T, const T*, int,  \
                                  const int*);                                                                    \
  template bool fill_cols_desc<T>(ColsDesc<T>&, const T*, int, int, int, int, const T*, T*, T, T, const T*, T*,  \
                                  size_t, const int*);                                                            \
  template hipError_t launch_bgemv_rows<T>(hipStream_t, const RowsDesc<T>*, const int*, int, int, size_t, int,    \
                                           const EventPair*);                                                     \
  template hipError_t launch_bgemv_cols<T>(hipStream_t, const ColsDesc<T>*, const int*, int, const int*, int,     \
                                           int, int, const EventPair*);                                           \
  template int k0_sym_max_n<T>();                                                                                 \
  template int k0_sym_grid<T>(int, int);                                                                          \
  template hipError_t launch_k0_sym_sweep<T>(hipStream_t, const T*, int, int, int, const T*, T*, size_t,          \
                                             const int*, const EventPair*);                                      \
  template hipError_t launch_k0_sym_reduce<T>(hipStream_t, int, int, const T*, T*, const int*, const EventPair*);  \
  template hipError_t launch_k0_sym_reduce_fold<T>(hipStream_t, int, int, const T*, T*, const PcgScalars*,       \
                                                   const T*, const T*, const T*, const T*, int, double*, int,    \
                                                   const EventPair*);                                             \
  template hipError_t launch_ph_reduce_fold<T>(hipStream_t, int, const T*, T*, const PcgScalars*, const T*,       \
                                               double*, int, const EventPair*);                                   \
  template int bk0_sym_grid<T>(int, int);                                                                         \
  template int k0_sym_width<T>(int);                                                                              \
  template bool fill_sym_desc<T>(SymDesc<T>&, const T*, int, int, int, const T*, T*, T*, size_t, const int*);     \
  template hipError_t launch_bk0_sym<T>(hipStream_t, const SymDesc<T>*, const int*, int, const int*, int, int,    \
                                        int, const EventPair*, const EventPair*);
QPG_GEMV_INST(double)
QPG_GEMV_INST(float)

}  // namespace qpg
