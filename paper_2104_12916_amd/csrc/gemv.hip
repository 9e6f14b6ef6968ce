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
// Lower-triangular operands (row i holds columns 0..i, zeros above) are read
// only up to the tile containing the diagonal.  Launch shapes come from tune().
#include <cstdlib>
#include <cstring>

#include "kernels.hpp"
#include "gemv_core.hpp"

namespace qpg {

Tune& tune() {
  static Tune t = [] {
    Tune v;
    const char* e = getenv("QPGPU_TUNE");
    if (!e) return v;
    char buf[256];
    strncpy(buf, e, sizeof(buf) - 1);
    buf[sizeof(buf) - 1] = 0;
    for (char* tok = strtok(buf, ","); tok; tok = strtok(nullptr, ",")) {
      char* eq = strchr(tok, '=');
      if (!eq) continue;
      *eq = 0;
      int val = atoi(eq + 1);
      if (!strcmp(tok, "rows_bpc") && val >= 1 && val <= kMaxRowsBpc) v.rows_bpc = val;
      if (!strcmp(tok, "rows_unroll") && (val == 4 || val == 8)) v.rows_unroll = val;
      if (!strcmp(tok, "cols_wide") && (val == 0 || val == 1)) v.cols_wide = val;
      if (!strcmp(tok, "cols_bpc") && val >= 1 && val <= kMaxColsBpc) v.cols_bpc = val;
      if (!strcmp(tok, "cols_unroll") && (val == 4 || val == 8)) v.cols_unroll = val;
      if (!strcmp(tok, "ld_pad") && val >= 0 && val <= 1024 && val % 64 == 0) v.ld_pad = val;
    }
    return v;
  }();
  return t;
}

// ---------------------------------------------------------------------------
// gemv_rows: y_i = alpha * (A x)_i [* sign_i] + beta * y0_i
//   shape kLower: row i uses columns [0, min(i + 1, k)).
//   sign: rows i >= nsplit are negated (applies Sigma = diag(I, -I)).
// TAG only separates launch sites in profiles (same code for every value):
// 0 generic, 1 C^T p, 2 Sigma M u, 3 M^T v (the CG-step operator sweeps),
// 4 X_P r, 5 X_P^T t (the P_H apply).
template <typename T, int TAG, int U>
__global__ void __launch_bounds__(256) gemv_rows_kernel(
    const T* __restrict__ A, int lda, int m, int k, int shape, const T* __restrict__ x,
    T* __restrict__ y, T alpha, T beta, const T* __restrict__ y0, int nsplit, const int* __restrict__ skip) {
  if (skip && *skip) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* xs = reinterpret_cast<T*>(smem_raw);
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int waves = blockDim.x / kWave;
  // rows are dealt round-robin over all waves of the grid, so every block sees
  // rows up to the last one
  const int maxlen = (shape == kLower) ? min(m, k) : k;
  const int lenR_max = round_chunk<T>(maxlen, lda);
  stage_x<T>(xs, x, k, lenR_max);
  for (int i = blockIdx.x * waves + wave; i < m; i += gridDim.x * waves) {
    int len = (shape == kLower) ? min(i + 1, k) : k;
    int lenR = round_chunk<T>(len, lda);
    T v = row_dot<T, U>(A + (size_t)i * lda, xs, lenR, lane);
    if (lane == 0) {
      v *= alpha;
      if (i >= nsplit) v = -v;
      if (y0) v += beta * y0[i];
      y[i] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// gemv_cols first pass.
//   WIDE = 0: the 4 waves of a workgroup split the rows of one 64-lane column
//             tile and are combined through LDS (block width = 1 tile).
//   WIDE = 1: each wave owns its own column tile (block width = 4 tiles) and
//             streams all rows of the chunk; no LDS.
// part[chunk * ps + col] receives the chunk's partial sum of column col.
template <typename T, int TAG, int WIDE, int U>
__global__ void __launch_bounds__(256) gemv_cols_part_kernel(
    const T* __restrict__ A, int lda, int m, int k, int shape, const T* __restrict__ x, T* __restrict__ part,
    int rows_per_chunk, const int* __restrict__ skip) {
  if (skip && *skip) return;
  constexpr int VE = Vec16<T>::n;
  constexpr int CW = kWave * VE;
  constexpr int BW = WIDE ? 4 * CW : CW;
  const int tile = blockIdx.x, chunk = blockIdx.y;
  const size_t ps = (size_t)gridDim.x * BW;
  const int b0 = tile * BW;
  const int first_chunk = (shape == kLower) ? (b0 / rows_per_chunk) : 0;
  if (chunk < first_chunk) return;
  const int r0 = chunk * rows_per_chunk;
  const int r1 = min(m, r0 + rows_per_chunk);
  if (WIDE) {
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int c0 = b0 + wave * CW;
    if (c0 >= k) return;  // this wave's tile lies past the last column (no further barrier)
    T acc[VE];
    cols_wave_partial<T, 8>(A, lda, r0, r1, c0, shape, x, acc);
#pragma unroll
    for (int e = 0; e < VE; ++e) part[(size_t)chunk * ps + c0 + lane * VE + e] = acc[e];
  } else {
    __shared__ T red[4][CW];
    cols_block_partial<T, U>(A, lda, r0, r1, b0, shape, x, red);
    if (threadIdx.x < CW) {
      const int jj = threadIdx.x;
      part[(size_t)chunk * ps + b0 + jj] = (red[0][jj] + red[1][jj]) + (red[2][jj] + red[3][jj]);
    }
  }
}

// Second pass: y_j = alpha * sum over chunks + beta * y0_j.  A 256-thread
// workgroup handles 16 columns; the 16 threads of a column load chunks
// ch = t, t + 16, ... (coalesced across columns) and combine them with a fixed
// butterfly, so the summation order is the same on every run.
constexpr int kRedCols = 16;
template <typename T>
__global__ void __launch_bounds__(256) gemv_cols_reduce_kernel(int k, int ps, int bw, int shape,
                                                               const T* __restrict__ part, int rows_per_chunk,
                                                               int nchunks, T* __restrict__ y, T alpha, T beta,
                                                               const T* __restrict__ y0,
                                                               const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int c = threadIdx.x % kRedCols, t = threadIdx.x / kRedCols;  // column in block, chunk lane
  const int col = blockIdx.x * kRedCols + c;
  T s = 0;
  if (col < k) {
    const int first_chunk = (shape == kLower) ? ((col / bw) * bw / rows_per_chunk) : 0;
    for (int ch = first_chunk + t; ch < nchunks; ch += 256 / kRedCols) s += part[(size_t)ch * ps + col];
  }
  // lanes of one column are kRedCols apart inside the wave (threads t*16 + c):
  // reduce the 4 chunk lanes of this wave, then the 4 waves through LDS
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
// host launchers
template <typename T>
int gemv_rows_grid(int m) {
  int blocks = (m + 3) / 4;
  int cap = dev_info().cu_count * tune().rows_bpc;
  return blocks < cap ? blocks : cap;
}

template <typename T, int TAG>
static void launch_rows_tag(dim3 grid, size_t smem, hipStream_t st, const EventPair* ev, const T* A, int lda, int m,
                            int k, int shape, const T* x, T* y, T alpha, T beta, const T* y0, int nsplit,
                            const int* skip) {
  if (tune().rows_unroll == 8)
    QPG_LAUNCH((gemv_rows_kernel<T, TAG, 8>), grid, dim3(256), (uint32_t)smem, st, ev, A, lda, m, k, shape, x, y,
               alpha, beta, y0, nsplit, skip);
  else
    QPG_LAUNCH((gemv_rows_kernel<T, TAG, 4>), grid, dim3(256), (uint32_t)smem, st, ev, A, lda, m, k, shape, x, y,
               alpha, beta, y0, nsplit, skip);
}

template <typename T>
hipError_t launch_gemv_rows(hipStream_t st, const T* A, int lda, int m, int k, int shape, const T* x, T* y,
                            T alpha, T beta, const T* y0, int nsplit, const int* skip, int tag, const EventPair* ev) {
  if (m <= 0) return hipSuccess;
  constexpr int CH = kWave * Vec16<T>::n;
  int maxlen = (shape == kLower) ? (m < k ? m : k) : k;
  int lenR = (maxlen + CH - 1) / CH * CH;
  if (lenR > lda) lenR = lda;
  size_t smem = (size_t)lenR * sizeof(T);
  if (smem > 150 * 1024) return hipErrorInvalidValue;
  if (nsplit < 0) nsplit = m;
  dim3 grid(gemv_rows_grid<T>(m));
  switch (tag) {
    case 2: launch_rows_tag<T, 2>(grid, smem, st, ev, A, lda, m, k, shape, x, y, alpha, beta, y0, nsplit, skip); break;
    case 4: launch_rows_tag<T, 4>(grid, smem, st, ev, A, lda, m, k, shape, x, y, alpha, beta, y0, nsplit, skip); break;
    default: launch_rows_tag<T, 0>(grid, smem, st, ev, A, lda, m, k, shape, x, y, alpha, beta, y0, nsplit, skip);
  }
  return hipGetLastError();
}

// Column tiling: block width bw (columns), chunks of rows_per_chunk rows.
template <typename T>
void gemv_cols_plan(int m, int k, int& rows_per_chunk, int& nchunks, int& bw) {
  constexpr int CW = kWave * Vec16<T>::n;
  bw = tune().cols_wide ? 4 * CW : CW;
  int tiles = (k + bw - 1) / bw;
  int target = dev_info().cu_count * tune().cols_bpc;
  int nc = target / (tiles > 0 ? tiles : 1);
  int maxc = (m + 15) / 16;
  if (nc > maxc) nc = maxc;
  if (nc < 1) nc = 1;
  int rpc = (m + nc - 1) / nc;
  rpc = (rpc + 15) / 16 * 16;
  if (rpc < 16) rpc = 16;
  rows_per_chunk = rpc;
  nchunks = (m + rpc - 1) / rpc;
}

size_t gemv_cols_part_elems(int max_ld) {
  // chunks <= max(1, target / tiles), so chunks * tiles * bw <= target * bw + tiles * bw
  return (size_t)dev_info().cu_count * kMaxColsBpc * 1024 + (size_t)max_ld + 4096;
}

template <typename T, int TAG>
static void launch_cols_tag(dim3 grid, hipStream_t st, const EventPair* ev, const T* A, int lda, int m, int k,
                            int shape, const T* x, T* part, int rpc, const int* skip) {
  if (tune().cols_wide)
    QPG_LAUNCH((gemv_cols_part_kernel<T, TAG, 1, 8>), grid, dim3(256), 0u, st, ev, A, lda, m, k, shape, x, part, rpc,
               skip);
  else if (tune().cols_unroll == 8)
    QPG_LAUNCH((gemv_cols_part_kernel<T, TAG, 0, 8>), grid, dim3(256), 0u, st, ev, A, lda, m, k, shape, x, part, rpc,
               skip);
  else
    QPG_LAUNCH((gemv_cols_part_kernel<T, TAG, 0, 4>), grid, dim3(256), 0u, st, ev, A, lda, m, k, shape, x, part, rpc,
               skip);
}

template <typename T>
hipError_t launch_gemv_cols(hipStream_t st, const T* A, int lda, int m, int k, int shape, const T* x, T* y,
                            T alpha, T beta, const T* y0, const GemvWork<T>& w, const int* skip, int tag,
                            const EventPair* ev) {
  if (k <= 0) return hipSuccess;
  if (m <= 0) return hipErrorInvalidValue;
  if (shape == kLower && k > m) return hipErrorInvalidValue;  // every column tile must meet a row chunk
  int rpc, nch, bw;
  gemv_cols_plan<T>(m, k, rpc, nch, bw);
  const int tiles = (k + bw - 1) / bw;
  if ((size_t)nch * tiles * bw > w.part_elems) return hipErrorInvalidValue;
  constexpr int CW = kWave * Vec16<T>::n;
  if ((k + CW - 1) / CW * CW > lda) return hipErrorInvalidValue;  // every active 64-lane tile reads inside the row
  dim3 grid(tiles, nch);
  switch (tag) {
    case 1: launch_cols_tag<T, 1>(grid, st, ev, A, lda, m, k, shape, x, w.part, rpc, skip); break;
    case 3: launch_cols_tag<T, 3>(grid, st, ev, A, lda, m, k, shape, x, w.part, rpc, skip); break;
    case 5: launch_cols_tag<T, 5>(grid, st, ev, A, lda, m, k, shape, x, w.part, rpc, skip); break;
    default: launch_cols_tag<T, 0>(grid, st, ev, A, lda, m, k, shape, x, w.part, rpc, skip);
  }
  hipLaunchKernelGGL(gemv_cols_reduce_kernel<T>, dim3((k + kRedCols - 1) / kRedCols), dim3(256), 0, st, k,
                     tiles * bw, bw, shape, w.part, rpc, nch, y, alpha, beta, y0, skip);
  return hipGetLastError();
}

template int gemv_rows_grid<double>(int);
template int gemv_rows_grid<float>(int);
template hipError_t launch_gemv_rows<double>(hipStream_t, const double*, int, int, int, int, const double*, double*,
                                             double, double, const double*, int, const int*, int, const EventPair*);
template hipError_t launch_gemv_rows<float>(hipStream_t, const float*, int, int, int, int, const float*, float*,
                                            float, float, const float*, int, const int*, int, const EventPair*);
template hipError_t launch_gemv_cols<double>(hipStream_t, const double*, int, int, int, int, const double*, double*,
                                             double, double, const double*, const GemvWork<double>&, const int*, int,
                                             const EventPair*);
template hipError_t launch_gemv_cols<float>(hipStream_t, const float*, int, int, int, int, const float*, float*,
                                            float, float, const float*, const GemvWork<float>&, const int*, int,
                                            const EventPair*);
template void gemv_cols_plan<double>(int, int, int&, int&, int&);
template void gemv_cols_plan<float>(int, int, int&, int&, int&);

}  // namespace qpg
