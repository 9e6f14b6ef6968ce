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
//   gemv_cols : y_j = sum_i A_ij x_i  -- a workgroup owns a column tile and a
//               chunk of rows and writes per-chunk partial sums; a second small
//               kernel adds them in chunk order.
//
// Lower-triangular operands (row i holds columns 0..i, zeros above) are read
// only up to the tile containing the diagonal.
#include "kernels.hpp"
#include "gemv_core.hpp"

namespace qpg {

// ---------------------------------------------------------------------------
// gemv_rows: y_i = alpha * (A x)_i [* sign_i] + beta * y0_i
//   shape kLower: row i uses columns [0, min(i + 1, k)).
//   sign: rows i >= nsplit are negated (applies Sigma = diag(I, -I)).
// TAG only separates launch sites in profiles (same code for every value):
// 0 generic, 1 C^T p, 2 Sigma M u, 3 M^T v (the CG-step operator sweeps),
// 4 X_P r, 5 X_P^T t (the P_H apply).
template <typename T, int TAG>
__global__ void __launch_bounds__(256) gemv_rows_kernel(
    const T* __restrict__ A, int lda, int m, int k, int shape, const T* __restrict__ x,
    T* __restrict__ y, T alpha, T beta, const T* __restrict__ y0, int nsplit, const int* __restrict__ skip) {
  if (skip && *skip) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* xs = reinterpret_cast<T*>(smem_raw);
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int waves = blockDim.x / kWave;
  // rows handled by this block: r = blockIdx.x*waves + wave + t*gridDim.x*waves
  int maxlen = k;
  if (shape == kLower) {
    int last_row = m - 1;  // rows are interleaved, so the block sees up to the last row
    maxlen = min(last_row + 1, k);
  }
  const int lenR_max = round_chunk<T>(maxlen, lda);
  stage_x<T>(xs, x, k, lenR_max);
  for (int i = blockIdx.x * waves + wave; i < m; i += gridDim.x * waves) {
    int len = (shape == kLower) ? min(i + 1, k) : k;
    int lenR = round_chunk<T>(len, lda);
    T v = row_dot<T>(A + (size_t)i * lda, xs, lenR, lane);
    if (lane == 0) {
      v *= alpha;
      if (i >= nsplit) v = -v;
      if (y0) v += beta * y0[i];
      y[i] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// gemv_cols: y_j = alpha * (A^T x)_j + beta * y0_j, j < k, in two passes.  The
// column kernel gives each workgroup one column tile (64 lanes x 16 B) and one
// chunk of rows and writes the chunk's partial sums; a second kernel adds the
// partials of each column in chunk order.  (A single kernel whose last
// workgroup reduces needs a device-scope release/acquire pair per workgroup,
// which measured 4-6x slower than the extra launch on gfx950.)
template <typename T, int TAG>
__global__ void __launch_bounds__(256) gemv_cols_part_kernel(
    const T* __restrict__ A, int lda, int m, int shape, const T* __restrict__ x, T* __restrict__ part,
    int rows_per_chunk, const int* __restrict__ skip) {
  if (skip && *skip) return;
  constexpr int CW = kWave * Vec16<T>::n;
  const int tile = blockIdx.x, chunk = blockIdx.y;
  const size_t ps = (size_t)gridDim.x * CW;
  const int c0 = tile * CW;
  const int first_chunk = (shape == kLower) ? (c0 / rows_per_chunk) : 0;
  if (chunk < first_chunk) return;
  const int r0 = chunk * rows_per_chunk;
  const int r1 = min(m, r0 + rows_per_chunk);
  __shared__ T red[4][CW];
  cols_block_partial<T>(A, lda, r0, r1, c0, shape, x, red);
  if (threadIdx.x < CW) {
    const int jj = threadIdx.x;
    part[(size_t)chunk * ps + c0 + jj] = (red[0][jj] + red[1][jj]) + (red[2][jj] + red[3][jj]);
  }
}

template <typename T>
__global__ void __launch_bounds__(256) gemv_cols_reduce_kernel(int k, int ps, int shape, const T* __restrict__ part,
                                                               int rows_per_chunk, int nchunks, T* __restrict__ y,
                                                               T alpha, T beta, const T* __restrict__ y0,
                                                               const int* __restrict__ skip) {
  if (skip && *skip) return;
  constexpr int CW = kWave * Vec16<T>::n;
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= k) return;
  const int first_chunk = (shape == kLower) ? ((col / CW) * CW / rows_per_chunk) : 0;
  T s = 0;
  for (int ch = first_chunk; ch < nchunks; ++ch) s += part[(size_t)ch * ps + col];
  T v = alpha * s;
  if (y0) v += beta * y0[col];
  y[col] = v;
}

// ---------------------------------------------------------------------------
// host launchers
template <typename T>
static int gemv_rows_grid(int m) {
  int cus = dev_info().cu_count;
  int blocks = (m + 3) / 4;
  int cap = cus * 2;
  return blocks < cap ? blocks : cap;
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
  if (ev) (void)hipEventRecord(ev->begin, st);
  if (tag == 2)
    hipLaunchKernelGGL((gemv_rows_kernel<T, 2>), grid, dim3(256), smem, st, A, lda, m, k, shape, x, y, alpha, beta,
                       y0, nsplit, skip);
  else if (tag == 4)
    hipLaunchKernelGGL((gemv_rows_kernel<T, 4>), grid, dim3(256), smem, st, A, lda, m, k, shape, x, y, alpha, beta,
                       y0, nsplit, skip);
  else
    hipLaunchKernelGGL((gemv_rows_kernel<T, 0>), grid, dim3(256), smem, st, A, lda, m, k, shape, x, y, alpha, beta,
                       y0, nsplit, skip);
  hipError_t e = hipGetLastError();
  if (ev) (void)hipEventRecord(ev->end, st);
  return e;
}

template <typename T>
void gemv_cols_plan(int m, int k, int& rows_per_chunk, int& nchunks) {
  constexpr int CW = kWave * Vec16<T>::n;
  int tiles = (k + CW - 1) / CW;
  int target = dev_info().cu_count * 4;
  int nc = target / (tiles > 0 ? tiles : 1);
  int maxc = (m + 31) / 32;
  if (nc > maxc) nc = maxc;
  if (nc < 1) nc = 1;
  int rpc = (m + nc - 1) / nc;
  rpc = (rpc + 15) / 16 * 16;
  if (rpc < 16) rpc = 16;
  rows_per_chunk = rpc;
  nchunks = (m + rpc - 1) / rpc;
}

template <typename T>
hipError_t launch_gemv_cols(hipStream_t st, const T* A, int lda, int m, int k, int shape, const T* x, T* y,
                            T alpha, T beta, const T* y0, const GemvWork<T>& w, const int* skip, int tag,
                            const EventPair* ev) {
  if (k <= 0) return hipSuccess;
  constexpr int CW = kWave * Vec16<T>::n;
  int tiles = (k + CW - 1) / CW;
  if (m <= 0) return hipErrorInvalidValue;
  if (shape == kLower && k > m) return hipErrorInvalidValue;  // every column tile must meet a row chunk
  int rpc, nch;
  gemv_cols_plan<T>(m, k, rpc, nch);
  if ((size_t)nch * tiles * CW > w.part_elems) return hipErrorInvalidValue;
  if (tiles * CW > lda) return hipErrorInvalidValue;
  dim3 grid(tiles, nch);
  if (ev) (void)hipEventRecord(ev->begin, st);
  if (tag == 1)
    hipLaunchKernelGGL((gemv_cols_part_kernel<T, 1>), grid, dim3(256), 0, st, A, lda, m, shape, x, w.part, rpc, skip);
  else if (tag == 3)
    hipLaunchKernelGGL((gemv_cols_part_kernel<T, 3>), grid, dim3(256), 0, st, A, lda, m, shape, x, w.part, rpc, skip);
  else if (tag == 5)
    hipLaunchKernelGGL((gemv_cols_part_kernel<T, 5>), grid, dim3(256), 0, st, A, lda, m, shape, x, w.part, rpc, skip);
  else
    hipLaunchKernelGGL((gemv_cols_part_kernel<T, 0>), grid, dim3(256), 0, st, A, lda, m, shape, x, w.part, rpc, skip);
  if (ev) (void)hipEventRecord(ev->end, st);
  hipLaunchKernelGGL(gemv_cols_reduce_kernel<T>, dim3((k + 255) / 256), dim3(256), 0, st, k, tiles * CW, shape, w.part,
                     rpc, nch, y, alpha, beta, y0, skip);
  return hipGetLastError();
}

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
template void gemv_cols_plan<double>(int, int, int&, int&);
template void gemv_cols_plan<float>(int, int, int&, int&);

}  // namespace qpg
