// Multi-vector kernels of the block PCG over QPs that share H, A and C (and so
// K0 and its inverse factor) but not c, b, d.  One CG step of k such QPs applies
// the same operator C K0^{-1}_{11} C^T to k direction vectors, so each matrix is
// streamed once for all k: every entry loaded from HBM meets k vectors held in
// LDS (2k flops per 8 bytes instead of 2), so the product is a dense contraction
// and runs on MFMA.
//
//   mv_rows : Y_v = alpha op(A) X_v for v < nv, op(A) a row sweep over a dense,
//             lower-trapezoid or upper-trapezoid matrix; rows >= nsplit negated.
//             A skinny GEMM on the FP64 matrix cores: workgroups own a tile of
//             rows and a slice of the columns (split K, so a tall operand still
//             yields hundreds of workgroups while each stages only its slice of
//             the vectors), write per-slice partials, and a second kernel adds
//             the slices in order.
//   bq_epilogue : per column j, q_j += d_j o p_j and p_j^T q_j (for the update).
//
// Vectors are column-major: X_v = X + v * ldx.
#include <algorithm>

#include "kernels.hpp"
#include "gemv_core.hpp"
#include "pcg.hpp"

namespace qpg {

typedef double v4d_t __attribute__((ext_vector_type(4)));

// Tile product on the FP64 matrix cores: a workgroup owns kMvRows = 64 rows (16 per
// wave) and a slice of KS = 256 columns, and forms the 64 x 16 NB block of
// A[rows, slice] X[slice, v] with v_mfma_f64_16x16x4 (lane l
// supplies A[l % 16][k] and X[k][l % 16] of its step, register r of the result
// holds row 4 r + l / 16, vector l % 16).  The slice is summed in a permuted
// order: at step t lane quarter q = l / 16 takes column 8 (t / 2) + 2 q + t % 2, so
// one 16-byte load gives a lane its columns of two steps and the four quarters of
// a row read 64 adjacent bytes per instruction (16 half-lines per load instead of
// 64 scattered pieces); loads are issued a batch ahead of the matrix
// instructions.  The vectors are staged in LDS already in step order
// (Bs[t][lane]: one contiguous 512-byte read per step, no bank conflicts), with
// 16-byte loads of column pairs (k = 16 on a dense 4096 x 4096 sweep: 34.6 against
// 36.2 us with 8-byte loads).  128 rows per workgroup (two MFMA blocks per
// wavefront) win on that square sweep (32.3 us) but lose on the solver's shapes,
// whose few row tiles then leave CUs without a second workgroup (M: 61 against
// 54 us).
constexpr int kMvKS = 256;                // columns per slice
constexpr int kMvQ = kMvKS / 4;           // steps per slice (columns per lane quarter)
constexpr int kMvBatch = 8;               // 16-byte loads per lane and row block in flight (16 steps)
constexpr int kMvRows = 64;               // rows per workgroup
constexpr int kMvRB = kMvRows / 64;       // 16-row MFMA blocks per wavefront

template <int NB>
__global__ void __launch_bounds__(256) mv_mfma_kernel(const double* __restrict__ A, int lda, int rows, int K,
                                                      int shape, const double* __restrict__ X, int ldx, int nv,
                                                      int vx, double* __restrict__ part, int ldp) {
  const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
  const int r0 = blockIdx.x * kMvRows, s = blockIdx.y;
  const int c0 = s * kMvKS, c1 = min(K, c0 + kMvKS);
  const int rlast = min(rows, r0 + kMvRows) - 1;
  const bool empty = (shape == kLower && c0 > rlast) || (shape == kUpper && c1 <= r0);
  __shared__ __align__(16) double Bs[NB][kMvQ][kWave];
  v4d_t acc[kMvRB][NB];
#pragma unroll
  for (int rb = 0; rb < kMvRB; ++rb)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[rb][b] = v4d_t{0.0, 0.0, 0.0, 0.0};
  const int q = lane / 16;
  if (!empty) {
    // stage X[slice, v] in step order: slice column c = 8 u + 2 q + h is step t = 2 u + h of quarter q;
    // columns c, c + 1 (one 16-byte load) are steps t, t + 1 of the same quarter
    if (vx) {
      for (int e = tid; e < NB * 16 * kMvKS / 2; e += 256) {
        const int cp = e % (kMvKS / 2), vv = e / (kMvKS / 2);
        const int b = vv / 16, v = vv % 16, c = 2 * cp, col = c0 + c;
        const int t = 2 * (c / 8), qq = (c % 8) / 2;
        v2d_t x = v2d_t{0.0, 0.0};
        if (vv < nv) {
          if (col + 1 < c1) x = *reinterpret_cast<const v2d_t*>(X + (size_t)vv * ldx + col);
          else if (col < c1) x.x = X[(size_t)vv * ldx + col];
        }
        Bs[b][t][qq * 16 + v] = x.x;
        Bs[b][t + 1][qq * 16 + v] = x.y;
      }
    } else {
      for (int e = tid; e < NB * 16 * kMvKS; e += 256) {
        const int c = e % kMvKS, vv = e / kMvKS;  // column of the slice (fastest: coalesced reads), vector
        const int b = vv / 16, v = vv % 16, col = c0 + c;
        const int t = 2 * (c / 8) + (c % 2), qq = (c % 8) / 2;
        Bs[b][t][qq * 16 + v] = (vv < nv && col < c1) ? X[(size_t)vv * ldx + col] : 0.0;
      }
    }
    int row[kMvRB], cend[kMvRB];
    const double* arow[kMvRB];
#pragma unroll
    for (int rb = 0; rb < kMvRB; ++rb) {
      row[rb] = r0 + wave * 16 * kMvRB + rb * 16 + lane % 16;  // the rows this lane supplies
      const int len = shape == kLower ? min(row[rb] + 1, K) : K;
      cend[rb] = min(len, c1);  // columns of the row inside the slice
      arow[rb] = A + (size_t)min(row[rb], rows - 1) * lda;
    }
    auto load_batch = [&](int t0, v2d_t (*a)[kMvBatch]) {
#pragma unroll
      for (int rb = 0; rb < kMvRB; ++rb)
#pragma unroll
        for (int u = 0; u < kMvBatch; ++u) {
          const int col = c0 + 8 * (t0 / 2 + u) + 2 * q;  // steps t0 + 2 u and t0 + 2 u + 1
          if (row[rb] < rows && col < cend[rb])
            a[rb][u] = __builtin_nontemporal_load(reinterpret_cast<const v2d_t*>(arow[rb] + col));
          else
            a[rb][u] = v2d_t{0.0, 0.0};
        }
    };
    v2d_t cur[kMvRB][kMvBatch], nxt[kMvRB][kMvBatch];
    load_batch(0, cur);
    __syncthreads();
#pragma unroll 1
    for (int t0 = 0; t0 < kMvQ; t0 += 2 * kMvBatch) {
      if (t0 + 2 * kMvBatch < kMvQ) load_batch(t0 + 2 * kMvBatch, nxt);
#pragma unroll
      for (int u = 0; u < kMvBatch; ++u) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int t = t0 + 2 * u + h;
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            const double bx = Bs[b][t][lane];
#pragma unroll
            for (int rb = 0; rb < kMvRB; ++rb)
              acc[rb][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(h ? cur[rb][u].y : cur[rb][u].x, bx, acc[rb][b], 0,
                                                                0, 0);
          }
        }
      }
#pragma unroll
      for (int rb = 0; rb < kMvRB; ++rb)
#pragma unroll
        for (int u = 0; u < kMvBatch; ++u) cur[rb][u] = nxt[rb][u];
    }
  }
  // register r of lane l of block rb: row r0 + 32 wave + 16 rb + 4 r + l / 16, vector 16 b + l % 16
#pragma unroll
  for (int rb = 0; rb < kMvRB; ++rb)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int v = 16 * b + lane % 16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = r0 + wave * 16 * kMvRB + rb * 16 + 4 * r + lane / 16;
        if (i < rows && v < nv) part[((size_t)s * nv + v) * ldp + i] = acc[rb][b][r];
      }
    }
}

// Y_v[i] = (i >= nsplit ? -alpha : alpha) * sum over slices of part (slice order).
__global__ void __launch_bounds__(256) mv_reduce_kernel(const double* __restrict__ part, int ldp, int S, int nv,
                                                        int rows, double* __restrict__ Y, int ldy, double alpha,
                                                        int nsplit) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)nv * rows) return;
  const int v = (int)(e / rows), i = (int)(e % rows);
  double t = 0.0;
  for (int s = 0; s < S; ++s) t += part[((size_t)s * nv + v) * ldp + i];
  Y[(size_t)v * ldy + i] = (i >= nsplit ? -alpha : alpha) * t;
}

template <int NB>
static void launch_mfma(hipStream_t st, const double* A, int lda, int rows, int K, int shape, const double* X,
                        int ldx, int nv, double* part, int ldp) {
  const dim3 grid((rows + kMvRows - 1) / kMvRows, (K + kMvKS - 1) / kMvKS);
  const int vx = (reinterpret_cast<uintptr_t>(X) & 15) == 0 && ldx % 2 == 0;  // 16-byte staging loads
  hipLaunchKernelGGL((mv_mfma_kernel<NB>), grid, dim3(256), 0, st, A, lda, rows, K, shape, X, ldx, nv, vx, part,
                     ldp);
}

size_t mv_part_elems(int rows, int K, int nv) {
  const int S = (K + kMvKS - 1) / kMvKS;
  return (size_t)S * std::min(nv, 32) * (size_t)rows;
}

hipError_t launch_mv_rows(hipStream_t st, const double* A, int lda, int rows, int K, int shape, const double* X,
                          int ldx, int nv, double* Y, int ldy, double alpha, int nsplit, double* part,
                          size_t part_elems) {
  if (rows <= 0 || nv <= 0) return hipSuccess;
  if (K <= 0 || lda < K || lda % 2 != 0 || ldx < K || ldy < rows) return hipErrorInvalidValue;
  if (mv_part_elems(rows, K, nv) > part_elems) return hipErrorInvalidValue;
  if (nsplit < 0) nsplit = rows;
  const int S = (K + kMvKS - 1) / kMvKS;
  for (int v0 = 0; v0 < nv; v0 += 32) {  // groups of at most 32 vectors
    const int g = std::min(32, nv - v0);
    const double* Xg = X + (size_t)v0 * ldx;
    if (g <= 16)
      launch_mfma<1>(st, A, lda, rows, K, shape, Xg, ldx, g, part, rows);
    else
      launch_mfma<2>(st, A, lda, rows, K, shape, Xg, ldx, g, part, rows);
    const size_t tot = (size_t)g * rows;
    hipLaunchKernelGGL(mv_reduce_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, part, rows, S, g,
                       rows, Y + (size_t)v0 * ldy, ldy, alpha, nsplit);
  }
  return hipGetLastError();
}

// q_j += d_j o p_j and bpart_j = p_j^T q_j for the solves that have not stopped
// (one workgroup per solve; the list is the PcgDesc of the block update).
__global__ void __launch_bounds__(256) bq_epilogue_kernel(const PcgDesc<double>* __restrict__ descs) {
  const PcgDesc<double> d = descs[blockIdx.x];
  const int done = d.sc->done;
  if (done) return;
  __shared__ double sh[16];
  double pq = 0.0;
  for (int i = threadIdx.x; i < d.m2; i += blockDim.x) {
    const double p = d.p[i];
    const double q = d.q[i] + d.dvec[i] * p;
    d.q[i] = q;
    pq += p * q;
  }
  pq = block_sum<double>(pq, sh);
  if (threadIdx.x == 0) d.bpart[0] = pq;
}

hipError_t bq_epilogue(hipStream_t st, const PcgDesc<double>* d, int count) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(bq_epilogue_kernel, dim3(count), dim3(256), 0, st, d);
  return hipGetLastError();
}

}  // namespace qpg
