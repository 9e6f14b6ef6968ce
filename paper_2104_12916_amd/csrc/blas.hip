// Dense FP64 factorization kernels for the once-per-QP setup (gfx950 MFMA).
//
//   gemm_f64      C = alpha op(A) op(B) + beta C, 64x64 tiles, v_mfma_f64_16x16x4
//                 through LDS; optional "lower only" output (SYRK-shaped updates)
//                 and k-range trimming for triangular operands.
//   chol_inv_leaf one workgroup factors a <= 64 x 64 SPD block in LDS and inverts
//                 the Cholesky factor (LL^T = A, X = L^{-1}).
//   chol_inv      recursive blocked driver: with A = [A11 .; A21 A22],
//                   (L11, X11) = chol_inv(A11);  L21 = A21 X11^T;
//                   A22 -= L21 L21^T and T = L21 X11 (one launch);
//                   (L22, X22) = chol_inv(A22);  X21 = -X22 T,
//                 so almost every flop runs in the MFMA GEMM.
#include <algorithm>
#include <cstring>

#include "kernels.hpp"

namespace qpg {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int GB = 64;   // tile
constexpr int GK = 16;   // k step

__device__ __forceinline__ void gemm_body(int M, int N, int K, double alpha, const double* __restrict__ A, int lda,
                                          int ta, const double* __restrict__ B, int ldb, int tb, double beta,
                                          double* __restrict__ C, int ldc, int flags, int bx, int by) {
  const int i0 = by * GB, j0 = bx * GB;
  if ((flags & kOutLower) && j0 > i0 + GB - 1) return;
  __shared__ double As[GK][GB + 4];
  __shared__ double Bs[GK][GB + 4];
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int wr = (wave / 2) * 32, wc = (wave % 2) * 32;
  // k range that can be nonzero for this tile
  int klo = 0, khi = K;
  if (flags & kALower) khi = min(khi, i0 + GB);       // op(A)[i][k] = 0 for k > i
  if (flags & kBUpper) khi = min(khi, j0 + GB);       // op(B)[k][j] = 0 for k > j
  if (flags & kBLower) klo = max(klo, j0);            // op(B)[k][j] = 0 for k < j
  if (flags & kAUpper) klo = max(klo, i0);            // op(A)[i][k] = 0 for k < i
  klo = klo / GK * GK;
  v4d acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4d{0, 0, 0, 0};

  double ra[4], rb[4];
  auto load_tiles = [&](int k0) {
    if (!ta) {  // op(A)[i][k] = A[i*lda + k]
      int r = tid / 4, kq = (tid % 4) * 4;
      int gi = i0 + r;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int gk = k0 + kq + e;
        ra[e] = (gi < M && gk < K) ? A[(size_t)gi * lda + gk] : 0.0;
      }
    } else {    // op(A)[i][k] = A[k*lda + i]
      int kr = tid / 16, iq = (tid % 16) * 4;
      int gk = k0 + kr;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int gi = i0 + iq + e;
        ra[e] = (gi < M && gk < K) ? A[(size_t)gk * lda + gi] : 0.0;
      }
    }
    if (!tb) {  // op(B)[k][j] = B[k*ldb + j]
      int kr = tid / 16, jq = (tid % 16) * 4;
      int gk = k0 + kr;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int gj = j0 + jq + e;
        rb[e] = (gj < N && gk < K) ? B[(size_t)gk * ldb + gj] : 0.0;
      }
    } else {    // op(B)[k][j] = B[j*ldb + k]
      int r = tid / 4, kq = (tid % 4) * 4;
      int gj = j0 + r;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int gk = k0 + kq + e;
        rb[e] = (gj < N && gk < K) ? B[(size_t)gj * ldb + gk] : 0.0;
      }
    }
  };
  auto store_tiles = [&]() {
    if (!ta) {
      int r = tid / 4, kq = (tid % 4) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) As[kq + e][r] = ra[e];
    } else {
      int kr = tid / 16, iq = (tid % 16) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) As[kr][iq + e] = ra[e];
    }
    if (!tb) {
      int kr = tid / 16, jq = (tid % 16) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) Bs[kr][jq + e] = rb[e];
    } else {
      int r = tid / 4, kq = (tid % 4) * 4;
#pragma unroll
      for (int e = 0; e < 4; ++e) Bs[kq + e][r] = rb[e];
    }
  };

  if (klo < khi) load_tiles(klo);
  for (int k0 = klo; k0 < khi; k0 += GK) {
    __syncthreads();
    store_tiles();
    __syncthreads();
    if (k0 + GK < khi) load_tiles(k0 + GK);
#pragma unroll
    for (int kk = 0; kk < GK / 4; ++kk) {
      const int kr = kk * 4 + lane / 16;
      double a0 = As[kr][wr + (lane % 16)];
      double a1 = As[kr][wr + 16 + (lane % 16)];
      double b0 = Bs[kr][wc + (lane % 16)];
      double b1 = Bs[kr][wc + 16 + (lane % 16)];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
  }
  // f64 16x16x4 result layout: register r of lane l holds D[4 r + l / 16][l % 16]
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int gi = i0 + wr + a * 16 + 4 * r + lane / 16;
        int gj = j0 + wc + b * 16 + (lane % 16);
        if (gi < M && gj < N) {
          double v = alpha * acc[a][b][r];
          double* cp = C + (size_t)gi * ldc + gj;
          if (beta != 0.0) v += beta * (*cp);
          *cp = v;
        }
      }
}

__global__ void __launch_bounds__(256) gemm_f64_kernel(int M, int N, int K, double alpha, const double* __restrict__ A,
                                                       int lda, int ta, const double* __restrict__ B, int ldb, int tb,
                                                       double beta, double* __restrict__ C, int ldc, int flags) {
  gemm_body(M, N, K, alpha, A, lda, ta, B, ldb, tb, beta, C, ldc, flags, blockIdx.x, blockIdx.y);
}

// One GEMM per blockIdx.z, same op/scalars for all; tiles outside a problem's
// M x N exit at once.
__global__ void __launch_bounds__(256) gemm_f64_batched_kernel(const GemmDesc* __restrict__ descs, int ta, int tb,
                                                               double alpha, double beta, int flags) {
  const GemmDesc g = descs[blockIdx.z];
  if ((int)blockIdx.y * GB >= g.M || (int)blockIdx.x * GB >= g.N) return;
  gemm_body(g.M, g.N, g.K, alpha, g.A, g.lda, ta, g.B, g.ldb, tb, beta, g.C, g.ldc, flags, blockIdx.x, blockIdx.y);
}

hipError_t gemm_f64(hipStream_t st, int ta, int tb, int M, int N, int K, double alpha, const double* A, int lda,
                    const double* B, int ldb, double beta, double* C, int ldc, int flags) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if ((M + GB - 1) / GB > 65535) return hipErrorInvalidValue;
  dim3 grid((N + GB - 1) / GB, (M + GB - 1) / GB);
  hipLaunchKernelGGL(gemm_f64_kernel, grid, dim3(256), 0, st, M, N, K, alpha, A, lda, ta, B, ldb, tb, beta, C, ldc,
                     flags);
  return hipGetLastError();
}

// Two independent GEMMs in one launch (blockIdx.z selects the problem).
struct GemmArgs {
  int ta, tb, M, N, K;
  double alpha;
  const double* A;
  int lda;
  const double* B;
  int ldb;
  double beta;
  double* C;
  int ldc, flags;
};

__global__ void __launch_bounds__(256) gemm_f64_pair_kernel(GemmArgs g0, GemmArgs g1) {
  const GemmArgs g = blockIdx.z == 0 ? g0 : g1;
  if ((int)blockIdx.y * GB >= g.M || (int)blockIdx.x * GB >= g.N) return;
  gemm_body(g.M, g.N, g.K, g.alpha, g.A, g.lda, g.ta, g.B, g.ldb, g.tb, g.beta, g.C, g.ldc, g.flags, blockIdx.x,
            blockIdx.y);
}

static hipError_t gemm_f64_pair(hipStream_t st, const GemmArgs& g0, const GemmArgs& g1) {
  const int gx = (std::max(g0.N, g1.N) + GB - 1) / GB, gy = (std::max(g0.M, g1.M) + GB - 1) / GB;
  if (gx <= 0 || gy <= 0) return hipSuccess;
  if (gy > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(gemm_f64_pair_kernel, dim3(gx, gy, 2), dim3(256), 0, st, g0, g1);
  return hipGetLastError();
}

// Batched form: blockIdx.z < count0 takes d0[z] with o0, the rest d1[z - count0] with o1.
__global__ void __launch_bounds__(256) gemm_f64_batched_pair_kernel(const GemmDesc* __restrict__ d0, int count0,
                                                                    GemmOp o0, const GemmDesc* __restrict__ d1,
                                                                    GemmOp o1) {
  const int z = blockIdx.z;
  const GemmDesc g = z < count0 ? d0[z] : d1[z - count0];
  const GemmOp o = z < count0 ? o0 : o1;
  if ((int)blockIdx.y * GB >= g.M || (int)blockIdx.x * GB >= g.N) return;
  gemm_body(g.M, g.N, g.K, o.alpha, g.A, g.lda, o.ta, g.B, g.ldb, o.tb, o.beta, g.C, g.ldc, o.flags, blockIdx.x,
            blockIdx.y);
}

// ---------------------------------------------------------------------------
constexpr int LEAF = 64;

// A pivot is rejected when it is not positive or falls below kPivRel times the
// largest diagonal entry of the whole input matrix (*dmax): for a singular
// matrix the computed pivot is a rounding residue of order eps * ||A||.
constexpr double kPivRel = 1e-13;

// Leaf: right-looking LDL^T of a <= 64 x 64 SPD block held in registers, then
// L = L_1 D^{1/2} and X = L^{-1} = D^{-1/2} L_1^{-1}.  Thread t owns the 4 x 4
// sub-block (rows 4 (t / 16) .., cols 4 (t % 16) ..) of both A and X.  Column j
// of the elimination applies
//     a_ik -= (a_ij / a_jj) a_kj   (j < k <= i),    x_ik -= (a_ij / a_jj) x_jk   (i > j),
// with X starting as I (its rows only mix with earlier rows, so it stays lower
// triangular).  The columns are taken four at a time: the owners of column
// block J publish it (and the owners of rows 4J..4J+3 those rows of X) in LDS,
// one barrier, and then every thread eliminates the 4 x 4 diagonal block and
// the block's part of the rows it needs, and applies the four column steps to
// its sub-blocks.  Each entry sees the same updates in the same order as with
// one column per step, with one barrier per four columns.
__device__ __forceinline__ void chol_inv_leaf_body(double* __restrict__ A, int lda, double* __restrict__ X, int ldx,
                                                   int nb, int* __restrict__ info, int code,
                                                   const double* __restrict__ dmax) {
  __shared__ double pan[2][LEAF][4];  // column block J of A (rows >= 4J), double-buffered
  __shared__ double xrow[2][4][LEAF];  // rows 4J..4J+3 of X as they enter block J
  __shared__ double piv[LEAF];
  const int t = threadIdx.x, tr = t >> 4, tc = t & 15, r0 = tr * 4, c0 = tc * 4;
  const double pmin = kPivRel * (*dmax);
  double a[4][4], x[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int i = r0 + r, k = c0 + c;
      a[r][c] = (i < nb && k <= i) ? A[(size_t)i * lda + k] : 0.0;
      x[r][c] = (i == k && i < nb) ? 1.0 : 0.0;
    }
  bool bad = false;
  const int nblk = (nb + 3) / 4;
  for (int J = 0; J < nblk; ++J) {
    const int buf = J & 1, j0 = 4 * J;
    if (tc == J && tr >= J) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) pan[buf][r0 + r][q] = a[r][q];
    }
    if (tr == J) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) xrow[buf][r][c0 + c] = x[r][c];
    }
    __syncthreads();
    // Diagonal block: E[i][q] (q <= i) ends as the eliminated value of a_{j0+i, j0+q}
    // at its own column step (E[p][p] is the pivot d_p).
    double E[4][4], dinv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) E[i][q] = q <= i ? pan[buf][j0 + i][q] : 0.0;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      double d = E[p][p];
      if (j0 + p < nb) {
        if (!(d > pmin) || !isfinite(d)) {  // same decision in every thread
          bad = true;
          d = 1.0;
        }
      } else {
        d = 1.0;  // past the block's end: the row and column are zero
      }
      E[p][p] = d;
      dinv[p] = 1.0 / d;
#pragma unroll
      for (int i = p + 1; i < 4; ++i) {
        const double coef = E[i][p] * dinv[p];
#pragma unroll
        for (int k = p + 1; k <= i; ++k) E[i][k] -= coef * E[k][p];
      }
    }
    if (t == 0) {
#pragma unroll
      for (int p = 0; p < 4; ++p) piv[j0 + p] = E[p][p];
    }
    // Row i >= j0 + 4 through the block's four steps: ev[p] = eliminated a_{i, j0+p},
    // cf[p] = ev[p] / d_p (the multiplier of step j0 + p).
    auto row_steps = [&](int i, double (&ev)[4], double (&cf)[4]) {
      double g[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) g[q] = pan[buf][i][q];
#pragma unroll
      for (int p = 0; p < 4; ++p) {
#pragma unroll
        for (int pp = 0; pp < p; ++pp) g[p] -= cf[pp] * E[p][pp];
        ev[p] = g[p];
        cf[p] = g[p] * dinv[p];
      }
    };
    double cfr[4][4], evr[4][4];  // this thread's rows r0 + r
    if (tr > J) {
#pragma unroll
      for (int r = 0; r < 4; ++r) row_steps(min(r0 + r, LEAF - 1), evr[r], cfr[r]);
    }
    // A: the owners of the column block keep its eliminated values; sub-blocks right of
    // it and on or below the diagonal take the four rank-one updates.
    if (tc == J && tr == J) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q <= r; ++q) a[r][q] = E[r][q];
    } else if (tc == J && tr > J) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
        if (r0 + r < nb) {
#pragma unroll
          for (int q = 0; q < 4; ++q) a[r][q] = evr[r][q];
        }
    } else if (tc > J && tr >= tc) {
      double evc[4][4], cfc[4][4];  // the rows k = c0 + c (columns of this sub-block)
#pragma unroll
      for (int c = 0; c < 4; ++c) row_steps(c0 + c, evc[c], cfc[c]);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = r0 + r;
        if (i >= nb) continue;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          if (c0 + c > i) continue;
#pragma unroll
          for (int p = 0; p < 4; ++p) a[r][c] -= cfr[r][p] * evc[c][p];
        }
      }
    }
    // X: rows j0..j0+3 first eliminate among themselves, then rows below take them.
    if (tr >= J) {
      double xf[4][4];
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int c = 0; c < 4; ++c) xf[p][c] = xrow[buf][p][c0 + c];
#pragma unroll
      for (int p = 1; p < 4; ++p)
#pragma unroll
        for (int pp = 0; pp < p; ++pp) {
          const double l = E[p][pp] * dinv[pp];
#pragma unroll
          for (int c = 0; c < 4; ++c) xf[p][c] -= l * xf[pp][c];
        }
      if (tr == J) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (r0 + r < nb) {
#pragma unroll
            for (int c = 0; c < 4; ++c) x[r][c] = xf[r][c];
          }
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (r0 + r >= nb) continue;
#pragma unroll
          for (int p = 0; p < 4; ++p)
#pragma unroll
            for (int c = 0; c < 4; ++c) x[r][c] -= cfr[r][p] * xf[p][c];
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = r0 + r;
    if (i >= nb) continue;
    const double si = sqrt(piv[i]);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int k = c0 + c;
      if (k >= nb) continue;
      if (k <= i) A[(size_t)i * lda + k] = a[r][c] / sqrt(piv[k]);
      X[(size_t)i * ldx + k] = x[r][c] / si;
    }
  }
  if (t == 0 && bad) *info = code;
}

__global__ void __launch_bounds__(256) chol_inv_leaf_kernel(double* __restrict__ A, int lda, double* __restrict__ X,
                                                            int ldx, int nb, int* __restrict__ info, int code,
                                                            const double* __restrict__ dmax) {
  chol_inv_leaf_body(A, lda, X, ldx, nb, info, code, dmax);
}

__global__ void __launch_bounds__(256) chol_inv_leaf_batched_kernel(const LeafDesc* __restrict__ descs) {
  const LeafDesc d = descs[blockIdx.x];
  chol_inv_leaf_body(d.A, d.lda, d.X, d.ldx, d.nb, d.info, d.code, d.dmax);
}

__global__ void fill2d_kernel(double* __restrict__ X, int ld, int rows, int cols, double v) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  int i = blockIdx.y;
  if (i < rows && j < cols) X[(size_t)i * ld + j] = v;
}

hipError_t fill2d_f64(hipStream_t st, double* X, int ld, int rows, int cols, double v) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  if (rows > 65535) return hipErrorInvalidValue;
  dim3 grid((cols + 255) / 256, rows);
  hipLaunchKernelGGL(fill2d_kernel, grid, dim3(256), 0, st, X, ld, rows, cols, v);
  return hipGetLastError();
}

// Split point of a node of n > LEAF rows: half of the smallest 64 * 2^k >= n.
// Splits therefore sit at fixed positions (multiples of powers of two), so the
// recursion of a problem is the same whether it runs alone or inside a batch
// whose largest problem is bigger (there the extra levels are left-only).
static int split_of(int n) {
  int v = LEAF;
  while (v < n) v *= 2;
  return v / 2;
}

// Recursive body.  A: n x n (lower part read, overwritten with scratch), X: n x n
// output (upper part must be zero on entry), tmp: chol_inv_tmp_elems(n) - 1
// doubles (a node keeps its n2 x n1 block of L21 X11 while its right child
// works past it; the deepest chain of such blocks stays below that size).
static hipError_t chol_inv_rec(hipStream_t st, double* A, int lda, double* X, int ldx, int n, double* tmp,
                               int* info, int code, const double* dmax) {
  hipError_t e;
  if (n <= LEAF) {
    hipLaunchKernelGGL(chol_inv_leaf_kernel, dim3(1), dim3(256), 0, st, A, lda, X, ldx, n, info, code, dmax);
    return hipGetLastError();
  }
  const int n1 = split_of(n);
  const int n2 = n - n1;
  double* A11 = A;
  double* A21 = A + (size_t)n1 * lda;
  double* A22 = A21 + n1;
  double* X11 = X;
  double* X21 = X + (size_t)n1 * ldx;
  double* X22 = X21 + n1;
  if ((e = chol_inv_rec(st, A11, lda, X11, ldx, n1, tmp, info, code, dmax)) != hipSuccess) return e;
  // L21 = A21 X11^T  (op(B) = X11^T is upper triangular) -> stored in X21
  if ((e = gemm_f64(st, 0, 1, n2, n1, n1, 1.0, A21, lda, X11, ldx, 0.0, X21, ldx, kBUpper)) != hipSuccess) return e;
  // one launch, both reading only L21 and X11: A22 -= L21 L21^T (lower part) and
  // tmp = L21 X11 (X11 lower)
  const GemmArgs s22{0, 1, n2, n2, n1, -1.0, X21, ldx, X21, ldx, 1.0, A22, lda, kOutLower};
  const GemmArgs t21{0, 0, n2, n1, n1, 1.0, X21, ldx, X11, ldx, 0.0, tmp, n1, kBLower};
  if ((e = gemm_f64_pair(st, s22, t21)) != hipSuccess) return e;
  double* tmp_right = tmp + (size_t)n2 * n1;  // past this node's block
  if ((e = chol_inv_rec(st, A22, lda, X22, ldx, n2, tmp_right, info, code, dmax)) != hipSuccess) return e;
  // X21 = -X22 tmp (X22 lower)
  if ((e = gemm_f64(st, 0, 0, n2, n1, n2, -1.0, X22, ldx, tmp, n1, 0.0, X21, ldx, kALower)) != hipSuccess) return e;
  return hipSuccess;
}

// Largest diagonal entry of A (n x n) into *out; one workgroup.
__device__ __forceinline__ void diag_max_body(const double* __restrict__ A, int lda, int n, double* __restrict__ out) {
  __shared__ double sh[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, A[(size_t)i * lda + i]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

__global__ void __launch_bounds__(256) diag_max_kernel(const double* __restrict__ A, int lda, int n,
                                                       double* __restrict__ out) {
  diag_max_body(A, lda, n, out);
}

__global__ void __launch_bounds__(256) diag_max_batched_kernel(const DiagDesc* __restrict__ descs) {
  const DiagDesc d = descs[blockIdx.x];
  diag_max_body(d.A, d.lda, d.n, d.out);
}

// tmp holds chol_inv_tmp_elems(n) doubles; its last element stores max diag(A).
hipError_t chol_inv_f64(hipStream_t st, double* A, int lda, double* X, int ldx, int n, double* tmp, int* info,
                        int code) {
  hipError_t e = fill2d_f64(st, X, ldx, n, n, 0.0);
  if (e != hipSuccess) return e;
  double* dmax = tmp + chol_inv_tmp_elems(n) - 1;
  hipLaunchKernelGGL(diag_max_kernel, dim3(1), dim3(256), 0, st, A, lda, n, dmax);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  return chol_inv_rec(st, A, lda, X, ldx, n, tmp, info, code, dmax);
}

size_t chol_inv_tmp_elems(int n) { return (size_t)(n / 2 + LEAF) * (size_t)(n + LEAF) + 1; }

// ---- batched factorizations ----------------------------------------------------
template <typename D>
size_t BatchedOps::push(const std::vector<D>& v) {
  const size_t off = (bytes_.size() + 255) / 256 * 256;
  bytes_.resize(off + v.size() * sizeof(D));
  if (!v.empty()) memcpy(bytes_.data() + off, v.data(), v.size() * sizeof(D));
  return off;
}

void BatchedOps::gemm(int ta, int tb, double alpha, double beta, int flags, const std::vector<GemmDesc>& d) {
  if (d.empty()) return;
  int mx = 0, nx = 0;
  for (const GemmDesc& g : d) {
    mx = std::max(mx, g.M);
    nx = std::max(nx, g.N);
  }
  if (mx <= 0 || nx <= 0) return;
  Op o{};
  o.kind = 1;
  o.count = (int)d.size();
  o.gx = (nx + GB - 1) / GB;
  o.gy = (mx + GB - 1) / GB;
  o.g0 = GemmOp{ta, tb, flags, alpha, beta};
  o.off = push(d);
  ops_.push_back(o);
}

void BatchedOps::gemm_pair(const GemmOp& o0, const std::vector<GemmDesc>& d0, const GemmOp& o1,
                           const std::vector<GemmDesc>& d1) {
  if (d0.empty() || d1.empty()) {
    if (!d0.empty()) gemm(o0.ta, o0.tb, o0.alpha, o0.beta, o0.flags, d0);
    if (!d1.empty()) gemm(o1.ta, o1.tb, o1.alpha, o1.beta, o1.flags, d1);
    return;
  }
  int mx = 0, nx = 0;
  for (const auto* d : {&d0, &d1})
    for (const GemmDesc& g : *d) {
      mx = std::max(mx, g.M);
      nx = std::max(nx, g.N);
    }
  if (mx <= 0 || nx <= 0) return;
  Op o{};
  o.kind = 3;
  o.count = (int)d0.size();
  o.count2 = (int)d1.size();
  o.gx = (nx + GB - 1) / GB;
  o.gy = (mx + GB - 1) / GB;
  o.g0 = o0;
  o.g1 = o1;
  o.off = push(d0);
  o.off2 = push(d1);
  ops_.push_back(o);
}

// Same recursion as chol_inv_rec over nodes of 64 * 2^k rows starting at 0; at
// every node a job takes the part of the node inside its own n (possibly none),
// which is exactly the node chol_inv_rec visits for that job alone.
void BatchedOps::rec(const std::vector<CholJob>& jobs, int off, int len) {
  if (len <= LEAF) {
    std::vector<LeafDesc> d;
    for (const CholJob& j : jobs) {
      const int nb = std::min(len, j.n - off);
      if (nb <= 0) continue;
      LeafDesc l;
      l.A = j.A + (size_t)off * j.lda + off;
      l.X = j.X + (size_t)off * j.ldx + off;
      l.info = j.info;
      l.dmax = j.tmp + chol_inv_tmp_elems(j.n) - 1;
      l.lda = j.lda;
      l.ldx = j.ldx;
      l.nb = nb;
      l.code = j.code;
      d.push_back(l);
    }
    if (d.empty()) return;
    Op o{};
    o.kind = 0;
    o.count = (int)d.size();
    o.off = push(d);
    ops_.push_back(o);
    return;
  }
  const int n1 = len / 2;
  rec(jobs, off, n1);
  std::vector<GemmDesc> g1, g2, g3, g4;
  std::vector<CholJob> right;  // jobs reaching the right child, scratch past this node's block
  for (const CholJob& j : jobs) {
    const int n2 = std::min(len, j.n - off) - n1;
    if (n2 <= 0) continue;
    double* A21 = j.A + (size_t)(off + n1) * j.lda + off;
    double* A22 = A21 + n1;
    double* X11 = j.X + (size_t)off * j.ldx + off;
    double* X21 = j.X + (size_t)(off + n1) * j.ldx + off;
    double* X22 = X21 + n1;
    g1.push_back(GemmDesc{A21, X11, X21, j.lda, j.ldx, j.ldx, n2, n1, n1});    // L21 = A21 X11^T
    g2.push_back(GemmDesc{X21, X21, A22, j.ldx, j.ldx, j.lda, n2, n2, n1});    // A22 -= L21 L21^T
    g3.push_back(GemmDesc{X21, X11, j.work, j.ldx, j.ldx, n1, n2, n1, n1});    // tmp = L21 X11
    g4.push_back(GemmDesc{X22, j.work, X21, j.ldx, n1, j.ldx, n2, n1, n2});    // X21 = -X22 tmp
    CholJob r = j;
    r.work = j.work + (size_t)n2 * n1;
    right.push_back(r);
  }
  gemm(0, 1, 1.0, 0.0, kBUpper, g1);
  gemm_pair(GemmOp{0, 1, kOutLower, -1.0, 1.0}, g2, GemmOp{0, 0, kBLower, 1.0, 0.0}, g3);
  rec(right, off + n1, len - n1);
  gemm(0, 0, -1.0, 0.0, kALower, g4);
}

void BatchedOps::chol_inv(const std::vector<CholJob>& jobs) {
  if (jobs.empty()) return;
  std::vector<DiagDesc> d;
  int len = LEAF;
  for (const CholJob& j : jobs) {
    d.push_back(DiagDesc{j.A, j.tmp + chol_inv_tmp_elems(j.n) - 1, j.lda, j.n});
    while (len < j.n) len *= 2;
  }
  Op o{};
  o.kind = 2;
  o.count = (int)d.size();
  o.off = push(d);
  ops_.push_back(o);
  std::vector<CholJob> js = jobs;
  for (CholJob& j : js) j.work = j.tmp;
  rec(js, 0, len);
}

hipError_t BatchedOps::run(hipStream_t st, const void* d_bytes) const {
  const char* base = static_cast<const char*>(d_bytes);
  for (const Op& o : ops_) {
    if (o.count > 65535) return hipErrorInvalidValue;
    switch (o.kind) {
      case 0:
        hipLaunchKernelGGL(chol_inv_leaf_batched_kernel, dim3(o.count), dim3(256), 0, st,
                           reinterpret_cast<const LeafDesc*>(base + o.off));
        break;
      case 1:
        if (o.gy > 65535) return hipErrorInvalidValue;
        hipLaunchKernelGGL(gemm_f64_batched_kernel, dim3(o.gx, o.gy, o.count), dim3(256), 0, st,
                           reinterpret_cast<const GemmDesc*>(base + o.off), o.g0.ta, o.g0.tb, o.g0.alpha, o.g0.beta,
                           o.g0.flags);
        break;
      case 3:
        if (o.gy > 65535 || o.count + o.count2 > 65535) return hipErrorInvalidValue;
        hipLaunchKernelGGL(gemm_f64_batched_pair_kernel, dim3(o.gx, o.gy, o.count + o.count2), dim3(256), 0, st,
                           reinterpret_cast<const GemmDesc*>(base + o.off), o.count, o.g0,
                           reinterpret_cast<const GemmDesc*>(base + o.off2), o.g1);
        break;
      default:
        hipLaunchKernelGGL(diag_max_batched_kernel, dim3(o.count), dim3(256), 0, st,
                           reinterpret_cast<const DiagDesc*>(base + o.off));
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace qpg
