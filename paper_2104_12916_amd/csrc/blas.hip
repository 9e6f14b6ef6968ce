// Dense FP64 factorization kernels for the once-per-QP setup (gfx950 MFMA).
//
//   gemm_f64      C = alpha op(A) op(B) + beta C, 64x64 tiles, v_mfma_f64_16x16x4
//                 through LDS; optional "lower only" output (SYRK-shaped updates)
//                 and k-range trimming for triangular operands.
//   chol_inv_leaf one workgroup factors a <= 64 x 64 SPD block in LDS and inverts
//                 the Cholesky factor (LL^T = A, X = L^{-1}).
//   chol_inv      recursive blocked driver: with A = [A11 .; A21 A22],
//                   (L11, X11) = chol_inv(A11);  L21 = A21 X11^T;
//                   A22 -= L21 L21^T;            (L22, X22) = chol_inv(A22);
//                   X21 = -X22 (L21 X11),
//                 so almost every flop runs in the MFMA GEMM.
#include "kernels.hpp"

namespace qpg {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int GB = 64;   // tile
constexpr int GK = 16;   // k step

__global__ void __launch_bounds__(256) gemm_f64_kernel(int M, int N, int K, double alpha, const double* __restrict__ A,
                                                       int lda, int ta, const double* __restrict__ B, int ldb, int tb,
                                                       double beta, double* __restrict__ C, int ldc, int flags) {
  const int i0 = blockIdx.y * GB, j0 = blockIdx.x * GB;
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

hipError_t gemm_f64(hipStream_t st, int ta, int tb, int M, int N, int K, double alpha, const double* A, int lda,
                    const double* B, int ldb, double beta, double* C, int ldc, int flags) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if ((M + GB - 1) / GB > 65535) return hipErrorInvalidValue;
  dim3 grid((N + GB - 1) / GB, (M + GB - 1) / GB);
  hipLaunchKernelGGL(gemm_f64_kernel, grid, dim3(256), 0, st, M, N, K, alpha, A, lda, ta, B, ldb, tb, beta, C, ldc,
                     flags);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
constexpr int LEAF = 64;

// A pivot is rejected when it is not positive or falls below kPivRel times the
// largest diagonal entry of the whole input matrix (*dmax): for a singular
// matrix the computed pivot is a rounding residue of order eps * ||A||.
constexpr double kPivRel = 1e-13;

__global__ void __launch_bounds__(256) chol_inv_leaf_kernel(double* __restrict__ A, int lda, double* __restrict__ X,
                                                            int ldx, int nb, int* __restrict__ info, int code,
                                                            const double* __restrict__ dmax) {
  __shared__ double L[LEAF][LEAF + 1];
  __shared__ double Xs[LEAF][LEAF + 1];
  __shared__ int bad;
  const int tid = threadIdx.x;
  const double pmin = kPivRel * (*dmax);
  if (tid == 0) bad = 0;
  for (int idx = tid; idx < LEAF * LEAF; idx += blockDim.x) {
    int i = idx / LEAF, k = idx % LEAF;
    L[i][k] = (i < nb && k <= i) ? A[(size_t)i * lda + k] : 0.0;
    Xs[i][k] = 0.0;
  }
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    double piv = L[j][j];
    __syncthreads();
    if (!(piv > pmin) || !isfinite(piv)) {
      if (tid == 0) bad = 1;
      piv = 1.0;
    }
    double dj = sqrt(piv);
    if (tid == 0) L[j][j] = dj;
    for (int i = j + 1 + tid; i < nb; i += blockDim.x) L[i][j] = L[i][j] / dj;
    __syncthreads();
    for (int idx = tid; idx < nb * nb; idx += blockDim.x) {
      int i = idx / nb, k = idx % nb;
      if (k > j && k <= i) L[i][k] -= L[i][j] * L[k][j];
    }
    __syncthreads();
  }
  // X = L^{-1}, one column per thread (forward substitution on unit vectors)
  if (tid < nb) {
    const int c = tid;
    Xs[c][c] = 1.0 / L[c][c];
    for (int i = c + 1; i < nb; ++i) {
      double s = 0.0;
      for (int k = c; k < i; ++k) s += L[i][k] * Xs[k][c];
      Xs[i][c] = -s / L[i][i];
    }
  }
  __syncthreads();
  for (int idx = tid; idx < nb * nb; idx += blockDim.x) {
    int i = idx / nb, k = idx % nb;
    if (k <= i) A[(size_t)i * lda + k] = L[i][k];
    X[(size_t)i * ldx + k] = Xs[i][k];
  }
  if (tid == 0 && bad) *info = code;
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

// Recursive body.  A: n x n (lower part read, overwritten with scratch), X: n x n
// output (upper part must be zero on entry), tmp: at least (n/2 + 64) * n doubles.
static hipError_t chol_inv_rec(hipStream_t st, double* A, int lda, double* X, int ldx, int n, double* tmp,
                               int* info, int code, const double* dmax) {
  hipError_t e;
  if (n <= LEAF) {
    hipLaunchKernelGGL(chol_inv_leaf_kernel, dim3(1), dim3(256), 0, st, A, lda, X, ldx, n, info, code, dmax);
    return hipGetLastError();
  }
  int n1 = ((n / 2) + LEAF - 1) / LEAF * LEAF;
  if (n1 >= n) n1 = n - LEAF;
  int n2 = n - n1;
  double* A11 = A;
  double* A21 = A + (size_t)n1 * lda;
  double* A22 = A21 + n1;
  double* X11 = X;
  double* X21 = X + (size_t)n1 * ldx;
  double* X22 = X21 + n1;
  if ((e = chol_inv_rec(st, A11, lda, X11, ldx, n1, tmp, info, code, dmax)) != hipSuccess) return e;
  // L21 = A21 X11^T  (op(B) = X11^T is upper triangular) -> stored in X21
  if ((e = gemm_f64(st, 0, 1, n2, n1, n1, 1.0, A21, lda, X11, ldx, 0.0, X21, ldx, kBUpper)) != hipSuccess) return e;
  // A22 -= L21 L21^T (lower part only)
  if ((e = gemm_f64(st, 0, 1, n2, n2, n1, -1.0, X21, ldx, X21, ldx, 1.0, A22, lda, kOutLower)) != hipSuccess) return e;
  if ((e = chol_inv_rec(st, A22, lda, X22, ldx, n2, tmp, info, code, dmax)) != hipSuccess) return e;
  // tmp = L21 X11 (X11 lower), then X21 = -X22 tmp (X22 lower)
  if ((e = gemm_f64(st, 0, 0, n2, n1, n1, 1.0, X21, ldx, X11, ldx, 0.0, tmp, n1, kBLower)) != hipSuccess) return e;
  if ((e = gemm_f64(st, 0, 0, n2, n1, n2, -1.0, X22, ldx, tmp, n1, 0.0, X21, ldx, kALower)) != hipSuccess) return e;
  return hipSuccess;
}

// Largest diagonal entry of A (n x n) into *out; one workgroup.
__global__ void __launch_bounds__(256) diag_max_kernel(const double* __restrict__ A, int lda, int n,
                                                       double* __restrict__ out) {
  __shared__ double sh[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) m = fmax(m, A[(size_t)i * lda + i]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
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

}  // namespace qpg
