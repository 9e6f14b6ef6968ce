// Dense FP64 factorization kernels for the once-per-QP setup (gfx950 MFMA).
//
//   gemm_f64      C = alpha op(A) op(B) + beta C, 64x64 or 32x32 tiles,
//                 v_mfma_f64_16x16x4 over double-buffered LDS slabs; optional
//                 "lower only" output (SYRK-shaped updates) and k-range trimming
//                 for triangular operands.
//   chol_inv_leaf one workgroup factors a <= 64 x 64 SPD block held in MFMA
//                 accumulators and inverts the Cholesky factor (LL^T = A, X = L^{-1}).
//   chol_inv_node one workgroup runs a whole node of <= 128 rows (two leaves and
//                 the three products between them, operands in LDS).
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
typedef double v2d __attribute__((ext_vector_type(2)));

// ---- tiled FP64 GEMM ----------------------------------------------------------
// A workgroup of 256 threads (2 x 2 wavefronts) owns a BM x BN tile of C; each
// wavefront a (BM/2) x (BN/2) block of 16 x 16 v_mfma_f64_16x16x4f64 accumulators.
// The k loop runs over BK-deep slabs of op(A) and op(B) staged in LDS, two
// buffers: the global loads of slab t+1 (16-byte vectors where the operand is
// aligned) are in flight while the matrix cores work on slab t, and one barrier
// per slab separates the buffers.  Each element of C is summed in the same order
// (k = klo, klo + 4, ... through the same instruction) whatever the tile shape,
// so the shape can be chosen per launch without changing results.
constexpr int GPAD = 4;   // LDS row padding (doubles)

// BK: depth of a k slab (16 measured fastest for both tile shapes in use).
template <int BM, int BN, int BK = 16>
struct GemmTile {
  static constexpr int GK = BK;                     // k slab
  // Slabs whose global loads are in flight in registers.  The large tile serves
  // launches of at least four tiles per CU and hides load latency across its
  // workgroups (one slab ahead keeps it at 96 VGPRs, five workgroups per CU; four
  // ahead cost 150 VGPRs and 25 % at 2048^3).  The small tile serves launches too
  // small for that, so it keeps eight slabs ahead (110 VGPRs): 1024^3 in 73 us
  // against 79 us one slab ahead.
  static constexpr int S = BM * BN >= 64 * 64 ? 1 : 8;
  static constexpr int WM = BM / 2, WN = BN / 2;    // per-wavefront block
  static constexpr int FM = WM / 16, FN = WN / 16;  // MFMA blocks per wavefront
  static constexpr int LA = BM * GK / 2 / 256;      // 16-byte loads per thread, A slab
  static constexpr int LB = BN * GK / 2 / 256;      // and B slab
  static constexpr int AS = BM + GPAD, BS = BN + GPAD;
  static constexpr size_t kLdsBytes = 2 * GK * (AS + BS) * sizeof(double);
};
constexpr size_t kLds64 = GemmTile<64, 64>::kLdsBytes, kLds32 = GemmTile<32, 32>::kLdsBytes;

// Elements idx, idx+1 of row p (zero at or past lim); one 16-byte load when allowed.
__device__ __forceinline__ v2d ld_pair(const double* __restrict__ p, int idx, int lim, bool vec) {
  if (vec && idx + 1 < lim) return *reinterpret_cast<const v2d*>(p + idx);
  v2d r;
  r.x = idx < lim ? p[idx] : 0.0;
  r.y = idx + 1 < lim ? p[idx + 1] : 0.0;
  return r;
}

template <int BM, int BN, int BK = GemmTile<BM, BN>::GK>
__device__ __forceinline__ void gemm_body(int M, int N, int K, double alpha, const double* __restrict__ A, int lda,
                                          int ta, const double* __restrict__ B, int ldb, int tb, double beta,
                                          double* __restrict__ C, int ldc, int flags, int bx, int by) {
  using G = GemmTile<BM, BN, BK>;
  constexpr int GK = G::GK;
  const int i0 = by * BM, j0 = bx * BN;
  if ((flags & kOutLower) && j0 > i0 + BM - 1) return;
  extern __shared__ double lds[];
  double* As = lds;                    // [2][GK][AS]
  double* Bs = lds + 2 * GK * G::AS;   // [2][GK][BS]
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  const int wr = (wave / 2) * G::WM, wc = (wave % 2) * G::WN;
  // k range that can be nonzero for this tile
  int klo = 0, khi = K;
  if (flags & kALower) khi = min(khi, i0 + BM);  // op(A)[i][k] = 0 for k > i
  if (flags & kBUpper) khi = min(khi, j0 + BN);  // op(B)[k][j] = 0 for k > j
  if (flags & kBLower) klo = max(klo, j0);       // op(B)[k][j] = 0 for k < j
  if (flags & kAUpper) klo = max(klo, i0);       // op(A)[i][k] = 0 for k < i
  klo = klo / GK * GK;
  // 16-byte loads need 16-byte aligned rows (every slab starts at an even index)
  const bool va = ((reinterpret_cast<uintptr_t>(A) & 15) == 0) && (lda % 2 == 0);
  const bool vb = ((reinterpret_cast<uintptr_t>(B) & 15) == 0) && (ldb % 2 == 0);

  v4d acc[G::FM][G::FN];
#pragma unroll
  for (int a = 0; a < G::FM; ++a)
#pragma unroll
    for (int b = 0; b < G::FN; ++b) acc[a][b] = v4d{0, 0, 0, 0};

  // Slab t (k0 = klo + t GK) goes through registers (stage t % S, its loads issued S
  // slabs ahead) into LDS buffer t % 2; one barrier per slab.
  constexpr int S = G::S;
  v2d ra[S][G::LA], rb[S][G::LB];
  auto load = [&](int k0, v2d (&xa)[G::LA], v2d (&xb)[G::LB]) {
#pragma unroll
    for (int e = 0; e < G::LA; ++e) {
      const int v = tid + 256 * e;
      if (!ta) {  // op(A)[i][k] = A[i lda + k]: pairs along k
        const int row = v / (GK / 2), kv = v % (GK / 2), gi = i0 + row;
        xa[e] = gi < M ? ld_pair(A + (size_t)gi * lda, k0 + 2 * kv, K, va) : v2d{0, 0};
      } else {    // op(A)[i][k] = A[k lda + i]: pairs along i
        const int kr = v / (BM / 2), iv = v % (BM / 2), gk = k0 + kr;
        xa[e] = gk < K ? ld_pair(A + (size_t)gk * lda, i0 + 2 * iv, M, va) : v2d{0, 0};
      }
    }
#pragma unroll
    for (int e = 0; e < G::LB; ++e) {
      const int v = tid + 256 * e;
      if (!tb) {  // op(B)[k][j] = B[k ldb + j]: pairs along j
        const int kr = v / (BN / 2), jv = v % (BN / 2), gk = k0 + kr;
        xb[e] = gk < K ? ld_pair(B + (size_t)gk * ldb, j0 + 2 * jv, N, vb) : v2d{0, 0};
      } else {    // op(B)[k][j] = B[j ldb + k]: pairs along k
        const int col = v / (GK / 2), kv = v % (GK / 2), gj = j0 + col;
        xb[e] = gj < N ? ld_pair(B + (size_t)gj * ldb, k0 + 2 * kv, K, vb) : v2d{0, 0};
      }
    }
  };
  auto store = [&](int buf, const v2d (&xa)[G::LA], const v2d (&xb)[G::LB]) {
    double* as = As + buf * GK * G::AS;
    double* bs = Bs + buf * GK * G::BS;
#pragma unroll
    for (int e = 0; e < G::LA; ++e) {
      const int v = tid + 256 * e;
      if (!ta) {
        const int row = v / (GK / 2), kv = v % (GK / 2);
        as[(2 * kv) * G::AS + row] = xa[e].x;
        as[(2 * kv + 1) * G::AS + row] = xa[e].y;
      } else {
        const int kr = v / (BM / 2), iv = v % (BM / 2);
        *reinterpret_cast<v2d*>(as + kr * G::AS + 2 * iv) = xa[e];
      }
    }
#pragma unroll
    for (int e = 0; e < G::LB; ++e) {
      const int v = tid + 256 * e;
      if (!tb) {
        const int kr = v / (BN / 2), jv = v % (BN / 2);
        *reinterpret_cast<v2d*>(bs + kr * G::BS + 2 * jv) = xb[e];
      } else {
        const int col = v / (GK / 2), kv = v % (GK / 2);
        bs[(2 * kv) * G::BS + col] = xb[e].x;
        bs[(2 * kv + 1) * G::BS + col] = xb[e].y;
      }
    }
  };
  auto compute = [&](int buf) {
    const double* as = As + buf * GK * G::AS;
    const double* bs = Bs + buf * GK * G::BS;
#pragma unroll
    for (int kk = 0; kk < GK / 4; ++kk) {
      const int kr = kk * 4 + lane / 16;
      double af[G::FM], bf[G::FN];
#pragma unroll
      for (int a = 0; a < G::FM; ++a) af[a] = as[kr * G::AS + wr + a * 16 + lane % 16];
#pragma unroll
      for (int b = 0; b < G::FN; ++b) bf[b] = bs[kr * G::BS + wc + b * 16 + lane % 16];
#pragma unroll
      for (int a = 0; a < G::FM; ++a)
#pragma unroll
        for (int b = 0; b < G::FN; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
    }
  };

  const int T = klo < khi ? (khi - klo + GK - 1) / GK : 0;  // slabs
#pragma unroll
  for (int u = 0; u < S; ++u)
    if (u < T) load(klo + u * GK, ra[u], rb[u]);
  if (T > 0) store(0, ra[0], rb[0]);
  if (S < T) load(klo + S * GK, ra[0], rb[0]);
  __syncthreads();
  for (int t0 = 0; t0 < T; t0 += S) {
#pragma unroll
    for (int u = 0; u < S; ++u) {
      const int t = t0 + u;
      if (t < T) {
        compute(t & 1);
        // slab t + 1 from its registers into the other buffer, then slab t + 1 + S into them
        const int nx = (u + 1) % S;
        if (t + 1 < T) store((t + 1) & 1, ra[nx], rb[nx]);
        if (t + 1 + S < T) load(klo + (t + 1 + S) * GK, ra[nx], rb[nx]);
        __syncthreads();
      }
    }
  }
  // f64 16x16x4 result layout: register r of lane l holds D[4 r + l / 16][l % 16]
#pragma unroll
  for (int a = 0; a < G::FM; ++a)
#pragma unroll
    for (int b = 0; b < G::FN; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = i0 + wr + a * 16 + 4 * r + lane / 16;
        const int gj = j0 + wc + b * 16 + (lane % 16);
        if (gi < M && gj < N && (!(flags & kOutLower) || gj <= gi)) {
          double v = alpha * acc[a][b][r];
          double* cp = C + (size_t)gi * ldc + gj;
          if (beta != 0.0) v += beta * (*cp);
          *cp = v;
        }
      }
}

// Tile shape of a launch covering `tiles` tiles of 64 x 64: that shape when it
// gives every CU at least four of them, else 32 x 32 (four times as many
// workgroups: a launch with few tiles is bound by the matrix cores of the CUs it
// occupies and by unhidden load latency, not by the smaller tile's extra L2
// traffic).  Measured on FP64 A B^T: 32 x 32 wins up to n = 1024 (80 us there
// against 128 us), 64 x 64 from n = 2048 (417 us against 515 us).
static bool use_tile64(long long tiles64) { return tiles64 >= (long long)dev_info().cu_count * 4; }

// Order of the tiles of a GEMM with a triangular operand, whose tiles' k ranges
// grow or shrink along one axis: the first half of the linear block indices takes
// the tiles from the heaviest down, the second half from the lightest up, so the
// workgroups dispatched together pair a long tile with a short one.  A bijection
// of the grid; other GEMMs keep the plain order.
__device__ __forceinline__ int2 tile_of_block(int flags) {
  const int tri = flags & (kALower | kBUpper | kBLower | kAUpper);
  if (tri != kALower && tri != kBUpper && tri != kBLower && tri != kAUpper)
    return make_int2((int)blockIdx.x, (int)blockIdx.y);
  const int gx = gridDim.x, gy = gridDim.y, total = gx * gy, half = total / 2;
  const int b = (int)blockIdx.y * gx + (int)blockIdx.x;
  const int idx = b < half ? b : total - 1 - (b - half);  // rank by work, heaviest first
  if (tri == kALower) return make_int2(idx % gx, gy - 1 - idx / gx);  // work grows with the tile row
  if (tri == kAUpper) return make_int2(idx % gx, idx / gx);           // work shrinks with the tile row
  if (tri == kBUpper) return make_int2(gx - 1 - idx / gy, idx % gy);  // work grows with the tile column
  return make_int2(idx / gy, idx % gy);                               // kBLower: shrinks with the column
}

static long long active_tiles(int M, int N, int bm, int bn, int flags) {
  const long long gy = (M + bm - 1) / bm, gx = (N + bn - 1) / bn;
  if (!(flags & kOutLower)) return gx * gy;
  long long t = 0;  // tiles on or below the diagonal
  for (long long y = 0; y < gy; ++y) t += std::min(gx, (y * bm + bm - 1) / bn + 1);
  return t;
}

template <int BM, int BN>
__global__ void __launch_bounds__(256, 2) gemm_f64_kernel(int M, int N, int K, double alpha,
                                                          const double* __restrict__ A, int lda, int ta,
                                                          const double* __restrict__ B, int ldb, int tb, double beta,
                                                          double* __restrict__ C, int ldc, int flags) {
  const int2 t = tile_of_block(flags);
  gemm_body<BM, BN>(M, N, K, alpha, A, lda, ta, B, ldb, tb, beta, C, ldc, flags, t.x, t.y);
}

// One GEMM per blockIdx.z, same op/scalars for all; tiles outside a problem's
// M x N exit at once.
template <int BM, int BN>
__global__ void __launch_bounds__(256, 2) gemm_f64_batched_kernel(const GemmDesc* __restrict__ descs, int ta, int tb,
                                                               double alpha, double beta, int flags) {
  const GemmDesc g = descs[blockIdx.z];
  if ((int)blockIdx.y * BM >= g.M || (int)blockIdx.x * BN >= g.N) return;
  gemm_body<BM, BN>(g.M, g.N, g.K, alpha, g.A, g.lda, ta, g.B, g.ldb, tb, beta, g.C, g.ldc, flags, blockIdx.x,
                    blockIdx.y);
}

hipError_t gemm_f64(hipStream_t st, int ta, int tb, int M, int N, int K, double alpha, const double* A, int lda,
                    const double* B, int ldb, double beta, double* C, int ldc, int flags) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (use_tile64(active_tiles(M, N, 64, 64, flags))) {
    if ((M + 63) / 64 > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL((gemm_f64_kernel<64, 64>), dim3((N + 63) / 64, (M + 63) / 64), dim3(256), kLds64, st, M, N,
                       K, alpha, A, lda, ta, B, ldb, tb, beta, C, ldc, flags);
  } else {
    if ((M + 31) / 32 > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL((gemm_f64_kernel<32, 32>), dim3((N + 31) / 32, (M + 31) / 32), dim3(256), kLds32, st, M, N,
                       K, alpha, A, lda, ta, B, ldb, tb, beta, C, ldc, flags);
  }
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

template <int BM, int BN>
__global__ void __launch_bounds__(256, 2) gemm_f64_pair_kernel(GemmArgs g0, GemmArgs g1) {
  const GemmArgs g = blockIdx.z == 0 ? g0 : g1;
  if ((int)blockIdx.y * BM >= g.M || (int)blockIdx.x * BN >= g.N) return;
  gemm_body<BM, BN>(g.M, g.N, g.K, g.alpha, g.A, g.lda, g.ta, g.B, g.ldb, g.tb, g.beta, g.C, g.ldc, g.flags,
                    blockIdx.x, blockIdx.y);
}

static hipError_t gemm_f64_pair(hipStream_t st, const GemmArgs& g0, const GemmArgs& g1) {
  const int mx = std::max(g0.M, g1.M), nx = std::max(g0.N, g1.N);
  if (mx <= 0 || nx <= 0) return hipSuccess;
  const long long t0 = active_tiles(g0.M, g0.N, 64, 64, g0.flags), t1 = active_tiles(g1.M, g1.N, 64, 64, g1.flags);
  const long long fill = (long long)dev_info().cu_count * 2;
  if (t0 >= fill && t1 >= fill) {
    // each fills the chip alone: two launches, each with its own tile shape and
    // tile order (a shared grid would leave half the output-lower tiles idle and
    // the triangular operand's tiles unsorted)
    hipError_t e = gemm_f64(st, g0.ta, g0.tb, g0.M, g0.N, g0.K, g0.alpha, g0.A, g0.lda, g0.B, g0.ldb, g0.beta, g0.C,
                            g0.ldc, g0.flags);
    if (e != hipSuccess) return e;
    return gemm_f64(st, g1.ta, g1.tb, g1.M, g1.N, g1.K, g1.alpha, g1.A, g1.lda, g1.B, g1.ldb, g1.beta, g1.C, g1.ldc,
                    g1.flags);
  }
  const long long tb = t0 + t1;
  if (use_tile64(tb)) {
    if ((mx + 63) / 64 > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL((gemm_f64_pair_kernel<64, 64>), dim3((nx + 63) / 64, (mx + 63) / 64, 2), dim3(256), kLds64,
                       st, g0, g1);
  } else {
    if ((mx + 31) / 32 > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL((gemm_f64_pair_kernel<32, 32>), dim3((nx + 31) / 32, (mx + 31) / 32, 2), dim3(256), kLds32,
                       st, g0, g1);
  }
  return hipGetLastError();
}

// Batched form: blockIdx.z < count0 takes d0[z] with o0, the rest d1[z - count0] with o1.
template <int BM, int BN>
__global__ void __launch_bounds__(256, 2) gemm_f64_batched_pair_kernel(const GemmDesc* __restrict__ d0, int count0,
                                                                    GemmOp o0, const GemmDesc* __restrict__ d1,
                                                                    GemmOp o1) {
  const int z = blockIdx.z;
  const GemmDesc g = z < count0 ? d0[z] : d1[z - count0];
  const GemmOp o = z < count0 ? o0 : o1;
  if ((int)blockIdx.y * BM >= g.M || (int)blockIdx.x * BN >= g.N) return;
  gemm_body<BM, BN>(g.M, g.N, g.K, o.alpha, g.A, g.lda, o.ta, g.B, g.ldb, o.tb, o.beta, g.C, g.ldc, o.flags,
                    blockIdx.x, blockIdx.y);
}

// ---------------------------------------------------------------------------
constexpr int LEAF = 64;

// A pivot is rejected when it is not positive or falls below kPivRel times the
// largest diagonal entry of the whole input matrix (*dmax): for a singular
// matrix the computed pivot is a rounding residue of order eps * ||A||.
constexpr double kPivRel = 1e-13;

// Leaf: right-looking LDL^T of a <= 64 x 64 SPD block A = L_1 D L_1^T, giving
// X = L^{-1} = D^{-1/2} L_1^{-1} for the Cholesky factor L = L_1 D^{1/2} (X starts
// as I and takes the same row operations, so it stays lower triangular; L itself
// is not stored, the callers use only its inverse).  The block is held as 16 x 16
// tiles in the accumulators of v_mfma_f64_16x16x4f64: wavefront I owns tile row
// I of A and of X (tiles K <= I).  Columns are eliminated four at a time, one
// barrier per column block J (columns j0 = 4J .. 4J+3): the owners publish those
// columns of A and rows j0 .. j0+3 of X in LDS; then every lane eliminates the
// 4 x 4 diagonal block itself, and each wavefront passes the rows of its operand
// tiles through the block's four steps (eliminated values ev_i and multipliers
// cf_i = ev_i / d) and the block's rows of X through their own steps (xf).  The
// updates of the trailing columns, a_ik -= sum_p cf_ip ev_kp, and of the rows of
// X below the block, x_i -= sum_p cf_ip xf_p, are rank-4 products: one MFMA per
// 16 x 16 tile, with the k = 4 operand slots holding p.  Each wavefront runs
// alone on its SIMD, so the code is shaped for latency: the wavefront index is a
// scalar (uniform branches), lane selections are selects, and the reciprocals of
// the pivots and of their square roots are Newton-refined hardware estimates
// instead of IEEE divisions.

// LDS of the leaf elimination.
struct alignas(16) LeafLds {
  double pan[2][LEAF][4];   // columns 4J..4J+3 of A (rows >= 4J), double-buffered
  double xrow[2][4][LEAF];  // rows 4J..4J+3 of X as they enter block J, double-buffered
  double rs[LEAF];          // 1 / sqrt(pivot)
};

// Accumulator layout of a 64 x 64 block over the four wavefronts: wavefront I
// holds tiles (I, K), K <= I; register r of lane l holds tile entry (4 r + l / 16, l % 16).
__device__ __forceinline__ void leaf_load(const double* __restrict__ A, int lda, int nb, v4d (&accA)[4],
                                          v4d (&accX)[4]) {
  const int tid = threadIdx.x, l = tid & 63, lr = l >> 4, lc = l & 15;
  const int I = __builtin_amdgcn_readfirstlane(tid >> 6);
#pragma unroll
  for (int K = 0; K < 4; ++K)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * I + 4 * r + lr, k = 16 * K + lc;
      accA[K][r] = (K <= I && i < nb && k <= i) ? A[(size_t)i * lda + k] : 0.0;
      accX[K][r] = (i == k && i < nb) ? 1.0 : 0.0;
    }
}

// v[s] for a lane-dependent s in 0..3 (selects; no indexed register access).
__device__ __forceinline__ double sel4(double v0, double v1, double v2, double v3, int s) {
  double r = v0;
  r = s == 1 ? v1 : r;
  r = s == 2 ? v2 : r;
  r = s == 3 ? v3 : r;
  return r;
}

// 1 / d and 1 / sqrt(d) for a positive normal d: the hardware estimate and two
// Newton steps (relative error a few units in the last place).
__device__ __forceinline__ double rcp_nr(double d) {
  double y = __builtin_amdgcn_rcp(d);
  double e = fma(-d, y, 1.0);
  y = fma(y, e, y);
  e = fma(-d, y, 1.0);
  return fma(y, e, y);
}
__device__ __forceinline__ double rsq_nr(double d) {
  double y = __builtin_amdgcn_rsq(d);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-d * y, y, 1.0);  // 1 - d y^2
    y = fma(0.5 * y, e, y);
  }
  return y;
}

// Elimination of the accumulators loaded by leaf_load; keeps X = L_1^{-1}
// (unscaled) in accX and 1 / sqrt(d) in sh.rs (L itself is not an output: the
// callers use only the inverse factor).  Returns true when a pivot is rejected.
__device__ __forceinline__ bool leaf_elim(LeafLds& sh, int nb, const double* __restrict__ dmax, v4d (&accA)[4],
                                          v4d (&accX)[4]) {
  const int tid = threadIdx.x, l = tid & 63, lr = l >> 4, lc = l & 15;
  const int I = __builtin_amdgcn_readfirstlane(tid >> 6);  // wavefront index, uniform
  const double pmin = kPivRel * (*dmax);
  bool bad = false;
  const int nblk = (nb + 3) / 4;
#pragma unroll
  for (int K0 = 0; K0 < 4; ++K0) {
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int J = 4 * K0 + jj;
      if (J < nblk) {
        const int buf = J & 1, j0 = 4 * J, c0 = 4 * jj;
        if (I >= K0 && lc >= c0 && lc < c0 + 4) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = 16 * I + 4 * r + lr;
            if (i >= j0) sh.pan[buf][i][lc - c0] = accA[K0][r];
          }
        }
        if (I == K0) {
#pragma unroll
          for (int K = 0; K <= K0; ++K) sh.xrow[buf][lr][16 * K + lc] = accX[K][jj];
        }
        __syncthreads();
        // Diagonal block: E[i][q] (q <= i) ends as the eliminated value of a_{j0+i, j0+q}
        // at its own column step (E[p][p] is the pivot d_p).
        double E[4][4], dinv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int q = 0; q < 4; ++q) E[i][q] = q <= i ? sh.pan[buf][j0 + i][q] : 0.0;
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          // a pivot past the block's end (zero row and column) or a rejected one
          // (the same decision in every thread) is replaced by 1
          const double d = E[p][p];
          const bool live = j0 + p < nb, ok = d > pmin && isfinite(d);
          bad = bad || (live && !ok);
          E[p][p] = live && ok ? d : 1.0;
          dinv[p] = rcp_nr(E[p][p]);
#pragma unroll
          for (int i = p + 1; i < 4; ++i) {
            const double coef = E[i][p] * dinv[p];
#pragma unroll
            for (int k = p + 1; k <= i; ++k) E[i][k] -= coef * E[k][p];
          }
        }
        if (I == 0 && lc == 0) sh.rs[j0 + lr] = rsq_nr(sel4(E[0][0], E[1][1], E[2][2], E[3][3], lr));
        if (I >= K0) {
          // Row 16 K + lc of each operand tile K (K0 <= K <= I) through the block's
          // four steps; this lane keeps slot p = lr: the eliminated value (B operand)
          // and, for its own tile row, the negated multiplier (A operand).  Rows at
          // or above the block contribute zero.
          double aop = 0.0, bop[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int K = K0; K < 4; ++K) {
            if (K > I) continue;
            const int row = 16 * K + lc;
            const bool below = row > j0 + 3;
            const v2d g01 = *reinterpret_cast<const v2d*>(&sh.pan[buf][row][0]);
            const v2d g23 = *reinterpret_cast<const v2d*>(&sh.pan[buf][row][2]);
            double g[4] = {g01.x, g01.y, g23.x, g23.y}, cf[4];
#pragma unroll
            for (int p = 0; p < 4; ++p) {
#pragma unroll
              for (int pp = 0; pp < p; ++pp) g[p] -= cf[pp] * E[p][pp];
              cf[p] = g[p] * dinv[p];
            }
            bop[K] = below ? sel4(g[0], g[1], g[2], g[3], lr) : 0.0;
            if (K == I) aop = below ? -sel4(cf[0], cf[1], cf[2], cf[3], lr) : 0.0;
          }
#pragma unroll
          for (int K = K0; K < 4; ++K)
            if (K <= I) accA[K] = __builtin_amdgcn_mfma_f64_16x16x4f64(aop, bop[K], accA[K], 0, 0, 0);
          // X: column 16 K + lc of the block's rows after their own steps (slot lr);
          // rows below take x_i -= sum_p cf_ip xf_p, the block's rows become xf
#pragma unroll
          for (int K = 0; K <= K0; ++K) {
            const int col = 16 * K + lc;
            double f[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              f[q] = sh.xrow[buf][q][col];
#pragma unroll
              for (int qq = 0; qq < q; ++qq) f[q] -= (E[q][qq] * dinv[qq]) * f[qq];
            }
            const double xv = sel4(f[0], f[1], f[2], f[3], lr);
            accX[K] = __builtin_amdgcn_mfma_f64_16x16x4f64(aop, xv, accX[K], 0, 0, 0);
            if (I == K0) accX[K][jj] = xv;
          }
        }
      }
    }
  }
  __syncthreads();
  return bad;
}

// X = D^{-1/2} L_1^{-1} (rows and columns < nb) into X, and with xs into LDS
// (64 x ldxs).
__device__ __forceinline__ void leaf_store_x(const LeafLds& sh, double* __restrict__ X, int ldx, int nb,
                                             const v4d (&accX)[4], double* xs = nullptr, int ldxs = 0) {
  const int tid = threadIdx.x, l = tid & 63, lr = l >> 4, lc = l & 15;
  const int I = __builtin_amdgcn_readfirstlane(tid >> 6);
#pragma unroll
  for (int K = 0; K < 4; ++K) {
    if (K > I) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * I + 4 * r + lr, k = 16 * K + lc;
      if (i >= nb || k >= nb) continue;
      const double x = accX[K][r] * sh.rs[i];
      X[(size_t)i * ldx + k] = x;
      if (xs) xs[i * ldxs + k] = x;
    }
  }
}

__device__ __forceinline__ void chol_inv_leaf_body(double* __restrict__ A, int lda, double* __restrict__ X,
                                                    int ldx, int nb, int* __restrict__ info, int code,
                                                    const double* __restrict__ dmax) {
  __shared__ LeafLds sh;
  v4d accA[4], accX[4];
  leaf_load(A, lda, nb, accA, accX);
  const bool bad = leaf_elim(sh, nb, dmax, accA, accX);
  leaf_store_x(sh, X, ldx, nb, accX);
  if (threadIdx.x == 0 && bad) *info = code;
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

// Node of 64 < n <= 128 rows in one workgroup, the recursive driver's steps
// for one node: (L11, X11) = leaf(A11); L21 = A21 X11^T; A22 -= L21 L21^T and
// T = L21 X11; (L22, X22) = leaf(A22); X21 = -X22 T.  A21, X11, L21, T and X22
// stay in LDS, and A22 is updated in the accumulators the second leaf starts
// from, so a node costs one launch instead of two leaves and three GEMMs.
constexpr int NLD = LEAF + 1;  // LDS row stride (doubles)

// acc[K] (tile (I, K) of a 64 x 64 product, wavefront I; K <= kmax_tile) += sign *
// sum_k opA(i, k) opB(k, j) over k < 64, operands read from LDS.
template <typename FA, typename FB>
__device__ __forceinline__ void node_mm(v4d (&acc)[4], int ktiles, double sign, FA&& opA, FB&& opB) {
  const int tid = threadIdx.x, l = tid & 63, lr = l >> 4, lc = l & 15;
  const int I = __builtin_amdgcn_readfirstlane(tid >> 6);
#pragma unroll 4
  for (int k0 = 0; k0 < LEAF; k0 += 4) {
    const double a = sign * opA(16 * I + lc, k0 + lr);
#pragma unroll
    for (int K = 0; K < 4; ++K)
      if (K < ktiles) acc[K] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, opB(k0 + lr, 16 * K + lc), acc[K], 0, 0, 0);
  }
}

struct NodeShared {
  LeafLds leaf;
  double a[LEAF * NLD];   // A21, later X22
  double x[LEAF * NLD];   // X11
  double lt[LEAF * NLD];  // L21
  double t[LEAF * NLD];   // T
};

__device__ __forceinline__ void chol_inv_node_body(double* __restrict__ A, int lda, double* __restrict__ X, int ldx,
                                                   int n, int* __restrict__ info, int code,
                                                   const double* __restrict__ dmax) {
  __shared__ NodeShared sh;
  const int tid = threadIdx.x, l = tid & 63, lr = l >> 4, lc = l & 15;
  const int I = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int n2 = n - LEAF;
  double* A21 = A + (size_t)LEAF * lda;
  double* A22 = A21 + LEAF;
  double* X21 = X + (size_t)LEAF * ldx;
  double* X22 = X21 + LEAF;
  // A21 into LDS (rows past n2 zero); X11's tile zeroed, the first leaf writes its
  // lower triangle and the products below read all of it
  for (int e = tid; e < LEAF * LEAF; e += 256) {
    const int i = e / LEAF, k = e % LEAF;
    sh.a[i * NLD + k] = i < n2 ? A21[(size_t)i * lda + k] : 0.0;
    sh.x[i * NLD + k] = 0.0;
  }
  v4d accA[4], accX[4];
  leaf_load(A, lda, LEAF, accA, accX);
  bool bad = leaf_elim(sh.leaf, LEAF, dmax, accA, accX);
  leaf_store_x(sh.leaf, X, ldx, LEAF, accX, sh.x, NLD);
  __syncthreads();
  // L21 = A21 X11^T
  v4d acc[4];
#pragma unroll
  for (int K = 0; K < 4; ++K) acc[K] = v4d{0, 0, 0, 0};
  node_mm(acc, 4, 1.0, [&](int i, int k) { return sh.a[i * NLD + k]; },
          [&](int k, int j) { return sh.x[j * NLD + k]; });
#pragma unroll
  for (int K = 0; K < 4; ++K)
#pragma unroll
    for (int r = 0; r < 4; ++r) sh.lt[(16 * I + 4 * r + lr) * NLD + 16 * K + lc] = acc[K][r];
  __syncthreads();
  // A22 -= L21 L21^T on the accumulators of the second leaf (tiles K <= I)
  leaf_load(A22, lda, n2, accA, accX);
  node_mm(accA, I + 1, -1.0, [&](int i, int k) { return sh.lt[i * NLD + k]; },
          [&](int k, int j) { return sh.lt[j * NLD + k]; });
  // T = L21 X11
#pragma unroll
  for (int K = 0; K < 4; ++K) acc[K] = v4d{0, 0, 0, 0};
  node_mm(acc, 4, 1.0, [&](int i, int k) { return sh.lt[i * NLD + k]; },
          [&](int k, int j) { return sh.x[k * NLD + j]; });
#pragma unroll
  for (int K = 0; K < 4; ++K)
#pragma unroll
    for (int r = 0; r < 4; ++r) sh.t[(16 * I + 4 * r + lr) * NLD + 16 * K + lc] = acc[K][r];
  // (L22, X22) = leaf(A22); X22 also into LDS (over A21, which is no longer read)
  bad = leaf_elim(sh.leaf, n2, dmax, accA, accX) || bad;
  for (int e = tid; e < LEAF * LEAF; e += 256) sh.a[(e / LEAF) * NLD + e % LEAF] = 0.0;
  __syncthreads();
  leaf_store_x(sh.leaf, X22, ldx, n2, accX, sh.a, NLD);
  __syncthreads();
  // X21 = -X22 T
#pragma unroll
  for (int K = 0; K < 4; ++K) acc[K] = v4d{0, 0, 0, 0};
  node_mm(acc, 4, -1.0, [&](int i, int k) { return sh.a[i * NLD + k]; },
          [&](int k, int j) { return sh.t[k * NLD + j]; });
#pragma unroll
  for (int K = 0; K < 4; ++K)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * I + 4 * r + lr, j = 16 * K + lc;
      if (i < n2) X21[(size_t)i * ldx + j] = acc[K][r];
    }
  if (tid == 0 && bad) *info = code;
}

__global__ void __launch_bounds__(256) chol_inv_node_kernel(double* __restrict__ A, int lda, double* __restrict__ X,
                                                            int ldx, int n, int* __restrict__ info, int code,
                                                            const double* __restrict__ dmax) {
  chol_inv_node_body(A, lda, X, ldx, n, info, code, dmax);
}

__global__ void __launch_bounds__(256) chol_inv_node_batched_kernel(const LeafDesc* __restrict__ descs) {
  const LeafDesc d = descs[blockIdx.x];
  chol_inv_node_body(d.A, d.lda, d.X, d.ldx, d.nb, d.info, d.code, d.dmax);
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
  if (n <= 2 * LEAF) {  // split at LEAF like the general node, in one workgroup
    hipLaunchKernelGGL(chol_inv_node_kernel, dim3(1), dim3(256), 0, st, A, lda, X, ldx, n, info, code, dmax);
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
  long long tiles = 0;
  for (const GemmDesc& g : d) tiles += active_tiles(g.M, g.N, 64, 64, flags);
  Op o{};
  o.kind = 1;
  o.count = (int)d.size();
  o.tile64 = use_tile64(tiles) ? 1 : 0;
  const int bt = o.tile64 ? 64 : 32;
  o.gx = (nx + bt - 1) / bt;
  o.gy = (mx + bt - 1) / bt;
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
  long long tiles = 0;
  for (const GemmDesc& g : d0) tiles += active_tiles(g.M, g.N, 64, 64, o0.flags);
  for (const GemmDesc& g : d1) tiles += active_tiles(g.M, g.N, 64, 64, o1.flags);
  Op o{};
  o.kind = 3;
  o.count = (int)d0.size();
  o.count2 = (int)d1.size();
  o.tile64 = use_tile64(tiles) ? 1 : 0;
  const int bt = o.tile64 ? 64 : 32;
  o.gx = (nx + bt - 1) / bt;
  o.gy = (mx + bt - 1) / bt;
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
  if (len <= 2 * LEAF) {
    // a job's part of the node: a leaf when it has at most LEAF rows, else a fused node
    std::vector<LeafDesc> leaves, nodes;
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
      (nb <= LEAF ? leaves : nodes).push_back(l);
    }
    for (int kind : {0, 4}) {
      const std::vector<LeafDesc>& d = kind == 0 ? leaves : nodes;
      if (d.empty()) continue;
      Op o{};
      o.kind = kind;
      o.count = (int)d.size();
      o.off = push(d);
      ops_.push_back(o);
    }
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
      case 4:
        hipLaunchKernelGGL(chol_inv_node_batched_kernel, dim3(o.count), dim3(256), 0, st,
                           reinterpret_cast<const LeafDesc*>(base + o.off));
        break;
      case 1: {
        if (o.gy > 65535) return hipErrorInvalidValue;
        const GemmDesc* d = reinterpret_cast<const GemmDesc*>(base + o.off);
        if (o.tile64)
          hipLaunchKernelGGL((gemm_f64_batched_kernel<64, 64>), dim3(o.gx, o.gy, o.count), dim3(256), kLds64, st, d,
                             o.g0.ta, o.g0.tb, o.g0.alpha, o.g0.beta, o.g0.flags);
        else
          hipLaunchKernelGGL((gemm_f64_batched_kernel<32, 32>), dim3(o.gx, o.gy, o.count), dim3(256), kLds32, st, d,
                             o.g0.ta, o.g0.tb, o.g0.alpha, o.g0.beta, o.g0.flags);
        break;
      }
      case 3: {
        if (o.gy > 65535 || o.count + o.count2 > 65535) return hipErrorInvalidValue;
        const GemmDesc* d0 = reinterpret_cast<const GemmDesc*>(base + o.off);
        const GemmDesc* d1 = reinterpret_cast<const GemmDesc*>(base + o.off2);
        if (o.tile64)
          hipLaunchKernelGGL((gemm_f64_batched_pair_kernel<64, 64>), dim3(o.gx, o.gy, o.count + o.count2),
                             dim3(256), kLds64, st, d0, o.count, o.g0, d1, o.g1);
        else
          hipLaunchKernelGGL((gemm_f64_batched_pair_kernel<32, 32>), dim3(o.gx, o.gy, o.count + o.count2),
                             dim3(256), kLds32, st, d0, o.count, o.g0, d1, o.g1);
        break;
      }
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
