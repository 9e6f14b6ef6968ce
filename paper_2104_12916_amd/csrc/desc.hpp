// Per-problem descriptors of the batched launches: one record per QP (and per
// sweep), so a single launch can stream the matrices of many QPs of different
// sizes.  A launch over a list of descriptors gets a prefix table of block
// counts; block b serves descriptor j with prefix[j] <= b < prefix[j + 1].
#pragma once
#include "common.hpp"

namespace qpg {

// y = alpha * A x [with rows >= nsplit negated] + beta * y0 over rows of A.
template <typename T>
struct RowsDesc {
  const T* A;
  const T* x;
  T* y;
  const T* y0;
  const int* skip;  // nonzero: the whole sweep is skipped (stopped CG solve)
  T alpha, beta;
  int lda, m, k, shape, nsplit;
  int nblocks;      // workgroups serving this sweep
};

// Column sweep y = alpha * A^T x + beta * y0: first pass over (tile, chunk)
// blocks writing part[chunk * ps + col], second pass over groups of columns.
template <typename T>
struct ColsDesc {
  const T* A;
  const T* x;
  T* part;
  T* y;
  const T* y0;
  const int* skip;
  T alpha, beta;
  int lda, m, k, shape;
  int rpc, nchunks, tiles;  // rows per chunk, chunks, 64-lane column tiles
  int nblocks;              // first pass: tiles * nchunks
  int rblocks;              // second pass: ceil(k / 16)
};

// One-pass w = M^T Sigma M u of one QP: G workgroups write partials
// part[g * ldp + j] (j < n), then rblocks workgroups add them into w.
template <typename T>
struct SymDesc {
  const T* M;      // L^{-1} (N x ldm); its first n columns are M
  const T* u;
  T* w;
  T* part;
  const int* skip;
  int ldm, N, n, ldp, G;
  int rblocks;     // ceil(n / 16)
};

// One CG solve of the reduced system (the vectors of one QP).
template <typename T>
struct PcgDesc {
  const T* C;     // m2 x n, leading dimension ldc; null: C = I (m2 = n)
  const T* w;     // input of the q sweep: w = [I 0] K0^{-1} [C^T p; 0]
  const T* dvec;  // diag(D)
  const T* wts;   // weights of the stop test (nu) or null
  const T* b;     // right-hand side
  T *x, *r, *z, *p, *q;
  double* bpart;  // per-workgroup partials of p^T q (qblocks entries)
  PcgScalars* sc;
  double rtol, wtol;
  int maxit;
  int ldc, n, m2, prec;
  int qblocks;    // workgroups of the q = C w + D p sweep
  int stage;      // 1: w staged in LDS; 0: w read from global memory (zero-padded to ldc)
};

// Map a flattened block index to its descriptor (binary search in prefix).
__device__ __forceinline__ int desc_of_block(const int* __restrict__ prefix, int ndesc, int b) {
  int lo = 0, hi = ndesc - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

}  // namespace qpg
