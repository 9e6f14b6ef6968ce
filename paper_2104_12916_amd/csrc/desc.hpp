// Per-problem descriptors of the batched launches: one record per QP (and per
// sweep), so a single launch can stream the matrices of many QPs of different
// sizes.  A launch over a list of descriptors gets a prefix table of block
// counts; block b serves descriptor j with prefix[j] <= b < prefix[j + 1].
#pragma once
#include <vector>

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

// Block b of a flattened batched launch: its descriptor j and its index among
// that descriptor's blocks.  The prefix table of a launch holds the ndesc
// first-block offsets followed by one entry per block, local << 16 | j (see
// with_block_map), so a workgroup finds its descriptor with one load instead of
// a binary search of dependent loads.
struct DescBlock {
  int j, local;
};
__device__ __forceinline__ DescBlock desc_of_block(const int* __restrict__ prefix, int ndesc, int b) {
  const int e = prefix[ndesc + b];
  return DescBlock{e & 0xffff, e >> 16};
}

// The prefix table of a launch over `total` blocks as it is uploaded: the
// first-block offsets, then the block map.  Empty when the encoding does not fit
// (more than 65536 descriptors or 32768 blocks of one descriptor).
inline std::vector<int> with_block_map(const std::vector<int>& prefix, int total) {
  std::vector<int> out(prefix);
  out.reserve(prefix.size() + (size_t)total);
  const int nd = (int)prefix.size();
  if (nd > 65536) return {};
  for (int j = 0; j < nd; ++j) {
    const int end = j + 1 < nd ? prefix[j + 1] : total;
    if (end - prefix[j] > 32768) return {};
    for (int b = prefix[j]; b < end; ++b) out.push_back(((b - prefix[j]) << 16) | j);
  }
  if ((int)out.size() != nd + total) return {};
  return out;
}

}  // namespace qpg
