// Internal launcher declarations (not part of the C ABI).
#pragma once
#include <vector>

#include "common.hpp"
#include "desc.hpp"

namespace qpg {

// gemv.hip -----------------------------------------------------------------
template <typename T>
hipError_t launch_gemv_rows(hipStream_t st, const T* A, int lda, int m, int k, int shape, const T* x, T* y, T alpha,
                            T beta, const T* y0, int nsplit, const int* skip, int tag = 0,
                            const EventPair* ev = nullptr);
template <typename T>
hipError_t launch_gemv_cols(hipStream_t st, const T* A, int lda, int m, int k, int shape, const T* x, T* y, T alpha,
                            T beta, const T* y0, const GemvWork<T>& w, const int* skip, int tag = 0,
                            const EventPair* ev = nullptr);
template <typename T>
void gemv_cols_plan(int m, int k, int& rows_per_chunk, int& nchunks, int& tiles, int target_blocks);
template <typename T>
int gemv_rows_grid(int m);
template <typename T>
size_t rows_smem_bytes(int m, int k, int shape, int lda);
size_t gemv_cols_part_elems(int max_ld);
// one-pass w = M^T Sigma M u (M = L^{-1}[:, :n], N x n lower trapezoid, Sigma =
// diag(I_n, -I_{N-n})): the sweep writes one partial of w per workgroup into
// part (G x k0_sym_ldp(n)), the reduce adds them in workgroup order into w
template <typename T>
int k0_sym_max_n();
template <typename T>
int k0_sym_grid(int N, int n);
int k0_sym_ldp(int n);
size_t k0_sym_part_elems(int n);  // partial elements for any tune().sym_wg
// Workgroups of the sum of the one-pass partials of an n-column product.
int k0_sym_reduce_grid(int n);
// The same sum inside the folded CG step (pcg.hpp): with the partials of
// p^T q = u^T w + p_new^T D p_new into al (one per workgroup), or, over the
// partials of the P_H apply (N = n = m2), with the partials of r^T z into rz.
template <typename T>
hipError_t launch_k0_sym_reduce_fold(hipStream_t st, int N, int n, const T* part, T* w, const PcgScalars* sc,
                                     const T* u, const T* z, const T* p, const T* dvec, int m2, double* al, int nal,
                                     const EventPair* ev);
template <typename T>
hipError_t launch_ph_reduce_fold(hipStream_t st, int m2, const T* part, T* z, const PcgScalars* sc, const T* r,
                                 double* rz, int nrz, const EventPair* ev);
template <typename T>
hipError_t launch_k0_sym_sweep(hipStream_t st, const T* M, int ldm, int N, int n, const T* u, T* part,
                               size_t part_elems, const int* skip, const EventPair* ev = nullptr);
template <typename T>
hipError_t launch_k0_sym_reduce(hipStream_t st, int N, int n, const T* part, T* w, const int* skip,
                                const EventPair* ev = nullptr);
// batched one-pass product over SymDesc lists: K = register-row width for the
// widest n of the list (k0_sym_width), workgroups per QP from bk0_sym_grid
template <typename T>
int bk0_sym_grid(int N, int n);
template <typename T>
int k0_sym_width(int n);
template <typename T>
bool fill_sym_desc(SymDesc<T>& d, const T* M, int ldm, int N, int n, const T* u, T* w, T* part, size_t part_elems,
                   const int* skip);
template <typename T>
hipError_t launch_bk0_sym(hipStream_t st, const SymDesc<T>* d, const int* prefix_sweep, int total_sweep,
                          const int* prefix_red, int total_red, int ndesc, int K, const EventPair* ev_sweep = nullptr,
                          const EventPair* ev_red = nullptr);
template <typename T>
size_t gemv_cols_need(int m, int k);   // single-problem launch shape
template <typename T>
size_t bgemv_cols_need(int m, int k);  // batched launch shape
// batched sweeps over descriptor lists (desc.hpp)
template <typename T>
void fill_rows_desc(RowsDesc<T>& d, const T* A, int lda, int m, int k, int shape, const T* x, T* y, T alpha, T beta,
                    const T* y0, int nsplit, const int* skip);
template <typename T>
bool fill_cols_desc(ColsDesc<T>& d, const T* A, int lda, int m, int k, int shape, const T* x, T* y, T alpha, T beta,
                    const T* y0, T* part, size_t part_elems, const int* skip);
template <typename T>
hipError_t launch_bgemv_rows(hipStream_t st, const RowsDesc<T>* ddesc, const int* dprefix, int ndesc, int total_blocks,
                             size_t smem, int tag, const EventPair* ev = nullptr);
template <typename T>
hipError_t launch_bgemv_cols(hipStream_t st, const ColsDesc<T>* ddesc, const int* dprefix_part, int total_part,
                             const int* dprefix_red, int total_red, int ndesc, int tag, const EventPair* ev = nullptr);

// dst = src^T (rows x cols source), float64 or rounded to float32
struct TransDesc {
  const double* src;
  void* dst;
  int lds, ldd, rows, cols, to_float;
};
hipError_t transpose_2d(hipStream_t st, const double* src, int lds, int rows, int cols, void* dst, int ldd,
                        int to_float);
hipError_t btranspose_2d(hipStream_t st, const TransDesc* d, int count, int max_rows, int max_cols);

// blas.hip -----------------------------------------------------------------
// Tile skip rules for GEMM operands with known zero blocks (indices in op()
// space): kALower: op(A) lower triangular (k <= i); kBLower: op(B) lower (k >= j);
// kAUpper: op(A) upper (k >= i); kBUpper: op(B) upper (k <= j); kOutLower: only
// output tiles that touch the lower triangle are computed.
enum TriFlags : int { kNone = 0, kALower = 1, kBLower = 2, kAUpper = 4, kBUpper = 8, kOutLower = 16 };
hipError_t gemm_f64(hipStream_t st, int ta, int tb, int M, int N, int K, double alpha, const double* A, int lda,
                    const double* B, int ldb, double beta, double* C, int ldc, int flags);
hipError_t fill2d_f64(hipStream_t st, double* X, int ld, int rows, int cols, double v);
hipError_t chol_inv_f64(hipStream_t st, double* A, int lda, double* X, int ldx, int n, double* tmp, int* info,
                        int code);
size_t chol_inv_tmp_elems(int n);

// Batched forms: one launch covers the same step of many independent problems.
struct GemmDesc {
  const double* A;
  const double* B;
  double* C;
  int lda, ldb, ldc;
  int M, N, K;
};
struct LeafDesc {
  double* A;
  double* X;
  int* info;
  const double* dmax;
  int lda, ldx, nb, code;
};
struct DiagDesc {
  const double* A;
  double* out;
  int lda, n;
};
// One chol_inv problem: A (n x n, lower part read and overwritten), X = chol(A)^{-1}
// (upper part must hold zeros on entry), tmp of chol_inv_tmp_elems(n) doubles.
struct CholJob {
  double* A;
  int lda;
  double* X;
  int ldx;
  int n;
  double* tmp;
  int* info;
  int code;
  double* work = nullptr;  // scratch of the node being recorded (BatchedOps sets it inside tmp)
};
// Operation of one list of a batched GEMM launch: C = alpha op(A) op(B) + beta C.
struct GemmOp {
  int ta, tb, flags;
  double alpha, beta;
};

// A recorded sequence of batched factorization launches.  Descriptor lists are
// appended to bytes() in 256-byte aligned sections; the caller copies bytes()
// to device memory and passes its address to run().
class BatchedOps {
 public:
  void gemm(int ta, int tb, double alpha, double beta, int flags, const std::vector<GemmDesc>& d);
  // Two independent lists with their own operations in one launch.
  void gemm_pair(const GemmOp& o0, const std::vector<GemmDesc>& d0, const GemmOp& o1,
                 const std::vector<GemmDesc>& d1);
  void chol_inv(const std::vector<CholJob>& jobs);
  bool empty() const { return ops_.empty(); }
  const std::vector<unsigned char>& bytes() const { return bytes_; }
  hipError_t run(hipStream_t st, const void* d_bytes) const;

 private:
  struct Op {
    int kind, count, count2, gx, gy, tile64;
    GemmOp g0, g1;
    size_t off, off2;
  };
  template <typename D>
  size_t push(const std::vector<D>& v);
  void rec(const std::vector<CholJob>& jobs, int off, int len);
  std::vector<Op> ops_;
  std::vector<unsigned char> bytes_;
};

}  // namespace qpg
