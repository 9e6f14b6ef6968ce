// Per-QP context of the library and the host-side steps shared by the
// single-QP entry points (api.hip) and the batch driver (batch.hip).  Every
// arithmetic step runs in the kernels of gemv.hip, blas.hip, pcg.hip and
// ipm.hip; these functions only order launches and copy scalar records.
#pragma once
#include <algorithm>
#include <cstdarg>
#include <iterator>
#include <map>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/qpgpu.h"
#include "kernels.hpp"
#include "pcg.hpp"

namespace qpg {

// First-fit sub-allocator over one device allocation (256-byte granules).
// Used by the batch so that admitting and retiring QPs never calls hipMalloc /
// hipFree (which synchronize the device) and so that admission can be decided
// by the bytes still free.  Host-side bookkeeping only; not thread-safe.
class Arena {
 public:
  hipError_t init(size_t bytes);
  void release();
  void* alloc(size_t bytes);  // nullptr when no free range is large enough
  void free(void* p);
  size_t capacity() const { return cap_; }
  size_t used() const { return used_bytes_; }
  size_t largest_free() const;

 private:
  char* base_ = nullptr;
  size_t cap_ = 0, used_bytes_ = 0;
  std::map<size_t, size_t> free_;               // offset -> size, coalesced
  std::unordered_map<size_t, size_t> live_;     // offset -> size
};

constexpr int kProfOps = 6;

// Buffers and shape a captured poll chunk of CG steps was recorded with.
struct CgGraphKey {
  size_t elem;
  int prec;
  const void *dvec, *wts, *x;
  int poll;
  bool operator==(const CgGraphKey& o) const {
    return elem == o.elem && prec == o.prec && dvec == o.dvec && wts == o.wts && x == o.x && poll == o.poll;
  }
};
constexpr int kStatsStride = 64;  // doubles per QP in the stats record

}  // namespace qpg

struct qp_ctx {
  int dev = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int n = 0, m1 = 0, m2 = 0, N = 0;
  int ldn = 0, ldN = 0, ldm2 = 0, ldm1 = 0;
  qp_options opt{};
  std::string err;
  size_t bytes = 0;
  std::vector<void*> allocs;
  // batch member: buffers come from two regions of the batch arena (the
  // persistent buffers, zeroed once, and the factorization scratch), and the
  // scalar records (sc, stats, info and their pinned mirrors) live in the
  // batch's pools
  qpg::Arena* arena = nullptr;
  bool pooled = false;
  struct Region {
    char* base = nullptr;
    size_t size = 0, used = 0;
  };
  Region main_rg, scratch_rg;
  Region* cur_rg = nullptr;  // region dalloc carves from (pooled contexts)

  // problem data (float64)
  double *H = nullptr, *c = nullptr, *A = nullptr, *b = nullptr, *C = nullptr, *d = nullptr;
  // inverse factor L^{-1} of K0 = L Sigma L^T (N x ldN, lower, explicit zeros above)
  double* Linv = nullptr;
  bool factored = false;
  bool c_identity = false;
  // shared-matrix member (qp_shared): H, A, C and every factor belong to the
  // master context; the member owns only its problem vectors and work vectors
  const qp_ctx* master = nullptr;
  bool keep_mt = false;  // store M^T even when the one-pass product applies (block PCG reads it)
  std::vector<int> cg_trace;  // CG steps (predictor, corrector) of each IPM iteration of the last solve  // C = I found at factorization (m2 = n): the CG step skips both C products
  // P_H data: T = C H^{-1} C^T (fixed), P = D + T and X_P = chol(P)^{-1} (per D)
  double *T = nullptr, *P = nullptr, *XP = nullptr, *ptmp = nullptr;
  bool ph_ready = false;
  // float32 copies for the mixed path
  float *Linv32 = nullptr, *C32 = nullptr, *XP32 = nullptr;
  // explicit reduced operator E = C K0^{-1}_{11} C^T (m2 x m2, full) for QP_KF_EXPLICIT
  double* E = nullptr;
  float* E32 = nullptr;
  // transposed copies for the implicit CG step (Tune::op_t): C^T (n x ldm2) and
  // M^T = (L^{-1}[:, :n])^T (n x ldN, upper trapezoid), so C^T p and M^T v are row sweeps
  double *CT = nullptr, *MT = nullptr;
  float *CT32 = nullptr, *MT32 = nullptr;
  // factorization scratch allocated ahead of time (batch admission); null: allocated by factor()
  double *fHw = nullptr, *fWt = nullptr, *fS = nullptr, *fG = nullptr, *ftmp = nullptr, *fYt = nullptr;
  double* fY = nullptr;  // Y = L^{-1}[:, :n] C^T (N x m2), explicit operator only

  // vectors (float64)
  double *x = nullptr, *lam = nullptr, *nu = nullptr, *s = nullptr;
  double *Hx = nullptr, *Atl = nullptr, *Ctn = nullptr, *Ax = nullptr, *Cx = nullptr;
  double *rg = nullptr, *re = nullptr, *ri = nullptr;
  double *dvec = nullptr, *rc = nullptr, *rhs = nullptr, *Cw = nullptr;
  double *vN1 = nullptr, *vN2 = nullptr, *vN3 = nullptr;  // N-long scratch
  double *dx = nullptr, *dlam = nullptr, *dnu = nullptr, *ds = nullptr;
  double *dx_a = nullptr, *dlam_a = nullptr, *dnu_a = nullptr, *ds_a = nullptr;
  // PCG vectors (float64)
  double *pr = nullptr, *pz = nullptr, *pp = nullptr, *pq = nullptr, *pt = nullptr;
  double *pu = nullptr, *pv = nullptr, *pw = nullptr;
  double *ir_r = nullptr, *ir_x = nullptr, *ir_d = nullptr;  // refinement residual, K_F dnu, correction
  // PCG vectors (float32)
  float *fr = nullptr, *fz = nullptr, *fp = nullptr, *fq = nullptr, *ft = nullptr, *fx = nullptr, *fb = nullptr;
  float *fu = nullptr, *fv = nullptr, *fw = nullptr, *fd = nullptr, *fwts = nullptr;
  // workspaces
  qpg::GemvWork<double> w64{};
  void* sympart = nullptr;  // per-workgroup partials of the one-pass K0 product
  size_t sympart_bytes = 0;
  void* phpart = nullptr;  // per-workgroup partials of the one-pass P_H apply X_P^T X_P r
  size_t phpart_bytes = 0;
  qpg::GemvWork<float> w32{};
  double* bpart = nullptr;  // per-workgroup partials of p^T q
  int bpart_cap = 0;
  double* fold = nullptr;  // partials handed between the kernels of the folded CG step (4 x fold_cap)
  int fold_cap = 0;
  qpg::PcgScalars* sc = nullptr;
  qpg::IpmScalars* isc = nullptr;
  double* stats = nullptr;
  int* info = nullptr;
  // sampled kernel durations (options.profile): CG-step sweeps in the order
  // C^T p, Sigma M u, M^T v, q = C w + D p, X_P r, X_P^T t
  qpg::EventPair prof_ev[qpg::kProfOps] = {};
  double prof_ms[qpg::kProfOps] = {};
  long long prof_n[qpg::kProfOps] = {};
  bool prof_ready = false;
  int last_cg = 0;  // CG steps of the last reduced solve (sizes the next solve's first poll chunk)
  // captured poll chunks of CG steps (options.cg_graph)
  std::vector<std::pair<qpg::CgGraphKey, hipGraphExec_t>> cg_graphs;
  // pinned host mirrors
  qpg::PcgScalars* h_sc = nullptr;
  qpg::IpmScalars* h_isc = nullptr;
  double* h_stats = nullptr;
  int* h_info = nullptr;
};

namespace qpg {
namespace detail {

struct Fail {
  qp_status st;
};

void set_err(qp_ctx* ctx, const char* fmt, ...);
void set_err_str(std::string& dst, const char* fmt, ...);

#define HIPCHK(ctx, expr)                                                                                   \
  do {                                                                                                      \
    hipError_t e_ = (expr);                                                                                 \
    if (e_ != hipSuccess) {                                                                                 \
      ::qpg::detail::set_err(ctx, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
      throw ::qpg::detail::Fail{e_ == hipErrorOutOfMemory ? QP_E_NOMEM : QP_E_DEVICE};                       \
    }                                                                                                       \
  } while (0)

void* dalloc_bytes(qp_ctx* ctx, size_t bytes);
template <typename T>
T* dalloc(qp_ctx* ctx, size_t elems) {
  return static_cast<T*>(dalloc_bytes(ctx, (elems ? elems : 1) * sizeof(T)));
}
void dfree(qp_ctx* ctx, void* p);
void free_all(qp_ctx* ctx);

int ld_for(int cols);
void upload_matrix(qp_ctx* ctx, double* dst, int ldd, const double* src, int rows, int cols, qp_mem where);
void upload_vec(qp_ctx* ctx, double* dst, const double* src, int n, qp_mem where);
void download_vec(qp_ctx* ctx, double* dst, const double* src, int n, qp_mem where);
void sync(qp_ctx* ctx);
void release_cg_graphs(qp_ctx* ctx);
bool finite_all(const double* v, size_t n);
qp_status check_problem(int n, int m1, int m2, const double* H, const double* c, const double* A, const double* b,
                        const double* C, const double* d, qp_mem where);
qp_status check_options(const qp_options& o);
qp_precond resolve_prec(const qp_ctx* ctx, qp_precond p);
int prec_mode(qp_precond p);

// Context set-up: sizes and leading dimensions, then every device buffer.
void init_dims(qp_ctx* ctx, int n, int m1, int m2, const qp_options& o);
void alloc_all(qp_ctx* ctx);
// Factorization scratch held from admission until the factor is done (batch).
void alloc_factor_scratch(qp_ctx* ctx);
void free_factor_scratch(qp_ctx* ctx);
// The same scratch placed in caller-provided device memory of factor_scratch_bytes
// bytes (256-byte aligned), and the pointers cleared again without freeing.
size_t factor_scratch_bytes(qp_ctx* ctx);
void place_factor_scratch(qp_ctx* ctx, char* base);
void forget_factor_scratch(qp_ctx* ctx);
// Device bytes alloc_all (+ the factorization scratch) takes, rounded as dalloc rounds.
size_t footprint_bytes(int n, int m1, int m2, const qp_options& o, bool pooled, bool with_scratch);
void upload_problem(qp_ctx* ctx, const double* H, const double* c, const double* A, const double* b,
                    const double* C, const double* d, qp_mem where);

// K0 = L Sigma L^T and its inverse factor; throws Fail on a bad pivot.
void factor(qp_ctx* ctx);
inline bool kf_explicit(const qp_ctx* ctx) { return ctx->opt.kf_form == QP_KF_EXPLICIT; }
// The implicit CG step reads the stored transposes (C^T, M^T) with row sweeps.
inline bool op_transposed(const qp_ctx* ctx) { return tune().op_t && !kf_explicit(ctx); }
// The implicit CG step forms M^T Sigma M u in one pass over M (n small enough
// for the register rows of the one-pass sweep); M^T is then not stored.
inline bool op_fused(const qp_ctx* ctx) {
  return tune().k0_sym && !kf_explicit(ctx) && !ctx->master && ctx->n <= k0_sym_max_n<double>();
}
// The P_H apply z = X_P^T (X_P r) runs as one pass over X_P (the one-pass sweep
// with N = n = m2 and no sign flips) instead of a row and a column sweep.
inline bool ph_fused(const qp_ctx* ctx) { return tune().k0_sym && ctx->m2 <= k0_sym_max_n<double>(); }
// The CG step of this solve folds the vector update into its operator sweeps
// (pcg.hpp, FoldParts): single-QP implicit step over the stored C^T with the
// one-pass K0 product, and for P_H the one-pass X_P apply.
inline bool cg_folded(const qp_ctx* ctx, int prec) {
  return (tune().cg_fold & (prec == kPrecH ? 2 : 1)) && ctx->fold && tune().op_t && tune().k0_sym && !ctx->master &&
         ctx->opt.kf_form == QP_KF_IMPLICIT && ctx->n <= k0_sym_max_n<double>() && !ctx->c_identity &&
         (prec != kPrecH || ctx->m2 <= k0_sym_max_n<double>());
}
inline bool store_mt(const qp_ctx* ctx) { return (op_transposed(ctx) && !op_fused(ctx)) || ctx->keep_mt; }
void ph_setup(qp_ctx* ctx);
void ph_factor(qp_ctx* ctx, const double* dvec);
void k0_solve_dev(qp_ctx* ctx, const double* in, double* out, double* tmpN);
void kf_apply_dev(qp_ctx* ctx, const double* dvec, const double* p, double* q);

// ---- CG buffers -----------------------------------------------------------
template <typename T>
struct PcgBufs {
  const T *Linv, *C, *XP, *E, *CT, *MT, *dvec, *wts;
  T *r, *z, *p, *q, *t, *u, *v, *w, *x;
  const GemvWork<T>* wk;
};
PcgBufs<double> bufs64(qp_ctx* ctx, const double* dvec, const double* wts, double* x);
PcgBufs<float> bufs32(qp_ctx* ctx);
// Iteration cap of one float32 sweep of the mixed solve: a little above the
// distinct-eigenvalue bound of the preconditioned operator.
int mixed_inner_cap(const qp_ctx* ctx, int prec);

// ---- interior point phases ------------------------------------------------
// Host-side bookkeeping of one QP's IPM run.
struct IpmRun {
  int prec = 0, maxit = 0, it = 0;
  long long cg_total = 0;
  long long cg64 = 0;  // mixed precision: CG steps of the float64 fallback runs
  int refin_total = 0, fallbacks = 0;
  int k1 = 0, k2 = 0;
  double score = 0, parts[5] = {0, 0, 0, 0, 0};
  double mu = 0, wtol = 0;
  int status = QP_E_NOCONV;
};
// Preconditioner, CG cap, P_H set-up and the initial point (launches only).
void ipm_start(qp_ctx* ctx, IpmRun& R);
// Residual products and statistics of the current iterate; with copy, also the
// asynchronous copy of the statistics to ctx->h_stats.
void ipm_eval_launch(qp_ctx* ctx, bool copy);
// After the statistics reached the host: KKT score and stop decision.
// Returns true when another iteration is due (then R.mu and R.wtol are set).
bool ipm_check(qp_ctx* ctx, IpmRun& R);
// r_nu pieces, D and the predictor right-hand side; with factor_ph also the
// P_H factor for the new D (launches only).
void ipm_predictor_setup(qp_ctx* ctx, IpmRun& R, bool factor_ph = true);
// Recovery and step of the predictor, then the corrector right-hand side.
void ipm_after_predictor(qp_ctx* ctx);
// Recovery and step of the corrector; closes the iteration.
void ipm_after_corrector(qp_ctx* ctx, IpmRun& R);
void ipm_fill_info(const qp_ctx* ctx, const IpmRun& R, qp_ipm_info* info);
double host_rel_kkt(const double* S, double parts[5]);

template <typename F>
qp_status guarded(qp_ctx* ctx, F&& f) {
  try {
    f();
    return QP_OK;
  } catch (const Fail& e) {
    return e.st;
  } catch (const std::exception& e) {
    set_err(ctx, "internal error: %s", e.what());
    return QP_E_DEVICE;
  } catch (...) {
    set_err(ctx, "internal error");
    return QP_E_DEVICE;
  }
}

}  // namespace detail
}  // namespace qpg
