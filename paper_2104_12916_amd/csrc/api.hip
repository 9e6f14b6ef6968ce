// C ABI of the library: the per-QP context (device buffers, stream, factor),
// the PCG driver and the interior point driver.  Every arithmetic step runs in
// the kernels of gemv.hip, blas.hip, pcg.hip and ipm.hip; this file only orders
// launches, polls convergence flags and copies small scalar records.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>
#include <chrono>
#include <cstdlib>

#include "../../include/qpgpu.h"
#include "kernels.hpp"
#include "pcg.hpp"

namespace qpg {

DevInfo& dev_info() {
  static DevInfo info = [] {
    DevInfo d;
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
      d.device = dev;
      int cus = 0;
      if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
        d.cu_count = cus;
    }
    return d;
  }();
  return info;
}

// Leading dimension of a matrix with `cols` columns: whole 256-element rows
// (every sweep reads full 64-lane x 16-byte chunks) plus tune().ld_pad.
static int ld_for(int cols) { return ((cols > 0 ? cols : 1) + 255) / 256 * 256 + tune().ld_pad; }

}  // namespace qpg

using namespace qpg;

constexpr int kProfOps = 6;

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

  // problem data (float64)
  double *H = nullptr, *c = nullptr, *A = nullptr, *b = nullptr, *C = nullptr, *d = nullptr;
  // inverse factor L^{-1} of K0 = L Sigma L^T (N x ldN, lower, explicit zeros above)
  double* Linv = nullptr;
  bool factored = false;
  // P_H data: T = C H^{-1} C^T (fixed), P = D + T and X_P = chol(P)^{-1} (per D)
  double *T = nullptr, *P = nullptr, *XP = nullptr, *ptmp = nullptr;
  bool ph_ready = false;
  // float32 copies for the mixed path
  float *Linv32 = nullptr, *C32 = nullptr, *XP32 = nullptr;

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
  GemvWork<double> w64{};
  GemvWork<float> w32{};
  double* bpart = nullptr;  // per-workgroup partials of p^T q
  int bpart_cap = 0;
  PcgScalars* sc = nullptr;
  IpmScalars* isc = nullptr;
  double* stats = nullptr;
  int* info = nullptr;
  // sampled kernel durations (options.profile): CG-step sweeps in the order
  // C^T p, Sigma M u, M^T v, q = C w + D p, X_P r, X_P^T t
  EventPair prof_ev[kProfOps] = {};
  double prof_ms[kProfOps] = {};
  long long prof_n[kProfOps] = {};
  bool prof_ready = false;
  // pinned host mirrors
  PcgScalars* h_sc = nullptr;
  IpmScalars* h_isc = nullptr;
  double* h_stats = nullptr;
  int* h_info = nullptr;
};

namespace {

struct Fail {
  qp_status st;
};

void set_err(qp_ctx* ctx, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (ctx) ctx->err = buf;
}

#define HIPCHK(ctx, expr)                                                                                   \
  do {                                                                                                      \
    hipError_t e_ = (expr);                                                                                 \
    if (e_ != hipSuccess) {                                                                                 \
      set_err(ctx, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__);              \
      throw Fail{e_ == hipErrorOutOfMemory ? QP_E_NOMEM : QP_E_DEVICE};                                      \
    }                                                                                                       \
  } while (0)

template <typename T>
T* dalloc(qp_ctx* ctx, size_t elems) {
  if (elems == 0) elems = 1;
  void* p = nullptr;
  size_t bytes = elems * sizeof(T);
  bytes = (bytes + 255) / 256 * 256;
  HIPCHK(ctx, hipMalloc(&p, bytes));
  HIPCHK(ctx, hipMemsetAsync(p, 0, bytes, ctx->stream));
  ctx->allocs.push_back(p);
  ctx->bytes += bytes;
  return static_cast<T*>(p);
}

void dfree(qp_ctx* ctx, void* p) {
  if (!p) return;
  for (size_t i = 0; i < ctx->allocs.size(); ++i)
    if (ctx->allocs[i] == p) {
      ctx->allocs.erase(ctx->allocs.begin() + i);
      break;
    }
  (void)hipFree(p);
}

// Copy a dense rows x cols row-major caller matrix (ld = cols) into a padded
// device matrix (ld = ldd).
void upload_matrix(qp_ctx* ctx, double* dst, int ldd, const double* src, int rows, int cols, qp_mem where) {
  if (rows <= 0 || cols <= 0) return;
  hipMemcpyKind kind = (where == QP_MEM_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  HIPCHK(ctx, hipMemcpy2DAsync(dst, (size_t)ldd * sizeof(double), src, (size_t)cols * sizeof(double),
                               (size_t)cols * sizeof(double), rows, kind, ctx->stream));
}

void upload_vec(qp_ctx* ctx, double* dst, const double* src, int n, qp_mem where) {
  if (n <= 0) return;
  hipMemcpyKind kind = (where == QP_MEM_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  HIPCHK(ctx, hipMemcpyAsync(dst, src, (size_t)n * sizeof(double), kind, ctx->stream));
}

void download_vec(qp_ctx* ctx, double* dst, const double* src, int n, qp_mem where) {
  if (n <= 0) return;
  hipMemcpyKind kind = (where == QP_MEM_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  HIPCHK(ctx, hipMemcpyAsync(dst, src, (size_t)n * sizeof(double), kind, ctx->stream));
}

void sync(qp_ctx* ctx) { HIPCHK(ctx, hipStreamSynchronize(ctx->stream)); }

bool finite_all(const double* v, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

qp_precond resolve_prec(const qp_ctx* ctx, qp_precond p) {
  if (p != QP_PREC_AUTO) return p;
  int bl = std::min(ctx->m2, ctx->n - ctx->m1);
  int bh = std::min(ctx->m2, ctx->m1);
  return bl <= bh ? QP_PREC_LOW_DOF : QP_PREC_FEW_EQ;
}

int prec_mode(qp_precond p) {
  return p == QP_PREC_LOW_DOF ? kPrecL : (p == QP_PREC_FEW_EQ ? kPrecH : kPrecNone);
}

// ---- K0 solves ------------------------------------------------------------
// out = K0^{-1} in = L^{-T} Sigma L^{-1} in  (full N-vectors, float64).
void k0_solve_dev(qp_ctx* ctx, const double* in, double* out, double* tmpN) {
  HIPCHK(ctx, launch_gemv_rows<double>(ctx->stream, ctx->Linv, ctx->ldN, ctx->N, ctx->N, kLower, in, tmpN, 1.0, 0.0,
                                       nullptr, ctx->n, nullptr));
  HIPCHK(ctx, launch_gemv_cols<double>(ctx->stream, ctx->Linv, ctx->ldN, ctx->N, ctx->N, kLower, tmpN, out, 1.0, 0.0,
                                       nullptr, ctx->w64, nullptr));
}

// w = [I 0] K0^{-1} [u; 0] = M^T Sigma M u with M = L^{-1}[:, :n].
template <typename T>
void k0_top_apply(qp_ctx* ctx, const T* Linv, const T* u, T* v, T* w, const GemvWork<T>& wk, const int* skip) {
  HIPCHK(ctx, launch_gemv_rows<T>(ctx->stream, Linv, ctx->ldN, ctx->N, ctx->n, kLower, u, v, T(1), T(0), nullptr,
                                  ctx->n, skip, 2));
  HIPCHK(ctx, launch_gemv_cols<T>(ctx->stream, Linv, ctx->ldN, ctx->N, ctx->n, kLower, v, w, T(1), T(0), nullptr, wk,
                                  skip, 3));
}

// ---- factorization --------------------------------------------------------
void factor(qp_ctx* ctx) {
  const int n = ctx->n, m1 = ctx->m1, N = ctx->N, ldn = ctx->ldn, ldN = ctx->ldN, ldm1 = ctx->ldm1;
  hipStream_t st = ctx->stream;
  double* Hw = dalloc<double>(ctx, (size_t)n * ldn);
  double* Wt = dalloc<double>(ctx, (size_t)m1 * ldn);
  double* S = dalloc<double>(ctx, (size_t)m1 * ldm1);
  double* tmpG = dalloc<double>(ctx, (size_t)m1 * ldn);
  double* tmp = dalloc<double>(ctx, chol_inv_tmp_elems(n > m1 ? n : m1));
  HIPCHK(ctx, hipMemsetAsync(ctx->info, 0, sizeof(int), st));
  HIPCHK(ctx, hipMemcpyAsync(Hw, ctx->H, (size_t)n * ldn * sizeof(double), hipMemcpyDeviceToDevice, st));
  double* XH = ctx->Linv;                        // rows 0..n-1, cols 0..n-1
  double* G = ctx->Linv + (size_t)n * ldN;       // rows n..N-1, cols 0..n-1
  double* XS = G + n;                            // rows n..N-1, cols n..N-1
  // X_H = L_H^{-1}
  HIPCHK(ctx, chol_inv_f64(st, Hw, ldn, XH, ldN, n, tmp, ctx->info, QP_E_NOT_SPD));
  // W^T = A X_H^T (m1 x n);  S = W^T W = A H^{-1} A^T (lower)
  HIPCHK(ctx, gemm_f64(st, 0, 1, m1, n, n, 1.0, ctx->A, ldn, XH, ldN, 0.0, Wt, ldn, kBUpper));
  HIPCHK(ctx, gemm_f64(st, 0, 1, m1, m1, n, 1.0, Wt, ldn, Wt, ldn, 0.0, S, ldm1, kOutLower));
  HIPCHK(ctx, hipMemcpyAsync(ctx->h_info, ctx->info, sizeof(int), hipMemcpyDeviceToHost, st));
  sync(ctx);
  if (*ctx->h_info != 0) {
    set_err(ctx, "Cholesky factorization of H failed: H is not positive definite");
    for (void* p : {(void*)Hw, (void*)Wt, (void*)S, (void*)tmpG, (void*)tmp}) dfree(ctx, p);
    throw Fail{QP_E_NOT_SPD};
  }
  // X_S = L_S^{-1}
  HIPCHK(ctx, chol_inv_f64(st, S, ldm1, XS, ldN, m1, tmp, ctx->info, QP_E_RANK));
  // G = -X_S W^T X_H  (bottom-left block of L^{-1})
  HIPCHK(ctx, gemm_f64(st, 0, 0, m1, n, n, 1.0, Wt, ldn, XH, ldN, 0.0, tmpG, ldn, kBLower));
  HIPCHK(ctx, gemm_f64(st, 0, 0, m1, n, m1, -1.0, XS, ldN, tmpG, ldn, 0.0, G, ldN, kALower));
  HIPCHK(ctx, hipMemcpyAsync(ctx->h_info, ctx->info, sizeof(int), hipMemcpyDeviceToHost, st));
  sync(ctx);
  int bad = *ctx->h_info;
  if (bad != 0) {
    set_err(ctx, "Cholesky factorization of A H^{-1} A^T failed: A is rank deficient");
    for (void* p : {(void*)Hw, (void*)Wt, (void*)S, (void*)tmpG, (void*)tmp}) dfree(ctx, p);
    throw Fail{QP_E_RANK};
  }
  for (void* p : {(void*)Hw, (void*)Wt, (void*)S, (void*)tmpG, (void*)tmp}) dfree(ctx, p);
  if (ctx->opt.precision == QP_MIXED) {
    HIPCHK(ctx, (convert_2d<double, float>(st, ctx->Linv, ldN, ctx->Linv32, ldN, N, N)));
  }
  ctx->factored = true;
}

// T = C H^{-1} C^T = (C X_H^T)(C X_H^T)^T, once per QP.
void ph_setup(qp_ctx* ctx) {
  if (ctx->ph_ready) return;
  const int n = ctx->n, m2 = ctx->m2;
  hipStream_t st = ctx->stream;
  double* Yt = dalloc<double>(ctx, (size_t)m2 * ctx->ldn);
  HIPCHK(ctx, gemm_f64(st, 0, 1, m2, n, n, 1.0, ctx->C, ctx->ldn, ctx->Linv, ctx->ldN, 0.0, Yt, ctx->ldn, kBUpper));
  HIPCHK(ctx, gemm_f64(st, 0, 1, m2, m2, n, 1.0, Yt, ctx->ldn, Yt, ctx->ldn, 0.0, ctx->T, ctx->ldm2, kOutLower));
  sync(ctx);
  dfree(ctx, Yt);
  ctx->ph_ready = true;
}

// X_P = chol(D + T)^{-1} for the current D (in ctx->dvec).
void ph_factor(qp_ctx* ctx, const double* dvec) {
  hipStream_t st = ctx->stream;
  const int m2 = ctx->m2;
  HIPCHK(ctx, add_diag_copy(st, m2, ctx->T, ctx->ldm2, dvec, ctx->P, ctx->ldm2));
  HIPCHK(ctx, hipMemsetAsync(ctx->info, 0, sizeof(int), st));
  HIPCHK(ctx, chol_inv_f64(st, ctx->P, ctx->ldm2, ctx->XP, ctx->ldm2, m2, ctx->ptmp, ctx->info, QP_E_INVALID));
  if (ctx->opt.precision == QP_MIXED)
    HIPCHK(ctx, (convert_2d<double, float>(st, ctx->XP, ctx->ldm2, ctx->XP32, ctx->ldm2, m2, m2)));
}

// ---- PCG driver -------------------------------------------------------------
struct PcgResult {
  int iters = 0;
  int done = 0;
};

template <typename T>
struct PcgBufs {
  const T *Linv, *C, *XP, *dvec, *wts;
  T *r, *z, *p, *q, *t, *u, *v, *w, *x;
  const GemvWork<T>* wk;
};

template <typename T>
PcgResult run_pcg(qp_ctx* ctx, const PcgBufs<T>& B, const T* rhs, int prec, double rtol, double wtol, int maxit) {
  hipStream_t st = ctx->stream;
  const int n = ctx->n, m2 = ctx->m2;
  const int* skip = &ctx->sc->done;
  HIPCHK(ctx, pcg_init<T>(st, m2, rhs, B.dvec, B.wts, B.x, B.r, B.z, B.p, prec, rtol, wtol, maxit, ctx->sc));
  auto ph_apply = [&](int init, const EventPair* ev) {
    HIPCHK(ctx, launch_gemv_rows<T>(st, B.XP, ctx->ldm2, m2, m2, kLower, B.r, B.t, T(1), T(0), nullptr, m2, skip, 4,
                                    ev ? &ev[4] : nullptr));
    HIPCHK(ctx, launch_gemv_cols<T>(st, B.XP, ctx->ldm2, m2, m2, kLower, B.t, B.z, T(1), T(0), nullptr, *B.wk, skip,
                                    5, ev ? &ev[5] : nullptr));
    HIPCHK(ctx, pcg_ph_update<T>(st, m2, B.r, B.z, B.p, init, ctx->sc));
  };
  if (prec == kPrecH) ph_apply(1, nullptr);
  const int poll = ctx->opt.poll_every > 0 ? ctx->opt.poll_every : 32;
  PcgResult res;
  long long launched = 0;
  const bool prof = ctx->opt.profile != 0;
  if (prof && !ctx->prof_ready) {
    for (int o = 0; o < kProfOps; ++o) {
      HIPCHK(ctx, hipEventCreate(&ctx->prof_ev[o].begin));
      HIPCHK(ctx, hipEventCreate(&ctx->prof_ev[o].end));
    }
    ctx->prof_ready = true;
  }
  int iter_before = 0;
  for (;;) {
    // the device stops at maxit; a host bound guards against a stop flag that never arrives
    if (launched > (long long)maxit + 2LL * poll) {
      set_err(ctx, "PCG made no progress after %lld launched steps", launched);
      throw Fail{QP_E_DEVICE};
    }
    launched += poll;
    for (int k = 0; k < poll; ++k) {
      const EventPair* ev = (prof && k == 0) ? ctx->prof_ev : nullptr;
      HIPCHK(ctx, launch_gemv_cols<T>(st, B.C, ctx->ldn, m2, n, kDense, B.p, B.u, T(1), T(0), nullptr, *B.wk, skip, 1,
                                      ev ? &ev[0] : nullptr));
      HIPCHK(ctx, launch_gemv_rows<T>(st, B.Linv, ctx->ldN, ctx->N, n, kLower, B.u, B.v, T(1), T(0), nullptr, n, skip,
                                      2, ev ? &ev[1] : nullptr));
      HIPCHK(ctx, launch_gemv_cols<T>(st, B.Linv, ctx->ldN, ctx->N, n, kLower, B.v, B.w, T(1), T(0), nullptr, *B.wk,
                                      skip, 3, ev ? &ev[2] : nullptr));
      HIPCHK(ctx, pcg_q<T>(st, B.C, ctx->ldn, m2, n, B.w, B.dvec, B.p, B.q, ctx->sc, ctx->bpart, ctx->bpart_cap,
                           ev ? &ev[3] : nullptr));
      HIPCHK(ctx, pcg_update<T>(st, m2, ctx->bpart, B.dvec, B.p, B.q, B.x, B.r, B.z, B.wts, prec, ctx->sc));
      if (prec == kPrecH) ph_apply(0, ev);
    }
    HIPCHK(ctx, hipMemcpyAsync(ctx->h_sc, ctx->sc, sizeof(PcgScalars), hipMemcpyDeviceToHost, st));
    sync(ctx);
    if (prof && ctx->h_sc->iter > iter_before) {
      // the sampled step ran (it was the first of the chunk and the solve had not stopped)
      const int nops = (prec == kPrecH) ? 6 : 4;
      for (int o = 0; o < nops; ++o) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, ctx->prof_ev[o].begin, ctx->prof_ev[o].end) == hipSuccess) {
          ctx->prof_ms[o] += ms;
          ctx->prof_n[o] += 1;
        }
      }
    }
    iter_before = ctx->h_sc->iter;
    if (ctx->h_sc->done) break;
  }
  res.iters = ctx->h_sc->iter;
  res.done = ctx->h_sc->done;
  return res;
}

PcgBufs<double> bufs64(qp_ctx* ctx, const double* dvec, const double* wts, double* x) {
  PcgBufs<double> B;
  B.Linv = ctx->Linv;
  B.C = ctx->C;
  B.XP = ctx->XP;
  B.dvec = dvec;
  B.wts = wts;
  B.r = ctx->pr;
  B.z = ctx->pz;
  B.p = ctx->pp;
  B.q = ctx->pq;
  B.t = ctx->pt;
  B.u = ctx->pu;
  B.v = ctx->pv;
  B.w = ctx->pw;
  B.x = x;
  B.wk = &ctx->w64;
  return B;
}

PcgBufs<float> bufs32(qp_ctx* ctx) {
  PcgBufs<float> B;
  B.Linv = ctx->Linv32;
  B.C = ctx->C32;
  B.XP = ctx->XP32;
  B.dvec = ctx->fd;
  B.wts = ctx->fwts;
  B.r = ctx->fr;
  B.z = ctx->fz;
  B.p = ctx->fp;
  B.q = ctx->fq;
  B.t = ctx->ft;
  B.u = ctx->fu;
  B.v = ctx->fv;
  B.w = ctx->fw;
  B.x = ctx->fx;
  B.wk = &ctx->w32;
  return B;
}

// q = K_F p in float64 (used by qp_kf_apply and the refinement residual).
void kf_apply_dev(qp_ctx* ctx, const double* dvec, const double* p, double* q) {
  hipStream_t st = ctx->stream;
  HIPCHK(ctx, launch_gemv_cols<double>(st, ctx->C, ctx->ldn, ctx->m2, ctx->n, kDense, p, ctx->pu, 1.0, 0.0, nullptr,
                                       ctx->w64, nullptr));
  k0_top_apply<double>(ctx, ctx->Linv, ctx->pu, ctx->pv, ctx->pw, ctx->w64, nullptr);
  HIPCHK(ctx, ew_mul(st, ctx->m2, dvec, p, ctx->pt));
  HIPCHK(ctx, launch_gemv_rows<double>(st, ctx->C, ctx->ldn, ctx->m2, ctx->n, kDense, ctx->pw, q, 1.0, 1.0, ctx->pt,
                                       ctx->m2, nullptr));
}

// Reduced solve used by both qp_pcg_solve and the IPM.  dvec, rhs, dnu, wts are
// device float64 vectors.  Returns CG steps; sets *done to the PCG stop code.
int reduced_solve(qp_ctx* ctx, int prec, const double* dvec, const double* rhs, double* dnu, const double* wts,
                  double rtol, double wtol, int maxit, int* done, int* refinements, int* fallback) {
  *refinements = 0;
  *fallback = 0;
  if (ctx->opt.precision != QP_MIXED) {
    PcgBufs<double> B = bufs64(ctx, dvec, wts, dnu);
    PcgResult r = run_pcg<double>(ctx, B, rhs, prec, rtol, wtol, maxit);
    *done = r.done;
    return r.iters;
  }
  // Mixed: float32 PCG sweeps on the residual equation K_F delta = r inside a
  // float64 refinement loop (r = rhs - K_F dnu recomputed with the float64
  // operator).  When a sweep does not converge within its cap or fails to
  // shrink ||r||_2 tenfold (the float32 recurrence stalls on ill-conditioned
  // systems) the remaining correction is solved by float64 PCG, which also sees
  // the total residual, so the stop tests are the same as in the float64 path.
  hipStream_t st = ctx->stream;
  const int m2 = ctx->m2;
  const int bound = prec == kPrecL ? std::min(m2, ctx->n - ctx->m1) : (prec == kPrecH ? std::min(m2, ctx->m1) : m2);
  const int inner_cap = std::max(200, 2 * (bound + 1));
  const double inner_rtol = 1e-5;
  int total = 0;
  HIPCHK(ctx, (convert_1d<double, float>(st, dvec, ctx->fd, m2)));
  if (wts) HIPCHK(ctx, (convert_1d<double, float>(st, wts, ctx->fwts, m2)));
  HIPCHK(ctx, fill_vec<double>(st, m2, 0.0, dnu));
  HIPCHK(ctx, hipMemcpyAsync(ctx->ir_r, rhs, (size_t)m2 * sizeof(double), hipMemcpyDeviceToDevice, st));
  int sweeps = 0;
  double prev_rr = -1.0;
  *done = 2;
  for (; sweeps < 30 && total < maxit; ++sweeps) {
    HIPCHK(ctx, (convert_1d<double, float>(st, ctx->ir_r, ctx->fb, m2)));
    PcgBufs<float> B = bufs32(ctx);
    B.wts = wts ? ctx->fwts : nullptr;
    PcgResult r = run_pcg<float>(ctx, B, ctx->fb, prec, inner_rtol, -1.0, std::min(inner_cap, maxit - total));
    total += r.iters;
    HIPCHK(ctx, ir_accumulate(st, m2, ctx->fx, dnu));
    // float64 residual r = rhs - K_F dnu, with its stop statistics
    kf_apply_dev(ctx, dvec, dnu, ctx->ir_x);
    HIPCHK(ctx, ir_residual(st, m2, rhs, ctx->ir_x, wts, ctx->ir_r, ctx->sc));
    HIPCHK(ctx, hipMemcpyAsync(ctx->h_sc, ctx->sc, sizeof(PcgScalars), hipMemcpyDeviceToHost, st));
    sync(ctx);
    const PcgScalars h = *ctx->h_sc;
    if (h.bb == 0.0 || h.rr <= rtol * rtol * h.bb || (wtol >= 0.0 && h.wmax <= wtol)) {
      *done = 1;
      ++sweeps;
      break;
    }
    const double ref_rr = prev_rr >= 0.0 ? prev_rr : h.bb;
    const bool stalled = r.done != 1 || h.rr > 1e-2 * ref_rr || !std::isfinite(h.rr);
    if (stalled && total < maxit) {
      // float64 PCG on the remaining correction, zero start, same stop tests
      PcgBufs<double> B64 = bufs64(ctx, dvec, wts, ctx->ir_d);
      const double rtol64 = h.rr > 0.0 ? rtol * std::sqrt(h.bb / h.rr) : rtol;
      PcgResult r64 = run_pcg<double>(ctx, B64, ctx->ir_r, prec, rtol64, wtol, maxit - total);
      total += r64.iters;
      HIPCHK(ctx, vec_add(st, m2, ctx->ir_d, dnu));
      *done = r64.done;
      *fallback = 1;
      ++sweeps;
      break;
    }
    prev_rr = h.rr;
  }
  *refinements = sweeps;
  return total;
}

double host_rel_kkt(const double* S, int m2, double parts[5]) {
  double pobj = 0.5 * S[kXHx] + S[kCx];
  double dobj = -0.5 * S[kXHx] + S[kBl] + S[kDn];
  double rho_d = S[kRdInf] / (1.0 + std::max(std::max(S[kHxInf], S[kCInf]), std::max(S[kAtlInf], S[kCtnInf])));
  double rho_e = S[kReInf] / (1.0 + std::max(S[kAxInf], S[kBInf]));
  double rho_p = std::max(S[kViolInf], 0.0) / (1.0 + S[kDInf]);
  double rho_g = std::fabs(pobj - dobj) / (1.0 + std::fabs(pobj));
  double rho_n = std::max(0.0, -S[kNuMin]) / (1.0 + S[kNuInf]);
  parts[0] = rho_d;
  parts[1] = rho_e;
  parts[2] = rho_p;
  parts[3] = rho_g;
  parts[4] = rho_n;
  (void)m2;
  return std::max(std::max(std::max(rho_d, rho_e), std::max(rho_p, rho_g)), rho_n);
}

// Residuals and statistics of the current iterate (x, lam, nu, s) -> host stats.
void eval_iterate(qp_ctx* ctx) {
  hipStream_t st = ctx->stream;
  const int n = ctx->n, m1 = ctx->m1, m2 = ctx->m2;
  HIPCHK(ctx, launch_gemv_rows<double>(st, ctx->H, ctx->ldn, n, n, kDense, ctx->x, ctx->Hx, 1.0, 0.0, nullptr, n,
                                       nullptr));
  HIPCHK(ctx, launch_gemv_rows<double>(st, ctx->A, ctx->ldn, m1, n, kDense, ctx->x, ctx->Ax, 1.0, 0.0, nullptr, m1,
                                       nullptr));
  HIPCHK(ctx, launch_gemv_rows<double>(st, ctx->C, ctx->ldn, m2, n, kDense, ctx->x, ctx->Cx, 1.0, 0.0, nullptr, m2,
                                       nullptr));
  HIPCHK(ctx, launch_gemv_cols<double>(st, ctx->A, ctx->ldn, m1, n, kDense, ctx->lam, ctx->Atl, 1.0, 0.0, nullptr,
                                       ctx->w64, nullptr));
  HIPCHK(ctx, launch_gemv_cols<double>(st, ctx->C, ctx->ldn, m2, n, kDense, ctx->nu, ctx->Ctn, 1.0, 0.0, nullptr,
                                       ctx->w64, nullptr));
  HIPCHK(ctx, ipm_stats(st, n, m1, m2, ctx->Hx, ctx->Atl, ctx->Ctn, ctx->Ax, ctx->Cx, ctx->x, ctx->c, ctx->lam, ctx->b,
                        ctx->nu, ctx->s, ctx->d, ctx->rg, ctx->re, ctx->ri, ctx->stats));
  HIPCHK(ctx, hipMemcpyAsync(ctx->h_stats, ctx->stats, kNumStats * sizeof(double), hipMemcpyDeviceToHost, st));
  sync(ctx);
}

// Recovery of eq. schur-delta-x (K0 form) and eq. delz for a given dnu.
void recover(qp_ctx* ctx, const double* dnu, double* dx, double* dlam, double* ds) {
  hipStream_t st = ctx->stream;
  const int n = ctx->n, m1 = ctx->m1, m2 = ctx->m2;
  // rhs = [r_g + C^T dnu; -r_e]
  HIPCHK(ctx, launch_gemv_cols<double>(st, ctx->C, ctx->ldn, m2, n, kDense, dnu, ctx->vN1, 1.0, 1.0, ctx->rg, ctx->w64,
                                       nullptr));
  HIPCHK(ctx, ipm_neg_copy(st, m1, ctx->re, ctx->vN1 + n));
  k0_solve_dev(ctx, ctx->vN1, ctx->vN2, ctx->vN3);
  HIPCHK(ctx, ipm_dirs(st, n, m1, m2, ctx->vN2, ctx->rc, ctx->nu, ctx->dvec, dnu, dx, dlam, ds));
}

void ipm_run(qp_ctx* ctx, qp_ipm_info* info) {
  hipStream_t st = ctx->stream;
  const int n = ctx->n, m1 = ctx->m1, m2 = ctx->m2;
  const qp_precond pc = resolve_prec(ctx, ctx->opt.prec);
  const int prec = prec_mode(pc);
  if (prec == kPrecH) ph_setup(ctx);
  const int maxit = ctx->opt.max_pcg > 0 ? ctx->opt.max_pcg : 20 * m2;
  // initial point: K0 [x0; -lam0] = [-c; b]; s0 = max(C x0 - d, 1); nu0 = 1
  HIPCHK(ctx, ipm_neg_copy(st, n, ctx->c, ctx->vN1));
  HIPCHK(ctx, hipMemcpyAsync(ctx->vN1 + n, ctx->b, (size_t)m1 * sizeof(double), hipMemcpyDeviceToDevice, st));
  k0_solve_dev(ctx, ctx->vN1, ctx->vN2, ctx->vN3);
  HIPCHK(ctx, launch_gemv_rows<double>(st, ctx->C, ctx->ldn, m2, n, kDense, ctx->vN2, ctx->Cx, 1.0, 0.0, nullptr, m2,
                                       nullptr));
  HIPCHK(ctx, ipm_init_point(st, n, m1, m2, ctx->vN2, ctx->Cx, ctx->d, ctx->x, ctx->lam, ctx->nu, ctx->s));
  IpmScalars hs{};
  hs.tau = ctx->opt.tau;
  HIPCHK(ctx, hipMemcpyAsync(ctx->isc, &hs, sizeof(IpmScalars), hipMemcpyHostToDevice, st));
  long long cg_total = 0;
  int refin_total = 0;
  int fallbacks = 0;
  int it = 0;
  double parts[5] = {0, 0, 0, 0, 0};
  double score = 0;
  int status = QP_E_NOCONV;
  for (;;) {
    eval_iterate(ctx);
    score = host_rel_kkt(ctx->h_stats, m2, parts);
    if (!std::isfinite(score)) {
      set_err(ctx, "non-finite iterate at IPM iteration %d", it);
      status = QP_E_NOCONV;
      break;
    }
    if (score <= ctx->opt.rtol_kkt) {
      status = QP_OK;
      break;
    }
    if (it >= ctx->opt.max_ipm) break;
    const double mu = ctx->h_stats[kSNu] / m2;
    // w = [I 0] K0^{-1} [-r_g; r_e];  C w feeds r_nu
    HIPCHK(ctx, ipm_neg_copy(st, n, ctx->rg, ctx->vN1));
    HIPCHK(ctx, hipMemcpyAsync(ctx->vN1 + n, ctx->re, (size_t)m1 * sizeof(double), hipMemcpyDeviceToDevice, st));
    k0_solve_dev(ctx, ctx->vN1, ctx->vN2, ctx->vN3);
    HIPCHK(ctx, launch_gemv_rows<double>(st, ctx->C, ctx->ldn, m2, n, kDense, ctx->vN2, ctx->Cw, 1.0, 0.0, nullptr,
                                         m2, nullptr));
    // predictor
    HIPCHK(ctx, ipm_rhs(st, m2, 0, ctx->ri, ctx->s, ctx->nu, ctx->Cw, nullptr, nullptr, ctx->isc, ctx->rc, ctx->rhs,
                        ctx->dvec));
    if (prec == kPrecH) ph_factor(ctx, ctx->dvec);
    const double wtol = ctx->opt.cg_theta * mu;
    int done = 0, refin = 0, fb = 0;
    int k1 = reduced_solve(ctx, prec, ctx->dvec, ctx->rhs, ctx->dnu_a, ctx->nu, ctx->opt.cg_rtol, wtol, maxit, &done,
                           &refin, &fb);
    refin_total += refin;
    fallbacks += fb;
    recover(ctx, ctx->dnu_a, ctx->dx_a, ctx->dlam_a, ctx->ds_a);
    HIPCHK(ctx, ipm_step(st, n, m1, m2, 0, ctx->x, ctx->lam, ctx->nu, ctx->s, ctx->dx_a, ctx->dlam_a, ctx->dnu_a,
                         ctx->ds_a, ctx->isc));
    // corrector
    HIPCHK(ctx, ipm_rhs(st, m2, 1, ctx->ri, ctx->s, ctx->nu, ctx->Cw, ctx->ds_a, ctx->dnu_a, ctx->isc, ctx->rc,
                        ctx->rhs, ctx->dvec));
    int k2 = reduced_solve(ctx, prec, ctx->dvec, ctx->rhs, ctx->dnu, ctx->nu, ctx->opt.cg_rtol, wtol, maxit, &done,
                           &refin, &fb);
    refin_total += refin;
    fallbacks += fb;
    recover(ctx, ctx->dnu, ctx->dx, ctx->dlam, ctx->ds);
    HIPCHK(ctx, ipm_step(st, n, m1, m2, 1, ctx->x, ctx->lam, ctx->nu, ctx->s, ctx->dx, ctx->dlam, ctx->dnu, ctx->ds,
                         ctx->isc));
    cg_total += k1 + k2;
    ++it;
    if (ctx->opt.verbose) {
      HIPCHK(ctx, hipMemcpyAsync(ctx->h_isc, ctx->isc, sizeof(IpmScalars), hipMemcpyDeviceToHost, st));
      sync(ctx);
      fprintf(stderr, "[qpgpu] it %3d mu %.3e sigma %.2e alpha %.4f cg %d+%d rel_kkt %.3e fallbacks %d\n", it, mu,
              ctx->h_isc->sigma, ctx->h_isc->alpha, k1, k2, score, fallbacks);
    }
  }
  if (info) {
    info->ipm_iters = it;
    info->pcg_iters_total = cg_total;
    info->rel_kkt = score;
    for (int k = 0; k < 5; ++k) info->rel_kkt_parts[k] = parts[k];
    info->obj = 0.5 * ctx->h_stats[kXHx] + ctx->h_stats[kCx];
    info->mu = ctx->h_stats[kSNu] / m2;
    info->status = status;
    info->refinements_total = refin_total;
    info->fp64_fallbacks = fallbacks;
  }
  if (status != QP_OK && ctx->err.empty()) set_err(ctx, "IPM stopped at rel_kkt %.3e after %d iterations", score, it);
  if (status != QP_OK) throw Fail{(qp_status)status};
}

void alloc_all(qp_ctx* ctx) {
  const int n = ctx->n, m1 = ctx->m1, m2 = ctx->m2, N = ctx->N;
  ctx->H = dalloc<double>(ctx, (size_t)n * ctx->ldn);
  ctx->c = dalloc<double>(ctx, n);
  ctx->A = dalloc<double>(ctx, (size_t)m1 * ctx->ldn);
  ctx->b = dalloc<double>(ctx, m1);
  ctx->C = dalloc<double>(ctx, (size_t)m2 * ctx->ldn);
  ctx->d = dalloc<double>(ctx, m2);
  ctx->Linv = dalloc<double>(ctx, (size_t)N * ctx->ldN);
  for (double** v : {&ctx->x, &ctx->Hx, &ctx->Atl, &ctx->Ctn, &ctx->rg, &ctx->dx, &ctx->dx_a, &ctx->pu, &ctx->pw})
    *v = dalloc<double>(ctx, n);
  for (double** v : {&ctx->lam, &ctx->Ax, &ctx->re, &ctx->dlam, &ctx->dlam_a}) *v = dalloc<double>(ctx, m1);
  for (double** v : {&ctx->nu, &ctx->s, &ctx->Cx, &ctx->ri, &ctx->dvec, &ctx->rc, &ctx->rhs, &ctx->Cw, &ctx->dnu,
                     &ctx->ds, &ctx->dnu_a, &ctx->ds_a, &ctx->pr, &ctx->pz, &ctx->pp, &ctx->pq, &ctx->pt, &ctx->ir_r,
                     &ctx->ir_x, &ctx->ir_d})
    *v = dalloc<double>(ctx, m2);
  for (double** v : {&ctx->vN1, &ctx->vN2, &ctx->vN3, &ctx->pv}) *v = dalloc<double>(ctx, N);
  // gemv_cols partial workspace: chunks * ld with chunks <= 4 * CUs / tiles
  int maxld = std::max(std::max(ctx->ldn, ctx->ldN), ctx->ldm2);
  size_t part = gemv_cols_part_elems(maxld);
  ctx->w64.part = dalloc<double>(ctx, part);
  ctx->w64.part_elems = part;
  ctx->bpart_cap = kMaxRowsBpc * dev_info().cu_count + 64;
  ctx->bpart = dalloc<double>(ctx, ctx->bpart_cap);
  ctx->sc = dalloc<PcgScalars>(ctx, 1);
  ctx->isc = dalloc<IpmScalars>(ctx, 1);
  ctx->stats = dalloc<double>(ctx, 64);
  ctx->info = dalloc<int>(ctx, 16);
  const qp_precond pc = resolve_prec(ctx, ctx->opt.prec);
  const bool need_ph = true;  // qp_pcg_solve may ask for P_H whatever the options say
  (void)pc;
  if (need_ph) {
    ctx->T = dalloc<double>(ctx, (size_t)m2 * ctx->ldm2);
    ctx->P = dalloc<double>(ctx, (size_t)m2 * ctx->ldm2);
    ctx->XP = dalloc<double>(ctx, (size_t)m2 * ctx->ldm2);
    ctx->ptmp = dalloc<double>(ctx, chol_inv_tmp_elems(m2));
  }
  if (ctx->opt.precision == QP_MIXED) {
    ctx->Linv32 = dalloc<float>(ctx, (size_t)N * ctx->ldN);
    ctx->C32 = dalloc<float>(ctx, (size_t)m2 * ctx->ldn);
    ctx->XP32 = dalloc<float>(ctx, (size_t)m2 * ctx->ldm2);
    for (float** v : {&ctx->fr, &ctx->fz, &ctx->fp, &ctx->fq, &ctx->ft, &ctx->fx, &ctx->fb, &ctx->fd, &ctx->fwts})
      *v = dalloc<float>(ctx, m2);
    for (float** v : {&ctx->fu, &ctx->fw}) *v = dalloc<float>(ctx, n);
    ctx->fv = dalloc<float>(ctx, N);
    ctx->w32.part = dalloc<float>(ctx, part);
    ctx->w32.part_elems = part;
  }
  HIPCHK(ctx, hipHostMalloc((void**)&ctx->h_sc, sizeof(PcgScalars), hipHostMallocDefault));
  HIPCHK(ctx, hipHostMalloc((void**)&ctx->h_isc, sizeof(IpmScalars), hipHostMallocDefault));
  HIPCHK(ctx, hipHostMalloc((void**)&ctx->h_stats, 64 * sizeof(double), hipHostMallocDefault));
  HIPCHK(ctx, hipHostMalloc((void**)&ctx->h_info, 16 * sizeof(int), hipHostMallocDefault));
}

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

}  // namespace

// ============================================================================
extern "C" {

void qp_default_options(qp_options* opt) {
  if (!opt) return;
  opt->rtol_kkt = 1e-9;
  opt->cg_theta = 0.1;
  opt->cg_rtol = 1e-12;
  opt->tau = 0.995;
  opt->max_ipm = 200;
  opt->max_pcg = 0;
  opt->poll_every = 32;
  opt->prec = QP_PREC_AUTO;
  opt->precision = QP_FP64;
  opt->verbose = 0;
  opt->profile = 0;
}

const char* qp_status_str(qp_status st) {
  switch (st) {
    case QP_OK: return "ok";
    case QP_E_INVALID: return "invalid argument";
    case QP_E_NOT_SPD: return "H is not positive definite";
    case QP_E_RANK: return "A is rank deficient";
    case QP_E_NOCONV: return "iteration limit reached";
    case QP_E_NOMEM: return "out of device memory";
    case QP_E_DEVICE: return "device error";
    case QP_E_STATE: return "call order violated";
  }
  return "unknown status";
}

const char* qp_last_error(const qp_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

size_t qp_ctx_bytes(const qp_ctx* ctx) { return ctx ? ctx->bytes : 0; }

qp_status qp_profile_get(qp_ctx* ctx, double avg_ms[6], long long samples[6], int reset) {
  if (!ctx || !avg_ms || !samples) return QP_E_INVALID;
  for (int o = 0; o < kProfOps; ++o) {
    samples[o] = ctx->prof_n[o];
    avg_ms[o] = ctx->prof_n[o] ? ctx->prof_ms[o] / (double)ctx->prof_n[o] : 0.0;
    if (reset) {
      ctx->prof_ms[o] = 0;
      ctx->prof_n[o] = 0;
    }
  }
  return QP_OK;
}

void qp_destroy(qp_ctx* ctx) {
  if (!ctx) return;
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  if (ctx->prof_ready)
    for (int o = 0; o < kProfOps; ++o) {
      (void)hipEventDestroy(ctx->prof_ev[o].begin);
      (void)hipEventDestroy(ctx->prof_ev[o].end);
    }
  for (void* p : ctx->allocs) (void)hipFree(p);
  for (void* p : {(void*)ctx->h_sc, (void*)ctx->h_isc, (void*)ctx->h_stats, (void*)ctx->h_info})
    if (p) (void)hipHostFree(p);
  if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

qp_status qp_setup(qp_ctx** out, int n, int m1, int m2, const double* H, const double* c, const double* A,
                   const double* b, const double* C, const double* d, qp_mem where, const qp_options* opt,
                   void* hip_stream) {
  if (!out) return QP_E_INVALID;
  *out = nullptr;
  if (n <= 0 || m1 <= 0 || m1 > n || m2 <= 0) return QP_E_INVALID;
  if (!H || !c || !A || !b || !C || !d) return QP_E_INVALID;
  if (where != QP_MEM_HOST && where != QP_MEM_DEVICE) return QP_E_INVALID;
  if ((long long)(n + m1) * (n + m1) > (1LL << 31) || (long long)m2 * m2 > (1LL << 31)) return QP_E_INVALID;
  qp_options o;
  qp_default_options(&o);
  if (opt) o = *opt;
  if (!(o.tau > 0 && o.tau < 1) || o.max_ipm < 0 || !(o.rtol_kkt > 0) || o.prec < QP_PREC_NONE ||
      o.prec > QP_PREC_AUTO || (o.precision != QP_FP64 && o.precision != QP_MIXED))
    return QP_E_INVALID;
  if (where == QP_MEM_HOST) {
    // finiteness and symmetry checks on the caller's host arrays
    if (!finite_all(H, (size_t)n * n) || !finite_all(c, n) || !finite_all(A, (size_t)m1 * n) ||
        !finite_all(b, m1) || !finite_all(C, (size_t)m2 * n) || !finite_all(d, m2))
      return QP_E_INVALID;
    double fro = 0, asym = 0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double h = H[(size_t)i * n + j];
        double t = h - H[(size_t)j * n + i];
        fro += h * h;
        asym += t * t;
      }
    if (std::sqrt(asym) > 1e-14 * std::max(1.0, std::sqrt(fro))) return QP_E_INVALID;
  }
  qp_ctx* ctx = new qp_ctx();
  ctx->n = n;
  ctx->m1 = m1;
  ctx->m2 = m2;
  ctx->N = n + m1;
  ctx->ldn = ld_for(n);
  ctx->ldN = ld_for(n + m1);
  ctx->ldm2 = ld_for(m2);
  ctx->ldm1 = ld_for(m1);
  ctx->opt = o;
  qp_status st = guarded(ctx, [&] {
    HIPCHK(ctx, hipGetDevice(&ctx->dev));
    (void)dev_info();
    if (hip_stream) {
      ctx->stream = static_cast<hipStream_t>(hip_stream);
    } else {
      HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
      ctx->own_stream = true;
    }
    alloc_all(ctx);
    upload_matrix(ctx, ctx->H, ctx->ldn, H, n, n, where);
    upload_vec(ctx, ctx->c, c, n, where);
    upload_matrix(ctx, ctx->A, ctx->ldn, A, m1, n, where);
    upload_vec(ctx, ctx->b, b, m1, where);
    upload_matrix(ctx, ctx->C, ctx->ldn, C, m2, n, where);
    upload_vec(ctx, ctx->d, d, m2, where);
    if (o.precision == QP_MIXED)
      HIPCHK(ctx, (convert_2d<double, float>(ctx->stream, ctx->C, ctx->ldn, ctx->C32, ctx->ldn, m2, n)));
    sync(ctx);
  });
  if (st != QP_OK) {
    qp_destroy(ctx);
    return st;
  }
  *out = ctx;
  return QP_OK;
}

qp_status qp_factor_K0(qp_ctx* ctx) {
  if (!ctx) return QP_E_INVALID;
  ctx->err.clear();
  return guarded(ctx, [&] {
    ctx->factored = false;
    ctx->ph_ready = false;
    factor(ctx);
    if (resolve_prec(ctx, ctx->opt.prec) == QP_PREC_FEW_EQ) ph_setup(ctx);
    sync(ctx);
  });
}

qp_status qp_k0_solve(qp_ctx* ctx, const double* rhs, double* out, qp_mem where) {
  if (!ctx || !rhs || !out) return QP_E_INVALID;
  if (!ctx->factored) {
    set_err(ctx, "qp_k0_solve before qp_factor_K0");
    return QP_E_STATE;
  }
  return guarded(ctx, [&] {
    upload_vec(ctx, ctx->vN1, rhs, ctx->N, where);
    k0_solve_dev(ctx, ctx->vN1, ctx->vN2, ctx->vN3);
    download_vec(ctx, out, ctx->vN2, ctx->N, where);
    sync(ctx);
  });
}

qp_status qp_kf_apply(qp_ctx* ctx, const double* dvec, const double* p, double* q, qp_mem where) {
  if (!ctx || !dvec || !p || !q) return QP_E_INVALID;
  if (!ctx->factored) {
    set_err(ctx, "qp_kf_apply before qp_factor_K0");
    return QP_E_STATE;
  }
  return guarded(ctx, [&] {
    upload_vec(ctx, ctx->dvec, dvec, ctx->m2, where);
    upload_vec(ctx, ctx->ir_r, p, ctx->m2, where);
    kf_apply_dev(ctx, ctx->dvec, ctx->ir_r, ctx->ir_x);
    download_vec(ctx, q, ctx->ir_x, ctx->m2, where);
    sync(ctx);
  });
}

qp_status qp_pcg_solve(qp_ctx* ctx, const double* dvec, const double* rhs, double* dnu, qp_mem where,
                       qp_precond prec, double rtol, int maxit, qp_pcg_info* info) {
  if (!ctx || !dvec || !rhs || !dnu) return QP_E_INVALID;
  if (prec < QP_PREC_NONE || prec > QP_PREC_AUTO || !(rtol >= 0)) return QP_E_INVALID;
  if (!ctx->factored) {
    set_err(ctx, "qp_pcg_solve before qp_factor_K0");
    return QP_E_STATE;
  }
  ctx->err.clear();
  int code = 0;
  qp_status st = guarded(ctx, [&] {
    const int m2 = ctx->m2;
    if (where == QP_MEM_HOST) {
      for (int i = 0; i < m2; ++i)
        if (!(dvec[i] > 0) || !std::isfinite(dvec[i]) || !std::isfinite(rhs[i])) {
          set_err(ctx, "dvec must be positive and finite, rhs finite");
          throw Fail{QP_E_INVALID};
        }
    }
    qp_precond pc = resolve_prec(ctx, prec);
    int mode = prec_mode(pc);
    upload_vec(ctx, ctx->dvec, dvec, m2, where);
    upload_vec(ctx, ctx->rhs, rhs, m2, where);
    if (mode == kPrecH) {
      ph_setup(ctx);
      ph_factor(ctx, ctx->dvec);
      HIPCHK(ctx, hipMemcpyAsync(ctx->h_info, ctx->info, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
      sync(ctx);
      if (*ctx->h_info) {
        set_err(ctx, "Cholesky of D + C H^{-1} C^T failed");
        throw Fail{QP_E_INVALID};
      }
    }
    int mi = maxit > 0 ? maxit : 10 * m2;
    int done = 0, refin = 0, fb = 0;
    int iters = reduced_solve(ctx, mode, ctx->dvec, ctx->rhs, ctx->dnu, nullptr, rtol, -1.0, mi, &done, &refin, &fb);
    // true residual in float64
    kf_apply_dev(ctx, ctx->dvec, ctx->dnu, ctx->ir_x);
    HIPCHK(ctx, ir_residual(ctx->stream, m2, ctx->rhs, ctx->ir_x, nullptr, ctx->ir_r, ctx->sc));
    HIPCHK(ctx, hipMemcpyAsync(ctx->h_sc, ctx->sc, sizeof(PcgScalars), hipMemcpyDeviceToHost, ctx->stream));
    download_vec(ctx, dnu, ctx->dnu, m2, where);
    sync(ctx);
    double rel = ctx->h_sc->bb > 0 ? std::sqrt(ctx->h_sc->rr / ctx->h_sc->bb) : 0.0;
    if (info) {
      info->iters = iters;
      info->rel_res = rel;
      info->refinements = refin;
      info->fp64_fallback = fb;
    }
    code = done;
    if (done == 3) {
      set_err(ctx, "PCG breakdown (p^T q <= 0)");
      throw Fail{QP_E_NOCONV};
    }
    if (done != 1) {
      set_err(ctx, "PCG reached %d iterations, relative residual %.3e", iters, rel);
      throw Fail{QP_E_NOCONV};
    }
  });
  if (info) info->status = st;
  (void)code;
  return st;
}

qp_status qp_op_time(qp_ctx* ctx, int op, qp_precision precision, int reps, double* avg_ms) {
  if (!ctx || !avg_ms || reps <= 0 || op < 0 || op > 4) return QP_E_INVALID;
  if (precision != QP_FP64 && precision != QP_MIXED) return QP_E_INVALID;
  if (precision == QP_MIXED && ctx->opt.precision != QP_MIXED) {
    set_err(ctx, "float32 operator copies exist only in a QP_MIXED context");
    return QP_E_STATE;
  }
  if (!ctx->factored) {
    set_err(ctx, "qp_op_time before qp_factor_K0");
    return QP_E_STATE;
  }
  ctx->err.clear();
  return guarded(ctx, [&] {
    hipStream_t st = ctx->stream;
    const int n = ctx->n, m2 = ctx->m2;
    hipEvent_t e0, e1;
    HIPCHK(ctx, hipEventCreate(&e0));
    HIPCHK(ctx, hipEventCreate(&e1));
    auto run = [&](auto tag) {
      using T = decltype(tag);
      PcgBufs<T> B;
      if constexpr (sizeof(T) == 8) {
        B = bufs64(ctx, ctx->dvec, nullptr, ctx->dnu);
      } else {
        B = bufs32(ctx);
        B.wts = nullptr;
      }
      // deterministic operands: p = 1, d = 1, a CG state that is far from convergence
      HIPCHK(ctx, fill_vec<T>(st, m2, T(1), const_cast<T*>(B.dvec)));
      HIPCHK(ctx, fill_vec<T>(st, m2, T(1), B.q));
      HIPCHK(ctx, pcg_init<T>(st, m2, B.q, B.dvec, nullptr, B.x, B.r, B.z, B.p, kPrecL, 0.0, -1.0, 1 << 30,
                              ctx->sc));
      HIPCHK(ctx, fill_vec<T>(st, n, T(1), B.u));
      HIPCHK(ctx, fill_vec<T>(st, ctx->N, T(1), B.v));
      HIPCHK(ctx, fill_vec<T>(st, n, T(1), B.w));
      auto launch = [&]() {
        switch (op) {
          case 0:
            HIPCHK(ctx, launch_gemv_cols<T>(st, B.C, ctx->ldn, m2, n, kDense, B.p, B.u, T(1), T(0), nullptr, *B.wk,
                                            nullptr, 1));
            break;
          case 1:
            HIPCHK(ctx, launch_gemv_rows<T>(st, B.Linv, ctx->ldN, ctx->N, n, kLower, B.u, B.v, T(1), T(0), nullptr, n,
                                            nullptr, 2));
            break;
          case 2:
            HIPCHK(ctx, launch_gemv_cols<T>(st, B.Linv, ctx->ldN, ctx->N, n, kLower, B.v, B.w, T(1), T(0), nullptr,
                                            *B.wk, nullptr, 3));
            break;
          case 3:
            HIPCHK(ctx, launch_gemv_rows<T>(st, B.C, ctx->ldn, m2, n, kDense, B.w, B.q, T(1), T(0), nullptr, m2,
                                            nullptr, 0));
            break;
          case 4: {
            const int* skip = &ctx->sc->done;
            HIPCHK(ctx, launch_gemv_cols<T>(st, B.C, ctx->ldn, m2, n, kDense, B.p, B.u, T(1), T(0), nullptr, *B.wk,
                                            skip, 1));
            k0_top_apply<T>(ctx, B.Linv, B.u, B.v, B.w, *B.wk, skip);
            HIPCHK(ctx, pcg_q<T>(st, B.C, ctx->ldn, m2, n, B.w, B.dvec, B.p, B.q, ctx->sc, ctx->bpart,
                                 ctx->bpart_cap));
            HIPCHK(ctx, pcg_update<T>(st, m2, ctx->bpart, B.dvec, B.p, B.q, B.x, B.r, B.z, nullptr, kPrecL, ctx->sc));
            break;
          }
        }
      };
      launch();  // warm-up
      HIPCHK(ctx, hipEventRecord(e0, st));
      for (int k = 0; k < reps; ++k) launch();
      HIPCHK(ctx, hipEventRecord(e1, st));
      HIPCHK(ctx, hipEventSynchronize(e1));
      float ms = 0;
      HIPCHK(ctx, hipEventElapsedTime(&ms, e0, e1));
      *avg_ms = ms / reps;
      if (op == 4) {
        HIPCHK(ctx, hipMemcpy(ctx->h_sc, ctx->sc, sizeof(PcgScalars), hipMemcpyDeviceToHost));
        if (ctx->h_sc->done) {
          set_err(ctx, "CG state stopped during the timing loop (done=%d)", ctx->h_sc->done);
          throw Fail{QP_E_NOCONV};
        }
      }
    };
    if (precision == QP_MIXED)
      run(float(0));
    else
      run(double(0));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  });
}

qp_status qp_ipm_solve(qp_ctx* ctx, double* x, double* lambda, double* nu, double* s, qp_mem where,
                       qp_ipm_info* info) {
  if (!ctx || !x || !lambda || !nu || !s) return QP_E_INVALID;
  if (!ctx->factored) {
    set_err(ctx, "qp_ipm_solve before qp_factor_K0");
    return QP_E_STATE;
  }
  ctx->err.clear();
  auto t0 = std::chrono::steady_clock::now();
  qp_status st = guarded(ctx, [&] { ipm_run(ctx, info); });
  qp_status st2 = guarded(ctx, [&] {
    download_vec(ctx, x, ctx->x, ctx->n, where);
    download_vec(ctx, lambda, ctx->lam, ctx->m1, where);
    download_vec(ctx, nu, ctx->nu, ctx->m2, where);
    download_vec(ctx, s, ctx->s, ctx->m2, where);
    sync(ctx);
  });
  auto t1 = std::chrono::steady_clock::now();
  if (info) {
    info->status = st;
    info->t_solve_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
  }
  return st != QP_OK ? st : st2;
}

}  // extern "C"
