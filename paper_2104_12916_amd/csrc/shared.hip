// QPs that share H, A and C: one factorization of K0, k right-hand sides.
//
// A qp_shared owns a master context (H, A, C, L^{-1}, C^T and M^T, factorized
// once) and up to k member contexts that alias those matrices and own only the
// per-QP vectors (c, b, d, the iterate, residuals, CG vectors).  Each member
// runs the interior point iteration of Sec. 2 with the phases of api.hip; the
// reduced solves of all members run together as a block PCG: every CG step
// applies C K0^{-1}_{11} C^T = C M^T Sigma M C^T to the k direction vectors with
// four multi-vector sweeps (block.hip), which stream each matrix once for all k,
// while the scalars, stop tests and preconditioner (P_L or none) stay per QP
// (the update kernel of the batched PCG, one workgroup per QP).  The members'
// IPMs advance in lockstep; a QP that has converged leaves the block.
#include <cmath>
#include <vector>

#include "ctx.hpp"

namespace qpg {
hipError_t launch_mv_rows(hipStream_t st, const double* A, int lda, int rows, int K, int shape, const double* X,
                          int ldx, int nv, double* Y, int ldy, double alpha, int nsplit, double* part,
                          size_t part_elems);
size_t mv_part_elems(int rows, int K, int nv);
hipError_t bq_epilogue(hipStream_t st, const PcgDesc<double>* d, int count);
}  // namespace qpg

using namespace qpg;
using namespace qpg::detail;

struct qp_shared {
  qp_ctx* master = nullptr;
  std::vector<qp_ctx*> members;
  // block vectors, column-major with leading dimension ld: P, R, Z, Q (m2),
  // U, W (n) and V (N) per QP
  int ld = 0, kcap = 0;
  double *P = nullptr, *U = nullptr, *V = nullptr, *W = nullptr, *Q = nullptr, *R = nullptr, *Z = nullptr;
  double* pq = nullptr;              // p_j^T q_j (one per QP)
  double* part = nullptr;            // per-slice partials of the multi-vector sweeps
  size_t part_elems = 0;
  PcgScalars* sc = nullptr;          // CG scalars (one per QP)
  PcgScalars* h_sc = nullptr;        // pinned mirror
  PcgDesc<double>* d_desc = nullptr; // device copy of the block's PcgDesc list
  PcgDesc<double>* h_desc = nullptr; // pinned staging of the list
  std::vector<void*> allocs;
  std::string err;
};

namespace {

qp_ctx* sink(qp_shared* sh) { return sh->master; }

template <typename T>
T* shalloc(qp_shared* sh, size_t elems) {
  void* p = nullptr;
  HIPCHK(sink(sh), hipMalloc(&p, std::max<size_t>(elems, 1) * sizeof(T)));
  sh->allocs.push_back(p);
  return static_cast<T*>(p);
}

// Members 0..k-1 and block workspace for k QPs.
void ensure_members(qp_shared* sh, int k) {
  qp_ctx* m = sh->master;
  while ((int)sh->members.size() < k) {
    qp_ctx* c = new qp_ctx();
    init_dims(c, m->n, m->m1, m->m2, m->opt);
    c->master = m;
    c->dev = m->dev;
    c->stream = m->stream;
    sh->members.push_back(c);
    alloc_all(c);
    c->H = m->H;
    c->A = m->A;
    c->C = m->C;
    c->Linv = m->Linv;
    c->CT = m->CT;
    c->MT = m->MT;
    c->factored = true;
    c->c_identity = m->c_identity;
  }
  if (k <= sh->kcap) return;
  for (void* p : sh->allocs) (void)hipFree(p);
  sh->allocs.clear();
  if (sh->h_sc) (void)hipHostFree(sh->h_sc);
  if (sh->h_desc) (void)hipHostFree(sh->h_desc);
  sh->h_sc = nullptr;
  sh->h_desc = nullptr;
  const int n = m->n, m2 = m->m2, N = m->N;
  sh->ld = (std::max(std::max(n, m2), N) + 63) / 64 * 64;
  const size_t blk = (size_t)sh->ld * k;
  for (double** v : {&sh->P, &sh->U, &sh->V, &sh->W, &sh->Q, &sh->R, &sh->Z}) *v = shalloc<double>(sh, blk);
  sh->pq = shalloc<double>(sh, k);
  sh->part_elems = std::max(std::max(mv_part_elems(n, m2, k), mv_part_elems(N, n, k)),
                            std::max(mv_part_elems(n, N, k), mv_part_elems(m2, n, k)));
  sh->part = shalloc<double>(sh, sh->part_elems);
  sh->sc = shalloc<PcgScalars>(sh, k);
  sh->d_desc = shalloc<PcgDesc<double>>(sh, k);
  HIPCHK(m, hipHostMalloc((void**)&sh->h_sc, k * sizeof(PcgScalars), hipHostMallocDefault));
  HIPCHK(m, hipHostMalloc((void**)&sh->h_desc, k * sizeof(PcgDesc<double>), hipHostMallocDefault));
  // the direction block is read past m2 (up to the padded length) by no kernel, but keep it defined
  HIPCHK(m, hipMemsetAsync(sh->P, 0, blk * sizeof(double), m->stream));
  sh->kcap = k;
}

struct BlockSolve {
  qp_ctx* c;
  double* x;          // solution (the member's dnu_a or dnu)
  const double* rhs;
  const double* wts;  // weights of the stop test (nu) or null
  double rtol, wtol;
  int maxit;
  int iters = 0, done = 0;
};

// Block PCG (P_L or none) over the listed solves; x starts at zero.
void block_pcg(qp_shared* sh, std::vector<BlockSolve>& js, int prec) {
  qp_ctx* m = sh->master;
  hipStream_t st = m->stream;
  const int k = (int)js.size();
  if (!k) return;
  const int n = m->n, m2 = m->m2, N = m->N, ld = sh->ld;
  for (int j = 0; j < k; ++j) {
    PcgDesc<double>& d = sh->h_desc[j];
    d = PcgDesc<double>{};
    d.C = nullptr;
    d.w = nullptr;
    d.dvec = js[j].c->dvec;
    d.wts = js[j].wts;
    d.b = js[j].rhs;
    d.x = js[j].x;
    d.r = sh->R + (size_t)j * ld;
    d.z = sh->Z + (size_t)j * ld;
    d.p = sh->P + (size_t)j * ld;
    d.q = (m->c_identity ? sh->W : sh->Q) + (size_t)j * ld;  // C = I: q = w + D p
    d.bpart = sh->pq + j;
    d.sc = sh->sc + j;
    d.rtol = js[j].rtol;
    d.wtol = js[j].wtol;
    d.maxit = js[j].maxit;
    d.ldc = m->ldn;
    d.n = n;
    d.m2 = m2;
    d.prec = prec;
    d.qblocks = 1;
    d.stage = 0;
  }
  HIPCHK(m, hipMemcpyAsync(sh->d_desc, sh->h_desc, k * sizeof(PcgDesc<double>), hipMemcpyHostToDevice, st));
  HIPCHK(m, bpcg_init<double>(st, sh->d_desc, k));
  const int poll = m->opt.poll_every > 0 ? m->opt.poll_every : 32;
  int maxit = 0;
  for (auto& j : js) maxit = std::max(maxit, j.maxit);
  long long launched = 0;
  for (;;) {
    if (launched > (long long)maxit + 2LL * poll) {
      set_err(m, "block PCG made no progress after %lld launched steps", launched);
      throw Fail{QP_E_DEVICE};
    }
    launched += poll;
    for (int s = 0; s < poll; ++s) {
      const double* U = sh->U;
      if (m->c_identity)
        U = sh->P;
      else
        HIPCHK(m, launch_mv_rows(st, m->CT, m->ldm2, n, m2, kDense, sh->P, ld, k, sh->U, ld, 1.0, n, sh->part,
                                 sh->part_elems));
      HIPCHK(m, launch_mv_rows(st, m->Linv, m->ldN, N, n, kLower, U, ld, k, sh->V, ld, 1.0, n, sh->part,
                               sh->part_elems));  // Sigma M u
      HIPCHK(m, launch_mv_rows(st, m->MT, m->ldN, n, N, kUpper, sh->V, ld, k, sh->W, ld, 1.0, n, sh->part,
                               sh->part_elems));  // M^T v
      if (!m->c_identity)
        HIPCHK(m, launch_mv_rows(st, m->C, m->ldn, m2, n, kDense, sh->W, ld, k, sh->Q, ld, 1.0, m2, sh->part,
                                 sh->part_elems));
      HIPCHK(m, bq_epilogue(st, sh->d_desc, k));
      HIPCHK(m, bpcg_update<double>(st, sh->d_desc, k));
    }
    HIPCHK(m, hipMemcpyAsync(sh->h_sc, sh->sc, k * sizeof(PcgScalars), hipMemcpyDeviceToHost, st));
    HIPCHK(m, hipStreamSynchronize(st));
    bool all = true;
    for (int j = 0; j < k; ++j) all = all && sh->h_sc[j].done;
    if (all) break;
  }
  for (int j = 0; j < k; ++j) {
    js[j].iters = sh->h_sc[j].iter;
    js[j].done = sh->h_sc[j].done;
  }
}

int block_prec(qp_shared* sh, qp_precond p) {
  if (p == QP_PREC_FEW_EQ) {
    set_err(sh->master, "shared-matrix solves take P_L or no preconditioner (P_H is per QP)");
    throw Fail{QP_E_INVALID};
  }
  return p == QP_PREC_NONE ? kPrecNone : kPrecL;  // QP_PREC_AUTO: P_L
}

}  // namespace

extern "C" {

qp_status qp_shared_setup(qp_shared** out, int n, int m1, int m2, const double* H, const double* A, const double* C,
                          qp_mem where, const qp_options* opt, void* hip_stream) {
  if (!out) return QP_E_INVALID;
  *out = nullptr;
  if (n <= 0 || m1 <= 0 || m1 > n || m2 <= 0 || !H || !A || !C) return QP_E_INVALID;
  qp_options o;
  qp_default_options(&o);
  if (opt) o = *opt;
  if (check_options(o) != QP_OK) return QP_E_INVALID;
  if (o.precision != QP_FP64 || o.kf_form != QP_KF_IMPLICIT || o.prec == QP_PREC_FEW_EQ) return QP_E_INVALID;
  // the master's own c, b, d are zero (each member brings its own)
  std::vector<double> zc(n, 0.0), zb(m1, 0.0), zd(m2, 0.0);
  const double *c0 = zc.data(), *b0 = zb.data(), *d0 = zd.data();
  qp_status pst = check_problem(n, m1, m2, H, c0, A, b0, C, d0, where);
  if (pst != QP_OK) return pst;
  qp_shared* sh = new qp_shared();
  qp_ctx* m = new qp_ctx();
  sh->master = m;
  init_dims(m, n, m1, m2, o);
  m->keep_mt = true;
  qp_status st = guarded(m, [&] {
    HIPCHK(m, hipGetDevice(&m->dev));
    (void)dev_info();
    if (hip_stream) {
      m->stream = static_cast<hipStream_t>(hip_stream);
    } else {
      HIPCHK(m, hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking));
      m->own_stream = true;
    }
    alloc_all(m);
    upload_matrix(m, m->H, m->ldn, H, n, n, where);
    upload_matrix(m, m->A, m->ldn, A, m1, n, where);
    upload_matrix(m, m->C, m->ldn, C, m2, n, where);
    HIPCHK(m, hipMemsetAsync(m->c, 0, n * sizeof(double), m->stream));
    HIPCHK(m, hipMemsetAsync(m->b, 0, m1 * sizeof(double), m->stream));
    HIPCHK(m, hipMemsetAsync(m->d, 0, m2 * sizeof(double), m->stream));
    factor(m);
    sync(m);
  });
  if (st != QP_OK) {
    sh->err = m->err;
    qp_shared_destroy(sh);
    return st;
  }
  *out = sh;
  return QP_OK;
}

qp_status qp_shared_pcg_solve(qp_shared* sh, int k, const double* dvec, const double* rhs, double* dnu, qp_mem where,
                              qp_precond prec, double rtol, int maxit, qp_pcg_info* info) {
  if (!sh || k <= 0 || !dvec || !rhs || !dnu || !(rtol >= 0)) return QP_E_INVALID;
  if (prec < QP_PREC_NONE || prec > QP_PREC_AUTO) return QP_E_INVALID;
  qp_ctx* m = sh->master;
  m->err.clear();
  TuneScope tune_scope(m->n);
  qp_status st = guarded(m, [&] {
    const int m2 = m->m2;
    const int mode = block_prec(sh, prec);
    if (where == QP_MEM_HOST)
      for (size_t i = 0; i < (size_t)k * m2; ++i)
        if (!(dvec[i] > 0) || !std::isfinite(dvec[i]) || !std::isfinite(rhs[i])) {
          set_err(m, "dvec must be positive and finite, rhs finite");
          throw Fail{QP_E_INVALID};
        }
    ensure_members(sh, k);
    std::vector<BlockSolve> js(k);
    for (int j = 0; j < k; ++j) {
      qp_ctx* c = sh->members[j];
      upload_vec(c, c->dvec, dvec + (size_t)j * m2, m2, where);
      upload_vec(c, c->rhs, rhs + (size_t)j * m2, m2, where);
      js[j] = BlockSolve{c, c->dnu, c->rhs, nullptr, rtol, -1.0, maxit > 0 ? maxit : 10 * m2};
    }
    block_pcg(sh, js, mode);
    // true residuals in float64, one QP at a time
    for (int j = 0; j < k; ++j) {
      qp_ctx* c = sh->members[j];
      kf_apply_dev(c, c->dvec, c->dnu, c->ir_x);
      HIPCHK(c, ir_residual(c->stream, m2, c->rhs, c->ir_x, nullptr, c->ir_r, c->sc));
      HIPCHK(c, hipMemcpyAsync(c->h_sc, c->sc, sizeof(PcgScalars), hipMemcpyDeviceToHost, c->stream));
      download_vec(c, dnu + (size_t)j * m2, c->dnu, m2, where);
      sync(c);
      const double rel = c->h_sc->bb > 0 ? std::sqrt(c->h_sc->rr / c->h_sc->bb) : 0.0;
      if (info) {
        info[j].iters = js[j].iters;
        info[j].rel_res = rel;
        info[j].refinements = 0;
        info[j].fp64_fallback = 0;
        info[j].status = js[j].done == 1 ? QP_OK : QP_E_NOCONV;
      }
    }
    for (int j = 0; j < k; ++j)
      if (js[j].done != 1) {
        set_err(m, "block PCG: solve %d stopped with code %d after %d steps", j, js[j].done, js[j].iters);
        throw Fail{QP_E_NOCONV};
      }
  });
  return st;
}

qp_status qp_shared_ipm_solve(qp_shared* sh, int k, const double* c, const double* b, const double* d, double* x,
                              double* lambda, double* nu, double* s, qp_mem where, qp_ipm_info* info) {
  if (!sh || k <= 0 || !c || !b || !d || !x || !lambda || !nu || !s) return QP_E_INVALID;
  qp_ctx* m = sh->master;
  m->err.clear();
  TuneScope tune_scope(m->n);
  const int n = m->n, m1 = m->m1, m2 = m->m2;
  std::vector<IpmRun> R(k);
  qp_status st = guarded(m, [&] {
    const int mode = block_prec(sh, m->opt.prec);
    ensure_members(sh, k);
    std::vector<qp_ctx*> mem(sh->members.begin(), sh->members.begin() + k);
    for (int j = 0; j < k; ++j) {
      qp_ctx* q = mem[j];
      upload_vec(q, q->c, c + (size_t)j * n, n, where);
      upload_vec(q, q->b, b + (size_t)j * m1, m1, where);
      upload_vec(q, q->d, d + (size_t)j * m2, m2, where);
      q->cg_trace.clear();
      q->opt.prec = mode == kPrecNone ? QP_PREC_NONE : QP_PREC_LOW_DOF;  // no P_H set-up on a member
      ipm_start(q, R[j]);
    }
    std::vector<int> active(k);
    for (int j = 0; j < k; ++j) active[j] = j;
    while (!active.empty()) {
      for (int j : active) ipm_eval_launch(mem[j], true);
      sync(m);
      std::vector<int> next;
      for (int j : active)
        if (ipm_check(mem[j], R[j])) next.push_back(j);
      active.swap(next);
      if (active.empty()) break;
      for (int j : active) ipm_predictor_setup(mem[j], R[j]);
      std::vector<BlockSolve> js;
      for (int j : active) {
        qp_ctx* q = mem[j];
        js.push_back(BlockSolve{q, q->dnu_a, q->rhs, q->nu, q->opt.cg_rtol, R[j].wtol, R[j].maxit});
      }
      block_pcg(sh, js, mode);
      for (size_t t = 0; t < active.size(); ++t) {
        R[active[t]].k1 = js[t].iters;
        ipm_after_predictor(mem[active[t]]);
      }
      for (size_t t = 0; t < active.size(); ++t) js[t].x = mem[active[t]]->dnu;
      block_pcg(sh, js, mode);
      for (size_t t = 0; t < active.size(); ++t) {
        R[active[t]].k2 = js[t].iters;
        ipm_after_corrector(mem[active[t]], R[active[t]]);
      }
    }
    for (int j = 0; j < k; ++j) {
      qp_ctx* q = mem[j];
      download_vec(q, x + (size_t)j * n, q->x, n, where);
      download_vec(q, lambda + (size_t)j * m1, q->lam, m1, where);
      download_vec(q, nu + (size_t)j * m2, q->nu, m2, where);
      download_vec(q, s + (size_t)j * m2, q->s, m2, where);
    }
    sync(m);
    for (int j = 0; j < k; ++j) {
      if (info) ipm_fill_info(mem[j], R[j], &info[j]);
      if (R[j].status != QP_OK) {
        set_err(m, "QP %d: IPM stopped at rel_kkt %.3e after %d iterations", j, R[j].score, R[j].it);
        throw Fail{(qp_status)R[j].status};
      }
    }
  });
  return st;
}

const char* qp_shared_last_error(const qp_shared* sh) {
  if (!sh) return "";
  if (sh->master && !sh->master->err.empty()) return sh->master->err.c_str();
  return sh->err.c_str();
}

void qp_shared_destroy(qp_shared* sh) {
  if (!sh) return;
  if (sh->master && sh->master->stream) (void)hipStreamSynchronize(sh->master->stream);
  for (void* p : sh->allocs) (void)hipFree(p);
  if (sh->h_sc) (void)hipHostFree(sh->h_sc);
  if (sh->h_desc) (void)hipHostFree(sh->h_desc);
  for (qp_ctx* c : sh->members) qp_destroy(c);
  qp_destroy(sh->master);
  delete sh;
}

}  // extern "C"
