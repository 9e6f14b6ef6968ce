// Batch driver: many independent QPs of different sizes in flight on one
// stream, each advancing through its own interior point iteration (Sec. 2
// predictor-corrector on the reduced system of eq. ineq-const-reduced).
//
// Scheduling is by ticks.  A tick runs one chunk of CG steps (poll_every of
// them) for every QP that is inside a reduced solve, as one launch per sweep
// over a descriptor list (desc.hpp) covering all of those QPs, so the K0
// inverse factors, the C matrices and the P_H factors of all of them stream
// through HBM in the same launches.  Then the host waits once, reads every
// QP's CG scalars and residual statistics, and moves each QP as far as it can
// go without another host decision: KKT check, right-hand side and P_H factor,
// start of the next solve, recovery and step, refinement residuals (mixed
// precision).  Those steps are batched too, over the QPs at the same point.  A
// QP whose solve ends early moves on at the next tick instead of waiting for
// the slowest QP, and QPs admitted between ticks start at the next one.  Each
// QP's arithmetic and launch shapes depend only on that QP, so its result does
// not depend on which other QPs share the batch or when they arrived.
//
// Admission is by memory: every QP's buffers come from one arena of the
// budget given at creation, so admitting and retiring QPs never calls hipMalloc
// or hipFree.  Results are copied to host memory when a QP finishes and its
// device memory returns to the arena at once.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <unordered_map>

#include "ctx.hpp"

using namespace qpg;
using namespace qpg::detail;

namespace {

using Clock = std::chrono::steady_clock;

enum SlotState : int { kQueued = 0, kRunning = 1, kFinished = 2 };

template <typename T>
struct BItem {
  qp_ctx* ctx = nullptr;
  PcgBufs<T> bufs{};
  const T* rhs = nullptr;
  int prec = 0;
  double rtol = 0, wtol = -1;
  int maxit = 0;
  int iters = 0, done = 0;
};

// Where a QP is in its interior point iteration (the batch advances each QP
// on its own; a tick moves every QP as far as it can go without a host decision).
enum Phase : int {
  kPhQueued = 0,     // admitted, not factored yet
  kPhAwaitStats = 1, // residual statistics launched; the KKT check needs them on the host
  kPhSolve = 2,      // a CG solve of a reduced system is running (in cg64 or cg32)
  kPhAwaitIR = 3,    // mixed precision: refinement residual launched; the next step needs it
  kPhDone = 4
};

struct Slot {
  qp_ctx* ctx = nullptr;
  long long ticket = 0;
  int pool = -1;
  int state = kQueued;
  int phase = kPhQueued;
  IpmRun R;
  // the reduced solve in flight: which system, CG steps and refinement state
  int which = 0;  // 0 predictor, 1 corrector
  int s_iters = 0, s_refin = 0, s_fb = 0, s_done = 0, last_done = 0;
  int s_iters64 = 0;  // mixed precision: CG steps of the float64 fallback run
  double prev_rr = -1.0, rtol64 = 0.0;
  long long launched = 0;  // CG steps launched for the current CG run
  BItem<double> it64{};    // current float64 CG run
  BItem<float> it32{};     // current float32 CG run (mixed precision)
  qp_status status = QP_OK;
  std::string err;
  int n = 0, m1 = 0, m2 = 0;
  std::vector<double> x, lam, nu, s;
  qp_ipm_info info{};
  Clock::time_point t_admit, t_done;
};

constexpr int kMaxSlots = 4096;  // QPs in flight at once (scalar pool entries)
constexpr int kInfoStride = 16;

}  // namespace

struct qp_batch {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int dev = 0;
  qp_options opt{};
  Arena arena;
  qp_ctx sink;  // error text and stream for batch-level failures
  // scalar pools indexed by Slot::pool
  PcgScalars *d_sc = nullptr, *h_sc = nullptr;
  double *d_stats = nullptr, *h_stats = nullptr;
  int *d_info = nullptr, *h_info = nullptr;
  IpmScalars* h_isc = nullptr;
  std::vector<int> free_pools;
  std::vector<Slot*> live;                          // queued and running, admission order
  std::vector<Slot*> cg64, cg32;                    // QPs whose current CG run is float64 / float32
  std::unordered_map<long long, Slot*> finished;    // waiting for qp_batch_collect
  long long next_ticket = 1;
  // descriptor staging: a ring of pinned host areas and their device copies;
  // an area is rewritten once the event after its last copy has passed
  struct StageArea {
    char *h = nullptr, *d = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool used = false;
  };
  static constexpr int kStageAreas = 32;
  StageArea stage[kStageAreas];
  int stage_next = 0;
  // per-QP records of the batched IPM kernels, indexed by pool entry
  IpmDesc* d_ipm = nullptr;
  long long rounds = 0;
  long long cg_launched = 0;  // batched CG steps launched
  // sampled sweeps (options.profile): the first CG step of every poll chunk is
  // stamped with HIP events; bytes are the algorithmic matrix bytes of that
  // launch over the QPs it covered.  Order: C^T p, Sigma M u, M^T v,
  // q = C w + D p, X_P r, X_P^T t.
  EventPair prof_ev[kProfOps] = {};
  bool prof_ready = false;
  double prof_ms[kProfOps] = {};
  double prof_bytes[kProfOps] = {};
  double prof_pending_bytes[kProfOps] = {};
  long long prof_n[kProfOps] = {};
};

namespace {

// ---- descriptor staging ---------------------------------------------------------
struct Packer {
  std::vector<std::pair<const void*, size_t>> parts;
  std::deque<std::vector<int>> owned;  // tables built for the upload (stable addresses)
  size_t total = 0;
  size_t add(const void* p, size_t bytes) {
    size_t off = total;
    parts.emplace_back(p, bytes);
    total += (bytes + 255) / 256 * 256;
    return off;
  }
  size_t add_owned(std::vector<int>&& v) {
    owned.push_back(std::move(v));
    return add(owned.back().data(), owned.back().size() * sizeof(int));
  }
};

// Copy the packed sections to the device.  Only called right after the stream
// was synchronized, so the pinned staging area is no longer being read.
void bsync(qp_batch* B) { HIPCHK(&B->sink, hipStreamSynchronize(B->stream)); }

// Copy the packed sections to the device through the next staging area and
// return the device address of the first section.  Launches that read the
// sections follow on the same stream.
const char* stage_upload(qp_batch* B, Packer& pk) {
  qp_ctx* sk = &B->sink;
  qp_batch::StageArea& a = B->stage[B->stage_next];
  B->stage_next = (B->stage_next + 1) % qp_batch::kStageAreas;
  if (a.used) HIPCHK(sk, hipEventSynchronize(a.ev));  // the host area's previous copy has been read
  if (pk.total > a.cap) {
    bsync(B);  // nothing in flight may still read the old device area
    if (a.h) (void)hipHostFree(a.h);
    if (a.d) (void)hipFree(a.d);
    a.h = a.d = nullptr;
    a.cap = 0;
    const size_t cap = std::max(pk.total * 2, (size_t)1 << 20);
    HIPCHK(sk, hipHostMalloc((void**)&a.h, cap, hipHostMallocDefault));
    HIPCHK(sk, hipMalloc((void**)&a.d, cap));
    a.cap = cap;
  }
  if (!a.ev) HIPCHK(sk, hipEventCreateWithFlags(&a.ev, hipEventDisableTiming));
  size_t off = 0;
  for (auto& pr : pk.parts) {
    if (pr.second) memcpy(a.h + off, pr.first, pr.second);
    off += (pr.second + 255) / 256 * 256;
  }
  HIPCHK(sk, hipMemcpyAsync(a.d, a.h, pk.total, hipMemcpyHostToDevice, B->stream));
  HIPCHK(sk, hipEventRecord(a.ev, B->stream));
  a.used = true;
  return a.d;
}

// Upload the descriptor lists of recorded factorization launches and run them.
void run_ops(qp_batch* B, const BatchedOps& ops) {
  if (ops.empty()) return;
  Packer pk;
  pk.add(ops.bytes().data(), ops.bytes().size());
  const char* base = stage_upload(B, pk);
  HIPCHK(&B->sink, ops.run(B->stream, base));
}

void sync_pools(qp_batch* B, int lo, int hi, bool stats) {
  qp_ctx* sk = &B->sink;
  if (hi >= lo && (lo < 0 || hi >= kMaxSlots)) {
    set_err(sk, "internal: pool range [%d, %d] outside the pools", lo, hi);
    throw Fail{QP_E_DEVICE};
  }
  if (hi >= lo) {
    HIPCHK(sk, hipMemcpyAsync(B->h_sc + lo, B->d_sc + lo, (size_t)(hi - lo + 1) * sizeof(PcgScalars),
                              hipMemcpyDeviceToHost, B->stream));
    if (stats) {
      HIPCHK(sk, hipMemcpyAsync(B->h_stats + (size_t)lo * kStatsStride, B->d_stats + (size_t)lo * kStatsStride,
                                (size_t)(hi - lo + 1) * kStatsStride * sizeof(double), hipMemcpyDeviceToHost,
                                B->stream));
      HIPCHK(sk, hipMemcpyAsync(B->h_info + (size_t)lo * kInfoStride, B->d_info + (size_t)lo * kInfoStride,
                                (size_t)(hi - lo + 1) * kInfoStride * sizeof(int), hipMemcpyDeviceToHost, B->stream));
    }
  }
  bsync(B);
}

// ---- batched PCG ------------------------------------------------------------------
template <typename T>
struct StepLists {
  std::vector<ColsDesc<T>> c1, c3, c5;  // C^T p, M^T v, X_P^T t as column sweeps
  std::vector<RowsDesc<T>> r1, r2, r3, r4;  // C^T p and M^T v over stored transposes; Sigma M u, X_P r
  std::vector<PcgDesc<T>> pd, ph;       // all solves; the P_H ones
  std::vector<SymDesc<T>> sy;           // one-pass M^T Sigma M u
  std::vector<SymDesc<T>> sph;          // one-pass X_P^T X_P r (P_H solves)
  std::vector<int> c1p, c1r, c3p, c3r, c5p, c5r, r1p, r2p, r3p, r4p, qp, syp, syr, sphp, sphr;
  int c1pt = 0, c1rt = 0, c3pt = 0, c3rt = 0, c5pt = 0, c5rt = 0, r1t = 0, r2t = 0, r3t = 0, r4t = 0, qt = 0;
  int sypt = 0, syrt = 0, syK = 1, sphpt = 0, sphrt = 0, sphK = 1;
  size_t r1smem = 0, r2smem = 0, r3smem = 0, r4smem = 0, qsmem = 0;
  // device addresses after upload
  const ColsDesc<T>*dc1, *dc3, *dc5;
  const RowsDesc<T>*dr1, *dr2, *dr3, *dr4;
  const PcgDesc<T>*dpd, *dph;
  const SymDesc<T>*dsy, *dsph;
  const int *dsphp, *dsphr;
  const int *dc1p, *dc1r, *dc3p, *dc3r, *dc5p, *dc5r, *dr1p, *dr2p, *dr3p, *dr4p, *dqp, *dsyp, *dsyr;
};

template <typename T>
void build_lists(qp_batch* B, std::vector<BItem<T>*>& act, StepLists<T>& L) {
  qp_ctx* sk = &B->sink;
  L = StepLists<T>{};
  for (BItem<T>* it : act) {
    qp_ctx* c = it->ctx;
    const PcgBufs<T>& b = it->bufs;
    const int* skip = &c->sc->done;
    const int n = c->n, m2 = c->m2, N = c->N;
    const bool expl = kf_explicit(c);
    ColsDesc<T> cd;
    RowsDesc<T> rd;
    GemvWork<T> wk = *b.wk;
    if (expl) goto pcg_desc;  // q = E p + D p: only the fused row sweep
    {
      // u = C^T p: a row sweep over the stored C^T, a column sweep over C, or u = p when C = I
      const T* u = b.u;
      if (c->c_identity) {
        u = b.p;
      } else if (op_transposed(c)) {
        fill_rows_desc<T>(rd, b.CT, c->ldm2, n, m2, kDense, b.p, b.u, T(1), T(0), nullptr, n, skip);
        L.r1p.push_back(L.r1t);
        L.r1t += rd.nblocks;
        L.r1.push_back(rd);
        L.r1smem = std::max(L.r1smem, rows_smem_bytes<T>(n, m2, kDense, c->ldm2));
      } else {
        if (!fill_cols_desc<T>(cd, b.C, c->ldn, m2, n, kDense, b.p, b.u, T(1), T(0), nullptr, wk.part,
                               wk.part_elems, skip)) {
          set_err(sk, "column sweep over C does not fit its workspace (m2=%d n=%d)", m2, n);
          throw Fail{QP_E_DEVICE};
        }
        L.c1p.push_back(L.c1pt);
        L.c1r.push_back(L.c1rt);
        L.c1pt += cd.nblocks;
        L.c1rt += cd.rblocks;
        L.c1.push_back(cd);
      }
      if (op_fused(c)) {  // w = M^T Sigma M u in one pass
        SymDesc<T> sd;
        if (!fill_sym_desc<T>(sd, b.Linv, c->ldN, N, n, u, b.w, static_cast<T*>(c->sympart),
                              c->sympart_bytes / sizeof(T), skip)) {
          set_err(sk, "one-pass K0 product does not fit its workspace (N=%d n=%d)", N, n);
          throw Fail{QP_E_DEVICE};
        }
        L.syp.push_back(L.sypt);
        L.syr.push_back(L.syrt);
        L.sypt += sd.G;
        L.syrt += sd.rblocks;
        L.syK = std::max(L.syK, k0_sym_width<T>(n));
        L.sy.push_back(sd);
        goto pcg_desc;
      }
      // v = Sigma M u, then w = M^T v over the stored M^T or as a column sweep over M
      fill_rows_desc<T>(rd, b.Linv, c->ldN, N, n, kLower, u, b.v, T(1), T(0), nullptr, n, skip);
      L.r2p.push_back(L.r2t);
      L.r2t += rd.nblocks;
      L.r2.push_back(rd);
      L.r2smem = std::max(L.r2smem, rows_smem_bytes<T>(N, n, kLower, c->ldN));
      if (op_transposed(c)) {
        fill_rows_desc<T>(rd, b.MT, c->ldN, n, N, kUpper, b.v, b.w, T(1), T(0), nullptr, n, skip);
        L.r3p.push_back(L.r3t);
        L.r3t += rd.nblocks;
        L.r3.push_back(rd);
        L.r3smem = std::max(L.r3smem, rows_smem_bytes<T>(n, N, kUpper, c->ldN));
      } else {
        if (!fill_cols_desc<T>(cd, b.Linv, c->ldN, N, n, kLower, b.v, b.w, T(1), T(0), nullptr, wk.part,
                               wk.part_elems, skip)) {
          set_err(sk, "column sweep over the inverse factor does not fit its workspace (N=%d n=%d)", N, n);
          throw Fail{QP_E_DEVICE};
        }
        L.c3p.push_back(L.c3pt);
        L.c3r.push_back(L.c3rt);
        L.c3pt += cd.nblocks;
        L.c3rt += cd.rblocks;
        L.c3.push_back(cd);
      }
    }
  pcg_desc:
    PcgDesc<T> pd;
    pd.C = expl ? b.E : (c->c_identity ? nullptr : b.C);  // null: q = w + D p
    pd.w = expl ? b.p : b.w;
    pd.dvec = b.dvec;
    pd.wts = b.wts;
    pd.b = it->rhs;
    pd.x = b.x;
    pd.r = b.r;
    pd.z = b.z;
    pd.p = b.p;
    pd.q = b.q;
    pd.bpart = c->bpart;
    pd.sc = c->sc;
    pd.rtol = it->rtol;
    pd.wtol = it->wtol;
    pd.maxit = it->maxit;
    pd.ldc = expl ? c->ldm2 : c->ldn;
    pd.n = expl ? m2 : n;
    pd.m2 = m2;
    pd.prec = it->prec;
    pd.qblocks = std::min(bpcg_q_blocks(m2), c->bpart_cap);
    pd.stage = pd.C ? tune().brows_stage : 0;
    L.qp.push_back(L.qt);
    L.qt += pd.qblocks;
    L.pd.push_back(pd);
    if (pd.stage) L.qsmem = std::max(L.qsmem, rows_smem_bytes<T>(m2, pd.n, kDense, pd.ldc));
    if (it->prec == kPrecH && ph_fused(c)) {  // z = X_P^T X_P r in one pass over X_P
      SymDesc<T> sd;
      if (!fill_sym_desc<T>(sd, b.XP, c->ldm2, m2, m2, b.r, b.z, static_cast<T*>(c->phpart),
                            c->phpart_bytes / sizeof(T), skip)) {
        set_err(sk, "one-pass P_H apply does not fit its workspace (m2=%d)", m2);
        throw Fail{QP_E_DEVICE};
      }
      L.sphp.push_back(L.sphpt);
      L.sphr.push_back(L.sphrt);
      L.sphpt += sd.G;
      L.sphrt += sd.rblocks;
      L.sphK = std::max(L.sphK, k0_sym_width<T>(m2));
      L.sph.push_back(sd);
      L.ph.push_back(pd);
    } else if (it->prec == kPrecH) {
      fill_rows_desc<T>(rd, b.XP, c->ldm2, m2, m2, kLower, b.r, b.t, T(1), T(0), nullptr, m2, skip);
      L.r4p.push_back(L.r4t);
      L.r4t += rd.nblocks;
      L.r4.push_back(rd);
      L.r4smem = std::max(L.r4smem, rows_smem_bytes<T>(m2, m2, kLower, c->ldm2));
      if (!fill_cols_desc<T>(cd, b.XP, c->ldm2, m2, m2, kLower, b.t, b.z, T(1), T(0), nullptr, wk.part,
                             wk.part_elems, skip)) {
        set_err(sk, "column sweep over X_P does not fit its workspace (m2=%d)", m2);
        throw Fail{QP_E_DEVICE};
      }
      L.c5p.push_back(L.c5pt);
      L.c5r.push_back(L.c5rt);
      L.c5pt += cd.nblocks;
      L.c5rt += cd.rblocks;
      L.c5.push_back(cd);
      L.ph.push_back(pd);
    }
  }
  // every prefix table has one entry per descriptor of its list, then its block map
  if (L.c1p.size() != L.c1.size() || L.c1r.size() != L.c1.size() || L.c3p.size() != L.c3.size() ||
      L.c3r.size() != L.c3.size() || L.c5p.size() != L.c5.size() || L.c5r.size() != L.c5.size() ||
      L.r1p.size() != L.r1.size() || L.r2p.size() != L.r2.size() || L.r3p.size() != L.r3.size() ||
      L.r4p.size() != L.r4.size() || L.qp.size() != L.pd.size() || L.syp.size() != L.sy.size() ||
      L.syr.size() != L.sy.size() || L.sphp.size() != L.sph.size() || L.sphr.size() != L.sph.size()) {
    set_err(sk, "batched launch lists are inconsistent");
    throw Fail{QP_E_DEVICE};
  }
  Packer pk;
  auto V = [&](auto& v) { return pk.add(v.data(), v.size() * sizeof(v[0])); };
  auto M = [&](const std::vector<int>& prefix, int total) {
    std::vector<int> m = with_block_map(prefix, total);
    if (m.size() != prefix.size() + (size_t)total) {
      set_err(sk, "batched launch too large for its block map (%d descriptors, %d blocks)", (int)prefix.size(),
              total);
      throw Fail{QP_E_DEVICE};
    }
    return pk.add_owned(std::move(m));
  };
  size_t o_c1 = V(L.c1), o_c3 = V(L.c3), o_c5 = V(L.c5), o_r1 = V(L.r1), o_r2 = V(L.r2), o_r3 = V(L.r3),
         o_r4 = V(L.r4), o_pd = V(L.pd), o_ph = V(L.ph), o_sy = V(L.sy), o_sph = V(L.sph);
  size_t o_c1p = M(L.c1p, L.c1pt), o_c1r = M(L.c1r, L.c1rt), o_c3p = M(L.c3p, L.c3pt), o_c3r = M(L.c3r, L.c3rt),
         o_c5p = M(L.c5p, L.c5pt), o_c5r = M(L.c5r, L.c5rt), o_r1p = M(L.r1p, L.r1t), o_r2p = M(L.r2p, L.r2t),
         o_r3p = M(L.r3p, L.r3t), o_r4p = M(L.r4p, L.r4t), o_qp = M(L.qp, L.qt), o_syp = M(L.syp, L.sypt),
         o_syr = M(L.syr, L.syrt), o_sphp = M(L.sphp, L.sphpt), o_sphr = M(L.sphr, L.sphrt);
  const char* base = stage_upload(B, pk);
  L.dsy = reinterpret_cast<const SymDesc<T>*>(base + o_sy);
  L.dsyp = reinterpret_cast<const int*>(base + o_syp);
  L.dsyr = reinterpret_cast<const int*>(base + o_syr);
  L.dsph = reinterpret_cast<const SymDesc<T>*>(base + o_sph);
  L.dsphp = reinterpret_cast<const int*>(base + o_sphp);
  L.dsphr = reinterpret_cast<const int*>(base + o_sphr);
  L.dc1 = reinterpret_cast<const ColsDesc<T>*>(base + o_c1);
  L.dc3 = reinterpret_cast<const ColsDesc<T>*>(base + o_c3);
  L.dc5 = reinterpret_cast<const ColsDesc<T>*>(base + o_c5);
  L.dr1 = reinterpret_cast<const RowsDesc<T>*>(base + o_r1);
  L.dr2 = reinterpret_cast<const RowsDesc<T>*>(base + o_r2);
  L.dr3 = reinterpret_cast<const RowsDesc<T>*>(base + o_r3);
  L.dr1p = reinterpret_cast<const int*>(base + o_r1p);
  L.dr3p = reinterpret_cast<const int*>(base + o_r3p);
  L.dr4 = reinterpret_cast<const RowsDesc<T>*>(base + o_r4);
  L.dpd = reinterpret_cast<const PcgDesc<T>*>(base + o_pd);
  L.dph = reinterpret_cast<const PcgDesc<T>*>(base + o_ph);
  L.dc1p = reinterpret_cast<const int*>(base + o_c1p);
  L.dc1r = reinterpret_cast<const int*>(base + o_c1r);
  L.dc3p = reinterpret_cast<const int*>(base + o_c3p);
  L.dc3r = reinterpret_cast<const int*>(base + o_c3r);
  L.dc5p = reinterpret_cast<const int*>(base + o_c5p);
  L.dc5r = reinterpret_cast<const int*>(base + o_c5r);
  L.dr2p = reinterpret_cast<const int*>(base + o_r2p);
  L.dr4p = reinterpret_cast<const int*>(base + o_r4p);
  L.dqp = reinterpret_cast<const int*>(base + o_qp);
}

// P_H apply z = X_P^T (X_P r) and the p update for the P_H solves of the lists.
template <typename T>
void launch_ph_apply(qp_batch* B, const StepLists<T>& L, int init, const EventPair* ev = nullptr) {
  qp_ctx* sk = &B->sink;
  const int nph = (int)L.ph.size();
  if (!nph) return;
  // one-pass QPs (profile slots 4 and 5: the sweep and its reduce), then any with X_P too wide for it
  const int ns = (int)L.sph.size(), nr = (int)L.r4.size(), nc = (int)L.c5.size();
  HIPCHK(sk, launch_bk0_sym<T>(B->stream, L.dsph, L.dsphp, L.sphpt, L.dsphr, L.sphrt, ns, L.sphK,
                               ev ? &ev[4] : nullptr, ev ? &ev[5] : nullptr));
  HIPCHK(sk, launch_bgemv_rows<T>(B->stream, L.dr4, L.dr4p, nr, L.r4t, L.r4smem, 4, ev && !ns ? &ev[4] : nullptr));
  HIPCHK(sk, launch_bgemv_cols<T>(B->stream, L.dc5, L.dc5p, L.c5pt, L.dc5r, L.c5rt, nc, 5,
                                  ev && !ns ? &ev[5] : nullptr));
  HIPCHK(sk, bpcg_ph_update<T>(B->stream, L.dph, nph, init));
}

// ---- batched IPM phases ---------------------------------------------------------------
IpmDesc ipm_desc_of(qp_ctx* c) {
  IpmDesc q{};
  q.n = c->n;
  q.m1 = c->m1;
  q.m2 = c->m2;
  q.c = c->c;
  q.b = c->b;
  q.d = c->d;
  q.x = c->x;
  q.lam = c->lam;
  q.nu = c->nu;
  q.s = c->s;
  q.Hx = c->Hx;
  q.Atl = c->Atl;
  q.Ctn = c->Ctn;
  q.Ax = c->Ax;
  q.Cx = c->Cx;
  q.rg = c->rg;
  q.re = c->re;
  q.ri = c->ri;
  q.stats = c->stats;
  q.dvec = c->dvec;
  q.rc = c->rc;
  q.rhs = c->rhs;
  q.Cw = c->Cw;
  q.vN1 = c->vN1;
  q.vN2 = c->vN2;
  q.dx = c->dx;
  q.dlam = c->dlam;
  q.dnu = c->dnu;
  q.ds = c->ds;
  q.dx_a = c->dx_a;
  q.dlam_a = c->dlam_a;
  q.dnu_a = c->dnu_a;
  q.ds_a = c->ds_a;
  q.ir_r = c->ir_r;
  q.ir_x = c->ir_x;
  q.ir_d = c->ir_d;
  q.pt = c->pt;
  q.fd = c->fd;
  q.fwts = c->fwts;
  q.fb = c->fb;
  q.fx = c->fx;
  q.isc = c->isc;
  q.sc = c->sc;
  return q;
}

// A launch's prefix table with its block map (desc.hpp); a list too large for the
// map's encoding is refused.
static size_t pack_prefix(Packer& pk, const std::vector<int>& prefix, int total) {
  std::vector<int> m = with_block_map(prefix, total);
  if (m.size() != prefix.size() + (size_t)total) throw Fail{QP_E_DEVICE};
  return pk.add_owned(std::move(m));
}

// One batched row sweep, one batched column sweep (float64), and the list of
// pool entries of the batched vector kernels.
struct RowsL {
  std::vector<RowsDesc<double>> d;
  std::vector<int> p;
  int t = 0;
  size_t smem = 0, od = 0, op = 0;
  void add(const double* A, int lda, int m, int k, int shape, const double* x, double* y, double beta,
           const double* y0, int nsplit) {
    if (m <= 0) return;
    RowsDesc<double> r;
    fill_rows_desc<double>(r, A, lda, m, k, shape, x, y, 1.0, beta, y0, nsplit, nullptr);
    p.push_back(t);
    t += r.nblocks;
    d.push_back(r);
    smem = std::max(smem, rows_smem_bytes<double>(m, k, shape, lda));
  }
  void pack(Packer& pk) {
    od = pk.add(d.data(), d.size() * sizeof(d[0]));
    op = pack_prefix(pk, p, t);
  }
  void launch(qp_batch* B, const char* base, int tag) const {
    HIPCHK(&B->sink, launch_bgemv_rows<double>(B->stream, reinterpret_cast<const RowsDesc<double>*>(base + od),
                                               reinterpret_cast<const int*>(base + op), (int)d.size(), t, smem, tag));
  }
};

struct ColsL {
  std::vector<ColsDesc<double>> d;
  std::vector<int> p, r;
  int tp = 0, tr = 0;
  size_t od = 0, op = 0, orr = 0;
  void add(qp_batch* B, qp_ctx* c, const double* A, int lda, int m, int k, int shape, const double* x, double* y,
           double beta, const double* y0) {
    if (k <= 0) return;
    ColsDesc<double> cd;
    if (!fill_cols_desc<double>(cd, A, lda, m, k, shape, x, y, 1.0, beta, y0, c->w64.part, c->w64.part_elems,
                                nullptr)) {
      set_err(&B->sink, "column sweep (m=%d k=%d) does not fit its workspace", m, k);
      throw Fail{QP_E_DEVICE};
    }
    p.push_back(tp);
    r.push_back(tr);
    tp += cd.nblocks;
    tr += cd.rblocks;
    d.push_back(cd);
  }
  void pack(Packer& pk) {
    od = pk.add(d.data(), d.size() * sizeof(d[0]));
    op = pack_prefix(pk, p, tp);
    orr = pack_prefix(pk, r, tr);
  }
  void launch(qp_batch* B, const char* base, int tag) const {
    HIPCHK(&B->sink, launch_bgemv_cols<double>(B->stream, reinterpret_cast<const ColsDesc<double>*>(base + od),
                                               reinterpret_cast<const int*>(base + op), tp,
                                               reinterpret_cast<const int*>(base + orr), tr, (int)d.size(), tag));
  }
};

struct PoolL {
  std::vector<int> v;
  size_t off = 0;
  explicit PoolL(const std::vector<Slot*>& ss) {
    for (Slot* s : ss) v.push_back(s->pool);
  }
  void pack(Packer& pk) { off = pk.add(v.data(), v.size() * sizeof(int)); }
  const int* dev(const char* base) const { return reinterpret_cast<const int*>(base + off); }
  int count() const { return (int)v.size(); }
};

// vN2 = K0^{-1} vN1 for every QP: the row sweep (with Sigma) and the column sweep over L^{-1}.
void add_k0_solve(qp_batch* B, RowsL& rl, ColsL& cl, qp_ctx* c) {
  rl.add(c->Linv, c->ldN, c->N, c->N, kLower, c->vN1, c->vN3, 0.0, nullptr, c->n);
  cl.add(B, c, c->Linv, c->ldN, c->N, c->N, kLower, c->vN3, c->vN2, 0.0, nullptr);
}

// Initial point of freshly factored QPs: K0 [x0; -lam0] = [-c; b], s0, nu0, scalars.
void bphase_start(qp_batch* B, const std::vector<Slot*>& ss) {
  if (ss.empty()) return;
  PoolL pl(ss);
  RowsL k0r, cx;
  ColsL k0c;
  for (Slot* s : ss) {
    qp_ctx* c = s->ctx;
    add_k0_solve(B, k0r, k0c, c);
    cx.add(c->C, c->ldn, c->m2, c->n, kDense, c->vN2, c->Cx, 0.0, nullptr, c->m2);
  }
  Packer pk;
  pl.pack(pk);
  k0r.pack(pk);
  k0c.pack(pk);
  cx.pack(pk);
  const char* base = stage_upload(B, pk);
  qp_ctx* sk = &B->sink;
  HIPCHK(sk, bipm_pack(B->stream, B->d_ipm, pl.dev(base), pl.count(), kPackInit));
  k0r.launch(B, base, 0);
  k0c.launch(B, base, 0);
  cx.launch(B, base, 0);
  HIPCHK(sk, bipm_init(B->stream, B->d_ipm, pl.dev(base), pl.count(), B->opt.tau));
}

// Residual products and statistics of every iterate (launches only).
void bphase_eval(qp_batch* B, const std::vector<Slot*>& ss) {
  PoolL pl(ss);
  RowsL rows;
  ColsL ca, cc;
  for (Slot* s : ss) {
    qp_ctx* c = s->ctx;
    rows.add(c->H, c->ldn, c->n, c->n, kDense, c->x, c->Hx, 0.0, nullptr, c->n);
    rows.add(c->A, c->ldn, c->m1, c->n, kDense, c->x, c->Ax, 0.0, nullptr, c->m1);
    rows.add(c->C, c->ldn, c->m2, c->n, kDense, c->x, c->Cx, 0.0, nullptr, c->m2);
    ca.add(B, c, c->A, c->ldn, c->m1, c->n, kDense, c->lam, c->Atl, 0.0, nullptr);
    cc.add(B, c, c->C, c->ldn, c->m2, c->n, kDense, c->nu, c->Ctn, 0.0, nullptr);
  }
  Packer pk;
  pl.pack(pk);
  rows.pack(pk);
  ca.pack(pk);
  cc.pack(pk);
  const char* base = stage_upload(B, pk);
  rows.launch(B, base, 0);
  ca.launch(B, base, 0);  // both column sweeps use the QP's one workspace: in turn
  cc.launch(B, base, 0);
  HIPCHK(&B->sink, bipm_stats(B->stream, B->d_ipm, pl.dev(base), pl.count()));
}

// r_nu pieces, D and the predictor right-hand side.
void bphase_predictor(qp_batch* B, const std::vector<Slot*>& ss) {
  PoolL pl(ss);
  RowsL k0r, cw;
  ColsL k0c;
  for (Slot* s : ss) {
    qp_ctx* c = s->ctx;
    add_k0_solve(B, k0r, k0c, c);
    cw.add(c->C, c->ldn, c->m2, c->n, kDense, c->vN2, c->Cw, 0.0, nullptr, c->m2);
  }
  Packer pk;
  pl.pack(pk);
  k0r.pack(pk);
  k0c.pack(pk);
  cw.pack(pk);
  const char* base = stage_upload(B, pk);
  qp_ctx* sk = &B->sink;
  HIPCHK(sk, bipm_pack(B->stream, B->d_ipm, pl.dev(base), pl.count(), kPackRhs));
  k0r.launch(B, base, 0);
  k0c.launch(B, base, 0);
  cw.launch(B, base, 0);
  HIPCHK(sk, bipm_rhs(B->stream, B->d_ipm, pl.dev(base), pl.count(), 0));
}

// Recovery of the directions for dnu (which 0: predictor, 1: corrector), the
// step, and for the predictor the corrector right-hand side.
void bphase_recover_step(qp_batch* B, const std::vector<Slot*>& ss, int which) {
  PoolL pl(ss);
  RowsL k0r;
  ColsL ct, k0c;
  for (Slot* s : ss) {
    qp_ctx* c = s->ctx;
    ct.add(B, c, c->C, c->ldn, c->m2, c->n, kDense, which ? c->dnu : c->dnu_a, c->vN1, 1.0, c->rg);
    add_k0_solve(B, k0r, k0c, c);
  }
  Packer pk;
  pl.pack(pk);
  ct.pack(pk);
  k0r.pack(pk);
  k0c.pack(pk);
  const char* base = stage_upload(B, pk);
  qp_ctx* sk = &B->sink;
  ct.launch(B, base, 0);
  HIPCHK(sk, bipm_pack(B->stream, B->d_ipm, pl.dev(base), pl.count(), kPackRecover));
  k0r.launch(B, base, 0);
  k0c.launch(B, base, 0);
  HIPCHK(sk, bipm_dirs(B->stream, B->d_ipm, pl.dev(base), pl.count(), which));
  HIPCHK(sk, bipm_step(B->stream, B->d_ipm, pl.dev(base), pl.count(), which));
  if (!which) HIPCHK(sk, bipm_rhs(B->stream, B->d_ipm, pl.dev(base), pl.count(), 1));
}

// ---- refinement steps ----------------------------------------------------------------
// Float64 residual r = rhs - K_F dnu of the listed QPs (dnu already updated by
// bir_acc, which also left pt = D dnu): C^T dnu, the M sweeps, C w + pt, then
// the residual statistics into each QP's PcgScalars.
void bphase_ir_residual(qp_batch* B, const std::vector<Slot*>& ss, int which) {
  PoolL pl(ss);
  ColsL ct, mt;
  RowsL mr, cr;
  for (Slot* s : ss) {
    qp_ctx* c = s->ctx;
    double* dnu = which ? c->dnu : c->dnu_a;
    if (kf_explicit(c)) {  // K_F dnu = E dnu + pt
      cr.add(c->E, c->ldm2, c->m2, c->m2, kDense, dnu, c->ir_x, 1.0, c->pt, c->m2);
      continue;
    }
    ct.add(B, c, c->C, c->ldn, c->m2, c->n, kDense, dnu, c->pu, 0.0, nullptr);
    mr.add(c->Linv, c->ldN, c->N, c->n, kLower, c->pu, c->pv, 0.0, nullptr, c->n);
    mt.add(B, c, c->Linv, c->ldN, c->N, c->n, kLower, c->pv, c->pw, 0.0, nullptr);
    cr.add(c->C, c->ldn, c->m2, c->n, kDense, c->pw, c->ir_x, 1.0, c->pt, c->m2);
  }
  Packer pk;
  pl.pack(pk);
  ct.pack(pk);
  mr.pack(pk);
  mt.pack(pk);
  cr.pack(pk);
  const char* base = stage_upload(B, pk);
  ct.launch(B, base, 0);
  mr.launch(B, base, 2);
  mt.launch(B, base, 3);
  cr.launch(B, base, 0);
  HIPCHK(&B->sink, bir_residual(B->stream, B->d_ipm, pl.dev(base), pl.count(), which));
}

// Vector kernel over the listed QPs with a freshly uploaded pool list.
template <typename F>
void bvec(qp_batch* B, const std::vector<Slot*>& ss, F&& launch) {
  if (ss.empty()) return;
  PoolL pl(ss);
  Packer pk;
  pl.pack(pk);
  const char* base = stage_upload(B, pk);
  HIPCHK(&B->sink, launch(pl.dev(base), pl.count()));
}

// ---- slots ------------------------------------------------------------------------------
void release_slot_memory(qp_batch* B, Slot* s) {
  if (s->ctx) {
    free_all(s->ctx);  // stream-ordered reuse: later work on the stream runs after this QP's
    delete s->ctx;
    s->ctx = nullptr;
  }
  if (s->pool >= 0) {
    B->free_pools.push_back(s->pool);
    s->pool = -1;
  }
}

// Copy the final iterate to host memory and free the QP's device memory.
void finish_slot(qp_batch* B, Slot* s, qp_status st) {
  qp_ctx* c = s->ctx;
  s->status = st;
  if (st != QP_OK && s->err.empty()) s->err = c && !c->err.empty() ? c->err : qp_status_str(st);
  if (c && s->state == kRunning) {
    s->x.resize(c->n);
    s->lam.resize(c->m1);
    s->nu.resize(c->m2);
    s->s.resize(c->m2);
    HIPCHK(c, hipMemcpyAsync(s->x.data(), c->x, (size_t)c->n * sizeof(double), hipMemcpyDeviceToHost, B->stream));
    HIPCHK(c, hipMemcpyAsync(s->lam.data(), c->lam, (size_t)c->m1 * sizeof(double), hipMemcpyDeviceToHost,
                             B->stream));
    HIPCHK(c, hipMemcpyAsync(s->nu.data(), c->nu, (size_t)c->m2 * sizeof(double), hipMemcpyDeviceToHost, B->stream));
    HIPCHK(c, hipMemcpyAsync(s->s.data(), c->s, (size_t)c->m2 * sizeof(double), hipMemcpyDeviceToHost, B->stream));
    bsync(B);
    ipm_fill_info(c, s->R, &s->info);
  }
  s->info.status = st;
  s->t_done = Clock::now();
  s->info.t_solve_ms = std::chrono::duration<double, std::milli>(s->t_done - s->t_admit).count();
  s->state = kFinished;
  s->phase = kPhDone;
  release_slot_memory(B, s);
  B->finished[s->ticket] = s;
}

// Run one per-QP phase; a failure of this QP alone (not of the device) retires it.
template <typename F>
bool per_qp(qp_batch* B, Slot* s, F&& f) {
  try {
    f();
    return true;
  } catch (const Fail& e) {
    if (e.st == QP_E_DEVICE) throw;
    s->err = s->ctx ? s->ctx->err : "";
    finish_slot(B, s, e.st);
    return false;
  }
}

// K0 = L Sigma L^T of every newly admitted QP at once (the steps of factor()
// and ph_setup(), each one batched launch per recursion node), then the
// initial point.  QPs whose H or A H^{-1} A^T has a bad pivot finish here.
void batched_factor(qp_batch* B, std::vector<Slot*> fresh) {
  auto drop_failed = [&](int code, const char* what) {
    std::vector<Slot*> ok;
    for (Slot* s : fresh) {
      if (B->h_info[(size_t)s->pool * kInfoStride] != 0) {
        set_err(s->ctx, "%s", what);
        s->err = s->ctx->err;
        finish_slot(B, s, (qp_status)code);
      } else {
        ok.push_back(s);
      }
    }
    fresh.swap(ok);
  };
  auto pool_range = [&](int& lo, int& hi) {
    lo = kMaxSlots;
    hi = -1;
    for (Slot* s : fresh) {
      lo = std::min(lo, s->pool);
      hi = std::max(hi, s->pool);
    }
  };
  BatchedOps o1;
  std::vector<CholJob> cj;
  std::vector<GemmDesc> gw, gs;
  // C = I test (info[1] is set when C differs from the identity)
  std::vector<MatOpDesc> idc;
  int id_rows = 0, id_cols = 0;
  for (Slot* s : fresh) {
    qp_ctx* c = s->ctx;
    HIPCHK(c, hipMemsetAsync(c->info, 0, 2 * sizeof(int), B->stream));
    if (c->m2 != c->n) continue;
    idc.push_back(MatOpDesc{c->C, nullptr, nullptr, c->info + 1, c->ldn, 0, 0, c->m2, c->n, kMatIdentity});
    id_rows = std::max(id_rows, c->m2);
    id_cols = std::max(id_cols, c->n);
  }
  if (!idc.empty()) {
    Packer pk;
    pk.add(idc.data(), idc.size() * sizeof(MatOpDesc));
    const char* base = stage_upload(B, pk);
    HIPCHK(&B->sink, bmatop(B->stream, reinterpret_cast<const MatOpDesc*>(base), (int)idc.size(), id_rows, id_cols));
  }
  for (Slot* s : fresh) {
    qp_ctx* c = s->ctx;
    HIPCHK(c, hipMemcpyAsync(c->fHw, c->H, (size_t)c->n * c->ldn * sizeof(double), hipMemcpyDeviceToDevice,
                             B->stream));
    double* XH = c->Linv;
    cj.push_back(CholJob{c->fHw, c->ldn, XH, c->ldN, c->n, c->ftmp, c->info, QP_E_NOT_SPD});
    gw.push_back(GemmDesc{c->A, XH, c->fWt, c->ldn, c->ldN, c->ldn, c->m1, c->n, c->n});       // W^T = A X_H^T
    gs.push_back(GemmDesc{c->fWt, c->fWt, c->fS, c->ldn, c->ldn, c->ldm1, c->m1, c->m1, c->n});  // S = W^T W
  }
  o1.chol_inv(cj);
  o1.gemm(0, 1, 1.0, 0.0, kBUpper, gw);
  o1.gemm(0, 1, 1.0, 0.0, kOutLower, gs);
  run_ops(B, o1);
  int lo, hi;
  pool_range(lo, hi);
  sync_pools(B, lo, hi, true);
  drop_failed(QP_E_NOT_SPD, "Cholesky factorization of H failed: H is not positive definite");
  if (fresh.empty()) return;
  for (Slot* s : fresh) s->ctx->c_identity = s->ctx->m2 == s->ctx->n && s->ctx->h_info[1] == 0;
  BatchedOps o2;
  std::vector<CholJob> cs;
  std::vector<GemmDesc> g1, g2, gy, gt;
  std::vector<MatOpDesc> ph_scale;  // diagonal form of P_H
  int ps_rows = 0, ps_cols = 0;
  for (Slot* s : fresh) {
    qp_ctx* c = s->ctx;
    const int n = c->n;
    double* XH = c->Linv;
    double* G = c->Linv + (size_t)n * c->ldN;
    double* XS = G + n;
    cs.push_back(CholJob{c->fS, c->ldm1, XS, c->ldN, c->m1, c->ftmp, c->info, QP_E_RANK});
    g1.push_back(GemmDesc{c->fWt, XH, c->fG, c->ldn, c->ldN, c->ldn, c->m1, n, n});      // W^T X_H
    g2.push_back(GemmDesc{XS, c->fG, G, c->ldN, c->ldn, c->ldN, c->m1, n, c->m1});       // G = -X_S W^T X_H
    if (s->R.prec == kPrecH || prec_mode(resolve_prec(c, c->opt.prec)) == kPrecH) {
      if (c->opt.ph_form == QP_PH_DIAG) {  // C diag(H)^{-1/2}
        ph_scale.push_back(MatOpDesc{c->C, c->H, c->fYt, nullptr, c->ldn, c->ldn, c->ldn, c->m2, n, kMatColScale});
        ps_rows = std::max(ps_rows, c->m2);
        ps_cols = std::max(ps_cols, n);
      } else {
        gy.push_back(GemmDesc{c->C, XH, c->fYt, c->ldn, c->ldN, c->ldn, c->m2, n, n});  // C X_H^T
      }
      gt.push_back(GemmDesc{c->fYt, c->fYt, c->T, c->ldn, c->ldn, c->ldm2, c->m2, c->m2, n});  // T = Y Y^T
    }
  }
  // explicit operator E = Y_1^T Y_1 - Y_2^T Y_2, Y = L^{-1}[:, :n] C^T (after G is final)
  std::vector<GemmDesc> ey, ee1, ee2;
  for (Slot* s : fresh) {
    qp_ctx* c = s->ctx;
    if (!kf_explicit(c)) continue;
    const int ld = c->ldm2;
    ey.push_back(GemmDesc{c->Linv, c->C, c->fY, c->ldN, c->ldn, ld, c->N, c->m2, c->n});
    ee1.push_back(GemmDesc{c->fY, c->fY, c->E, ld, ld, ld, c->m2, c->m2, c->n});
    const double* Y2 = c->fY + (size_t)c->n * ld;
    ee2.push_back(GemmDesc{Y2, Y2, c->E, ld, ld, ld, c->m2, c->m2, c->m1});
  }
  o2.chol_inv(cs);
  o2.gemm(0, 0, 1.0, 0.0, kBLower, g1);
  o2.gemm(0, 0, -1.0, 0.0, kALower, g2);
  o2.gemm(0, 1, 1.0, 0.0, kBUpper, gy);
  o2.gemm(0, 1, 1.0, 0.0, kOutLower, gt);
  o2.gemm(0, 1, 1.0, 0.0, kALower, ey);
  o2.gemm(1, 0, 1.0, 0.0, kNone, ee1);
  o2.gemm(1, 0, -1.0, 1.0, kNone, ee2);
  if (!ph_scale.empty()) {  // before T = Y Y^T, which o2 runs
    Packer pk;
    pk.add(ph_scale.data(), ph_scale.size() * sizeof(MatOpDesc));
    const char* base = stage_upload(B, pk);
    HIPCHK(&B->sink, bmatop(B->stream, reinterpret_cast<const MatOpDesc*>(base), (int)ph_scale.size(), ps_rows,
                            ps_cols));
  }
  run_ops(B, o2);
  pool_range(lo, hi);
  sync_pools(B, lo, hi, true);
  drop_failed(QP_E_RANK, "Cholesky factorization of A H^{-1} A^T failed: A is rank deficient");
  std::vector<Mat2dDesc> cv;
  int max_rows = 0, max_cols = 0;
  for (Slot* s : fresh) {
    qp_ctx* c = s->ctx;
    if (c->opt.precision == QP_MIXED) {
      cv.push_back(Mat2dDesc{c->Linv, c->Linv32, nullptr, c->ldN, c->ldN, c->N, c->N, 1, 1});
      max_rows = std::max(max_rows, c->N);
      max_cols = std::max(max_cols, c->N);
      if (kf_explicit(c)) cv.push_back(Mat2dDesc{c->E, c->E32, nullptr, c->ldm2, c->ldm2, c->m2, c->m2, 0, 1});
    }
    c->factored = true;
    c->ph_ready = prec_mode(resolve_prec(c, c->opt.prec)) == kPrecH;
    IpmRun& R = s->R;
    R = IpmRun{};
    R.prec = prec_mode(resolve_prec(c, c->opt.prec));
    R.maxit = c->opt.max_pcg > 0 ? c->opt.max_pcg : 20 * c->m2;
    s->state = kRunning;
  }
  if (!cv.empty()) {
    Packer pk;
    pk.add(cv.data(), cv.size() * sizeof(Mat2dDesc));
    const char* base = stage_upload(B, pk);
    HIPCHK(&B->sink, bmat2d(B->stream, reinterpret_cast<const Mat2dDesc*>(base), (int)cv.size(), max_rows, max_cols));
  }
  // transposed copies for the implicit CG step: C^T and M^T (and their float32 copies)
  std::vector<TransDesc> tr;
  int tr_rows = 0, tr_cols = 0;
  for (Slot* s : fresh) {
    qp_ctx* c = s->ctx;
    if (!op_transposed(c)) continue;
    const bool ct = !c->c_identity;  // C = I needs no C^T
    if (ct) tr.push_back(TransDesc{c->C, c->CT, c->ldn, c->ldm2, c->m2, c->n, 0});
    if (store_mt(c)) tr.push_back(TransDesc{c->Linv, c->MT, c->ldN, c->ldN, c->N, c->n, 0});
    if (c->opt.precision == QP_MIXED) {
      if (ct) tr.push_back(TransDesc{c->C, c->CT32, c->ldn, c->ldm2, c->m2, c->n, 1});
      if (store_mt(c)) tr.push_back(TransDesc{c->Linv, c->MT32, c->ldN, c->ldN, c->N, c->n, 1});
    }
    tr_rows = std::max(tr_rows, c->N);
    tr_cols = std::max(tr_cols, c->n);
  }
  if (!tr.empty()) {
    Packer pk;
    pk.add(tr.data(), tr.size() * sizeof(TransDesc));
    const char* base = stage_upload(B, pk);
    HIPCHK(&B->sink, btranspose_2d(B->stream, reinterpret_cast<const TransDesc*>(base), (int)tr.size(), tr_rows,
                                   tr_cols));
  }
  bphase_start(B, fresh);
  // the scratch regions were read by the factorization launches: release them once those ran
  bsync(B);
  for (Slot* s : fresh)
    if (s->ctx) free_factor_scratch(s->ctx);
}

// X_P = chol(D + C H^{-1} C^T)^{-1} for the new D of every P_H QP, batched.
void batched_ph_factor(qp_batch* B, const std::vector<Slot*>& go) {
  std::vector<Mat2dDesc> add, cv;
  std::vector<CholJob> cj;
  int mr = 0;
  for (Slot* s : go) {
    if (s->R.prec != kPrecH) continue;
    qp_ctx* c = s->ctx;
    add.push_back(Mat2dDesc{c->T, c->P, c->dvec, c->ldm2, c->ldm2, c->m2, c->m2, 1, 0});
    cj.push_back(CholJob{c->P, c->ldm2, c->XP, c->ldm2, c->m2, c->ptmp, c->info, QP_E_INVALID});
    if (c->opt.precision == QP_MIXED) cv.push_back(Mat2dDesc{c->XP, c->XP32, nullptr, c->ldm2, c->ldm2, c->m2, c->m2, 1, 1});
    mr = std::max(mr, c->m2);
  }
  if (cj.empty()) return;
  Packer pk;
  const size_t oa = pk.add(add.data(), add.size() * sizeof(Mat2dDesc));
  const size_t oc = pk.add(cv.data(), cv.size() * sizeof(Mat2dDesc));
  const char* base = stage_upload(B, pk);
  HIPCHK(&B->sink, bmat2d(B->stream, reinterpret_cast<const Mat2dDesc*>(base + oa), (int)add.size(), mr, mr));
  BatchedOps o;
  o.chol_inv(cj);
  run_ops(B, o);
  if (!cv.empty())
    HIPCHK(&B->sink, bmat2d(B->stream, reinterpret_cast<const Mat2dDesc*>(base + oc), (int)cv.size(), mr, mr));
}

// ---- the scheduler -----------------------------------------------------------------------
// Start CG runs (their BItem<T> already filled): initial residual and direction,
// and for P_H the first preconditioner apply; the QPs join the CG pool.
template <typename T>
void start_cg(qp_batch* B, const std::vector<Slot*>& ss, std::vector<Slot*>& pool) {
  if (ss.empty()) return;
  std::vector<BItem<T>*> items;
  for (Slot* s : ss) {
    BItem<T>* it;
    if constexpr (sizeof(T) == 8)
      it = &s->it64;
    else
      it = &s->it32;
    it->iters = it->done = 0;
    items.push_back(it);
    s->launched = 0;
    s->phase = kPhSolve;
    pool.push_back(s);
  }
  StepLists<T> L;
  build_lists<T>(B, items, L);
  HIPCHK(&B->sink, bpcg_init<T>(B->stream, L.dpd, (int)items.size()));
  launch_ph_apply<T>(B, L, 1);
}

void fill_cg64(Slot* s, double* x, const double* rhs, double rtol, int maxit) {
  qp_ctx* c = s->ctx;
  s->it64 = BItem<double>{};
  s->it64.ctx = c;
  s->it64.bufs = bufs64(c, c->dvec, c->nu, x);
  s->it64.rhs = rhs;
  s->it64.prec = s->R.prec;
  s->it64.rtol = rtol;
  s->it64.wtol = s->R.wtol;
  s->it64.maxit = maxit;
}

// Next float32 sweep of the mixed refinement: fb = r, CG on K_F delta = r.
void next_sweep(qp_batch* B, const std::vector<Slot*>& ss) {
  if (ss.empty()) return;
  bvec(B, ss, [&](const int* l, int n) { return bir_prep(B->stream, B->d_ipm, l, n); });
  for (Slot* s : ss) {
    qp_ctx* c = s->ctx;
    s->it32 = BItem<float>{};
    s->it32.ctx = c;
    s->it32.bufs = bufs32(c);
    s->it32.rhs = c->fb;
    s->it32.prec = s->R.prec;
    s->it32.rtol = 1e-5;
    s->it32.wtol = -1.0;
    s->it32.maxit = std::min(mixed_inner_cap(c, s->R.prec), s->R.maxit - s->s_iters);
  }
  start_cg<float>(B, ss, B->cg32);
}

// Begin the reduced solve `which` (0 predictor, 1 corrector) of the listed QPs.
void start_solve(qp_batch* B, const std::vector<Slot*>& ss, int which) {
  if (ss.empty()) return;
  for (Slot* s : ss) {
    s->which = which;
    s->s_iters = s->s_refin = s->s_fb = s->s_iters64 = 0;
    s->s_done = 2;
    s->last_done = 0;
    s->prev_rr = -1.0;
  }
  if (B->opt.precision != QP_MIXED) {
    for (Slot* s : ss) fill_cg64(s, which ? s->ctx->dnu : s->ctx->dnu_a, s->ctx->rhs, s->ctx->opt.cg_rtol, s->R.maxit);
    start_cg<double>(B, ss, B->cg64);
    return;
  }
  bvec(B, ss, [&](const int* l, int n) { return bir_begin(B->stream, B->d_ipm, l, n, which); });
  next_sweep(B, ss);
}

// A reduced solve has ended: record it and move the QP on (recovery and step;
// after the corrector also the next iteration's residual statistics).
void solves_done(qp_batch* B, std::vector<Slot*>& d0, std::vector<Slot*>& d1) {
  for (auto* v : {&d0, &d1})
    for (Slot* s : *v) {
      IpmRun& R = s->R;
      (s->which ? R.k2 : R.k1) = s->s_iters;
      R.refin_total += s->s_refin;
      R.fallbacks += s->s_fb;
      R.cg64 += s->s_iters64;
    }
  if (!d0.empty()) {
    bphase_recover_step(B, d0, 0);
    start_solve(B, d0, 1);
  }
  if (!d1.empty()) {
    bphase_recover_step(B, d1, 1);
    for (Slot* s : d1) {
      s->R.cg_total += s->R.k1 + s->R.k2;
      ++s->R.it;
      s->phase = kPhAwaitStats;
    }
    bphase_eval(B, d1);
  }
}

void sync_live_pools(qp_batch* B) {
  int lo = kMaxSlots, hi = -1;
  for (Slot* s : B->live) {
    if (s->pool < 0) continue;  // retired in this tick
    lo = std::min(lo, s->pool);
    hi = std::max(hi, s->pool);
  }
  sync_pools(B, lo, hi, true);
}

// CG steps for every QP of a pool: poll_every steps, one launch per sweep.
template <typename T>
void launch_chunk(qp_batch* B, const std::vector<Slot*>& pool, int poll, bool sample) {
  if (pool.empty()) return;
  std::vector<BItem<T>*> items;
  for (Slot* s : pool) {
    BItem<T>* it;
    if constexpr (sizeof(T) == 8)
      it = &s->it64;
    else
      it = &s->it32;
    if (s->launched > (long long)it->maxit + 2LL * poll) {
      set_err(&B->sink, "batched PCG made no progress after %lld launched steps", s->launched);
      throw Fail{QP_E_DEVICE};
    }
    s->launched += poll;
    items.push_back(it);
  }
  // largest QPs first: their workgroups start first and the small ones fill in behind
  std::stable_sort(items.begin(), items.end(),
                   [](const BItem<T>* a, const BItem<T>* b) { return a->ctx->n > b->ctx->n; });
  StepLists<T> L;
  build_lists<T>(B, items, L);
  qp_ctx* sk = &B->sink;
  const int na = (int)items.size();
  for (int k = 0; k < poll; ++k) {
    const EventPair* ev = (sample && k == 0) ? B->prof_ev : nullptr;
    // lists are empty where they do not apply (explicit operators; transposes or not)
    const int n1 = (int)L.c1.size(), n2 = (int)L.r2.size(), n3 = (int)L.c3.size();
    const int t1 = (int)L.r1.size(), t3 = (int)L.r3.size(), ns = (int)L.sy.size();
    // profile slots 1 and 2: the one-pass sweep and its reduce when the list has
    // one-pass QPs, else the two triangular sweeps
    const EventPair* e1 = ev && !ns ? &ev[1] : nullptr;
    const EventPair* e2 = ev && !ns ? &ev[2] : nullptr;
    HIPCHK(sk, launch_bgemv_cols<T>(B->stream, L.dc1, L.dc1p, L.c1pt, L.dc1r, L.c1rt, n1, 1, ev && n1 ? &ev[0] : nullptr));
    HIPCHK(sk, launch_bgemv_rows<T>(B->stream, L.dr1, L.dr1p, t1, L.r1t, L.r1smem, 1, ev && t1 ? &ev[0] : nullptr));
    HIPCHK(sk, launch_bk0_sym<T>(B->stream, L.dsy, L.dsyp, L.sypt, L.dsyr, L.syrt, ns, L.syK, ev ? &ev[1] : nullptr,
                                 ev ? &ev[2] : nullptr));
    HIPCHK(sk, launch_bgemv_rows<T>(B->stream, L.dr2, L.dr2p, n2, L.r2t, L.r2smem, 2, e1));
    HIPCHK(sk, launch_bgemv_cols<T>(B->stream, L.dc3, L.dc3p, L.c3pt, L.dc3r, L.c3rt, n3, 3, e2 && n3 ? e2 : nullptr));
    HIPCHK(sk, launch_bgemv_rows<T>(B->stream, L.dr3, L.dr3p, t3, L.r3t, L.r3smem, 3, e2 && t3 ? e2 : nullptr));
    HIPCHK(sk, bpcg_q<T>(B->stream, L.dpd, L.dqp, na, L.qt, L.qsmem, ev ? &ev[3] : nullptr));
    HIPCHK(sk, bpcg_update<T>(B->stream, L.dpd, na));
    launch_ph_apply<T>(B, L, 0, ev);
  }
  if (sample) {
    // every QP of the chunk was iterating when it started, so the sampled step covered all of them
    for (int o = 0; o < kProfOps; ++o) B->prof_pending_bytes[o] = 0;
    for (Slot* s : pool) {
      const qp_ctx* c = s->ctx;
      const double mn = (double)c->n * (c->n + 1) / 2 + (double)c->m1 * c->n;
      const double cn = (double)c->m2 * c->n, xp = (double)c->m2 * (c->m2 + 1) / 2;
      if (kf_explicit(c)) {
        B->prof_pending_bytes[3] += (double)c->m2 * c->m2 * sizeof(T);
      } else {
        B->prof_pending_bytes[0] += cn * sizeof(T);
        B->prof_pending_bytes[1] += mn * sizeof(T);
        if (!op_fused(c)) B->prof_pending_bytes[2] += mn * sizeof(T);  // the one pass reads M once
        B->prof_pending_bytes[3] += cn * sizeof(T);
      }
      if (s->R.prec == kPrecH) {
        B->prof_pending_bytes[4] += xp * sizeof(T);
        if (!ph_fused(c)) B->prof_pending_bytes[5] += xp * sizeof(T);  // the one pass reads X_P once
      }
    }
  }
}

bool advance(qp_batch* B);

// One scheduling tick: admit and factor new QPs, run one poll chunk of CG
// steps for every QP inside a reduced solve, wait once, then move every QP as
// far as it can go (KKT checks, refinement decisions, recovery and step, the
// next solve) before the next chunk.
void tick(qp_batch* B) {
  qp_ctx* sk = &B->sink;
  // (1) QPs admitted since the last tick: factor, initial point, statistics
  std::vector<Slot*> fresh;
  for (Slot* s : B->live)
    if (s->state == kQueued) fresh.push_back(s);
  auto prune = [&] {
    std::vector<Slot*> keep;
    for (Slot* s : B->live)
      if (s->state != kFinished) keep.push_back(s);
    B->live.swap(keep);
  };
  if (!fresh.empty()) {
    batched_factor(B, fresh);
    prune();  // QPs whose factorization failed have left (and given back their pool entry)
    std::vector<Slot*> ok;
    for (Slot* s : fresh)
      if (s->state == kRunning) {
        s->phase = kPhAwaitStats;
        ok.push_back(s);
      }
    if (!ok.empty()) bphase_eval(B, ok);
  }
  // (2) one chunk of CG steps
  const int poll = B->opt.poll_every > 0 ? B->opt.poll_every : 32;
  const bool prof = B->opt.profile != 0;
  if (prof && !B->prof_ready) {
    for (int o = 0; o < kProfOps; ++o) {
      HIPCHK(sk, hipEventCreate(&B->prof_ev[o].begin));
      HIPCHK(sk, hipEventCreate(&B->prof_ev[o].end));
    }
    B->prof_ready = true;
  }
  const bool s32 = prof && !B->cg32.empty();
  const bool s64 = prof && !s32 && !B->cg64.empty();
  launch_chunk<double>(B, B->cg64, poll, s64);
  launch_chunk<float>(B, B->cg32, poll, s32);
  if (!B->cg64.empty() || !B->cg32.empty()) B->cg_launched += poll;
  // (3) wait; every QP's CG scalars, statistics and factorization status on the host
  sync_live_pools(B);
  if (s32 || s64) {
    for (int o = 0; o < kProfOps; ++o) {
      if (B->prof_pending_bytes[o] == 0) continue;
      float ms = 0;
      if (hipEventElapsedTime(&ms, B->prof_ev[o].begin, B->prof_ev[o].end) == hipSuccess) {
        B->prof_ms[o] += ms;
        B->prof_bytes[o] += B->prof_pending_bytes[o];
        B->prof_n[o] += 1;
      }
    }
  }
  B->rounds += 1;
  // (4) decisions and the launches they lead to; a QP may need a few host
  // decisions in a row (refinement residual, KKT check) before its next CG run,
  // so repeat with a short wait for the small kernels in between
  for (int pass = 0; pass < 4; ++pass) {
    if (pass > 0) sync_live_pools(B);
    if (!advance(B)) break;
  }
  prune();
}

// Read the host copies of every QP's scalars and move each QP on; returns true
// when some QP now waits for a result launched here (one more pass helps it).
bool advance(qp_batch* B) {
  {
    std::vector<Slot*> keep;  // QPs retired by an earlier pass have left
    for (Slot* s : B->live)
      if (s->state != kFinished) keep.push_back(s);
    B->live.swap(keep);
  }
  std::vector<Slot*> pred, d0, d1, ir0, ir1, fb, sw;
  const bool mixed = B->opt.precision == QP_MIXED;
  auto done_solve = [&](Slot* s) { (s->which ? d1 : d0).push_back(s); };
  // CG runs that stopped
  std::vector<Slot*> keep64, keep32;
  for (Slot* s : B->cg64) {
    const PcgScalars& h = B->h_sc[s->pool];
    if (!h.done) {
      keep64.push_back(s);
      continue;
    }
    s->s_iters += h.iter;
    if (!mixed) {
      s->s_done = h.done;
      done_solve(s);
    } else {
      // float64 leg of a mixed solve: add the correction
      s->s_iters64 += h.iter;
      s->s_done = h.done;
      s->s_fb = 1;
      fb.push_back(s);
    }
  }
  for (Slot* s : B->cg32) {
    const PcgScalars& h = B->h_sc[s->pool];
    if (!h.done) {
      keep32.push_back(s);
      continue;
    }
    s->s_iters += h.iter;
    s->last_done = h.done;
    (s->which ? ir1 : ir0).push_back(s);
  }
  B->cg64.swap(keep64);
  B->cg32.swap(keep32);
  // refinement residuals that reached the host: converged, stalled, or sweep again
  std::vector<Slot*> to64;
  for (Slot* s : B->live) {
    if (s->phase == kPhAwaitIR) {
      const PcgScalars h = B->h_sc[s->pool];
      s->s_refin += 1;
      const double rt = s->ctx->opt.cg_rtol;
      if (h.bb == 0.0 || h.rr <= rt * rt * h.bb || (s->R.wtol >= 0.0 && h.wmax <= s->R.wtol)) {
        s->s_done = 1;
        done_solve(s);
        continue;
      }
      const double ref_rr = s->prev_rr >= 0.0 ? s->prev_rr : h.bb;
      const bool stalled = s->last_done != 1 || h.rr > 1e-2 * ref_rr || !std::isfinite(h.rr);
      if (stalled && s->s_iters < s->R.maxit) {
        s->rtol64 = h.rr > 0.0 ? rt * std::sqrt(h.bb / h.rr) : rt;
        to64.push_back(s);
        continue;
      }
      s->prev_rr = h.rr;
      if (s->s_refin < 30 && s->s_iters < s->R.maxit)
        sw.push_back(s);
      else {
        s->s_done = 2;
        done_solve(s);
      }
    } else if (s->phase == kPhAwaitStats) {
      if (!ipm_check(s->ctx, s->R)) {
        qp_status st = (qp_status)s->R.status;
        if (st != QP_OK && s->ctx->err.empty())
          set_err(s->ctx, "IPM stopped at rel_kkt %.3e after %d iterations", s->R.score, s->R.it);
        finish_slot(B, s, st);
        continue;
      }
      pred.push_back(s);
    }
  }
  // (5) launches, grouped by kind over all QPs
  if (!fb.empty()) {  // float64 corrections of stalled mixed solves are done: dnu += correction
    std::vector<Slot*> f0, f1;
    for (Slot* s : fb) (s->which ? f1 : f0).push_back(s);
    bvec(B, f0, [&](const int* l, int n) { return bir_fb_add(B->stream, B->d_ipm, l, n, 0); });
    bvec(B, f1, [&](const int* l, int n) { return bir_fb_add(B->stream, B->d_ipm, l, n, 1); });
    for (Slot* s : fb) done_solve(s);
  }
  for (int w = 0; w < 2; ++w) {  // float32 sweeps that stopped: accumulate, float64 residual
    std::vector<Slot*>& ir = w ? ir1 : ir0;
    if (ir.empty()) continue;
    bvec(B, ir, [&](const int* l, int n) { return bir_acc(B->stream, B->d_ipm, l, n, w); });
    bphase_ir_residual(B, ir, w);
    for (Slot* s : ir) s->phase = kPhAwaitIR;
  }
  if (!to64.empty()) {
    for (Slot* s : to64) fill_cg64(s, s->ctx->ir_d, s->ctx->ir_r, s->rtol64, s->R.maxit - s->s_iters);
    start_cg<double>(B, to64, B->cg64);
  }
  next_sweep(B, sw);
  if (!pred.empty()) {
    bphase_predictor(B, pred);
    batched_ph_factor(B, pred);
    start_solve(B, pred, 0);
  }
  solves_done(B, d0, d1);
  for (Slot* s : B->live)
    if (s->state != kFinished && (s->phase == kPhAwaitStats || s->phase == kPhAwaitIR)) return true;
  return false;
}

template <typename F>
qp_status batch_guard(qp_batch* B, F&& f) {
  try {
    f();
    return QP_OK;
  } catch (const Fail& e) {
    return e.st;
  } catch (const std::exception& e) {
    set_err(&B->sink, "internal error: %s", e.what());
    return QP_E_DEVICE;
  } catch (...) {
    set_err(&B->sink, "internal error");
    return QP_E_DEVICE;
  }
}

}  // namespace

// ============================================================================
extern "C" {

void qp_batch_destroy(qp_batch* B) {
  if (!B) return;
  if (B->stream) (void)hipStreamSynchronize(B->stream);
  if (B->prof_ready)
    for (int o = 0; o < kProfOps; ++o) {
      (void)hipEventDestroy(B->prof_ev[o].begin);
      (void)hipEventDestroy(B->prof_ev[o].end);
    }
  for (Slot* s : B->live) {
    release_slot_memory(B, s);
    delete s;
  }
  for (auto& kv : B->finished) delete kv.second;
  B->arena.release();
  for (void* p : {(void*)B->d_sc, (void*)B->d_stats, (void*)B->d_info, (void*)B->d_ipm})
    if (p) (void)hipFree(p);
  for (void* p : {(void*)B->h_sc, (void*)B->h_stats, (void*)B->h_info, (void*)B->h_isc})
    if (p) (void)hipHostFree(p);
  for (auto& a : B->stage) {
    if (a.h) (void)hipHostFree(a.h);
    if (a.d) (void)hipFree(a.d);
    if (a.ev) (void)hipEventDestroy(a.ev);
  }
  if (B->own_stream && B->stream) (void)hipStreamDestroy(B->stream);
  delete B;
}

qp_status qp_batch_create(qp_batch** out, const qp_options* opt, size_t hbm_budget_bytes, void* hip_stream) {
  if (!out) return QP_E_INVALID;
  *out = nullptr;
  qp_options o;
  qp_default_options(&o);
  if (opt) o = *opt;
  if (check_options(o) != QP_OK) return QP_E_INVALID;
  qp_batch* B = new qp_batch();
  B->opt = o;
  qp_status st = batch_guard(B, [&] {
    qp_ctx* sk = &B->sink;
    HIPCHK(sk, hipGetDevice(&B->dev));
    (void)dev_info();
    if (hip_stream) {
      B->stream = static_cast<hipStream_t>(hip_stream);
    } else {
      HIPCHK(sk, hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking));
      B->own_stream = true;
    }
    sk->stream = B->stream;
    size_t budget = hbm_budget_bytes;
    if (budget == 0) {
      size_t fr = 0, tot = 0;
      HIPCHK(sk, hipMemGetInfo(&fr, &tot));
      budget = fr / 10 * 8;
    }
    HIPCHK(sk, B->arena.init(budget));
    HIPCHK(sk, hipMalloc((void**)&B->d_sc, kMaxSlots * sizeof(PcgScalars)));
    HIPCHK(sk, hipMalloc((void**)&B->d_stats, (size_t)kMaxSlots * kStatsStride * sizeof(double)));
    HIPCHK(sk, hipMalloc((void**)&B->d_info, (size_t)kMaxSlots * kInfoStride * sizeof(int)));
    HIPCHK(sk, hipMemsetAsync(B->d_sc, 0, kMaxSlots * sizeof(PcgScalars), B->stream));
    HIPCHK(sk, hipMemsetAsync(B->d_stats, 0, (size_t)kMaxSlots * kStatsStride * sizeof(double), B->stream));
    HIPCHK(sk, hipMemsetAsync(B->d_info, 0, (size_t)kMaxSlots * kInfoStride * sizeof(int), B->stream));
    HIPCHK(sk, hipHostMalloc((void**)&B->h_sc, kMaxSlots * sizeof(PcgScalars), hipHostMallocDefault));
    HIPCHK(sk, hipHostMalloc((void**)&B->h_stats, (size_t)kMaxSlots * kStatsStride * sizeof(double),
                             hipHostMallocDefault));
    HIPCHK(sk, hipHostMalloc((void**)&B->h_info, (size_t)kMaxSlots * kInfoStride * sizeof(int),
                             hipHostMallocDefault));
    HIPCHK(sk, hipHostMalloc((void**)&B->h_isc, kMaxSlots * sizeof(IpmScalars), hipHostMallocDefault));
    HIPCHK(sk, hipMalloc((void**)&B->d_ipm, kMaxSlots * sizeof(IpmDesc)));
    for (int k = kMaxSlots - 1; k >= 0; --k) B->free_pools.push_back(k);
    HIPCHK(sk, hipStreamSynchronize(B->stream));
  });
  if (st != QP_OK) {
    qp_batch_destroy(B);
    return st;
  }
  *out = B;
  return QP_OK;
}

qp_status qp_batch_admit(qp_batch* B, int n, int m1, int m2, const double* H, const double* c, const double* A,
                         const double* b, const double* C, const double* d, qp_mem where, long long* ticket) {
  if (!B || !ticket) return QP_E_INVALID;
  *ticket = 0;
  qp_status pst = check_problem(n, m1, m2, H, c, A, b, C, d, where);
  if (pst != QP_OK) {
    set_err(&B->sink, "invalid QP (n=%d m1=%d m2=%d)", n, m1, m2);
    return pst;
  }
  const size_t need = footprint_bytes(n, m1, m2, B->opt, true, true);
  if (B->free_pools.empty() || need > B->arena.capacity() - B->arena.used()) {
    set_err(&B->sink, "not enough batch memory for the QP (%zu bytes needed, %zu free)", need,
            B->arena.capacity() - B->arena.used());
    return QP_E_NOMEM;
  }
  Slot* s = new Slot();
  s->pool = B->free_pools.back();
  B->free_pools.pop_back();
  s->n = n;
  s->m1 = m1;
  s->m2 = m2;
  qp_ctx* ctx = new qp_ctx();
  s->ctx = ctx;
  init_dims(ctx, n, m1, m2, B->opt);
  ctx->dev = B->dev;
  ctx->stream = B->stream;
  ctx->arena = &B->arena;
  ctx->pooled = true;
  ctx->sc = B->d_sc + s->pool;
  ctx->h_sc = B->h_sc + s->pool;
  ctx->stats = B->d_stats + (size_t)s->pool * kStatsStride;
  ctx->h_stats = B->h_stats + (size_t)s->pool * kStatsStride;
  ctx->info = B->d_info + (size_t)s->pool * kInfoStride;
  ctx->h_info = B->h_info + (size_t)s->pool * kInfoStride;
  ctx->h_isc = B->h_isc + s->pool;
  qp_status st = guarded(ctx, [&] {
    alloc_all(ctx);
    alloc_factor_scratch(ctx);
    upload_problem(ctx, H, c, A, b, C, d, where);
    const IpmDesc q = ipm_desc_of(ctx);
    HIPCHK(ctx, hipMemcpyAsync(B->d_ipm + s->pool, &q, sizeof(IpmDesc), hipMemcpyHostToDevice, B->stream));
    // the caller's arrays (and q) may be released when this call returns
    sync(ctx);
  });
  if (st != QP_OK) {
    B->sink.err = ctx->err;
    release_slot_memory(B, s);
    delete s;
    return st;
  }
  s->ticket = B->next_ticket++;
  s->t_admit = Clock::now();
  s->state = kQueued;
  B->live.push_back(s);
  *ticket = s->ticket;
  return QP_OK;
}

qp_status qp_batch_step(qp_batch* B, int max_rounds, int* n_done) {
  if (!B || max_rounds <= 0) return QP_E_INVALID;
  B->sink.err.clear();
  qp_status st = batch_guard(B, [&] {
    for (int r = 0; r < max_rounds && !B->live.empty(); ++r) tick(B);
  });
  if (n_done) *n_done = (int)B->finished.size();
  return st;
}

qp_status qp_batch_finished(qp_batch* B, long long* tickets, int cap, int* count) {
  if (!B || !count || cap < 0 || (cap > 0 && !tickets)) return QP_E_INVALID;
  std::vector<long long> t;
  for (auto& kv : B->finished) t.push_back(kv.first);
  std::sort(t.begin(), t.end());
  int k = 0;
  for (; k < cap && k < (int)t.size(); ++k) tickets[k] = t[k];
  *count = k;
  return QP_OK;
}

qp_status qp_batch_collect(qp_batch* B, long long ticket, double* x, double* lambda, double* nu, double* s,
                           qp_mem where, qp_ipm_info* info) {
  if (!B || !x || !lambda || !nu || !s) return QP_E_INVALID;
  if (where != QP_MEM_HOST && where != QP_MEM_DEVICE) return QP_E_INVALID;
  auto f = B->finished.find(ticket);
  if (f == B->finished.end()) {
    for (Slot* l : B->live)
      if (l->ticket == ticket) {
        set_err(&B->sink, "ticket %lld has not finished", ticket);
        return QP_E_STATE;
      }
    set_err(&B->sink, "unknown ticket %lld", ticket);
    return QP_E_INVALID;
  }
  Slot* sl = f->second;
  qp_status st = batch_guard(B, [&] {
    auto put = [&](double* dst, const std::vector<double>& v) {
      if (v.empty()) return;
      if (where == QP_MEM_HOST)
        memcpy(dst, v.data(), v.size() * sizeof(double));
      else
        HIPCHK(&B->sink, hipMemcpy(dst, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice));
    };
    put(x, sl->x);
    put(lambda, sl->lam);
    put(nu, sl->nu);
    put(s, sl->s);
  });
  if (st != QP_OK) return st;
  if (info) *info = sl->info;
  qp_status result = sl->status;
  if (result != QP_OK) B->sink.err = sl->err;
  B->finished.erase(f);
  delete sl;
  return result;
}

qp_status qp_batch_query(const qp_batch* B, int* in_flight, int* finished, size_t* bytes_used,
                         size_t* bytes_capacity, long long* rounds) {
  if (!B) return QP_E_INVALID;
  if (in_flight) *in_flight = (int)B->live.size();
  if (finished) *finished = (int)B->finished.size();
  if (bytes_used) *bytes_used = B->arena.used();
  if (bytes_capacity) *bytes_capacity = B->arena.capacity();
  if (rounds) *rounds = B->rounds;
  return QP_OK;
}

size_t qp_batch_footprint(const qp_options* opt, int n, int m1, int m2) {
  qp_options o;
  qp_default_options(&o);
  if (opt) o = *opt;
  if (n <= 0 || m1 <= 0 || m1 > n || m2 <= 0 || check_options(o) != QP_OK) return 0;
  return footprint_bytes(n, m1, m2, o, true, true);
}

const char* qp_batch_last_error(const qp_batch* B) { return B ? B->sink.err.c_str() : ""; }

qp_status qp_batch_profile_get(qp_batch* B, double avg_ms[6], double avg_bytes[6], long long samples[6], int reset) {
  if (!B || !avg_ms || !avg_bytes || !samples) return QP_E_INVALID;
  for (int o = 0; o < kProfOps; ++o) {
    samples[o] = B->prof_n[o];
    avg_ms[o] = B->prof_n[o] ? B->prof_ms[o] / (double)B->prof_n[o] : 0.0;
    avg_bytes[o] = B->prof_n[o] ? B->prof_bytes[o] / (double)B->prof_n[o] : 0.0;
    if (reset) {
      B->prof_ms[o] = B->prof_bytes[o] = 0;
      B->prof_n[o] = 0;
    }
  }
  return QP_OK;
}

}  // extern "C"
