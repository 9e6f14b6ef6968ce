// Kernels of one preconditioned CG step on the inequality-constraint reduced
// system K_F dnu = r_nu (eq. ineq-const-reduced), K_F applied in implicit form:
//
//   u = C^T p                      gemv_cols over C               (gemv.hip)
//   v = Sigma M u                  gemv_rows over the inverse factor
//   w = M^T v                      gemv_cols over the inverse factor
//   q = C w + D p, partial p^T q   pcg_q (this file)
//   alpha, dnu, r, z, beta, p      pcg_update (one workgroup)
//
// M = first n columns of L^{-1}, where K0 = L Sigma L^T, so w = [I 0] K0^{-1} [u; 0]
// and q = K_F p.  With P_L = D (eq. preconditioner-1) or no preconditioner,
// pcg_update applies z = P^{-1} r itself.  With P_H = D + C H^{-1} C^T
// (eq. preconditioner-2) the update stops after r and the preconditioner solve
// z = X_P^T (X_P r), X_P = chol(P_H)^{-1}, runs as a gemv_rows and a gemv_cols
// over X_P, followed by pcg_ph_update (r^T z, beta, p).
//
// Scalars live in device memory (PcgScalars); every kernel returns at once
// when the stop flag is set, so the host only polls every few steps.  The
// reductions over workgroup partials run in a single workgroup in a fixed
// order, so a solve is bitwise reproducible.  Each kernel also has a batched
// form over PcgDesc lists (one CG solve per QP) that runs the same body.
#include "kernels.hpp"
#include "gemv_core.hpp"
#include "pcg.hpp"

namespace qpg {

constexpr int kUpd = 1024;  // threads of the single-workgroup update kernels

__device__ __forceinline__ void pcg_check_stop(PcgScalars* sc, double rr, double wmax) {
  sc->rr = rr;
  sc->wmax = wmax;
  sc->iter += 1;
  if (rr <= sc->tol2 || (sc->wtol >= 0.0 && wmax <= sc->wtol)) sc->done = 1;
  else if (sc->iter >= sc->maxit) sc->done = 2;
}

// --------------------------------------------------------------------------
// device bodies

// x = 0, r = b, (z = P^{-1} r, p = z, rho = r^T z for P_L / none), stop tests.
template <typename T>
__device__ __forceinline__ void init_body(int m2, const T* __restrict__ b, const T* __restrict__ dvec,
                                          const T* __restrict__ wts, T* __restrict__ x, T* __restrict__ r,
                                          T* __restrict__ z, T* __restrict__ p, int prec, double rtol, double wtol,
                                          int maxit, PcgScalars* __restrict__ sc) {
  __shared__ double sh[16];
  double bb = 0, rz = 0, wm = 0;
  for (int i = threadIdx.x; i < m2; i += blockDim.x) {
    T bi = b[i];
    x[i] = 0;
    r[i] = bi;
    bb += (double)bi * bi;
    if (wts) wm = fmax(wm, fabs((double)wts[i] * bi));
    if (prec != kPrecH) {
      T zi = (prec == kPrecL) ? bi / dvec[i] : bi;
      z[i] = zi;
      p[i] = zi;
      rz += (double)bi * zi;
    }
  }
  bb = block_sum<double>(bb, sh);
  rz = block_sum<double>(rz, sh);
  wm = block_max<double>(wm, sh);
  if (threadIdx.x == 0) {
    sc->bb = bb;
    sc->rr = bb;
    sc->tol2 = rtol * rtol * bb;
    sc->wtol = wtol;
    sc->wmax = wm;
    sc->maxit = maxit;
    sc->iter = 0;
    sc->rho = rz;
    sc->rho_next = rz;
    sc->fresh = 1;
    sc->alpha = sc->beta = sc->pq = 0;
    sc->done = (bb == 0.0 || bb <= sc->tol2 || (wtol >= 0.0 && wm <= wtol)) ? 1 : 0;
    if (!sc->done && maxit <= 0) sc->done = 2;
  }
}

// Rows of q = C w + D p dealt to workgroup bid of nb (one wavefront per row,
// w staged in LDS), and the workgroup's partial of p^T q into bpart[bid].
template <typename T, int U>
__device__ __forceinline__ void q_body(const T* __restrict__ C, int ldc, int m2, int n, const T* __restrict__ w,
                                       const T* __restrict__ dvec, const T* __restrict__ p, T* __restrict__ q,
                                       double* __restrict__ bpart, int bid, int nb, T* ws, int stage,
                                       const int* __restrict__ done, int nt = 1) {
  // the stop flag (the same for every workgroup) is tested once the first
  // row's loads are in flight; a stopped solve leaves q and bpart untouched
  const int sk = *done;
  __shared__ double sh[16];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave, waves = blockDim.x / kWave;
  const int lenR = round_chunk<T>(n, ldc);
  if (stage) stage_x<T>(ws, w, n, lenR);  // else w is read through the caches
  double pq = 0;
  // p_i and d_i of a row are loaded before its dot (lane 0), so their latency
  // hides behind the row's
  // (unconditional loads at a clamped index, m2 >= 1: a load under a branch is
  // waited for at the branch's end)
  const int step = nb * waves;
  int i = bid * waves + wave;
  T pn = p[min(i, m2 - 1)], dn = dvec[min(i, m2 - 1)];
  for (; i < m2; i += step) {
    T v;
    if (!C)  // C = I: q = w + D p
      v = w[i];
    else if (nt)
      v = stage ? row_dot<T, U>(C + (size_t)i * ldc, ws, lenR, lane)
                : row_dot_gx<T, U>(C + (size_t)i * ldc, w, lenR, n, lane);
    else
      v = stage ? row_dot<T, U, false>(C + (size_t)i * ldc, ws, lenR, lane)
                : row_dot_gx<T, U, false>(C + (size_t)i * ldc, w, lenR, n, lane);
    if (sk) return;
    const T pi = pn, di = dn;
    if (i + step < m2) {
      pn = p[i + step];
      dn = dvec[i + step];
    }
    if (lane == 0) {
      T qi = v + di * pi;
      q[i] = qi;
      pq += (double)pi * qi;
    }
  }
  if (sk) return;  // waves without rows
  pq = block_sum<double>(pq, sh);
  if (threadIdx.x == 0) bpart[bid] = pq;
}

// The vector part of the step: alpha = rho / p^T q, dnu += alpha p,
// r -= alpha q, stop tests; for P_L / none also z, rho' = r^T z, beta, p.
// When every thread holds at most kKeep elements, z and p stay in registers
// between the two passes.  Per-thread partial sums follow the element order
// i = tid, tid + blockDim, ... in both branches, so the result is the same.
// kKeep: entries per thread held in registers (a template parameter of the body).

template <typename T>
__device__ __forceinline__ void update_elem(int i, T a, const T* __restrict__ dvec, const T* __restrict__ p,
                                            const T* __restrict__ q, T* __restrict__ x, T* __restrict__ r,
                                            T* __restrict__ z, const T* __restrict__ wts, int prec, double& rr,
                                            double& wm, double& rz, T& zi, T& pi) {
  pi = p[i];
  const T ri = r[i] - a * q[i];
  x[i] += a * pi;
  r[i] = ri;
  rr += (double)ri * ri;
  if (wts) wm = fmax(wm, fabs((double)wts[i] * ri));
  if (prec != kPrecH) {
    zi = (prec == kPrecL) ? ri / dvec[i] : ri;
    z[i] = zi;
    rz += (double)ri * zi;
  }
}

template <typename T>
__device__ __forceinline__ void update_elem_pre(int i, T a, T di, T pi, T qi, T xi, T ri0, T wi, T* __restrict__ x,
                                                T* __restrict__ r, T* __restrict__ z, bool has_w, int prec,
                                                double& rr, double& wm, double& rz, T& zi) {
  const T ri = ri0 - a * qi;
  x[i] = xi + a * pi;
  r[i] = ri;
  rr += (double)ri * ri;
  if (has_w) wm = fmax(wm, fabs((double)wi * ri));
  if (prec != kPrecH) {
    zi = (prec == kPrecL) ? ri / di : ri;
    z[i] = zi;
    rz += (double)ri * zi;
  }
}

// Stops at once (before any write) when the solve's stop flag is set.
template <typename T, int kKeep = 4>
__device__ __forceinline__ void update_body(int m2, int nparts, const double* __restrict__ bpart,
                                            const T* __restrict__ dvec, T* __restrict__ p, const T* __restrict__ q,
                                            T* __restrict__ x, T* __restrict__ r, T* __restrict__ z,
                                            const T* __restrict__ wts, int prec, PcgScalars* __restrict__ sc) {
  __shared__ double sh[16];
  __shared__ double sh3[3][16];
  __shared__ double alpha_s, beta_s;
  __shared__ int stop_s;
  const int bd = blockDim.x;
  const bool keep = m2 <= kKeep * bd;
  // every load of the step is issued before the first wait: the stop flag, the
  // p^T q partials and (when they fit in registers) this thread's entries
  const int done0 = sc->done;
  const double rho0 = sc->rho, tol2 = sc->tol2, wtol = sc->wtol;
  const int iter0 = sc->iter, maxit = sc->maxit;
  double s = 0;
  for (int b = threadIdx.x; b < nparts; b += bd) s += bpart[b];
  T pd[kKeep], pp[kKeep], pq_[kKeep], px[kKeep], pr[kKeep], pw[kKeep];
  if (keep) {
#pragma unroll
    for (int k = 0; k < kKeep; ++k) {
      const int i = threadIdx.x + k * bd;
      const bool in = i < m2;
      pp[k] = in ? p[i] : T(0);
      pq_[k] = in ? q[i] : T(0);
      px[k] = in ? x[i] : T(0);
      pr[k] = in ? r[i] : T(0);
      pd[k] = (in && prec == kPrecL) ? dvec[i] : T(1);
      pw[k] = (in && wts) ? wts[i] : T(0);
    }
  }
  if (done0) return;
  const double pq = block_sum<double>(s, sh);
  if (threadIdx.x == 0) {
    sc->pq = pq;
    if (!(pq > 0.0) || !isfinite(pq)) {
      sc->done = 3;
      stop_s = 1;
    } else {
      stop_s = 0;
      alpha_s = rho0 / pq;
      sc->alpha = alpha_s;
    }
  }
  __syncthreads();
  if (stop_s) return;
  const T a = (T)alpha_s;
  double rr = 0, rz = 0, wm = 0;
  T zk[kKeep], pk[kKeep];
  if (keep) {
#pragma unroll
    for (int k = 0; k < kKeep; ++k) {
      const int i = threadIdx.x + k * bd;
      pk[k] = pp[k];
      if (i < m2)
        update_elem_pre<T>(i, a, pd[k], pp[k], pq_[k], px[k], pr[k], pw[k], x, r, z, wts != nullptr, prec, rr, wm, rz,
                           zk[k]);
    }
  } else {
    T zi, pi;
    for (int i = threadIdx.x; i < m2; i += bd) update_elem<T>(i, a, dvec, p, q, x, r, z, wts, prec, rr, wm, rz, zi, pi);
  }
  block_sum2_max1(rr, rz, wm, sh3);
  if (threadIdx.x == 0) {
    // the stop test of pcg_check_stop on the values read at entry
    int dn = 0;
    if (rr <= tol2 || (wtol >= 0.0 && wm <= wtol)) dn = 1;
    else if (iter0 + 1 >= maxit) dn = 2;
    sc->rr = rr;
    sc->wmax = wm;
    sc->iter = iter0 + 1;
    if (dn) sc->done = dn;
    stop_s = dn;
    if (!dn && prec != kPrecH) {
      beta_s = rz / rho0;
      sc->beta = beta_s;
      sc->rho = rz;
    }
  }
  __syncthreads();
  if (stop_s || prec == kPrecH) return;
  const T bt = (T)beta_s;
  if (keep) {
#pragma unroll
    for (int k = 0; k < kKeep; ++k) {
      const int i = threadIdx.x + k * bd;
      if (i < m2) p[i] = zk[k] + bt * pk[k];
    }
  } else {
    for (int i = threadIdx.x; i < m2; i += bd) p[i] = z[i] + bt * p[i];
  }
}

// After z = P_H^{-1} r: rho' = r^T z, beta = rho' / rho (0 on the first step),
// p = z + beta p.
template <typename T>
__device__ __forceinline__ void ph_update_body(int m2, const T* __restrict__ r, const T* __restrict__ z,
                                               T* __restrict__ p, int init, PcgScalars* __restrict__ sc) {
  __shared__ double sh[16];
  __shared__ double beta_s;
  double rz = 0;
  for (int i = threadIdx.x; i < m2; i += blockDim.x) rz += (double)r[i] * z[i];
  rz = block_sum<double>(rz, sh);
  if (threadIdx.x == 0) {
    beta_s = init ? 0.0 : rz / sc->rho;
    sc->beta = beta_s;
    sc->rho = rz;
  }
  __syncthreads();
  const T bt = (T)beta_s;
  for (int i = threadIdx.x; i < m2; i += blockDim.x) p[i] = init ? z[i] : z[i] + bt * p[i];
}

// --------------------------------------------------------------------------
// single-solve kernels
template <typename T>
__global__ void __launch_bounds__(kUpd) pcg_init_kernel(int m2, const T* __restrict__ b, const T* __restrict__ dvec,
                                                        const T* __restrict__ wts, T* __restrict__ x,
                                                        T* __restrict__ r, T* __restrict__ z, T* __restrict__ p,
                                                        int prec, double rtol, double wtol, int maxit,
                                                        PcgScalars* __restrict__ sc) {
  init_body<T>(m2, b, dvec, wts, x, r, z, p, prec, rtol, wtol, maxit, sc);
}

template <typename T, int U>
__global__ void __launch_bounds__(256) pcg_q_kernel(const T* __restrict__ C, int ldc, int m2, int n,
                                                    const T* __restrict__ w, const T* __restrict__ dvec,
                                                    const T* __restrict__ p, T* __restrict__ q,
                                                    const PcgScalars* __restrict__ sc, double* __restrict__ bpart,
                                                    int stage, int nt) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  q_body<T, U>(C, ldc, m2, n, w, dvec, p, q, bpart, blockIdx.x, gridDim.x, reinterpret_cast<T*>(smem_raw), stage,
               &sc->done, nt);
}

template <typename T, int BD>
__global__ void __launch_bounds__(BD) pcg_update_kernel(int m2, int nparts, const double* __restrict__ bpart,
                                                        const T* __restrict__ dvec, T* __restrict__ p,
                                                        const T* __restrict__ q, T* __restrict__ x,
                                                        T* __restrict__ r, T* __restrict__ z,
                                                        const T* __restrict__ wts, int prec,
                                                        PcgScalars* __restrict__ sc) {
  update_body<T, (4096 / BD > 4 ? 4096 / BD : 4)>(m2, nparts, bpart, dvec, p, q, x, r, z, wts, prec, sc);
}

template <typename T>
__global__ void __launch_bounds__(kUpd) pcg_ph_update_kernel(int m2, const T* __restrict__ r,
                                                             const T* __restrict__ z, T* __restrict__ p, int init,
                                                             PcgScalars* __restrict__ sc) {
  if (sc->done) return;
  ph_update_body<T>(m2, r, z, p, init, sc);
}

// --------------------------------------------------------------------------
// batched kernels over PcgDesc lists: one workgroup per solve for the vector
// kernels, a flattened grid with a prefix table for the q sweep
template <typename T>
__global__ void __launch_bounds__(kUpd) bpcg_init_kernel(const PcgDesc<T>* __restrict__ descs) {
  const PcgDesc<T> d = descs[blockIdx.x];
  init_body<T>(d.m2, d.b, d.dvec, d.wts, d.x, d.r, d.z, d.p, d.prec, d.rtol, d.wtol, d.maxit, d.sc);
}

template <typename T, int U>
__global__ void __launch_bounds__(256) bpcg_q_kernel(const PcgDesc<T>* __restrict__ descs,
                                                     const int* __restrict__ prefix, int ndesc) {
  const DescBlock db = desc_of_block(prefix, ndesc, blockIdx.x);
  const PcgDesc<T> d = descs[db.j];
  extern __shared__ __align__(16) unsigned char smem_raw[];
  q_body<T, U>(d.C, d.ldc, d.m2, d.n, d.w, d.dvec, d.p, d.q, d.bpart, db.local, d.qblocks,
               reinterpret_cast<T*>(smem_raw), d.stage, &d.sc->done);
}

template <typename T>
__global__ void __launch_bounds__(kUpd) bpcg_update_kernel(const PcgDesc<T>* __restrict__ descs) {
  const PcgDesc<T> d = descs[blockIdx.x];
  update_body<T>(d.m2, d.qblocks, d.bpart, d.dvec, d.p, d.q, d.x, d.r, d.z, d.wts, d.prec, d.sc);
}

template <typename T>
__global__ void __launch_bounds__(kUpd) bpcg_ph_update_kernel(const PcgDesc<T>* __restrict__ descs, int init) {
  const PcgDesc<T> d = descs[blockIdx.x];
  if (d.sc->done) return;
  ph_update_body<T>(d.m2, d.r, d.z, d.p, init, d.sc);
}

// --------------------------------------------------------------------------
template <typename T>
hipError_t pcg_init(hipStream_t st, int m2, const T* b, const T* dvec, const T* wts, T* x, T* r, T* z, T* p,
                    int prec, double rtol, double wtol, int maxit, PcgScalars* sc) {
  hipLaunchKernelGGL(pcg_init_kernel<T>, dim3(1), dim3(kUpd), 0, st, m2, b, dvec, wts, x, r, z, p, prec, rtol, wtol,
                     maxit, sc);
  return hipGetLastError();
}

template <typename T>
int pcg_q_grid(int m2) {
  return gemv_rows_grid<T>(m2);
}

template <typename T>
hipError_t pcg_q(hipStream_t st, const T* C, int ldc, int m2, int n, const T* w, const T* dvec, const T* p, T* q,
                 const PcgScalars* sc, double* bpart, int bpart_cap, const EventPair* ev, int stage) {
  if (!tune().rows_stage || !C) stage = 0;  // a null C stands for the identity (m2 = n)
  size_t smem = stage ? rows_smem_bytes<T>(m2, n, kDense, ldc) : 0;
  if (smem > 150 * 1024) return hipErrorInvalidValue;
  const int grid = pcg_q_grid<T>(m2);
  if (grid > bpart_cap) return hipErrorInvalidValue;
  const int nt = tune().ld_nt & 1;
  if (tune().rows_unroll == 16)
    QPG_LAUNCH((pcg_q_kernel<T, 16>), dim3(grid), dim3(256), (uint32_t)smem, st, ev, C, ldc, m2, n, w, dvec, p, q, sc,
               bpart, stage, nt);
  else if (tune().rows_unroll == 8)
    QPG_LAUNCH((pcg_q_kernel<T, 8>), dim3(grid), dim3(256), (uint32_t)smem, st, ev, C, ldc, m2, n, w, dvec, p, q, sc,
               bpart, stage, nt);
  else
    QPG_LAUNCH((pcg_q_kernel<T, 4>), dim3(grid), dim3(256), (uint32_t)smem, st, ev, C, ldc, m2, n, w, dvec, p, q, sc,
               bpart, stage, nt);
  return hipGetLastError();
}

template <typename T>
hipError_t pcg_update(hipStream_t st, int m2, const double* bpart, const T* dvec, T* p, const T* q, T* x, T* r, T* z,
                      const T* wts, int prec, PcgScalars* sc) {
  switch (tune().upd_threads) {
    case 256:
      hipLaunchKernelGGL((pcg_update_kernel<T, 256>), dim3(1), dim3(256), 0, st, m2, pcg_q_grid<T>(m2), bpart, dvec,
                         p, q, x, r, z, wts, prec, sc);
      break;
    case 512:
      hipLaunchKernelGGL((pcg_update_kernel<T, 512>), dim3(1), dim3(512), 0, st, m2, pcg_q_grid<T>(m2), bpart, dvec,
                         p, q, x, r, z, wts, prec, sc);
      break;
    default:
      hipLaunchKernelGGL((pcg_update_kernel<T, kUpd>), dim3(1), dim3(kUpd), 0, st, m2, pcg_q_grid<T>(m2), bpart,
                         dvec, p, q, x, r, z, wts, prec, sc);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t pcg_ph_update(hipStream_t st, int m2, const T* r, const T* z, T* p, int init, PcgScalars* sc) {
  hipLaunchKernelGGL(pcg_ph_update_kernel<T>, dim3(1), dim3(kUpd), 0, st, m2, r, z, p, init, sc);
  return hipGetLastError();
}

// ---- folded-update CG step ------------------------------------------------------
// Scalars of the solve read at a kernel's entry.
struct FoldState {
  double rho, tol2, wtol;
  int iter, maxit;
};

// A thread's first kFoldPre partials of each kind, loaded at a kernel's entry
// so that their latency overlaps the kernel's other loads.
constexpr int kFoldPre = 2;
struct FoldPre {
  double rz[kFoldPre], rr[kFoldPre], wm[kFoldPre];
};
// Every load is issued unconditionally (indices clamped into the arrays, which
// hold at least one entry) and masked afterwards: a load under a branch makes
// the compiler wait for it at the branch's end, which would serialise them.
__device__ __forceinline__ FoldPre fold_load(const FoldParts& fp) {
  FoldPre f;
  const int lz = max(fp.nrz - 1, 0), lw = max(fp.nrw - 1, 0);
#pragma unroll
  for (int k = 0; k < kFoldPre; ++k) {
    const int b = threadIdx.x + k * blockDim.x;
    const double vz = fp.rz[min(b, lz)], vr = fp.rr[min(b, lw)], vw = fp.wm[min(b, lw)];
    f.rz[k] = b < fp.nrz ? vz : 0.0;
    f.rr[k] = b < fp.nrw ? vr : 0.0;
    f.wm[k] = b < fp.nrw ? vw : 0.0;
  }
  return f;
}

// Stop test of the update the last q sweep made, from its partials in a fixed
// order (the preloaded ones, then the rest), so every workgroup that calls it
// gets the same rz, rr, wm and code.
__device__ __forceinline__ int fold_reduce_test(const FoldParts& fp, const FoldPre& f, const FoldState& s,
                                                double& rz, double& rr, double& wm, double (*sh3)[16]) {
  rz = 0;
  rr = 0;
  wm = 0;
#pragma unroll
  for (int k = 0; k < kFoldPre; ++k) {
    rz += f.rz[k];
    rr += f.rr[k];
    wm = fmax(wm, f.wm[k]);
  }
  const int b0 = threadIdx.x + kFoldPre * blockDim.x;
  for (int b = b0; b < fp.nrz; b += blockDim.x) rz += fp.rz[b];
  for (int b = b0; b < fp.nrw; b += blockDim.x) {
    rr += fp.rr[b];
    wm = fmax(wm, fp.wm[b]);
  }
  block_sum2_max1(rz, rr, wm, sh3);
  if (rr <= s.tol2 || (s.wtol >= 0.0 && wm <= s.wtol)) return 1;
  if (s.iter + 1 >= s.maxit) return 2;
  return 0;
}

// u = C^T p_new with p_new = z + beta p_old, as C^T z + beta C^T p_old: both dots
// of a row of the stored C^T from one load of the row.  beta = rho' / rho comes
// from the partials of rho' = r^T z, reduced by every workgroup after its first
// row; workgroup 0 records the update in the solve's scalars.  With recur set,
// C^T p_old is the u of the previous step (C^T applied to the same p_old, which
// the q sweep stored), so each row takes one dot, C^T z, and reads one vector:
// u = C^T z + beta u_old.  The first step of a solve (p = z) takes u = C^T z.
template <typename T, int U, bool RECUR>
__global__ void __launch_bounds__(256) fold_ct_kernel(const T* __restrict__ CT, int ldct, int n, int m2,
                                                      const T* __restrict__ z, const T* __restrict__ p,
                                                      T* __restrict__ u, PcgScalars* __restrict__ sc, FoldParts fp,
                                                      int nt) {
  __shared__ double sh3[3][16];
  // a stopped solve returns before any other load (the steps launched past a
  // stop cost one launch each); then the partials of the last update's test are
  // issued together with this wavefront's first row
  if (sc->done) return;
  const int fresh = sc->fresh;
  const FoldState s{sc->rho, sc->tol2, sc->wtol, sc->iter, sc->maxit};
  const FoldPre pre = fold_load(fp);
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave, waves = blockDim.x / kWave;
  const int lenR = round_chunk<T>(m2, ldct);
  const int stride = gridDim.x * waves;
  // (the two forms are separate instantiations: the two-dot form needs twice
  // the vector registers, which would cost the one-dot form its occupancy)
  auto dots = [&](int i, T& d1, T& d2) {
    const T* row = CT + (size_t)i * ldct;
    if constexpr (RECUR) {
      const T uo = u[i];  // unconditional (see fold_load)
      d2 = fresh ? T(0) : uo;
      d1 = nt ? row_dot_gx<T, U, true>(row, z, lenR, m2, lane) : row_dot_gx<T, U, false>(row, z, lenR, m2, lane);
    } else if (nt) {
      row_dot2_gx<T, U, true>(row, z, p, lenR, m2, lane, d1, d2);
    } else {
      row_dot2_gx<T, U, false>(row, z, p, lenR, m2, lane, d1, d2);
    }
  };
  int i = blockIdx.x * waves + wave;
  T d1 = 0, d2 = 0;
  if (i < n) dots(i, d1, d2);
  double beta = 0.0;  // the first step of a solve: p = z from the initialisation
  if (!fresh) {
    double rz, rr, wm;
    const int dn = fold_reduce_test(fp, pre, s, rz, rr, wm, sh3);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc->rr = rr;
      sc->wmax = wm;
      sc->iter = s.iter + 1;
      if (dn) {
        sc->done = dn;
      } else {
        sc->beta = rz / s.rho;
        sc->rho_next = rz;
      }
    }
    if (dn) return;
    beta = rz / s.rho;
  } else if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc->rho_next = s.rho;
  }
  const T bt = (T)beta;
  if (i < n && lane == 0) u[i] = fresh ? d1 : d1 + bt * d2;
  for (i += stride; i < n; i += stride) {
    dots(i, d1, d2);
    if (lane == 0) u[i] = fresh ? d1 : d1 + bt * d2;
  }
}

// q = C w + D p_new, p = p_new = z + beta p_old, alpha = rho / p^T q (p^T q from
// the partials of the K0 sum), dnu += alpha p, r -= alpha q, z = P_L^{-1} r (or
// r without a preconditioner; P_H computes z afterwards), and the per-workgroup
// partials of the next stop test.  Workgroup 0 records alpha and rho.
template <typename T, int U>
__global__ void __launch_bounds__(256) fold_q_kernel(const T* __restrict__ C, int ldc, int m2, int n,
                                                     const T* __restrict__ w, const T* __restrict__ dvec,
                                                     T* __restrict__ p, T* __restrict__ q, T* __restrict__ x,
                                                     T* __restrict__ r, T* __restrict__ z, const T* __restrict__ wts,
                                                     int prec, PcgScalars* __restrict__ sc, FoldParts fp, int nt) {
  __shared__ double sh[16];
  __shared__ double sh3[3][16];
  if (sc->done) return;  // before any other load (see fold_ct_kernel)
  const double rho = sc->rho_next;
  const T bt = (T)sc->beta;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave, waves = blockDim.x / kWave;
  const int lenR = round_chunk<T>(n, ldc);
  const int stride = gridDim.x * waves;
  auto dot = [&](int i) {
    const T* row = C + (size_t)i * ldc;
    return nt ? row_dot_gx<T, U>(row, w, lenR, n, lane) : row_dot_gx<T, U, false>(row, w, lenR, n, lane);
  };
  int i = blockIdx.x * waves + wave;
  // the p^T q partials and the vector entries of this wavefront's first row are
  // loaded before its dot, so their latency hides behind the row's
  // (unconditional loads at clamped indices, masked afterwards: see fold_load)
  const double a0 = fp.al[min((int)threadIdx.x, max(fp.nal - 1, 0))];
  const int ic = min(i, m2 - 1);
  const T e_d = dvec[ic], e_z = z[ic], e_p = p[ic], e_x = x[ic], e_r = r[ic], e_w = wts ? wts[ic] : T(0);
  T v = 0;
  if (i < m2) v = dot(i);
  double pq = (int)threadIdx.x < fp.nal ? a0 : 0.0;
  for (int b = threadIdx.x + blockDim.x; b < fp.nal; b += blockDim.x) pq += fp.al[b];
  pq = block_sum<double>(pq, sh);
  if (!(pq > 0.0) || !isfinite(pq)) {  // the same decision in every workgroup
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc->pq = pq;
      sc->done = 3;
    }
    return;
  }
  const T a = (T)(rho / pq);
  double rz = 0, rr = 0, wm = 0;
  auto upd = [&](int ii, T vv, T di, T zi0, T pi0, T xi, T ri0, T wi) {
    const T pi = zi0 + bt * pi0;
    const T qi = vv + di * pi;
    p[ii] = pi;
    q[ii] = qi;
    x[ii] = xi + a * pi;
    const T ri = ri0 - a * qi;
    r[ii] = ri;
    rr += (double)ri * ri;
    if (wts) wm = fmax(wm, fabs((double)wi * ri));
    if (prec != kPrecH) {
      const T zi = (prec == kPrecL) ? ri / di : ri;
      z[ii] = zi;
      rz += (double)ri * zi;
    }
  };
  if (i < m2 && lane == 0) upd(i, v, e_d, e_z, e_p, e_x, e_r, e_w);
  for (i += stride; i < m2; i += stride) {
    v = dot(i);
    if (lane == 0) upd(i, v, dvec[i], z[i], p[i], x[i], r[i], wts ? wts[i] : T(0));
  }
  block_sum2_max1(rz, rr, wm, sh3);
  if (threadIdx.x == 0) {
    if (prec != kPrecH) fp.rz[blockIdx.x] = rz;
    fp.rr[blockIdx.x] = rr;
    fp.wm[blockIdx.x] = wm;
    if (blockIdx.x == 0) {
      sc->pq = pq;
      sc->alpha = rho / pq;
      sc->rho = rho;
      sc->fresh = 0;
    }
  }
}

// The stop test of the last update of a chunk (same code as fold_ct's), so the
// host's poll sees a finished solve; leaves the scalars alone otherwise.
__global__ void __launch_bounds__(256) fold_test_kernel(PcgScalars* __restrict__ sc, FoldParts fp) {
  __shared__ double sh3[3][16];
  if (sc->done || sc->fresh) return;
  const FoldState s{sc->rho, sc->tol2, sc->wtol, sc->iter, sc->maxit};
  double rz, rr, wm;
  const int dn = fold_reduce_test(fp, fold_load(fp), s, rz, rr, wm, sh3);
  if (dn && threadIdx.x == 0) {
    sc->rr = rr;
    sc->wmax = wm;
    sc->iter = s.iter + 1;
    sc->done = dn;
  }
}

template <typename T>
hipError_t fold_ct(hipStream_t st, const T* CT, int ldct, int n, int m2, const T* z, const T* p, T* u,
                   PcgScalars* sc, const FoldParts& fp, const EventPair* ev) {
  if (n <= 0) return hipSuccess;
  const dim3 grid(gemv_rows_grid<T>(n));
  const int nt = tune().ld_nt & 1;
  const bool recur = tune().cg_fold & 4;
  if (recur && tune().rows_unroll >= 8)
    QPG_LAUNCH((fold_ct_kernel<T, 8, true>), grid, dim3(256), 0u, st, ev, CT, ldct, n, m2, z, p, u, sc, fp, nt);
  else if (recur)
    QPG_LAUNCH((fold_ct_kernel<T, 4, true>), grid, dim3(256), 0u, st, ev, CT, ldct, n, m2, z, p, u, sc, fp, nt);
  else  // two dots per row: half the matrix loads in flight, the same registers
    QPG_LAUNCH((fold_ct_kernel<T, 4, false>), grid, dim3(256), 0u, st, ev, CT, ldct, n, m2, z, p, u, sc, fp, nt);
  return hipGetLastError();
}

template <typename T>
hipError_t fold_q(hipStream_t st, const T* C, int ldc, int m2, int n, const T* w, const T* dvec, T* p, T* q, T* x,
                  T* r, T* z, const T* wts, int prec, PcgScalars* sc, const FoldParts& fp, const EventPair* ev) {
  const int grid = pcg_q_grid<T>(m2);
  if (grid > fp.nrw || (prec != kPrecH && grid > fp.nrz)) return hipErrorInvalidValue;
  const int nt = tune().ld_nt & 1;
  if (tune().rows_unroll >= 8)
    QPG_LAUNCH((fold_q_kernel<T, 8>), dim3(grid), dim3(256), 0u, st, ev, C, ldc, m2, n, w, dvec, p, q, x, r, z, wts,
               prec, sc, fp, nt);
  else
    QPG_LAUNCH((fold_q_kernel<T, 4>), dim3(grid), dim3(256), 0u, st, ev, C, ldc, m2, n, w, dvec, p, q, x, r, z, wts,
               prec, sc, fp, nt);
  return hipGetLastError();
}

hipError_t fold_test(hipStream_t st, PcgScalars* sc, const FoldParts& fp) {
  hipLaunchKernelGGL(fold_test_kernel, dim3(1), dim3(256), 0, st, sc, fp);
  return hipGetLastError();
}

// ---- batched launchers ------------------------------------------------------
int bpcg_q_blocks(int m2) { return m2 > 16 ? (m2 + 15) / 16 : 1; }

template <typename T>
hipError_t bpcg_init(hipStream_t st, const PcgDesc<T>* d, int ndesc) {
  if (ndesc <= 0) return hipSuccess;
  hipLaunchKernelGGL(bpcg_init_kernel<T>, dim3(ndesc), dim3(kUpd), 0, st, d);
  return hipGetLastError();
}

template <typename T>
hipError_t bpcg_q(hipStream_t st, const PcgDesc<T>* d, const int* prefix, int ndesc, int total_blocks, size_t smem,
                  const EventPair* ev) {
  if (ndesc <= 0 || total_blocks <= 0) return hipSuccess;
  if (smem > 150 * 1024) return hipErrorInvalidValue;
  if (tune().brows_unroll == 8)
    QPG_LAUNCH((bpcg_q_kernel<T, 8>), dim3(total_blocks), dim3(256), (uint32_t)smem, st, ev, d, prefix, ndesc);
  else
    QPG_LAUNCH((bpcg_q_kernel<T, 4>), dim3(total_blocks), dim3(256), (uint32_t)smem, st, ev, d, prefix, ndesc);
  return hipGetLastError();
}

template <typename T>
hipError_t bpcg_update(hipStream_t st, const PcgDesc<T>* d, int ndesc) {
  if (ndesc <= 0) return hipSuccess;
  hipLaunchKernelGGL(bpcg_update_kernel<T>, dim3(ndesc), dim3(kUpd), 0, st, d);
  return hipGetLastError();
}

template <typename T>
hipError_t bpcg_ph_update(hipStream_t st, const PcgDesc<T>* d, int ndesc, int init) {
  if (ndesc <= 0) return hipSuccess;
  hipLaunchKernelGGL(bpcg_ph_update_kernel<T>, dim3(ndesc), dim3(kUpd), 0, st, d, init);
  return hipGetLastError();
}

#define QPG_PCG_INST(T)                                                                                           \
  template hipError_t pcg_init<T>(hipStream_t, int, const T*, const T*, const T*, T*, T*, T*, T*, int, double,   \
                                  double, int, PcgScalars*);                                                      \
  template int pcg_q_grid<T>(int);                                                                                \
  template hipError_t pcg_q<T>(hipStream_t, const T*, int, int, int, const T*, const T*, const T*, T*,            \
                               const PcgScalars*, double*, int, const EventPair*, int);                           \
  template hipError_t pcg_update<T>(hipStream_t, int, const double*, const T*, T*, const T*, T*, T*, T*,          \
                                    const T*, int, PcgScalars*);                                                  \
  template hipError_t pcg_ph_update<T>(hipStream_t, int, const T*, const T*, T*, int, PcgScalars*);               \
  template hipError_t bpcg_init<T>(hipStream_t, const PcgDesc<T>*, int);                                          \
  template hipError_t bpcg_q<T>(hipStream_t, const PcgDesc<T>*, const int*, int, int, size_t, const EventPair*);  \
  template hipError_t bpcg_update<T>(hipStream_t, const PcgDesc<T>*, int);                                        \
  template hipError_t bpcg_ph_update<T>(hipStream_t, const PcgDesc<T>*, int, int);                             \
  template hipError_t fold_ct<T>(hipStream_t, const T*, int, int, int, const T*, const T*, T*, PcgScalars*,       \
                                 const FoldParts&, const EventPair*);                                             \
  template hipError_t fold_q<T>(hipStream_t, const T*, int, int, int, const T*, const T*, T*, T*, T*, T*, T*,     \
                                const T*, int, PcgScalars*, const FoldParts&, const EventPair*);
QPG_PCG_INST(double)
QPG_PCG_INST(float)

}  // namespace qpg
