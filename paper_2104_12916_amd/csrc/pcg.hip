// Fused kernels of one preconditioned CG step on the inequality-constraint
// reduced system K_F dnu = r_nu (eq. ineq-const-reduced), K_F applied in
// implicit form:
//
//   u = C^T p                      gemv_cols over C            (gemv.hip)
//   v = Sigma M u                  gemv_rows over the inverse factor
//   w = M^T v                      gemv_cols over the inverse factor
//   q = C w + D p, then the CG update                           (this file)
//
// M = first n columns of L^{-1}, where K0 = L Sigma L^T, so w = [I 0] K0^{-1} [u; 0]
// and q = K_F p.  The last workgroup of the q kernel finishes the dot product
// p^T q and performs the whole vector update of the step (alpha, dnu, r, the
// P_L = D preconditioner of eq. preconditioner-1, r^T z, beta, p), so a
// P_L/unpreconditioned step is four launches.  With P_H (eq. preconditioner-2)
// the preconditioner solve z = X_P^T (X_P r), X_P = chol(D + C H^{-1} C^T)^{-1},
// adds a gemv_rows and the pcg_prec_cols kernel below, whose last workgroup
// forms r^T z, beta and p.
//
// Scalars live in device memory (PcgScalars); kernels launched after
// convergence return immediately, so the host only polls every few steps.
#include "kernels.hpp"
#include "gemv_core.hpp"
#include "pcg.hpp"

namespace qpg {

__device__ __forceinline__ void pcg_check_stop(PcgScalars* sc, double rr, double wmax) {
  sc->rr = rr;
  sc->wmax = wmax;
  sc->iter += 1;
  if (rr <= sc->tol2 || (sc->wtol >= 0.0 && wmax <= sc->wtol)) sc->done = 1;
  else if (sc->iter >= sc->maxit) sc->done = 2;
}

// --------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) pcg_init_kernel(int m2, const T* __restrict__ b, const T* __restrict__ dvec,
                                                       const T* __restrict__ wts, T* __restrict__ x, T* __restrict__ r,
                                                       T* __restrict__ z, T* __restrict__ p, int prec, double rtol,
                                                       double wtol, int maxit, PcgScalars* __restrict__ sc) {
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
    sc->alpha = sc->beta = sc->pq = 0;
    sc->done = (bb == 0.0 || bb <= sc->tol2 || (wtol >= 0.0 && wm <= wtol)) ? 1 : 0;
    if (!sc->done && maxit <= 0) sc->done = 2;
  }
}

// --------------------------------------------------------------------------
// q = C w + D p over rows of C (one wavefront per row, w in LDS), then the step.
template <typename T>
__global__ void __launch_bounds__(256) pcg_q_kernel(const T* __restrict__ C, int ldc, int m2, int n,
                                                    const T* __restrict__ w, const T* __restrict__ dvec,
                                                    T* __restrict__ p, T* __restrict__ q, T* __restrict__ x,
                                                    T* __restrict__ r, T* __restrict__ z, const T* __restrict__ wts,
                                                    int prec, PcgScalars* __restrict__ sc, double* __restrict__ bpart,
                                                    unsigned* __restrict__ counter) {
  if (sc->done) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* ws = reinterpret_cast<T*>(smem_raw);
  __shared__ double sh[16];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave, waves = blockDim.x / kWave;
  const int lenR = round_chunk<T>(n, ldc);
  stage_x<T>(ws, w, n, lenR);
  double pq = 0;
  for (int i = blockIdx.x * waves + wave; i < m2; i += gridDim.x * waves) {
    T v = row_dot<T>(C + (size_t)i * ldc, ws, lenR, lane);
    if (lane == 0) {
      T pi = p[i];
      T qi = v + dvec[i] * pi;
      q[i] = qi;
      pq += (double)pi * qi;
    }
  }
  pq = block_sum<double>(pq, sh);
  if (threadIdx.x == 0) bpart[blockIdx.x] = pq;
  if (!last_block(counter, gridDim.x)) return;

  // ---- last workgroup: the vector part of the CG step -------------------
  double s = 0;
  for (int b = threadIdx.x; b < (int)gridDim.x; b += blockDim.x) s += bpart[b];
  pq = block_sum<double>(s, sh);
  __shared__ double alpha_s, beta_s;
  __shared__ int stop_s;
  if (threadIdx.x == 0) {
    sc->pq = pq;
    if (!(pq > 0.0) || !isfinite(pq)) {
      sc->done = 3;
      stop_s = 1;
    } else {
      stop_s = 0;
      alpha_s = sc->rho / pq;
      sc->alpha = alpha_s;
    }
  }
  __syncthreads();
  if (stop_s) return;
  const T a = (T)alpha_s;
  double rr = 0, rz = 0, wm = 0;
  for (int i = threadIdx.x; i < m2; i += blockDim.x) {
    T pi = p[i];
    T ri = r[i] - a * q[i];
    x[i] += a * pi;
    r[i] = ri;
    rr += (double)ri * ri;
    if (wts) wm = fmax(wm, fabs((double)wts[i] * ri));
    if (prec != kPrecH) {
      T zi = (prec == kPrecL) ? ri / dvec[i] : ri;
      z[i] = zi;
      rz += (double)ri * zi;
    }
  }
  rr = block_sum<double>(rr, sh);
  wm = block_max<double>(wm, sh);
  rz = block_sum<double>(rz, sh);
  if (threadIdx.x == 0) {
    pcg_check_stop(sc, rr, wm);
    stop_s = sc->done;
    if (!stop_s && prec != kPrecH) {
      beta_s = rz / sc->rho;
      sc->beta = beta_s;
      sc->rho = rz;
    }
  }
  __syncthreads();
  if (stop_s || prec == kPrecH) return;
  const T bt = (T)beta_s;
  for (int i = threadIdx.x; i < m2; i += blockDim.x) p[i] = z[i] + bt * p[i];
}

// --------------------------------------------------------------------------
// P_H apply, second half: z = X_P^T t (column tiles of the lower-triangular X_P),
// then r^T z, beta and p = z + beta p in the last workgroup of the grid.
template <typename T>
__global__ void __launch_bounds__(256) pcg_prec_cols_kernel(const T* __restrict__ XP, int ldp, int m2,
                                                            const T* __restrict__ t, const T* __restrict__ r,
                                                            T* __restrict__ z, T* __restrict__ p, int init,
                                                            PcgScalars* __restrict__ sc, T* __restrict__ part,
                                                            double* __restrict__ tpart, unsigned* __restrict__ counters,
                                                            int rows_per_chunk, int nchunks) {
  if (sc->done) return;
  constexpr int CW = kWave * Vec16<T>::n;
  __shared__ double sh[16];
  const int tile = blockIdx.x, chunk = blockIdx.y;
  const int ntiles = gridDim.x;
  const int c0 = tile * CW;
  const int first_chunk = c0 / rows_per_chunk;
  if (chunk < first_chunk) return;
  const int r0 = chunk * rows_per_chunk;
  const int r1 = min(m2, r0 + rows_per_chunk);
  __shared__ T red[4][CW];
  cols_block_partial<T>(XP, ldp, r0, r1, c0, kLower, t, red);
  if (threadIdx.x < CW) {
    const int jj = threadIdx.x;
    part[(size_t)chunk * ldp + c0 + jj] = (red[0][jj] + red[1][jj]) + (red[2][jj] + red[3][jj]);
  }
  if (!last_block(&counters[tile], (unsigned)(nchunks - first_chunk))) return;
  double rz = 0;
  for (int jj = threadIdx.x; jj < CW; jj += blockDim.x) {
    int col = c0 + jj;
    T s = 0;
    for (int ch = first_chunk; ch < nchunks; ++ch) s += part[(size_t)ch * ldp + col];
    if (col < m2) {
      z[col] = s;
      rz += (double)r[col] * s;
    }
  }
  rz = block_sum<double>(rz, sh);
  if (threadIdx.x == 0) tpart[tile] = rz;
  if (!last_block(&counters[ntiles], (unsigned)ntiles)) return;
  double s2 = 0;
  for (int b = threadIdx.x; b < ntiles; b += blockDim.x) s2 += tpart[b];
  rz = block_sum<double>(s2, sh);
  __shared__ double beta_s;
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
template <typename T>
hipError_t pcg_init(hipStream_t st, int m2, const T* b, const T* dvec, const T* wts, T* x, T* r, T* z, T* p,
                    int prec, double rtol, double wtol, int maxit, PcgScalars* sc) {
  hipLaunchKernelGGL(pcg_init_kernel<T>, dim3(1), dim3(256), 0, st, m2, b, dvec, wts, x, r, z, p, prec, rtol, wtol,
                     maxit, sc);
  return hipGetLastError();
}

template <typename T>
int pcg_q_grid(int m2) {
  int blocks = (m2 + 3) / 4;
  int cap = dev_info().cu_count * 2;
  return blocks < cap ? blocks : cap;
}

template <typename T>
hipError_t pcg_q(hipStream_t st, const T* C, int ldc, int m2, int n, const T* w, const T* dvec, T* p, T* q, T* x,
                 T* r, T* z, const T* wts, int prec, PcgScalars* sc, double* bpart, unsigned* counter) {
  constexpr int CH = kWave * Vec16<T>::n;
  int lenR = (n + CH - 1) / CH * CH;
  if (lenR > ldc) lenR = ldc;
  size_t smem = (size_t)lenR * sizeof(T);
  if (smem > 150 * 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(pcg_q_kernel<T>, dim3(pcg_q_grid<T>(m2)), dim3(256), smem, st, C, ldc, m2, n, w, dvec, p, q, x,
                     r, z, wts, prec, sc, bpart, counter);
  return hipGetLastError();
}

template <typename T>
hipError_t pcg_prec_cols(hipStream_t st, const T* XP, int ldp, int m2, const T* t, const T* r, T* z, T* p, int init,
                         PcgScalars* sc, const GemvWork<T>& w, double* tpart) {
  constexpr int CW = kWave * Vec16<T>::n;
  int tiles = (m2 + CW - 1) / CW;
  int rpc, nch;
  gemv_cols_plan<T>(m2, m2, rpc, nch);
  if ((size_t)nch * ldp > w.part_elems || tiles + 1 > w.n_counters || tiles * CW > ldp) return hipErrorInvalidValue;
  hipLaunchKernelGGL(pcg_prec_cols_kernel<T>, dim3(tiles, nch), dim3(256), 0, st, XP, ldp, m2, t, r, z, p, init, sc,
                     w.part, tpart, w.counters, rpc, nch);
  return hipGetLastError();
}

#define QPG_PCG_INST(T)                                                                                           \
  template hipError_t pcg_init<T>(hipStream_t, int, const T*, const T*, const T*, T*, T*, T*, T*, int, double,   \
                                  double, int, PcgScalars*);                                                      \
  template int pcg_q_grid<T>(int);                                                                                \
  template hipError_t pcg_q<T>(hipStream_t, const T*, int, int, int, const T*, const T*, T*, T*, T*, T*, T*,      \
                               const T*, int, PcgScalars*, double*, unsigned*);                                   \
  template hipError_t pcg_prec_cols<T>(hipStream_t, const T*, int, int, const T*, const T*, T*, T*, int,          \
                                       PcgScalars*, const GemvWork<T>&, double*);
QPG_PCG_INST(double)
QPG_PCG_INST(float)

}  // namespace qpg
