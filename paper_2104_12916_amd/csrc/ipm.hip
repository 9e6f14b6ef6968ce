// FP64 vector kernels of the outer interior point iteration (Sec. 2 and 4):
// residuals of eq. rhs-KKT4 with the statistics of the relative KKT score, the
// reduced right-hand side r_nu (eq. ineq-const-reduced) and D = V^{-1} S
// (eq. diag-d), the recovered directions (eqs. schur-delta-x, delz), and the
// Mehrotra predictor-corrector step.  All are small O(n + m) kernels; the
// reductions use one workgroup so their summation order is fixed.
#include <algorithm>

#include "kernels.hpp"
#include "gemv_core.hpp"
#include "pcg.hpp"

namespace qpg {

constexpr int kRedThreads = 1024;

__device__ __forceinline__ void ipm_stats_body(
    int n, int m1, int m2, const double* __restrict__ Hx, const double* __restrict__ Atl,
    const double* __restrict__ Ctn, const double* __restrict__ Ax, const double* __restrict__ Cx,
    const double* __restrict__ x, const double* __restrict__ c, const double* __restrict__ lam,
    const double* __restrict__ b, const double* __restrict__ nu, const double* __restrict__ s,
    const double* __restrict__ d, double* __restrict__ rg, double* __restrict__ re, double* __restrict__ ri,
    double* __restrict__ stats) {
  __shared__ double sh[16];
  double rd_inf = 0, hx_inf = 0, c_inf = 0, atl_inf = 0, ctn_inf = 0, xhx = 0, cx = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double g = -Hx[i] - c[i] + Atl[i] + Ctn[i];
    rg[i] = g;
    rd_inf = fmax(rd_inf, fabs(g));
    hx_inf = fmax(hx_inf, fabs(Hx[i]));
    c_inf = fmax(c_inf, fabs(c[i]));
    atl_inf = fmax(atl_inf, fabs(Atl[i]));
    ctn_inf = fmax(ctn_inf, fabs(Ctn[i]));
    xhx += x[i] * Hx[i];
    cx += c[i] * x[i];
  }
  double re_inf = 0, ax_inf = 0, b_inf = 0, bl = 0;
  for (int i = threadIdx.x; i < m1; i += blockDim.x) {
    double e = Ax[i] - b[i];
    re[i] = e;
    re_inf = fmax(re_inf, fabs(e));
    ax_inf = fmax(ax_inf, fabs(Ax[i]));
    b_inf = fmax(b_inf, fabs(b[i]));
    bl += b[i] * lam[i];
  }
  double viol = 0, d_inf = 0, dn = 0, nu_min = INFINITY, nu_inf = 0, snu = 0, ri_inf = 0, s_min = INFINITY;
  for (int i = threadIdx.x; i < m2; i += blockDim.x) {
    double e = Cx[i] - d[i] - s[i];
    ri[i] = e;
    ri_inf = fmax(ri_inf, fabs(e));
    viol = fmax(viol, d[i] - Cx[i]);
    d_inf = fmax(d_inf, fabs(d[i]));
    dn += d[i] * nu[i];
    nu_min = fmin(nu_min, nu[i]);
    nu_inf = fmax(nu_inf, fabs(nu[i]));
    snu += s[i] * nu[i];
    s_min = fmin(s_min, s[i]);
  }
  double vals[kNumStats];
  vals[kRdInf] = block_max(rd_inf, sh);
  vals[kHxInf] = block_max(hx_inf, sh);
  vals[kCInf] = block_max(c_inf, sh);
  vals[kAtlInf] = block_max(atl_inf, sh);
  vals[kCtnInf] = block_max(ctn_inf, sh);
  vals[kReInf] = block_max(re_inf, sh);
  vals[kAxInf] = block_max(ax_inf, sh);
  vals[kBInf] = block_max(b_inf, sh);
  vals[kViolInf] = block_max(viol, sh);
  vals[kDInf] = block_max(d_inf, sh);
  vals[kXHx] = block_sum(xhx, sh);
  vals[kCx] = block_sum(cx, sh);
  vals[kBl] = block_sum(bl, sh);
  vals[kDn] = block_sum(dn, sh);
  vals[kNuMin] = -block_max(-nu_min, sh);
  vals[kNuInf] = block_max(nu_inf, sh);
  vals[kSNu] = block_sum(snu, sh);
  vals[kRiInf] = block_max(ri_inf, sh);
  vals[kSMin] = -block_max(-s_min, sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < kNumStats; ++k) stats[k] = vals[k];
}

__global__ void __launch_bounds__(kRedThreads) ipm_stats_kernel(
    int n, int m1, int m2, const double* __restrict__ Hx, const double* __restrict__ Atl,
    const double* __restrict__ Ctn, const double* __restrict__ Ax, const double* __restrict__ Cx,
    const double* __restrict__ x, const double* __restrict__ c, const double* __restrict__ lam,
    const double* __restrict__ b, const double* __restrict__ nu, const double* __restrict__ s,
    const double* __restrict__ d, double* __restrict__ rg, double* __restrict__ re, double* __restrict__ ri,
    double* __restrict__ stats) {
  ipm_stats_body(n, m1, m2, Hx, Atl, Ctn, Ax, Cx, x, c, lam, b, nu, s, d, rg, re, ri, stats);
}

hipError_t ipm_stats(hipStream_t st, int n, int m1, int m2, const double* Hx, const double* Atl, const double* Ctn,
                     const double* Ax, const double* Cx, const double* x, const double* c, const double* lam,
                     const double* b, const double* nu, const double* s, const double* d, double* rg, double* re,
                     double* ri, double* stats) {
  hipLaunchKernelGGL(ipm_stats_kernel, dim3(1), dim3(kRedThreads), 0, st, n, m1, m2, Hx, Atl, Ctn, Ax, Cx, x, c, lam,
                     b, nu, s, d, rg, re, ri, stats);
  return hipGetLastError();
}

// r_c (predictor: S V e; corrector: S V e + dS_aff dV_aff e - sigma mu e),
// r_a = r_i + V^{-1} r_c (eq. augmented), r_nu = -r_a + C w with
// w = [I 0] K0^{-1} [-r_g; r_e] (eq. ineq-const-reduced in K0 form), D = S V^{-1}.
__global__ void ipm_rhs_kernel(int m2, int corrector, const double* __restrict__ ri, const double* __restrict__ s,
                               const double* __restrict__ nu, const double* __restrict__ Cw,
                               const double* __restrict__ dsa, const double* __restrict__ dna,
                               const IpmScalars* __restrict__ isc, double* __restrict__ rc, double* __restrict__ rhs,
                               double* __restrict__ dvec) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m2) return;
  double si = s[i], ni = nu[i];
  double r = si * ni;
  if (corrector) r += dsa[i] * dna[i] - isc->sigma * isc->mu;
  rc[i] = r;
  rhs[i] = -(ri[i] + r / ni) + Cw[i];
  dvec[i] = si / ni;
}

hipError_t ipm_rhs(hipStream_t st, int m2, int corrector, const double* ri, const double* s, const double* nu,
                   const double* Cw, const double* dsa, const double* dna, const IpmScalars* isc, double* rc,
                   double* rhs, double* dvec) {
  hipLaunchKernelGGL(ipm_rhs_kernel, dim3((m2 + 255) / 256), dim3(256), 0, st, m2, corrector, ri, s, nu, Cw, dsa, dna,
                     isc, rc, rhs, dvec);
  return hipGetLastError();
}

__global__ void neg_copy_kernel(int m, const double* __restrict__ src, double* __restrict__ dst) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) dst[i] = -src[i];
}

hipError_t ipm_neg_copy(hipStream_t st, int m, const double* src, double* dst) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(neg_copy_kernel, dim3((m + 255) / 256), dim3(256), 0, st, m, src, dst);
  return hipGetLastError();
}

// sol = K0^{-1} [r_g + C^T dnu; -r_e] = [dx; -dlam]  (eq. schur-delta-x in K0 form),
// ds = -V^{-1} r_c - D dnu (eq. delz).
__global__ void ipm_dirs_kernel(int n, int m1, int m2, const double* __restrict__ sol, const double* __restrict__ rc,
                                const double* __restrict__ nu, const double* __restrict__ dvec,
                                const double* __restrict__ dnu, double* __restrict__ dx, double* __restrict__ dlam,
                                double* __restrict__ ds) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dx[i] = sol[i];
  if (i < m1) dlam[i] = -sol[n + i];
  if (i < m2) ds[i] = -rc[i] / nu[i] - dvec[i] * dnu[i];
}

hipError_t ipm_dirs(hipStream_t st, int n, int m1, int m2, const double* sol, const double* rc, const double* nu,
                    const double* dvec, const double* dnu, double* dx, double* dlam, double* ds) {
  int m = n > m2 ? n : m2;
  hipLaunchKernelGGL(ipm_dirs_kernel, dim3((m + 255) / 256), dim3(256), 0, st, n, m1, m2, sol, rc, nu, dvec, dnu, dx,
                     dlam, ds);
  return hipGetLastError();
}

// Largest alpha with v + alpha dv >= 0 (INFINITY when no component decreases).
__device__ __forceinline__ double ratio(double v, double dv) { return dv < 0.0 ? -v / dv : INFINITY; }

// Predictor: alpha_aff, mu_aff, sigma = (mu_aff / mu)^3.
// Corrector: alpha = min(1, tau alpha_max) and the update of (x, lam, nu, s).
__device__ __forceinline__ void ipm_step_body(int n, int m1, int m2, int corrector, double* __restrict__ x,
                                              double* __restrict__ lam, double* __restrict__ nu,
                                              double* __restrict__ s, const double* __restrict__ dx,
                                              const double* __restrict__ dlam, const double* __restrict__ dnu,
                                              const double* __restrict__ ds, IpmScalars* __restrict__ isc) {
  __shared__ double sh[16];
  __shared__ double alpha_s;
  double amax = INFINITY, snu = 0;
  for (int i = threadIdx.x; i < m2; i += blockDim.x) {
    amax = fmin(amax, fmin(ratio(s[i], ds[i]), ratio(nu[i], dnu[i])));
    snu += s[i] * nu[i];
  }
  amax = -block_max(-amax, sh);
  snu = block_sum(snu, sh);
  if (!corrector) {
    double a = fmin(1.0, amax);
    double acc = 0;
    for (int i = threadIdx.x; i < m2; i += blockDim.x) acc += (s[i] + a * ds[i]) * (nu[i] + a * dnu[i]);
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) {
      double mu = snu / m2;
      double mua = acc / m2;
      double ratio_mu = mua / mu;
      isc->mu = mu;
      isc->alpha_aff = a;
      isc->mu_aff = mua;
      isc->sigma = ratio_mu * ratio_mu * ratio_mu;
    }
    return;
  }
  if (threadIdx.x == 0) {
    double a = fmin(1.0, isc->tau * amax);
    isc->alpha_max = amax;
    isc->alpha = a;
    alpha_s = a;
  }
  __syncthreads();
  const double a = alpha_s;
  for (int i = threadIdx.x; i < n; i += blockDim.x) x[i] += a * dx[i];
  for (int i = threadIdx.x; i < m1; i += blockDim.x) lam[i] += a * dlam[i];
  for (int i = threadIdx.x; i < m2; i += blockDim.x) {
    nu[i] += a * dnu[i];
    s[i] += a * ds[i];
  }
}

__global__ void __launch_bounds__(kRedThreads) ipm_step_kernel(int n, int m1, int m2, int corrector,
                                                               double* __restrict__ x, double* __restrict__ lam,
                                                               double* __restrict__ nu, double* __restrict__ s,
                                                               const double* __restrict__ dx,
                                                               const double* __restrict__ dlam,
                                                               const double* __restrict__ dnu,
                                                               const double* __restrict__ ds,
                                                               IpmScalars* __restrict__ isc) {
  ipm_step_body(n, m1, m2, corrector, x, lam, nu, s, dx, dlam, dnu, ds, isc);
}

hipError_t ipm_step(hipStream_t st, int n, int m1, int m2, int corrector, double* x, double* lam, double* nu,
                    double* s, const double* dx, const double* dlam, const double* dnu, const double* ds,
                    IpmScalars* isc) {
  hipLaunchKernelGGL(ipm_step_kernel, dim3(1), dim3(kRedThreads), 0, st, n, m1, m2, corrector, x, lam, nu, s, dx, dlam,
                     dnu, ds, isc);
  return hipGetLastError();
}

// Initial point: sol = K0^{-1} [-c; b] = [x0; -lam0]; s0 = max(C x0 - d, 1); nu0 = 1.
__global__ void ipm_init_kernel(int n, int m1, int m2, const double* __restrict__ sol, const double* __restrict__ Cx,
                                const double* __restrict__ d, double* __restrict__ x, double* __restrict__ lam,
                                double* __restrict__ nu, double* __restrict__ s) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = sol[i];
  if (i < m1) lam[i] = -sol[n + i];
  if (i < m2) {
    s[i] = fmax(Cx[i] - d[i], 1.0);
    nu[i] = 1.0;
  }
}

hipError_t ipm_init_point(hipStream_t st, int n, int m1, int m2, const double* sol, const double* Cx,
                          const double* d, double* x, double* lam, double* nu, double* s) {
  int m = n > m2 ? n : m2;
  hipLaunchKernelGGL(ipm_init_kernel, dim3((m + 255) / 256), dim3(256), 0, st, n, m1, m2, sol, Cx, d, x, lam, nu, s);
  return hipGetLastError();
}

// P = T + D on the lower triangle (the P_H matrix of eq. preconditioner-2).
__global__ void add_diag_copy_kernel(int m, const double* __restrict__ T, int ldt, const double* __restrict__ dvec,
                                     double* __restrict__ P, int ldp) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  int i = blockIdx.y;
  if (i >= m || j > i) return;
  double v = T[(size_t)i * ldt + j];
  if (i == j) v += dvec[i];
  P[(size_t)i * ldp + j] = v;
}

hipError_t add_diag_copy(hipStream_t st, int m, const double* T, int ldt, const double* dvec, double* P, int ldp) {
  if (m > 65535) return hipErrorInvalidValue;
  dim3 grid((m + 255) / 256, m);
  hipLaunchKernelGGL(add_diag_copy_kernel, grid, dim3(256), 0, st, m, T, ldt, dvec, P, ldp);
  return hipGetLastError();
}


__global__ void ew_mul_kernel(int m, const double* __restrict__ a, const double* __restrict__ b,
                              double* __restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) out[i] = a[i] * b[i];
}

hipError_t ew_mul(hipStream_t st, int m, const double* a, const double* b, double* out) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(ew_mul_kernel, dim3((m + 255) / 256), dim3(256), 0, st, m, a, b, out);
  return hipGetLastError();
}

// dnu += dx32 (iterative refinement accumulates the float32 correction in float64).
__global__ void ir_accumulate_kernel(int m, const float* __restrict__ fx, double* __restrict__ x) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) x[i] += (double)fx[i];
}

__global__ void vec_add_kernel(int m, const double* __restrict__ a, double* __restrict__ y) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) y[i] += a[i];
}

hipError_t vec_add(hipStream_t st, int m, const double* a, double* y) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(vec_add_kernel, dim3((m + 255) / 256), dim3(256), 0, st, m, a, y);
  return hipGetLastError();
}

hipError_t ir_accumulate(hipStream_t st, int m, const float* fx, double* x) {
  hipLaunchKernelGGL(ir_accumulate_kernel, dim3((m + 255) / 256), dim3(256), 0, st, m, fx, x);
  return hipGetLastError();
}

// r = rhs - Kx in float64 with ||r||^2, ||rhs||^2 and max |w_i r_i| into sc.
__device__ __forceinline__ void ir_residual_body(int m, const double* __restrict__ rhs, const double* __restrict__ Kx,
                                                 const double* __restrict__ w, double* __restrict__ r,
                                                 PcgScalars* __restrict__ sc) {
  __shared__ double sh[16];
  double rr = 0, bb = 0, wm = 0;
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    double ri = rhs[i] - Kx[i];
    r[i] = ri;
    rr += ri * ri;
    bb += rhs[i] * rhs[i];
    if (w) wm = fmax(wm, fabs(w[i] * ri));
  }
  rr = block_sum(rr, sh);
  bb = block_sum(bb, sh);
  wm = block_max(wm, sh);
  if (threadIdx.x == 0) {
    sc->rr = rr;
    sc->bb = bb;
    sc->wmax = wm;
  }
}

__global__ void __launch_bounds__(kRedThreads) ir_residual_kernel(int m, const double* __restrict__ rhs,
                                                                  const double* __restrict__ Kx,
                                                                  const double* __restrict__ w,
                                                                  double* __restrict__ r,
                                                                  PcgScalars* __restrict__ sc) {
  ir_residual_body(m, rhs, Kx, w, r, sc);
}

hipError_t ir_residual(hipStream_t st, int m, const double* rhs, const double* Kx, const double* w, double* r,
                       PcgScalars* sc) {
  hipLaunchKernelGGL(ir_residual_kernel, dim3(1), dim3(kRedThreads), 0, st, m, rhs, Kx, w, r, sc);
  return hipGetLastError();
}

// ---- batched forms (one workgroup of kRedThreads per QP) ---------------------------
// The reductions call the bodies above with the same block size, so a QP's
// statistics, step lengths and refinement residuals are computed in the same
// order whether it runs alone or in a batch; element-wise steps are exact.
#define QPG_BENTRY const IpmDesc& q = tab[list[blockIdx.x]]

__global__ void __launch_bounds__(kRedThreads) bipm_stats_kernel(const IpmDesc* __restrict__ tab,
                                                                 const int* __restrict__ list) {
  QPG_BENTRY;
  ipm_stats_body(q.n, q.m1, q.m2, q.Hx, q.Atl, q.Ctn, q.Ax, q.Cx, q.x, q.c, q.lam, q.b, q.nu, q.s, q.d, q.rg, q.re,
                 q.ri, q.stats);
}

// vN1 = [-r_g; r_e] (rhs), vN1[n:] = -r_e (recover; top half written by the C^T sweep),
// vN1 = [-c; b] (initial point).
__global__ void __launch_bounds__(kRedThreads) bipm_pack_kernel(const IpmDesc* __restrict__ tab,
                                                                const int* __restrict__ list, int mode) {
  QPG_BENTRY;
  if (mode != kPackRecover)
    for (int i = threadIdx.x; i < q.n; i += blockDim.x) q.vN1[i] = mode == kPackRhs ? -q.rg[i] : -q.c[i];
  for (int i = threadIdx.x; i < q.m1; i += blockDim.x)
    q.vN1[q.n + i] = mode == kPackRhs ? q.re[i] : (mode == kPackRecover ? -q.re[i] : q.b[i]);
}

__global__ void __launch_bounds__(kRedThreads) bipm_rhs_kernel(const IpmDesc* __restrict__ tab,
                                                               const int* __restrict__ list, int corrector) {
  QPG_BENTRY;
  const IpmScalars* isc = q.isc;
  for (int i = threadIdx.x; i < q.m2; i += blockDim.x) {
    double si = q.s[i], ni = q.nu[i];
    double r = si * ni;
    if (corrector) r += q.ds_a[i] * q.dnu_a[i] - isc->sigma * isc->mu;
    q.rc[i] = r;
    q.rhs[i] = -(q.ri[i] + r / ni) + q.Cw[i];
    q.dvec[i] = si / ni;
  }
}

__global__ void __launch_bounds__(kRedThreads) bipm_dirs_kernel(const IpmDesc* __restrict__ tab,
                                                                const int* __restrict__ list, int which) {
  QPG_BENTRY;
  double* dx = which ? q.dx : q.dx_a;
  double* dlam = which ? q.dlam : q.dlam_a;
  double* ds = which ? q.ds : q.ds_a;
  const double* dnu = which ? q.dnu : q.dnu_a;
  for (int i = threadIdx.x; i < q.n; i += blockDim.x) dx[i] = q.vN2[i];
  for (int i = threadIdx.x; i < q.m1; i += blockDim.x) dlam[i] = -q.vN2[q.n + i];
  for (int i = threadIdx.x; i < q.m2; i += blockDim.x) ds[i] = -q.rc[i] / q.nu[i] - q.dvec[i] * dnu[i];
}

__global__ void __launch_bounds__(kRedThreads) bipm_step_kernel(const IpmDesc* __restrict__ tab,
                                                                const int* __restrict__ list, int corrector) {
  QPG_BENTRY;
  if (corrector)
    ipm_step_body(q.n, q.m1, q.m2, 1, q.x, q.lam, q.nu, q.s, q.dx, q.dlam, q.dnu, q.ds, q.isc);
  else
    ipm_step_body(q.n, q.m1, q.m2, 0, q.x, q.lam, q.nu, q.s, q.dx_a, q.dlam_a, q.dnu_a, q.ds_a, q.isc);
}

// Initial point from vN2 = K0^{-1} [-c; b] and Cx = C x0; IPM scalars reset with tau.
__global__ void __launch_bounds__(kRedThreads) bipm_init_kernel(const IpmDesc* __restrict__ tab,
                                                                const int* __restrict__ list, double tau) {
  QPG_BENTRY;
  for (int i = threadIdx.x; i < q.n; i += blockDim.x) q.x[i] = q.vN2[i];
  for (int i = threadIdx.x; i < q.m1; i += blockDim.x) q.lam[i] = -q.vN2[q.n + i];
  for (int i = threadIdx.x; i < q.m2; i += blockDim.x) {
    q.s[i] = fmax(q.Cx[i] - q.d[i], 1.0);
    q.nu[i] = 1.0;
  }
  if (threadIdx.x == 0) {
    IpmScalars z{};
    z.tau = tau;
    *q.isc = z;
  }
}

__global__ void __launch_bounds__(kRedThreads) bir_begin_kernel(const IpmDesc* __restrict__ tab,
                                                                const int* __restrict__ list, int which) {
  QPG_BENTRY;
  double* dnu = which ? q.dnu : q.dnu_a;
  for (int i = threadIdx.x; i < q.m2; i += blockDim.x) {
    q.fd[i] = (float)q.dvec[i];
    q.fwts[i] = (float)q.nu[i];
    dnu[i] = 0.0;
    q.ir_r[i] = q.rhs[i];
  }
}

__global__ void __launch_bounds__(kRedThreads) bir_prep_kernel(const IpmDesc* __restrict__ tab,
                                                               const int* __restrict__ list) {
  QPG_BENTRY;
  for (int i = threadIdx.x; i < q.m2; i += blockDim.x) q.fb[i] = (float)q.ir_r[i];
}

__global__ void __launch_bounds__(kRedThreads) bir_acc_kernel(const IpmDesc* __restrict__ tab,
                                                              const int* __restrict__ list, int which) {
  QPG_BENTRY;
  double* dnu = which ? q.dnu : q.dnu_a;
  for (int i = threadIdx.x; i < q.m2; i += blockDim.x) {
    const double v = dnu[i] + (double)q.fx[i];
    dnu[i] = v;
    q.pt[i] = q.dvec[i] * v;
  }
}

__global__ void __launch_bounds__(kRedThreads) bir_residual_kernel(const IpmDesc* __restrict__ tab,
                                                                   const int* __restrict__ list, int which) {
  QPG_BENTRY;
  (void)which;
  ir_residual_body(q.m2, q.rhs, q.ir_x, q.nu, q.ir_r, q.sc);
}

__global__ void __launch_bounds__(kRedThreads) bir_fb_add_kernel(const IpmDesc* __restrict__ tab,
                                                                 const int* __restrict__ list, int which) {
  QPG_BENTRY;
  double* dnu = which ? q.dnu : q.dnu_a;
  for (int i = threadIdx.x; i < q.m2; i += blockDim.x) dnu[i] += q.ir_d[i];
}

__global__ void bmat2d_kernel(const Mat2dDesc* __restrict__ descs) {
  const Mat2dDesc m = descs[blockIdx.z];
  const int i = blockIdx.y;
  if (i >= m.rows) return;
  const int jend = m.lower ? min(i + 1, m.cols) : m.cols;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < jend; j += gridDim.x * blockDim.x) {
    double v = m.src[(size_t)i * m.lds + j];
    if (m.diag && i == j) v += m.diag[i];
    if (m.to_float)
      static_cast<float*>(m.dst)[(size_t)i * m.ldd + j] = (float)v;
    else
      static_cast<double*>(m.dst)[(size_t)i * m.ldd + j] = v;
  }
}

#define QPG_BLAUNCH(kern, ...)                                                                              \
  do {                                                                                                      \
    if (count <= 0) return hipSuccess;                                                                      \
    hipLaunchKernelGGL(kern, dim3(count), dim3(kRedThreads), 0, st, tab, list, ##__VA_ARGS__);             \
    return hipGetLastError();                                                                               \
  } while (0)

hipError_t bipm_stats(hipStream_t st, const IpmDesc* tab, const int* list, int count) {
  QPG_BLAUNCH(bipm_stats_kernel);
}
hipError_t bipm_pack(hipStream_t st, const IpmDesc* tab, const int* list, int count, int mode) {
  QPG_BLAUNCH(bipm_pack_kernel, mode);
}
hipError_t bipm_rhs(hipStream_t st, const IpmDesc* tab, const int* list, int count, int corrector) {
  QPG_BLAUNCH(bipm_rhs_kernel, corrector);
}
hipError_t bipm_dirs(hipStream_t st, const IpmDesc* tab, const int* list, int count, int which) {
  QPG_BLAUNCH(bipm_dirs_kernel, which);
}
hipError_t bipm_step(hipStream_t st, const IpmDesc* tab, const int* list, int count, int corrector) {
  QPG_BLAUNCH(bipm_step_kernel, corrector);
}
hipError_t bipm_init(hipStream_t st, const IpmDesc* tab, const int* list, int count, double tau) {
  QPG_BLAUNCH(bipm_init_kernel, tau);
}
hipError_t bir_begin(hipStream_t st, const IpmDesc* tab, const int* list, int count, int which) {
  QPG_BLAUNCH(bir_begin_kernel, which);
}
hipError_t bir_prep(hipStream_t st, const IpmDesc* tab, const int* list, int count) {
  QPG_BLAUNCH(bir_prep_kernel);
}
hipError_t bir_acc(hipStream_t st, const IpmDesc* tab, const int* list, int count, int which) {
  QPG_BLAUNCH(bir_acc_kernel, which);
}
hipError_t bir_residual(hipStream_t st, const IpmDesc* tab, const int* list, int count, int which) {
  QPG_BLAUNCH(bir_residual_kernel, which);
}
hipError_t bir_fb_add(hipStream_t st, const IpmDesc* tab, const int* list, int count, int which) {
  QPG_BLAUNCH(bir_fb_add_kernel, which);
}

hipError_t bmat2d(hipStream_t st, const Mat2dDesc* d, int count, int max_rows, int max_cols) {
  if (count <= 0 || max_rows <= 0 || max_cols <= 0) return hipSuccess;
  if (max_rows > 65535 || count > 65535) return hipErrorInvalidValue;
  const int gx = std::min((max_cols + 255) / 256, 16);
  hipLaunchKernelGGL(bmat2d_kernel, dim3(gx, max_rows, count), dim3(256), 0, st, d);
  return hipGetLastError();
}

// Once-per-QP matrix passes over C: kMatIdentity sets *flag to 1 when C != I
// (an entry differs from the identity's; the flag starts at 0), kMatColScale
// writes dst = C diag(H)^{-1/2} for the diagonal form of P_H.
__device__ __forceinline__ void matop_body(const MatOpDesc& d, int i0, int di, int j0, int dj) {
  bool bad = false;
  for (int i = i0; i < d.rows; i += di) {
    const double* row = d.src + (size_t)i * d.lds;
    for (int j = j0; j < d.cols; j += dj) {
      const double v = row[j];
      if (d.op == kMatIdentity) {
        bad |= v != (i == j ? 1.0 : 0.0);
      } else {
        d.dst[(size_t)i * d.ldd + j] = v / sqrt(d.h[(size_t)j * d.ldh + j]);
      }
    }
  }
  if (bad) *d.flag = 1;  // every writer stores the same value
}

__global__ void __launch_bounds__(256) matop_kernel(MatOpDesc d) {
  matop_body(d, blockIdx.y, gridDim.y, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

__global__ void __launch_bounds__(256) bmatop_kernel(const MatOpDesc* __restrict__ descs) {
  const MatOpDesc d = descs[blockIdx.z];
  matop_body(d, blockIdx.y, gridDim.y, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

static dim3 matop_grid(int rows, int cols, int count) {
  return dim3(std::min((cols + 255) / 256, 16), std::min(rows, 4096), count);
}

hipError_t matop(hipStream_t st, const MatOpDesc& d) {
  if (d.rows <= 0 || d.cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(matop_kernel, matop_grid(d.rows, d.cols, 1), dim3(256), 0, st, d);
  return hipGetLastError();
}

hipError_t bmatop(hipStream_t st, const MatOpDesc* d, int count, int max_rows, int max_cols) {
  if (count <= 0 || max_rows <= 0 || max_cols <= 0) return hipSuccess;
  if (count > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(bmatop_kernel, matop_grid(max_rows, max_cols, count), dim3(256), 0, st, d);
  return hipGetLastError();
}

template <typename S, typename D>
__global__ void convert_2d_kernel(const S* __restrict__ src, int lds, D* __restrict__ dst, int ldd, int rows,
                                  int cols) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  int i = blockIdx.y;
  if (i < rows && j < cols) dst[(size_t)i * ldd + j] = (D)src[(size_t)i * lds + j];
}

template <typename S, typename D>
hipError_t convert_2d(hipStream_t st, const S* src, int lds, D* dst, int ldd, int rows, int cols) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  if (rows > 65535) return hipErrorInvalidValue;
  dim3 grid((cols + 255) / 256, rows);
  hipLaunchKernelGGL((convert_2d_kernel<S, D>), grid, dim3(256), 0, st, src, lds, dst, ldd, rows, cols);
  return hipGetLastError();
}

template <typename S, typename D>
__global__ void convert_1d_kernel(const S* __restrict__ src, D* __restrict__ dst, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (D)src[i];
}

template <typename S, typename D>
hipError_t convert_1d(hipStream_t st, const S* src, D* dst, int n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((convert_1d_kernel<S, D>), dim3((n + 255) / 256), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

template <typename T>
__global__ void fill_vec_kernel(int n, T v, T* __restrict__ x) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

template <typename T>
hipError_t fill_vec(hipStream_t st, int n, T v, T* x) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_vec_kernel<T>, dim3((n + 255) / 256), dim3(256), 0, st, n, v, x);
  return hipGetLastError();
}
template hipError_t fill_vec<double>(hipStream_t, int, double, double*);
template hipError_t fill_vec<float>(hipStream_t, int, float, float*);

template hipError_t convert_2d<double, float>(hipStream_t, const double*, int, float*, int, int, int);
template hipError_t convert_2d<double, double>(hipStream_t, const double*, int, double*, int, int, int);
template hipError_t convert_1d<double, float>(hipStream_t, const double*, float*, int);
template hipError_t convert_1d<float, double>(hipStream_t, const float*, double*, int);

}  // namespace qpg
