// Launchers of the fused CG-step kernels (pcg.hip) and the IPM vector kernels
// (ipm.hip).  Internal to the library.
#pragma once
#include "common.hpp"
#include "desc.hpp"

namespace qpg {

enum PrecMode : int { kPrecNone = 0, kPrecL = 1, kPrecH = 2 };

template <typename T>
hipError_t pcg_init(hipStream_t st, int m2, const T* b, const T* dvec, const T* wts, T* x, T* r, T* z, T* p, int prec,
                    double rtol, double wtol, int maxit, PcgScalars* sc);
template <typename T>
int pcg_q_grid(int m2);
// q = C w + D p and the per-workgroup partials of p^T q; C null means C = I (m2 = n).
template <typename T>
hipError_t pcg_q(hipStream_t st, const T* C, int ldc, int m2, int n, const T* w, const T* dvec, const T* p, T* q,
                 const PcgScalars* sc, double* bpart, int bpart_cap, const EventPair* ev = nullptr, int stage = 1);
template <typename T>
hipError_t pcg_update(hipStream_t st, int m2, const double* bpart, const T* dvec, T* p, const T* q, T* x, T* r, T* z,
                      const T* wts, int prec, PcgScalars* sc);
template <typename T>
hipError_t pcg_ph_update(hipStream_t st, int m2, const T* r, const T* z, T* p, int init, PcgScalars* sc);
// ---- CG step with the vector update folded into the operator sweeps ------------
// The step's kernels: fold_ct (u = C^T z + beta C^T p_old, and the stop test and
// beta of the previous update from its partials), the one-pass K0 product and the
// sum of its partials with the partials of p^T q = u^T w + p^T D p, then fold_q
// (q = C w + D p, p = z + beta p_old, alpha, dnu, r, z and the partials of the
// next test); with P_H the one-pass X_P apply and its sum with the partials of
// r^T z.  fold_test closes a chunk of steps so the host sees a stop at once.
struct FoldParts {
  double* al;  // partials of p^T q (u^T w + p^T D p), one per workgroup of the K0 sum
  int nal;
  double* rz;  // partials of r^T z (q sweep, or the sum of the P_H apply)
  int nrz;
  double *rr, *wm;  // partials of ||r||^2 and max |w r| (q sweep)
  int nrw;
};
template <typename T>
hipError_t fold_ct(hipStream_t st, const T* CT, int ldct, int n, int m2, const T* z, const T* p, T* u,
                   PcgScalars* sc, const FoldParts& fp, const EventPair* ev);
template <typename T>
hipError_t fold_q(hipStream_t st, const T* C, int ldc, int m2, int n, const T* w, const T* dvec, T* p, T* q, T* x,
                  T* r, T* z, const T* wts, int prec, PcgScalars* sc, const FoldParts& fp, const EventPair* ev);
hipError_t fold_test(hipStream_t st, PcgScalars* sc, const FoldParts& fp);

// batched forms: descriptor list in device memory, one solve per entry
int bpcg_q_blocks(int m2);
template <typename T>
hipError_t bpcg_init(hipStream_t st, const PcgDesc<T>* d, int ndesc);
template <typename T>
hipError_t bpcg_q(hipStream_t st, const PcgDesc<T>* d, const int* prefix, int ndesc, int total_blocks, size_t smem,
                  const EventPair* ev = nullptr);
template <typename T>
hipError_t bpcg_update(hipStream_t st, const PcgDesc<T>* d, int ndesc);
template <typename T>
hipError_t bpcg_ph_update(hipStream_t st, const PcgDesc<T>* d, int ndesc, int init);

// ---- IPM (ipm.hip) -------------------------------------------------------
// Scalars of one IPM iteration, resident in device memory.
struct IpmScalars {
  double mu;        // s^T nu / m2 at the current iterate
  double sigma;     // centering parameter from the predictor
  double alpha_aff;
  double mu_aff;
  double alpha;     // step taken
  double alpha_max;
  double tau;
  double pad;
};

// Stats of the current iterate used for the relative KKT score.
enum StatIdx : int {
  kRdInf = 0, kHxInf, kCInf, kAtlInf, kCtnInf,   // dual residual and its terms
  kReInf, kAxInf, kBInf,                         // equality residual
  kViolInf, kDInf,                               // inequality violation max(d - Cx, 0)
  kXHx, kCx, kBl, kDn,                           // objective pieces
  kNuMin, kNuInf, kSNu, kRiInf, kSMin,
  kNumStats
};

// Per-QP record of the batched IPM kernels: every vector of one QP's interior
// point state (fixed for the QP's lifetime).  A batched launch takes the table
// and a list of entries; workgroup b serves entry list[b].
struct IpmDesc {
  int n, m1, m2, pad;
  const double *c, *b, *d;
  double *x, *lam, *nu, *s;
  double *Hx, *Atl, *Ctn, *Ax, *Cx, *rg, *re, *ri, *stats;
  double *dvec, *rc, *rhs, *Cw, *vN1, *vN2;
  double *dx, *dlam, *dnu, *ds, *dx_a, *dlam_a, *dnu_a, *ds_a;
  double *ir_r, *ir_x, *ir_d, *pt;
  float *fd, *fwts, *fb, *fx;
  IpmScalars* isc;
  PcgScalars* sc;
};

// dst = (D)(src + diag on the diagonal) over rows x cols (lower: j <= i only).
struct Mat2dDesc {
  const double* src;
  void* dst;
  const double* diag;
  int lds, ldd, rows, cols, lower, to_float;
};

// Once-per-QP passes over C (ipm.hip): identity test and diag(H)^{-1/2} column scaling.
enum MatOp : int { kMatIdentity = 0, kMatColScale = 1 };
struct MatOpDesc {
  const double* src;  // C (rows x cols, leading dimension lds)
  const double* h;    // H (kMatColScale)
  double* dst;        // C diag(H)^{-1/2} (kMatColScale)
  int* flag;          // set to 1 when C != I (kMatIdentity)
  int lds, ldh, ldd, rows, cols, op;
};
hipError_t matop(hipStream_t st, const MatOpDesc& d);
hipError_t bmatop(hipStream_t st, const MatOpDesc* d, int count, int max_rows, int max_cols);

hipError_t ipm_stats(hipStream_t st, int n, int m1, int m2, const double* Hx, const double* Atl, const double* Ctn,
                     const double* Ax, const double* Cx, const double* x, const double* c, const double* lam,
                     const double* b, const double* nu, const double* s, const double* d, double* rg, double* re,
                     double* ri, double* stats);
hipError_t ipm_rhs(hipStream_t st, int m2, int corrector, const double* ri, const double* s, const double* nu,
                   const double* Cw, const double* dsa, const double* dna, const IpmScalars* isc, double* rc,
                   double* rhs, double* dvec);
hipError_t ipm_neg_copy(hipStream_t st, int m, const double* src, double* dst);
hipError_t ipm_dirs(hipStream_t st, int n, int m1, int m2, const double* sol, const double* rc, const double* nu,
                    const double* dvec, const double* dnu, double* dx, double* dlam, double* ds);
hipError_t ipm_step(hipStream_t st, int n, int m1, int m2, int corrector, double* x, double* lam, double* nu,
                    double* s, const double* dx, const double* dlam, const double* dnu, const double* ds,
                    IpmScalars* isc);
hipError_t ipm_init_point(hipStream_t st, int n, int m1, int m2, const double* sol, const double* Cx,
                          const double* d, double* x, double* lam, double* nu, double* s);
hipError_t ew_mul(hipStream_t st, int m, const double* a, const double* b, double* out);
hipError_t ir_accumulate(hipStream_t st, int m, const float* fx, double* x);
hipError_t vec_add(hipStream_t st, int m, const double* a, double* y);
hipError_t ir_residual(hipStream_t st, int m, const double* rhs, const double* Kx, const double* w, double* r,
                       PcgScalars* sc);
hipError_t add_diag_copy(hipStream_t st, int m, const double* T, int ldt, const double* dvec, double* P, int ldp);
// Batched IPM steps over `count` entries of an IpmDesc table (list: entry
// indices in device memory).  `which` selects the predictor (0) or corrector
// (1) vectors where both exist.
enum PackMode : int { kPackRhs = 0, kPackRecover = 1, kPackInit = 2 };
hipError_t bipm_stats(hipStream_t st, const IpmDesc* tab, const int* list, int count);
hipError_t bipm_pack(hipStream_t st, const IpmDesc* tab, const int* list, int count, int mode);
hipError_t bipm_rhs(hipStream_t st, const IpmDesc* tab, const int* list, int count, int corrector);
hipError_t bipm_dirs(hipStream_t st, const IpmDesc* tab, const int* list, int count, int which);
hipError_t bipm_step(hipStream_t st, const IpmDesc* tab, const int* list, int count, int corrector);
hipError_t bipm_init(hipStream_t st, const IpmDesc* tab, const int* list, int count, double tau);
// mixed refinement: begin (fd, fwts, dnu = 0, ir_r = rhs), fb = ir_r, dnu += fx
// with pt = D dnu, residual into sc, dnu += ir_d
hipError_t bir_begin(hipStream_t st, const IpmDesc* tab, const int* list, int count, int which);
hipError_t bir_prep(hipStream_t st, const IpmDesc* tab, const int* list, int count);
hipError_t bir_acc(hipStream_t st, const IpmDesc* tab, const int* list, int count, int which);
hipError_t bir_residual(hipStream_t st, const IpmDesc* tab, const int* list, int count, int which);
hipError_t bir_fb_add(hipStream_t st, const IpmDesc* tab, const int* list, int count, int which);
hipError_t bmat2d(hipStream_t st, const Mat2dDesc* d, int count, int max_rows, int max_cols);
template <typename T>
hipError_t fill_vec(hipStream_t st, int n, T v, T* x);
template <typename S, typename D>
hipError_t convert_2d(hipStream_t st, const S* src, int lds, D* dst, int ldd, int rows, int cols);
template <typename S, typename D>
hipError_t convert_1d(hipStream_t st, const S* src, D* dst, int n);

}  // namespace qpg
