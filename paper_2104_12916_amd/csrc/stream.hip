// HBM read-rate probe (diagnostic, host entry point qp_hbm_read_time).
//
// Every CG-step kernel streams a matrix from HBM, so the rate a plain streaming
// read reaches on this device is the practical ceiling of those kernels (the
// published 8 TB/s is the interface peak).  The probe reads a buffer several
// times the 256 MB last-level cache with the loads the sweeps use (16-byte
// non-temporal loads, 8 in flight per lane, a grid-stride pass), and times
// back-to-back launches with HIP events.
#include <hip/hip_runtime.h>

#include "../../include/qpgpu.h"
#include "common.hpp"
#include "kernels.hpp"

namespace qpg {
namespace {

typedef double v2d_probe_t __attribute__((ext_vector_type(2)));
constexpr int kProbeBT = 256;
constexpr int kProbeInflight = 8;

__global__ void __launch_bounds__(kProbeBT) hbm_read_kernel(const v2d_probe_t* __restrict__ p, size_t n2,
                                                            double* __restrict__ out) {
  const size_t stride = (size_t)gridDim.x * kProbeBT;
  size_t i = (size_t)blockIdx.x * kProbeBT + threadIdx.x;
  double acc = 0.0;
  for (; i + (kProbeInflight - 1) * stride < n2; i += kProbeInflight * stride) {
    v2d_probe_t v[kProbeInflight];
#pragma unroll
    for (int k = 0; k < kProbeInflight; ++k) v[k] = __builtin_nontemporal_load(p + i + k * stride);
#pragma unroll
    for (int k = 0; k < kProbeInflight; ++k) acc += v[k].x + v[k].y;
  }
  for (; i < n2; i += stride) {
    const v2d_probe_t v = p[i];
    acc += v.x + v.y;
  }
  out[(size_t)blockIdx.x * kProbeBT + threadIdx.x] = acc;  // one value per thread keeps every load live
}

// Deterministic operand entries in [-0.5, 0.5) (an integer hash of the index),
// plus `shift` on the diagonal of a square n x n operand (ld columns).
__global__ void dense_fill_kernel(double* __restrict__ a, int rows, int ld, int n, double shift, unsigned seed) {
  const size_t total = (size_t)rows * ld;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / ld), j = (int)(e % ld);
    // symmetric in (i, j) so the square operand of the factorization is symmetric
    unsigned h = (unsigned)(i < j ? i : j) * 2654435761u ^ (unsigned)(i < j ? j : i) * 40503u ^ seed;
    h ^= h >> 15;
    h *= 2246822519u;
    h ^= h >> 13;
    double v = (double)(h & 0xffffff) / 16777216.0 - 0.5;
    if (i == j && i < n) v += shift;
    a[e] = v;
  }
}

}  // namespace
}  // namespace qpg

extern "C" qp_status qp_dense_time(int op, int n, int reps, double* avg_ms) {
  if (!avg_ms || reps <= 0 || n < 1 || n > 16384 || op < 0 || op > 2) return QP_E_INVALID;
  const int ld = (n + 255) / 256 * 256 + 64;
  const size_t elems = (size_t)n * ld;
  double *a = nullptr, *b = nullptr, *c = nullptr, *tmp = nullptr;
  int* info = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  qp_status st = QP_OK;
  float ms = 0.f;
  const size_t tmp_elems = qpg::chol_inv_tmp_elems(n);
  if (hipMalloc(&a, elems * sizeof(double)) != hipSuccess || hipMalloc(&b, elems * sizeof(double)) != hipSuccess ||
      hipMalloc(&c, elems * sizeof(double)) != hipSuccess ||
      hipMalloc(&tmp, tmp_elems * sizeof(double)) != hipSuccess || hipMalloc(&info, sizeof(int)) != hipSuccess) {
    st = QP_E_NOMEM;
  } else if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    st = QP_E_DEVICE;
  } else {
    const int grid = qpg::dev_info().cu_count * 4;
    hipLaunchKernelGGL(qpg::dense_fill_kernel, dim3(grid), dim3(256), 0, nullptr, a, n, ld, n, op == 2 ? n : 0.0, 1u);
    hipLaunchKernelGGL(qpg::dense_fill_kernel, dim3(grid), dim3(256), 0, nullptr, b, n, ld, n, 0.0, 2u);
    auto run = [&]() -> hipError_t {
      switch (op) {
        case 0: return qpg::gemm_f64(nullptr, 0, 1, n, n, n, 1.0, a, ld, b, ld, 0.0, c, ld, qpg::kNone);
        case 1: return qpg::gemm_f64(nullptr, 0, 1, n, n, n, 1.0, a, ld, b, ld, 0.0, c, ld, qpg::kBUpper);
        default:
          // the factorization overwrites its input: restore it from the copy in b first
          if (hipMemcpyAsync(c, b, elems * sizeof(double), hipMemcpyDeviceToDevice, nullptr) != hipSuccess)
            return hipErrorUnknown;
          return qpg::chol_inv_f64(nullptr, c, ld, a, ld, n, tmp, info, 1);
      }
    };
    if (op == 2)  // b keeps the SPD matrix, a receives the inverse factor
      hipLaunchKernelGGL(qpg::dense_fill_kernel, dim3(grid), dim3(256), 0, nullptr, b, n, ld, n, (double)n, 1u);
    bool ok = hipMemset(info, 0, sizeof(int)) == hipSuccess && run() == hipSuccess;  // warm-up
    ok = ok && hipEventRecord(e0, nullptr) == hipSuccess;
    for (int r = 0; ok && r < reps; ++r) ok = run() == hipSuccess;
    ok = ok && hipEventRecord(e1, nullptr) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
         hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
    int h_info = 0;
    if (ok && op == 2) ok = hipMemcpy(&h_info, info, sizeof(int), hipMemcpyDeviceToHost) == hipSuccess;
    if (!ok)
      st = QP_E_DEVICE;
    else if (h_info != 0)
      st = QP_E_NOT_SPD;
    else
      *avg_ms = (double)ms / reps;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  for (void* p : {(void*)a, (void*)b, (void*)c, (void*)tmp, (void*)info})
    if (p) (void)hipFree(p);
  return st;
}

extern "C" qp_status qp_hbm_read_time(size_t bytes, int wg_per_cu, int reps, double* avg_ms) {
  if (!avg_ms || reps <= 0 || bytes < 16 || bytes % 16 != 0 || wg_per_cu < 1 || wg_per_cu > 32)
    return QP_E_INVALID;
  const int grid = qpg::dev_info().cu_count * wg_per_cu;
  void* buf = nullptr;
  double* out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  qp_status st = QP_OK;
  float ms = 0.f;
  if (hipMalloc(&buf, bytes) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&out), (size_t)grid * qpg::kProbeBT * sizeof(double)) != hipSuccess) {
    st = QP_E_NOMEM;
  } else if (hipMemset(buf, 0, bytes) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
             hipEventCreate(&e1) != hipSuccess) {
    st = QP_E_DEVICE;
  } else {
    const auto* p = static_cast<const qpg::v2d_probe_t*>(buf);
    const size_t n2 = bytes / 16;
    hipLaunchKernelGGL(qpg::hbm_read_kernel, dim3(grid), dim3(qpg::kProbeBT), 0, nullptr, p, n2, out);  // warm-up
    bool ok = hipEventRecord(e0, nullptr) == hipSuccess;
    for (int r = 0; r < reps; ++r)
      hipLaunchKernelGGL(qpg::hbm_read_kernel, dim3(grid), dim3(qpg::kProbeBT), 0, nullptr, p, n2, out);
    ok = ok && hipGetLastError() == hipSuccess && hipEventRecord(e1, nullptr) == hipSuccess &&
         hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
    if (ok)
      *avg_ms = (double)ms / reps;
    else
      st = QP_E_DEVICE;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (out) (void)hipFree(out);
  if (buf) (void)hipFree(buf);
  return st;
}
