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

}  // namespace
}  // namespace qpg

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
