// qp_factor_K0_static: the once-per-QP factorization of qp_factor_K0 with its
// set-up scratch taken from a fixed device array instead of hipMalloc, for
// callers that cannot allocate device memory.
//
// The array below is a file-scope device variable of this translation unit.  Its
// name denotes a host-side stand-in in host code; the device address of the copy
// held on each GPU comes from hipGetSymbolAddress, looked up once per device (with
// that device current) and kept in a table.  Only that address is ever handed to
// kernels or copies.
#include <mutex>

#include "ctx.hpp"

// The set-up scratch of qp_factor_K0_static; every GPU holds its own copy until
// the process ends.
static __device__ __align__(256) unsigned char scratch[QPGPU_STATIC_SCRATCH_BYTES];

namespace qpg {
namespace {

constexpr size_t kStaticScratchBytes = QPGPU_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

struct StaticScratch {
  std::mutex lock;      // held for a whole call: one user of a device's array at a time
  char* ptr = nullptr;  // device address of this device's copy (null until looked up)
};
StaticScratch g_dev[kMaxDevices];

// Device address of `scratch` on device dev (current).  Called with g_dev[dev].lock held.
hipError_t scratch_address(int dev, char** out) {
  StaticScratch& s = g_dev[dev];
  if (!s.ptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    s.ptr = static_cast<char*>(p);
  }
  *out = s.ptr;
  return hipSuccess;
}

// Makes `dev` current for the scope and restores the caller's device.
class DeviceScope {
 public:
  explicit DeviceScope(int dev) {
    if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
    err_ = (prev_ == dev) ? hipSuccess : hipSetDevice(dev);
  }
  ~DeviceScope() {
    if (prev_ >= 0 && err_ == hipSuccess) (void)hipSetDevice(prev_);
  }
  hipError_t err() const { return err_; }

 private:
  int prev_ = -1;
  hipError_t err_ = hipSuccess;
};

}  // namespace
}  // namespace qpg

using namespace qpg;
using namespace qpg::detail;

extern "C" {

qp_status qp_factor_K0_static(qp_ctx* ctx) {
  if (!ctx) return QP_E_INVALID;
  ctx->err.clear();
  if (ctx->dev < 0 || ctx->dev >= kMaxDevices) {
    set_err(ctx, "qp_factor_K0_static: device %d outside the %d the library tracks", ctx->dev, kMaxDevices);
    return QP_E_INVALID;
  }
  if (ctx->pooled || ctx->master) {
    set_err(ctx, "qp_factor_K0_static: batch and shared-matrix member contexts factor through their owner");
    return QP_E_STATE;
  }
  const size_t need = factor_scratch_bytes(ctx);
  if (need > kStaticScratchBytes) {
    set_err(ctx, "qp_factor_K0_static: the factorization of n=%d, m1=%d, m2=%d needs %zu bytes of scratch, "
            "more than the static %zu",
            ctx->n, ctx->m1, ctx->m2, need, kStaticScratchBytes);
    return QP_E_INVALID;
  }
  DeviceScope ds(ctx->dev);
  if (ds.err() != hipSuccess) {
    set_err(ctx, "hipSetDevice(%d) failed: %s", ctx->dev, hipGetErrorString(ds.err()));
    return QP_E_DEVICE;
  }
  std::lock_guard<std::mutex> g(g_dev[ctx->dev].lock);
  char* base = nullptr;
  const hipError_t e = scratch_address(ctx->dev, &base);
  if (e != hipSuccess) {
    set_err(ctx, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    return QP_E_DEVICE;
  }
  // Every scratch buffer of the factorization is written before it is read, so
  // what an earlier call left in the array needs no clearing.
  place_factor_scratch(ctx, base);
  const qp_status st = guarded(ctx, [&] {
    ctx->factored = false;
    ctx->ph_ready = false;
    factor(ctx);
    if (resolve_prec(ctx, ctx->opt.prec) == QP_PREC_FEW_EQ) ph_setup(ctx);
    sync(ctx);
  });
  if (st != QP_OK) (void)hipStreamSynchronize(ctx->stream);  // no launch may still read the array
  forget_factor_scratch(ctx);
  return st;
}

}  // extern "C"
