// Gauss-Newton Hessian-vector product for callers that cannot allocate device
// memory: the same kernels as mfr_hess_vec, with the workspace taken from a
// fixed device array of this file instead of a caller buffer.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/mfr.h"
#include "ctx_internal.h"

using namespace mfr;

namespace {

constexpr size_t kScratchBytes = MFR_NOALLOC_SCRATCH_BYTES;

// One copy per GPU, allocated when the code object is loaded on it and held
// until the process ends.  Host code never passes this name to a kernel or a
// copy: it stands for the host-side shadow, not the device address; the
// address comes from hipGetSymbolAddress, per device.
__device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array, looked up once per
// device (with that device current).
mfr_status scratch_address(void** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(MFR_EINVAL, "device %d outside 0..%d", dev, kMaxDevices - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p || reinterpret_cast<uintptr_t>(p) % 256 != 0)
      return fail(MFR_EHIP, "scratch array of device %d has no usable address", dev);
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return MFR_OK;
}

}  // namespace

extern "C" {

mfr_status mfr_hess_vec_noalloc(const mfr_grid* grid, void* hip_stream, const float* R, const float* T,
                                const float* u, const float* p, float* q) {
  size_t need = 0;
  MFR_TRY(mfr_workspace_size(grid, &need));
  if (need > kScratchBytes)
    return fail(MFR_ENOMEM,
                "the problem needs %zu bytes of workspace; mfr_hess_vec_noalloc has %zu (use mfr_create with a "
                "caller workspace)",
                need, kScratchBytes);
  MFR_TRY(check_ptr(R, "R"));
  MFR_TRY(check_ptr(T, "T"));
  MFR_TRY(check_ptr(u, "u"));
  MFR_TRY(check_ptr(p, "p"));
  MFR_TRY(check_ptr(q, "q"));
  if (q == u || q == p) return fail(MFR_EINVAL, "q must not alias u or p");
  void* ws = nullptr;
  MFR_TRY(scratch_address(&ws));
  // A host-side context on the stack over the scratch array: table uploads,
  // the zero-bordered template copy, the voxel-tile kernel and the node pass,
  // exactly as mfr_create / mfr_set_images / mfr_hess_vec enqueue them.  The
  // kernels take their parameters by value, so the context may end before they
  // run.  Every scratch entry the kernels read is written earlier in the same
  // call, so nothing needs clearing between calls.
  mfr_ctx c{};
  MFR_TRY(ctx_init(&c, grid, hip_stream, ws, kScratchBytes));
  MFR_TRY(mfr_set_images(&c, R, T));
  return enqueue_hess_vec(&c, u, p, q);
}

}  // extern "C"
