// Fixed device scratch of the allocation-free entry point
// (dg_block_smooth_noalloc): a file-scope device array that every GPU the
// library runs on holds from the loading of this code object until the
// process ends.  Host code never passes the array's name to a kernel (in
// host code it only names a host-side stand-in); it looks up the array's
// device address once per device with hipGetSymbolAddress, with that
// device current, and hands that address to the kernels as their scratch
// pointer.
#include <hip/hip_runtime.h>

#include <mutex>

#include "dg_internal.h"

namespace dgmg {

// 128 MiB: the ping-pong vector of a 32 M-DOF FP32 problem (or a 16 M-DOF
// FP64 one) plus the per-cell iteration counts
constexpr size_t kScratchBytes = size_t(128) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

size_t scratch_capacity() { return kScratchBytes; }

// Device address of `scratch` on `device`, which must be the current
// device; looked up on the first call per device and kept.
int scratch_device_ptr(int device, void **out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) {
    set_error("scratch: device index out of range");
    return DG_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) {
      set_error("hipGetSymbolAddress(scratch) returned NULL");
      return DG_EDEVICE;
    }
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return DG_OK;
}

}  // namespace dgmg
