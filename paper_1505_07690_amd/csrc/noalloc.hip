// The stabilised reconstruction for callers that cannot allocate device
// memory: the workspace is a static device array of this library instead of
// a caller buffer.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "os3d_internal.h"

namespace os3d {

constexpr size_t kScratchBytes = (size_t)64 << 20;  // 64 MiB per device, held until the process ends
constexpr int kMaxDevices = 64;

// Never pass `scratch` itself to a kernel or a copy from host code: on the
// host it names a stand-in, not the device memory.  Host code uses the
// address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

// This device's copy of `scratch`, looked up on the first call per device.
static int scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    set_error("os3d_reconstruct_noalloc: no current device (or more than 64 devices)");
    return OS3D_EDEVICE;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error(std::string("os3d_reconstruct_noalloc: hipGetSymbolAddress(scratch) failed: ") +
                hipGetErrorString(e));
      return OS3D_EDEVICE;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return OS3D_OK;
}

}  // namespace os3d

using namespace os3d;

extern "C" os3d_status os3d_reconstruct_noalloc(const os3d_bank* b, const void* U, int32_t dtype,
                                                 const float* scales, int32_t batch, float* f_out, void* stream) {
  if (!b) { set_error("bank is NULL"); return OS3D_EINVAL; }
  if (!U || !f_out) { set_error("input or output is NULL"); return OS3D_EINVAL; }
  if (batch < 1) { set_error("batch must be >= 1"); return OS3D_EINVAL; }
  if (dtype != OS3D_C64 && dtype != OS3D_BF16X2 && dtype != OS3D_F16X2) {
    set_error("unknown score dtype");
    return OS3D_EINVAL;
  }
  if (dtype != OS3D_C64 && !scales) { set_error("scales is NULL for a 16-bit score dtype"); return OS3D_EINVAL; }
  const int nb = reduce_pair_batch(b, (long long)kScratchBytes);
  if (nb < 1) {
    set_error("os3d_reconstruct_noalloc: the reconstruction of a " + std::to_string(b->V) + "-voxel volume needs " +
              std::to_string(2 * b->V * 8) + " bytes of scratch at least; the static scratch holds " +
              std::to_string(kScratchBytes) + " bytes (use os3d_reconstruct with a workspace)");
    return OS3D_ENOMEM;
  }
  void* ws = nullptr;
  int rc = scratch_address(&ws);
  if (rc) return (os3d_status)rc;
  return (os3d_status)launch_reduce(b, U, dtype, scales, batch, f_out, ws, true, stream, nb);
}
