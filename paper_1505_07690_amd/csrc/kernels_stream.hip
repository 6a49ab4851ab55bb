// Plain streaming kernels for measuring the HBM rates a copy, a read and a
// write reach on this GPU (measurement support, not a method step): the
// practical ceilings the transform's passes compare with.
#include <hip/hip_runtime.h>

#include <string>

#include "os3d_internal.h"

namespace os3d {

constexpr int kStreamThreads = 512;
constexpr int kStreamBlocks = 2048;  // 8 workgroups per CU

typedef float nt_float4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kStreamThreads) void k_stream_copy(const float4* __restrict__ src,
                                                                float4* __restrict__ dst, long long n) {
  const long long stride = (long long)gridDim.x * kStreamThreads;
  for (long long i = (long long)blockIdx.x * kStreamThreads + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// Sum of the buffer per workgroup into part[blockIdx.x] (keeps the loads live).
template <bool NT>
__global__ __launch_bounds__(kStreamThreads) void k_stream_read(const float4* __restrict__ src, long long n,
                                                                float* __restrict__ part) {
  __shared__ float red[kStreamThreads / 64];
  const long long stride = (long long)gridDim.x * kStreamThreads;
  float s = 0.f;
  for (long long i = (long long)blockIdx.x * kStreamThreads + threadIdx.x; i < n; i += stride) {
    float4 v;
    if constexpr (NT) {
      const nt_float4 w = __builtin_nontemporal_load((const nt_float4*)(src + i));
      v = make_float4(w.x, w.y, w.z, w.w);
    } else {
      v = src[i];
    }
    s += (v.x + v.y) + (v.z + v.w);
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.f;
    for (int w = 0; w < kStreamThreads / 64; ++w) t += red[w];
    part[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(kStreamThreads) void k_stream_write(float4* __restrict__ dst, long long n, float value) {
  const long long stride = (long long)gridDim.x * kStreamThreads;
  const float4 v = make_float4(value, value, value, value);
  for (long long i = (long long)blockIdx.x * kStreamThreads + threadIdx.x; i < n; i += stride) dst[i] = v;
}

}  // namespace os3d

using namespace os3d;

extern "C" os3d_status os3d_stream_probe(int32_t kind, const void* src, void* dst, size_t bytes, void* stream) {
  if (kind < 0 || kind > 3) { set_error("os3d_stream_probe: kind must be 0 (copy), 1 (read), 2 (write) or 3 (read, non-temporal)"); return OS3D_EINVAL; }
  if (bytes == 0 || bytes % 16) { set_error("os3d_stream_probe: bytes must be a positive multiple of 16"); return OS3D_EINVAL; }
  if ((kind != 2 && (!src || (uintptr_t)src % 16)) || !dst || (uintptr_t)dst % 16) {
    set_error("os3d_stream_probe: buffers must be non-NULL and 16-byte aligned");
    return OS3D_EINVAL;
  }
  hipStream_t st = (hipStream_t)stream;
  const long long n = (long long)(bytes / 16);
  if (kind == 0)
    hipLaunchKernelGGL(k_stream_copy, dim3(kStreamBlocks), dim3(kStreamThreads), 0, st, (const float4*)src,
                       (float4*)dst, n);
  else if (kind == 1)
    hipLaunchKernelGGL(k_stream_read<false>, dim3(kStreamBlocks), dim3(kStreamThreads), 0, st, (const float4*)src, n,
                       (float*)dst);
  else if (kind == 3)
    hipLaunchKernelGGL(k_stream_read<true>, dim3(kStreamBlocks), dim3(kStreamThreads), 0, st, (const float4*)src, n,
                       (float*)dst);
  else
    hipLaunchKernelGGL(k_stream_write, dim3(kStreamBlocks), dim3(kStreamThreads), 0, st, (float4*)dst, n, 1.0f);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(std::string("os3d_stream_probe: ") + hipGetErrorString(e));
    return OS3D_EDEVICE;
  }
  return OS3D_OK;
}
