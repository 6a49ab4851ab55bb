// Plain streaming kernels for measuring the HBM rates a copy, a read and a
// write reach on this GPU (measurement support, not a method step): the
// practical ceilings the transform's passes compare with.
#include <hip/hip_runtime.h>

#include <string>

#include "os3d_internal.h"

namespace os3d {

// One-shot grids (every thread moves a fixed few 16-byte values and exits):
// on this GPU they reach higher write and copy rates than grid-stride loops
// over a fixed number of workgroups (measured 6.9 against 4.1 TB/s for a
// write of 2 GiB, 5.9 against 4.6 TB/s for a copy).
constexpr int kStreamThreads = 256;
constexpr int kStreamPer = 4;  // 16-byte values per thread

typedef float nt_float4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kStreamThreads) void k_stream_copy(const float4* __restrict__ src,
                                                                float4* __restrict__ dst, long long n) {
  const long long b = (long long)blockIdx.x * kStreamThreads * kStreamPer + threadIdx.x;
  float4 v[kStreamPer];
#pragma unroll
  for (int r = 0; r < kStreamPer; ++r)
    if (b + r * kStreamThreads < n) {
      const nt_float4 w = __builtin_nontemporal_load((const nt_float4*)(src + b + r * kStreamThreads));
      v[r] = make_float4(w.x, w.y, w.z, w.w);
    }
#pragma unroll
  for (int r = 0; r < kStreamPer; ++r)
    if (b + r * kStreamThreads < n) dst[b + r * kStreamThreads] = v[r];
}

// Per-workgroup sums into part[blockIdx.x % kParts] (keeps the loads live;
// the values written are not meaningful as a sum).
constexpr int kParts = 2048;

template <bool NT>
__global__ __launch_bounds__(kStreamThreads) void k_stream_read(const float4* __restrict__ src, long long n,
                                                                float* __restrict__ part) {
  __shared__ float red[kStreamThreads / 64];
  const long long b = (long long)blockIdx.x * kStreamThreads * kStreamPer + threadIdx.x;
  float s = 0.f;
#pragma unroll
  for (int r = 0; r < kStreamPer; ++r)
    if (b + r * kStreamThreads < n) {
      float4 v;
      if constexpr (NT) {
        const nt_float4 w = __builtin_nontemporal_load((const nt_float4*)(src + b + r * kStreamThreads));
        v = make_float4(w.x, w.y, w.z, w.w);
      } else {
        v = src[b + r * kStreamThreads];
      }
      s += (v.x + v.y) + (v.z + v.w);
    }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    float t = 0.f;
    for (int w = 0; w < kStreamThreads / 64; ++w) t += red[w];
    part[blockIdx.x % kParts] = t;
  }
}

__global__ __launch_bounds__(kStreamThreads) void k_stream_write(float4* __restrict__ dst, long long n, float value) {
  const long long b = (long long)blockIdx.x * kStreamThreads * kStreamPer + threadIdx.x;
  const float4 v = make_float4(value, value, value, value);
#pragma unroll
  for (int r = 0; r < kStreamPer; ++r)
    if (b + r * kStreamThreads < n) dst[b + r * kStreamThreads] = v;
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
  const long long per_block = (long long)kStreamThreads * kStreamPer;
  const long long blocks = (n + per_block - 1) / per_block;
  if (blocks > 0x7fffffffLL) { set_error("os3d_stream_probe: buffer too large"); return OS3D_EINVAL; }
  const dim3 grid((unsigned)blocks);
  if (kind == 0)
    hipLaunchKernelGGL(k_stream_copy, grid, dim3(kStreamThreads), 0, st, (const float4*)src, (float4*)dst, n);
  else if (kind == 1)
    hipLaunchKernelGGL(k_stream_read<false>, grid, dim3(kStreamThreads), 0, st, (const float4*)src, n, (float*)dst);
  else if (kind == 3)
    hipLaunchKernelGGL(k_stream_read<true>, grid, dim3(kStreamThreads), 0, st, (const float4*)src, n, (float*)dst);
  else
    hipLaunchKernelGGL(k_stream_write, grid, dim3(kStreamThreads), 0, st, (float4*)dst, n, 1.0f);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(std::string("os3d_stream_probe: ") + hipGetErrorString(e));
    return OS3D_EDEVICE;
  }
  return OS3D_OK;
}
