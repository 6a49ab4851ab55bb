// Kernel launch of libos3d.  When the per-kernel timer is on, prof_start has
// left a pair of events pending; the next launch takes them and the runtime
// stamps them with the kernel's own start and end inside the dispatch
// (hipExtLaunchKernel), so timing adds no packets between dependent kernels.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

namespace os3d {

// Takes the events prof_start left pending on this thread (false if none).
bool prof_take(hipEvent_t* e0, hipEvent_t* e1);

template <typename K, typename... Args>
inline void launch_k(K kernel, dim3 grid, dim3 block, unsigned lds, hipStream_t st, Args... args) {
  hipEvent_t e0, e1;
  if (prof_take(&e0, &e1))
    hipExtLaunchKernelGGL(kernel, grid, block, lds, st, e0, e1, 0, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, lds, st, args...);
}

}  // namespace os3d
