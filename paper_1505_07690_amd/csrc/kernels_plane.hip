// Two-pass 3D DFT for volumes whose (y, x) planes fit in LDS (Ny = Nx = 64
// or 128): one pass transforms z lines (the per-axis kernels of
// kernels_fft.hip, with the bank multiply or the orientation sum fused in),
// the other transforms whole planes in one workgroup, so every transform
// moves its intermediate through HBM once instead of twice.
//
// k_plane: one workgroup per (z plane, pair slot).  The plane is loaded with
// fully coalesced accesses into LDS (with the fused load of the pass), then
// the x lines and the y lines are transformed in LDS by 16 x R2 Cooley-Tukey
// steps (radix-16 over elements s + TL r, twiddles W_N^(jj r'), radix-R2),
// and the last stage stores straight to global memory with consecutive
// lanes on consecutive x (fused store of the pass).
#include <hip/hip_runtime.h>

#include "fft_pass.h"

namespace os3d {

template <int NP>
struct PlaneCfg {
  static constexpr int T = NP * NP / 16;  // threads: 16 values each
  static constexpr int TL = NP / 16;      // threads per line
  static constexpr int R2 = NP / 16;      // second-stage radix
  static constexpr int B2 = 16 / R2;      // second-stage butterflies per thread
  static constexpr int RS = NP + NP / 16 + 1;  // LDS row stride (float2)
};

__device__ __forceinline__ int ppad(int x) { return x + (x >> 4); }

template <int NP, int LM, int SM, int DT>
__global__ __launch_bounds__(PlaneCfg<NP>::T) void k_plane(PassArgs a) {
  using C = PlaneCfg<NP>;
  extern __shared__ float2 P[];  // [NP][RS]
  __shared__ float2 twl[NP];
  const int t = threadIdx.x;
  const int j = blockIdx.y;
  const long long base = (long long)blockIdx.x * NP * NP;
  for (int i = t; i < NP; i += C::T) {
    float2 w = a.tw[i];
    if (a.sgn > 0.f) w.y = -w.y;
    twl[i] = w;
  }
  // coalesced fused load of the plane: element e = t + T r
  {
    float2 v[16];
    float asum = 0.f;
    load_k<LM, DT, 16>(a, j, base + t, C::T, v, asum);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int e = t + C::T * r;
      P[(e / NP) * C::RS + ppad(e % NP)] = v[r];
    }
  }
  __syncthreads();
  // x lines: thread (row y, slot s)
  {
    const int y = t / C::TL, s = t % C::TL;
    float2* row = P + y * C::RS;
    float2 v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = row[ppad(s + C::TL * r)];
    dft16(v, a.sgn);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) row[ppad(s * 16 + r)] = v[r];
    __syncthreads();
    float2 u[C::B2][C::R2];
#pragma unroll
    for (int q = 0; q < C::B2; ++q) {
      const int jj = s + C::TL * q;
#pragma unroll
      for (int r = 0; r < C::R2; ++r) u[q][r] = row[ppad(jj + 16 * r)];
#pragma unroll
      for (int r = 1; r < C::R2; ++r) u[q][r] = cmul(u[q][r], twl[jj * r]);
      dft_r<C::R2>(u[q], a.sgn);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < C::B2; ++q)
#pragma unroll
      for (int p = 0; p < C::R2; ++p) row[ppad(s + C::TL * q + 16 * p)] = u[q][p];
  }
  __syncthreads();
  // y lines: thread (column x, slot s); the last stage stores to memory
  {
    const int x = t % NP, s = t / NP;
    float2* col = P + ppad(x);
    float2 v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = col[(s + C::TL * r) * C::RS];
    dft16(v, a.sgn);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) col[(s * 16 + r) * C::RS] = v[r];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < C::B2; ++q) {
      const int jj = s + C::TL * q;
      float2 u[C::R2];
#pragma unroll
      for (int r = 0; r < C::R2; ++r) u[r] = col[(jj + 16 * r) * C::RS];
#pragma unroll
      for (int r = 1; r < C::R2; ++r) u[r] = cmul(u[r], twl[jj * r]);
      dft_r<C::R2>(u, a.sgn);
      float2 dummy[C::R2];
      store_k<SM, DT, C::R2>(a, j, base + (long long)jj * NP + x, 16LL * NP, u, dummy);
    }
  }
}

template <int NP, int LM, int SM, int DT>
static void launch_plane_np(const PassArgs& a, int grid_y, hipStream_t st) {
  using C = PlaneCfg<NP>;
  const size_t lds = (size_t)NP * C::RS * sizeof(float2);
  static bool attr_set = false;
  if (!attr_set) {
    (void)hipFuncSetAttribute((const void*)k_plane<NP, LM, SM, DT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    attr_set = true;
  }
  hipLaunchKernelGGL((k_plane<NP, LM, SM, DT>), dim3((unsigned)a.Nz, grid_y), dim3(C::T), lds, st, a);
}

template <int LM, int SM, int DT>
static void launch_plane_dt(const PassArgs& a, int grid_y, hipStream_t st) {
  if (a.Nx == 128)
    launch_plane_np<128, LM, SM, DT>(a, grid_y, st);
  else
    launch_plane_np<64, LM, SM, DT>(a, grid_y, st);
}

template <int LM, int SM>
void launch_plane(const PassArgs& a, int grid_y, hipStream_t st) {
  if constexpr (LM == LM_UIN || SM == SM_UOUT) {
    if (a.dtype == OS3D_BF16X2) launch_plane_dt<LM, SM, OS3D_BF16X2>(a, grid_y, st);
    else if (a.dtype == OS3D_F16X2) launch_plane_dt<LM, SM, OS3D_F16X2>(a, grid_y, st);
    else launch_plane_dt<LM, SM, OS3D_C64>(a, grid_y, st);
  } else {
    launch_plane_dt<LM, SM, OS3D_C64>(a, grid_y, st);
  }
}

template void launch_plane<LM_REAL, SM_C>(const PassArgs&, int, hipStream_t);
template void launch_plane<LM_C, SM_UOUT>(const PassArgs&, int, hipStream_t);
template void launch_plane<LM_C, SM_PHI>(const PassArgs&, int, hipStream_t);
template void launch_plane<LM_C, SM_REAL>(const PassArgs&, int, hipStream_t);
template void launch_plane<LM_UIN, SM_C>(const PassArgs&, int, hipStream_t);
template void launch_plane<LM_C, SM_C>(const PassArgs&, int, hipStream_t);

}  // namespace os3d
