// Two-pass 3D DFT for volumes whose (y, x) planes fit in LDS (Ny = Nx = 64
// or 128): one pass transforms z lines (the per-axis kernels of
// kernels_fft.hip, with the bank multiply or the orientation sum fused in),
// the other transforms whole planes in one workgroup, so every transform
// moves its intermediate through HBM once instead of twice.
//
// k_plane: a workgroup loops over (pair slot, z plane) tasks, prefetching the
// next task's values while it transforms the current plane.  The plane is
// loaded with fully coalesced accesses into LDS (fused load of the pass), then
// the x lines and the y lines are transformed in LDS by 16 x R2 Cooley-Tukey
// steps (radix-16 over elements s + TL r, twiddles W_N^(jj r'), radix-R2),
// and the last stage stores straight to global memory with consecutive
// lanes on consecutive x (fused store of the pass).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <type_traits>
#include <unordered_set>

#include "fft_pass.h"
#include "launch.h"

namespace os3d {

template <int NP>
struct PlaneCfg {
  static constexpr int T = NP * NP / 16;  // threads: 16 values each
  static constexpr int TL = NP / 16;      // threads per line
  static constexpr int R2 = NP / 16;      // second-stage radix
  static constexpr int B2 = 16 / R2;      // second-stage butterflies per thread
  // LDS row stride (float2): 8 (NP = 128) or 16 (NP = 64) rows of a wave
  // start on distinct bank groups, so the row stages run at the minimum two
  // passes per wave-wide access
  static constexpr int RS = NP + NP / 16;
};

__device__ __forceinline__ int ppad(int x) { return x + (x >> 4); }

// The 16 values a thread loads for one plane, issued as raw loads and
// turned into complex values later, so that the loads of the next plane
// are in flight while the current one is transformed.  Buffer loads: one
// VGPR offset per thread (the element's byte offset in its volume, < 2^32
// for these shapes) and the value index in a scalar offset, so the 16 or 32
// loads in flight hold no per-load address registers.
constexpr int kBufDword3 = 0x00020000;  // raw 32-bit records, no format conversion
constexpr int kNT = 2;                  // cache policy: non-temporal (streamed once)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t volume_rsrc(const void* base, long long bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kBufDword3);
}

template <int LM, int DT>
struct PlaneIn;

template <int DT>
struct PlaneIn<LM_C, DT> {
  float2 r[16];
  __device__ __forceinline__ void issue(const PassArgs& a, int j, long long e0, int T) {
    const auto rs = volume_rsrc(a.src_c + j * a.src_stride, a.V * 8);
    const int vo = (int)(e0 * 8);
#pragma unroll
    for (int i = 0; i < 16; ++i)
      r[i] = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rs, vo, i * T * 8, kNT));
  }
  __device__ __forceinline__ void issue2(const PassArgs&, int, long long, int) {}
  __device__ __forceinline__ void get(const PassArgs&, int, float2 (&v)[16]) const {
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = r[i];
  }
};

template <int DT>
struct PlaneIn<LM_REAL, DT> {
  float r[16];
  __device__ __forceinline__ void issue(const PassArgs& a, int, long long e0, int T) {
    const auto rs = volume_rsrc(a.src_r, a.V * 4);
    const int vo = (int)(e0 * 4);
#pragma unroll
    for (int i = 0; i < 16; ++i)
      r[i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, vo, i * T * 4, kNT));
  }
  __device__ __forceinline__ void issue2(const PassArgs&, int, long long, int) {}
  __device__ __forceinline__ void get(const PassArgs&, int, float2 (&v)[16]) const {
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = make_float2(r[i], 0.f);
  }
};

template <int DT>
__device__ __forceinline__ float2 score_word(unsigned int q, float s) {
  float re, im;
  if constexpr (DT == OS3D_F16X2) {
    re = __half2float(__ushort_as_half((unsigned short)(q & 0xffffu)));
    im = __half2float(__ushort_as_half((unsigned short)(q >> 16)));
  } else {
    re = __uint_as_float((q & 0xffffu) << 16);
    im = __uint_as_float(q & 0xffff0000u);
  }
  return make_float2(re * s, im * s);
}

// U_n + conj(U_-n) of a stored pair (or U_n alone); 16-bit values times
// their orientation's scale.
template <int DT>
struct PlaneIn<LM_UIN, DT> {
  static constexpr int WB = (DT == OS3D_C64) ? 8 : 4;  // bytes per stored value
  using Word = typename std::conditional<DT == OS3D_C64, float2, unsigned int>::type;
  Word ra[16], rb[16];
  __device__ __forceinline__ static Word ld(__amdgpu_buffer_rsrc_t rs, int vo, int so) {
    if constexpr (DT == OS3D_C64)
      return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rs, vo, so, kNT));
    else
      return __builtin_amdgcn_raw_buffer_load_b32(rs, vo, so, kNT);
  }
  // the two members of the pair are issued at two points of the previous
  // plane's work, which keeps the registers in flight within the budget
  __device__ __forceinline__ void issue(const PassArgs& a, int j, long long e0, int T) {
    const char* U = (const char*)a.U;
    const int ia = a.oa[j];
    const auto rsa = volume_rsrc(U + (long long)ia * a.V * WB, a.V * WB);
#pragma unroll
    for (int i = 0; i < 16; ++i) ra[i] = ld(rsa, (int)(e0 * WB), i * T * WB);
  }
  __device__ __forceinline__ void issue2(const PassArgs& a, int j, long long e0, int T) {
    const char* U = (const char*)a.U;
    const int ib = a.ob[j];
    if (ib >= 0) {
      const auto rsb = volume_rsrc(U + (long long)ib * a.V * WB, a.V * WB);
#pragma unroll
      for (int i = 0; i < 16; ++i) rb[i] = ld(rsb, (int)(e0 * WB), i * T * WB);
    }
  }
  __device__ __forceinline__ static float2 val(Word w, float s) {
    if constexpr (DT == OS3D_C64)
      return w;
    else
      return score_word<DT>(w, s);
  }
  __device__ __forceinline__ void get(const PassArgs& a, int j, float2 (&v)[16]) const {
    const int ia = a.oa[j], ib = a.ob[j];
    float sa = 1.f, sb = 1.f;
    if constexpr (DT != OS3D_C64) {
      sa = a.scales[ia];
      if (ib >= 0) sb = a.scales[ib];
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = val(ra[i], sa);
    if (ib >= 0) {
#pragma unroll
      for (int i = 0; i < 16; ++i) v[i] = cadd(v[i], cconj(val(rb[i], sb)));
    }
  }
};

// x lines of the plane in LDS, in place: thread (row y, slot s).  The
// caller synchronises before and after.
template <int NP, bool INV>
__device__ __forceinline__ void plane_rows(float2* P, const float2* twl, int t) {
  using C = PlaneCfg<NP>;
  constexpr float sg = INV ? 1.f : -1.f;
  const int y = t / C::TL, s = t % C::TL;
  float2* row = P + y * C::RS;
  float2 v[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = row[ppad(s + C::TL * r)];
  dft16(v, sg);
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 16; ++r) row[ppad(s * 16 + r)] = v[r];
  __syncthreads();
  // butterfly (s, q) reads and writes only the positions jj + 16 r of the
  // row, jj = s + TL q, and jj is unique to (s, q): in place, no barrier
#pragma unroll
  for (int q = 0; q < C::B2; ++q) {
    const int jj = s + C::TL * q;
    float2 u[C::R2];
#pragma unroll
    for (int r = 0; r < C::R2; ++r) u[r] = row[ppad(jj + 16 * r)];
#pragma unroll
    for (int r = 1; r < C::R2; ++r) u[r] = cmul(u[r], INV ? cconj(twl[jj * r]) : twl[jj * r]);
    dft_r<C::R2>(u, sg);
#pragma unroll
    for (int p = 0; p < C::R2; ++p) row[ppad(jj + 16 * p)] = u[p];
  }
}

// y lines: thread (column x, slot s).  mid() runs between the first stage's
// write-back and its barrier; the second stage hands the outputs y = jj + 16 p
// of butterfly (s, q) to sink(jj, x, u) (in place into LDS is safe: jj is
// unique to (s, q)).
template <int NP, bool INV, class Mid, class Sink>
__device__ __forceinline__ void plane_cols(float2* P, const float2* twl, int t, Mid mid, Sink sink) {
  using C = PlaneCfg<NP>;
  constexpr float sg = INV ? 1.f : -1.f;
  const int x = t % NP, s = t / NP;
  float2* col = P + ppad(x);
  float2 v[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = col[(s + C::TL * r) * C::RS];
  dft16(v, sg);
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 16; ++r) col[(s * 16 + r) * C::RS] = v[r];
  mid();
  __syncthreads();
#pragma unroll
  for (int q = 0; q < C::B2; ++q) {
    const int jj = s + C::TL * q;
    float2 u[C::R2];
#pragma unroll
    for (int r = 0; r < C::R2; ++r) u[r] = col[(jj + 16 * r) * C::RS];
#pragma unroll
    for (int r = 1; r < C::R2; ++r) u[r] = cmul(u[r], INV ? cconj(twl[jj * r]) : twl[jj * r]);
    dft_r<C::R2>(u, sg);
    sink(jj, x, u);
  }
}

// The thread's 16 coalesced values (element e = t + T r of the plane) into LDS.
template <int NP>
__device__ __forceinline__ void plane_put(float2* P, int t, const float2 (&v)[16]) {
  using C = PlaneCfg<NP>;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int e = t + C::T * r;
    P[(e / NP) * C::RS + ppad(e % NP)] = v[r];
  }
}

// Persistent over tasks (pair slot j, z plane): task = j * Nz + z, strided
// by the grid; the loads of task + gridDim.x are issued before the current
// plane's LDS stages and stores.  INV: inverse DFT (+1 exponent).
template <int NP, int LM, int SM, int DT, bool INV>
__global__ __launch_bounds__(PlaneCfg<NP>::T) void k_plane(PassArgs a) {
  using C = PlaneCfg<NP>;
  extern __shared__ float2 P[];  // [NP][RS]
  __shared__ float2 twl[NP];     // exp(-2 pi i m / NP)
  const int t = threadIdx.x;
  const int ntask = a.Nz * a.nb;
  for (int i = t; i < NP; i += C::T) twl[i] = a.tw[i];
  // a pair of complex64 128^2 planes in flight (64 VGPRs) does not fit next
  // to the transform's registers: that pass loads its plane when it starts it
  constexpr bool kPrefetch = !(LM == LM_UIN && DT == OS3D_C64 && NP == 128);
  PlaneIn<LM, DT> in;
  int task = blockIdx.x;
  if (kPrefetch && task < ntask) {
    in.issue(a, task / a.Nz, (long long)(task % a.Nz) * NP * NP + t, C::T);
    in.issue2(a, task / a.Nz, (long long)(task % a.Nz) * NP * NP + t, C::T);
  }
  for (; task < ntask; task += gridDim.x) {
    const int j = task / a.Nz;
    const long long base = (long long)(task % a.Nz) * NP * NP;
    if (!kPrefetch) {
      in.issue(a, j, base + t, C::T);
      in.issue2(a, j, base + t, C::T);
    }
    {
      float2 v[16];
      in.get(a, j, v);
      plane_put<NP>(P, t, v);
    }
    const int next = task + gridDim.x;
    if (kPrefetch && next < ntask) in.issue(a, next / a.Nz, (long long)(next % a.Nz) * NP * NP + t, C::T);
    __syncthreads();
    plane_rows<NP, INV>(P, twl, t);
    __syncthreads();
    plane_cols<NP, INV>(
        P, twl, t,
        [&]() {
          if (kPrefetch && next < ntask) in.issue2(a, next / a.Nz, (long long)(next % a.Nz) * NP * NP + t, C::T);
        },
        [&](int jj, int x, const float2 (&u)[C::R2]) {
          float2 dummy[C::R2];
          store_k<SM, DT, C::R2>(a, j, base + (long long)jj * NP + x, 16LL * NP, u, dummy);
        });
    __syncthreads();  // the plane buffer is rewritten by the next task
  }
}

// Processing via scores on the plane path, both directions in one kernel:
// the z-inverse-transformed plane of pair slot j (src) -> inverse plane DFT
// -> Phi on the scores -> forward plane DFT -> back to the same place
// (in place: a task owns its plane).  The scores never reach memory.
template <int NP>
__global__ __launch_bounds__(PlaneCfg<NP>::T) void k_plane_phi(PassArgs a) {
  using C = PlaneCfg<NP>;
  extern __shared__ float2 P[];
  __shared__ float2 twl[NP];
  const int t = threadIdx.x;
  const int ntask = a.Nz * a.nb;
  for (int i = t; i < NP; i += C::T) twl[i] = a.tw[i];
  // the 128^2 variant needs its registers for Phi: it loads each plane when it starts it
  constexpr bool kPrefetch = NP != 128;
  PlaneIn<LM_C, OS3D_C64> in;
  int task = blockIdx.x;
  if (kPrefetch && task < ntask) in.issue(a, task / a.Nz, (long long)(task % a.Nz) * NP * NP + t, C::T);
  for (; task < ntask; task += gridDim.x) {
    const int j = task / a.Nz;
    const long long base = (long long)(task % a.Nz) * NP * NP;
    if (!kPrefetch) in.issue(a, j, base + t, C::T);
    {
      float2 v[16];
      in.get(a, j, v);
      plane_put<NP>(P, t, v);
    }
    const int next = task + gridDim.x;
    if (kPrefetch && next < ntask) in.issue(a, next / a.Nz, (long long)(next % a.Nz) * NP * NP + t, C::T);
    __syncthreads();
    plane_rows<NP, true>(P, twl, t);
    __syncthreads();
    plane_cols<NP, true>(
        P, twl, t, []() {},
        [&](int jj, int x, const float2 (&u)[C::R2]) {
#pragma unroll
          for (int p = 0; p < C::R2; ++p) P[(jj + 16 * p) * C::RS + ppad(x)] = phi_apply(a, j, u[p]);
        });
    __syncthreads();
    plane_rows<NP, false>(P, twl, t);
    __syncthreads();
    plane_cols<NP, false>(
        P, twl, t, []() {},
        [&](int jj, int x, const float2 (&u)[C::R2]) {
          float2* d = a.dst_c + j * a.dst_stride + base + (long long)jj * NP + x;
#pragma unroll
          for (int p = 0; p < C::R2; ++p) d[(long long)p * 16 * NP] = u[p];
        });
    __syncthreads();
  }
}

static int cu_count() {
  static int n = 0;
  if (n == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
      n = 256;
  }
  return n;
}

// Raises the dynamic-LDS limit of each plane kernel once.
static void reserve_lds(const void* kernel, size_t lds) {
  static std::mutex mu;
  static std::unordered_set<const void*> done;
  std::lock_guard<std::mutex> lock(mu);
  if (done.insert(kernel).second)
    (void)hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <class K>
static void launch_persistent(K kernel, int NP, long long ntask, size_t lds, int threads, const PassArgs& a,
                              hipStream_t st) {
  reserve_lds((const void*)kernel, lds);
  // one workgroup per CU for 128^2 planes (LDS), four for 64^2; each loops over its tasks
  const int per_cu = (NP == 128) ? 1 : 4;
  const unsigned grid = (unsigned)std::min<long long>(ntask, (long long)cu_count() * per_cu);
  launch_k(kernel, dim3(grid), dim3(threads), lds, st, a);
}

template <int NP, int LM, int SM, int DT>
static void launch_plane_np(const PassArgs& a, int grid_y, hipStream_t st) {
  using C = PlaneCfg<NP>;
  const size_t lds = (size_t)NP * C::RS * sizeof(float2);
  const long long ntask = (long long)a.Nz * grid_y;
  if (a.sgn > 0.f)
    launch_persistent(k_plane<NP, LM, SM, DT, true>, NP, ntask, lds, C::T, a, st);
  else
    launch_persistent(k_plane<NP, LM, SM, DT, false>, NP, ntask, lds, C::T, a, st);
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

void launch_plane_phi(const PassArgs& a, int grid_y, hipStream_t st) {
  const long long ntask = (long long)a.Nz * grid_y;
  if (a.Nx == 128)
    launch_persistent(k_plane_phi<128>, 128, ntask, (size_t)128 * PlaneCfg<128>::RS * sizeof(float2),
                      PlaneCfg<128>::T, a, st);
  else
    launch_persistent(k_plane_phi<64>, 64, ntask, (size_t)64 * PlaneCfg<64>::RS * sizeof(float2),
                      PlaneCfg<64>::T, a, st);
}

template void launch_plane<LM_REAL, SM_C>(const PassArgs&, int, hipStream_t);
template void launch_plane<LM_C, SM_UOUT>(const PassArgs&, int, hipStream_t);
template void launch_plane<LM_C, SM_REAL>(const PassArgs&, int, hipStream_t);
template void launch_plane<LM_UIN, SM_C>(const PassArgs&, int, hipStream_t);

}  // namespace os3d
