// Arguments and fused per-value loads and stores shared by the DFT pass
// kernels (the three-pass path of kernels_fft.hip and the two-pass 256^3 path
// of kernels_fft4.hip).
#pragma once
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "fft_radix.h"
#include "os3d_internal.h"

namespace os3d {

constexpr int kMaxBatch = 64;    // orientation pairs per launch

enum LoadMode { LM_REAL = 0, LM_C = 1, LM_MULBANK = 2, LM_UIN = 3, LM_DIVM = 4 };
enum StoreMode { SM_C = 0, SM_UOUT = 1, SM_ACCUM = 2, SM_REAL = 3, SM_PHI = 4 };

struct PassArgs {
  int axis;  // 0 = z, 1 = y, 2 = x
  int Nz, Ny, Nx;
  long long V;
  int N, nst;
  int radix[kMaxStages];
  int W, LS;            // lines per tile, LDS line stride (float2)
  long long lines;      // V / N
  const float2* tw;     // exp(-2 pi i j / N)
  float sgn;            // -1: forward DFT, +1: inverse DFT
  int nb;               // pairs in this launch
  // sources
  const float* src_r;
  const float2* src_c;
  long long src_stride;  // per pair (elements)
  const float* psi;      // bank rows (without kappa)
  float kappa;           // the bank's normaliser: LM_MULBANK multiplies by kappa psi, LM_DIVM by kappa
  int rows[kMaxBatch];
  int oa[kMaxBatch], ob[kMaxBatch];  // stored member, partner (-1 if none)
  const void* U;
  int dtype;
  const float* scales;   // [N_o] of this volume
  const float* M;
  float eps;
  int divide;
  // destinations
  float2* dst_c;
  long long dst_stride;
  float* dst_r;
  void* Uout;
  float out_scale;
  float* partial;        // [nb][tiles] sums of |value| (scale bound), or null
  const float* tsc;      // 256^3 fp16 intermediates: scales of the writing workgroups [nb][1024]
  float* tsc_out;        // where the writing pass puts them
  int accumulate;        // SM_ACCUM: 1 adds to X, 0 overwrites
  int phi_kind;          // SM_PHI: 0 identity, 1 |U|^phi_p sgn(U)
  float phi_p;
};

__device__ __forceinline__ long long gaddr(const PassArgs& a, long long line, int n) {
  if (a.axis == 2) return line * a.Nx + n;
  if (a.axis == 1) {
    long long z = line / a.Nx, x = line - z * a.Nx;
    return (z * a.Ny + n) * a.Nx + x;
  }
  return (long long)n * a.Ny * a.Nx + line;
}

__device__ __forceinline__ int lidx(int LS, int w, int n) { return w * LS + n + (n >> 4); }

// Non-temporal loads for values a pass streams through once (a plain read
// kernel reaches 6.3 TB/s on this GPU, 7.0 TB/s with the hint).  Measured per
// kernel: they speed up the bank-row and intermediate reads of the
// orientation-sum passes and the z-line and plane passes, and slow down the
// other 256^3 passes, which keep plain loads.
typedef float nt_float2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 ldnt(const float2* p) {
  const nt_float2 v = __builtin_nontemporal_load((const nt_float2*)p);
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ float ldnt(const float* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ unsigned int ldnt(const unsigned int* p) { return __builtin_nontemporal_load(p); }

__device__ __forceinline__ unsigned int bf16_rne(float x) {
  unsigned int u = __float_as_uint(x);
  unsigned int lsb = (u >> 16) & 1u;
  return (u + 0x7fffu + lsb) >> 16;
}

// Score element i as complex float (16-bit pairs times their scale s).  The
// storage type is a template parameter so that the loads of a pass are not
// separated by branches and can all be in flight together.
// A stored 16-bit pair times its scale s.
template <int DT>
__device__ __forceinline__ float2 score_value(unsigned int q, float s) {
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

template <int DT>
__device__ __forceinline__ float2 load_score(const void* U, long long i, float s) {
  if constexpr (DT == OS3D_C64)
    return ((const float2*)U)[i];
  else
    return score_value<DT>(((const unsigned int*)U)[i], s);
}


template <int DT>
__device__ __forceinline__ void store_score(void* U, long long i, float2 v, float inv_s) {
  if constexpr (DT == OS3D_C64) {
    ((float2*)U)[i] = v;
  } else {
    const float re = v.x * inv_s, im = v.y * inv_s;
    unsigned int q;
    if constexpr (DT == OS3D_F16X2)
      q = (unsigned int)__half_as_ushort(__float2half_rn(re)) |
          ((unsigned int)__half_as_ushort(__float2half_rn(im)) << 16);
    else
      q = bf16_rne(re) | (bf16_rne(im) << 16);
    ((unsigned int*)U)[i] = q;
  }
}

// Fused first-pass load of element g (line position) for pair slot j.
template <int LM, int DT = OS3D_C64>
__device__ __forceinline__ float2 load_elem(const PassArgs& a, int j, long long g, float& asum) {
  if constexpr (LM == LM_REAL) {
    return make_float2(a.src_r[g], 0.f);
  } else if constexpr (LM == LM_C) {
    return a.src_c[j * a.src_stride + g];
  } else if constexpr (LM == LM_MULBANK) {
    const float p = a.psi[(long long)a.rows[j] * a.V + g] * a.kappa;
    const float2 v = cscale(a.src_c[g], p);
    if (a.partial) asum += sqrtf(v.x * v.x + v.y * v.y);  // scale bound of 16-bit storage only
    return v;
  } else if constexpr (LM == LM_UIN) {
    const int ia = a.oa[j], ib = a.ob[j];
    const float sa = a.scales ? a.scales[ia] : 1.f;
    float2 v = load_score<DT>(a.U, (long long)ia * a.V + g, sa);
    if (ib >= 0) {
      const float sb = a.scales ? a.scales[ib] : 1.f;
      v = cadd(v, cconj(load_score<DT>(a.U, (long long)ib * a.V + g, sb)));
    }
    return v;
  } else {  // LM_DIVM
    const float2 v = a.src_c[g];
    return cscale(v, a.divide ? a.kappa / fmaxf(a.M[g], a.eps) : a.kappa);
  }
}

// Phi of processing via scores applied to one transformed value v (times
// out_scale = 1/V), times 2 for a stored antipodal pair: for real f the pair
// contributes Phi(U_n) + conj(Phi(U_-n)) = 2 Phi(U_n) to the reconstruction.
// |U|^(p-1) = 2^((p-1)/2 log2 |U|^2) with the hardware base-2 logarithm
// and exponential (about 1 ulp each; powf costs ~170 instructions).  The
// hardware logarithm flushes denormal inputs to zero, so a score whose
// components are both below 2^-60 is scaled by 2^96 before it is squared
// (every such |U|^2, down to the smallest denormal component, is then a
// normal number) and log2 |U|^2 is corrected by -192.
__device__ __forceinline__ float2 phi_apply(const PassArgs& a, int j, float2 v) {
  const float2 u = cscale(v, a.out_scale);
  const float mult = (a.ob[j] >= 0) ? 2.f : 1.f;
  if (a.phi_kind == 1) {
    const bool tiny = fmaxf(fabsf(u.x), fabsf(u.y)) < 0x1p-60f;
    const float2 w = tiny ? cscale(u, 0x1p96f) : u;
    const float l2 = __builtin_amdgcn_logf(w.x * w.x + w.y * w.y) - (tiny ? 192.f : 0.f);
    const float f = __builtin_amdgcn_exp2f(0.5f * (a.phi_p - 1.f) * l2);
    return cscale(u, (u.x != 0.f || u.y != 0.f) ? mult * f : 0.f);
  }
  return cscale(u, mult);
}

// Fused last-pass store of element g for pair slot j (SM_ACCUM adds into acc).
template <int SM, int DT = OS3D_C64>
__device__ __forceinline__ void store_elem(const PassArgs& a, int j, long long g, float2 v, float2& acc) {
  if constexpr (SM == SM_C) {
    a.dst_c[j * a.dst_stride + g] = v;
  } else if constexpr (SM == SM_UOUT) {
    const float2 u = cscale(v, a.out_scale);
    const int ia = a.oa[j], ib = a.ob[j];
    const float inv_s = a.scales ? 1.f / a.scales[ia] : 1.f;
    store_score<DT>(a.Uout, (long long)ia * a.V + g, u, inv_s);
    if (ib >= 0) store_score<DT>(a.Uout, (long long)ib * a.V + g, cconj(u), inv_s);
  } else if constexpr (SM == SM_ACCUM) {
    const float p = a.psi[(long long)a.rows[j] * a.V + g];
    acc = make_float2(acc.x + p * v.x, acc.y + p * v.y);
  } else if constexpr (SM == SM_PHI) {
    a.dst_c[j * a.dst_stride + g] = phi_apply(a, j, v);
  } else {  // SM_REAL
    a.dst_r[g] = v.x * a.out_scale;
  }
}

__device__ __forceinline__ void accum_flush(const PassArgs& a, long long g, float2 acc) {
  float2 x = acc;
  if (a.accumulate) x = cadd(a.dst_c[g], x);
  a.dst_c[g] = x;
}


// K values of one thread at the affine positions g0 + r d (r < K), for pair
// slot j.  Uniform conditions (partner present, division, scales) are
// decided once, outside the unrolled loops, so that each group of loads sits
// in one basic block and is issued back to back.
template <int LM, int DT, int K>
__device__ __forceinline__ void load_k(const PassArgs& a, int j, long long g0, long long d, float2 (&v)[K],
                                       float& asum) {
  if constexpr (LM == LM_REAL) {
#pragma unroll
    for (int r = 0; r < K; ++r) v[r] = make_float2(a.src_r[g0 + r * d], 0.f);
  } else if constexpr (LM == LM_C) {
    const float2* p = a.src_c + j * a.src_stride;
#pragma unroll
    for (int r = 0; r < K; ++r) v[r] = ldnt(p + g0 + r * d);
  } else if constexpr (LM == LM_MULBANK) {
    const float* pr = a.psi + (long long)a.rows[j] * a.V;
    float ps[K];
#pragma unroll
    for (int r = 0; r < K; ++r) ps[r] = ldnt(pr + g0 + r * d);
#pragma unroll
    for (int r = 0; r < K; ++r) v[r] = a.src_c[g0 + r * d];
#pragma unroll
    for (int r = 0; r < K; ++r) v[r] = cscale(v[r], ps[r] * a.kappa);
    if (a.partial) {  // scale bound of 16-bit storage only
#pragma unroll
      for (int r = 0; r < K; ++r) asum += sqrtf(v[r].x * v[r].x + v[r].y * v[r].y);
    }
  } else if constexpr (LM == LM_UIN) {
    const int ia = a.oa[j], ib = a.ob[j];
    float sa = 1.f, sb = 1.f;
    if constexpr (DT != OS3D_C64) {
      sa = a.scales[ia];
      if (ib >= 0) sb = a.scales[ib];
    }
    const long long ba = (long long)ia * a.V + g0;
#pragma unroll
    for (int r = 0; r < K; ++r) v[r] = load_score<DT>(a.U, ba + r * d, sa);
    if (ib >= 0) {
      const long long bb = (long long)ib * a.V + g0;
      float2 w[K];
#pragma unroll
      for (int r = 0; r < K; ++r) w[r] = load_score<DT>(a.U, bb + r * d, sb);
#pragma unroll
      for (int r = 0; r < K; ++r) v[r] = cadd(v[r], cconj(w[r]));
    }
  } else {  // LM_DIVM
#pragma unroll
    for (int r = 0; r < K; ++r) v[r] = a.src_c[g0 + r * d];
    if (a.divide) {
      float m[K];
#pragma unroll
      for (int r = 0; r < K; ++r) m[r] = a.M[g0 + r * d];
#pragma unroll
      for (int r = 0; r < K; ++r) v[r] = cscale(v[r], a.kappa / fmaxf(m[r], a.eps));
    } else {
#pragma unroll
      for (int r = 0; r < K; ++r) v[r] = cscale(v[r], a.kappa);
    }
  }
}

// K values of one thread stored at g0 + r d for pair slot j; SM_ACCUM adds
// psi_hat_j * value into acc[r] instead.
template <int SM, int DT, int K>
__device__ __forceinline__ void store_k(const PassArgs& a, int j, long long g0, long long d, const float2 (&v)[K],
                                        float2 (&acc)[K]) {
  if constexpr (SM == SM_C) {
    float2* p = a.dst_c + j * a.dst_stride;
#pragma unroll
    for (int r = 0; r < K; ++r) p[g0 + r * d] = v[r];
  } else if constexpr (SM == SM_UOUT) {
    const int ia = a.oa[j], ib = a.ob[j];
    const float inv_s = (DT != OS3D_C64) ? 1.f / a.scales[ia] : 1.f;
    const long long ba = (long long)ia * a.V + g0;
#pragma unroll
    for (int r = 0; r < K; ++r) store_score<DT>(a.Uout, ba + r * d, cscale(v[r], a.out_scale), inv_s);
    if (ib >= 0) {
      const long long bb = (long long)ib * a.V + g0;
#pragma unroll
      for (int r = 0; r < K; ++r) store_score<DT>(a.Uout, bb + r * d, cconj(cscale(v[r], a.out_scale)), inv_s);
    }
  } else if constexpr (SM == SM_ACCUM) {
    const float* pr = a.psi + (long long)a.rows[j] * a.V;
    float ps[K];
#pragma unroll
    for (int r = 0; r < K; ++r) ps[r] = ldnt(pr + g0 + r * d);
#pragma unroll
    for (int r = 0; r < K; ++r) acc[r] = make_float2(acc[r].x + ps[r] * v[r].x, acc[r].y + ps[r] * v[r].y);
  } else if constexpr (SM == SM_PHI) {
    // the reconstruction's input for the pair (phi_apply)
    float2* p = a.dst_c + j * a.dst_stride;
#pragma unroll
    for (int r = 0; r < K; ++r) p[g0 + r * d] = phi_apply(a, j, v[r]);
  } else {  // SM_REAL
#pragma unroll
    for (int r = 0; r < K; ++r) a.dst_r[g0 + r * d] = v[r].x * a.out_scale;
  }
}

// X (+)= acc at g0 + r d, the read of X (when adding) issued as one group.
template <int K>
__device__ __forceinline__ void flush_k(const PassArgs& a, long long g0, long long d, const float2 (&acc)[K]) {
  if (a.accumulate) {
    float2 x[K];
#pragma unroll
    for (int r = 0; r < K; ++r) x[r] = a.dst_c[g0 + r * d];
#pragma unroll
    for (int r = 0; r < K; ++r) a.dst_c[g0 + r * d] = cadd(x[r], acc[r]);
  } else {
#pragma unroll
    for (int r = 0; r < K; ++r) a.dst_c[g0 + r * d] = acc[r];
  }
}

// Per-kernel timer slots (os3d_profile_*): first / middle / last pass of the
// DFT of f, of the forward transform, of the reconstruction's orientation
// sum and of its final inverse DFT.
enum ProfKernel {
  kProfDftFirst = 0, kProfDftMid, kProfDftLast, kProfFwdFirst, kProfScales, kProfFwdMid, kProfFwdLast,
  kProfRecFirst, kProfRecMid, kProfRecLast, kProfInvFirst, kProfInvMid, kProfInvLast, kProfBank, kProfCount
};

void launch_scales(const float* partial, int ntiles, const PassArgs& a, int dtype, float* scales, int nb,
                   hipStream_t st);
int forward4(const os3d_bank* b, const float* f, int batch, void* U, int dtype, float* scales, void* ws, int nbmax,
             void* stream);
int reduce4(const os3d_bank* b, const void* U, int dtype, const float* scales, int batch, float* f_out, void* ws,
            bool divide_M, int nbmax, void* stream);
template <int LM, int SM>
void launch_plane(const PassArgs& a, int grid_y, hipStream_t st);
void launch_plane_phi(const PassArgs& a, int grid_y, hipStream_t st);
int process4(const os3d_bank* b, const float* f, int batch, int phi_kind, float phi_p, float* f_out, void* ws,
             int nbmax, void* stream);

}  // namespace os3d
