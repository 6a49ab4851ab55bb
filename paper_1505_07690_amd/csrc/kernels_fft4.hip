// Two-pass 3D DFT of 256^3 volumes (four-step split of the y axis).
//
// A 256^3 DFT is six radix-16 stages.  The y axis is split as
// y = n1 + 16 n2 (input) and ky = 16 k1 + k2 (output):
//   step A: 16-point DFT over n2 for each n1, then the twiddle w^(n1 k2);
//   step C: 16-point DFT over n1 for each k2.
// The natural side (real-space rows, x contiguous) does the x DFT and one
// y step; the frequency side (tiles of layout4.h) does the other y step and
// the z DFT.  Each pass reads and writes every value once, so a 3D transform
// makes one round trip of its intermediate T through memory instead of two.
//
// A workgroup is 1024 threads working on four independent sub-problems of
// 16 x 256 values (four z planes on the natural side, four kx on the
// frequency side).  Every thread holds 16 values in registers; each pass is
// three radix-16 DFTs separated by two LDS exchanges.  A workgroup of the
// writing pass and one of the reading pass share 16 values of T (128
// bytes); T groups four such runs of neighbouring reading workgroups, so
// that the writer stores runs of 512 bytes and the reader loads 128-byte
// runs that come four to a 512-byte block:
//   inverse direction (frequency -> space), written by the frequency side:
//     T[((k2 * 16 + zbh) * 16 + n1) * 4096 + kxb * 64 + zbl * 16 + zz * 4 + kxx]
//   forward direction (space -> frequency), written by the natural side:
//     T[((k2 * 16 + kbh) * 16 + n1) * 4096 + zb * 64 + kbl * 16 + zz * 4 + kxx]
// with z = 4 zb + zz, zb = 4 zbh + zbl, kx = 4 kxb + kxx, kxb = 4 kbh + kbl.
// (Measured on the writes alone: the frequency side, whose workgroups loop
// over the pairs of a launch, stores 128-byte runs at 2.9 TB/s and
// 512-byte runs at 5.4 TB/s; the reads keep the rate of whole 128 KB tiles
// when the four readers of a block run side by side, see reader_tile.)
#include <hip/hip_runtime.h>

#include <algorithm>

#include "fft_pass.h"
#include "launch.h"
#include "layout4.h"

namespace os3d {

constexpr int k4Threads = 1024;
constexpr int k4LS = 256 + 16 + 1;  // LDS line stride (float2), padded every 16
constexpr int k4Sub = 16 * k4LS + 4;  // one sub-problem: 16 lines of 256; the extra 4 values shift
                                     // successive sub-problems by 8 banks, so lanes that interleave
                                     // sub-problems hit distinct banks

__device__ __forceinline__ int pad4(int n) { return n + (n >> 4); }

// Tile of a natural-side workgroup of the inverse direction.  The four tiles
// zb = 4 zbh + zbl (zbl = 0..3) read the four 128-byte quarters of the same
// 512-byte blocks of T; workgroups are dispatched to the eight XCDs in turn
// (blockIdx mod 8), so the four go to consecutive slots of one XCD and run
// side by side (measured: 3.09 against 3.58 ms per launch of 40 pairs when
// they land on four different XCDs).
__device__ __forceinline__ int reader_tile(int b) {
  const int xcd = b & 7, i = b >> 3;
  return (((i >> 2) << 3) + xcd) * 4 + (i & 3);
}

// 16-bit intermediates.  With bf16 score storage the intermediate T of a
// pair is stored as fp16 pairs (4 instead of 8 bytes a value, the same
// element order, packed into the first half of the pair's slot), each
// writing workgroup's values with its own power-of-two scale s =
// 2^(e - 15) from a bound m <= 2^e of their components.  The natural side
// takes the largest |component| of its 16384 values; the frequency side of
// the forward direction takes the sum of |v| over its 16384 inputs, which
// bounds every value it writes (each is a sum of some of them times
// unit-modulus twiddles) and which the 16-bit scores' scale bound reduces
// anyway.  Every value is finite and those down to 2^-29 m are normal
// (about 1.4e-4 relative RMS, well below bf16 storage's
// 1.7e-3; the reconstruction's division by max(M, eps) amplifies errors
// spread into the spectrum's corners, which rules out bf16 intermediates
// and keeps fp16 scores on complex64 intermediates).  The scales, one
// float per writing workgroup and pair, follow the pairs' values in the
// intermediate buffer.  A reading workgroup gathers its 16 values per
// thread from 16 writers and looks up each one's scale.
__device__ __forceinline__ float t16_scale(float m) {
  if (!(m > 0.f)) return 1.f;
  int e;
  frexpf(m, &e);  // m <= 2^e
  return ldexpf(1.f, e - 15);
}

__device__ __forceinline__ unsigned int pack_f16(float2 v, float inv) {
  return (unsigned int)__half_as_ushort(__float2half_rn(v.x * inv)) |
         ((unsigned int)__half_as_ushort(__float2half_rn(v.y * inv)) << 16);
}

__device__ __forceinline__ float2 unpack_f16(unsigned int q, float s) {
  return make_float2(__half2float(__ushort_as_half((unsigned short)(q & 0xffffu))) * s,
                     __half2float(__ushort_as_half((unsigned short)(q >> 16))) * s);
}

// The scale of this workgroup's 16 values per thread (all threads get it).
// red: 16 floats of LDS; the caller synchronises before red is reused.
__device__ __forceinline__ float tile_scale(const float2 (&u)[16], float* red) {
  float m = 0.f;
#pragma unroll
  for (int r = 0; r < 16; ++r) m = fmaxf(m, fmaxf(fabsf(u[r].x), fabsf(u[r].y)));
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  float b = red[0];
#pragma unroll
  for (int w = 1; w < 16; ++w) b = fmaxf(b, red[w]);
  return t16_scale(b);
}

// exp(sg 2 pi i m / 256) for the direction sg of the kernel (the table holds sg = -1)
template <int SG>
__device__ __forceinline__ void load_twiddles(const PassArgs& a, float2* twl) {
  for (int i = threadIdx.x; i < 256; i += k4Threads) {
    float2 v = a.tw[i];
    if (SG > 0) v.y = -v.y;
    twl[i] = v;
  }
}

// Each kernel runs one direction: the frequency-to-space kernels the inverse
// DFT (+1), the space-to-frequency kernels the forward DFT (-1).  The sign is
// a compile-time constant so that the multiplications by +-i and +-1 of the
// radix-16 butterflies fold into operand negations.
constexpr float kInv = 1.f, kFwd = -1.f;

// Frequency side of the inverse direction: Phi tile (kxb, n1) -> T.
// The spectrum tile (F, or X / max(M, eps)) is loaded once for the pair
// batch of the launch; per pair: multiply by the bank row (the next row is
// prefetched while the current pair is transformed), z DFT (two stages),
// step A over n2 and the twiddle w^(n1 k2).  Consecutive workgroups take
// consecutive kxb, so the 128-byte runs they write into T are adjacent.
template <int LM, bool T16 = false>
__global__ __launch_bounds__(k4Threads) void k4_inv_phi(PassArgs a) {
  __shared__ float2 lds[4 * k4Sub];
  __shared__ float2 twl[256];
  __shared__ float red[16];
  const int t = threadIdx.x;
  const int kxb = blockIdx.x & 63, n1 = blockIdx.x >> 6, tile = kxb * 16 + n1;
  const int g = t & 3, s = (t >> 2) & 15, n2 = t >> 6;
  load_twiddles<1>(a, twl);
  const long long base = (long long)tile << 14;
  float2 spec[16];
  if constexpr (LM == LM_MULBANK) {  // F times the bank's normaliser, once for the launch
#pragma unroll
    for (int r = 0; r < 16; ++r) spec[r] = cscale(a.src_c[base + t + r * 1024], a.kappa);
  } else {
    float unused = 0.f;
    load_k<LM, OS3D_C64, 16>(a, 0, base + t, 1024, spec, unused);
  }
  float pnx[16];
  if constexpr (LM == LM_MULBANK) {
    const float* prow = a.psi + (long long)a.rows[0] * a.V + base + t;
#pragma unroll
    for (int r = 0; r < 16; ++r) pnx[r] = prow[r * 1024];
  }
  const int z = t >> 2, zb = z >> 2, zz = z & 3;
  static_assert(!T16 || LM == LM_MULBANK, "fp16 intermediates are scaled by the tile's bound sum");
  // the scale bound of 16-bit storage (and the fp16 intermediates' scale):
  // the sum of |v| over the tile, its wave totals passed through LDS at the
  // first exchange's barrier
  const bool bound = LM == LM_MULBANK && (T16 || a.partial != nullptr);
  for (int j = 0; j < a.nb; ++j) {
    float2 v[16];
    float wave_abs = 0.f;
    if constexpr (LM == LM_MULBANK) {
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = cscale(spec[r], pnx[r]);
      if (j + 1 < a.nb) {
        const float* prow = a.psi + (long long)a.rows[j + 1] * a.V + base + t;
#pragma unroll
        for (int r = 0; r < 16; ++r) pnx[r] = prow[r * 1024];
      }
      if (bound) {
        // the hardware square root (1 ulp) is ample for a bound that is
        // rounded up to a power of two
#pragma unroll
        for (int r = 0; r < 16; ++r) wave_abs += __builtin_amdgcn_sqrtf(v[r].x * v[r].x + v[r].y * v[r].y);
        for (int o = 32; o > 0; o >>= 1) wave_abs += __shfl_xor(wave_abs, o);
      }
    } else {
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = spec[r];
    }
    dft16(v, kInv);
    float2* S = lds + g * k4Sub + n2 * k4LS;
    // the previous pair's step-A reads (and its reads of red) are done
    if (j > 0) __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) S[pad4(s * 16 + r)] = v[r];
    if (bound && (t & 63) == 0) red[t >> 6] = wave_abs;
    __syncthreads();
    float tile_abs = 0.f;  // sum of |v| over the workgroup's tile, every thread
    if (bound) {
      tile_abs = red[0];
#pragma unroll
      for (int w = 1; w < 16; ++w) tile_abs += red[w];
      if (t == 0 && a.partial) a.partial[(long long)j * gridDim.x + blockIdx.x] = tile_abs;
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = S[pad4(s + 16 * r)];
#pragma unroll
    for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], twl[s * r]);
    dft16(v, kInv);
#pragma unroll
    for (int r = 0; r < 16; ++r) S[pad4(s + 16 * r)] = v[r];
    __syncthreads();
    float2 u[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) u[q] = lds[g * k4Sub + q * k4LS + pad4(z)];
    dft16(u, kInv);
#pragma unroll
    for (int k2 = 1; k2 < 16; ++k2) u[k2] = cmul(u[k2], twl[n1 * k2]);
    const long long o = (long long)((zb >> 2) * 16 + n1) * 4096 + kxb * 64 + (zb & 3) * 16 + zz * 4 + g;
    if constexpr (!T16) {
      float2* T = a.dst_c + (long long)j * a.dst_stride;
#pragma unroll
      for (int k2 = 0; k2 < 16; ++k2) T[(long long)k2 * (256 * 4096) + o] = u[k2];
    } else {
      // every value of the tile's T is a sum of some of its 16384 values
      // times unit-modulus twiddles, so sum |v| bounds them all: no
      // reduction of its own
      const float sT = t16_scale(tile_abs);
      unsigned int* T = (unsigned int*)a.dst_c + (long long)j * a.dst_stride;
      const float inv = 1.f / sT;  // a power of two: exact
#pragma unroll
      for (int k2 = 0; k2 < 16; ++k2) T[(long long)k2 * (256 * 4096) + o] = pack_f16(u[k2], inv);
      // at the tile index, so that a reader's 16 writers' scales are adjacent
      if (t == 0) a.tsc_out[(long long)j * gridDim.x + tile] = sT;
    }
  }
}

// Natural side of the inverse direction: T tile (k2, zb) -> rows of four z
// planes.  Step C over n1, then the x DFT (two stages), then the fused store.
// v: the thread's 16 values of the tile in T (value q from the writer n1 = q).
template <int SM, int DT>
__device__ __forceinline__ void inv_nat_tile(const PassArgs& a, float2* lds, const float2* twl, int j, int k2, int zb,
                                             float2 (&v)[16]) {
  const int t = threadIdx.x;
  dft16(v, kInv);  // over n1 -> k1
  {
    const int g = (t >> 2) & 3, kx = (t >> 4) * 4 + (t & 3);
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) lds[g * k4Sub + k1 * k4LS + pad4(kx)] = v[k1];
  }
  __syncthreads();
  const int g = t >> 8, k1 = (t >> 4) & 15, s = t & 15;
  float2* S = lds + g * k4Sub + k1 * k4LS;
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = S[pad4(s + 16 * r)];
  dft16(v, kInv);
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 16; ++r) S[pad4(s * 16 + r)] = v[r];
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = S[pad4(s + 16 * r)];
#pragma unroll
  for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], twl[s * r]);
  dft16(v, kInv);
  const long long row = ((long long)(4 * zb + g) * 256 + (16 * k1 + k2)) * 256;
  float2 dummy[16];
  store_k<SM, DT, 16>(a, j, row + s, 16, v, dummy);
}

// Offset of this thread's 16 values of tile (k2, zb) in pair slot j's T.
__device__ __forceinline__ long long inv_nat_src(const PassArgs& a, int j, int k2, int zb) {
  const int t = threadIdx.x;
  return (long long)j * a.src_stride + (long long)(k2 * 16 + (zb >> 2)) * 16 * 4096 + (t >> 4) * 64 + (zb & 3) * 16 +
         (t & 15);
}

// Scales of this thread's 16 writers (tiles (t / 16) * 16 + q of the
// frequency side), adjacent in the scale array.
__device__ __forceinline__ void inv_nat_scales(const PassArgs& a, int j, float (&sT)[16]) {
  const float4* sc = (const float4*)(a.tsc + (long long)j * 1024 + (threadIdx.x >> 4) * 16);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float4 c = sc[q];
    sT[4 * q] = c.x;
    sT[4 * q + 1] = c.y;
    sT[4 * q + 2] = c.z;
    sT[4 * q + 3] = c.w;
  }
}

template <int SM, int DT, bool T16 = false>
__global__ __launch_bounds__(k4Threads) void k4_inv_nat(PassArgs a) {
  __shared__ float2 lds[4 * k4Sub];
  __shared__ float2 twl[256];
  const int tile = reader_tile(blockIdx.x), k2 = tile >> 6, zb = tile & 63;
  const int j = blockIdx.y;
  load_twiddles<1>(a, twl);
  const long long to = inv_nat_src(a, j, k2, zb);
  float2 v[16];
  if constexpr (!T16) {
    const float2* T = a.src_c + to;
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = T[q * 4096];
  } else {
    const unsigned int* T = (const unsigned int*)a.src_c + to;
    unsigned int w[16];
    float sT[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) w[q] = T[q * 4096];
    inv_nat_scales(a, j, sT);
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = unpack_f16(w[q], sT[q]);
  }
  inv_nat_tile<SM, DT>(a, lds, twl, j, k2, zb, v);
}

// The score passes of the bf16 form (the forward's last pass here, the
// reconstruction's first pass below) are persistent: a workgroup per CU
// loops over the launch's (pair slot j, block) tasks, task = 1024 j +
// block in the order of the one-tile-per-workgroup grid, and issues the next
// task's loads before it transforms the current tile.  A workgroup holds a
// whole CU's LDS, so with one tile per workgroup each tile's load latency
// is exposed; fp16 intermediates and 16-bit scores make a tile half the
// bytes of a complex64 one, which doubles its weight (bf16 form: 1.88 ->
// 1.58 ms and 1.73 -> 1.52 ms per launch of 40.5 pairs; the complex64
// passes and those of the fp16 form, whose intermediates are complex64,
// gained nothing this way and keep one tile per workgroup).  The
// grid is a multiple of 8, so a task runs on its block's XCD (task mod 8 =
// block mod 8) and the four readers of a block of T still run side by side.
__global__ __launch_bounds__(k4Threads) void k4_inv_nat_scores(PassArgs a) {
  __shared__ float2 lds[4 * k4Sub];
  __shared__ float2 twl[256];
  load_twiddles<1>(a, twl);
  const int ntask = 1024 * a.nb;
  unsigned int w[16];
  float sT[16];
  auto issue = [&](int task) {
    const int tile = reader_tile(task & 1023), j = task >> 10;
    const unsigned int* T = (const unsigned int*)a.src_c + inv_nat_src(a, j, tile >> 6, tile & 63);
#pragma unroll
    for (int q = 0; q < 16; ++q) w[q] = T[q * 4096];
    inv_nat_scales(a, j, sT);
  };
  int task = blockIdx.x;
  if (task < ntask) issue(task);
  for (; task < ntask; task += gridDim.x) {
    const int tile = reader_tile(task & 1023), j = task >> 10;
    float2 v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = unpack_f16(w[q], sT[q]);
    if (task + gridDim.x < ntask) issue(task + gridDim.x);
    inv_nat_tile<SM_UOUT, OS3D_BF16X2>(a, lds, twl, j, tile >> 6, tile & 63, v);
    __syncthreads();  // the tile's LDS is rewritten by the next task
  }
}

// Natural side of the forward direction: rows y = n1 + 16 n2 of four z
// planes -> T.  x DFT (two stages), then step A over n2 with w^(n1 k2).
// Consecutive workgroups take consecutive n1: sixteen of them read all 256
// rows of the same four planes.  Block wg = 16 zb + n1 of pair slot j; v: the
// thread's 16 values of row `fwd_nat_row(wg)` at x = s + 16 r.
__device__ __forceinline__ long long fwd_nat_row(int wg) {
  const int t = threadIdx.x;
  const int zb = wg >> 4, n1 = wg & 15, g = t >> 8, n2 = (t >> 4) & 15;
  return ((long long)(4 * zb + g) * 256 + (n1 + 16 * n2)) * 256;
}

template <bool T16>
__device__ __forceinline__ void fwd_nat_tile(const PassArgs& a, float2* lds, const float2* twl, float* red, int j,
                                             int wg, float2 (&v)[16]) {
  const int t = threadIdx.x;
  const int zb = wg >> 4, n1 = wg & 15;
  const int g = t >> 8, n2 = (t >> 4) & 15, s = t & 15;
  dft16(v, kFwd);
  float2* S = lds + g * k4Sub + n2 * k4LS;
#pragma unroll
  for (int r = 0; r < 16; ++r) S[pad4(s * 16 + r)] = v[r];
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = S[pad4(s + 16 * r)];
#pragma unroll
  for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], twl[s * r]);
  dft16(v, kFwd);
#pragma unroll
  for (int r = 0; r < 16; ++r) S[pad4(s + 16 * r)] = v[r];
  __syncthreads();
  const int zz = (t >> 2) & 3, kxx = t & 3, kxb = t >> 4, kx = kxb * 4 + kxx;
  float2 u[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) u[q] = lds[zz * k4Sub + q * k4LS + pad4(kx)];
  dft16(u, kFwd);
#pragma unroll
  for (int k2 = 1; k2 < 16; ++k2) u[k2] = cmul(u[k2], twl[n1 * k2]);
  const long long o = (long long)((kxb >> 2) * 16 + n1) * 4096 + zb * 64 + (kxb & 3) * 16 + zz * 4 + kxx;
  if constexpr (!T16) {
    float2* T = a.dst_c + (long long)j * a.dst_stride;
#pragma unroll
    for (int k2 = 0; k2 < 16; ++k2) T[(long long)k2 * (256 * 4096) + o] = u[k2];
  } else {
    const float sT = tile_scale(u, red);
    unsigned int* T = (unsigned int*)a.dst_c + (long long)j * a.dst_stride;
    const float inv = 1.f / sT;  // a power of two: exact
#pragma unroll
    for (int k2 = 0; k2 < 16; ++k2) T[(long long)k2 * (256 * 4096) + o] = pack_f16(u[k2], inv);
    if (t == 0) a.tsc_out[(long long)j * 1024 + wg] = sT;
  }
}

template <int LM, int DT, bool T16 = false>
__global__ __launch_bounds__(k4Threads) void k4_fwd_nat(PassArgs a) {
  __shared__ float2 lds[4 * k4Sub];
  __shared__ float2 twl[256];
  __shared__ float red[16];
  const int j = blockIdx.y;
  load_twiddles<-1>(a, twl);
  float2 v[16];
  float asum = 0.f;
  load_k<LM, DT, 16>(a, j, fwd_nat_row(blockIdx.x) + (threadIdx.x & 15), 16, v, asum);
  fwd_nat_tile<T16>(a, lds, twl, red, j, blockIdx.x, v);
}

// The reconstruction's first pass of the bf16 form, persistent (as
// k4_inv_nat_scores): the next task's two 16-bit score rows are in flight
// while the current tile is transformed.
__global__ __launch_bounds__(k4Threads) void k4_fwd_nat_scores(PassArgs a) {
  __shared__ float2 lds[4 * k4Sub];
  __shared__ float2 twl[256];
  __shared__ float red[16];
  load_twiddles<-1>(a, twl);
  const int ntask = 1024 * a.nb;
  const int s = threadIdx.x & 15;
  unsigned int qa[16], qb[16];
  auto issue = [&](int task) {
    const int j = task >> 10;
    const long long row = fwd_nat_row(task & 1023) + s;
    const unsigned int* Ua = (const unsigned int*)a.U + (long long)a.oa[j] * a.V + row;
#pragma unroll
    for (int r = 0; r < 16; ++r) qa[r] = Ua[r * 16];
    const int ib = a.ob[j];
    if (ib >= 0) {
      const unsigned int* Ub = (const unsigned int*)a.U + (long long)ib * a.V + row;
#pragma unroll
      for (int r = 0; r < 16; ++r) qb[r] = Ub[r * 16];
    }
  };
  int task = blockIdx.x;
  if (task < ntask) issue(task);
  for (; task < ntask; task += gridDim.x) {
    const int j = task >> 10;
    const int ia = a.oa[j], ib = a.ob[j];
    float2 v[16];
    const float sa = a.scales[ia];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = score_value<OS3D_BF16X2>(qa[r], sa);
    if (ib >= 0) {
      const float sb = a.scales[ib];
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = cadd(v[r], cconj(score_value<OS3D_BF16X2>(qb[r], sb)));
    }
    if (task + gridDim.x < ntask) issue(task + gridDim.x);
    fwd_nat_tile<true>(a, lds, twl, red, j, task & 1023, v);
    __syncthreads();  // the tile's LDS (and red) are rewritten by the next task
  }
}

// Natural side of both directions, for processing via scores: inverse T
// tile (k2, zb) -> step C and the inverse x DFT -> the scores of rows
// y = k2 + 16 k1 of four z planes -> Phi -> the forward x DFT and step A
// (n1 = k2, n2 = k1) -> forward T.  After the inverse x DFT a thread holds
// x = s + 16 r of row (g, k1), which is exactly what the forward pass loads
// into that thread, so the scores never leave the registers.
__global__ __launch_bounds__(k4Threads) void k4_nat_phi(PassArgs a) {
  __shared__ float2 lds[4 * k4Sub];
  __shared__ float2 twl[256];  // exp(-2 pi i m / 256); conjugated for the inverse direction
  const int t = threadIdx.x;
  const int tile = reader_tile(blockIdx.x), c = tile >> 6, zb = tile & 63;
  const int j = blockIdx.y;
  for (int i = t; i < 256; i += k4Threads) twl[i] = a.tw[i];
  const float2* T = a.src_c + (long long)j * a.src_stride + (long long)(c * 16 + (zb >> 2)) * 16 * 4096 +
                    (t >> 4) * 64 + (zb & 3) * 16 + (t & 15);
  float2 v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) v[q] = T[q * 4096];
  dft16(v, 1.f);  // over n1 -> k1
  {
    const int g = (t >> 2) & 3, kx = (t >> 4) * 4 + (t & 3);
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) lds[g * k4Sub + k1 * k4LS + pad4(kx)] = v[k1];
  }
  __syncthreads();
  const int g = t >> 8, k1 = (t >> 4) & 15, s = t & 15;
  float2* S = lds + g * k4Sub + k1 * k4LS;
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = S[pad4(s + 16 * r)];
  dft16(v, 1.f);
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 16; ++r) S[pad4(s * 16 + r)] = v[r];
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = S[pad4(s + 16 * r)];
#pragma unroll
  for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], cconj(twl[s * r]));
  dft16(v, 1.f);
  // V U at (z = 4 zb + g, y = 16 k1 + c, x = s + 16 r) -> Phi
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = phi_apply(a, j, v[r]);
  // forward direction on the same rows
  dft16(v, -1.f);
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 16; ++r) S[pad4(s * 16 + r)] = v[r];
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = S[pad4(s + 16 * r)];
#pragma unroll
  for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], twl[s * r]);
  dft16(v, -1.f);
#pragma unroll
  for (int r = 0; r < 16; ++r) S[pad4(s + 16 * r)] = v[r];
  __syncthreads();
  const int zz = (t >> 2) & 3, kxx = t & 3, kxb = t >> 4, kx = kxb * 4 + kxx;
  float2 u[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) u[q] = lds[zz * k4Sub + q * k4LS + pad4(kx)];
  dft16(u, -1.f);
#pragma unroll
  for (int k2 = 1; k2 < 16; ++k2) u[k2] = cmul(u[k2], twl[c * k2]);
  float2* Tf = a.dst_c + (long long)j * a.dst_stride;
  const long long o = (long long)((kxb >> 2) * 16 + c) * 4096 + zb * 64 + (kxb & 3) * 16 + zz * 4 + kxx;
#pragma unroll
  for (int k2 = 0; k2 < 16; ++k2) Tf[(long long)k2 * (256 * 4096) + o] = u[k2];
}

// Frequency side of the forward direction: T tile (k2, kxb) -> Phi tile
// (kxb, n1 = k2).  Step C over n1, then the z DFT (two stages), then the
// fused store (F) or the weighted orientation sum over the pair batch (X).
template <int SM, bool T16 = false>
__global__ __launch_bounds__(k4Threads) void k4_fwd_phi(PassArgs a) {
  __shared__ float2 lds[4 * k4Sub];
  __shared__ float2 twl[256];
  const int t = threadIdx.x;
  // fp16 intermediates: the four readers of a block load 64-byte quarters
  // of its 128-byte lines, so they run side by side on one XCD (one L2)
  const int tile = T16 ? reader_tile(blockIdx.x) : blockIdx.x, k2 = tile >> 6, kxb = tile & 63;
  load_twiddles<-1>(a, twl);
  const long long pbase = (long long)(kxb * 16 + k2) << 14;
  const int jb = (SM == SM_ACCUM) ? 0 : blockIdx.y;
  const int je = (SM == SM_ACCUM) ? a.nb : blockIdx.y + 1;
  float2 acc[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = make_float2(0.f, 0.f);
  const long long tb = (long long)(k2 * 16 + (kxb >> 2)) * 16 * 4096 + (t >> 4) * 64 + (kxb & 3) * 16 + (t & 15);
  unsigned int wn[16];  // fp16 intermediates: the next pair's words, in flight during this pair
  if constexpr (T16) {
    const unsigned int* T = (const unsigned int*)a.src_c + (long long)jb * a.src_stride + tb;
#pragma unroll
    for (int q = 0; q < 16; ++q) wn[q] = ldnt(T + q * 4096);
  }
  for (int j = jb; j < je; ++j) {
    float2 v[16];
    if constexpr (!T16) {
      const float2* T = a.src_c + (long long)j * a.src_stride + tb;
#pragma unroll
      for (int q = 0; q < 16; ++q) v[q] = ldnt(T + q * 4096);
    } else {
      // value q was written by the natural-side workgroup (zb = t / 16, n1 = q)
      const float* sc = a.tsc + (long long)j * 1024 + (t >> 4) * 16;
#pragma unroll
      for (int q = 0; q < 16; ++q) v[q] = unpack_f16(wn[q], sc[q]);
    }
    dft16(v, kFwd);  // over n1 -> k1
    {
      const int g = t & 3, z = t >> 2;
#pragma unroll
      for (int k1 = 0; k1 < 16; ++k1) lds[g * k4Sub + k1 * k4LS + pad4(z)] = v[k1];
    }
    if constexpr (T16) {
      if (j + 1 < je) {
        const unsigned int* T = (const unsigned int*)a.src_c + (long long)(j + 1) * a.src_stride + tb;
#pragma unroll
        for (int q = 0; q < 16; ++q) wn[q] = ldnt(T + q * 4096);
      }
    }
    __syncthreads();
    const int g = t & 3, s = (t >> 2) & 15, k1 = t >> 6;
    float2* S = lds + g * k4Sub + k1 * k4LS;
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = S[pad4(s + 16 * r)];
    dft16(v, kFwd);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) S[pad4(s * 16 + r)] = v[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = S[pad4(s + 16 * r)];
#pragma unroll
    for (int r = 1; r < 16; ++r) v[r] = cmul(v[r], twl[s * r]);
    dft16(v, kFwd);
    // kz = s + 16 r sits at Phi position pbase + r * 1024 + t
    store_k<SM, OS3D_C64, 16>(a, j, pbase + t, 1024, v, acc);
    if constexpr (SM == SM_ACCUM) __syncthreads();
  }
  if constexpr (SM == SM_ACCUM) flush_k<16>(a, pbase + t, 1024, acc);
}

// Workgroups of a persistent score pass: one per CU, rounded down to a
// multiple of the 8 XCDs, at most one per task.
static unsigned persistent_grid(long long ntask) {
  static const int n = [] {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 8)
      cus = 256;
    return cus / 8 * 8;
  }();
  return (unsigned)std::min<long long>(ntask, n);
}

static int check(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return OS3D_EDEVICE;
  }
  return OS3D_OK;
}

static PassArgs base_args(const os3d_bank* b, float sgn) {
  PassArgs a = {};
  a.Nz = a.Ny = a.Nx = 256;
  a.V = b->V;
  a.N = 256;
  a.tw = (const float2*)b->d.tw[0];
  a.sgn = sgn;
  a.nb = 1;
  return a;
}

#define OS3D_LAUNCH4(kernel, kid, alg, a, gy)                                                  \
  do {                                                                                         \
    void* tok_ = prof_start(st, kid);                                                               \
    launch_k(kernel, dim3(1024), dim3(k4Threads), 0, st, a);                         \
    prof_stop(tok_, st, kid, alg, 0.0);                                                        \
    if ((rc = check(#kernel))) return rc;                                                      \
  } while (0)

int forward4(const os3d_bank* b, const float* f, int batch, void* U, int dtype, float* scales, void* ws, int nbmax,
             void* stream) {
  hipStream_t st = (hipStream_t)stream;
  const long long V = b->V;
  float2* F = (float2*)ws;
  float2* T = F + V;  // nbmax intermediates
  float* partial = (float*)(T + (long long)nbmax * V);
  // bf16 scores: fp16 intermediates in the first half of T, their scales after them
  float* tsc = (float*)((unsigned int*)T + (long long)nbmax * V);
  const size_t ubytes = (dtype == OS3D_C64) ? 8 : 4;
  const bool quant = dtype != OS3D_C64;
  const bool t16 = dtype == OS3D_BF16X2;
  int rc;
  for (int bi = 0; bi < batch; ++bi) {
    {  // F = DFT(f) into the frequency tiles
      PassArgs a = base_args(b, -1.f);
      a.src_r = f + (long long)bi * V;
      a.dst_c = T;
      OS3D_LAUNCH4((k4_fwd_nat<LM_REAL, OS3D_C64>), kProfDftFirst, 4.0 * V, a, 1);
      PassArgs c = base_args(b, -1.f);
      c.src_c = T;
      c.dst_c = F;
      OS3D_LAUNCH4((k4_fwd_phi<SM_C>), kProfDftLast, 0.0, c, 1);
    }

    void* Ub = (char*)U + (size_t)bi * b->n_orients * V * ubytes;
    float* sc = scales ? scales + (long long)bi * b->n_orients : nullptr;
    for (int r0 = 0; r0 < b->n_unique; r0 += nbmax) {
      const int nb = std::min(nbmax, b->n_unique - r0);
      PassArgs z = base_args(b, 1.f);
      z.nb = nb;
      double nor = 0.0;
      for (int jj = 0; jj < nb; ++jj) {
        const int o = b->rep[r0 + jj];
        z.rows[jj] = r0 + jj;
        z.oa[jj] = o;
        z.ob[jj] = b->partner[o];
        nor += (z.ob[jj] >= 0) ? 2.0 : 1.0;
      }
      z.src_c = F;
      z.psi = b->d.psi;
      z.kappa = (float)b->kappa;
      z.dst_c = T;
      z.dst_stride = V;
      z.partial = quant ? partial : nullptr;
      z.tsc = tsc;
      z.tsc_out = tsc;
      {
        void* tok = prof_start(st, kProfFwdFirst);
        if (t16)
          launch_k((k4_inv_phi<LM_MULBANK, true>), dim3(1024), dim3(k4Threads), 0, st, z);
        else
          launch_k((k4_inv_phi<LM_MULBANK>), dim3(1024), dim3(k4Threads), 0, st, z);
        prof_stop(tok, st, kProfFwdFirst, 0.0, 0.0);
        if ((rc = check("k4_inv_phi"))) return rc;
      }
      if (quant) {
        void* tok = prof_start(st, kProfScales);
        launch_scales(partial, 1024, z, dtype, sc, nb, st);
        prof_stop(tok, st, kProfScales, 0.0, 0.0);
        if ((rc = check("k_scales"))) return rc;
      }
      PassArgs x = z;
      x.partial = nullptr;
      x.src_c = T;
      x.src_stride = V;
      x.Uout = Ub;
      x.dtype = dtype;
      x.scales = quant ? sc : nullptr;
      x.out_scale = 1.f / (float)V;
      {
        void* tok = prof_start(st, kProfFwdLast);
        if (dtype == OS3D_C64)
          launch_k((k4_inv_nat<SM_UOUT, OS3D_C64>), dim3(1024, nb), dim3(k4Threads), 0, st, x);
        else if (dtype == OS3D_BF16X2)
          launch_k(k4_inv_nat_scores, dim3(persistent_grid(1024LL * nb)), dim3(k4Threads), 0, st, x);
        else
          launch_k((k4_inv_nat<SM_UOUT, OS3D_F16X2>), dim3(1024, nb), dim3(k4Threads), 0, st, x);
        prof_stop(tok, st, kProfFwdLast, nor * (double)V * (double)ubytes, 0.0);
        if ((rc = check("k4_inv_nat"))) return rc;
      }
    }
  }
  return OS3D_OK;
}

int reduce4(const os3d_bank* b, const void* U, int dtype, const float* scales, int batch, float* f_out, void* ws,
            bool divide_M, int nbmax, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  const long long V = b->V;
  float2* X = (float2*)ws;
  float2* T = X + V;
  // bf16 scores: fp16 intermediates in the first half of T, their scales after them
  float* tsc = (float*)((unsigned int*)T + (long long)nbmax * V);
  const size_t ubytes = (dtype == OS3D_C64) ? 8 : 4;
  int rc;
  for (int bi = 0; bi < batch; ++bi) {
    const void* Ub = (const char*)U + (size_t)bi * b->n_orients * V * ubytes;
    const float* sc = scales ? scales + (long long)bi * b->n_orients : nullptr;
    for (int r0 = 0; r0 < b->n_unique; r0 += nbmax) {
      const int nb = std::min(nbmax, b->n_unique - r0);
      PassArgs x = base_args(b, -1.f);
      x.nb = nb;
      double nor = 0.0;
      for (int jj = 0; jj < nb; ++jj) {
        const int o = b->rep[r0 + jj];
        x.rows[jj] = r0 + jj;
        x.oa[jj] = o;
        x.ob[jj] = b->partner[o];
        nor += (x.ob[jj] >= 0) ? 2.0 : 1.0;
      }
      x.U = Ub;
      x.dtype = dtype;
      x.scales = (dtype == OS3D_C64) ? nullptr : sc;
      x.dst_c = T;
      x.dst_stride = V;
      x.tsc = tsc;
      x.tsc_out = tsc;
      {
        void* tok = prof_start(st, kProfRecFirst);
        if (dtype == OS3D_C64)
          launch_k((k4_fwd_nat<LM_UIN, OS3D_C64>), dim3(1024, nb), dim3(k4Threads), 0, st, x);
        else if (dtype == OS3D_BF16X2)
          launch_k(k4_fwd_nat_scores, dim3(persistent_grid(1024LL * nb)), dim3(k4Threads), 0, st, x);
        else
          launch_k((k4_fwd_nat<LM_UIN, OS3D_F16X2>), dim3(1024, nb), dim3(k4Threads), 0, st, x);
        prof_stop(tok, st, kProfRecFirst, nor * (double)V * (double)ubytes, 0.0);
        if ((rc = check("k4_fwd_nat"))) return rc;
      }
      PassArgs z = x;
      z.src_c = T;
      z.src_stride = V;
      z.psi = b->d.psi;
      z.kappa = (float)b->kappa;
      z.dst_c = X;
      z.accumulate = (r0 > 0) ? 1 : 0;
      if (dtype == OS3D_BF16X2)
        OS3D_LAUNCH4((k4_fwd_phi<SM_ACCUM, true>), kProfRecLast, 0.0, z, 1);
      else
        OS3D_LAUNCH4((k4_fwd_phi<SM_ACCUM>), kProfRecLast, 0.0, z, 1);
    }
    PassArgs z = base_args(b, 1.f);
    z.src_c = X;
    z.M = b->d.M;
    z.kappa = (float)b->kappa;
    z.eps = (float)b->params.eps;
    z.divide = divide_M ? 1 : 0;
    z.dst_c = T;
    OS3D_LAUNCH4((k4_inv_phi<LM_DIVM>), kProfInvFirst, 0.0, z, 1);
    PassArgs x = base_args(b, 1.f);
    x.src_c = T;
    x.dst_r = f_out + (long long)bi * V;
    x.out_scale = 1.f / (float)V;
    OS3D_LAUNCH4((k4_inv_nat<SM_REAL, OS3D_C64>), kProfInvLast, 4.0 * V, x, 1);
  }
  return OS3D_OK;
}

// Processing via scores, Eq. (23) with the stabilised inverse: per pair
// batch, the frequency-side pass of the inverse direction, then one
// natural-side kernel for both directions with Phi in registers (the scores
// never reach memory), then the frequency-side accumulation of the
// orientation sum.
int process4(const os3d_bank* b, const float* f, int batch, int phi_kind, float phi_p, float* f_out, void* ws,
             int nbmax, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  const long long V = b->V;
  float2* F = (float2*)ws;
  float2* X = F + V;
  float2* T = X + V;
  float2* Z = T + (long long)nbmax * V;
  int rc;
  for (int bi = 0; bi < batch; ++bi) {
    {
      PassArgs a = base_args(b, -1.f);
      a.src_r = f + (long long)bi * V;
      a.dst_c = T;
      OS3D_LAUNCH4((k4_fwd_nat<LM_REAL, OS3D_C64>), kProfDftFirst, 4.0 * V, a, 1);
      PassArgs c = base_args(b, -1.f);
      c.src_c = T;
      c.dst_c = F;
      OS3D_LAUNCH4((k4_fwd_phi<SM_C>), kProfDftLast, 0.0, c, 1);
    }
    for (int r0 = 0; r0 < b->n_unique; r0 += nbmax) {
      const int nb = std::min(nbmax, b->n_unique - r0);
      PassArgs z = base_args(b, 1.f);
      z.nb = nb;
      for (int jj = 0; jj < nb; ++jj) {
        const int o = b->rep[r0 + jj];
        z.rows[jj] = r0 + jj;
        z.oa[jj] = o;
        z.ob[jj] = b->partner[o];
      }
      z.src_c = F;
      z.psi = b->d.psi;
      z.kappa = (float)b->kappa;
      z.dst_c = T;
      z.dst_stride = V;
      OS3D_LAUNCH4((k4_inv_phi<LM_MULBANK>), kProfFwdFirst, 0.0, z, 1);
      PassArgs x = z;
      x.src_c = T;
      x.src_stride = V;
      x.dst_c = Z;
      x.dst_stride = V;
      x.out_scale = 1.f / (float)V;
      x.phi_kind = phi_kind;
      x.phi_p = phi_p;
      {
        void* tok = prof_start(st, kProfFwdLast);
        launch_k(k4_nat_phi, dim3(1024, nb), dim3(k4Threads), 0, st, x);
        prof_stop(tok, st, kProfFwdLast, 0.0, 0.0);
        if ((rc = check("k4_nat_phi"))) return rc;
      }
      PassArgs w = base_args(b, -1.f);
      w.nb = nb;
      for (int jj = 0; jj < nb; ++jj) w.rows[jj] = z.rows[jj];
      w.src_c = Z;
      w.src_stride = V;
      w.psi = b->d.psi;
      w.dst_c = X;
      w.dst_stride = 0;
      w.accumulate = (r0 > 0) ? 1 : 0;
      OS3D_LAUNCH4((k4_fwd_phi<SM_ACCUM>), kProfRecLast, 0.0, w, 1);
    }
    PassArgs z = base_args(b, 1.f);
    z.src_c = X;
    z.M = b->d.M;
    z.kappa = (float)b->kappa;
    z.eps = (float)b->params.eps;
    z.divide = 1;
    z.dst_c = T;
    OS3D_LAUNCH4((k4_inv_phi<LM_DIVM>), kProfInvFirst, 0.0, z, 1);
    PassArgs x = base_args(b, 1.f);
    x.src_c = T;
    x.dst_r = f_out + (long long)bi * V;
    x.out_scale = 1.f / (float)V;
    OS3D_LAUNCH4((k4_inv_nat<SM_REAL, OS3D_C64>), kProfInvLast, 4.0 * V, x, 1);
  }
  return OS3D_OK;
}

}  // namespace os3d
