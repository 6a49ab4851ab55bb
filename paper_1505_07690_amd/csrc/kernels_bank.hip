// Wavelet-bank synthesis on gfx950 (Sec. 3, Eqs. 9-19).
//
// For every DFT frequency k the rotated angular profiles of all stored bank
// rows are one row of a dense contraction
//     h[k, i] = sum_{(l,m)} Y_lm(w_hat_k) S[(l,m), i]
// (S: steering matrix a_l sqrt(4 pi/(2l+1)) Y_lm(n_i), the addition-theorem
// form of the Wigner-D rotation of Eqs. 17-19).  It runs on the fp16 matrix
// cores with FP32-level accuracy: each operand is split into fp16 hi + lo
// parts, x = hi + lo to 2^-22 relative, and
//     x y ~ hi_x hi_y + hi_x lo_y + lo_x hi_y
// (three v_mfma_f32_16x16x32_f16, FP32 accumulation; the dropped lo lo term
// is below 2^-22 relative).  Y_lm is scaled by 2^13 and S by 2^e_S first so
// that neither part meets fp16's subnormal range; the product is scaled back
// by 2^-(13 + e_S).
//
// Each wave owns 64 frequency points and works alone: every lane runs the
// FP64 normalised recursion for its point's Q_l^m, one K entry pair (cos,
// sin) per step, multiplies by Re / Im (x + iy)^m (the sinus power is in
// that factor), splits into hi / lo and writes the word to the wave's LDS
// ring (one K-block, [word pair][point][2 words]).  When the K-block is
// complete the wave reads it back in the MFMA's A-operand order (lane t:
// point t % 16 of each 16-point row block, entries 8 (t / 16) .. + 7) and
// runs the block against the steering operands, which the host packed in
// the B-operand order and which the wave loads from memory (L2-resident)
// while it generates the block.  The epilogue multiplies by the FP64 radial window
// g(rho) (Eq. 10), applies the Nyquist and DC rules, writes the bank rows
// and accumulates sum_i psi_i^2 (Eq. 9) and sum_i psi_i in FP64 with a
// fixed-order cross-lane tree; the workgroup's sums of both over the
// normalisation band go to one partial record per workgroup.  The rows are
// stored without the normaliser kappa (known only once every partial is
// in): the transforms apply kappa as a scalar where they multiply by the
// bank.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "launch.h"
#include "layout4.h"
#include "os3d_internal.h"

namespace os3d {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __fp16 fp16x2 __attribute__((ext_vector_type(2)));

constexpr int kBankPts = 256;    // frequency points per workgroup (four independent waves)
constexpr int kRingRows = 8;     // word pairs of one K-block
constexpr int kRingStride = 144; // words per ring row (64 points x 2 words + 16): rows 2 apart fall 32 banks apart
constexpr double kYScale = 8192.0;  // 2^13

struct BankArgs {
  int layout;  // storage order of the frequency points (natural or four-step tiles)
  int Nz, Ny, Nx;
  long long V;
  int L, n_rows, ncb, kblocks;
  int mb;             // first order of recursion chain B
  double t_inv;       // 1 / t of Eq. (10)
  int taylor_N;
  double dc_value;    // a_0 / sqrt(4 pi)
  float out_scale;    // 2^-(13 + e_S)
  const uint4* S;     // [kblocks][ncb][2 (hi, lo)][64 lanes] B operands, ncb a multiple of the sweep's
  const double* tab;  // recursion steps [kblocks * 8][chain A, B][c0, c1], then order-start masks
  float* psi;         // [n_rows][V]
  double* Mh;         // [V]
  double* part;       // [gridDim.x][3]: band sums of Mh and of sum_i psi_i, band count
};

__device__ inline double omega_of(int k, int n) {
  int kt = (k < (n + 1) / 2) ? k : k - n;
  return 2.0 * 3.14159265358979323846 * (double)kt / (double)n;
}

__device__ inline bool is_nyquist(int k, int n) { return (n % 2 == 0) && (k == n / 2); }

// Radial window of Eq. (10): exp(-x) sum_{j <= N} x^j / j!, x = rho^2 / t.
__device__ inline double radial_g(double rho2, double t_inv, int N) {
  double x = rho2 * t_inv;
  double term = exp(-x), acc = term;
  for (int j = 1; j <= N; ++j) {
    term = term * x / (double)j;
    acc += term;
  }
  return acc;
}

typedef _Float16 half2v __attribute__((ext_vector_type(2)));

// fp16 hi / lo parts of q c and q s (round to nearest even), packed low
// half first.  The products are rounded to FP32 once and held in registers
// (the empty asm): otherwise the compiler may fuse a product into the fp16
// conversion on one path and not on the other, and the hi part in the word
// would differ from the one the residual subtracts (hi + lo then misses q c
// by an fp16 ulp).  The residual subtracts the packed hi values themselves.
__device__ __forceinline__ void split_pair(float q, float c, float s, unsigned& hi, unsigned& lo) {
  float u = q * c, v = q * s;
  asm volatile("" : "+v"(u), "+v"(v));
  half2v h;
  h.x = (_Float16)u;
  h.y = (_Float16)v;
  hi = __builtin_bit_cast(unsigned, h);
  asm volatile("" : "+v"(hi));  // unpack the packed word (no second conversion)
  const half2v hh = __builtin_bit_cast(half2v, hi);
  half2v l;
  l.x = (_Float16)(u - (float)hh.x);
  l.y = (_Float16)(v - (float)hh.y);
  lo = __builtin_bit_cast(unsigned, l);
}

// The recursion runs as two independent chains, A over the orders 0..M and
// B over M + 1..L, which fill the even and odd words of the K order: two
// dependency chains in flight per lane.  Per word pair the table holds one
// record (c0, c1) per chain, Q = c0 (z Q') - c1 Q'' (Q', Q'': the chain's
// two previous values): inside an order c0 = alpha_lm and c1 = alpha_lm
// beta_lm of the normalised recursion; where an order starts c0 = 0 and
// c1 = -Q_m^m, and the chain sets Q'' = 1 first; zero records past a
// chain's end.  After the records, one 32-bit mask per K-block marks the
// pairs that start an order (bit i: chain A, bit 8 + i: chain B).  The
// table is read-only during the synthesis: read through the constant
// address space, the uniform records become scalar loads (one per pair) and
// the masks scalar bit tests, which do not wait behind the vector loads of
// the steering operands.
struct StepPair {
  double a[2], b[2];  // chain A, chain B: c0, c1
};
typedef const StepPair __attribute__((address_space(4)))* ctab_t;
typedef const unsigned __attribute__((address_space(4)))* cmask_t;

__device__ __forceinline__ StepPair load_steps(ctab_t p) {
  StepPair r;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    r.a[j] = p->a[j];
    r.b[j] = p->b[j];
  }
  return r;
}

__device__ __forceinline__ double rec_step(const double* r, double uz, double& q1, double& q2) {
  const double q = fma(r[0], uz * q1, -(r[1] * q2));
  q2 = q1;
  q1 = q;
  return q;
}

template <int NCB>
__global__ __launch_bounds__(256, 2) void k_bank_synth(BankArgs a) {
  __shared__ unsigned ring[4][2][kRingRows * kRingStride];  // per wave: hi plane, lo plane
  __shared__ double gsh[kBankPts];
  __shared__ double Msh[kBankPts];
  __shared__ int flags[kBankPts];  // bit 0: DC, bit 1: in the normalisation band

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const long long p0 = (long long)blockIdx.x * kBankPts;
  const long long pw = p0 + wave * 64;  // the wave's first point
  const long long p = p0 + tid;
  const bool valid = p < a.V;
  const ctab_t tab = (ctab_t)a.tab;
  const cmask_t starts = (cmask_t)(tab + a.kblocks * 8);  // after the records
  unsigned* hiP = ring[wave][0];
  unsigned* loP = ring[wave][1];

  // this lane's frequency point
  double ux = 0.0, uy = 0.0, uz = 1.0, g = 0.0;
  int dc = 0;
  bool band = false;  // the normalisation band: 0 < rho <= rho_N / 2, no Nyquist plane
  if (valid) {
    int kz, ky, kx;
    pos_to_k(a.layout, p, a.Nz, a.Ny, a.Nx, kz, ky, kx);
    double wx = omega_of(kx, a.Nx), wy = omega_of(ky, a.Ny), wz = omega_of(kz, a.Nz);
    double r2 = wx * wx + wy * wy + wz * wz;
    if (r2 > 0.0) {
      double r = sqrt(r2);
      ux = wx / r;
      uy = wy / r;
      uz = wz / r;
    } else {
      dc = 1;
    }
    bool nyq = is_nyquist(kx, a.Nx) || is_nyquist(ky, a.Ny) || is_nyquist(kz, a.Nz);
    g = nyq ? 0.0 : radial_g(r2, a.t_inv, a.taylor_N);
    const double hn = 0.5 * 3.14159265358979323846;
    band = !nyq && r2 > 0.0 && r2 <= hn * hn;
  }
  gsh[tid] = g;
  flags[tid] = dc | (band ? 2 : 0);
  Msh[tid] = 0.0;
  double asum = 0.0;  // this lane's share of the band sum of sum_i psi_raw
  // the points are wave-private: a wave-level fence orders the LDS traffic
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

  const bool vec_store = (a.V % 4 == 0) && (pw + 64 <= a.V);
  for (int cb0 = 0; cb0 < a.ncb; cb0 += NCB) {
    floatx4 acc[4][NCB];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < NCB; ++c) acc[r][c] = floatx4{0.f, 0.f, 0.f, 0.f};

    // chain A starts at m = 0 ((x + iy)^0 = 1, no sqrt 2), chain B at m = mb
    const double sc = 1.4142135623730950488 * kYScale;
    double qa1 = 0.0, qa2 = 0.0, qb1 = 0.0, qb2 = 0.0;  // the chains' two previous values
    double cra = 1.0, cia = 0.0, crb = 1.0, cib = 0.0;  // (x + iy)^m of each chain
    for (int m = 0; m < a.mb; ++m) {
      const double nr = crb * ux - cib * uy, ni = crb * uy + cib * ux;
      crb = nr;
      cib = ni;
    }
    float crsa = (float)kYScale, cisa = 0.f;  // times sqrt 2 (m > 0) and 2^13, in FP32
    float crsb = (float)(crb * sc), cisb = (float)(cib * sc);
    for (int kb = 0; kb < a.kblocks; ++kb) {
      // the block's steering operands: in flight while the block is generated
      uint4 bop[NCB][2];
#pragma unroll
      for (int c = 0; c < NCB; ++c)
#pragma unroll
        for (int h = 0; h < 2; ++h)
          bop[c][h] = a.S[(((long long)kb * a.ncb + cb0 + c) * 2 + h) * 64 + lane];
      // generate the block's 8 word pairs (uniform control flow)
      const unsigned st = starts[kb];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const StepPair r = load_steps(tab + kb * 8 + i);  // one scalar load of both records
        const bool later = kb > 0 || i > 0;  // not the chains' first order
        if ((st >> i) & 1u) {  // chain A starts an order
          qa2 = 1.0;
          if (later) {  // (x + iy)^(m+1)
            const double nr = cra * ux - cia * uy, ni = cra * uy + cia * ux;
            cra = nr;
            cia = ni;
            crsa = (float)(nr * sc);
            cisa = (float)(ni * sc);
          }
        }
        if ((st >> (8 + i)) & 1u) {  // chain B
          qb2 = 1.0;
          if (later) {
            const double nr = crb * ux - cib * uy, ni = crb * uy + cib * ux;
            crb = nr;
            cib = ni;
            crsb = (float)(nr * sc);
            cisb = (float)(ni * sc);
          }
        }
        const float qa = (float)rec_step(r.a, uz, qa1, qa2);
        const float qb = (float)rec_step(r.b, uz, qb1, qb2);
        uint2 hw, lw;  // (chain A word, chain B word)
        split_pair(qa, crsa, cisa, hw.x, lw.x);
        split_pair(qb, crsb, cisb, hw.y, lw.y);
        *(uint2*)&hiP[i * kRingStride + 2 * lane] = hw;
        *(uint2*)&loP[i * kRingStride + 2 * lane] = lw;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // A operands of the four 16-point row blocks: lane t takes the words
      // 4 (t / 16) .. + 3, i.e. the pairs 2 (t / 16) and + 1
      half8 ah[4], al[4];
      const int p0r = 2 * (lane >> 4);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int col = 2 * (r * 16 + (lane & 15));
        const uint2 h0 = *(const uint2*)&hiP[p0r * kRingStride + col];
        const uint2 h1 = *(const uint2*)&hiP[(p0r + 1) * kRingStride + col];
        const uint2 l0 = *(const uint2*)&loP[p0r * kRingStride + col];
        const uint2 l1 = *(const uint2*)&loP[(p0r + 1) * kRingStride + col];
        ah[r] = __builtin_bit_cast(half8, uint4{h0.x, h0.y, h1.x, h1.y});
        al[r] = __builtin_bit_cast(half8, uint4{l0.x, l0.y, l1.x, l1.y});
      }
      // the ring is rewritten by the next block only after these reads
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // hi hi, hi lo, lo hi: each pass over all 4 x NCB accumulators before
      // the next touches one again (the operands of absent column blocks are
      // zero: no branches between the MFMAs)
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < NCB; ++c)
          acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[r], __builtin_bit_cast(half8, bop[c][0]), acc[r][c], 0, 0,
                                                             0);
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < NCB; ++c)
          acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[r], __builtin_bit_cast(half8, bop[c][1]), acc[r][c], 0, 0,
                                                             0);
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < NCB; ++c)
          acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[r], __builtin_bit_cast(half8, bop[c][0]), acc[r][c], 0, 0,
                                                             0);
    }

    // epilogue: psi_raw = g * h (DC: isotropic), bank rows, FP64 sums of
    // squares and of values.  Lane t holds column t % 16 and the four
    // consecutive points 4 (t / 16) .. + 3 of each row block.
    double mh[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int i = 0; i < 4; ++i) mh[r][i] = 0.0;
#pragma unroll
    for (int c = 0; c < NCB; ++c) {
      const int col = (cb0 + c) * 16 + (lane & 15);
      const bool colok = col < a.n_rows;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int pt0 = wave * 64 + r * 16 + 4 * (lane >> 4);
        float vv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int pt = pt0 + i;
          const int fl = flags[pt];
          // columns past the rows have zero steering operands (h = 0) and
          // no DC value: they add exact zeros
          const double h = (fl & 1) ? (colok ? a.dc_value : 0.0) : (double)(acc[r][c][i] * a.out_scale);
          const float v = (float)(gsh[pt] * h);
          vv[i] = v;
          mh[r][i] += (double)v * (double)v;
          asum += (fl & 2) ? (double)v : 0.0;
        }
        if (colok) {
          float* dst = a.psi + (long long)col * a.V + p0 + pt0;
          if (vec_store) {
            *(float4*)dst = float4{vv[0], vv[1], vv[2], vv[3]};
          } else {
#pragma unroll
            for (int i = 0; i < 4; ++i)
              if (p0 + pt0 + i < a.V) dst[i] = vv[i];
          }
        }
      }
    }
    // sum over the 16 lanes that share (lane >> 4): fixed xor tree, then
    // into the point's running sum (one owner lane per point)
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        double s = mh[r][i];
        s += __shfl_xor(s, 1);
        s += __shfl_xor(s, 2);
        s += __shfl_xor(s, 4);
        s += __shfl_xor(s, 8);
        if ((lane & 15) == 0) Msh[wave * 64 + r * 16 + 4 * (lane >> 4) + i] += s;
      }
  }
  __syncthreads();
  const double mt = Msh[tid];
  if (valid) a.Mh[p] = mt;
  // the workgroup's band sums, by a fixed tree (deterministic), in the ring's
  // memory
  double* tm = (double*)&ring[0][0][0];
  double* ta = tm + kBankPts;
  double* tc = ta + kBankPts;
  tm[tid] = band ? mt : 0.0;
  ta[tid] = asum;
  tc[tid] = band ? 1.0 : 0.0;
  __syncthreads();
  for (int w = kBankPts / 2; w > 0; w >>= 1) {
    if (tid < w) {
      tm[tid] += tm[tid + w];
      ta[tid] += ta[tid + w];
      tc[tid] += tc[tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) {
    a.part[3 * (long long)blockIdx.x] = tm[0];
    a.part[3 * (long long)blockIdx.x + 1] = ta[0];
    a.part[3 * (long long)blockIdx.x + 2] = tc[0];
  }
}

// S: k -> -k mod N on every axis, on storage positions.
__device__ inline long long mirror_index(int layout, long long p, int Nz, int Ny, int Nx) {
  int kz, ky, kx;
  pos_to_k(layout, p, Nz, Ny, Nx, kz, ky, kx);
  return k_to_pos(layout, (Nz - kz) % Nz, (Ny - ky) % Ny, (Nx - kx) % Nx, Ny, Nx);
}

// kappa and the approximate-reconstruction normaliser from the synthesis
// workgroups' band partials, summed in a fixed order (deterministic).  The
// band is symmetric under k -> -k, so for an antipodal set the partner's
// terms (the stored row read at -k) add the same band sums again:
//   kappa = (mean over the band of M0)^(-1/2), M0[k] = Mh[k] (+ Mh[-k]);
//   S = kappa x (mean over the band of sum over every orientation of psi_raw).
// out[0] = kappa, out[1] = S.
__global__ __launch_bounds__(1024) void k_bank_reduce(const double* part, long long nparts, int paired, double* out) {
  __shared__ double sm[1024], sa[1024], sc[1024];
  const int tid = threadIdx.x;
  double m = 0.0, av = 0.0, c = 0.0;
  for (long long i = tid; i < nparts; i += 1024) {
    m += part[3 * i];
    av += part[3 * i + 1];
    c += part[3 * i + 2];
  }
  sm[tid] = m;
  sa[tid] = av;
  sc[tid] = c;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if (tid < w) {
      sm[tid] += sm[tid + w];
      sa[tid] += sa[tid + w];
      sc[tid] += sc[tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) {
    const double f = paired ? 2.0 : 1.0;
    const double cnt = sc[0];
    const double mean_m = f * sm[0] / cnt;
    const double kappa = (cnt > 0.0 && mean_m > 0.0) ? 1.0 / sqrt(mean_m) : 1.0;
    out[0] = kappa;
    out[1] = (cnt > 0.0) ? kappa * f * sa[0] / cnt : 1.0;
  }
}

// M = kappa^2 M0 (Eq. 9 with its constants in kappa), M0[k] = Mh[k] (+ Mh[-k]
// for an antipodal set: the partner's row is the stored row at -k).
__global__ __launch_bounds__(256) void k_M_finalize(const double* Mh, float* M, int paired, int layout, int Nz,
                                                    int Ny, int Nx, long long V, const double* kappa_p) {
  const double kappa = *kappa_p;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < V; p += stride) {
    const double m0 = Mh[p] + (paired ? Mh[mirror_index(layout, p, Nz, Ny, Nx)] : 0.0);
    M[p] = (float)(kappa * kappa * m0);
  }
}

// f_out[b] = Re(sum_i U[b][i]) / S: the orientation integral of Eq. (6), one
// pass over the scores, fixed summation order (deterministic).  A thread
// sums VPT consecutive voxels, loading 16 bytes per orientation (two
// complex64 or four packed 16-bit scores) when VPT > 1; the per-voxel
// order of the sum is the same for every VPT.
template <int DT>
__device__ __forceinline__ float approx_re(unsigned int q) {
  if constexpr (DT == OS3D_F16X2)
    return __half2float(__ushort_as_half((unsigned short)(q & 0xffffu)));
  else
    return __uint_as_float((q & 0xffffu) << 16);
}

typedef float nt_f2 __attribute__((ext_vector_type(2)));
typedef float nt_f4 __attribute__((ext_vector_type(4)));
typedef unsigned int nt_u4 __attribute__((ext_vector_type(4)));

template <int DT, int VPT>
__global__ __launch_bounds__(256) void k_approx_reconstruct(const void* U, const float* scales, int n_orients,
                                                            long long V, float inv_norm, float* out) {
  const long long p = ((long long)blockIdx.x * 256 + threadIdx.x) * VPT;
  if (p >= V) return;
  if constexpr (VPT == 1) {  // one voxel per thread: the plain loop measured fastest
    float acc = 0.f;
    for (int i = 0; i < n_orients; ++i) {
      const long long e = (long long)i * V + p;
      if constexpr (DT == OS3D_C64)
        acc += __builtin_nontemporal_load((const nt_f2*)U + e).x;
      else
        acc += approx_re<DT>(__builtin_nontemporal_load((const unsigned int*)U + e)) * scales[i];
    }
    out[p] = acc * inv_norm;
  } else {
    float acc[VPT];
#pragma unroll
    for (int v = 0; v < VPT; ++v) acc[v] = 0.f;
#pragma unroll 4
    for (int i = 0; i < n_orients; ++i) {
      const long long e = (long long)i * V + p;
      // every score is read once: non-temporal loads
      if constexpr (DT == OS3D_C64) {
        static_assert(VPT == 2, "complex64 scores: two per 16-byte load");
        const nt_f4 w = __builtin_nontemporal_load((const nt_f4*)((const float2*)U + e));
        acc[0] += w.x;
        acc[1] += w.z;
      } else {
        static_assert(VPT == 4, "16-bit scores: four per 16-byte load");
        const float sc = scales[i];
        const nt_u4 w = __builtin_nontemporal_load((const nt_u4*)((const unsigned int*)U + e));
        acc[0] += approx_re<DT>(w.x) * sc;
        acc[1] += approx_re<DT>(w.y) * sc;
        acc[2] += approx_re<DT>(w.z) * sc;
        acc[3] += approx_re<DT>(w.w) * sc;
      }
    }
#pragma unroll
    for (int v = 0; v < VPT; ++v) out[p + v] = acc[v] * inv_norm;
  }
}


// Natural-order export: out[k] = scale x row[pos(k)] (or row[pos(-k)] for
// the second member of an antipodal pair).
__global__ __launch_bounds__(256) void k_export(const float* row, int mirrored, int layout, int Nz, int Ny, int Nx,
                                                long long V, float scale, float* out) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x; p < V; p += stride) {
    int kx = (int)(p % Nx);
    int ky = (int)((p / Nx) % Ny);
    int kz = (int)(p / ((long long)Nx * Ny));
    if (mirrored) {
      kx = (Nx - kx) % Nx;
      ky = (Ny - ky) % Ny;
      kz = (Nz - kz) % Nz;
    }
    out[p] = scale * row[k_to_pos(layout, kz, ky, kx, Ny, Nx)];
  }
}

static int check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return OS3D_EDEVICE;
  }
  return OS3D_OK;
}

int launch_build_bank(os3d_bank* b, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  const int L = b->L, nn = L + 1;
  BankArgs a;
  a.layout = b->layout;
  a.Nz = (int)b->dims[0];
  a.Ny = (int)b->dims[1];
  a.Nx = (int)b->dims[2];
  a.V = b->V;
  a.L = L;
  a.n_rows = b->n_unique;
  const double rhoN = 3.14159265358979323846;
  const double t = 2.0 * (b->params.gamma * rhoN) * (b->params.gamma * rhoN) / (1.0 + 2.0 * b->params.taylor_N);
  a.t_inv = 1.0 / t;
  a.taylor_N = b->params.taylor_N;
  a.S = (const uint4*)b->d.S;
  a.tab = b->d.tab;
  a.psi = b->d.psi;
  a.Mh = b->d.Mh;
  a.part = b->d.part;
  a.dc_value = b->dc_value;
  a.ncb = synth_padded_blocks(b->Npad / 16);
  a.kblocks = b->kblocks;
  a.mb = b->synth_mb;
  a.out_scale = b->synth_scale;
  const long long nblk = (b->V + kBankPts - 1) / kBankPts;
  void* tok = prof_start(st, PROF_BANK);
  switch (synth_sweep_blocks(b->Npad / 16)) {  // 16-column blocks per sweep
    case 1: launch_k(k_bank_synth<1>, dim3((unsigned)nblk), dim3(256), 0, st, a); break;
    case 2: launch_k(k_bank_synth<2>, dim3((unsigned)nblk), dim3(256), 0, st, a); break;
    case 3: launch_k(k_bank_synth<3>, dim3((unsigned)nblk), dim3(256), 0, st, a); break;
    case 4: launch_k(k_bank_synth<4>, dim3((unsigned)nblk), dim3(256), 0, st, a); break;
    case 5: launch_k(k_bank_synth<5>, dim3((unsigned)nblk), dim3(256), 0, st, a); break;
    default: launch_k(k_bank_synth<6>, dim3((unsigned)nblk), dim3(256), 0, st, a); break;
  }
  // algorithmic work of the contraction: 2 V (L+1)^2 n_rows flops
  prof_stop(tok, st, PROF_BANK, 0.0, 2.0 * (double)b->V * (double)(nn * nn) * (double)b->n_unique);
  int rc = check_launch("k_bank_synth");
  if (rc) return rc;
  launch_k(k_bank_reduce, dim3(1), dim3(1024), 0, st, (const double*)b->d.part, nblk, b->paired,
           b->d.part + 3 * nblk);
  if ((rc = check_launch("k_bank_reduce"))) return rc;
  const unsigned fin_blocks = (unsigned)std::min<long long>((b->V + 255) / 256, 8192);
  launch_k(k_M_finalize, dim3(fin_blocks), dim3(256), 0, st, (const double*)b->d.Mh, b->d.M, b->paired, b->layout,
           a.Nz, a.Ny, a.Nx, a.V, (const double*)(b->d.part + 3 * nblk));
  if ((rc = check_launch("k_M_finalize"))) return rc;
  double kn[2] = {0.0, 0.0};
  if (hipMemcpyAsync(kn, b->d.part + 3 * nblk, 2 * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    set_error("os3d_build_bank: reading kappa failed");
    return OS3D_EDEVICE;
  }
  b->kappa = kn[0];
  b->approx_norm = kn[1];
  return OS3D_OK;
}

template <int DT, int VPT>
static void launch_approx_k(const void* Ub, const float* sc, const os3d_bank* b, float inv_norm, float* o,
                            hipStream_t st) {
  const unsigned nblk = (unsigned)((b->V / VPT + 255) / 256);
  launch_k(k_approx_reconstruct<DT, VPT>, dim3(nblk), dim3(256), 0, st, Ub, sc, b->n_orients, b->V, inv_norm, o);
}

int launch_approx(const os3d_bank* b, const void* U, int dtype, const float* scales, int batch, float* f_out,
                  void* stream) {
  hipStream_t st = (hipStream_t)stream;
  const size_t ubytes = (dtype == OS3D_C64) ? 8 : 4;
  const float inv_norm = (float)(1.0 / b->approx_norm);
  for (int bi = 0; bi < batch; ++bi) {
    const void* Ub = (const char*)U + (size_t)bi * b->n_orients * b->V * ubytes;
    const float* sc = scales ? scales + (long long)bi * b->n_orients : nullptr;
    float* o = f_out + (long long)bi * b->V;
    // 16-byte loads when every orientation's row starts 16-byte aligned and
    // the volume is large enough to keep the GPU busy with fewer threads
    // (at 128^3 one voxel per thread measured faster: 0.16 against 0.20 ms)
    const bool al = ((uintptr_t)Ub % 16) == 0 && b->V >= (8LL << 20);
    if (dtype == OS3D_C64) {
      if (al && b->V % 2 == 0)
        launch_approx_k<OS3D_C64, 2>(Ub, sc, b, inv_norm, o, st);
      else
        launch_approx_k<OS3D_C64, 1>(Ub, sc, b, inv_norm, o, st);
    } else if (dtype == OS3D_BF16X2) {
      if (al && b->V % 4 == 0)
        launch_approx_k<OS3D_BF16X2, 4>(Ub, sc, b, inv_norm, o, st);
      else
        launch_approx_k<OS3D_BF16X2, 1>(Ub, sc, b, inv_norm, o, st);
    } else {
      if (al && b->V % 4 == 0)
        launch_approx_k<OS3D_F16X2, 4>(Ub, sc, b, inv_norm, o, st);
      else
        launch_approx_k<OS3D_F16X2, 1>(Ub, sc, b, inv_norm, o, st);
    }
    int rc = check_launch("k_approx_reconstruct");
    if (rc) return rc;
  }
  return OS3D_OK;
}

int launch_export_psi(const os3d_bank* b, int i, float* out, void* stream) {
  const float* row = b->d.psi + (long long)b->row_of[i] * b->V;
  const unsigned nb = (unsigned)std::min<long long>((b->V + 255) / 256, 8192);
  launch_k(k_export, dim3(nb), dim3(256), 0, (hipStream_t)stream, row, b->conj_of[i], b->layout,
                     (int)b->dims[0], (int)b->dims[1], (int)b->dims[2], b->V, (float)b->kappa, out);
  return check_launch("k_export");
}

int launch_export_M(const os3d_bank* b, float* out, void* stream) {
  const unsigned nb = (unsigned)std::min<long long>((b->V + 255) / 256, 8192);
  launch_k(k_export, dim3(nb), dim3(256), 0, (hipStream_t)stream, b->d.M, 0, b->layout, (int)b->dims[0],
                     (int)b->dims[1], (int)b->dims[2], b->V, 1.f, out);
  return check_launch("k_export");
}

}  // namespace os3d
