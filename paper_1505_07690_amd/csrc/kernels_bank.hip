// Wavelet-bank synthesis on gfx950 (Sec. 3, Eqs. 9-19).
//
// For every DFT frequency k the rotated angular profiles of all stored bank
// rows are one row of a dense contraction
//     h[k, i] = sum_{(l,m)} Y_lm(w_hat_k) S[(l,m), i]
// (S: steering matrix a_l sqrt(4 pi/(2l+1)) Y_lm(n_i), the addition-theorem
// form of the Wigner-D rotation of Eqs. 17-19).  Each workgroup owns 256
// frequency points: every thread generates its point's associated Legendre
// values Q_l^m for one order m at a time with the FP64 normalised recursion
// and rounds them to FP32 into LDS; the real harmonics of that order are
// Q_l^m times the real and imaginary parts of (x + iy)^m, applied in
// registers to the MFMA A operand.  The four waves run
// v_mfma_f32_16x16x4_f32 over the chunk against the chunk's rows of S
// (prefetched during the recursion and staged in LDS).  The epilogue
// multiplies by the FP64 radial window g(rho) (Eq. 10), applies the Nyquist
// and DC rules, writes the bank rows and accumulates sum_i psi_i^2 (Eq. 9)
// and sum_i psi_i in FP64 with a fixed-order cross-lane tree; the
// workgroup's sums of both over the normalisation band go to one partial
// record per workgroup.  The rows are stored without the normaliser kappa
// (known only once every partial is in): the transforms apply kappa as a
// scalar where they multiply by the bank.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "launch.h"
#include "layout4.h"
#include "os3d_internal.h"

namespace os3d {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kBankPts = 256;   // frequency points per workgroup
constexpr int kYStride = 272;   // LDS row stride (floats) of the K-chunk buffer
constexpr int kColBlocks = 3;                  // 16-column MFMA blocks per sweep (at most)
constexpr int kColsPerSweep = 16 * kColBlocks;
constexpr int kStageRegs = 11;                 // steering values prefetched per thread and chunk

struct BankArgs {
  int layout;  // storage order of the frequency points (natural or four-step tiles)
  int Nz, Ny, Nx;
  long long V;
  int L, Npad, n_rows, maxpad;
  double t_inv;      // 1 / t of Eq. (10)
  int taylor_N;
  double dc_value;   // a_0 / sqrt(4 pi)
  const float* S;    // [K][Npad]
  const double* tab; // qmm[L+1] | alm[(L+1)^2] | blm[(L+1)^2]
  const int* koff;   // chunk offsets [L+1] | padded lengths [L+1]
  float* psi;        // [n_rows][V]
  double* Mh;        // [V]
  double* part;      // [gridDim.x][3]: band sums of Mh and of sum_i psi_i, band count
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

// One K-chunk per m: the rows Q_l^m (l = m..L, times sqrt 2 for m > 0) of
// the 256 points are generated once into LDS; the cos rows of the chunk are
// Q cos(m phi) and the sin rows Q sin(m phi), so the A operand of either half
// is the same LDS value times the point's (x + iy)^m real or imaginary part,
// applied in registers.  Half the LDS of storing both halves: three
// workgroups per CU.
template <int NS, int CB>
__global__ __launch_bounds__(256, 3) void k_bank_synth(BankArgs a) {
  extern __shared__ float Ybuf[];  // [qpad_max][kYStride], then cos and sin steering rows [2][qpad_max][cols]
  __shared__ double gsh[kBankPts];
  __shared__ double Msh[kBankPts];
  __shared__ double Ash[kBankPts];
  __shared__ float crsh[kBankPts], cish[kBankPts];
  __shared__ int dcsh[kBankPts], bandsh[kBankPts];

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const long long p0 = (long long)blockIdx.x * kBankPts;
  const long long p = p0 + tid;
  const bool valid = p < a.V;
  const int L = a.L, nn = L + 1;
  const double* qmm = a.tab;
  const double* alm = a.tab + nn;
  const double* blm = a.tab + nn + nn * nn;
  const int* koff = a.koff;
  float* Scos = Ybuf + a.maxpad * kYStride;

  // this thread's frequency point
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
  dcsh[tid] = dc;
  bandsh[tid] = band ? 1 : 0;
  Msh[tid] = 0.0;
  double asum = 0.0;  // this lane's share of the band sum of sum_i psi_raw

  constexpr int kCols = 16 * CB;  // columns per sweep
  // NS sweeps of kCols columns share each order's recursion: one FP64 pass of
  // Q_l^m per order and column group, the steering rows of every sweep
  // staged in turn
  // steering values prefetched in registers during the recursion (fewer when
  // two sweeps' accumulators are live)
  constexpr int SR = (NS == 1) ? kStageRegs : 4;
  for (int c0 = 0; c0 < a.Npad; c0 += NS * kCols) {
    floatx4 acc[NS][4][CB];
#pragma unroll
    for (int w = 0; w < NS; ++w)
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < CB; ++c) acc[w][r][c] = floatx4{0.f, 0.f, 0.f, 0.f};

    double cr = 1.0, ci = 0.0;  // (x + i y)^m of the unit frequency direction
    for (int m = 0; m <= L; ++m) {
      if (m > 0) {
        double nr = cr * ux - ci * uy, ni = cr * uy + ci * ux;
        cr = nr;
        ci = ni;
      }
      const int nq = nn - m;            // rows l = m..L
      const int qpad = (nq + 3) & ~3;
      // issue the loads of the chunk's cos and sin steering rows (the first
      // sweep's columns) first, branch-free, so that they complete during
      // the recursion
      const float* Sm = a.S + (long long)koff[m] * a.Npad;
      const int half = qpad * kCols;
      float sv[SR];
#pragma unroll
      for (int u = 0; u < SR; ++u) {
        const int idx = u * kBankPts + tid;
        const int part = idx >= half, id2 = idx - part * half;
        const int kr = id2 / kCols, cc = id2 - kr * kCols;
        const bool ok = idx < 2 * half && kr < nq && c0 + cc < a.Npad && (m > 0 || part == 0);
        const float v = Sm[ok ? (long long)(kr + part * nq) * a.Npad + c0 + cc : 0];
        sv[u] = ok ? v : 0.f;
      }
      // Q_l^m for l = m..L (sinus power factored out), FP64 recursion
      {
        double q2 = 0.0, q1 = qmm[m];
        const double sc = (m == 0) ? 1.0 : 1.4142135623730950488;
        for (int l = m; l <= L; ++l) {
          double q;
          if (l == m)
            q = qmm[m];
          else if (l == m + 1)
            q = sqrt(2.0 * m + 3.0) * uz * qmm[m];
          else
            q = alm[l * nn + m] * (uz * q1 - blm[l * nn + m] * q2);
          if (l > m) q2 = q1;
          q1 = q;
          Ybuf[(l - m) * kYStride + tid] = (float)(sc * q);
        }
        for (int kk = nq; kk < qpad; ++kk) Ybuf[kk * kYStride + tid] = 0.f;
        crsh[tid] = (float)cr;
        cish[tid] = (float)ci;
      }
#pragma unroll
      for (int w = 0; w < NS; ++w) {
        const int cs = c0 + w * kCols;
        if (cs >= a.Npad) break;  // uniform
        if (w == 0) {
          // stage the first sweep's rows in LDS (the values past SR * 256 are
          // loaded in the loop below)
#pragma unroll
          for (int u = 0; u < SR; ++u)
            if (u * kBankPts + tid < 2 * half) Scos[u * kBankPts + tid] = sv[u];
        } else {
          __syncthreads();  // every wave is done with the previous sweep's rows
        }
        for (int idx = (w == 0 ? SR * kBankPts : 0) + tid; idx < 2 * half; idx += kBankPts) {
          const int part = idx >= half, id2 = idx - part * half;
          const int kr = id2 / kCols, cc = id2 - kr * kCols;
          const bool ok = kr < nq && cs + cc < a.Npad && (m > 0 || part == 0);
          Scos[idx] = ok ? Sm[(long long)(kr + part * nq) * a.Npad + cs + cc] : 0.f;
        }
        __syncthreads();
        float crv[4], civ[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          crv[r] = crsh[wave * 64 + r * 16 + (lane & 15)];
          civ[r] = cish[wave * 64 + r * 16 + (lane & 15)];
        }
        const float* Sc = Scos;
        const float* Ss = Scos + half;  // the sin rows follow the cos rows
        // the cos rows, then (m > 0: m is uniform, a scalar branch) the sin
        // rows, which are zero for m = 0; two loops also keep fewer steering
        // values live than one loop over both (measured 25.9 against 26.6 ms
        // at 256^3 x 81 rows, L = 24)
        for (int k0 = 0; k0 < qpad; k0 += 4) {
          const int kr = k0 + (lane >> 4);
          float q[4], bc[CB];
#pragma unroll
          for (int r = 0; r < 4; ++r) q[r] = Ybuf[kr * kYStride + wave * 64 + r * 16 + (lane & 15)];
#pragma unroll
          for (int c = 0; c < CB; ++c) bc[c] = Sc[kr * kCols + c * 16 + (lane & 15)];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const float ac = q[r] * crv[r];
#pragma unroll
            for (int c = 0; c < CB; ++c)
              acc[w][r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(ac, bc[c], acc[w][r][c], 0, 0, 0);
          }
        }
        if (m > 0) {
          for (int k0 = 0; k0 < qpad; k0 += 4) {
            const int kr = k0 + (lane >> 4);
            float q[4], bs[CB];
#pragma unroll
            for (int r = 0; r < 4; ++r) q[r] = Ybuf[kr * kYStride + wave * 64 + r * 16 + (lane & 15)];
#pragma unroll
            for (int c = 0; c < CB; ++c) bs[c] = Ss[kr * kCols + c * 16 + (lane & 15)];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const float as = q[r] * civ[r];
#pragma unroll
              for (int c = 0; c < CB; ++c)
                acc[w][r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(as, bs[c], acc[w][r][c], 0, 0, 0);
            }
          }
        }
      }
      __syncthreads();
    }

    // epilogue: psi_raw = g * h (DC: isotropic), bank rows, FP64 sums of
    // squares and of values
#pragma unroll
    for (int w = 0; w < NS; ++w) {
      const int cs = c0 + w * kCols;
      if (cs >= a.Npad) break;
      const int ncb = min(kCols, a.Npad - cs) / 16;
      double mh[4][4];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int i = 0; i < 4; ++i) mh[r][i] = 0.0;
#pragma unroll
      for (int c = 0; c < CB; ++c) {
        if (c >= ncb) continue;
        const int col = cs + c * 16 + (lane & 15);
        const bool colok = col < a.n_rows;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int pt = wave * 64 + r * 16 + 4 * (lane >> 4) + i;
            const long long gp = p0 + pt;
            double h = dcsh[pt] ? a.dc_value : (double)acc[w][r][c][i];
            float v = (float)(gsh[pt] * h);
            if (colok && gp < a.V) a.psi[(long long)col * a.V + gp] = v;
            if (colok) {
              mh[r][i] += (double)v * (double)v;
              if (bandsh[pt]) asum += (double)v;
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
  }
  __syncthreads();
  const double mt = Msh[tid];
  if (valid) a.Mh[p] = mt;
  // the workgroup's band sums, by a fixed tree (deterministic); Msh and
  // Ash are reused as the tree's buffers
  double cnt = band ? 1.0 : 0.0;
  double ms = band ? mt : 0.0, as = asum;
  __syncthreads();
  Msh[tid] = ms;
  Ash[tid] = as;
  gsh[tid] = cnt;
  __syncthreads();
  for (int w = kBankPts / 2; w > 0; w >>= 1) {
    if (tid < w) {
      Msh[tid] += Msh[tid + w];
      Ash[tid] += Ash[tid + w];
      gsh[tid] += gsh[tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) {
    a.part[3 * (long long)blockIdx.x] = Msh[0];
    a.part[3 * (long long)blockIdx.x + 1] = Ash[0];
    a.part[3 * (long long)blockIdx.x + 2] = gsh[0];
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
        acc += ((const float2*)U)[e].x;
      else
        acc += approx_re<DT>(((const unsigned int*)U)[e]) * scales[i];
    }
    out[p] = acc * inv_norm;
  } else {
    float acc[VPT];
#pragma unroll
    for (int v = 0; v < VPT; ++v) acc[v] = 0.f;
#pragma unroll 4
    for (int i = 0; i < n_orients; ++i) {
      const long long e = (long long)i * V + p;
      if constexpr (DT == OS3D_C64) {
        static_assert(VPT == 2, "complex64 scores: two per 16-byte load");
        const float4 w = *(const float4*)((const float2*)U + e);
        acc[0] += w.x;
        acc[1] += w.z;
      } else {
        static_assert(VPT == 4, "16-bit scores: four per 16-byte load");
        const float sc = scales[i];
        const uint4 w = *(const uint4*)((const unsigned int*)U + e);
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
  a.Npad = b->Npad;
  a.n_rows = b->n_unique;
  const double rhoN = 3.14159265358979323846;
  const double t = 2.0 * (b->params.gamma * rhoN) * (b->params.gamma * rhoN) / (1.0 + 2.0 * b->params.taylor_N);
  a.t_inv = 1.0 / t;
  a.taylor_N = b->params.taylor_N;
  a.S = b->d.S;
  a.tab = b->d.tab;
  a.koff = (const int*)(b->d.tab + nn + 2 * nn * nn);
  a.psi = b->d.psi;
  a.Mh = b->d.Mh;
  a.part = b->d.part;
  a.dc_value = b->dc_value;
  // LDS rows per chunk: the L + 1 - m values Q_l^m, padded to 4 (largest at m = 0)
  const int maxpad = (nn + 3) / 4 * 4;
  a.maxpad = maxpad;
  const long long nblk = (b->V + kBankPts - 1) / kBankPts;
  // the stored rows in one sweep of 32 or 48 columns, or two 48-column
  // sweeps per recursion
  const int cb = (b->Npad <= 32) ? 2 : 3;
  const int ns = (b->Npad > kColsPerSweep) ? 2 : 1;
  size_t lds = (size_t)maxpad * (kYStride + 2 * 16 * cb) * sizeof(float);
  const void* kfn = ns == 2 ? (const void*)k_bank_synth<2, 3>
                            : (cb == 2 ? (const void*)k_bank_synth<1, 2> : (const void*)k_bank_synth<1, 3>);
  if (hipFuncSetAttribute(kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) {
    set_error("k_bank_synth: cannot reserve LDS");
    return OS3D_EDEVICE;
  }
  void* tok = prof_start(st, PROF_BANK);
  if (ns == 2)
    launch_k(k_bank_synth<2, 3>, dim3((unsigned)nblk), dim3(256), lds, st, a);
  else if (cb == 2)
    launch_k(k_bank_synth<1, 2>, dim3((unsigned)nblk), dim3(256), lds, st, a);
  else
    launch_k(k_bank_synth<1, 3>, dim3((unsigned)nblk), dim3(256), lds, st, a);
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
