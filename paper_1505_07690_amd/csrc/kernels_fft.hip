// 3D DFT passes of the orientation-score transform (Eqs. 7-8) on gfx950.
//
// A pass computes the length-N DFT of every line of a volume along one axis.
// A workgroup owns W consecutive lines (W * N <= 4096): it stages them in
// LDS with coalesced global accesses (x-lines are contiguous; y- and z-lines
// are read as W consecutive x positions per row), runs the mixed-radix
// Stockham stages (radix 16, 8, 4, 2, 5, 3) between two LDS buffers, and
// writes the lines back.  The first and last pass of each 3D transform fuse
// the per-voxel work of the method into their global loads and stores:
//   * spectral multiply psi_hat_i * F (forward, Eq. 7),
//   * antipodal pair store U_n and U_{-n} = conj(U_n), optionally rounded to
//     16-bit pairs with a per-orientation power-of-two scale,
//   * pair load U_n + conj(U_{-n}) and the weighted orientation sum
//     X += psi_hat_n * DFT(.) over a batch of pairs (Eq. 8),
//   * X / max(M, eps) (Sec. 3.1) and the real part of the inverse.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>

#include "fft_pass.h"
#include "launch.h"
#include "layout4.h"

namespace os3d {

constexpr int kThreads = 256;
constexpr int kTile = 4096;      // complex elements per workgroup tile
constexpr int kEPT = kTile / kThreads;

template <int R>
__device__ __forceinline__ void stage(const PassArgs& a, const float2* __restrict__ cur, float2* __restrict__ nxt,
                                      int Ns, int nl) {
  const int N = a.N, NR = N / R, tstep = N / (Ns * R);
  const int total = a.W * NR;
  for (int b = threadIdx.x; b < total; b += kThreads) {
    const int w = b / NR, j = b - w * NR;
    if (w >= nl) continue;
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = cur[lidx(a.LS, w, j + r * NR)];
    const int k = j % Ns;
    if (Ns > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        float2 t = a.tw[k * r * tstep];
        if (a.sgn > 0.f) t.y = -t.y;
        v[r] = cmul(v[r], t);
      }
    }
    dft_r<R>(v, a.sgn);
    const int base = (j - k) * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) nxt[lidx(a.LS, w, base + r * Ns)] = v[r];
  }
}

template <int LM, int SM, int DT>
__global__ __launch_bounds__(kThreads) void k_pass(PassArgs a) {
  extern __shared__ float2 lds[];
  __shared__ float red[kThreads];
  const int tile = blockIdx.x;
  const long long line0 = (long long)tile * a.W;
  const int nl = (int)min((long long)a.W, a.lines - line0);
  const int tsize = a.W * a.N;
  const bool contiguous = (a.axis == 2);
  const int bufsz = a.W * a.LS;
  float2* buf0 = lds;
  float2* buf1 = lds + bufsz;

  // SM_ACCUM walks the whole pair batch inside one workgroup; other modes take
  // their pair from blockIdx.y.
  const int jb = (SM == SM_ACCUM) ? 0 : blockIdx.y;
  const int je = (SM == SM_ACCUM) ? a.nb : blockIdx.y + 1;
  float2 acc[kEPT];
#pragma unroll
  for (int e = 0; e < kEPT; ++e) acc[e] = make_float2(0.f, 0.f);

  for (int j = jb; j < je; ++j) {
    // ---------------------------------------------------------------- load
    float asum = 0.f;
#pragma unroll
    for (int e = 0; e < kEPT; ++e) {
      const int idx = threadIdx.x + e * kThreads;
      if (idx < tsize) {
        int w, n;
        if (contiguous) {
          w = idx / a.N;
          n = idx - w * a.N;
        } else {
          n = idx / a.W;
          w = idx - n * a.W;
        }
        if (w < nl) {
          const long long g = gaddr(a, line0 + w, n);
          const float2 v = load_elem<LM, DT>(a, j, g, asum);
          buf0[lidx(a.LS, w, n)] = v;
        }
      }
    }
    if constexpr (LM == LM_MULBANK) {
      if (a.partial) {
        red[threadIdx.x] = asum;
        __syncthreads();
        for (int s = kThreads / 2; s > 0; s >>= 1) {
          if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
          __syncthreads();
        }
        if (threadIdx.x == 0) a.partial[(long long)j * gridDim.x + tile] = red[0];
      }
    }
    __syncthreads();

    // -------------------------------------------------------------- stages
    float2* cur = buf0;
    float2* nxt = buf1;
    int Ns = 1;
    for (int s = 0; s < a.nst; ++s) {
      const int R = a.radix[s];
      switch (R) {
        case 16: stage<16>(a, cur, nxt, Ns, nl); break;
        case 8: stage<8>(a, cur, nxt, Ns, nl); break;
        case 4: stage<4>(a, cur, nxt, Ns, nl); break;
        case 2: stage<2>(a, cur, nxt, Ns, nl); break;
        case 5: stage<5>(a, cur, nxt, Ns, nl); break;
        default: stage<3>(a, cur, nxt, Ns, nl); break;
      }
      __syncthreads();
      float2* t = cur;
      cur = nxt;
      nxt = t;
      Ns *= R;
    }

    // --------------------------------------------------------------- store
#pragma unroll
    for (int e = 0; e < kEPT; ++e) {
      const int idx = threadIdx.x + e * kThreads;
      if (idx < tsize) {
        int w, n;
        if (contiguous) {
          w = idx / a.N;
          n = idx - w * a.N;
        } else {
          n = idx / a.W;
          w = idx - n * a.W;
        }
        if (w < nl) {
          const long long g = gaddr(a, line0 + w, n);
          store_elem<SM, DT>(a, j, g, cur[lidx(a.LS, w, n)], acc[e]);
        }
      }
    }
    if constexpr (SM == SM_ACCUM) __syncthreads();  // buf0 is reloaded for the next pair
  }

  if constexpr (SM == SM_ACCUM) {
#pragma unroll
    for (int e = 0; e < kEPT; ++e) {
      const int idx = threadIdx.x + e * kThreads;
      if (idx < tsize) {
        int w, n;
        if (contiguous) {
          w = idx / a.N;
          n = idx - w * a.N;
        } else {
          n = idx / a.W;
          w = idx - n * a.W;
        }
        if (w < nl) {
          const long long g = gaddr(a, line0 + w, n);
          accum_flush(a, g, acc[e]);
        }
      }
    }
  }
}


// ---------------------------------------------------------------------------
// Power-of-two lines, N = 16 * R2 with R2 in {4, 8, 16}: every thread keeps
// 16 elements of one line in registers.  Stage 1 is a radix-16 DFT of the
// elements s + (N/16) r loaded straight from global memory; one LDS exchange
// transposes the line; stage 2 applies the twiddles W_N^(j r) (LDS table) and
// radix-R2 DFTs whose outputs are already in natural order, stored straight
// to global memory.  Tiles are N/16 threads per line x (256 / (N/16)) lines.
// ---------------------------------------------------------------------------
template <int N>
struct FastCfg {
  static constexpr int TL = N / 16;        // threads per line
  static constexpr int W = 256 / TL;       // lines per workgroup
  static constexpr int R2 = N / 16;        // second-stage radix
  static constexpr int B2 = 16 / R2;       // second-stage butterflies per thread
  static constexpr int LS = N + N / 16 + 1;
};

__device__ __forceinline__ int padn(int n) { return n + (n >> 4); }

template <int N, int AXIS>
__device__ __forceinline__ long long gaddr_t(const PassArgs& a, long long line, int n) {
  if constexpr (AXIS == 2) {
    return line * N + n;
  } else if constexpr (AXIS == 1) {
    const long long z = line / a.Nx, x = line - z * a.Nx;
    return (z * N + n) * a.Nx + x;
  } else {
    return (long long)n * a.Ny * a.Nx + line;
  }
}

template <int N, int AXIS, int LM, int SM, int DT>
__global__ __launch_bounds__(kThreads) void k_fast(PassArgs a) {
  using C = FastCfg<N>;
  __shared__ float2 buf[C::W * C::LS];
  __shared__ float2 twl[N];
  __shared__ float red[kThreads];
  const int t = threadIdx.x;
  int w, s;
  if constexpr (AXIS == 2) {
    s = t % C::TL;
    w = t / C::TL;
  } else {
    w = t % C::W;
    s = t / C::W;
  }
  const long long line = (long long)blockIdx.x * C::W + w;
  const bool valid = line < a.lines;
  for (int i = t; i < N; i += kThreads) {
    float2 v = a.tw[i];
    if (a.sgn > 0.f) v.y = -v.y;
    twl[i] = v;
  }
  const int jb = (SM == SM_ACCUM) ? 0 : blockIdx.y;
  const int je = (SM == SM_ACCUM) ? a.nb : blockIdx.y + 1;
  float2 acc[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) acc[e] = make_float2(0.f, 0.f);
  __syncthreads();

  for (int j = jb; j < je; ++j) {
    float2 v[16];
    float asum = 0.f;
    if (valid) {
      const long long g0 = gaddr_t<N, AXIS>(a, line, s);
      const long long dn = gaddr_t<N, AXIS>(a, line, s + C::TL) - g0;
      load_k<LM, DT, 16>(a, j, g0, dn, v, asum);
    } else {
#pragma unroll
      for (int r = 0; r < 16; ++r) v[r] = make_float2(0.f, 0.f);
    }
    if constexpr (LM == LM_MULBANK) {
      if (a.partial) {
        red[t] = asum;
        __syncthreads();
        for (int h = kThreads / 2; h > 0; h >>= 1) {
          if (t < h) red[t] += red[t + h];
          __syncthreads();
        }
        if (t == 0) a.partial[(long long)j * gridDim.x + blockIdx.x] = red[0];
      }
    }
    dft16(v, a.sgn);
#pragma unroll
    for (int r = 0; r < 16; ++r) buf[w * C::LS + padn(s * 16 + r)] = v[r];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < C::B2; ++q) {
      const int jj = s + C::TL * q;
      float2 u[C::R2];
#pragma unroll
      for (int r = 0; r < C::R2; ++r) u[r] = buf[w * C::LS + padn(jj + 16 * r)];
#pragma unroll
      for (int r = 1; r < C::R2; ++r) u[r] = cmul(u[r], twl[jj * r]);
      dft_r<C::R2>(u, a.sgn);
      if (valid) {
        const long long g0 = gaddr_t<N, AXIS>(a, line, jj);
        const long long dn = gaddr_t<N, AXIS>(a, line, jj + 16) - g0;
        float2 ac[C::R2];
#pragma unroll
        for (int r = 0; r < C::R2; ++r) ac[r] = acc[q * C::R2 + r];
        store_k<SM, DT, C::R2>(a, j, g0, dn, u, ac);
#pragma unroll
        for (int r = 0; r < C::R2; ++r) acc[q * C::R2 + r] = ac[r];
      }
    }
    __syncthreads();
  }
  if constexpr (SM == SM_ACCUM) {
    if (valid) {
#pragma unroll
      for (int q = 0; q < C::B2; ++q) {
        const long long g0 = gaddr_t<N, AXIS>(a, line, s + C::TL * q);
        const long long dn = gaddr_t<N, AXIS>(a, line, s + C::TL * q + 16) - g0;
        float2 ac[C::R2];
#pragma unroll
        for (int r = 0; r < C::R2; ++r) ac[r] = acc[q * C::R2 + r];
        flush_k<C::R2>(a, g0, dn, ac);
      }
    }
  }
}

// Per-orientation power-of-two scale for 16-bit score storage from the
// bound max|U_i| <= (1/V) sum_k |psi_hat_i[k] F[k]|: fp16 maps the bound to
// at most 2^15, bf16 to at most 1.  Fixed-order FP64 sum (deterministic).
__global__ __launch_bounds__(256) void k_scales(const float* partial, int ntiles, PassArgs a, int dtype,
                                                float* scales) {
  __shared__ double red[256];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int t = threadIdx.x; t < ntiles; t += 256) s += (double)partial[(long long)j * ntiles + t];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double bound = red[0] / (double)a.V * (1.0 + 1e-5);
    float sc = 1.f;
    if (bound > 0.0) {
      int e;
      frexp(bound, &e);  // bound <= 2^e
      sc = (float)ldexp(1.0, dtype == OS3D_F16X2 ? e - 15 : e);
    }
    scales[a.oa[j]] = sc;
    if (a.ob[j] >= 0) scales[a.ob[j]] = sc;
  }
}

void launch_scales(const float* partial, int ntiles, const PassArgs& a, int dtype, float* scales, int nb,
                   hipStream_t st) {
  launch_k(k_scales, dim3(nb), dim3(256), 0, st, partial, ntiles, a, dtype, scales);
}

static int check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return OS3D_EDEVICE;
  }
  return OS3D_OK;
}

static void setup_axis(const os3d_bank* b, int axis, PassArgs& a) {
  a.axis = axis;
  a.Nz = (int)b->dims[0];
  a.Ny = (int)b->dims[1];
  a.Nx = (int)b->dims[2];
  a.V = b->V;
  const AxisPlan& p = b->plan[axis];
  a.N = p.n;
  a.nst = p.nstages;
  for (int s = 0; s < kMaxStages; ++s) a.radix[s] = (s < p.nstages) ? p.radix[s] : 0;
  a.W = std::min(256, std::max(1, kTile / a.N));
  a.LS = a.N + (a.N >> 4) + 1;
  a.lines = a.V / a.N;
  a.tw = (const float2*)b->d.tw[axis];
}

static size_t pass_lds(const PassArgs& a) { return (size_t)2 * a.W * a.LS * sizeof(float2); }

// Lines per workgroup of the kernel that run_pass launches for this pass.
static int tile_lines(const PassArgs& a) {
  if (a.N == 256) return FastCfg<256>::W;
  if (a.N == 128) return FastCfg<128>::W;
  if (a.N == 64) return FastCfg<64>::W;
  return a.W;
}

// ---------------------------------------------------------------------------
// Optional per-kernel timing: a pair of HIP events per launch, stamped by the
// runtime with the kernel's start and end (launch_k), with the algorithmic
// bytes each launch must move; every launch, or only those of one slot (so
// that timing one kernel leaves the others' launches untouched).
// Process-wide and meant for one host thread (the benchmark); events are
// reused across enable calls.
// ---------------------------------------------------------------------------
static_assert((int)kProfBank == (int)PROF_BANK, "profiler slot of the bank kernel");
static const char* kKernelNames[kProfCount] = {
    "dft_f_first_real_in", "dft_f_mid", "dft_f_last", "fwd_first_mul_bank", "fwd_scales", "fwd_mid",
    "fwd_last_store_scores", "rec_first_load_scores", "rec_mid", "rec_last_accumulate", "inv_first_divide_M",
    "inv_mid", "inv_last_real_out", "bank_synth_mfma"};

struct ProfRec {
  int kid;
  hipEvent_t e0, e1;
  double alg_bytes, alg_flops;
  bool launched;
};
static int g_prof_mode = 0;  // 0 off, 1 every launch, 2 + k only the launches of slot k
static std::vector<ProfRec> g_prof;
static std::vector<hipEvent_t> g_event_pool;
static thread_local ProfRec* t_pending = nullptr;

static bool take_event(hipEvent_t* e) {
  if (!g_event_pool.empty()) {
    *e = g_event_pool.back();
    g_event_pool.pop_back();
    return true;
  }
  return hipEventCreate(e) == hipSuccess;
}

void* prof_start(void* stream, int kid) {
  (void)stream;
  if (g_prof_mode == 0 || (g_prof_mode >= 2 && kid != g_prof_mode - 2)) return nullptr;
  ProfRec* r = new ProfRec();
  r->launched = false;
  if (!take_event(&r->e0)) {
    delete r;
    return nullptr;
  }
  if (!take_event(&r->e1)) {
    g_event_pool.push_back(r->e0);
    delete r;
    return nullptr;
  }
  t_pending = r;
  return r;
}

bool prof_take(hipEvent_t* e0, hipEvent_t* e1) {
  ProfRec* r = t_pending;
  if (!r) return false;
  t_pending = nullptr;
  r->launched = true;
  *e0 = r->e0;
  *e1 = r->e1;
  return true;
}

void prof_stop(void* token, void* stream, int kid, double alg_bytes, double alg_flops) {
  (void)stream;
  if (!token) return;
  ProfRec* r = (ProfRec*)token;
  if (t_pending == r) t_pending = nullptr;
  if (r->launched) {
    r->kid = kid;
    r->alg_bytes = alg_bytes;
    r->alg_flops = alg_flops;
    g_prof.push_back(*r);
  } else {  // no launch between start and stop: nothing to time
    g_event_pool.push_back(r->e0);
    g_event_pool.push_back(r->e1);
  }
  delete r;
}

template <int LM, int SM, int N, int AXIS, int DT>
static void launch_fast(const PassArgs& a, int grid_y, hipStream_t st) {
  const long long tiles = (a.lines + FastCfg<N>::W - 1) / FastCfg<N>::W;
  launch_k((k_fast<N, AXIS, LM, SM, DT>), dim3((unsigned)tiles, grid_y), dim3(kThreads), 0, st, a);
}

template <int LM, int SM, int N, int DT>
static void launch_fast_axis(const PassArgs& a, int grid_y, hipStream_t st) {
  if constexpr (LM == LM_UIN || SM == SM_UOUT) {
    launch_fast<LM, SM, N, 2, DT>(a, grid_y, st);  // scores are read and written along x only
  } else {
    if (a.axis == 0) launch_fast<LM, SM, N, 0, DT>(a, grid_y, st);
    else if (a.axis == 1) launch_fast<LM, SM, N, 1, DT>(a, grid_y, st);
    else launch_fast<LM, SM, N, 2, DT>(a, grid_y, st);
  }
}

template <int LM, int SM, int DT>
static void launch_pass_dt(const PassArgs& a, int grid_y, hipStream_t st) {
  if (a.N == 256) {
    launch_fast_axis<LM, SM, 256, DT>(a, grid_y, st);
  } else if (a.N == 128) {
    launch_fast_axis<LM, SM, 128, DT>(a, grid_y, st);
  } else if (a.N == 64) {
    launch_fast_axis<LM, SM, 64, DT>(a, grid_y, st);
  } else {
    const long long tiles = (a.lines + a.W - 1) / a.W;
    static bool attr_set = false;
    if (!attr_set) {
      (void)hipFuncSetAttribute((const void*)k_pass<LM, SM, DT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                96 * 1024);
      attr_set = true;
    }
    launch_k((k_pass<LM, SM, DT>), dim3((unsigned)tiles, grid_y), dim3(kThreads), pass_lds(a), st, a);
  }
}

template <int LM, int SM>
static int run_pass(int kid, double alg, const PassArgs& a, int grid_y, hipStream_t st) {
  void* tok = prof_start(st, kid);
  if constexpr (LM == LM_UIN || SM == SM_UOUT) {
    if (a.dtype == OS3D_BF16X2) launch_pass_dt<LM, SM, OS3D_BF16X2>(a, grid_y, st);
    else if (a.dtype == OS3D_F16X2) launch_pass_dt<LM, SM, OS3D_F16X2>(a, grid_y, st);
    else launch_pass_dt<LM, SM, OS3D_C64>(a, grid_y, st);
  } else {
    launch_pass_dt<LM, SM, OS3D_C64>(a, grid_y, st);
  }
  prof_stop(tok, st, kid, alg, 0.0);
  return check_launch(kKernelNames[kid]);
}

// Whole-plane pass of the two-pass path (kernels_plane.hip).
template <int LM, int SM>
static int run_plane(int kid, double alg, const PassArgs& a, int grid_y, hipStream_t st) {
  void* tok = prof_start(st, kid);
  launch_plane<LM, SM>(a, grid_y, st);
  prof_stop(tok, st, kid, alg, 0.0);
  return check_launch(kKernelNames[kid]);
}

// Arguments of a whole-plane pass (the x twiddles serve both plane axes).
static PassArgs plane_args(const os3d_bank* b, float sgn, int nb) {
  PassArgs a = {};
  setup_axis(b, 2, a);
  a.sgn = sgn;
  a.nb = nb;
  return a;
}

// Algorithmic score bytes of one launch over nb stored rows: every stored
// row stands for one orientation, or two with its antipode.
static double score_bytes(const os3d_bank* b, const PassArgs& a, int nb, size_t ubytes) {
  int n = 0;
  for (int j = 0; j < nb; ++j) n += (a.ob[j] >= 0) ? 2 : 1;
  return (double)n * (double)b->V * (double)ubytes;
}

// Orientation pairs per launch: larger batches amortise the spectrum loads
// and the orientation-sum read-modify-write and keep more workgroups in
// flight; each pair costs one intermediate volume of workspace.
static int pair_batch(const os3d_bank* b) {
  int nb = kMaxBatch;
  if (const char* e = getenv("OS3D_PAIR_BATCH")) nb = atoi(e);
  nb = std::max(1, std::min(std::min(nb, kMaxBatch), b->n_unique));
  // one complex intermediate volume per pair of a launch: at most 8 GiB of them
  nb = (int)std::max(1LL, std::min((long long)nb, (8LL << 30) / (b->V * (long long)sizeof(float2))));
  // the same number of pairs in every launch (no short last launch)
  const int launches = (b->n_unique + nb - 1) / nb;
  return (b->n_unique + launches - 1) / launches;
}

size_t workspace_bytes(const os3d_bank* b) {
  const int nb = pair_batch(b);
  long long max_tiles = 0;
  for (int ax = 0; ax < 3; ++ax) {
    const int n = b->plan[ax].n;
    const int W = std::min(256, std::max(1, kTile / n));
    max_tiles = std::max(max_tiles, (long long)((b->V / n + W - 1) / W));  // fast kernels use W = 4096 / n too
  }
  // F or X, one intermediate per pair of the batch; processing via scores (F, X, and two
  // buffers per pair of a half batch) needs one volume more
  return (size_t)(2 + std::max(nb, 2)) * b->V * sizeof(float2) + (size_t)nb * max_tiles * sizeof(float) + 256;
}

// forward DFT of one real volume into F (three passes, in place after the first)
static int dft_real_volume(const os3d_bank* b, const float* f, float2* F, hipStream_t st) {
  int rc;
  if (b->plane) {
    PassArgs a = plane_args(b, -1.f, 1);
    a.src_r = f;
    a.dst_c = F;
    if ((rc = run_plane<LM_REAL, SM_C>(kProfDftFirst, 4.0 * b->V, a, 1, st))) return rc;
    PassArgs c = {};
    setup_axis(b, 0, c);
    c.sgn = -1.f;
    c.nb = 1;
    c.src_c = F;
    c.dst_c = F;
    return run_pass<LM_C, SM_C>(kProfDftLast, 0.0, c, 1, st);
  }
  PassArgs a = {};
  setup_axis(b, 2, a);
  a.sgn = -1.f;
  a.nb = 1;
  a.src_r = f;
  a.dst_c = F;
  if ((rc = run_pass<LM_REAL, SM_C>(kProfDftFirst, 4.0 * b->V, a, 1, st))) return rc;
  for (int ax : {1, 0}) {
    PassArgs c = {};
    setup_axis(b, ax, c);
    c.sgn = -1.f;
    c.nb = 1;
    c.src_c = F;
    c.dst_c = F;
    if ((rc = run_pass<LM_C, SM_C>(ax == 1 ? kProfDftMid : kProfDftLast, 0.0, c, 1, st))) return rc;
  }
  return OS3D_OK;
}

int launch_forward(const os3d_bank* b, const float* f, int batch, void* U, int dtype, float* scales, void* ws,
                   void* stream) {
  if (b->layout == kLayoutFour256) return forward4(b, f, batch, U, dtype, scales, ws, pair_batch(b), stream);
  hipStream_t st = (hipStream_t)stream;
  const long long V = b->V;
  const int nbmax = pair_batch(b);
  float2* F = (float2*)ws;
  float2* T = F + V;
  float* partial = (float*)(T + (long long)nbmax * V);
  const size_t ubytes = (dtype == OS3D_C64) ? 8 : 4;
  int rc;
  for (int bi = 0; bi < batch; ++bi) {
    if ((rc = dft_real_volume(b, f + (long long)bi * V, F, st))) return rc;
    void* Ub = (char*)U + (size_t)bi * b->n_orients * V * ubytes;
    float* sc = scales ? scales + (long long)bi * b->n_orients : nullptr;
    for (int r0 = 0; r0 < b->n_unique; r0 += nbmax) {
      const int nb = std::min(nbmax, b->n_unique - r0);
      PassArgs z = {};
      setup_axis(b, 0, z);
      z.sgn = 1.f;
      z.nb = nb;
      for (int j = 0; j < nb; ++j) {
        const int o = b->rep[r0 + j];
        z.rows[j] = r0 + j;
        z.oa[j] = o;
        z.ob[j] = b->partner[o];
      }
      z.src_c = F;
      z.psi = b->d.psi;
      z.kappa = (float)b->kappa;
      z.dst_c = T;
      z.dst_stride = V;
      const bool quant = dtype != OS3D_C64;
      z.partial = quant ? partial : nullptr;
      if ((rc = run_pass<LM_MULBANK, SM_C>(kProfFwdFirst, 0.0, z, nb, st))) return rc;
      if (quant) {
        const long long tiles = (z.lines + tile_lines(z) - 1) / tile_lines(z);
        void* tok = prof_start(st, kProfScales);
        launch_k(k_scales, dim3(nb), dim3(256), 0, st, partial, (int)tiles, z, dtype, sc);
        prof_stop(tok, st, kProfScales, 0.0, 0.0);
        if ((rc = check_launch("k_scales"))) return rc;
      }
      if (b->plane) {
        PassArgs x = plane_args(b, 1.f, nb);
        for (int j = 0; j < nb; ++j) {
          x.oa[j] = z.oa[j];
          x.ob[j] = z.ob[j];
        }
        x.src_c = T;
        x.src_stride = V;
        x.Uout = Ub;
        x.dtype = dtype;
        x.scales = quant ? sc : nullptr;
        x.out_scale = 1.f / (float)V;
        if ((rc = run_plane<LM_C, SM_UOUT>(kProfFwdLast, score_bytes(b, z, nb, ubytes), x, nb, st))) return rc;
        continue;
      }
      PassArgs y = {};
      setup_axis(b, 1, y);
      y.sgn = 1.f;
      y.nb = nb;
      y.src_c = T;
      y.src_stride = V;
      y.dst_c = T;
      y.dst_stride = V;
      if ((rc = run_pass<LM_C, SM_C>(kProfFwdMid, 0.0, y, nb, st))) return rc;
      PassArgs x = {};
      setup_axis(b, 2, x);
      x.sgn = 1.f;
      x.nb = nb;
      for (int j = 0; j < nb; ++j) {
        x.oa[j] = z.oa[j];
        x.ob[j] = z.ob[j];
      }
      x.src_c = T;
      x.src_stride = V;
      x.Uout = Ub;
      x.dtype = dtype;
      x.scales = quant ? sc : nullptr;
      x.out_scale = 1.f / (float)V;
      if ((rc = run_pass<LM_C, SM_UOUT>(kProfFwdLast, score_bytes(b, z, nb, ubytes), x, nb, st))) return rc;
    }
  }
  return OS3D_OK;
}

int reduce_pair_batch(const os3d_bank* b, long long ws_bytes) {
  // X and one intermediate volume per pair of a launch
  const long long vol = b->V * (long long)sizeof(float2);
  const int fit = (int)std::min<long long>(kMaxBatch, ws_bytes / vol - 1);
  if (fit < 1) return 0;
  int nb = std::min(pair_batch(b), fit);
  const int launches = (b->n_unique + nb - 1) / nb;
  return (b->n_unique + launches - 1) / launches;
}

int launch_reduce(const os3d_bank* b, const void* U, int dtype, const float* scales, int batch, float* f_out,
                  void* ws, bool divide_M, void* stream, int nb_limit) {
  const int nbmax = nb_limit > 0 ? nb_limit : pair_batch(b);
  if (b->layout == kLayoutFour256)
    return reduce4(b, U, dtype, scales, batch, f_out, ws, divide_M, nbmax, stream);
  hipStream_t st = (hipStream_t)stream;
  const long long V = b->V;
  float2* X = (float2*)ws;
  float2* T = X + V;
  const size_t ubytes = (dtype == OS3D_C64) ? 8 : 4;
  int rc;
  for (int bi = 0; bi < batch; ++bi) {
    const void* Ub = (const char*)U + (size_t)bi * b->n_orients * V * ubytes;
    const float* sc = scales ? scales + (long long)bi * b->n_orients : nullptr;
    for (int r0 = 0; r0 < b->n_unique; r0 += nbmax) {
      const int nb = std::min(nbmax, b->n_unique - r0);
      PassArgs x = {};
      setup_axis(b, 2, x);
      x.sgn = -1.f;
      x.nb = nb;
      for (int j = 0; j < nb; ++j) {
        const int o = b->rep[r0 + j];
        x.rows[j] = r0 + j;
        x.oa[j] = o;
        x.ob[j] = b->partner[o];
      }
      x.U = Ub;
      x.dtype = dtype;
      x.scales = (dtype == OS3D_C64) ? nullptr : sc;
      x.dst_c = T;
      x.dst_stride = V;
      if (b->plane) {  // x was set up on the x axis: the plane pass's twiddles
        if ((rc = run_plane<LM_UIN, SM_C>(kProfRecFirst, score_bytes(b, x, nb, ubytes), x, nb, st))) return rc;
      } else {
        if ((rc = run_pass<LM_UIN, SM_C>(kProfRecFirst, score_bytes(b, x, nb, ubytes), x, nb, st))) return rc;
        PassArgs y = {};
        setup_axis(b, 1, y);
        y.sgn = -1.f;
        y.nb = nb;
        y.src_c = T;
        y.src_stride = V;
        y.dst_c = T;
        y.dst_stride = V;
        if ((rc = run_pass<LM_C, SM_C>(kProfRecMid, 0.0, y, nb, st))) return rc;
      }
      PassArgs z = {};
      setup_axis(b, 0, z);
      z.sgn = -1.f;
      z.nb = nb;
      for (int j = 0; j < nb; ++j) z.rows[j] = x.rows[j];
      z.src_c = T;
      z.src_stride = V;
      z.psi = b->d.psi;
      z.kappa = (float)b->kappa;
      z.dst_c = X;
      z.accumulate = (r0 > 0) ? 1 : 0;
      if ((rc = run_pass<LM_C, SM_ACCUM>(kProfRecLast, 0.0, z, 1, st))) return rc;
    }
    // X / max(M, eps) (reconstruction) or X (adjoint), inverse DFT, real part
    PassArgs z = {};
    setup_axis(b, 0, z);
    z.sgn = 1.f;
    z.nb = 1;
    z.src_c = X;
    z.M = b->d.M;
    z.kappa = (float)b->kappa;
    z.eps = (float)b->params.eps;
    z.divide = divide_M ? 1 : 0;
    z.dst_c = X;
    if ((rc = run_pass<LM_DIVM, SM_C>(kProfInvFirst, 0.0, z, 1, st))) return rc;
    if (b->plane) {
      PassArgs x = plane_args(b, 1.f, 1);
      x.src_c = X;
      x.dst_r = f_out + (long long)bi * V;
      x.out_scale = 1.f / (float)V;
      if ((rc = run_plane<LM_C, SM_REAL>(kProfInvLast, 4.0 * b->V, x, 1, st))) return rc;
      continue;
    }
    PassArgs y = {};
    setup_axis(b, 1, y);
    y.sgn = 1.f;
    y.nb = 1;
    y.src_c = X;
    y.dst_c = X;
    if ((rc = run_pass<LM_C, SM_C>(kProfInvMid, 0.0, y, 1, st))) return rc;
    PassArgs x = {};
    setup_axis(b, 2, x);
    x.sgn = 1.f;
    x.nb = 1;
    x.src_c = X;
    x.dst_r = f_out + (long long)bi * V;
    x.out_scale = 1.f / (float)V;
    if ((rc = run_pass<LM_C, SM_REAL>(kProfInvLast, 4.0 * b->V, x, 1, st))) return rc;
  }
  return OS3D_OK;
}

// Processing via scores, Eq. (23) with the stabilised inverse, on the
// three-pass path (see process4 for the structure).
int launch_process(const os3d_bank* b, const float* f, int batch, int phi_kind, float phi_p, float* f_out, void* ws,
                   void* stream) {
  // the plane path transforms in place (F, X and one volume per pair); the
  // others keep the reconstruction's input in a second volume per pair
  // the largest batch the workspace allows: spreading the pairs evenly over
  // the same number of launches measured slower (a launch costs less the
  // more pairs it carries)
  const int nbp = b->plane ? pair_batch(b) : std::max(1, pair_batch(b) / 2);
  if (b->layout == kLayoutFour256) return process4(b, f, batch, phi_kind, phi_p, f_out, ws, nbp, stream);
  hipStream_t st = (hipStream_t)stream;
  const long long V = b->V;
  float2* F = (float2*)ws;
  float2* X = F + V;
  float2* T = X + V;
  float2* Z = T + (long long)nbp * V;
  int rc;
  for (int bi = 0; bi < batch; ++bi) {
    if ((rc = dft_real_volume(b, f + (long long)bi * V, F, st))) return rc;
    for (int r0 = 0; r0 < b->n_unique; r0 += nbp) {
      const int nb = std::min(nbp, b->n_unique - r0);
      PassArgs z = {};
      setup_axis(b, 0, z);
      z.sgn = 1.f;
      z.nb = nb;
      for (int j = 0; j < nb; ++j) {
        const int o = b->rep[r0 + j];
        z.rows[j] = r0 + j;
        z.oa[j] = o;
        z.ob[j] = b->partner[o];
      }
      z.src_c = F;
      z.psi = b->d.psi;
      z.kappa = (float)b->kappa;
      z.dst_c = T;
      z.dst_stride = V;
      if ((rc = run_pass<LM_MULBANK, SM_C>(kProfFwdFirst, 0.0, z, nb, st))) return rc;
      if (b->plane) {  // inverse plane DFT, Phi, forward plane DFT in one kernel, in place
        PassArgs x = z;
        setup_axis(b, 2, x);
        x.src_c = T;
        x.src_stride = V;
        x.dst_c = T;
        x.dst_stride = V;
        x.out_scale = 1.f / (float)V;
        x.phi_kind = phi_kind;
        x.phi_p = phi_p;
        {
          void* tok = prof_start(st, kProfFwdLast);
          launch_plane_phi(x, nb, st);
          prof_stop(tok, st, kProfFwdLast, 0.0, 0.0);
          if ((rc = check_launch("k_plane_phi"))) return rc;
        }
        PassArgs w = z;
        setup_axis(b, 0, w);
        w.sgn = -1.f;
        w.src_c = T;
        w.src_stride = V;
        w.psi = b->d.psi;
        w.dst_c = X;
        w.dst_stride = 0;
        w.accumulate = (r0 > 0) ? 1 : 0;
        if ((rc = run_pass<LM_C, SM_ACCUM>(kProfRecLast, 0.0, w, 1, st))) return rc;
        continue;
      }
      PassArgs y = z;
      setup_axis(b, 1, y);
      y.src_c = T;
      y.src_stride = V;
      if ((rc = run_pass<LM_C, SM_C>(kProfFwdMid, 0.0, y, nb, st))) return rc;
      PassArgs x = z;
      setup_axis(b, 2, x);
      x.src_c = T;
      x.src_stride = V;
      x.dst_c = Z;
      x.dst_stride = V;
      x.out_scale = 1.f / (float)V;
      x.phi_kind = phi_kind;
      x.phi_p = phi_p;
      if ((rc = run_pass<LM_C, SM_PHI>(kProfFwdLast, 0.0, x, nb, st))) return rc;
      PassArgs u = z;
      setup_axis(b, 2, u);
      u.sgn = -1.f;
      u.src_c = Z;
      u.src_stride = V;
      u.dst_c = T;
      u.dst_stride = V;
      if ((rc = run_pass<LM_C, SM_C>(kProfRecFirst, 0.0, u, nb, st))) return rc;
      PassArgs v = u;
      setup_axis(b, 1, v);
      v.src_c = T;
      if ((rc = run_pass<LM_C, SM_C>(kProfRecMid, 0.0, v, nb, st))) return rc;
      PassArgs w = u;
      setup_axis(b, 0, w);
      w.src_c = T;
      w.psi = b->d.psi;
      w.dst_c = X;
      w.dst_stride = 0;
      w.accumulate = (r0 > 0) ? 1 : 0;
      if ((rc = run_pass<LM_C, SM_ACCUM>(kProfRecLast, 0.0, w, 1, st))) return rc;
    }
    PassArgs z = {};
    setup_axis(b, 0, z);
    z.sgn = 1.f;
    z.nb = 1;
    z.src_c = X;
    z.M = b->d.M;
    z.kappa = (float)b->kappa;
    z.eps = (float)b->params.eps;
    z.divide = 1;
    z.dst_c = X;
    if ((rc = run_pass<LM_DIVM, SM_C>(kProfInvFirst, 0.0, z, 1, st))) return rc;
    if (b->plane) {
      PassArgs x = plane_args(b, 1.f, 1);
      x.src_c = X;
      x.dst_r = f_out + (long long)bi * V;
      x.out_scale = 1.f / (float)V;
      if ((rc = run_plane<LM_C, SM_REAL>(kProfInvLast, 4.0 * b->V, x, 1, st))) return rc;
      continue;
    }
    PassArgs y = {};
    setup_axis(b, 1, y);
    y.sgn = 1.f;
    y.nb = 1;
    y.src_c = X;
    y.dst_c = X;
    if ((rc = run_pass<LM_C, SM_C>(kProfInvMid, 0.0, y, 1, st))) return rc;
    PassArgs x = {};
    setup_axis(b, 2, x);
    x.sgn = 1.f;
    x.nb = 1;
    x.src_c = X;
    x.dst_r = f_out + (long long)bi * V;
    x.out_scale = 1.f / (float)V;
    if ((rc = run_pass<LM_C, SM_REAL>(kProfInvLast, 4.0 * b->V, x, 1, st))) return rc;
  }
  return OS3D_OK;
}

int profile_enable(int on) {
  for (auto& r : g_prof) {
    g_event_pool.push_back(r.e0);
    g_event_pool.push_back(r.e1);
  }
  g_prof.clear();
  if (on < 0 || on >= 2 + kProfCount) return OS3D_EINVAL;
  g_prof_mode = on;
  return OS3D_OK;
}

int profile_get(int idx, const char** name, long long* launches, double* total_ms, double* alg_bytes,
                double* alg_flops) {
  if (idx < 0 || idx >= kProfCount) return OS3D_EINVAL;
  *name = kKernelNames[idx];
  long long n = 0;
  double ms = 0.0, by = 0.0, fl = 0.0;
  for (auto& r : g_prof) {
    if (r.kid != idx) continue;
    float t = 0.f;
    if (hipEventSynchronize(r.e1) != hipSuccess || hipEventElapsedTime(&t, r.e0, r.e1) != hipSuccess) return OS3D_EDEVICE;
    ++n;
    ms += t;
    by += r.alg_bytes;
    fl += r.alg_flops;
  }
  *launches = n;
  *total_ms = ms;
  *alg_bytes = by;
  *alg_flops = fl;
  return OS3D_OK;
}

int profile_count() { return kProfCount; }

}  // namespace os3d
