// C ABI of libos3d: argument validation, bank layout and plan, dispatch to
// the HIP launchers.  See include/os3d.h for the contract of each call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "os3d_internal.h"

namespace os3d {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

static int fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// element-wise kernels launch one work-item per voxel: keep V within 2^31
static constexpr long long kMaxVoxels = 1LL << 31;

static int check_params(const os3d_wavelet_params* p) {
  if (!p) return fail(OS3D_EINVAL, "params is NULL");
  if (p->L < 0 || p->L > kMaxL) return fail(OS3D_EINVAL, "L must be in [0, 64]");
  if (!(p->s_theta > 0.0) || !std::isfinite(p->s_theta)) return fail(OS3D_EINVAL, "s_theta must be > 0");
  if (p->k < 0 || p->k > 16) return fail(OS3D_EINVAL, "k must be in [0, 16]");
  if (p->taylor_N < 0 || p->taylor_N > 200) return fail(OS3D_EINVAL, "taylor_N must be in [0, 200]");
  if (!(p->gamma > 0.0 && p->gamma < 1.0)) return fail(OS3D_EINVAL, "gamma must be in (0, 1)");
  if (!(p->eps > 0.0) || !std::isfinite(p->eps)) return fail(OS3D_EINVAL, "eps must be > 0");
  if (p->variant != OS3D_CAKE && p->variant != OS3D_PLATE) return fail(OS3D_EINVAL, "unknown variant");
  if (p->coeffs != OS3D_COEFFS_LSQ && p->coeffs != OS3D_COEFFS_QUADRATURE)
    return fail(OS3D_EINVAL, "unknown coefficient method");
  return OS3D_OK;
}

static int check_dims(const int64_t* dims) {
  if (!dims) return fail(OS3D_EINVAL, "dims is NULL");
  for (int d = 0; d < 3; ++d) {
    if (dims[d] < 2) return fail(OS3D_EINVAL, "every dim must be >= 2");
    if (dims[d] > kMaxDim || !factor235(dims[d]))
      return fail(OS3D_EUNSUPPORTED, "dims must be <= 4096 with prime factors 2, 3, 5 only");
  }
  if (dims[0] * dims[1] * dims[2] > kMaxVoxels)
    return fail(OS3D_EUNSUPPORTED, "the volume must hold at most 2^31 voxels");
  return OS3D_OK;
}

static int check_orients(const double* o, int n) {
  if (!o) return fail(OS3D_EINVAL, "orients is NULL");
  if (n < 1 || n > 4096) return fail(OS3D_EINVAL, "n_orients must be in [1, 4096]");
  for (int i = 0; i < n; ++i) {
    double r = std::sqrt(o[3 * i] * o[3 * i] + o[3 * i + 1] * o[3 * i + 1] + o[3 * i + 2] * o[3 * i + 2]);
    if (!(std::fabs(r - 1.0) <= 1e-9)) return fail(OS3D_EINVAL, "orientation " + std::to_string(i) + " is not a unit vector");
  }
  return OS3D_OK;
}

// Stored rows: one per antipodal pair when the whole set pairs up, else one per orientation.
static void make_rows(const double* o, int n, std::vector<int>& partner, std::vector<int>& rep, std::vector<int>& row_of,
                      std::vector<int>& conj_of, int& paired) {
  pair_orientations(o, n, partner);
  paired = 1;
  for (int i = 0; i < n; ++i)
    if (partner[i] < 0 || partner[partner[i]] != i) paired = 0;
  rep.clear();
  row_of.assign(n, -1);
  conj_of.assign(n, 0);
  if (!paired) partner.assign(n, -1);
  for (int i = 0; i < n; ++i) {
    if (paired && partner[i] < i) continue;
    row_of[i] = (int)rep.size();
    rep.push_back(i);
  }
  if (paired)
    for (int i = 0; i < n; ++i)
      if (row_of[i] < 0) {
        row_of[i] = row_of[partner[i]];
        conj_of[i] = 1;
      }
}

struct BankLayout {
  size_t psi, M, Mh, S, tab, part, tw[3], total;
};

static BankLayout layout(const int64_t dims[3], int n_unique, int L) {
  BankLayout b;
  const size_t V = (size_t)dims[0] * dims[1] * dims[2];
  const int Npad = (n_unique + 15) / 16 * 16;
  size_t o = 0;
  b.psi = o;
  o = align256(o + (size_t)n_unique * V * sizeof(float));
  b.M = o;
  o = align256(o + V * sizeof(float));
  b.Mh = o;
  o = align256(o + V * sizeof(double));
  b.S = o;
  o = align256(o + (size_t)synth_kblocks(L) * synth_padded_blocks(Npad / 16) * 2 * 64 * 16);
  b.tab = o;
  // the synthesis' recursion records, then its order-start masks (packed into doubles)
  o = align256(o + ((size_t)synth_kblocks(L) * 8 * 4 + (synth_kblocks(L) + 1) / 2) * sizeof(double));
  b.part = o;  // band partials of the synthesis workgroups (3 each), then kappa and S
  o = align256(o + (3 * ((V + 255) / 256) + 2) * sizeof(double));
  for (int d = 0; d < 3; ++d) {
    b.tw[d] = o;
    o = align256(o + (size_t)dims[d] * 2 * sizeof(float));
  }
  b.total = o;
  return b;
}

size_t bank_bytes(const int64_t dims[3], int n_unique, int L) { return layout(dims, n_unique, L).total; }

}  // namespace os3d

using namespace os3d;

extern "C" {

const char* os3d_last_error(void) { return g_last_error.c_str(); }

const char* os3d_version(void) { return "os3d 0.1 (gfx950)"; }

os3d_status os3d_wavelet_coeffs(const os3d_wavelet_params* p, double* c_out, double* a_out) {
  int rc = check_params(p);
  if (rc) return (os3d_status)rc;
  std::vector<double> c, a;
  wavelet_coeffs(*p, c, a);
  if (c_out) std::copy(c.begin(), c.end(), c_out);
  if (a_out) std::copy(a.begin(), a.end(), a_out);
  return OS3D_OK;
}

os3d_status os3d_steering_matrix(const os3d_wavelet_params* p, const double* orients, int32_t n, double* S_out) {
  int rc = check_params(p);
  if (rc) return (os3d_status)rc;
  if ((rc = check_orients(orients, n))) return (os3d_status)rc;
  if (!S_out) return (os3d_status)fail(OS3D_EINVAL, "S_out is NULL");
  std::vector<double> c, a;
  wavelet_coeffs(*p, c, a);
  steering_std(*p, orients, n, a, S_out);
  return OS3D_OK;
}

os3d_status os3d_bank_bytes(const int64_t dims[3], const double* orients, int32_t n, const os3d_wavelet_params* p,
                            size_t* bytes) {
  int rc;
  if ((rc = check_dims(dims))) return (os3d_status)rc;
  if ((rc = check_orients(orients, n))) return (os3d_status)rc;
  if ((rc = check_params(p))) return (os3d_status)rc;
  if (!bytes) return (os3d_status)fail(OS3D_EINVAL, "bytes is NULL");
  std::vector<int> partner, rep, row_of, conj_of;
  int paired;
  make_rows(orients, n, partner, rep, row_of, conj_of, paired);
  *bytes = bank_bytes(dims, (int)rep.size(), p->L);
  return OS3D_OK;
}

os3d_status os3d_build_bank(const int64_t dims[3], const double* orients, int32_t n, const os3d_wavelet_params* p,
                            void* bank_dev, size_t bank_bytes_given, void* stream, os3d_bank** out) {
  int rc;
  if ((rc = check_dims(dims))) return (os3d_status)rc;
  if ((rc = check_orients(orients, n))) return (os3d_status)rc;
  if ((rc = check_params(p))) return (os3d_status)rc;
  if (!bank_dev || !out) return (os3d_status)fail(OS3D_EINVAL, "bank_dev or out is NULL");
  if (p->L > kMaxBankL)
    return (os3d_status)fail(OS3D_EUNSUPPORTED, "bank synthesis supports L <= " + std::to_string(kMaxBankL));
  // kappa averages M over {k != 0, rho <= rho_N / 2, off the Nyquist planes}:
  // the axis frequency 2 pi / N is inside only for N >= 4
  if (std::max(dims[0], std::max(dims[1], dims[2])) < 4)
    return (os3d_status)fail(OS3D_EINVAL, "the normalisation band is empty: some dim must be >= 4");
  os3d_bank* b = new (std::nothrow) os3d_bank();
  if (!b) return (os3d_status)fail(OS3D_ENOMEM, "host allocation failed");
  for (int d = 0; d < 3; ++d) b->dims[d] = dims[d];
  b->V = dims[0] * dims[1] * dims[2];
  b->n_orients = n;
  b->params = *p;
  b->L = p->L;
  make_rows(orients, n, b->partner, b->rep, b->row_of, b->conj_of, b->paired);
  b->n_unique = (int)b->rep.size();
  b->Npad = (b->n_unique + 15) / 16 * 16;
  // 256^3 volumes take the two-pass transform and its frequency tiles
  b->layout = (dims[0] == 256 && dims[1] == 256 && dims[2] == 256) ? 1 : 0;
  b->plane = (b->layout == 0 && dims[1] == dims[2] && (dims[2] == 64 || dims[2] == 128)) ? 1 : 0;
  if (const char* e = std::getenv("OS3D_THREE_PASS"))
    if (e[0] == '1') b->layout = b->plane = 0;
  const BankLayout lay = layout(dims, b->n_unique, p->L);
  if (bank_bytes_given < lay.total) {
    delete b;
    return (os3d_status)fail(OS3D_ENOMEM, "bank buffer too small: need " + std::to_string(lay.total) + " bytes");
  }
  char* base = (char*)bank_dev;
  b->base = bank_dev;
  b->bytes = lay.total;
  b->d.psi = (float*)(base + lay.psi);
  b->d.M = (float*)(base + lay.M);
  b->d.Mh = (double*)(base + lay.Mh);
  b->d.S = (uint32_t*)(base + lay.S);
  b->d.tab = (double*)(base + lay.tab);
  b->d.part = (double*)(base + lay.part);
  for (int d = 0; d < 3; ++d) b->d.tw[d] = (float*)(base + lay.tw[d]);
  for (int d = 0; d < 3; ++d) {
    std::vector<int> r = radix_schedule((int)dims[d]);
    b->plan[d].n = (int)dims[d];
    b->plan[d].nstages = (int)r.size();
    for (int s = 0; s < kMaxStages; ++s) b->plan[d].radix[s] = s < (int)r.size() ? r[s] : 0;
  }

  // host FP64 design: coefficients, steering matrix as MFMA operands, recursion tables, twiddles
  std::vector<double> c, a;
  wavelet_coeffs(*p, c, a);
  b->dc_value = a[0] / std::sqrt(4.0 * 3.14159265358979323846);
  const int L = p->L, nn = L + 1;
  std::vector<double> Sstd((size_t)nn * nn * b->n_unique);
  std::vector<double> rep_or(3 * b->n_unique);
  for (int r = 0; r < b->n_unique; ++r)
    for (int c3 = 0; c3 < 3; ++c3) rep_or[3 * r + c3] = orients[3 * b->rep[r] + c3];
  steering_std(*p, rep_or.data(), b->n_unique, a, Sstd.data());
  // fp16 hi / lo operands: S 2^e_S = hi + lo, e_S putting max |S| in
  // [2^14, 2^15) (fp16 holds up to 65504); the device scales Y_lm by 2^13
  // and the product back by synth_scale = 2^-(13 + e_S)
  double smax = 0.0;
  for (double v : Sstd) smax = std::max(smax, std::fabs(v));
  const int eS = smax > 0.0 ? 14 - (int)std::floor(std::log2(smax)) : 0;
  b->synth_scale = (float)std::ldexp(1.0, -(13 + eS));
  b->kblocks = synth_kblocks(L);
  const int ncb = synth_padded_blocks(b->Npad / 16);
  // operand order of v_mfma_f32_16x16x32_f16's B: lane t holds column t % 16
  // and the eight K entries 8 (t / 16) .. + 7, two per word (low half first)
  std::vector<uint32_t> S((size_t)b->kblocks * ncb * 2 * 64 * 4, 0u);
  const std::vector<int> order = synth_word_order(L);
  for (int kb = 0; kb < b->kblocks; ++kb)
    for (int cb = 0; cb < ncb; ++cb)
      for (int t = 0; t < 64; ++t) {
        const int col = cb * 16 + (t & 15);
        for (int j = 0; j < 8; ++j) {
          const int e = kb * 32 + 8 * (t >> 4) + j;  // entry: word e / 2, cos (even) or sin (odd)
          const int lm = order[e >> 1];
          const int l = lm / (L + 1), m = lm % (L + 1);
          const bool sn = (e & 1) == 1;
          float v = 0.f;
          if (col < b->n_unique && lm >= 0 && !(m == 0 && sn)) {
            const int idx = l * l + l + (sn ? -m : m);
            v = (float)std::ldexp(Sstd[(size_t)idx * b->n_unique + col], eS);
          }
          const _Float16 hi = (_Float16)v;
          const _Float16 lo = (_Float16)(v - (float)hi);
          uint16_t hb, lb;
          std::memcpy(&hb, &hi, 2);
          std::memcpy(&lb, &lo, 2);
          const size_t w = ((((size_t)kb * ncb + cb) * 2) * 64 + t) * 4 + j / 2;
          const int sh = (j & 1) * 16;
          S[w] |= (uint32_t)hb << sh;
          S[w + 64 * 4] |= (uint32_t)lb << sh;
        }
      }
  ShTables t = sh_tables(L);
  // the recursion steps in the synthesis order, per word pair the records
  // (c0, c1) of chains A and B, Q = c0 (z Q') - c1 Q'': inside an order
  // (alpha, alpha beta), where an order starts (0, -Q_m^m) with Q'' set to 1
  // by the device (zero records past a chain's end); then per K-block a mask
  // with bit i (chain A) or 8 + i (chain B) set where pair i starts an order
  // (the chain then also multiplies its (x + iy)^m by x + iy, except at its
  // first order)
  const int M = synth_split(L);
  std::vector<double> tab((size_t)b->kblocks * 8 * 4 + (b->kblocks + 1) / 2, 0.0);
  std::vector<uint32_t> starts(b->kblocks, 0u);
  auto put_chain = [&](int chain, int m0, int m1) {
    int i = 0;
    for (int m = m0; m <= m1; ++m)
      for (int l = m; l <= L; ++l, ++i) {
        double* r = &tab[(size_t)4 * i + 2 * chain];
        if (l == m) {
          r[1] = -t.qmm[m];
          starts[i / 8] |= 1u << (8 * chain + i % 8);
        } else if (l == m + 1) {
          r[0] = std::sqrt(2.0 * m + 3.0);
        } else {
          r[0] = t.alm[l * nn + m];
          r[1] = t.alm[l * nn + m] * t.blm[l * nn + m];
        }
      }
  };
  put_chain(0, 0, M);
  put_chain(1, M + 1, L);
  std::memcpy(&tab[(size_t)b->kblocks * 8 * 4], starts.data(), starts.size() * sizeof(uint32_t));
  b->synth_mb = M + 1;
  std::vector<float> tw[3];
  for (int d = 0; d < 3; ++d) {
    const int N = (int)dims[d];
    tw[d].resize(2 * N);
    for (int j = 0; j < N; ++j) {
      const double ang = -2.0 * 3.14159265358979323846 * (double)j / (double)N;
      tw[d][2 * j] = (float)std::cos(ang);
      tw[d][2 * j + 1] = (float)std::sin(ang);
    }
  }
  hipStream_t st = (hipStream_t)stream;
  bool ok = hipMemcpyAsync(b->d.S, S.data(), S.size() * sizeof(uint32_t), hipMemcpyHostToDevice, st) == hipSuccess &&
            hipMemcpyAsync(b->d.tab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice, st) == hipSuccess;
  for (int d = 0; d < 3 && ok; ++d)
    ok = hipMemcpyAsync(b->d.tw[d], tw[d].data(), tw[d].size() * sizeof(float), hipMemcpyHostToDevice, st) ==
         hipSuccess;
  if (!ok) {
    delete b;
    return (os3d_status)fail(OS3D_EDEVICE, "os3d_build_bank: host-to-device copy failed");
  }
  rc = launch_build_bank(b, stream);
  if (rc) {
    (void)hipStreamSynchronize(st);
    delete b;
    return (os3d_status)rc;
  }
  *out = b;
  return OS3D_OK;
}

os3d_status os3d_free_bank(os3d_bank* b) {
  delete b;
  return OS3D_OK;
}

os3d_status os3d_get_bank_info(const os3d_bank* b, os3d_bank_info* info) {
  if (!b || !info) return (os3d_status)fail(OS3D_EINVAL, "bank or info is NULL");
  for (int d = 0; d < 3; ++d) info->dims[d] = b->dims[d];
  info->n_orients = b->n_orients;
  info->n_unique = b->n_unique;
  info->paired = b->paired;
  info->kappa = b->kappa;
  info->approx_norm = b->approx_norm;
  info->M_dev = b->d.M;
  return OS3D_OK;
}

os3d_status os3d_bank_psi(const os3d_bank* b, int32_t i, float* psi_dev, void* stream) {
  if (!b || !psi_dev) return (os3d_status)fail(OS3D_EINVAL, "bank or psi_dev is NULL");
  if (i < 0 || i >= b->n_orients) return (os3d_status)fail(OS3D_EINVAL, "orientation index out of range");
  return (os3d_status)launch_export_psi(b, i, psi_dev, stream);
}

os3d_status os3d_bank_M(const os3d_bank* b, float* M_dev, void* stream) {
  if (!b || !M_dev) return (os3d_status)fail(OS3D_EINVAL, "bank or M_dev is NULL");
  return (os3d_status)launch_export_M(b, M_dev, stream);
}

os3d_status os3d_workspace_bytes(const os3d_bank* b, size_t* bytes) {
  if (!b || !bytes) return (os3d_status)fail(OS3D_EINVAL, "bank or bytes is NULL");
  *bytes = workspace_bytes(b);
  return OS3D_OK;
}

static int check_compute(const os3d_bank* b, const void* in, int batch, const void* out, int dtype, const void* scales,
                         const void* ws, size_t ws_bytes, bool scales_are_output) {
  if (!b) return fail(OS3D_EINVAL, "bank is NULL");
  if (!in || !out) return fail(OS3D_EINVAL, "input or output is NULL");
  if (batch < 1) return fail(OS3D_EINVAL, "batch must be >= 1");
  if (dtype != OS3D_C64 && dtype != OS3D_BF16X2 && dtype != OS3D_F16X2) return fail(OS3D_EINVAL, "unknown score dtype");
  if (dtype != OS3D_C64 && !scales)
    return fail(OS3D_EINVAL, scales_are_output ? "scales output is NULL for a 16-bit score dtype"
                                               : "scales is NULL for a 16-bit score dtype");
  if (!ws) return fail(OS3D_EINVAL, "workspace is NULL");
  if (ws_bytes < workspace_bytes(b))
    return fail(OS3D_ENOMEM, "workspace too small: need " + std::to_string(workspace_bytes(b)) + " bytes");
  return OS3D_OK;
}

os3d_status os3d_forward(const os3d_bank* b, const float* f, int32_t batch, void* U, int32_t dtype, float* scales,
                         void* ws, size_t ws_bytes, void* stream) {
  int rc = check_compute(b, f, batch, U, dtype, scales, ws, ws_bytes, true);
  if (rc) return (os3d_status)rc;
  return (os3d_status)launch_forward(b, f, batch, U, dtype, scales, ws, stream);
}

os3d_status os3d_adjoint(const os3d_bank* b, const void* U, int32_t dtype, const float* scales, int32_t batch,
                         float* f_out, void* ws, size_t ws_bytes, void* stream) {
  int rc = check_compute(b, U, batch, f_out, dtype, scales, ws, ws_bytes, false);
  if (rc) return (os3d_status)rc;
  return (os3d_status)launch_reduce(b, U, dtype, scales, batch, f_out, ws, false, stream);
}

os3d_status os3d_reconstruct(const os3d_bank* b, const void* U, int32_t dtype, const float* scales, int32_t batch,
                             float* f_out, void* ws, size_t ws_bytes, void* stream) {
  int rc = check_compute(b, U, batch, f_out, dtype, scales, ws, ws_bytes, false);
  if (rc) return (os3d_status)rc;
  return (os3d_status)launch_reduce(b, U, dtype, scales, batch, f_out, ws, true, stream);
}

os3d_status os3d_reconstruct_approx(const os3d_bank* b, const void* U, int32_t dtype, const float* scales,
                                    int32_t batch, float* f_out, void* stream) {
  if (!b) return (os3d_status)fail(OS3D_EINVAL, "bank is NULL");
  if (!U || !f_out) return (os3d_status)fail(OS3D_EINVAL, "input or output is NULL");
  if (batch < 1) return (os3d_status)fail(OS3D_EINVAL, "batch must be >= 1");
  if (dtype != OS3D_C64 && dtype != OS3D_BF16X2 && dtype != OS3D_F16X2)
    return (os3d_status)fail(OS3D_EINVAL, "unknown score dtype");
  if (dtype != OS3D_C64 && !scales) return (os3d_status)fail(OS3D_EINVAL, "scales is NULL for a 16-bit score dtype");
  return (os3d_status)launch_approx(b, U, dtype, scales, batch, f_out, stream);
}

os3d_status os3d_process(const os3d_bank* b, const float* f, int32_t batch, int32_t phi, double phi_power,
                         float* f_out, void* ws, size_t ws_bytes, void* stream) {
  int rc = check_compute(b, f, batch, f_out, OS3D_C64, nullptr, ws, ws_bytes, false);
  if (rc) return (os3d_status)rc;
  if (phi != OS3D_PHI_IDENTITY && phi != OS3D_PHI_SOFT_THRESHOLD) return (os3d_status)fail(OS3D_EINVAL, "unknown phi");
  if (phi == OS3D_PHI_SOFT_THRESHOLD && !(phi_power > 0.0 && phi_power <= 16.0))
    return (os3d_status)fail(OS3D_EINVAL, "phi_power must be in (0, 16]");
  return (os3d_status)launch_process(b, f, batch, phi, (float)phi_power, f_out, ws, stream);
}

os3d_status os3d_profile_enable(int32_t on) {
  int rc = profile_enable(on);
  if (rc) return (os3d_status)fail(rc, "os3d_profile_enable: on must be 0, 1 or 2 + a kernel slot");
  return OS3D_OK;
}

os3d_status os3d_profile_count(int32_t* n) {
  if (!n) return (os3d_status)fail(OS3D_EINVAL, "n is NULL");
  *n = profile_count();
  return OS3D_OK;
}

os3d_status os3d_profile_get(int32_t idx, const char** name, int64_t* launches, double* total_ms, double* alg_bytes,
                             double* alg_flops) {
  if (!name || !launches || !total_ms || !alg_bytes || !alg_flops)
    return (os3d_status)fail(OS3D_EINVAL, "output pointer is NULL");
  long long n = 0;
  int rc = profile_get(idx, name, &n, total_ms, alg_bytes, alg_flops);
  *launches = n;
  if (rc) return (os3d_status)fail(rc, "os3d_profile_get: bad index or event failure");
  return OS3D_OK;
}

}  // extern "C"
