// Internal declarations of libos3d (not part of the C ABI).
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/os3d.h"

namespace os3d {

// Largest SH order of the device bank synthesis (its fp16 operands hold
// |Y_lm| <= sqrt((2L + 1) / 4 pi) scaled by 2^13).
constexpr int kMaxBankL = 62;

constexpr int kMaxL = 64;
constexpr int kMaxDim = 4096;
constexpr int kMaxStages = 14;

// ---------------------------------------------------------------- host FP64 setup
double bspline(int k, double x);
void legendre(int L, double x, double* P);               // P[0..L]
std::vector<double> geodesic_icosahedron(int freq);      // 3 * (10 freq^2 + 2)
bool zonal_fit(int L, const std::vector<double>& pts, const std::vector<double>& values,
               std::vector<double>& c);                   // least squares, Householder QR
void cake_coeffs(int L, const double* c, int variant, double* a);
void wavelet_coeffs(const os3d_wavelet_params& p, std::vector<double>& c, std::vector<double>& a);

// Real spherical-harmonic recursion coefficients shared by the host steering
// matrix and the device generator (so both use one convention):
//   Q_m^m = qmm[m];  Q_{m+1}^m = sqrt(2m+3) z Q_m^m;
//   Q_l^m = alm[l*(L+1)+m] (z Q_{l-1}^m - blm[l*(L+1)+m] Q_{l-2}^m)
//   Y_l0 = Q_l^0,  Y_lm = sqrt2 Q_l^m Re((x+iy)^m),  Y_l-m = sqrt2 Q_l^m Im((x+iy)^m)
struct ShTables {
  int L;
  std::vector<double> qmm, alm, blm;
};
ShTables sh_tables(int L);
void real_sh(const ShTables& t, const double n[3], double* Y);  // index l*l + l + m

// Contraction order (K) of the bank synthesis.  The orders m = 0..L are
// split into two chains of the recursion, A = 0..M and B = M + 1..L, M
// balancing their lengths (one step per (l, m), l = m..L, orders ascending);
// word 2i is step i of chain A, word 2i + 1 step i of chain B (zero past a
// chain's end).  A word holds the entries (cos, sin) of its (l, m) as two
// fp16 values (the sin entry of m = 0 is zero); 16 words (32 entries) are
// one K-block of the 16x16x32 fp16 MFMA.
int synth_split(int L);                                        // M
int synth_pairs(int L);                                        // steps of the longer chain
int synth_words(int L);                                        // 2 synth_pairs(L)
int synth_kblocks(int L);                                      // ceil(words / 16)
// The stored rows go through the synthesis in sweeps of at most
// kSynthMaxBlocks 16-column blocks, the sweeps evenly filled; the packed
// steering operands hold synth_padded_blocks (zero past the rows).
constexpr int kSynthMaxBlocks = 6;
int synth_sweep_blocks(int ncb);                               // blocks per sweep
int synth_padded_blocks(int ncb);                              // sweeps x blocks per sweep
bool synth_entry(int L, int e, int& l, int& m, bool& sin_part);  // false for a zero entry
std::vector<int> synth_word_order(int L);  // per word of the K-blocks: l (L + 1) + m, or -1

void steering_std(const os3d_wavelet_params& p, const double* orients, int n, const std::vector<double>& a,
                  double* S);  // [(L+1)^2][n], standard order

// Antipodal pairing: partner[i] = j with n_j = -n_i (|n_i + n_j| < 1e-9) or -1.
void pair_orientations(const double* orients, int n, std::vector<int>& partner);

bool factor235(int64_t n);
std::vector<int> radix_schedule(int n);  // radices in {16, 8, 4, 2, 5, 3}

// ---------------------------------------------------------------- device plan
struct AxisPlan {
  int n;
  int nstages;
  int radix[kMaxStages];
};

struct DevPtrs {
  float* psi;      // [n_unique][V] float32 g h without kappa (the transforms apply kappa)
  float* M;        // [V]
  double* Mh;      // [V] FP64 sum over stored rows of raw psi^2 (build scratch)
  uint32_t* S;     // steering matrix as fp16 hi / lo MFMA operands: [kblocks][padded blocks][2][64][4 words]
  double* tab;     // recursion steps of the synthesis: [kblocks * 8][chain A, B][c0, c1],
                   // then [kblocks] 32-bit order-start masks
  double* part;    // band partials of the synthesis, then kappa and S
  float* tw[3];    // twiddles exp(-2 pi i j / N_d), j < N_d, per axis (z, y, x)
};

}  // namespace os3d

struct os3d_bank {
  int64_t dims[3];
  int64_t V;
  int n_orients;
  int n_unique;
  int paired;
  int layout;                 // frequency storage order: 0 natural, 1 four-step tiles of 256^3
  int plane;                  // natural order with Ny = Nx in {64, 128}: z-line pass + whole-plane pass
  int L;
  int Npad;
  int kblocks;                // K-blocks of the synthesis contraction
  int synth_mb;               // first order of the synthesis' second recursion chain
  float synth_scale;          // 2^-(13 + e_S): undoes the fp16 operand scaling
  double kappa;
  double dc_value;            // a_0 / sqrt(4 pi): the sphere average of h, used at k = 0
  double approx_norm;         // band mean of sum_i psi_hat_i (approximate reconstruction)
  os3d_wavelet_params params;
  std::vector<int> partner;   // per orientation: antipode index or -1
  std::vector<int> row_of;    // per orientation: stored bank row
  std::vector<int> conj_of;   // per orientation: 1 when it is the second member of a pair (psi(Sk))
  std::vector<int> rep;       // per stored row: orientation index of the stored member
  os3d::AxisPlan plan[3];     // z, y, x
  os3d::DevPtrs d;
  void* base;
  size_t bytes;
};

namespace os3d {
// Device-side entry points implemented in the .hip files.
int launch_build_bank(os3d_bank* b, void* stream);
int launch_forward(const os3d_bank* b, const float* f, int batch, void* U, int dtype, float* scales, void* ws,
                   void* stream);
// nb_limit > 0 caps the orientation pairs per launch (the workspace then
// needs X and nb_limit intermediate volumes); 0 takes the default batch.
int launch_reduce(const os3d_bank* b, const void* U, int dtype, const float* scales, int batch, float* f_out,
                  void* ws, bool divide_M, void* stream, int nb_limit = 0);
// Largest even pair batch whose reduction intermediates (X and one volume
// per pair) fit ws_bytes; 0 if not even one pair fits.
int reduce_pair_batch(const os3d_bank* b, long long ws_bytes);
int launch_export_psi(const os3d_bank* b, int i, float* out, void* stream);
int launch_process(const os3d_bank* b, const float* f, int batch, int phi_kind, float phi_p, float* f_out, void* ws,
                   void* stream);
int launch_approx(const os3d_bank* b, const void* U, int dtype, const float* scales, int batch, float* f_out,
                  void* stream);
int launch_export_M(const os3d_bank* b, float* out, void* stream);
size_t workspace_bytes(const os3d_bank* b);
int profile_enable(int on);
// Launch bracketing for the per-kernel timer: prof_start returns a token (or
// null when timing is off) and leaves its events for the one launch that
// follows (launch_k in launch.h); prof_stop files that launch under slot kid.
void* prof_start(void* stream, int kid);
void prof_stop(void* token, void* stream, int kid, double alg_bytes, double alg_flops);
enum ProfSlot { PROF_BANK = 13 };
int profile_get(int idx, const char** name, long long* launches, double* total_ms, double* alg_bytes,
                double* alg_flops);
int profile_count();
size_t bank_bytes(const int64_t dims[3], int n_unique, int L);
void set_error(const std::string& msg);
}  // namespace os3d
