/*
 * os3d: the discrete invertible 3D orientation-score transform with cake
 * wavelets (Janssen, Duits & Breeuwer, "Invertible Orientation Scores of 3D
 * Images"), on AMD Instinct MI355X (gfx950).
 *
 * C ABI.  Every call returns an os3d_status (0 = OK) and never throws; the
 * message of the last non-OK status of the calling thread is returned by
 * os3d_last_error().
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - A volume is float32 [Nz][Ny][Nx] with x fastest (dims[] = {Nz, Ny, Nx}).
 *   Every dim must be >= 2 and have no prime factor other than 2, 3 and 5
 *   (others: OS3D_EUNSUPPORTED); the largest supported dim is 4096 and the largest
 *   volume 2^31 voxels (larger: OS3D_EUNSUPPORTED).
 * - Orientations are float64 host arrays [N_o][3] of (x, y, z) unit vectors,
 *   in the caller's order (the set V of Sec. 2.1).  Scores keep that order.
 * - The DFT is unnormalised, F[k] = sum_x f[x] exp(-2 pi i k.x / N); its
 *   inverse carries 1/V (V = Nz Ny Nx).  Frequencies are
 *   omega_d = 2 pi kt_d / N_d, kt_d in [-N_d/2, N_d/2), Nyquist radius pi.
 * - A score U is [B][N_o][Nz][Ny][Nx].  OS3D_C64 stores interleaved float32
 *   (re, im).  OS3D_BF16X2 / OS3D_F16X2 store two 16-bit floats (re, im)
 *   per voxel; the stored value times scales[b][i] (float32, a power of two)
 *   is the score.
 * - Device pointers are HIP device memory on the current device, owned by the
 *   caller; the library never allocates device memory.  `stream` is a
 *   hipStream_t passed as void* (NULL = the default stream).  Compute calls
 *   only enqueue work on `stream` and return; os3d_build_bank synchronises
 *   `stream` once at its end.
 * - Argument errors are detected before any work is enqueued and return
 *   OS3D_EINVAL; a failed launch returns OS3D_EDEVICE.
 */
#ifndef OS3D_H
#define OS3D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  OS3D_OK = 0,
  OS3D_EINVAL = -1,        /* invalid argument (null pointer, bad size, non-unit orientation, ...) */
  OS3D_ENOMEM = -2,        /* a caller-provided buffer is smaller than required */
  OS3D_EUNSUPPORTED = -3,  /* a dim with a prime factor other than 2, 3, 5, above 4096, or V > 2^31 */
  OS3D_EDEVICE = -4        /* a HIP runtime call or kernel launch failed */
} os3d_status;

typedef enum {
  OS3D_C64 = 0,      /* complex float32, 8 B per voxel-orientation */
  OS3D_BF16X2 = 1,   /* (re, im) bfloat16 pair times a per-(b, i) power-of-two scale, 4 B */
  OS3D_F16X2 = 2     /* (re, im) IEEE half pair times a per-(b, i) power-of-two scale, 4 B */
} os3d_score_dtype;

typedef enum {
  OS3D_CAKE = 0,     /* h = Funk(A) + antisym(A): real line detector, imaginary edge detector (Eqs. 12-14) */
  OS3D_PLATE = 1     /* h = A: real plate detector (Sec. 3.1, Fig. 4) */
} os3d_variant;

typedef enum {
  OS3D_COEFFS_LSQ = 0,        /* c_l by least squares (the pseudo-inverse) over the frequency-15 geodesic
                                 icosahedron, as in Sec. 3.2 */
  OS3D_COEFFS_QUADRATURE = 1  /* c_l = 2 pi int_0^pi A(theta) Y_l0(theta) sin(theta) dtheta, composite
                                 64-node Gauss-Legendre in theta split at the B-spline knots */
} os3d_coeffs;

typedef enum {
  OS3D_PHI_IDENTITY = 0,        /* Phi(U) = U: Upsilon = W^+ W, the band filter M / max(M, eps) */
  OS3D_PHI_SOFT_THRESHOLD = 1   /* Phi(U) = |U|^p sgn(U), sgn(U) = U / |U| (Fig. 7: p = 1.5) */
} os3d_phi;

/* Cake-wavelet parameters (Sec. 3).
 *   L         spherical-harmonic order of the window expansion (Eq. 15), 0 <= L <= 64
 *   s_theta   width of the orientation window A = B^k(theta / s_theta) (Eq. 11), > 0
 *   k         B-spline order (Eq. 11), 0 <= k <= 16
 *   taylor_N  Taylor order N of the radial window (Eq. 10), 0 <= N <= 200
 *   gamma     inflection point of the radial window at gamma * rho_N (Sec. 3.1), 0 < gamma < 1
 *   eps       floor in M -> max(M, eps) of the stabilised inverse (Sec. 3.1), > 0
 *             (M vanishes on the Nyquist planes of even dims)
 *   variant   os3d_variant
 *   coeffs    os3d_coeffs: how the SH coefficients of A are obtained */
typedef struct {
  int32_t L;
  double s_theta;
  int32_t k;
  int32_t taylor_N;
  double gamma;
  double eps;
  int32_t variant;
  int32_t coeffs;
} os3d_wavelet_params;

/* Opaque host handle of a built bank: dims, orientation pairing, kappa and
 * pointers into the caller's bank buffer.  Immutable after os3d_build_bank;
 * calls on different streams may share it. */
typedef struct os3d_bank os3d_bank;

typedef struct {
  int64_t dims[3];       /* Nz, Ny, Nx */
  int32_t n_orients;     /* N_o */
  int32_t n_unique;      /* stored bank rows: N_o/2 when the set is antipodally closed, else N_o */
  int32_t paired;        /* 1 when every orientation has its antipode in the set */
  double kappa;          /* normaliser: the band mean of M is 1 */
  double approx_norm;    /* S: band mean of sum_i psi_hat_i, normaliser of os3d_reconstruct_approx */
  const float* M_dev;    /* M[k] on the device, frequency order of os3d_bank_M */
} os3d_bank_info;

/* Host-only wavelet design (Sec. 3.1-3.2), FP64, no device needed.
 * c_out[0..L]: coefficients c_{l,0} of A (Eq. 15) by the method p->coeffs
 * selects (least squares over the frequency-15 geodesic icosahedron, or the
 * quadrature projection);
 * a_out[0..L]: coefficients of h (cake: 2 pi P_l(0) c_l + (1 - (-1)^l) c_l,
 * Eqs. 12-16; plate: c_l).  Either output may be NULL. */
os3d_status os3d_wavelet_coeffs(const os3d_wavelet_params* p, double* c_out, double* a_out);

/* Host-only steering matrix (Eqs. 17-19 via the addition theorem), FP64:
 * S_out[(l*l + l + m) * n_orients + i] = a_l sqrt(4 pi / (2l + 1)) Y_lm(n_i)
 * for the library's real orthonormal spherical harmonics Y_lm,
 * -l <= m <= l, so that sum_lm Y_lm(w) S[lm, i] = h(angle(w, n_i)).
 * S_out holds (L+1)^2 * n_orients doubles. */
os3d_status os3d_steering_matrix(const os3d_wavelet_params* p, const double* orients, int32_t n_orients,
                                 double* S_out);

/* Bytes of the device buffer a bank needs (bank rows, M, build scratch and
 * constant tables). */
os3d_status os3d_bank_bytes(const int64_t dims[3], const double* orients, int32_t n_orients,
                            const os3d_wavelet_params* p, size_t* bytes);

/* Builds the sampled bank psi_hat_i[k] = kappa g(rho_k) h(w_k . n_i) (real;
 * Eqs. 10-19; 0 on Nyquist planes; a_0/sqrt(4 pi) at k = 0) and
 * M[k] = sum_i psi_hat_i[k]^2 (Eq. 9, constants absorbed into kappa) into
 * bank_dev (os3d_bank_bytes bytes, caller-owned, must outlive the handle).
 * The contraction over spherical harmonics runs on the matrix cores.
 * Synchronises `stream` at the end.  *out receives a new handle.
 * L > 62 returns OS3D_EUNSUPPORTED (the host-only calls accept L <= 64).
 * A grid whose dims are all < 4 has no frequency in the normalisation band
 * of kappa and returns OS3D_EINVAL. */
os3d_status os3d_build_bank(const int64_t dims[3], const double* orients, int32_t n_orients,
                            const os3d_wavelet_params* p, void* bank_dev, size_t bank_bytes,
                            void* stream, os3d_bank** out);

/* Frees the host handle (not the caller's device buffer).  NULL is a no-op. */
os3d_status os3d_free_bank(os3d_bank* bank);

os3d_status os3d_get_bank_info(const os3d_bank* bank, os3d_bank_info* info);

/* Writes psi_hat_i (float32 [Nz][Ny][Nx], natural DFT index order) of the
 * caller's orientation i into psi_dev (device). */
os3d_status os3d_bank_psi(const os3d_bank* bank, int32_t i, float* psi_dev, void* stream);

/* Writes M[k] = sum_i psi_hat_i[k]^2, the discrete stability function of
 * Eq. (9) with its constants absorbed into kappa (float32 [Nz][Ny][Nx],
 * natural DFT index order), into M_dev (device, caller-owned).  The copy
 * is enqueued on `stream`.  kappa and the library's own M (in its internal
 * frequency order) are reported by os3d_get_bank_info. */
os3d_status os3d_bank_M(const os3d_bank* bank, float* M_dev, void* stream);

/* Bytes of workspace that os3d_forward / os3d_adjoint / os3d_reconstruct /
 * os3d_process need for this bank (independent of the batch size and score
 * dtype).  A call uses the workspace until its work on `stream` has
 * finished: calls that may overlap (different streams) need workspaces of
 * their own; the bank itself is read-only and may be shared. */
os3d_status os3d_workspace_bytes(const os3d_bank* bank, size_t* bytes);

/* Discrete orientation score, Eq. (7): U[b][i] = IDFT(psi_hat_i DFT(f[b])),
 * the circular correlation of f with conj(psi_i).
 * f: device float32 [B][Nz][Ny][Nx]; U: device score (dtype as above);
 * scales: device float32 [B][N_o] written for 16-bit dtypes (may be NULL for
 * OS3D_C64); ws: device workspace of os3d_workspace_bytes bytes. */
os3d_status os3d_forward(const os3d_bank* bank, const float* f, int32_t batch, void* U,
                         int32_t dtype, float* scales, void* ws, size_t ws_bytes, void* stream);

/* Real adjoint of os3d_forward (the orientation sum of Eq. (8) without the
 * division by M): f_out[b] = Re IDFT(sum_i psi_hat_i DFT(U[b][i])).
 * U may be any complex score (not only one produced by os3d_forward). */
os3d_status os3d_adjoint(const os3d_bank* bank, const void* U, int32_t dtype, const float* scales,
                         int32_t batch, float* f_out, void* ws, size_t ws_bytes, void* stream);

/* Stabilised exact reconstruction, Eq. (8) with M -> max(M, eps) (Sec. 3.1):
 * f_out[b] = Re IDFT(sum_i psi_hat_i DFT(U[b][i]) / max(M, eps)). */
os3d_status os3d_reconstruct(const os3d_bank* bank, const void* U, int32_t dtype, const float* scales,
                             int32_t batch, float* f_out, void* ws, size_t ws_bytes, void* stream);

/* Approximate reconstruction, Eq. (6): the integral of the score over the
 * orientations, f_out[b] = Re(sum_i U[b][i]) / S, where S normalises the
 * discrete area element so that sum_i psi_hat_i averages 1 over the band
 * (|omega| <= rho_N / 2, the band of kappa).  No DFT: one pass over the scores
 * (Sec. 3.1 names it as the alternative to the stabilised inverse).
 * Arguments as for os3d_reconstruct; no workspace. */
os3d_status os3d_reconstruct_approx(const os3d_bank* bank, const void* U, int32_t dtype, const float* scales,
                                    int32_t batch, float* f_out, void* stream);

/* Processing via invertible orientation scores, Eq. (23) with the
 * stabilised inverse: f_out[b] = Re W^+ (Phi(W f[b])) for a pointwise
 * operation Phi on the scores (os3d_phi; phi_power is p of the soft
 * threshold, 0 < p <= 16).  Both kinds satisfy Phi(conj U) = conj Phi(U), so
 * for real f an antipodal pair contributes 2 Phi(U_n) to the orientation sum
 * and the scores never reach memory.  f, f_out: float32 [B][Nz][Ny][Nx];
 * ws: os3d_workspace_bytes bytes. */
os3d_status os3d_process(const os3d_bank* bank, const float* f, int32_t batch, int32_t phi, double phi_power,
                         float* f_out, void* ws, size_t ws_bytes, void* stream);

/* os3d_reconstruct without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops that
 * must not call hipMalloc): the library's own static device scratch array
 * (64 MiB, held on every device the library runs on until the process ends)
 * takes the place of the workspace, and the call allocates nothing.  It
 * holds the orientation sum and the intermediates of as many orientation
 * pairs per launch as fit (at least one): volumes up to 2^22 voxels, e.g.
 * 128^3 or 160 x 128 x 128; a larger volume returns OS3D_ENOMEM before any
 * work is enqueued.  Every call on one device shares that device's scratch:
 * calls that overlap on one device (different streams or threads without
 * ordering between them) race and give wrong results.  The result equals
 * os3d_reconstruct's up to the summation order of the orientation pairs
 * (FP32 rounding).  Other arguments and errors as for os3d_reconstruct. */
os3d_status os3d_reconstruct_noalloc(const os3d_bank* bank, const void* U, int32_t dtype, const float* scales,
                                     int32_t batch, float* f_out, void* stream);

/* Per-kernel timing (not a method step: measurement support).  While
 * enabled, a timed launch carries two HIP events that the runtime stamps
 * with the kernel's start and end on its launch stream, and the algorithmic
 * bytes that launch must move are recorded with it (scores written or read:
 * orientations x V x bytes per score; the real input and output volumes:
 * 4 V).  on = 0: off; 1: every launch; 2 + k: only the launches of kernel
 * slot k (0 <= k < os3d_profile_count), so that timing one kernel adds
 * nothing to the others.  Other values return OS3D_EINVAL.  Enabling or
 * disabling clears the records.  Not thread-safe; host memory only. */
os3d_status os3d_profile_enable(int32_t on);

/* Number of kernel slots that os3d_profile_get reports. */
os3d_status os3d_profile_count(int32_t* n_kernels);

/* Kernel slot idx: its name (static string), number of recorded launches,
 * summed event time in ms (waits for the recorded events), summed
 * algorithmic bytes and summed algorithmic flops (the bank contraction:
 * 2 V (L+1)^2 rows). */
os3d_status os3d_profile_get(int32_t idx, const char** name, int64_t* launches, double* total_ms,
                             double* alg_bytes, double* alg_flops);

/* Streaming probe (measurement support, not a method step): one pass of a
 * plain kernel over `bytes` bytes on `stream`, to measure the HBM rates a
 * copy, a read and a write reach on this GPU.  kind 0: copy src -> dst;
 * 1: read src (dst receives up to 2048 float values that keep the loads
 * live, so it must hold 8 KiB); 2: write dst (src unused, may be NULL);
 * 3: read src with non-temporal loads (dst as for 1).  bytes must be a positive multiple of
 * 16 and the buffers 16-byte aligned device memory, else OS3D_EINVAL. */
os3d_status os3d_stream_probe(int32_t kind, const void* src, void* dst, size_t bytes, void* stream);

/* Message of the calling thread's last non-OK status ("" if none). */
const char* os3d_last_error(void);

/* Library version string. */
const char* os3d_version(void);

#ifdef __cplusplus
}
#endif

#endif /* OS3D_H */
