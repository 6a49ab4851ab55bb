"""FP64 CPU oracle of the discrete invertible 3D orientation-score transform
with cake wavelets (Janssen, Duits & Breeuwer, "Invertible Orientation Scores
of 3D Images").

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline of the benchmark may import this module.  It shares no code, table
or constant generator with the HIP library: it has its own DFT (the DFT
matrix applied per axis), its own radix-2 FFT (a cross-check), its own
Legendre recursion, its own B-spline and its own geodesic sphere.  The
library primitives it calls are numpy's ``linalg.pinv`` (the least-squares
fit), ``tensordot`` (applying the DFT matrices), ``linalg.norm`` and, for
the quadrature coefficient option, ``polynomial.legendre.leggauss`` (nodes
and weights).

Parity unpinned (nothing outside this module fixes the value): the absolute
level of the least-squares coefficients c_l of ``sh_coeffs_A`` (the paper
prints none; they are bounded against the quadrature projection of
``sh_coeffs_A_quadrature``, which has closed-form pins, at about twice the
measured gap: 5.6e-5 at L = 8, 8.1e-5 at L = 16, 4.6e-4 at L = 24), and the
uniformity of M over the band (only its band mean is fixed, through kappa).

Conventions (the readings of the paper this module fixes; every one is also
a parameter or a documented constant of the library):

* Volumes are arrays ``[Nz][Ny][Nx]`` (x fastest); orientations are (x, y, z)
  unit vectors.
* DFT: ``F[k] = sum_x f[x] exp(-2 pi i k.x / N)``, unnormalised; the inverse
  carries 1/V.  The continuous (2 pi)^(3/2) constants of Eqs. (2), (3), (5)
  and (9) and the area element 4 pi / N_o are absorbed into one scale kappa
  fixed by requiring M to average 1 over a band (Sec. 2, requirement 2 of
  Sec. 3: M close to 1).
* Frequencies: omega_d = 2 pi kt_d / N_d with kt_d = k_d for k_d < N_d/2,
  else k_d - N_d; the Nyquist radius is rho_N = pi on every axis (Sec. 3.1).
* Every Nyquist plane (kt_d = -N_d/2 on an even axis) gets psi_hat = 0: the
  radial window must vanish there (Sec. 3.1), and this keeps real inputs
  mapping to conjugate pairs of scores.
* At omega = 0 the angle is undefined; psi_hat takes the sphere average of
  the angular profile, a_0 / sqrt(4 pi).
* kappa = (mean over the band of sum_i (g h_i)^2)^(-1/2); the band is every
  non-zero, non-Nyquist frequency with rho <= rho_N / 2.
"""
from __future__ import annotations

import math

import numpy as np

RHO_N = math.pi

__all__ = [
    "WaveletParams", "dft_matrix", "dft_axis", "dft3", "idft3", "fft_radix2",
    "legendre_P", "assoc_legendre_normalized", "real_sh", "bspline", "radial_g",
    "geodesic_icosahedron", "sh_coeffs_A", "sh_coeffs_A_quadrature",
    "cake_coeffs", "angular_profile", "freq_grid", "steering_matrix",
    "build_bank", "bank_values", "band_kappa", "forward", "adjoint", "reconstruct",
    "forward_bruteforce", "spatial_wavelets", "quantize_scores", "fit_zonal", "approx_norm",
    "reconstruct_approx", "soft_threshold", "process", "freq_at", "band_kappa_streamed",
    "M_at", "bank_row", "score_scale_bound", "score_scales",
]


class WaveletParams:
    """Parameters of the cake wavelet (Sec. 3): SH order L, window width
    s_theta and B-spline order k (Eq. 11), Taylor order N_T and inflection
    fraction gamma of the radial window (Eq. 10), stabiliser eps (Sec. 3.1)."""

    def __init__(self, L=16, s_theta=0.7, k=2, taylor_N=20, gamma=0.8, eps=1e-3, variant="cake", coeffs="lsq"):
        self.L = int(L)
        self.s_theta = float(s_theta)
        self.k = int(k)
        self.taylor_N = int(taylor_N)
        self.gamma = float(gamma)
        self.eps = float(eps)
        self.variant = variant  # "cake" (Eq. 14) or "plate" (h = A, Fig. 4)
        self.coeffs = coeffs    # "lsq" (pseudo-inverse fit, Sec. 3.2) or "quadrature" (projection)

    def __repr__(self):
        return (f"WaveletParams(L={self.L}, s_theta={self.s_theta}, k={self.k}, "
                f"taylor_N={self.taylor_N}, gamma={self.gamma}, eps={self.eps}, variant={self.variant!r}, "
                f"coeffs={self.coeffs!r})")


# ---------------------------------------------------------------------------
# Discrete Fourier transform (the definition, applied one axis at a time)
# ---------------------------------------------------------------------------

def dft_matrix(n, sign):
    """W[j, k] = exp(sign * 2 pi i (j k mod n) / n); the phase is reduced
    in integers first so that large n loses no accuracy."""
    j = np.arange(n, dtype=np.int64)
    ph = np.outer(j, j) % n
    return np.exp(sign * 2j * np.pi * ph.astype(np.float64) / n)


def dft_axis(a, axis, sign):
    axis = axis % a.ndim
    W = dft_matrix(a.shape[axis], sign)
    out = np.tensordot(W, a, axes=([1], [axis]))
    return np.moveaxis(out, 0, axis)


def dft3(a):
    """Unnormalised 3D DFT over the last three axes (exponent sign -1)."""
    a = np.asarray(a, dtype=np.complex128)
    for ax in (-3, -2, -1):
        a = dft_axis(a, ax, -1.0)
    return a


def idft3(a):
    """Inverse 3D DFT over the last three axes, with the 1/V factor."""
    a = np.asarray(a, dtype=np.complex128)
    v = a.shape[-1] * a.shape[-2] * a.shape[-3]
    for ax in (-3, -2, -1):
        a = dft_axis(a, ax, +1.0)
    return a / v


def fft_radix2(x, sign=-1.0):
    """Recursive decimation-in-time radix-2 FFT of a 1D array whose length is
    a power of two (a cross-check of the DFT matrix)."""
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[0]
    if n == 1:
        return x.copy()
    if n % 2:
        raise ValueError("length must be a power of two")
    even = fft_radix2(x[0::2], sign)
    odd = fft_radix2(x[1::2], sign)
    tw = np.exp(sign * 2j * np.pi * np.arange(n // 2) / n) * odd
    return np.concatenate([even + tw, even - tw])


# ---------------------------------------------------------------------------
# Legendre functions and real spherical harmonics
# ---------------------------------------------------------------------------

def legendre_P(L, x):
    """P_0..P_L at x by Bonnet's recursion (l+1) P_{l+1} = (2l+1) x P_l - l P_{l-1}.
    Returns [L+1, *x.shape]."""
    x = np.asarray(x, dtype=np.float64)
    P = np.empty((L + 1,) + x.shape)
    P[0] = 1.0
    if L >= 1:
        P[1] = x
    for l in range(1, L):
        P[l + 1] = ((2 * l + 1) * x * P[l] - l * P[l - 1]) / (l + 1)
    return P


def assoc_legendre_normalized(L, theta):
    """pbar[l, m] = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) P_l^m(cos theta) for
    0 <= m <= l <= L, without the Condon-Shortley phase, by the standard
    normalised column recursion (sectoral seed, then three-term recursion in
    l at fixed m).  Returns [L+1, L+1, *theta.shape] (zero for m > l)."""
    th = np.asarray(theta, dtype=np.float64)
    c, s = np.cos(th), np.sin(th)
    p = np.zeros((L + 1, L + 1) + th.shape)
    p[0, 0] = 1.0 / math.sqrt(4.0 * math.pi)
    for m in range(1, L + 1):
        p[m, m] = math.sqrt((2.0 * m + 1.0) / (2.0 * m)) * s * p[m - 1, m - 1]
    for m in range(0, L):
        p[m + 1, m] = math.sqrt(2.0 * m + 3.0) * c * p[m, m]
    for m in range(0, L + 1):
        for l in range(m + 2, L + 1):
            a = math.sqrt((4.0 * l * l - 1.0) / (l * l - m * m))
            b = math.sqrt(((l - 1.0) ** 2 - m * m) / (4.0 * (l - 1.0) ** 2 - 1.0))
            p[l, m] = a * (c * p[l - 1, m] - b * p[l - 2, m])
    return p


def real_sh(L, theta, phi):
    """Real orthonormal spherical harmonics, index l*l + l + m:
    Y_l0 = pbar_l0, Y_lm = sqrt2 pbar_lm cos(m phi), Y_l,-m = sqrt2 pbar_lm sin(m phi)."""
    th = np.asarray(theta, dtype=np.float64)
    ph = np.asarray(phi, dtype=np.float64)
    p = assoc_legendre_normalized(L, th)
    Y = np.zeros(((L + 1) ** 2,) + th.shape)
    r2 = math.sqrt(2.0)
    for l in range(L + 1):
        Y[l * l + l] = p[l, 0]
        for m in range(1, l + 1):
            Y[l * l + l + m] = r2 * p[l, m] * np.cos(m * ph)
            Y[l * l + l - m] = r2 * p[l, m] * np.sin(m * ph)
    return Y


# ---------------------------------------------------------------------------
# Wavelet design (Sec. 3)
# ---------------------------------------------------------------------------

def bspline(k, x):
    """Centred cardinal B-spline of order k, B^k = B^(k-1) * B^0 (Eq. 11), in
    its closed form (1/k!) sum_j (-1)^j C(k+1, j) (x + (k+1)/2 - j)_+^k."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    for j in range(k + 2):
        t = x + (k + 1) / 2.0 - j
        if k == 0:
            tp = (t > 0).astype(np.float64)
        else:
            tp = np.where(t > 0, t, 0.0) ** k
        out += (-1) ** j * math.comb(k + 1, j) * tp
    return out / math.factorial(k)


def radial_g(rho, gamma, taylor_N, rho_N=RHO_N):
    """Radial window of Eq. (10): exp(-x) sum_{j<=N} x^j / j!, x = rho^2 / t,
    with t = 2 (gamma rho_N)^2 / (1 + 2N) placing the inflection point at
    gamma rho_N (Sec. 3.1)."""
    rho = np.asarray(rho, dtype=np.float64)
    t = 2.0 * (gamma * rho_N) ** 2 / (1.0 + 2.0 * taylor_N)
    x = rho * rho / t
    term = np.exp(-x)
    acc = term.copy()
    for j in range(1, taylor_N + 1):
        term = term * x / j
        acc = acc + term
    return acc


def geodesic_icosahedron(freq):
    """Class-I geodesic sphere: every face of the icosahedron whose vertices
    are the cyclic permutations of (0, +-1, +-phi) is split into freq^2
    triangles by planar barycentric points, which are projected onto the unit
    sphere.  10 freq^2 + 2 distinct points."""
    p = (1.0 + 5.0 ** 0.5) / 2.0
    v = []
    for a in (-1.0, 1.0):
        for b in (-p, p):
            v += [(0.0, a, b), (a, b, 0.0), (b, 0.0, a)]
    v = np.array(v)
    d = np.linalg.norm(v[:, None] - v[None, :], axis=2)
    e = d[d > 0].min()
    adj = np.abs(d - e) < 1e-9
    pts = []
    for i in range(12):
        for j in range(i + 1, 12):
            for k in range(j + 1, 12):
                if adj[i, j] and adj[i, k] and adj[j, k]:
                    for a in range(freq + 1):
                        for b in range(freq + 1 - a):
                            c = freq - a - b
                            pts.append((a * v[i] + b * v[j] + c * v[k]) / freq)
    pts = np.array(pts)
    pts /= np.linalg.norm(pts, axis=1, keepdims=True)
    key = np.round(pts * 1e9).astype(np.int64)
    _, idx = np.unique(key, axis=0, return_index=True)
    return pts[np.sort(idx)]


def _window_A(theta, params):
    """Orientation distribution A(theta) = B^k(theta / s_theta) (Sec. 3.1)."""
    return bspline(params.k, np.asarray(theta) / params.s_theta)


def fit_zonal(fun, L, freq=15):
    """Coefficients c_l (l = 0..L) of the zonal expansion sum_l c_l Y_l^0
    fitted to fun(theta) by the pseudo-inverse of the sampled synthesis
    matrix over the points of the frequency-`freq` geodesic icosahedron
    (Sec. 3.2: only m = 0 is needed for a z-symmetric window)."""
    pts = geodesic_icosahedron(freq)
    z = np.clip(pts[:, 2], -1.0, 1.0)
    P = legendre_P(L, z)
    Y0 = (np.sqrt((2 * np.arange(L + 1) + 1) / (4 * math.pi))[:, None] * P).T
    return np.linalg.pinv(Y0) @ fun(np.arccos(z))


def sh_coeffs_A(params, freq=15):
    """c_{l,0} of the window A = B^k(theta / s_theta) (Sec. 3.2)."""
    return fit_zonal(lambda th: _window_A(th, params), params.L, freq)


def sh_coeffs_A_quadrature(params, nodes=64):
    """Projection c_l = 2 pi int_0^pi A(theta) Y_l^0(theta) sin(theta) dtheta
    by composite Gauss-Legendre in theta split at the B-spline knots: the
    alternative to the least-squares fit (params.coeffs = "quadrature"),
    differing from it by the fit's discretisation error only."""
    L, k, s = params.L, params.k, params.s_theta
    knots = [0.0] + [s * (j - (k + 1) / 2.0) for j in range(k + 2)
                     if 0.0 < s * (j - (k + 1) / 2.0) < math.pi] + [math.pi]
    knots = sorted(set(knots))
    xg, wg = np.polynomial.legendre.leggauss(nodes)
    c = np.zeros(L + 1)
    for a, b in zip(knots[:-1], knots[1:]):
        th = 0.5 * (b - a) * xg + 0.5 * (b + a)
        w = 0.5 * (b - a) * wg
        P = legendre_P(L, np.cos(th))
        Yl0 = np.sqrt((2 * np.arange(L + 1) + 1) / (4 * math.pi))[:, None] * P
        c += 2 * math.pi * (Yl0 * (_window_A(th, params) * np.sin(th) * w)[None, :]).sum(axis=1)
    return c


def cake_coeffs(c, variant="cake"):
    """Angular-profile coefficients a_l.  Cake wavelet (Eq. 14): the Funk
    transform (Eq. 16) maps c_l to 2 pi P_l(0) c_l and gives the real line
    detector (Eq. 13); antisymmetrisation maps c_l to (1 - (-1)^l) c_l and
    gives the imaginary edge detector (Eq. 12).  Plate detector (Fig. 4):
    a_l = c_l (h = A)."""
    c = np.asarray(c, dtype=np.float64)
    if variant == "plate":
        return c.copy()
    L = c.shape[0] - 1
    P0 = legendre_P(L, np.array(0.0))
    l = np.arange(L + 1)
    return 2 * math.pi * P0 * c + (1 - (-1.0) ** l) * c


def angular_profile(a, cosang):
    """h(theta) = sum_l a_l Y_l^0(theta) as a function of cos(theta)."""
    L = a.shape[0] - 1
    P = legendre_P(L, cosang)
    w = np.asarray(a) * np.sqrt((2 * np.arange(L + 1) + 1) / (4 * math.pi))
    return np.tensordot(w, P, axes=(0, 0))


def steering_matrix(a, orients):
    """S[l*l+l+m, i] = a_l sqrt(4 pi/(2l+1)) Y_lm(n_i): by the addition
    theorem sum_lm Y_lm(w) S[lm, i] = sum_l a_l Y_l^0 evaluated at the angle
    between w and n_i, i.e. the rotated profile h_{n_i} of Eqs. (17)-(19)."""
    n = np.asarray(orients, dtype=np.float64)
    th = np.arccos(np.clip(n[:, 2], -1, 1))
    ph = np.arctan2(n[:, 1], n[:, 0])
    L = a.shape[0] - 1
    Y = real_sh(L, th, ph)
    S = np.zeros_like(Y)
    for l in range(L + 1):
        S[l * l:(l + 1) ** 2] = a[l] * math.sqrt(4 * math.pi / (2 * l + 1)) * Y[l * l:(l + 1) ** 2]
    return S


# ---------------------------------------------------------------------------
# The sampled wavelet bank and M
# ---------------------------------------------------------------------------

def _axis_omega(n):
    k = np.arange(n)
    kt = np.where(k < (n + 1) // 2, k, k - n)
    nyq = (k == n // 2) if n % 2 == 0 else np.zeros(n, dtype=bool)
    return 2 * math.pi * kt / n, nyq


def freq_grid(shape):
    """omega_z, omega_y, omega_x (broadcastable) and the Nyquist-plane mask."""
    nz, ny, nx = shape
    wz, qz = _axis_omega(nz)
    wy, qy = _axis_omega(ny)
    wx, qx = _axis_omega(nx)
    wz, wy, wx = wz[:, None, None], wy[None, :, None], wx[None, None, :]
    nyq = qz[:, None, None] | qy[None, :, None] | qx[None, None, :]
    return wz, wy, wx, nyq


def bank_values(wz, wy, wx, nyq, orients, a, params):
    """psi_hat_i (before kappa) at given frequencies: g(rho) h(w_hat . n_i);
    0 on Nyquist planes; a_0/sqrt(4 pi) at the origin.  Returns
    [N_o, *broadcast shape]."""
    wz, wy, wx = np.broadcast_arrays(wz, wy, wx)
    nyq = np.broadcast_to(nyq, wz.shape)
    rho = np.sqrt(wx * wx + wy * wy + wz * wz)
    g = radial_g(rho, params.gamma, params.taylor_N)
    safe = np.where(rho > 0, rho, 1.0)
    out = np.empty((len(orients),) + wz.shape)
    for i, n in enumerate(np.asarray(orients, dtype=np.float64)):
        c = (wx * n[0] + wy * n[1] + wz * n[2]) / safe
        h = angular_profile(a, np.clip(c, -1.0, 1.0))
        h = np.where(rho > 0, h, a[0] / math.sqrt(4 * math.pi))
        out[i] = np.where(nyq, 0.0, g * h)
    return out


def band_kappa(raw_M, shape):
    """kappa = (mean over the band of the un-normalised M)^(-1/2)."""
    wz, wy, wx, nyq = freq_grid(shape)
    rho = np.sqrt(wx * wx + wy * wy + wz * wz)
    band = (rho > 0) & (rho <= RHO_N / 2) & ~nyq
    if not band.any():
        # every dim < 4: no non-zero frequency within half the Nyquist radius
        raise ValueError(f"the normalisation band of grid {shape} is empty (some dim must be >= 4)")
    return 1.0 / math.sqrt(float(np.mean(raw_M[band])))


def build_bank(shape, orients, params):
    """The sampled bank psi_hat [N_o][Nz][Ny][Nx] (real, FP64), M = sum_i
    psi_hat_i^2 (Eq. 9 with its constants absorbed into kappa), kappa, and
    the coefficient vectors (c, a)."""
    shape = tuple(int(s) for s in shape)
    c = sh_coeffs_A_quadrature(params) if params.coeffs == "quadrature" else sh_coeffs_A(params)
    a = cake_coeffs(c, params.variant)
    wz, wy, wx, nyq = freq_grid(shape)
    raw = bank_values(wz, wy, wx, nyq, orients, a, params)
    M0 = np.sum(raw * raw, axis=0)
    kappa = band_kappa(M0, shape)
    return dict(psi_hat=raw * kappa, M=M0 * kappa * kappa, kappa=kappa, c=c, a=a,
                shape=shape, orients=np.asarray(orients, dtype=np.float64), params=params)


def spatial_wavelets(bank):
    """psi_i = IDFT(psi_hat_i): the discrete wavelets in the spatial domain."""
    return idft3(bank["psi_hat"])


# ---------------------------------------------------------------------------
# The transform, its adjoint and its stabilised inverse
# ---------------------------------------------------------------------------

def forward(f, bank):
    """Discrete orientation score of Eq. (7): U_i = IDFT(psi_hat_i DFT(f)),
    i.e. the circular correlation of f with conj(psi_i).  [N_o][Nz][Ny][Nx] complex."""
    F = dft3(np.asarray(f, dtype=np.float64))
    return idft3(bank["psi_hat"] * F[None])


def _orientation_sum(U, bank):
    X = np.zeros(bank["shape"], dtype=np.complex128)
    for i in range(U.shape[0]):
        X += bank["psi_hat"][i] * dft3(U[i])
    return X


def adjoint(U, bank):
    """Real adjoint of the forward map: Re IDFT(sum_i psi_hat_i DFT(U_i))
    (the orientation sum of Eq. 8 without the division by M)."""
    return np.real(idft3(_orientation_sum(np.asarray(U), bank)))


def reconstruct(U, bank, eps=None):
    """Stabilised exact reconstruction, Eq. (8) with M replaced by max(M, eps)
    (Sec. 3.1): Re IDFT(sum_i psi_hat_i DFT(U_i) / max(M, eps))."""
    eps = bank["params"].eps if eps is None else eps
    X = _orientation_sum(np.asarray(U), bank)
    return np.real(idft3(X / np.maximum(bank["M"], eps)))


def approx_norm(bank):
    """S = mean over the band of sum_i psi_hat_i[k]: the discrete area element
    of Eq. (6) normalised so that the orientation sum of the bank averages 1."""
    wz, wy, wx, nyq = freq_grid(bank["shape"])
    rho = np.sqrt(wx * wx + wy * wy + wz * wz)
    band = (rho > 0) & (rho <= RHO_N / 2) & ~nyq
    return float(np.mean(np.sum(bank["psi_hat"], axis=0)[band]))


def reconstruct_approx(U, bank):
    """Approximate reconstruction of Eq. (6): the integral of the score over
    the orientations, Re(sum_i U_i) / S (no inverse filter)."""
    return np.real(np.sum(np.asarray(U), axis=0)) / approx_norm(bank)


def soft_threshold(U, p):
    """Phi(U) = |U|^p sgn(U), sgn(U) = U / |U| (0 where U = 0): the pointwise
    score operation of Fig. 7 (p = 1.5 there), applied to the complex score."""
    U = np.asarray(U)
    m = np.abs(U)
    out = np.zeros_like(U)
    nz = m > 0
    out[nz] = U[nz] * m[nz] ** (p - 1.0)
    return out


def process(f, bank, phi="soft_threshold", p=1.5):
    """Processing via invertible orientation scores, Eq. (23): the stabilised
    reconstruction of Phi applied to the score of f."""
    U = forward(f, bank)
    if phi == "soft_threshold":
        U = soft_threshold(U, p)
    elif phi != "identity":
        raise ValueError(phi)
    return reconstruct(U, bank)


def forward_bruteforce(f, bank):
    """Eq. (7) literally: U_i[x] = sum_x' conj(psi_i[(x' - x) mod N]) f[x']
    with psi_i = IDFT(psi_hat_i).  O(V^2 N_o): tiny volumes only."""
    f = np.asarray(f, dtype=np.float64)
    psi = spatial_wavelets(bank)
    nz, ny, nx = f.shape
    U = np.zeros((psi.shape[0],) + f.shape, dtype=np.complex128)
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                sh = psi[:, (zz - z) % nz, (yy - y) % ny, (xx - x) % nx]
                U[:, z, y, x] = np.sum(np.conj(sh) * f[None], axis=(1, 2, 3))
    return U


# ---------------------------------------------------------------------------
# Reduced-precision score storage (per-orientation power-of-two scale)
# ---------------------------------------------------------------------------

def _bf16_round(x32):
    b = np.asarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def score_scale_bound(F, psi_hat_i):
    """Bound of max |Re U_i|, |Im U_i| known before the inverse DFT: since
    U_i = IDFT(psi_hat_i F), every |U_i[x]| <= (1/V) sum_k |psi_hat_i[k] F[k]|."""
    F = np.asarray(F)
    return float(np.sum(np.abs(np.asarray(psi_hat_i) * F)) / F.size)


def score_scales(bounds, fmt):
    """Per-orientation power-of-two scale of 16-bit storage from the bounds
    of score_scale_bound: s_i = 2^e_i with bound_i = m 2^e_i, m in [0.5, 1)
    (the smallest power of two above the bound), for bf16; 2^(e_i - 15) for
    fp16, so that U_i / s_i stays below 2^15 < 65504."""
    out = np.ones(len(bounds))
    for i, b in enumerate(bounds):
        if b > 0:
            e = math.frexp(b)[1]
            out[i] = math.ldexp(1.0, e - 15 if fmt == "fp16" else e)
    return out


def quantize_scores(U, fmt, s):
    """Store U_i / s_i as a pair of 16-bit floats (round to nearest even)
    with the per-orientation scales s (score_scales).  Returns the
    dequantised values."""
    U = np.asarray(U)
    out = np.empty_like(U, dtype=np.complex128)
    for i in range(U.shape[0]):
        re = (U[i].real / s[i]).astype(np.float32)
        im = (U[i].imag / s[i]).astype(np.float32)
        if fmt == "fp16":
            re, im = re.astype(np.float16).astype(np.float64), im.astype(np.float16).astype(np.float64)
        elif fmt == "bf16":
            re, im = _bf16_round(re).astype(np.float64), _bf16_round(im).astype(np.float64)
        else:
            raise ValueError(fmt)
        out[i] = (re + 1j * im) * s[i]
    return out


# ---------------------------------------------------------------------------
# The same bank quantities without the full grid in memory (large volumes)
# ---------------------------------------------------------------------------

def freq_at(shape, idx):
    """omega_z, omega_y, omega_x and the Nyquist-plane flag at flat frequency
    indices idx (natural order, x fastest)."""
    nz, ny, nx = shape
    idx = np.asarray(idx, dtype=np.int64)
    kz, r = np.divmod(idx, ny * nx)
    ky, kx = np.divmod(r, nx)
    (wz, qz), (wy, qy), (wx, qx) = _axis_omega(nz), _axis_omega(ny), _axis_omega(nx)
    return wz[kz], wy[ky], wx[kx], qz[kz] | qy[ky] | qx[kx]


def _band_indices(shape):
    """Flat indices of the kappa band (0 < rho <= rho_N / 2, no Nyquist plane)."""
    wz, wy, wx, nyq = freq_grid(shape)
    rho2 = wx * wx + wy * wy + wz * wz
    band = (rho2 > 0) & (rho2 <= (RHO_N / 2) ** 2) & ~nyq
    return np.flatnonzero(band)


def band_kappa_streamed(shape, orients, a, params, chunk=1 << 17):
    """kappa of build_bank (the band mean of sum_i (g h_i)^2 to the power
    -1/2) visiting only the band's frequencies, a chunk at a time."""
    idx = _band_indices(shape)
    if idx.size == 0:
        raise ValueError(f"the normalisation band of grid {shape} is empty (some dim must be >= 4)")
    tot = 0.0
    for c0 in range(0, idx.size, chunk):
        wz, wy, wx, nyq = freq_at(shape, idx[c0:c0 + chunk])
        raw = bank_values(wz, wy, wx, nyq, orients, a, params)
        tot += float(np.sum(raw * raw))
    return 1.0 / math.sqrt(tot / idx.size)


def M_at(shape, idx, orients, a, params, kappa, chunk=1 << 15):
    """M = sum_i psi_hat_i^2 (Eq. 9) at flat frequency indices idx."""
    idx = np.asarray(idx, dtype=np.int64)
    out = np.empty(idx.size)
    for c0 in range(0, idx.size, chunk):
        wz, wy, wx, nyq = freq_at(shape, idx[c0:c0 + chunk])
        raw = bank_values(wz, wy, wx, nyq, orients, a, params)
        out[c0:c0 + chunk] = kappa * kappa * np.sum(raw * raw, axis=0)
    return out


def bank_row(shape, orient, a, params, kappa, slab=16):
    """psi_hat of one orientation over the whole grid [Nz][Ny][Nx] (kappa
    times g h, build_bank's row), evaluated a z-slab at a time."""
    wz, wy, wx, nyq = freq_grid(shape)
    out = np.empty(tuple(shape))
    n = np.asarray(orient, dtype=np.float64)[None]
    for z0 in range(0, shape[0], slab):
        out[z0:z0 + slab] = kappa * bank_values(wz[z0:z0 + slab], wy, wx, nyq[z0:z0 + slab], n, a, params)[0]
    return out
