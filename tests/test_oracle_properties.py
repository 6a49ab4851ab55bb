"""Property tests with hypothesis: random grids (every dim a product of 2, 3
and 5), random orientation sets with and without antipodes, random window
parameters.  Each example checks what the paper and the mathematics fix for
any such input: Eq. (7) as a literal circular correlation, the Gram identity
W^H W = M (Eq. 9), the adjoint identity, conjugate antipodal scores of a real
volume, M with band mean 1 (requirement 2 of Sec. 3 through kappa) and even
for antipodal sets, and the pair identity behind the halved reconstruction.
The last test draws wavelet parameters and checks the host C++ design of the
C ABI against the oracle.  CPU only."""
import numpy as np
from hypothesis import HealthCheck, assume, given, settings
from hypothesis import strategies as st

import oracle as O
from paper_1505_07690_amd import os3d

DIMS = st.sampled_from([2, 3, 4, 5, 6, 8, 9, 10, 12])
SETTINGS = settings(max_examples=30, deadline=None, suppress_health_check=[HealthCheck.too_slow])


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


@st.composite
def cases(draw):
    shape = (draw(DIMS), draw(DIMS), draw(DIMS))
    assume(max(shape) >= 4)  # a non-empty normalisation band
    seed = draw(st.integers(0, 2 ** 31 - 1))
    rng = np.random.default_rng(seed)
    n_half = draw(st.integers(1, 5))
    v = rng.standard_normal((n_half, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    paired = draw(st.booleans())
    orients = np.vstack([v, -v]) if paired else v
    params = O.WaveletParams(L=draw(st.integers(0, 12)), s_theta=draw(st.floats(0.3, 1.5)),
                             k=draw(st.integers(0, 3)), variant=draw(st.sampled_from(["cake", "plate"])))
    return shape, orients, paired, params, rng


@SETTINGS
@given(cases())
def test_transform_identities_on_random_inputs(case):
    shape, n, paired, p, rng = case
    b = O.build_bank(shape, n, p)
    f = rng.standard_normal(shape)
    U = O.forward(f, b)
    F = O.dft3(f)
    # W^H W is the Fourier multiplier M
    assert rel(O.adjoint(U, b), np.real(O.idft3(b["M"] * F))) < 1e-12
    # <W f, Z> = <f, W^H Z> (real parts) for a general complex Z
    Z = rng.standard_normal(U.shape) + 1j * rng.standard_normal(U.shape)
    lhs = np.real(np.vdot(U, Z))
    assert abs(lhs - np.sum(f * O.adjoint(Z, b))) < 1e-11 * max(1.0, np.linalg.norm(U) * np.linalg.norm(Z))
    # M is non-negative with band mean 1; even when the set is closed under
    # antipodes (psi_-n(w) = psi_n(-w)), not in general
    M = b["M"]
    assert np.min(M) >= 0.0
    if paired:
        assert np.max(np.abs(M - np.roll(np.flip(M, axis=(0, 1, 2)), 1, axis=(0, 1, 2)))) < 1e-12 * np.max(M)
    wz, wy, wx, nyq = O.freq_grid(shape)
    rho = np.sqrt(wx ** 2 + wy ** 2 + wz ** 2)
    band = (rho > 0) & (rho <= np.pi / 2) & ~nyq
    assert abs(np.mean(M[band]) - 1.0) < 1e-12
    if paired:
        h = len(n) // 2
        # a real volume has conjugate scores on antipodal orientations
        assert rel(U[h:], np.conj(U[:h])) < 1e-12
        # the reconstruction from pairs (Z_n + conj Z_-n, one row each) is the full one
        X = np.zeros(shape, dtype=complex)
        for i in range(h):
            X += b["psi_hat"][i] * O.dft3(Z[i] + np.conj(Z[h + i]))
        pair = np.real(O.idft3(X / np.maximum(M, p.eps)))
        assert rel(pair, O.reconstruct(Z, b)) < 1e-12


@settings(max_examples=15, deadline=None)
@given(st.integers(0, 2 ** 31 - 1), st.sampled_from([(2, 3, 4), (4, 4, 2), (3, 5, 4), (6, 2, 5)]))
def test_fft_path_equals_literal_correlation(seed, shape):
    """Eq. (7) literally, U_i(x) = sum_y conj(psi_i(y - x)) f(y), on tiny grids."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((3, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    b = O.build_bank(shape, v, O.WaveletParams(L=6, s_theta=0.8))
    f = rng.standard_normal(shape)
    assert rel(O.forward(f, b), O.forward_bruteforce(f, b)) < 1e-12


@SETTINGS
@given(L=st.integers(0, 40), s=st.floats(0.25, 2.0), k=st.integers(0, 4),
       coeffs=st.sampled_from(["lsq", "quadrature"]), variant=st.sampled_from(["cake", "plate"]))
def test_host_design_matches_oracle_on_random_parameters(L, s, k, coeffs, variant):
    """The host C++ coefficient setup (Sec. 3.2, Eqs. 12-16) of the C ABI
    against the oracle for random L, s_theta, k, method and variant."""
    p = O.WaveletParams(L=L, s_theta=s, k=k, coeffs=coeffs, variant=variant)
    c_lib, a_lib = os3d.wavelet_coeffs(p)
    c_or = O.sh_coeffs_A(p) if coeffs == "lsq" else O.sh_coeffs_A_quadrature(p)
    a_or = O.cake_coeffs(c_or, variant)
    scale = max(1.0, np.max(np.abs(c_or)))
    assert np.max(np.abs(c_lib - c_or)) < 1e-10 * scale
    assert np.max(np.abs(a_lib - a_or)) < 1e-10 * max(1.0, np.max(np.abs(a_or)))
