"""The C-ABI library on the CPU: it loads, exports every declared symbol,
its host-only FP64 wavelet design (the coefficient setup and steering
matrix) matches the oracle, and argument errors come back as status codes
before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_1505_07690_amd import inputs
from paper_1505_07690_amd import os3d

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^\s*(?:os3d_status|const char\s*\*)\s*(os3d_[A-Za-z_0-9]+)\s*\(", txt, re.M))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = os3d.lib()
    syms = declared_symbols()
    assert len(syms) == 21, syms
    for s in syms:
        assert hasattr(L, s), s
    assert L.os3d_version().decode().startswith("os3d")


@pytest.mark.parametrize("L,s,variant", [(8, 1.31, "cake"), (16, 0.7, "cake"), (24, 0.356, "cake"),
                                         (16, 0.6, "plate"), (4, 2.0, "cake")])
def test_host_coefficients_match_oracle(L, s, variant):
    """Sec. 3.2: least-squares c_l on the geodesic sphere; Eqs. 12-16: a_l."""
    p = O.WaveletParams(L=L, s_theta=s, variant=variant)
    c_lib, a_lib = os3d.wavelet_coeffs(p)
    c_or = O.sh_coeffs_A(p)
    a_or = O.cake_coeffs(c_or, variant)
    assert np.max(np.abs(c_lib - c_or)) < 1e-12 * max(1.0, np.max(np.abs(c_or)))
    assert np.max(np.abs(a_lib - a_or)) < 1e-12 * max(1.0, np.max(np.abs(a_or)))


@pytest.mark.parametrize("L,s,k", [(8, 1.31, 2), (24, 0.356, 2), (16, 0.5, 3), (6, 1.0, 0)])
def test_host_quadrature_coefficients_match_oracle(L, s, k):
    """The quadrature projection option: composite Gauss-Legendre at the
    B-spline knots, host C++ against the oracle."""
    p = O.WaveletParams(L=L, s_theta=s, k=k, coeffs="quadrature")
    c_lib, a_lib = os3d.wavelet_coeffs(p)
    c_or = O.sh_coeffs_A_quadrature(p)
    assert np.max(np.abs(c_lib - c_or)) < 1e-13 * max(1.0, np.max(np.abs(c_or)))
    assert np.max(np.abs(a_lib - O.cake_coeffs(c_or))) < 1e-12 * max(1.0, np.max(np.abs(c_or)))


def test_host_steering_matrix_blocks():
    """Eqs. 17-19 by the addition theorem: for every l,
    sum_m S[lm, i] S[lm, j] = a_l^2 (4 pi / (2l+1)) (2l+1)/(4 pi) P_l(n_i . n_j),
    independent of the sign and ordering conventions of the real harmonics."""
    p = O.WaveletParams(L=16, s_theta=0.7)
    n = inputs.icosahedral_orientations(1)
    S = os3d.steering_matrix(p, n)
    a = O.cake_coeffs(O.sh_coeffs_A(p))
    G = n @ n.T
    P = O.legendre_P(16, np.clip(G, -1, 1))
    for l in range(17):
        blk = S[l * l:(l + 1) ** 2]
        assert np.max(np.abs(blk.T @ blk - a[l] ** 2 * P[l])) < 1e-12


def test_host_steering_reproduces_profile():
    """sum_lm Y_lm(w) S[lm, i] = h(w . n_i) with the oracle's real harmonics
    (same orthonormal basis up to per-(l, m) signs, which cancel in S Y)."""
    p = O.WaveletParams(L=12, s_theta=0.9)
    n = inputs.icosahedral_orientations(0)
    S_lib = os3d.steering_matrix(p, n)
    S_or = O.steering_matrix(O.cake_coeffs(O.sh_coeffs_A(p)), n)
    # both are steering matrices for some orthonormal real basis: their Gram
    # matrices over the orientations agree
    assert np.max(np.abs(S_lib.T @ S_lib - S_or.T @ S_or)) < 1e-11


def test_errors_are_status_codes():
    L = os3d.lib()
    n = inputs.icosahedral_orientations(0)
    good = os3d.make_params(L=8, s_theta=1.3)
    nbytes = ctypes.c_size_t()
    dims = (ctypes.c_int64 * 3)(8, 8, 8)
    assert L.os3d_bank_bytes(dims, n.ctypes.data, 12, ctypes.byref(good), ctypes.byref(nbytes)) == 0
    assert nbytes.value > 12 // 2 * 512 * 4
    bad_dims = (ctypes.c_int64 * 3)(8, 7, 8)
    assert L.os3d_bank_bytes(bad_dims, n.ctypes.data, 12, ctypes.byref(good), ctypes.byref(nbytes)) == -3
    huge = (ctypes.c_int64 * 3)(1024, 2048, 2048)  # every dim allowed, 2^32 voxels in all
    assert L.os3d_bank_bytes(huge, n.ctypes.data, 12, ctypes.byref(good), ctypes.byref(nbytes)) == -3
    assert b"2^31" in L.os3d_last_error()
    largest = (ctypes.c_int64 * 3)(512, 2048, 2048)
    assert L.os3d_bank_bytes(largest, n.ctypes.data, 12, ctypes.byref(good), ctypes.byref(nbytes)) == 0
    assert nbytes.value > 6 * (1 << 31) * 4
    tiny = (ctypes.c_int64 * 3)(8, 1, 8)
    assert L.os3d_bank_bytes(tiny, n.ctypes.data, 12, ctypes.byref(good), ctypes.byref(nbytes)) == -1
    for field, val in [("L", -1), ("L", 65), ("s_theta", 0.0), ("k", -1), ("taylor_N", -2), ("gamma", 1.0),
                       ("gamma", 0.0), ("eps", 0.0), ("variant", 7), ("coeffs", 2)]:
        p = os3d.make_params(L=8, s_theta=1.3)
        setattr(p, field, val)
        assert L.os3d_bank_bytes(dims, n.ctypes.data, 12, ctypes.byref(p), ctypes.byref(nbytes)) == -1, field
        assert L.os3d_last_error().decode() != ""
    nonunit = n.copy()
    nonunit[3] *= 1.001
    assert L.os3d_bank_bytes(dims, nonunit.ctypes.data, 12, ctypes.byref(good), ctypes.byref(nbytes)) == -1
    assert b"unit" in L.os3d_last_error()
    # build with a NULL device buffer is rejected before any device call
    h = ctypes.c_void_p()
    assert L.os3d_build_bank(dims, n.ctypes.data, 12, ctypes.byref(good), None, 0, None, ctypes.byref(h)) == -1
    # the device synthesis stops at L = 62 (before touching the buffer)
    high = os3d.make_params(L=63, s_theta=1.3)
    fake = ctypes.c_void_p(8)
    assert L.os3d_build_bank(dims, n.ctypes.data, 12, ctypes.byref(high), fake, 1 << 40, None, ctypes.byref(h)) == -3
    assert b"L <= 62" in L.os3d_last_error()
    # a grid with an empty normalisation band (every dim < 4)
    small = (ctypes.c_int64 * 3)(2, 3, 3)
    assert L.os3d_build_bank(small, n.ctypes.data, 12, ctypes.byref(good), fake, 1 << 40, None, ctypes.byref(h)) == -1
    assert b"band is empty" in L.os3d_last_error()
    # compute calls with a NULL bank
    assert L.os3d_forward(None, None, 1, None, 0, None, None, 0, None) == -1
    assert L.os3d_reconstruct(None, None, 0, None, 1, None, None, 0, None) == -1
    assert L.os3d_adjoint(None, None, 0, None, 1, None, None, 0, None) == -1
    assert L.os3d_reconstruct_approx(None, None, 0, None, 1, None, None) == -1
    assert L.os3d_process(None, None, 1, 0, 1.5, None, None, 0, None) == -1
    assert L.os3d_free_bank(None) == 0
    # timing modes: off, every launch, one slot; nothing else
    nslots = ctypes.c_int32()
    assert L.os3d_profile_count(ctypes.byref(nslots)) == 0
    for mode in (0, 1, 2, 2 + nslots.value - 1, 0):
        assert L.os3d_profile_enable(mode) == 0, mode
    for mode in (-1, 2 + nslots.value):
        assert L.os3d_profile_enable(mode) == -1, mode
    assert os3d.profile_slots()[-1] == "bank_synth_mfma"


def test_bank_bytes_halved_for_antipodal_sets():
    """Antipodally closed sets store one bank row per pair."""
    p = os3d.make_params(L=8, s_theta=1.3)
    n = inputs.icosahedral_orientations(0)
    V = 16 ** 3
    full = os3d.bank_bytes((16, 16, 16), n, p)
    # six random directions have no antipodes: one row each, as many rows as the 6 pairs
    v = np.random.default_rng(0).standard_normal((6, 3))
    six = os3d.bank_bytes((16, 16, 16), v / np.linalg.norm(v, axis=1, keepdims=True), p)
    assert six == full
    # a 13th, unpaired orientation disables pairing: 13 rows
    odd = os3d.bank_bytes((16, 16, 16), np.vstack([n, [[0.0, 0.0, 1.0]]]), p)
    assert odd - full >= 7 * V * 4
