"""Symmetries and identities of the transform checked on the GPU path:
pyritohedral rotation covariance (Sec. 2: the cubic grid and the icosahedral
sets are mapped to themselves), the delta response (Eq. 7: reflected
conjugate wavelets, against the oracle's spatial wavelets), shift
covariance, the wavelet parity of requirement 6 (Sec. 3), the Gram identity
W^H W = M and the norm identity (Eq. 5 / Theorem 1) against the oracle's M.
Shift covariance and the norm identity also run at 256^3."""
import numpy as np
import pytest

import oracle as O
from paper_1505_07690_amd import inputs

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    from paper_1505_07690_amd import os3d
    os3d.lib()
    return t


def _bank(shape, level, L):
    from paper_1505_07690_amd import os3d
    n = inputs.icosahedral_orientations(level)
    p = O.WaveletParams(L=L, s_theta=inputs.s_theta_for(len(n)))
    return n, p, os3d.Bank(shape, n, p)


def test_pyritohedral_covariance_gpu(torch):
    """W[f o R^-1](x, R n_i) = W[f](R^-1 x, n_i) for cyclic axis permutations
    and sign flips (exact on the grid given psi_hat = 0 on Nyquist planes)."""
    from paper_1505_07690_amd import os3d
    N = 32
    n, p, gb = _bank((N, N, N), 1, 16)
    f = np.random.default_rng(8).standard_normal((N, N, N)).astype(np.float32)
    U = os3d.forward(torch.from_numpy(f).cuda(), gb)[0].cpu().numpy()
    idx = np.indices((N, N, N)).reshape(3, -1)
    xyz = idx[::-1]
    for perm in [(1, 2, 0), (2, 0, 1)]:
        for signs in [(1, 1, 1), (-1, 1, 1), (1, -1, -1)]:
            R = np.zeros((3, 3))
            for r in range(3):
                R[r, perm[r]] = signs[r]
            src = (R.T @ xyz).astype(int) % N
            g = np.ascontiguousarray(f[src[2], src[1], src[0]].reshape(N, N, N))
            Ug = os3d.forward(torch.from_numpy(g).cuda(), gb)[0].cpu().numpy()
            Rn = n @ R.T
            match = np.argmin(np.linalg.norm(Rn[:, None] - n[None], axis=2), axis=1)
            rhs = U[:, src[2], src[1], src[0]].reshape(len(n), N, N, N)
            assert rel(Ug[match], rhs) < 1e-6, (perm, signs)


def test_delta_response_is_reflected_conjugate_wavelet(torch):
    from paper_1505_07690_amd import os3d
    shape = (12, 16, 20)
    n, p, gb = _bank(shape, 1, 16)
    f = np.zeros(shape, dtype=np.float32)
    f[0, 0, 0] = 1.0
    U = os3d.forward(torch.from_numpy(f).cuda(), gb)[0].cpu().numpy()
    psi = O.spatial_wavelets(O.build_bank(shape, n, p))
    refl = np.conj(np.roll(np.flip(psi, axis=(1, 2, 3)), 1, axis=(1, 2, 3)))
    assert rel(U, refl) < 1e-5
    # requirement 6: Re psi even, Im psi odd (so Re U is even, Im U odd in x)
    mirror = np.roll(np.flip(U, axis=(1, 2, 3)), 1, axis=(1, 2, 3))
    scale = np.max(np.abs(U))
    assert np.max(np.abs(U.real - mirror.real)) < 1e-6 * scale
    assert np.max(np.abs(U.imag + mirror.imag)) < 1e-6 * scale
    assert np.max(np.abs(U.imag)) > 1e-3 * scale


@pytest.mark.parametrize("shape,level,L", [((20, 24, 16), 1, 16), ((256, 256, 256), 2, 24)],
                         ids=["20x24x16", "256cube_No162"])
def test_shift_covariance_gpu(torch, shape, level, L):
    """A circular shift of f shifts every score by the same amount (up to
    FP32 rounding: the DFT phases differ)."""
    from paper_1505_07690_amd import os3d
    n, p, gb = _bank(shape, level, L)
    f = torch.from_numpy(inputs.tubes(shape, 6, 1.5, 0.1, 0, 3)).cuda()
    fs = torch.roll(f, shifts=(3, -5, 7), dims=(0, 1, 2)).contiguous()
    U, _ = os3d.forward(f, gb)
    Us, _ = os3d.forward(fs, gb)
    for i0 in range(0, len(n), 27):  # orientation blocks bound the temporaries at 256^3
        a = torch.roll(U[i0:i0 + 27], shifts=(3, -5, 7), dims=(1, 2, 3))
        b = Us[i0:i0 + 27]
        err = (torch.linalg.norm((a - b).flatten()) / torch.linalg.norm(a.flatten())).item()
        assert err < 1e-5, i0
        del a, b


def test_gram_and_norm_identities_against_oracle_M(torch):
    """adjoint(forward(f)) = Re IDFT(M F) and sum_i ||U_i||^2 = (1/V) sum_k M |F|^2
    with M, F from the oracle."""
    from paper_1505_07690_amd import os3d
    shape = (16, 24, 20)
    n, p, gb = _bank(shape, 1, 16)
    ob = O.build_bank(shape, n, p)
    f = np.random.default_rng(4).standard_normal(shape).astype(np.float32)
    fg = torch.from_numpy(f).cuda()
    U, _ = os3d.forward(fg, gb)
    adj = os3d.adjoint(U, gb).cpu().numpy()
    F = O.dft3(f.astype(np.float64))
    assert rel(adj, np.real(O.idft3(ob["M"] * F))) < 1e-5
    lhs = torch.sum(torch.abs(U).double() ** 2).item()
    rhs = float(np.sum(ob["M"] * np.abs(F) ** 2) / np.prod(shape))
    assert abs(lhs - rhs) < 1e-5 * rhs


def test_norm_identity_headline(torch):
    """Eq. (5) in its M-weighted form at 256^3 x 162 (M from the GPU bank is
    checked against the oracle in the bank tests; here the identity ties the
    scores to it): sum_i ||U_i||^2 = (1/V) sum_k M |F|^2."""
    from paper_1505_07690_amd import os3d
    shape = (256, 256, 256)
    n, p, gb = _bank(shape, 2, 24)
    f = torch.from_numpy(inputs.tubes(shape, 8, (1.0, 3.0), 0.2, 0, 5)).cuda()
    U, _ = os3d.forward(f, gb)
    lhs = sum(torch.sum(torch.view_as_real(U[i]).double() ** 2).item() for i in range(len(n)))
    del U
    F = torch.fft.fftn(f.double())
    rhs = (torch.sum(gb.M().double() * torch.abs(F) ** 2) / f.numel()).item()
    assert abs(lhs - rhs) < 1e-5 * rhs
