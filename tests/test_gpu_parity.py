"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle, on
seeded inputs at oracle-sized shapes: the bank and M (Eqs. 9-19), the
forward transform (Eq. 7), its adjoint and the stabilised reconstruction
(Eq. 8 with max(M, eps)).  FP32 paths: relative L2 error <= 1e-5."""
import numpy as np
import pytest

import oracle as O
from paper_1505_07690_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-5


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1505_07690_amd import os3d
    os3d.lib()  # the HIP library must be there: no fallback
    return torch


def _case(shape, orients, params, vol):
    from paper_1505_07690_amd import os3d
    import torch
    ob = O.build_bank(shape, orients, params)
    gb = os3d.Bank(shape, orients, params)
    f = torch.from_numpy(np.ascontiguousarray(vol, dtype=np.float32)).cuda()
    return ob, gb, f


def _oracle_params(L, n_or, variant="cake", gamma=0.8):
    return O.WaveletParams(L=L, s_theta=inputs.s_theta_for(n_or), variant=variant, gamma=gamma)


CASES = {
    # config A: 32^3 crossing tubes, 12 icosahedron orientations, L = 8
    "A32": lambda: ((32, 32, 32), inputs.icosahedral_orientations(0), _oracle_params(8, 12),
                    inputs.config_volume("A")),
    # non-cubic, ragged tile counts, 42 orientations, L = 16
    "r12x10x18": lambda: ((12, 10, 18), inputs.icosahedral_orientations(1), _oracle_params(16, 42),
                          inputs.tubes((12, 10, 18), 2, 1.2, 0.1, 0, 5)),
    # odd dims (no Nyquist plane on z, y), radix 3 and 5
    "odd15x9x10": lambda: ((15, 9, 10), inputs.icosahedral_orientations(0), _oracle_params(8, 12),
                           inputs.tubes((15, 9, 10), 2, 1.0, 0.2, 0, 6)),
    # a set without antipodes (no pairing) and the plate-detector variant
    "unpaired_plate": lambda: ((16, 12, 20), _random_orients(7, 3), _oracle_params(6, 7, "plate"),
                               inputs.tubes((16, 12, 20), 3, 1.5, 0.1, 0, 7)),
    # power-of-two axes of the register-resident kernels (64 on every axis)
    "fast64": lambda: ((64, 64, 64), inputs.icosahedral_orientations(0), _oracle_params(8, 12),
                       inputs.tubes((64, 64, 64), 3, 1.5, 0.1, 0, 9)),
    # 128 / 64 / 256 on z / y / x: each fast line length on a different axis, ragged tile count on none
    "fast128x64x256": lambda: ((128, 64, 256), inputs.icosahedral_orientations(0), _oracle_params(4, 12),
                               inputs.tubes((128, 64, 256), 3, 1.5, 0.1, 0, 10)),
    # 256 on z, 128 on y, tiny x: a y-tile wraps across z planes
    "fast256x128x4": lambda: ((256, 128, 4), inputs.icosahedral_orientations(0), _oracle_params(4, 12),
                              inputs.tubes((256, 128, 4), 2, 1.0, 0.1, 0, 11)),
    # quadrature coefficients, B-spline order 3 and a narrow window (bank variants)
    "quad_k3": lambda: ((12, 16, 10), inputs.icosahedral_orientations(1),
                        O.WaveletParams(L=12, s_theta=0.5, k=3, coeffs="quadrature"),
                        inputs.tubes((12, 16, 10), 2, 1.2, 0.1, 0, 12)),
    # the smallest grid with a normalisation band: radices 2, 3, 4, mostly Nyquist planes
    "tiny234": lambda: ((2, 3, 4), inputs.icosahedral_orientations(0), _oracle_params(4, 12),
                        inputs.tubes((2, 3, 4), 1, 1.0, 0.1, 0, 13)),
    # the longest supported axis (4096 = 2^12) through the LDS Stockham kernel, odd sizes beside it
    "axis4096": lambda: ((2, 3, 4096), inputs.icosahedral_orientations(0), _oracle_params(4, 12),
                         inputs.tubes((2, 3, 4096), 2, 1.0, 0.1, 0, 14)),
    # whole-plane path: 128 x 128 planes over a z axis of 20 (radix 4 x 5 in the z pass)
    "plane128": lambda: ((20, 128, 128), inputs.icosahedral_orientations(0), _oracle_params(4, 12),
                         inputs.tubes((20, 128, 128), 3, 1.5, 0.1, 0, 15)),
    # platonic sets: the tetrahedron has no antipodes (pair path off), the dodecahedron has
    "tetra": lambda: ((12, 10, 16), inputs.platonic_orientations("tetrahedron"), _oracle_params(6, 4),
                      inputs.tubes((12, 10, 16), 2, 1.2, 0.1, 0, 18)),
    "dodeca": lambda: ((16, 12, 10), inputs.platonic_orientations("dodecahedron"), _oracle_params(10, 20),
                       inputs.tubes((16, 12, 10), 2, 1.2, 0.1, 0, 19)),
    # degenerate banks: L = 0 (every profile isotropic) and a single orientation
    "L0": lambda: ((10, 12, 8), inputs.icosahedral_orientations(0), _oracle_params(0, 12),
                   inputs.tubes((10, 12, 8), 2, 1.2, 0.1, 0, 20)),
    "single": lambda: ((12, 8, 10), np.array([[0.0, 0.0, 1.0]]), _oracle_params(8, 12),
                       inputs.tubes((12, 8, 10), 2, 1.2, 0.1, 0, 21)),
    # the bank synthesis takes the stored rows in 16-column blocks, up to six
    # per sweep of its recursion, the sweeps evenly filled: 81 rows of the
    # 162-orientation set (six blocks, the last one partly filled), 60, 70
    # and 40 unpaired rows (four, five and three blocks), 110 unpaired rows
    # (two sweeps of four blocks, the second one partly filled)
    "ico162": lambda: ((10, 12, 8), inputs.icosahedral_orientations(2), _oracle_params(12, 162),
                       inputs.tubes((10, 12, 8), 2, 1.2, 0.1, 0, 22)),
    "rand60": lambda: ((8, 10, 12), _random_orients(60, 23), _oracle_params(8, 60),
                       inputs.tubes((8, 10, 12), 2, 1.2, 0.1, 0, 24)),
    "rand70": lambda: ((9, 8, 10), _random_orients(70, 29), _oracle_params(10, 70),
                       inputs.tubes((9, 8, 10), 2, 1.2, 0.1, 0, 30)),
    "rand110": lambda: ((8, 10, 12), _random_orients(110, 31), _oracle_params(6, 110),
                        inputs.tubes((8, 10, 12), 2, 1.2, 0.1, 0, 32)),
    "rand40": lambda: ((10, 8, 12), _random_orients(40, 25), _oracle_params(10, 40),
                       inputs.tubes((10, 8, 12), 2, 1.2, 0.1, 0, 26)),
    # the two non-power-of-two shapes of the serving workload (12 orientations
    # to bound the oracle's time): radix 3 and 5 on the three-pass path, and
    # sets without antipodes on the whole-plane path (every pair slot unpaired)
    "plane128_tetra": lambda: ((12, 128, 128), inputs.platonic_orientations("tetrahedron"), _oracle_params(6, 4),
                               inputs.tubes((12, 128, 128), 3, 1.5, 0.1, 0, 51)),
    "plane64_rand5": lambda: ((16, 64, 64), _random_orients(5, 53), _oracle_params(8, 5),
                              inputs.tubes((16, 64, 64), 3, 1.5, 0.1, 0, 52)),
    # a z axis of 160 under 128 x 128 planes on the plane path
    "serve96x80x64": lambda: ((96, 80, 64), inputs.icosahedral_orientations(0), _oracle_params(24, 12),
                              inputs.tubes((96, 80, 64), 12, (1.0, 3.0), 0.2, 0, 27)),
    "serve160x128x128": lambda: ((160, 128, 128), inputs.icosahedral_orientations(0), _oracle_params(16, 12),
                                 inputs.tubes((160, 128, 128), 12, (1.0, 3.0), 0.2, 0, 28)),
    # the ends of the synthesis' K order: L = 1 and L = 3 (a few words, the
    # chains one or two orders long) and L = 62, the largest order the
    # synthesis takes (|Y_lm| 2^13 up to 25.8k of fp16's 65504, the recursion
    # to m = 62)
    "L1": lambda: ((8, 6, 10), inputs.icosahedral_orientations(0), _oracle_params(1, 12),
                   inputs.tubes((8, 6, 10), 2, 1.2, 0.1, 0, 34)),
    "L3": lambda: ((10, 8, 6), inputs.icosahedral_orientations(1), _oracle_params(3, 42),
                   inputs.tubes((10, 8, 6), 2, 1.2, 0.1, 0, 35)),
    "L62": lambda: ((6, 8, 10), inputs.icosahedral_orientations(0), _oracle_params(62, 12),
                    inputs.tubes((6, 8, 10), 2, 1.2, 0.1, 0, 36)),
    # small N with radix-2 only and a long axis
    "long4x6x64": lambda: ((4, 6, 64), inputs.icosahedral_orientations(0), _oracle_params(4, 12),
                           inputs.tubes((4, 6, 64), 2, 1.0, 0.1, 0, 8)),
}


def _random_orients(n, seed):
    v = np.random.default_rng(seed).standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request, torch_dev):
    shape, orients, params, vol = CASES[request.param]()
    ob, gb, f = _case(shape, orients, params, vol)
    return dict(name=request.param, shape=shape, orients=orients, params=params, vol=vol, ob=ob, gb=gb, f=f)


def test_bank_and_M_parity(case):
    ob, gb = case["ob"], case["gb"]
    psi = np.stack([gb.psi(i).cpu().numpy() for i in range(len(case["orients"]))])
    assert rel(psi, ob["psi_hat"]) < TOL
    assert rel(gb.M().cpu().numpy(), ob["M"]) < TOL
    assert abs(gb.kappa - ob["kappa"]) < 1e-6 * ob["kappa"]
    unpaired = ("unpaired_plate", "tetra", "single", "rand60", "rand40", "rand70", "rand110", "plane128_tetra",
                "plane64_rand5")
    assert gb.paired == (case["name"] not in unpaired)


def test_forward_parity(case):
    from paper_1505_07690_amd import os3d
    U, _ = os3d.forward(case["f"], case["gb"])
    Uo = O.forward(case["vol"].astype(np.float64), case["ob"])
    assert rel(U.cpu().numpy(), Uo) < TOL


def test_reconstruct_and_adjoint_parity(case):
    from paper_1505_07690_amd import os3d
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    No = len(case["orients"])
    # a general complex score (not in the range of W)
    Un = (rng.standard_normal((No,) + case["shape"]) + 1j * rng.standard_normal((No,) + case["shape"]))
    Ug = torch.from_numpy(Un.astype(np.complex64)).cuda()
    rec = os3d.reconstruct(Ug, case["gb"]).cpu().numpy()
    adj = os3d.adjoint(Ug, case["gb"]).cpu().numpy()
    Un32 = Un.astype(np.complex64).astype(np.complex128)
    assert rel(rec, O.reconstruct(Un32, case["ob"])) < TOL
    assert rel(adj, O.adjoint(Un32, case["ob"])) < TOL


def test_roundtrip_reconstruction(case):
    """reconstruct(forward(f)) on the GPU equals the oracle's (Eq. 8)."""
    from paper_1505_07690_amd import os3d
    U, _ = os3d.forward(case["f"], case["gb"])
    rec = os3d.reconstruct(U, case["gb"]).cpu().numpy()
    ref = O.reconstruct(O.forward(case["vol"].astype(np.float64), case["ob"]), case["ob"])
    assert rel(rec, ref) < TOL


def test_bruteforce_correlation_8cube(torch_dev):
    """Eq. (7) literally (direct circular correlation with conj(psi)) on 8^3."""
    from paper_1505_07690_amd import os3d
    shape = (8, 8, 8)
    n = inputs.icosahedral_orientations(0)
    p = _oracle_params(8, 12)
    vol = np.random.default_rng(0).standard_normal(shape).astype(np.float32)
    ob, gb, f = _case(shape, n, p, vol)
    U, _ = os3d.forward(f, gb)
    assert rel(U.cpu().numpy(), O.forward_bruteforce(vol.astype(np.float64), ob)) < TOL


def test_exact_reconstruction_bandlimited(torch_dev):
    from paper_1505_07690_amd import os3d
    shape = (32, 32, 32)
    n = inputs.icosahedral_orientations(1)
    p = _oracle_params(16, 42)
    vol = inputs.bandlimited(shape, 0.75, seed=4)
    gb = os3d.Bank(shape, n, p)
    f = torch_dev.from_numpy(vol).cuda()
    U, _ = os3d.forward(f, gb)
    rec = os3d.reconstruct(U, gb).cpu().numpy()
    assert rel(rec, vol) < TOL


def test_batch_and_determinism(torch_dev):
    from paper_1505_07690_amd import os3d
    shape = (16, 16, 16)
    n = inputs.icosahedral_orientations(1)
    p = _oracle_params(16, 42)
    gb = os3d.Bank(shape, n, p)
    vols = np.stack([inputs.tubes(shape, 2, 1.2, 0.1, 0, s) for s in range(3)])
    fb = torch_dev.from_numpy(vols).cuda()
    U, _ = os3d.forward(fb, gb)
    U2, _ = os3d.forward(fb, gb)
    assert torch_dev.equal(U, U2)
    for b in range(3):
        Ub, _ = os3d.forward(fb[b].contiguous(), gb)
        assert torch_dev.equal(U[b], Ub)
    rec = os3d.reconstruct(U, gb)
    for b in range(3):
        assert torch_dev.equal(rec[b], os3d.reconstruct(U[b].contiguous(), gb))
    ob = O.build_bank(shape, n, p)
    for b in range(3):
        assert rel(U[b].cpu().numpy(), O.forward(vols[b].astype(np.float64), ob)) < TOL


def test_antipodal_pairs_are_conjugate(torch_dev):
    from paper_1505_07690_amd import os3d
    shape = (16, 16, 16)
    n = inputs.icosahedral_orientations(0)
    gb = os3d.Bank(shape, n, _oracle_params(8, 12))
    f = torch_dev.from_numpy(inputs.tubes(shape, 2, 1.2, 0.1, 0, 2)).cuda()
    U, _ = os3d.forward(f, gb)
    d = np.linalg.norm(n[:, None] + n[None], axis=2)
    j = np.argmin(d, axis=1)
    assert torch_dev.equal(U[j], torch_dev.conj(U).resolve_conj())


@pytest.mark.parametrize("fmt,bound,shape", [("bf16", 4e-3, (32, 32, 32)), ("fp16", 5e-4, (32, 32, 32)),
                                             ("bf16", 4e-3, (24, 64, 64)), ("fp16", 5e-4, (24, 64, 64))],
                         ids=["bf16_three_pass", "fp16_three_pass", "bf16_plane", "fp16_plane"])
def test_reduced_precision_storage(torch_dev, fmt, bound, shape):
    """16-bit score storage with per-orientation power-of-two scales: error of
    U and of the reconstruction against the FP64 oracle (three-pass path and
    z-line + whole-plane path)."""
    from paper_1505_07690_amd import os3d
    n = inputs.icosahedral_orientations(1)
    p = _oracle_params(16, 42)
    vol = inputs.config_volume("A") if shape == (32, 32, 32) else inputs.tubes(shape, 3, 1.5, 0.1, 0, 16)
    ob, gb, f = _case(shape, n, p, vol)
    Uq, sc = os3d.forward(f, gb, dtype=fmt)
    s = sc.cpu().numpy()
    assert np.all(np.log2(s) == np.round(np.log2(s)))
    # the scales are the bound reading: the smallest power of two above
    # (1/V) sum_k |psi_hat_i F| (times 2^-15 for fp16), up to one step where
    # the bound lies within 1e-5 of a power of two
    F = O.dft3(vol.astype(np.float64))
    bounds = np.array([O.score_scale_bound(F, ob["psi_hat"][i]) for i in range(len(n))])
    s_or = O.score_scales(bounds, fmt)
    frac = np.array([np.frexp(b)[0] for b in bounds])
    near = (frac > 1 - 1e-5) | (frac < 0.5 * (1 + 1e-5))
    d_e = np.log2(s) - np.log2(s_or)
    assert np.all((d_e == 0) | (near & (np.abs(d_e) == 1))), (s, s_or)
    U = os3d.unpack16(Uq, sc, fmt).cpu().numpy()
    Uo = O.forward(vol.astype(np.float64), ob)
    assert rel(U, Uo) < bound
    rec = os3d.reconstruct(Uq, gb, scales=sc, dtype=fmt).cpu().numpy()
    assert rel(rec, O.reconstruct(Uo, ob)) < bound
    # the antipodal partner is stored as the exact conjugate code
    d = np.linalg.norm(n[:, None] + n[None], axis=2)
    j = np.argmin(d, axis=1)
    Uc = os3d.unpack16(Uq, sc, fmt)
    assert torch_dev.equal(Uc[j], torch_dev.conj(Uc).resolve_conj())


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
@pytest.mark.parametrize("shape", [(12, 128, 128), (16, 64, 64)], ids=["plane128", "plane64"])
def test_reduced_precision_unpaired_plane(torch_dev, fmt, shape):
    """16-bit storage on the whole-plane path with a set without antipodes
    (the tetrahedron): the scores within the storage bound of the FP64
    oracle's, and the reconstruction against the oracle's reconstruction of
    the same dequantised scores — the plane path keeps complex64
    intermediates, so within the FP32 tolerance.  (With 4 orientations the
    division by max(M, eps) amplifies the storage error itself, so the
    reconstruction is not compared with the oracle's from exact scores.)"""
    from paper_1505_07690_amd import os3d
    n = inputs.platonic_orientations("tetrahedron")
    ob, gb, f = _case(shape, n, _oracle_params(6, 4), inputs.tubes(shape, 3, 1.5, 0.1, 0, 54))
    assert not gb.paired
    Uq, sc = os3d.forward(f, gb, dtype=fmt)
    Ud = os3d.unpack16(Uq, sc, fmt).cpu().numpy()
    Uo = O.forward(f.cpu().numpy().astype(np.float64), ob)
    assert rel(Ud, Uo) < {"bf16": 4e-3, "fp16": 5e-4}[fmt]
    rec = os3d.reconstruct(Uq, gb, scales=sc, dtype=fmt).cpu().numpy()
    assert rel(rec, O.reconstruct(Ud.astype(np.complex128), ob)) < TOL


def test_approximate_reconstruction_parity(case):
    """Eq. (6) on the GPU (one pass over the scores) against the oracle, for
    a general complex score and for 16-bit storage."""
    from paper_1505_07690_amd import os3d
    import torch
    rng = np.random.default_rng(2)
    No = len(case["orients"])
    Un = (rng.standard_normal((No,) + case["shape"]) + 1j * rng.standard_normal((No,) + case["shape"]))
    Un32 = Un.astype(np.complex64)
    got = os3d.reconstruct_approx(torch.from_numpy(Un32).cuda(), case["gb"]).cpu().numpy()
    assert abs(case["gb"].approx_norm - O.approx_norm(case["ob"])) < 1e-6 * abs(O.approx_norm(case["ob"]))
    assert rel(got, O.reconstruct_approx(Un32.astype(np.complex128), case["ob"])) < TOL
    want = O.reconstruct_approx(O.forward(case["vol"].astype(np.float64), case["ob"]), case["ob"])
    for fmt, bound in (("fp16", 5e-4), ("bf16", 4e-3)):
        Uq, sc = os3d.forward(case["f"], case["gb"], dtype=fmt)
        got16 = os3d.reconstruct_approx(Uq, case["gb"], scales=sc, dtype=fmt).cpu().numpy()
        assert rel(got16, want) < bound, fmt
    # a score tensor that starts off the 16-byte grid takes the one-voxel loads
    # (as do volumes below 2^23 voxels; the full-size tests cover the other path)
    Ub = torch.empty(Un32.size + 2, dtype=torch.complex64, device="cuda")
    Uo = Ub[1:1 + Un32.size].view(Un32.shape)
    Uo.copy_(torch.from_numpy(Un32).cuda())
    got_off = os3d.reconstruct_approx(Uo, case["gb"]).cpu().numpy()
    assert rel(got_off, O.reconstruct_approx(Un32.astype(np.complex128), case["ob"])) < TOL


@pytest.mark.parametrize("phi,power", [("identity", 1.0), ("soft_threshold", 1.5)])
def test_process_parity(case, phi, power):
    """Eq. (23), W^+ Phi(W f), fused on the GPU (Phi applied in the forward
    transform's last pass) against the oracle."""
    from paper_1505_07690_amd import os3d
    got = os3d.process(case["f"], case["gb"], phi, power).cpu().numpy()
    want = O.process(case["vol"].astype(np.float64), case["ob"], phi, power)
    assert rel(got, want) < TOL


@pytest.mark.parametrize("power", [1.0, 0.5])
@pytest.mark.parametrize("shape", [(16, 16, 16), (12, 64, 64)], ids=["three_pass", "plane"])
def test_process_soft_threshold_of_tiny_scores(torch_dev, shape, power):
    """The soft threshold of Fig. 7 on a volume scaled by 1e-20: |U|^2 is
    below the smallest normal float there, and the result must still match
    the oracle (no NaN from the logarithm of a flushed square)."""
    from paper_1505_07690_amd import os3d
    n = inputs.icosahedral_orientations(0)
    p = _oracle_params(8, 12)
    vol = (inputs.tubes(shape, 2, 1.2, 0.1, 0, 29).astype(np.float64) * 1e-20).astype(np.float32)
    ob, gb, f = _case(shape, n, p, vol)
    got = os3d.process(f, gb, "soft_threshold", power).cpu().numpy()
    assert np.all(np.isfinite(got))
    assert rel(got, O.process(vol.astype(np.float64), ob, "soft_threshold", power)) < TOL


def test_projection_parity(case):
    """The projection W W^+ onto the orientation scores (Corollary of
    Appendix A), composed from the reconstruction and the forward transform,
    and its square, against the oracle with the same eps."""
    from paper_1505_07690_amd import os3d
    import torch
    if np.prod(case["shape"]) > 1 << 20:
        pytest.skip("four oracle transforms of every orientation take minutes at this size")
    rng = np.random.default_rng(3)
    No = len(case["orients"])
    Un = (rng.standard_normal((No,) + case["shape"]) + 1j * rng.standard_normal((No,) + case["shape"]))
    Un = Un.astype(np.complex64)
    P1, _ = os3d.forward(os3d.reconstruct(torch.from_numpy(Un).cuda(), case["gb"]), case["gb"])
    P2, _ = os3d.forward(os3d.reconstruct(P1, case["gb"]), case["gb"])
    ob = case["ob"]
    W1 = O.forward(O.reconstruct(Un.astype(np.complex128), ob), ob)
    W2 = O.forward(O.reconstruct(W1, ob), ob)
    assert rel(P1.cpu().numpy(), W1) < TOL
    assert rel(P2.cpu().numpy(), W2) < TOL


def test_three_pass_path_on_plane_shapes(torch_dev, monkeypatch):
    """Shapes with 64^2 or 128^2 planes take the z-line + whole-plane path;
    the three-pass path (forced for this bank) gives the same transform."""
    from paper_1505_07690_amd import os3d
    shape = (16, 64, 64)
    n = inputs.icosahedral_orientations(0)
    p = _oracle_params(8, 12)
    vol = inputs.tubes(shape, 3, 1.5, 0.1, 0, 17)
    ob = O.build_bank(shape, n, p)
    f = torch_dev.from_numpy(vol).cuda()
    monkeypatch.setenv("OS3D_THREE_PASS", "1")
    g3 = os3d.Bank(shape, n, p)
    monkeypatch.delenv("OS3D_THREE_PASS")
    g2 = os3d.Bank(shape, n, p)
    Uo = O.forward(vol.astype(np.float64), ob)
    ro = O.reconstruct(Uo, ob)
    for gb in (g3, g2):
        U, _ = os3d.forward(f, gb)
        assert rel(U.cpu().numpy(), Uo) < TOL
        assert rel(os3d.reconstruct(U, gb).cpu().numpy(), ro) < TOL


def _smooth235(m):
    for q in (2, 3, 5):
        while m % q == 0:
            m //= q
    return m == 1


def _sweep_case(seed):
    """A seeded draw outside the hand-picked cases: each axis one of the
    supported lengths (prime factors 2, 3, 5) from 2 to 48, odd or even, an
    orientation set with or without antipodes, L from 0 to 12, bank variant
    cake or plate."""
    rng = np.random.default_rng(1000 + seed)
    lengths = [m for m in range(2, 49) if _smooth235(m)]
    shape = tuple(int(lengths[i]) for i in rng.integers(0, len(lengths), 3))
    if max(shape) < 4:  # the normalisation band needs one axis of 4 or more
        shape = (shape[0], shape[1], 4)
    kind = int(rng.integers(4))
    if kind == 0:
        n = inputs.icosahedral_orientations(0)
    elif kind == 1:
        n = inputs.platonic_orientations("octahedron")
    elif kind == 2:
        n = inputs.platonic_orientations("tetrahedron")
    else:
        n = _random_orients(int(rng.integers(1, 21)), 2000 + seed)
    L = int(rng.integers(0, 13))
    variant = "plate" if rng.random() < 0.25 else "cake"
    return shape, n, _oracle_params(L, len(n), variant)


@pytest.mark.parametrize("seed", range(24))
def test_seeded_shape_sweep(torch_dev, seed):
    """Bank, M, forward, reconstruction of a general complex score,
    processing via scores and the approximate reconstruction against the
    oracle for a seeded draw of grid, orientation set, L and variant; every
    third draw also runs a batch of two volumes, whose elements must equal
    the volumes run alone; then 16-bit storage (bf16 for even seeds, fp16 for odd): the
    scores within the storage bound, their reconstruction against the
    oracle's reconstruction of the same dequantised scores (complex64
    intermediates on these paths: the FP32 tolerance)."""
    from paper_1505_07690_amd import os3d
    shape, n, p = _sweep_case(seed)
    vol = inputs.tubes(shape, 2, 1.2, 0.1, 0, 3000 + seed)
    ob, gb, f = _case(shape, n, p, vol)
    psi = np.stack([gb.psi(i).cpu().numpy() for i in range(len(n))])
    assert rel(psi, ob["psi_hat"]) < TOL, (shape, len(n), p.L)
    assert rel(gb.M().cpu().numpy(), ob["M"]) < TOL
    U, _ = os3d.forward(f, gb)
    assert rel(U.cpu().numpy(), O.forward(vol.astype(np.float64), ob)) < TOL, (shape, len(n), p.L)
    rng = np.random.default_rng(seed)
    Un = (rng.standard_normal((len(n),) + shape) + 1j * rng.standard_normal((len(n),) + shape)).astype(np.complex64)
    rec = os3d.reconstruct(torch_dev.from_numpy(Un).cuda(), gb).cpu().numpy()
    assert rel(rec, O.reconstruct(Un.astype(np.complex128), ob)) < TOL, (shape, len(n), p.L)
    Uo = O.forward(vol.astype(np.float64), ob)
    # processing via scores (Eq. 23, soft threshold) and the approximate
    # reconstruction (Eq. 6)
    gp = os3d.process(f, gb, "soft_threshold", 1.5).cpu().numpy()
    assert rel(gp, O.reconstruct(O.soft_threshold(Uo, 1.5), ob)) < TOL, (shape, len(n), p.L)
    ga = os3d.reconstruct_approx(torch_dev.from_numpy(Un).cuda(), gb).cpu().numpy()
    assert rel(ga, O.reconstruct_approx(Un.astype(np.complex128), ob)) < TOL, (shape, len(n), p.L)
    fmt = "bf16" if seed % 2 == 0 else "fp16"
    Uq, sc = os3d.forward(f, gb, dtype=fmt)
    Ud = os3d.unpack16(Uq, sc, fmt).cpu().numpy()
    assert rel(Ud, Uo) < {"bf16": 4e-3, "fp16": 5e-4}[fmt], (shape, fmt)
    rq = os3d.reconstruct(Uq, gb, scales=sc, dtype=fmt).cpu().numpy()
    assert rel(rq, O.reconstruct(Ud.astype(np.complex128), ob)) < TOL, (shape, fmt)
    if seed % 3 == 0:
        # a batch of two volumes: each element equals its volume run alone
        g = torch_dev.from_numpy(inputs.tubes(shape, 2, 1.2, 0.1, 0, 4000 + seed)).cuda()
        for dt in ("c64", fmt):
            Ub, sb = os3d.forward(torch_dev.stack([f, g]), gb, dtype=dt)
            U1, s1 = os3d.forward(f, gb, dtype=dt)
            U2, s2 = os3d.forward(g, gb, dtype=dt)
            assert torch_dev.equal(Ub[0], U1) and torch_dev.equal(Ub[1], U2), (shape, dt)
            kw = {} if dt == "c64" else dict(dtype=dt)
            rb = os3d.reconstruct(Ub, gb, scales=sb, **kw)
            assert torch_dev.equal(rb[0], os3d.reconstruct(U1, gb, scales=s1, **kw)), (shape, dt)
            assert torch_dev.equal(rb[1], os3d.reconstruct(U2, gb, scales=s2, **kw)), (shape, dt)


@pytest.mark.parametrize("seed", range(8))
def test_seeded_plane_sweep(torch_dev, seed):
    """The whole-plane path (64^2 or 128^2 planes) for seeded draws of the z
    length, orientation set and L: bank, forward and reconstruction of a
    general complex score against the oracle, and 16-bit storage as in the
    grid sweep."""
    from paper_1505_07690_amd import os3d
    rng = np.random.default_rng(5000 + seed)
    lengths = [m for m in range(2, 49) if _smooth235(m)]
    npl = (64, 128)[int(rng.integers(2))]
    shape = (int(lengths[int(rng.integers(len(lengths)))]), npl, npl)
    n = (inputs.icosahedral_orientations(0) if rng.random() < 0.5
         else _random_orients(int(rng.integers(1, 9)), 6000 + seed))
    p = _oracle_params(int(rng.integers(0, 13)), len(n))
    vol = inputs.tubes(shape, 2, 1.5, 0.1, 0, 7000 + seed)
    ob, gb, f = _case(shape, n, p, vol)
    assert rel(np.stack([gb.psi(i).cpu().numpy() for i in range(len(n))]), ob["psi_hat"]) < TOL
    Uo = O.forward(vol.astype(np.float64), ob)
    U, _ = os3d.forward(f, gb)
    assert rel(U.cpu().numpy(), Uo) < TOL, (shape, len(n), p.L)
    del U
    Un = (rng.standard_normal((len(n),) + shape) + 1j * rng.standard_normal((len(n),) + shape)).astype(np.complex64)
    rec = os3d.reconstruct(torch_dev.from_numpy(Un).cuda(), gb).cpu().numpy()
    assert rel(rec, O.reconstruct(Un.astype(np.complex128), ob)) < TOL, (shape, len(n), p.L)
    fmt = "bf16" if seed % 2 == 0 else "fp16"
    Uq, sc = os3d.forward(f, gb, dtype=fmt)
    Ud = os3d.unpack16(Uq, sc, fmt).cpu().numpy()
    assert rel(Ud, Uo) < {"bf16": 4e-3, "fp16": 5e-4}[fmt], (shape, fmt)
    rq = os3d.reconstruct(Uq, gb, scales=sc, dtype=fmt).cpu().numpy()
    assert rel(rq, O.reconstruct(Ud.astype(np.complex128), ob)) < TOL, (shape, fmt)
