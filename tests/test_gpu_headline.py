"""The headline workload, 256^3 x 162 orientations with L = 24 (the 256^3
crossing-tube volume: 40 tubes, sigma in U[1, 4], noise 0.3, seed 2),
against the FP64 oracle with nothing divided out (Sec. 2.1, Eqs. 7-9;
Sec. 3.1-3.2, Eqs. 10-19).

The oracle runs in this process, streamed so that it never holds the full
162-row bank:

* kappa over the whole normalisation band (1.1 M frequencies x 162
  orientations);
* M (Eq. 9) at about 2e5 sampled frequencies, a quarter of them within 0.1
  rho_N of the Nyquist radius;
* eight whole bank rows (every 16-column block of the contraction), each
  orientation's partner read through the reflected row;
* the scores of those eight stored orientations and of their antipodal
  partners, complex64 and 16-bit storage, with the 16-bit scales checked
  against the bound reading;
* the reconstruction (Eq. 8 with max(M, eps)) of the forward scores in each
  storage mode, compared in the frequency domain at the sampled frequencies:
  by Parseval the relative L2 error over uniformly sampled frequencies
  estimates the relative L2 error of the volume.

It prints one PRECISION line (JSON) with the relative L2 errors per storage
mode against the oracle.
"""
import json
import math

import numpy as np
import pytest

import oracle as O
from paper_1505_07690_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-5
BOUNDS = {"c64": TOL, "fp16": 5e-4, "bf16": 4e-3}


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


@pytest.fixture(scope="module")
def hl():
    import torch
    assert torch.cuda.is_available()
    from paper_1505_07690_amd import os3d
    c = inputs.CONFIGS["C"]
    shape = tuple(c["shape"])
    n = inputs.icosahedral_orientations(c["level"])
    p = O.WaveletParams(L=c["L"], s_theta=inputs.s_theta_for(len(n)))
    print(f"headline: building the bank {shape} x {len(n)}, L = {p.L}", flush=True)
    gb = os3d.Bank(shape, n, p)
    a = O.cake_coeffs(O.sh_coeffs_A(p))
    print("headline: oracle kappa over the band", flush=True)
    kappa = O.band_kappa_streamed(shape, n, a, p)
    vol = inputs.config_volume("C")
    print("headline: oracle DFT of the volume", flush=True)
    F = O.dft3(vol.astype(np.float64))
    d = np.linalg.norm(n[:, None] + n[None], axis=2)
    partner = np.argmin(d, axis=1)
    reps = [i for i in range(len(n)) if partner[i] > i]
    assert len(reps) == 81 and gb.n_unique == 81
    # sampled frequencies: uniform, plus the shell within 0.1 rho_N of Nyquist
    rng = np.random.default_rng(12)
    V = int(np.prod(shape))
    uni = np.unique(rng.integers(0, V, 150_000))
    wz, wy, wx, nyq = O.freq_at(shape, np.arange(V, dtype=np.int64)[::7])
    rho = np.sqrt(wz * wz + wy * wy + wx * wx)
    shell = np.arange(V, dtype=np.int64)[::7][(rho > 0.9 * np.pi) & ~nyq]
    near = rng.choice(shell, 50_000, replace=False)
    print("headline: oracle M at sampled frequencies", flush=True)
    M_uni = O.M_at(shape, uni, n, a, p, kappa)
    M_near = O.M_at(shape, near, n, a, p, kappa)
    return dict(torch=torch, os3d=os3d, shape=shape, n=n, p=p, gb=gb, a=a, kappa=kappa, vol=vol, F=F,
                partner=partner, reps=reps, uni=uni, near=near, M_uni=M_uni, M_near=M_near, report={})


def _scores(hl):
    """The forward scores of the volume in the three storage modes (computed
    once per module)."""
    if "Us" not in hl:
        f = hl["torch"].from_numpy(hl["vol"]).cuda()
        hl["Us"] = {"c64": hl["os3d"].forward(f, hl["gb"])}
        for fmt in ("bf16", "fp16"):
            hl["Us"][fmt] = hl["os3d"].forward(f, hl["gb"], dtype=fmt)
    return hl["Us"]


# stored rows in every 16-column block of the contraction (rows 16 j .. 16 j + 15)
ROWS = (0, 13, 29, 47, 48, 61, 72, 80)


def test_headline_kappa_and_M(hl):
    gb, kappa = hl["gb"], hl["kappa"]
    assert abs(gb.kappa - kappa) < TOL * kappa, (gb.kappa, kappa)
    M = hl["gb"].M().cpu().numpy().astype(np.float64).ravel()
    for idx, want in ((hl["uni"], hl["M_uni"]), (hl["near"], hl["M_near"])):
        got = M[idx]
        assert rel(got, want) < TOL
        assert np.max(np.abs(got - want)) < TOL * np.max(hl["M_uni"])
    hl["report"]["kappa_rel"] = abs(gb.kappa - kappa) / kappa
    hl["report"]["M_rel_l2_sampled"] = rel(M[hl["uni"]], hl["M_uni"])


def test_headline_bank_rows_scores_and_scales(hl):
    """Eight whole bank rows and the scores of their orientations and
    partners, complex64 and 16-bit, against the oracle; the 16-bit scales
    are the oracle's bound reading (the smallest power of two above
    (1/V) sum_k |psi_hat_i F|, times 2^-15 for fp16), exactly, except
    where that bound lies within 1e-5 of a power of two."""
    torch, os3d, gb, shape = hl["torch"], hl["os3d"], hl["gb"], hl["shape"]
    n, a, p, kappa, F, partner = hl["n"], hl["a"], hl["p"], hl["kappa"], hl["F"], hl["partner"]
    Us = _scores(hl)
    num = {m: 0.0 for m in Us}
    den = 0.0
    peak = {m: 0.0 for m in ("bf16", "fp16")}
    for r in ROWS:
        i = hl["reps"][r]
        j = int(partner[i])
        print(f"headline: row {r} (orientations {i}, {j})", flush=True)
        psi = O.bank_row(shape, n[i], a, p, kappa)
        assert rel(gb.psi(i).cpu().numpy(), psi) < TOL, r
        # the partner's row is the same row read at -k
        psi_j = np.roll(np.flip(psi, axis=(0, 1, 2)), 1, axis=(0, 1, 2))
        assert rel(gb.psi(j).cpu().numpy(), psi_j) < TOL, r
        Uo = O.idft3(psi * F)
        bound = O.score_scale_bound(F, psi)
        del psi, psi_j
        U, _ = Us["c64"]
        got = U[i].cpu().numpy()
        assert rel(got, Uo) < TOL, r
        assert torch.equal(U[j], torch.conj(U[i]).resolve_conj())
        num["c64"] += float(np.sum(np.abs(got - Uo) ** 2))
        den += float(np.sum(np.abs(Uo) ** 2))
        for fmt in ("bf16", "fp16"):
            Uq, sc = Us[fmt]
            s_gpu = float(sc[i].item())
            assert float(sc[j].item()) == s_gpu
            s_or = float(O.score_scales([bound], fmt)[0])
            e_gpu, e_or = math.log2(s_gpu), math.log2(s_or)
            assert e_gpu == round(e_gpu)
            frac = math.frexp(bound)[0]  # bound = frac 2^e, frac in [0.5, 1)
            near_pow2 = frac > 1 - 1e-5 or frac < 0.5 * (1 + 1e-5)
            assert e_gpu == e_or or (near_pow2 and abs(e_gpu - e_or) == 1), (fmt, r, s_gpu, s_or, bound)
            top = 2.0 ** 15 if fmt == "fp16" else 1.0
            uq = os3d.unpack16(Uq[i:i + 1], sc[i:i + 1], fmt)[0].cpu().numpy()
            num[fmt] += float(np.sum(np.abs(uq - Uo) ** 2))
            umax = max(np.abs(uq.real).max(), np.abs(uq.imag).max())
            peak[fmt] = max(peak[fmt], float(umax) / (s_gpu * top))
            assert umax / s_gpu < top
        del Uo
    errs = {m: math.sqrt(num[m] / den) for m in num}
    for m, e in errs.items():
        assert e < BOUNDS[m], (m, e)
    hl["report"]["U_rel_l2"] = errs
    hl["report"]["U_sampled_orientations"] = 2 * len(ROWS)
    hl["report"]["max_abs_U_over_scale_range"] = peak


def test_headline_reconstruction(hl):
    """The stabilised reconstruction (Eq. 8, M -> max(M, eps)) of the
    forward scores in each storage mode: the DFT of the GPU's volume at the
    sampled frequencies against F M / max(M, eps) from the oracle."""
    torch, os3d, gb = hl["torch"], hl["os3d"], hl["gb"]
    eps = hl["p"].eps
    F = hl["F"].ravel()
    idx = np.concatenate([hl["uni"], hl["near"]])
    M = np.concatenate([hl["M_uni"], hl["M_near"]])
    want = F[idx] * M / np.maximum(M, eps)
    nu = hl["uni"].size
    errs = {}
    for mode in ("c64", "bf16", "fp16"):
        U, sc = _scores(hl).pop(mode)
        kw = {} if mode == "c64" else dict(scales=sc, dtype=mode)
        rec = os3d.reconstruct(U, gb, **kw).cpu().numpy().astype(np.float64)
        del U, sc
        print(f"headline: oracle DFT of the {mode} reconstruction", flush=True)
        got = O.dft3(rec).ravel()[idx]
        e_uni = rel(got[:nu], want[:nu])
        e_near = rel(got[nu:], want[nu:])
        assert e_uni < BOUNDS[mode], (mode, e_uni)
        assert e_near < 10 * BOUNDS[mode], (mode, e_near)
        errs[mode] = e_uni
        hl["report"].setdefault("rec_rel_l2_near_nyquist", {})[mode] = e_near
    hl["report"]["rec_rel_l2"] = errs
    print("PRECISION " + json.dumps(hl["report"], default=float), flush=True)


def test_headline_adjoint_of_one_pair_against_oracle(hl):
    """W* of a general complex score supported on one antipodal pair (Eq. 8
    without the division by M), over the whole grid, against the oracle
    with its own kappa."""
    torch, os3d, gb, shape = hl["torch"], hl["os3d"], hl["gb"], hl["shape"]
    n, a, p, kappa = hl["n"], hl["a"], hl["p"], hl["kappa"]
    i = hl["reps"][40]
    j = int(hl["partner"][i])
    rng = np.random.default_rng(9)
    Ui = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)
    Uj = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)
    hl.pop("Us", None)  # free the scores of the other tests
    Ug = torch.zeros((len(n),) + shape, dtype=torch.complex64, device="cuda")
    Ug[i] = torch.from_numpy(Ui).cuda()
    Ug[j] = torch.from_numpy(Uj).cuda()
    adj = os3d.adjoint(Ug, gb).cpu().numpy()
    del Ug
    psi = O.bank_row(shape, n[i], a, p, kappa)
    X = psi * O.dft3(Ui.astype(np.complex128))
    psi = np.roll(np.flip(psi, axis=(0, 1, 2)), 1, axis=(0, 1, 2))  # the partner's row: the same row at -k
    X += psi * O.dft3(Uj.astype(np.complex128))
    assert rel(adj, np.real(O.idft3(X))) < TOL
