"""The Python binding checks every tensor (device, shape, storage type,
contiguity, batch) before it hands a pointer to the C ABI, so a wrong
argument raises in Python instead of reaching the kernels.  CPU only: a
stand-in bank object carries the geometry, and every case must raise before
any library call."""
import types

import pytest
import torch

from paper_1505_07690_amd import os3d


def _bank(device="cpu"):
    def no_workspace():
        raise AssertionError("validation must fail before the workspace is touched")
    return types.SimpleNamespace(shape=(4, 6, 8), n_orients=12, device=torch.device(device), handle=None,
                                 workspace=no_workspace)


def test_volume_checks():
    b = _bank()
    with pytest.raises(ValueError, match="shape"):
        os3d.forward(torch.zeros(4, 6, 9), b)
    with pytest.raises(ValueError, match="float32"):
        os3d.forward(torch.zeros(4, 6, 8, dtype=torch.float64), b)
    with pytest.raises(ValueError, match="contiguous"):
        os3d.forward(torch.zeros(8, 6, 4).permute(2, 1, 0), b)
    with pytest.raises(ValueError, match="empty"):
        os3d.forward(torch.zeros(0, 4, 6, 8), b)
    with pytest.raises(ValueError, match="expected f"):
        os3d.process(torch.zeros(4, 6), b)
    with pytest.raises(ValueError, match="must be on"):
        os3d.forward(torch.zeros(4, 6, 8), _bank("meta"))


def test_output_and_scale_checks():
    b = _bank()
    f = torch.zeros(2, 4, 6, 8)
    with pytest.raises(ValueError, match="out"):
        os3d.forward(f, b, out=torch.zeros((2, 11, 4, 6, 8), dtype=torch.complex64))
    with pytest.raises(ValueError, match="out"):
        os3d.forward(f, b, dtype="bf16", out=torch.zeros((2, 12, 4, 6, 8), dtype=torch.complex64))
    with pytest.raises(ValueError, match="scales"):
        os3d.forward(f, b, dtype="fp16", out=torch.zeros((2, 12, 4, 6, 8), dtype=torch.int32),
                     scales=torch.zeros(2, 11))
    with pytest.raises(ValueError, match="out"):
        os3d.process(f, b, out=torch.zeros(1, 4, 6, 8))


def test_score_checks():
    b = _bank()
    U = torch.zeros((12, 4, 6, 8), dtype=torch.complex64)
    with pytest.raises(ValueError, match="shape"):
        os3d.reconstruct(torch.zeros((11, 4, 6, 8), dtype=torch.complex64), b)
    with pytest.raises(ValueError, match="complex64"):
        os3d.adjoint(U.real.contiguous(), b)
    with pytest.raises(ValueError, match="int32"):
        os3d.reconstruct(U, b, dtype="bf16", scales=torch.zeros(12))
    with pytest.raises(ValueError, match="scales"):
        os3d.reconstruct(torch.zeros((12, 4, 6, 8), dtype=torch.int32), b, dtype="fp16")
    with pytest.raises(ValueError, match="contiguous"):
        os3d.reconstruct_approx(torch.zeros((8, 6, 4, 12), dtype=torch.complex64).permute(3, 2, 1, 0), b)
    with pytest.raises(ValueError, match="out"):
        os3d.reconstruct(U, b, out=torch.zeros(4, 6, 7))


def test_bank_must_live_on_a_gpu():
    with pytest.raises(ValueError, match="GPU"):
        os3d.Bank((4, 6, 8), [[0.0, 0.0, 1.0]], os3d.make_params(L=4), device="cpu")
