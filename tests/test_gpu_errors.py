"""Argument errors of the compute calls with a real bank: every bad call
returns its status code before any work is enqueued, and the library keeps
working afterwards (a bad call does not poison the next good one)."""
import ctypes

import numpy as np
import pytest

import oracle as O
from paper_1505_07690_amd import inputs

pytestmark = pytest.mark.gpu


def test_compute_call_errors_and_recovery():
    import torch
    from paper_1505_07690_amd import os3d
    L = os3d.lib()
    shape = (16, 12, 20)
    n = inputs.icosahedral_orientations(0)
    p = O.WaveletParams(L=8, s_theta=inputs.s_theta_for(12))
    bank = os3d.Bank(shape, n, p)
    vol = inputs.tubes(shape, 2, 1.5, 0.1, 0, 50)
    f = torch.from_numpy(vol).cuda()
    U = torch.empty((12,) + shape, dtype=torch.complex64, device="cuda")
    out = torch.empty(shape, dtype=torch.float32, device="cuda")
    ws = bank.workspace()
    h, fp, up, op, wp = bank.handle, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(U.data_ptr()), \
        ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr())
    # batch 0, unknown dtype, 16-bit without scales, missing or short workspace
    assert L.os3d_forward(h, fp, 0, up, 0, None, wp, ws.numel(), None) == -1
    assert L.os3d_forward(h, fp, 1, up, 7, None, wp, ws.numel(), None) == -1
    assert L.os3d_forward(h, fp, 1, up, 1, None, wp, ws.numel(), None) == -1
    assert b"scales" in L.os3d_last_error()
    assert L.os3d_forward(h, fp, 1, up, 0, None, None, ws.numel(), None) == -1
    assert L.os3d_forward(h, fp, 1, up, 0, None, wp, ws.numel() - 1, None) == -2
    assert L.os3d_reconstruct(h, up, 0, None, 0, op, wp, ws.numel(), None) == -1
    assert L.os3d_reconstruct_approx(h, up, 2, None, 1, op, None) == -1
    assert L.os3d_process(h, fp, 1, 3, 1.5, op, wp, ws.numel(), None) == -1
    assert L.os3d_process(h, fp, 1, 1, 0.0, op, wp, ws.numel(), None) == -1
    assert L.os3d_bank_psi(h, 12, op, None) == -1
    # the next good calls are unaffected
    U2, _ = os3d.forward(f, bank)
    rec = os3d.reconstruct(U2, bank).cpu().numpy()
    ob = O.build_bank(shape, n, p)
    want = O.reconstruct(O.forward(vol.astype(np.float64), ob), ob)
    assert np.linalg.norm(rec - want) / np.linalg.norm(want) < 1e-5
