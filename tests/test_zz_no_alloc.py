"""The reconstruction entry point that allocates nothing (its workspace is
the library's static device scratch), through the C ABI, against
os3d_reconstruct with a caller workspace: two calls in a row, the second on
a smaller volume, each within the FP32 tolerance (relative L2 1e-5; the pair
batches differ, so the summation order of the orientation sum does too)."""
import ctypes

import numpy as np
import pytest

from paper_1505_07690_amd import inputs

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    from paper_1505_07690_amd import os3d
    os3d.lib()
    return t


def _case(torch, shape, level, L, seed, dtype):
    from paper_1505_07690_amd import os3d
    n = inputs.icosahedral_orientations(level)
    bank = os3d.Bank(shape, n, os3d.make_params(L=L, s_theta=inputs.s_theta_for(len(n))))
    f = inputs.tubes_device(shape, 12, (1.0, 3.0), 0.2, 0, seed)
    U, sc = os3d.forward(f, bank, dtype=dtype)
    return bank, U, sc


def _noalloc_raw(torch, bank, U, sc, dtype):
    """The entry point called through ctypes with raw pointers."""
    from paper_1505_07690_amd import os3d
    out = torch.empty(bank.shape, dtype=torch.float32, device="cuda")
    rc = os3d.lib().os3d_reconstruct_noalloc(bank.handle, ctypes.c_void_p(U.data_ptr()), os3d.DTYPES[dtype],
                                            ctypes.c_void_p(sc.data_ptr() if sc is not None else 0), 1,
                                            ctypes.c_void_p(out.data_ptr()),
                                            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, os3d.lib().os3d_last_error()
    return out


@pytest.mark.parametrize("dtype", ["c64", "bf16"])
def test_noalloc_matches_the_workspace_entry_point_twice(torch, dtype):
    from paper_1505_07690_amd import os3d
    # a large call (128^3 x 42: three pairs per launch fit the scratch) then a smaller one (64^3 x 12)
    for shape, level, L, seed in (((128, 128, 128), 1, 16, 41), ((64, 64, 64), 0, 8, 42)):
        bank, U, sc = _case(torch, shape, level, L, seed, dtype)
        got = _noalloc_raw(torch, bank, U, sc, dtype)
        want = os3d.reconstruct(U, bank, scales=sc, dtype=dtype)
        torch.cuda.synchronize()
        assert rel(got.cpu().numpy(), want.cpu().numpy()) < 1e-5, (shape, dtype)
        # the Python binding of the same entry point
        got2 = os3d.reconstruct_noalloc(U, bank, scales=sc, dtype=dtype)
        assert torch.equal(got2, got)


def test_noalloc_rejects_a_volume_beyond_the_scratch(torch):
    from paper_1505_07690_amd import os3d
    shape = (256, 256, 128)  # 2^23 voxels: X and one pair need 128 MiB
    n = np.array([[0.0, 0.6, 0.8], [0.0, -0.6, -0.8]])
    bank = os3d.Bank(shape, n, os3d.make_params(L=4, s_theta=0.7))
    U = torch.zeros((2,) + shape, dtype=torch.complex64, device="cuda")
    out = torch.empty(shape, dtype=torch.float32, device="cuda")
    rc = os3d.lib().os3d_reconstruct_noalloc(bank.handle, ctypes.c_void_p(U.data_ptr()), 0, None, 1,
                                            ctypes.c_void_p(out.data_ptr()), None)
    assert rc == os3d.OS3DError(-2, "").code == -2
    assert b"static scratch" in os3d.lib().os3d_last_error()
