"""The backward rule of the autograd function, grad_f = Re W^H grad_U with
W^H Z = sum_i IDFT(psi_hat_i DFT(Z_i)) (the library's adjoint), checked under
PyTorch's complex-gradient convention by torch.autograd.gradcheck on a tiny
FP64 CPU stand-in of W built from the oracle's bank.  The library itself runs
on the GPU (its backward is checked there against the oracle and finite
differences); this test pins the rule it implements.  CPU only."""
import numpy as np
import torch

import oracle as O
from paper_1505_07690_amd import inputs


def _stand_in(psi):
    psi_t = torch.from_numpy(psi)

    class W(torch.autograd.Function):
        @staticmethod
        def forward(ctx, f):
            return torch.fft.ifftn(psi_t * torch.fft.fftn(f, dim=(-3, -2, -1)), dim=(-3, -2, -1))

        @staticmethod
        def backward(ctx, g):
            # the rule of the autograd function: Re sum_i IDFT(psi_i DFT(g_i))
            return torch.real(torch.fft.ifftn(psi_t * torch.fft.fftn(g, dim=(-3, -2, -1)), dim=(-3, -2, -1)).sum(0))

    return W.apply


def test_backward_rule_passes_gradcheck():
    shape = (4, 3, 5)
    n = inputs.icosahedral_orientations(0)
    b = O.build_bank(shape, n, O.WaveletParams(L=6, s_theta=1.3))
    W = _stand_in(b["psi_hat"])
    f = torch.from_numpy(np.random.default_rng(0).standard_normal(shape)).requires_grad_(True)
    assert torch.autograd.gradcheck(W, (f,), eps=1e-6, atol=1e-8, rtol=1e-6)


def test_backward_rule_gives_the_gradient_of_a_weighted_energy():
    """For L = sum w |U|^2 the rule gives W^H (2 w U), which is what the GPU
    test compares the library's gradient with."""
    shape = (4, 4, 3)
    n = inputs.icosahedral_orientations(0)
    b = O.build_bank(shape, n, O.WaveletParams(L=6, s_theta=1.3))
    W = _stand_in(b["psi_hat"])
    rng = np.random.default_rng(1)
    f0 = rng.standard_normal(shape)
    w = torch.from_numpy(rng.random((len(n),) + shape))
    f = torch.from_numpy(f0).requires_grad_(True)
    U = W(f)
    torch.sum(w * torch.abs(U) ** 2).backward()
    want = O.adjoint(2 * w.numpy() * O.forward(f0, b), b)
    assert np.max(np.abs(f.grad.numpy() - want)) < 1e-12 * np.max(np.abs(want))
