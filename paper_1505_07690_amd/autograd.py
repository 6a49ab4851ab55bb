"""The forward transform as a torch.autograd.Function whose backward is the
library's adjoint (both through the C ABI).

For real f and U = W f, the gradient of a real loss L(U) with respect to f is
Re(W^H dL/dU) with PyTorch's complex-gradient convention (dL/dU =
dL/dRe U + i dL/dIm U); W^H U = sum_i IDFT(psi_hat_i DFT(U_i)) because every
psi_hat_i is real, which is exactly os3d_adjoint.
"""
import torch

from . import os3d


class OS3DFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, bank):
        U, _ = os3d.forward(f.contiguous(), bank)
        ctx.bank = bank
        return U

    @staticmethod
    def backward(ctx, grad_U):
        grad_f = os3d.adjoint(grad_U.contiguous(), ctx.bank)
        return grad_f, None


def orientation_score(f, bank):
    """U = W f with gradient support (float32 f [B, Nz, Ny, Nx] on the GPU)."""
    return OS3DFunction.apply(f, bank)
