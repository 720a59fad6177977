"""The discrete free energy as a differentiable PyTorch function.

G(X) is the energy of the current labels at atom positions X (the discrete
form of the paper's free-energy functional plus bonds); its gradient with
respect to X at fixed labels is minus the adjoint forces (the Appendix
gradient taken as the exact derivative of the discrete energy).  With
``relax_interface`` the labels are first relaxed to a local minimum at X
(Step 2 of the algorithm), so the gradient is the one Step 3 of the
algorithm descends along.  The energy, the forces and the interface
relaxation all run in the library's kernels; this module only moves
positions in and the gradient out.
"""
from __future__ import annotations

import numpy as np
import torch

from .vesis import Context


class _FreeEnergy(torch.autograd.Function):
    @staticmethod
    def forward(fctx, xyz: torch.Tensor, vctx: Context, relax_interface: bool, max_sweeps: int):
        x = xyz.detach()
        if x.dtype != torch.float64 or not x.is_contiguous():
            x = x.to(torch.float64).contiguous()
        vctx.set_positions(x)
        if relax_interface:
            vctx.minimize(max_sweeps)
        G = vctx.energy()["total"]
        if xyz.requires_grad:
            f = torch.from_numpy(vctx.forces()).to(device=xyz.device, dtype=xyz.dtype)
            fctx.save_for_backward(f)
        return torch.tensor(G, dtype=xyz.dtype, device=xyz.device)

    @staticmethod
    def backward(fctx, grad_out):
        (f,) = fctx.saved_tensors
        return -grad_out * f, None, None, None


def free_energy(vctx: Context, xyz: torch.Tensor, relax_interface: bool = False,
                max_sweeps: int = 20000) -> torch.Tensor:
    """G at positions ``xyz`` (an N x 3 tensor on the context's device).

    Differentiable in ``xyz``; the labels held by ``vctx`` stay fixed unless
    ``relax_interface`` relaxes them at ``xyz`` first."""
    if not isinstance(xyz, torch.Tensor) or not xyz.is_cuda:
        raise TypeError("xyz must be a CUDA tensor on the context's device")
    if tuple(xyz.shape) != (vctx.natoms, 3):
        raise ValueError(f"xyz must be ({vctx.natoms}, 3), got {tuple(xyz.shape)}")
    return _FreeEnergy.apply(xyz, vctx, bool(relax_interface), int(max_sweeps))


def gradient(vctx: Context) -> np.ndarray:
    """dG/dX at the context's current positions and labels (N x 3, host)."""
    return -vctx.forces()
