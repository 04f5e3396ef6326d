"""First guesses for the multigrid solve (the iteration of Sec. 2 starts from
any phi; the paper reports it insensitive to that start, Sec. 2 and Sec. 6).

* zero: phi = 0 (the paper's timings);
* interpolated: the problem coarsened by 2 per axis is solved by the same
  multigrid library to a loose tolerance, then linearly up-sampled;
* learned: the U-Net of this library, run at 1/stride resolution and
  linearly up-sampled.

Every step runs in the library's kernels; this module only wires calls.
"""
from __future__ import annotations

import os

import torch

from . import mg

WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "unet_holes64.safetensors")


class InterpolatedGuess:
    """Coarse solve + up-sampling.  The coarse hierarchy depends on the mask
    only and is built once (like the fine one)."""

    def __init__(self, mask: torch.Tensor, h: float, stride: int = 2, tol: float = 1e-4, **options):
        if stride != 2:
            raise ValueError("the interpolated guess coarsens by 2 per axis")
        self.stride = stride
        self.tol = tol
        self.mask = mask
        zero = torch.zeros(mask.shape, dtype=torch.float64, device=mask.device)
        _, mask_c, _ = mg.coarsen_problem(zero, mask, None, stride)
        self.mask_c = mask_c
        self.H = mg.Hierarchy(mask_c, h * stride, **options)
        self.phi_c = torch.zeros(mask_c.shape, dtype=torch.float64, device=mask.device)
        self.last_info = None

    def __call__(self, rho: torch.Tensor, dirichlet=None, out=None) -> torch.Tensor:
        rho_c, _, b_c = mg.coarsen_problem(rho, self.mask, dirichlet, self.stride)
        self.phi_c.zero_()
        _, self.last_info = self.H.solve(rho_c, self.phi_c, b_c, tol=self.tol)
        return mg.upsample_guess(self.phi_c, self.mask, out=out)

    def close(self):
        self.H.close()


def load_network(path: str = WEIGHTS, seed: int = 0) -> mg.UNet:
    """The U-Net with trained weights from ``path`` (raises if absent)."""
    if not os.path.exists(path):
        raise FileNotFoundError(f"no trained weights at {path}; run python -m paper_1104_1703_amd.train_unet")
    net = mg.UNet(seed=seed)
    net.load(path)
    return net


def learned_guess(net: mg.UNet, rho, mask, dirichlet=None, stride: int = 4, out=None) -> torch.Tensor:
    return net.infer(rho, mask, dirichlet, stride=stride, out=out)
