"""One-way solve of nested refined levels (Sec. 3 one-way interface,
Sec. 5.1 accuracy tests) on the GPU path.

Each level is solved by the library's multigrid after the next coarser one,
with Dirichlet values interpolated from it (``mg_amr_dirichlet``); the
gradient of each level's potential is the paper's 5-point difference with
the values beyond the level taken from the coarser level (``mg_amr_grad5``).
The test problem is the 3D analogue of the paper's ln profile around the box
centre (inputs from ``gen``); the outermost level takes its exact values as
Dirichlet data.
"""
from __future__ import annotations

import torch

from . import gen, mg


class Level:
    def __init__(self, shape, h, origin, mask, rho, B, phi, grad, info):
        self.shape, self.h, self.origin = shape, h, origin
        self.mask, self.rho, self.B, self.phi, self.grad, self.info = mask, rho, B, phi, grad, info


def solve_nested(n: int, depth: int, r0: float = 0.1, tol: float = 1e-12, guess: str = "zero", device="cuda",
                 **options):
    """Levels 0..depth of ``gen.nested_levels(n, depth)``, each an n^3 box
    (outer layer = boundary), solved one way from the coarsest; returns the
    list of ``Level`` (device tensors) and the wall time in ms of the whole
    chain (interface values, solves, gradients; hierarchy builds excluded).
    guess = "interp" starts each refined level from the coarser solution
    interpolated to its cell centres (the paper's multilevel first guess,
    Sec. 5.2), which is the interior of its Dirichlet field; "zero" from 0."""
    geo = gen.nested_levels(n, depth)
    inputs = []
    for shape, h, origin in geo:
        phi_e, rho, _ = gen.ln_profile(gen.level_centres(shape, h, origin), r0)
        mask = torch.from_numpy(gen.frame_mask(shape)).to(device)
        inputs.append((mask, torch.from_numpy(rho).to(device), torch.from_numpy(phi_e).to(device)))
    hier = [mg.Hierarchy(m, h, **options) for (m, _, _), (_, h, _) in zip(inputs, geo)]
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    levels = []
    for k, ((shape, h, origin), (mask, rho, phi_e), H) in enumerate(zip(geo, inputs, hier)):
        if k == 0:
            B = phi_e
        else:
            c = levels[-1]
            B = mg.amr_dirichlet(c.phi, c.h, c.origin, shape, h, origin)
        phi0 = B.clone() if (k > 0 and guess == "interp") else None
        phi, info = H.solve(rho, phi0, B, tol=tol)
        if k == 0:
            grad = mg.amr_grad5(phi, mask, h, origin, bnd=B)
        else:
            grad = mg.amr_grad5(phi, mask, h, origin, coarse=(c.phi, c.h, c.origin))
        levels.append(Level(shape, h, origin, mask, rho, B, phi, grad, info))
    ev1.record()
    ev1.synchronize()
    ms = ev0.elapsed_time(ev1)
    for H in hier:
        H.close()
    return levels, ms
