"""One-way nested levels (AMR) in plain numpy: interface Dirichlet values,
the 5-point gradient and the composite-grid truncation errors.

TEST INFRASTRUCTURE ONLY: imported by ``tests/`` and ``bench.py``'s
accuracy study.  The GPU library never loads it.

Follows Sec. 5.1 (accuracy tests) and the one-way interface scheme of Sec. 3:
a refined level is solved after the coarser one, with Dirichlet values on its
boundary faces interpolated linearly from the coarser solution, and the
gradient of the potential (the paper's 5-point difference) takes the values
it needs beyond a level's boundary from the coarser level by the same linear
interpolation (Fig. "force-ramses").

A level is a box array (nz, ny, nx) of cells of width h whose lower corner
sits at ``origin`` = (x0, y0, z0); cell (i, j, k) has its centre at
origin + ((i, j, k) + 1/2) h.  Values live at cell centres.  Linear
interpolation between cell centres in 3D is trilinear.
"""
from __future__ import annotations

import numpy as np

from paper_1104_1703_amd.gen import frame_mask, level_centres as centres, ln_profile, nested_levels


def interp(phi_c, hc, origin_c, pts):
    """Trilinear interpolation of the cell-centred field phi_c (nz, ny, nx) at
    the points pts (..., 3) given as (x, y, z).  The 8 surrounding centres
    must lie inside the array.  Weights (1 - t, t) per axis; the 8 terms are
    summed with z slowest, then y, then x."""
    pts = np.asarray(pts, dtype=np.float64)
    out = np.zeros(pts.shape[:-1])
    idx, frac = [], []
    for a in range(3):
        s = (pts[..., a] - origin_c[a]) / hc - 0.5
        base = np.floor(s)
        idx.append(base.astype(np.int64))
        frac.append(s - base)
    nz, ny, nx = phi_c.shape
    I, J, K = idx
    if (I.min() < 0 or J.min() < 0 or K.min() < 0 or I.max() + 1 >= nx or J.max() + 1 >= ny
            or K.max() + 1 >= nz):
        raise ValueError("interpolation stencil outside the coarse array")
    wx = (1.0 - frac[0], frac[0])
    wy = (1.0 - frac[1], frac[1])
    wz = (1.0 - frac[2], frac[2])
    for c in range(2):
        for b in range(2):
            for a in range(2):
                w = wz[c] * wy[b] * wx[a]
                out = out + w * phi_c[K + c, J + b, I + a]
    return out


def patch_dirichlet(phi_c, hc, origin_c, shape, hf, origin_f):
    """Dirichlet field B (cell-centred, as the solver reads it: the face value
    between an active cell i and an inactive cell j is (B_i + B_j)/2) for a
    refined patch whose outer layer is its boundary and whose interior is
    active.  Interior cells get the interpolated coarse potential at their
    centre; a frame cell face-adjacent to exactly one interior cell gets
    2 g - B_i, g being the interpolated coarse potential at the centre of the
    shared face, so that (B_i + B_j)/2 = g; other frame cells get 0."""
    nz, ny, nx = shape
    B = np.zeros(shape)
    ctr = centres(shape, hf, origin_f)
    inner = (slice(1, nz - 1), slice(1, ny - 1), slice(1, nx - 1))
    B[inner] = interp(phi_c, hc, origin_c, ctr[inner])
    # the six faces of the interior block, one axis at a time
    for ax, n in ((0, nx), (1, ny), (2, nz)):
        for side in (0, 1):
            frame_i = 0 if side == 0 else n - 1
            act_i = 1 if side == 0 else n - 2
            sl_f = [slice(1, nz - 1), slice(1, ny - 1), slice(1, nx - 1)]
            sl_a = list(sl_f)
            arr_ax = 2 - ax  # array axis of coordinate ax
            sl_f[arr_ax] = slice(frame_i, frame_i + 1)
            sl_a[arr_ax] = slice(act_i, act_i + 1)
            face = 0.5 * (ctr[tuple(sl_f)] + ctr[tuple(sl_a)])
            g = interp(phi_c, hc, origin_c, face)
            B[tuple(sl_f)] = 2.0 * g - B[tuple(sl_a)]
    return B


def grad5(phi, active, h, origin, coarse=None, bnd=None, exact=None):
    """Gradient of the potential on the active cells of a level by the
    paper's 5-point difference (Sec. 5.1):
        d/dx phi = (4/3) (phi[i+1] - phi[i-1]) / (2 h) - (1/3) (phi[i+2] - phi[i-2]) / (4 h),
    each of the 4 values taken from phi where that cell is an active cell of
    the level, else interpolated from the coarser level ``coarse`` =
    (phi_c, hc, origin_c) at that cell's centre; without a coarser level,
    from the Dirichlet field ``bnd`` (the outermost level's boundary values)
    where the cell is inside the array, NaN beyond.  ``exact`` (a function of
    the points) replaces both for the paper's control run with exact values
    at the interfaces.  Returns (3, nz, ny, nx) with components (x, y, z);
    inactive cells get 0."""
    nz, ny, nx = phi.shape
    out = np.zeros((3,) + phi.shape)
    act = active.astype(bool)
    kk, jj, ii = np.nonzero(act)
    for ax in range(3):
        vals = []
        for off in (1, -1, 2, -2):
            i2, j2, k2 = ii.copy(), jj.copy(), kk.copy()
            if ax == 0:
                i2 += off
            elif ax == 1:
                j2 += off
            else:
                k2 += off
            inside = (i2 >= 0) & (i2 < nx) & (j2 >= 0) & (j2 < ny) & (k2 >= 0) & (k2 < nz)
            v = np.full(ii.shape, np.nan)
            ci, cj, ck = np.clip(i2, 0, nx - 1), np.clip(j2, 0, ny - 1), np.clip(k2, 0, nz - 1)
            own = inside & act[ck, cj, ci]
            v[own] = phi[ck[own], cj[own], ci[own]]
            rest = ~own
            if exact is not None:
                pts = np.stack([origin[0] + (i2[rest] + 0.5) * h, origin[1] + (j2[rest] + 0.5) * h,
                                origin[2] + (k2[rest] + 0.5) * h], axis=-1)
                v[rest] = exact(pts)
            elif coarse is not None:
                pts = np.stack([origin[0] + (i2[rest] + 0.5) * h, origin[1] + (j2[rest] + 0.5) * h,
                                origin[2] + (k2[rest] + 0.5) * h], axis=-1)
                v[rest] = interp(coarse[0], coarse[1], coarse[2], pts)
            else:
                frame = rest & inside
                v[frame] = bnd[ck[frame], cj[frame], ci[frame]]
            vals.append(v)
        p1, m1, p2, m2 = vals
        out[ax][kk, jj, ii] = (4.0 / 3.0) * (p1 - m1) / (2.0 * h) - (1.0 / 3.0) * (p2 - m2) / (4.0 * h)
    return out


# ------------------------------------------------------------------ study --
# (inputs: the profile, the level geometry and masks come from the seeded
# input module shared with the GPU path)


def solve_nested(n, depth, r0, solve, exact_interface=False):
    """One-way solve of the nested levels: level 0 with the exact potential as
    its Dirichlet field, each finer level with Dirichlet values interpolated
    from the level above (or, for the paper's control run, the exact
    potential).  ``solve(mask, h, rho, B) -> phi`` is any FP64 solver of one
    level (the oracle's multigrid in the tests).  Returns
    [(phi, rho, B, shape, h, origin)] per level."""
    out = []
    for k, (shape, h, origin) in enumerate(nested_levels(n, depth)):
        ctr = centres(shape, h, origin)
        phi_e, rho, _ = ln_profile(ctr, r0)
        if k == 0 or exact_interface:
            B = phi_e
        else:
            pc, _, _, _, hc, oc = out[-1]
            B = patch_dirichlet(pc, hc, oc, shape, h, origin)
        phi = solve(frame_mask(shape), h, rho, B)
        out.append((phi, rho, B, shape, h, origin))
    return out


def nested_grads(levels, r0=None, exact_interface=False):
    """grad5 on every level: level 0 with its Dirichlet field beyond its
    active cells, each finer level with the level above (or the exact
    potential of the ln profile with parameter r0 for the control run)."""
    grads = []
    for k, (phi, _, B, shape, h, origin) in enumerate(levels):
        active = frame_mask(shape) == 1
        if k > 0 and exact_interface:
            grads.append(grad5(phi, active, h, origin, exact=lambda p: ln_profile(p, r0)[0]))
        elif k == 0:
            grads.append(grad5(phi, active, h, origin, bnd=B))
        else:
            pc, _, _, _, hc, oc = levels[k - 1]
            grads.append(grad5(phi, active, h, origin, coarse=(pc, hc, oc)))
    return grads


def composite_errors(levels, grads, r0):
    """Truncation errors over the composite grid: each point counted on the
    finest level that covers it (a level's active cells minus those covered
    by the next level's active region), volume-weighted L2 and L-infinity of
    the potential error and of the gradient error's Euclidean length, the
    latter relative to the largest exact gradient length.  Level-0 cells
    whose 5-point stencil leaves the array are left out."""
    e_phi, e_g, vol = [], [], []
    gmax = 0.0
    for k, (phi, _, _, shape, h, origin) in enumerate(levels):
        ctr = centres(shape, h, origin)
        phi_e, _, grad_e = ln_profile(ctr, r0)
        use = frame_mask(shape) == 1
        if k + 1 < len(levels):
            _, _, _, fs, fh, fo = levels[k + 1]
            lo = np.array(fo) + fh           # the next level's active region
            hi = np.array(fo) + (np.array(fs[::-1]) - 1) * fh
            inside = np.all((ctr > lo) & (ctr < hi), axis=-1)
            use &= ~inside
        if k == 0:
            core = np.zeros(shape, dtype=bool)
            core[2:-2, 2:-2, 2:-2] = True
            use &= core
        e_phi.append(np.abs(phi - phi_e)[use])
        g = np.moveaxis(grads[k], 0, -1)
        e_g.append(np.linalg.norm(g - grad_e, axis=-1)[use])
        vol.append(np.full(use.sum(), h ** 3))
        gmax = max(gmax, float(np.linalg.norm(grad_e, axis=-1)[use].max()))
    e_phi, e_g, vol = np.concatenate(e_phi), np.concatenate(e_g), np.concatenate(vol)
    return {"phi_linf": float(e_phi.max()), "phi_l2": float(np.sqrt((vol * e_phi ** 2).sum() / vol.sum())),
            "grad_linf": float(e_g.max() / gmax), "grad_l2": float(np.sqrt((vol * e_g ** 2).sum() / vol.sum()) / gmax)}
