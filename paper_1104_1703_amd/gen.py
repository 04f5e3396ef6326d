"""Seeded synthetic inputs for the masked multigrid Poisson solver.

This module only draws geometry and fields (masks, densities, Dirichlet
values).  It holds none of the solver's arithmetic, so both the CPU oracle
(test infrastructure) and the GPU path read inputs from here.

Conventions shared by every generator:
  * arrays are C-contiguous ``(nz, ny, nx)`` with x fastest;
  * the unit cube is split into cells of width ``h = 1/n`` (per axis, the
    longest axis sets ``h`` for non-cubic patches), cell centres at
    ``(i + 1/2) h``;
  * ``mask`` is int8 with +1 inside the domain and -1 outside (the colouring
    of the paper's Sec. 3), and the outermost layer of cells is always -1;
  * ``rho`` and ``dirichlet`` are float64; ``dirichlet`` is a cell-centred
    field whose face average between an active and an inactive cell is the
    Dirichlet value on that face.

The workloads stand in for the paper's AMR grids (Sec. 5, Table 1), which are
not available: a sphere, a sphere with holes, uneven masked patches, a porous
box and a learned-guess training set.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "Problem",
    "centres",
    "sphere_problem",
    "holes_problem",
    "porous_problem",
    "patch_problems",
    "random_small_problem",
    "training_sample",
    "nested_levels",
    "level_centres",
    "frame_mask",
    "ln_profile",
]


class Problem:
    """One Poisson problem: mask, density and cell-centred Dirichlet field."""

    def __init__(self, mask, rho, dirichlet, h, name=""):
        self.mask = np.ascontiguousarray(mask, dtype=np.int8)
        self.rho = np.ascontiguousarray(rho, dtype=np.float64)
        self.dirichlet = None if dirichlet is None else np.ascontiguousarray(dirichlet, dtype=np.float64)
        self.h = float(h)
        self.name = name

    @property
    def shape(self):
        return self.mask.shape

    @property
    def n_active(self):
        return int((self.mask == 1).sum())


def centres(n: int, h: float | None = None) -> np.ndarray:
    """Cell-centre coordinates ``(i + 1/2) h`` for ``i < n``."""
    if h is None:
        h = 1.0 / n
    return (np.arange(n, dtype=np.float64) + 0.5) * h


def _frame(mask: np.ndarray) -> np.ndarray:
    mask[0, :, :] = -1
    mask[-1, :, :] = -1
    mask[:, 0, :] = -1
    mask[:, -1, :] = -1
    mask[:, :, 0] = -1
    mask[:, :, -1] = -1
    return mask


def _r2(n: int, c=(0.5, 0.5, 0.5)) -> np.ndarray:
    x = centres(n)
    dz = (x - c[2])[:, None, None] ** 2
    dy = (x - c[1])[None, :, None] ** 2
    dx = (x - c[0])[None, None, :] ** 2
    return dz + dy + dx


def _carve_spheres(mask: np.ndarray, cen: np.ndarray, rad: np.ndarray, h: float) -> None:
    """Set mask = -1 for every cell whose centre lies strictly inside a sphere.

    Each sphere is tested only inside its index bounding box; the test is
    the same ``|x - c|^2 < r^2`` comparison everywhere.
    """
    nz, ny, nx = mask.shape
    for (cx, cy, cz), r in zip(cen, rad):
        lo = [max(0, int(np.floor((c - r) / h - 0.5))) for c in (cx, cy, cz)]
        hi = [min(n, int(np.ceil((c + r) / h + 0.5)) + 1) for c, n in zip((cx, cy, cz), (nx, ny, nz))]
        if lo[0] >= hi[0] or lo[1] >= hi[1] or lo[2] >= hi[2]:
            continue
        xs = (np.arange(lo[0], hi[0]) + 0.5) * h - cx
        ys = (np.arange(lo[1], hi[1]) + 0.5) * h - cy
        zs = (np.arange(lo[2], hi[2]) + 0.5) * h - cz
        d2 = zs[:, None, None] ** 2 + ys[None, :, None] ** 2 + xs[None, None, :] ** 2
        sub = mask[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        sub[d2 < r * r] = -1


def _gaussian_sum(n: int, cen, sig, amp) -> np.ndarray:
    """Sum of isotropic Gaussians ``A exp(-|x-c|^2 / 2 s^2)`` (separable)."""
    x = centres(n)
    out = np.zeros((n, n, n), dtype=np.float64)
    for (cx, cy, cz), s, a in zip(cen, sig, amp):
        ex = np.exp(-((x - cx) ** 2) / (2 * s * s))
        ey = np.exp(-((x - cy) ** 2) / (2 * s * s))
        ez = np.exp(-((x - cz) ** 2) / (2 * s * s))
        out += a * (ez[:, None, None] * ey[None, :, None]) * ex[None, None, :]
    return out


def sphere_problem(n: int = 32, R: float = 0.4, a: float = 0.2) -> Problem:
    """Sphere of radius ``R`` centred in the unit cube; rho = 1 inside ``a``.

    Dirichlet value 0 on the staircase boundary (cells outside ``R`` are
    inactive).  At n = 32 this is the 32^3 plain-FP64 workload.
    """
    r2 = _r2(n)
    mask = np.where(r2 < R * R, 1, -1).astype(np.int8)
    _frame(mask)
    rho = np.where(r2 < a * a, 1.0, 0.0)
    return Problem(mask, rho, None, 1.0 / n, name=f"sphere{n}")


def holes_problem(n: int = 256, seed: int = 2, n_holes: int = 64, r_lo: float = 0.02, r_hi: float = 0.1,
                  R: float = 0.45, n_gauss: int = 32, s_lo: float = 0.01, s_hi: float = 0.05) -> Problem:
    """Outer sphere (radius ``R``) minus ``n_holes`` random spheres.

    Draw order from ``default_rng(seed)``: hole centres (n_holes, 3) in
    U[0,1), hole radii U[r_lo, r_hi), Gaussian centres (n_gauss, 3),
    Gaussian widths U[s_lo, s_hi), Gaussian amplitudes N(0,1).
    Dirichlet value 0 everywhere.  At n = 256, seed 2 this is the 256^3
    masked workload.
    """
    rng = np.random.default_rng(seed)
    hc = rng.random((n_holes, 3))
    hr = rng.uniform(r_lo, r_hi, n_holes)
    gc = rng.random((n_gauss, 3))
    gs = rng.uniform(s_lo, s_hi, n_gauss)
    ga = rng.standard_normal(n_gauss)
    h = 1.0 / n
    mask = np.where(_r2(n) < R * R, 1, -1).astype(np.int8)
    _carve_spheres(mask, hc, hr, h)
    _frame(mask)
    rho = _gaussian_sum(n, gc, gs, ga)
    return Problem(mask, rho, None, h, name=f"holes{n}_s{seed}")


def _grf_k2(n: int, rng) -> np.ndarray:
    """Gaussian random field with power spectrum ~ k^-2, unit variance."""
    w = rng.standard_normal((n, n, n))
    wk = np.fft.rfftn(w)
    del w
    kz = np.fft.fftfreq(n)[:, None, None]
    ky = np.fft.fftfreq(n)[None, :, None]
    kx = np.fft.rfftfreq(n)[None, None, :]
    kk = np.sqrt(kz * kz + ky * ky + kx * kx)
    with np.errstate(divide="ignore"):
        amp = np.where(kk > 0, 1.0 / np.where(kk > 0, kk, 1.0), 0.0)
    wk *= amp
    del amp, kk
    g = np.fft.irfftn(wk, s=(n, n, n), axes=(0, 1, 2))
    g -= g.mean()
    g /= g.std()
    return g


def porous_problem(n: int = 512, seed: int = 4, n_holes: int = 4096, r_lo: float = 0.005,
                   r_hi: float = 0.02) -> Problem:
    """Box with a 1-cell frame minus ``n_holes`` small random spheres.

    Draw order from ``default_rng(seed)``: hole centres, hole radii, then
    the white noise of the k^-2 Gaussian random field used as rho.
    Dirichlet value 0.  At n = 512 this is the mixed-precision workload.
    """
    rng = np.random.default_rng(seed)
    hc = rng.random((n_holes, 3))
    hr = rng.uniform(r_lo, r_hi, n_holes)
    h = 1.0 / n
    mask = np.ones((n, n, n), dtype=np.int8)
    _carve_spheres(mask, hc, hr, h)
    _frame(mask)
    rho = _grf_k2(n, rng)
    return Problem(mask, rho, None, h, name=f"porous{n}_s{seed}")


def _trilinear_up(coarse: np.ndarray, shape) -> np.ndarray:
    """Trilinear interpolation of a (nz/2+1, ny/2+1, nx/2+1) node field to fine centres."""
    out = coarse
    for axis, n in enumerate(shape):
        m = out.shape[axis]
        # fine centre (i + 1/2) in fine units -> coarse node coordinate (i + 1/2)/2
        t = (np.arange(n) + 0.5) / 2.0
        i0 = np.clip(np.floor(t).astype(int), 0, m - 2)
        w = t - i0
        a = np.take(out, i0, axis=axis)
        b = np.take(out, i0 + 1, axis=axis)
        sh = [1] * out.ndim
        sh[axis] = n
        w = w.reshape(sh)
        out = a * (1 - w) + b * w
    return out


def _edge(rng, lo=16, hi=128, mult=8) -> int:
    e = float(np.exp(rng.uniform(np.log(lo), np.log(hi))))
    return int(min(hi, max(lo, mult * round(e / mult))))


def patch_problems(count: int = 512, seed: int = 3, active_frac: float = 0.6):
    """Uneven masked patches standing in for AMR-level patches.

    Each patch gets its own generator from ``SeedSequence(seed).spawn``.
    Edges are log-uniform in [16, 128], rounded to a multiple of 8.  The
    mask thresholds blurred white noise at the (1 - active_frac) quantile;
    the Dirichlet field is trilinear from a half-resolution N(0,1) node
    field; rho = exp(N(0,1)) per cell.
    """
    from scipy.ndimage import gaussian_filter

    out = []
    for k, ss in enumerate(np.random.SeedSequence(seed).spawn(count)):
        rng = np.random.default_rng(ss)
        nx, ny, nz = _edge(rng), _edge(rng), _edge(rng)
        shape = (nz, ny, nx)
        noise = rng.standard_normal(shape)
        sig = max(2.0, min(shape) / 8.0)
        sm = gaussian_filter(noise, sig, mode="wrap")
        thr = np.quantile(sm, 1.0 - active_frac)
        mask = np.where(sm > thr, 1, -1).astype(np.int8)
        _frame(mask)
        coarse = rng.standard_normal((nz // 2 + 1, ny // 2 + 1, nx // 2 + 1))
        bnd = _trilinear_up(coarse, shape)
        rho = np.exp(rng.standard_normal(shape))
        h = 1.0 / max(shape)
        out.append(Problem(mask, rho, bnd, h, name=f"patch{k}"))
    return out


def random_small_problem(shape, seed: int, active_frac: float = 0.7, with_dirichlet: bool = True,
                         blur: float = 0.0) -> Problem:
    """Small random problem for parity and edge-case tests.

    Mask: i.i.d. (or blurred) noise thresholded to ``active_frac``, frame -1.
    rho ~ N(0,1); Dirichlet ~ N(0,1) when requested.
    """
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal(shape)
    if blur > 0:
        from scipy.ndimage import gaussian_filter
        noise = gaussian_filter(noise, blur, mode="wrap")
    thr = np.quantile(noise, 1.0 - active_frac)
    mask = np.where(noise > thr, 1, -1).astype(np.int8)
    _frame(mask)
    rho = rng.standard_normal(shape)
    bnd = rng.standard_normal(shape) if with_dirichlet else None
    return Problem(mask, rho, bnd, 1.0 / max(shape), name=f"rand{shape}_s{seed}")


def training_sample(n: int = 64, seed: int = 10000) -> Problem:
    """One learned-guess training sample drawn like the 256^3 holes workload
    (same physical radii and widths), at ``n^3``."""
    return holes_problem(n=n, seed=seed)


# ------------------------------------------------------- nested levels (AMR)
def nested_levels(n: int, depth: int):
    """Geometry of nested refined levels around the box centre, standing in
    for the paper's quasi-Lagrangian AMR of a centrally concentrated profile
    (Sec. 5.1): level 0 is the unit box as an n^3 array, level k an n^3 array
    of cells 1/(n 2^k) covering the central 1/2^k of the box.  Each level's
    outer layer of cells is its boundary.  Returns [(shape, h, origin)] with
    origin = (x0, y0, z0) the lower corner of the array."""
    levels = []
    for k in range(depth + 1):
        h = 1.0 / (n * 2 ** k)
        o = 0.5 - 0.5 * n * h
        levels.append(((n, n, n), h, (o, o, o)))
    return levels


def level_centres(shape, h: float, origin) -> np.ndarray:
    """Cell-centre coordinates (nz, ny, nx, 3) as (x, y, z) of an array of
    cells of width h whose lower corner is at origin."""
    nz, ny, nx = shape
    x = origin[0] + (np.arange(nx) + 0.5) * h
    y = origin[1] + (np.arange(ny) + 0.5) * h
    z = origin[2] + (np.arange(nz) + 0.5) * h
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return np.stack([X, Y, Z], axis=-1)


def frame_mask(shape) -> np.ndarray:
    """All cells active except the outer layer."""
    m = -np.ones(shape, dtype=np.int8)
    m[1:-1, 1:-1, 1:-1] = 1
    return m


def ln_profile(pts: np.ndarray, r0: float = 0.1):
    """3D analogue of the paper's accuracy-test profile (Sec. 5.1) around the
    box centre: phi = ln((r/r0)^2 + 1), rho = Laplacian(phi) =
    (6 r0^2 + 2 r^2) / (r^2 + r0^2)^2 and grad(phi) = 2 (x - c) / (r^2 + r0^2).
    Returns (phi, rho, grad) at the points (..., 3)."""
    d = pts - 0.5
    r2 = (d ** 2).sum(-1)
    phi = np.log(r2 / r0 ** 2 + 1.0)
    rho = (6.0 * r0 ** 2 + 2.0 * r2) / (r2 + r0 ** 2) ** 2
    grad = 2.0 * d / (r2 + r0 ** 2)[..., None]
    return phi, rho, grad
