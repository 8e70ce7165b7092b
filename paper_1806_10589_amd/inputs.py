"""Seeded synthetic inputs: solid masks and random distribution perturbations.

This module holds no lattice-Boltzmann arithmetic. It is the one source of
inputs that both the HIP path and the CPU oracle consume, so that the two are
compared on identical data.

Masks are ``uint8`` arrays of shape ``(nz, ny, nx)`` (x fastest), 1 = solid.

The sphere packs stand in for the micro-CT sandstone sub-volume that the paper
drives its two-fluid experiment with (Results, Bentheimer section): overlapping
solid spheres with uniform centres and uniform radii, rasterised with the
minimum-image distance in x and y (the box is periodic across its sides), and
six pure-fluid reservoir layers at each z end as in the paper's drainage set-up.
"""
from __future__ import annotations

import numpy as np


def slit_channel(nx: int = 16, ny: int = 16, nz: int = 64) -> np.ndarray:
    """Plane channel: solid columns x = 0 and x = nx-1, fluid elsewhere."""
    m = np.zeros((nz, ny, nx), np.uint8)
    m[:, :, 0] = 1
    m[:, :, nx - 1] = 1
    return m


def square_duct(width: int, nz: int) -> np.ndarray:
    """Square tube: fluid interior width x width, one solid voxel layer around it."""
    n = width + 2
    m = np.ones((nz, n, n), np.uint8)
    m[:, 1:-1, 1:-1] = 0
    return m


def random_mask(shape, solid_fraction: float, seed: int) -> np.ndarray:
    """Independent random solid voxels (for brute-force tests on tiny boxes)."""
    rng = np.random.default_rng(seed)
    return (rng.random(shape) < solid_fraction).astype(np.uint8)


def carve_reservoirs(mask: np.ndarray, layers: int) -> np.ndarray:
    """Copy of ``mask`` with its first and last ``layers`` z-planes set to fluid."""
    m = np.array(mask, dtype=np.uint8, copy=True)
    if layers > 0:
        m[:layers] = 0
        m[-layers:] = 0
    return m


def sphere_pack(n: int | tuple, porosity: float, seed: int, rmin: float = 6.0,
                rmax: float = 10.0, reservoir_layers: int = 0, batch: int = 64):
    """Overlapping solid spheres until the porosity drops to ``porosity``.

    Centres are uniform in the box, radii uniform in [rmin, rmax]. A voxel
    (i, j, k) is solid when its minimum-image distance to a centre (periodic
    in x and y, not in z) is at most the radius. Spheres are drawn from
    ``numpy.random.default_rng(seed)`` (PCG64) and added one at a time in draw
    order until the sample's porosity is at or below the target. Reservoir
    layers are carved afterwards.

    Returns ``(mask, achieved_porosity, n_spheres)``; the porosity is that of
    the sample before the reservoirs are carved.
    """
    if isinstance(n, (tuple, list)):
        nz, ny, nx = (int(v) for v in n)
    else:
        nz = ny = nx = int(n)
    rng = np.random.default_rng(seed)
    solid = np.zeros((nz, ny, nx), np.uint8)
    total = nx * ny * nz
    n_solid = 0
    n_spheres = 0
    target_solid = (1.0 - porosity) * total
    rr = int(np.ceil(rmax))
    off = np.arange(-rr, rr + 1)
    while n_solid < target_solid:
        cs = rng.random((batch, 3)) * np.array([nx, ny, nz])
        rs = rmin + (rmax - rmin) * rng.random(batch)
        for (cx, cy, cz), r in zip(cs, rs):
            if n_solid >= target_solid:
                break
            ix = (np.floor(cx).astype(int) + off)
            iy = (np.floor(cy).astype(int) + off)
            iz = (np.floor(cz).astype(int) + off)
            iz = iz[(iz >= 0) & (iz < nz)]
            dx = ix - cx
            dy = iy - cy
            dz = iz - cz
            dx = dx - nx * np.round(dx / nx)
            dy = dy - ny * np.round(dy / ny)
            d2 = dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2
            hit = d2 <= r * r
            xs = np.mod(ix, nx)
            ys = np.mod(iy, ny)
            sub = solid[np.ix_(iz, ys, xs)]
            new = hit & (sub == 0)
            n_new = int(new.sum())
            if n_new:
                sub[new] = 1
                solid[np.ix_(iz, ys, xs)] = sub
                n_solid += n_new
            n_spheres += 1
    achieved = 1.0 - n_solid / total
    mask = carve_reservoirs(solid, reservoir_layers)
    return mask, achieved, n_spheres


def uniform_noise(shape, seed: int, low: float = -1.0, high: float = 1.0) -> np.ndarray:
    """Float64 uniform noise in [low, high) (used to perturb distributions)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(low, high, size=shape)


def pore_sites(mask: np.ndarray) -> np.ndarray:
    """Flat raster indices (x + nx*(y + ny*z)) of the pore voxels, in raster order.

    This is the site order of the sparse lattice: z slowest, x fastest.
    """
    return np.flatnonzero(np.asarray(mask).reshape(-1) == 0)
