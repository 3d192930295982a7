"""Seeded EM-like image stacks (stand-in for the paper's uint8 EM sections, Section 2.1).

The paper's data (Kasthuri S1, AC3/AC4) is not available, so every workload uses
this generator. Recipe, per slice z of a volume with seed s:

* ``rng = numpy.random.default_rng([s, z])`` (PCG64).
* Voronoi cells: a Poisson(H*W/spacing^2) number of seeds placed uniformly in the
  slice (mean cell spacing 32 px, about 1000 cells per 1024^2 slice).
* Cell interiors take an intensity drawn from U(140, 220), one per cell.
* A pixel is on a membrane ridge iff d2 - d1 < ridge (2 px), where d1, d2 are its
  distances to the nearest and second-nearest seed; ridge pixels are set to 40.
* Gaussian blur, sigma 1.5 (truncate 4 sigma, reflecting borders), then additive
  N(0, noise^2) noise with noise = 12, then rint and clip to [0, 255] as uint8.

Slices are independent, so any slice can be regenerated alone.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
from scipy.ndimage import gaussian_filter
from scipy.spatial import cKDTree


def em_slice(seed: int, z: int, H: int, W: int, *, spacing: float = 32.0,
             ridge: float = 2.0, blur: float = 1.5, noise: float = 12.0,
             workers: int = 1) -> np.ndarray:
    """One H x W uint8 slice; deterministic in (seed, z, H, W, parameters)."""
    rng = np.random.default_rng([int(seed), int(z)])
    n = max(2, int(rng.poisson(H * W / (spacing * spacing))))
    pts = rng.uniform((0.0, 0.0), (float(H), float(W)), size=(n, 2))
    level = rng.uniform(140.0, 220.0, size=n)
    yy, xx = np.meshgrid(np.arange(H, dtype=np.float64) + 0.5,
                         np.arange(W, dtype=np.float64) + 0.5, indexing="ij")
    d, idx = cKDTree(pts).query(np.stack([yy.ravel(), xx.ravel()], axis=1), k=2,
                                workers=workers)
    img = level[idx[:, 0]]
    img[(d[:, 1] - d[:, 0]) < ridge] = 40.0
    img = gaussian_filter(img.reshape(H, W), blur, mode="reflect", truncate=4.0)
    img = img + rng.normal(0.0, noise, size=(H, W))
    return np.clip(np.rint(img), 0, 255).astype(np.uint8)


def em_volume(seed: int, Z: int, H: int, W: int, *, threads: int | None = None,
              **kw) -> np.ndarray:
    """Z x H x W uint8 volume; slice z is ``em_slice(seed, z, H, W)``."""
    out = np.empty((Z, H, W), dtype=np.uint8)
    if threads is None:
        threads = min(16, os.cpu_count() or 1)

    def one(z):
        out[z] = em_slice(seed, z, H, W, **kw)

    if threads <= 1 or Z == 1:
        for z in range(Z):
            one(z)
    else:
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(one, range(Z)))
    return out
