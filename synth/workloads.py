"""Workload shapes and seeded draws (tile lists, training patches).

Configurations (sizes of the synthetic stand-ins for the paper's EM stacks):

* ``tiny``      - net A, FP32, one 256x256 slice, seed 1.
* ``plain``     - net B, FP32, 32 x 1024 x 1024, seed 2.
* ``precision`` - net B, BF16 / FP8, 128 x 2048 x 2048, seed 3; errors are taken on
  slices 0-3, output window [0,256)^2, plus three seeded windows.
* ``batch``     - net B, BF16, 512 tiles, side L = round(exp(U(ln 64, ln 1024))),
  1-8 slices, 8-px input halo; seed 4.
* ``student``   - net S, BF16; teacher maps from FP32 net B over 64 volumes of
  16 x 512 x 512 (seeds 5000..5063); batch 16 patches of 128 x 128.

Blocks of the volume are processed independently with a halo of input context
(the paper segments blocks independently, Section 2.1, "Block merging").
"""
from __future__ import annotations

import numpy as np

from .em import em_slice

CONFIGS = {
    "tiny": {"net": "A", "precision": "fp32", "shape": (1, 256, 256), "seed": 1},
    "plain": {"net": "B", "precision": "fp32", "shape": (32, 1024, 1024), "seed": 2},
    "precision": {"net": "B", "precision": ("bf16", "fp8"), "shape": (128, 2048, 2048),
                  "seed": 3},
    "batch": {"net": "B", "precision": "bf16", "n_tiles": 512, "side": (64, 1024),
              "slices": (1, 8), "halo": 8, "seed": 4},
    "student": {"net": "S", "precision": "bf16", "train_volumes": 64,
                "train_shape": (16, 512, 512), "train_seed0": 5000, "batch": 16,
                "patch": 128, "lr": 1e-3},
}


def batch_tiles(n: int = 512, seed: int = 4, side=(64, 1024), slices=(1, 8), halo: int = 8):
    """Tile geometry list: dicts with z, h, w (input incl. halo), halo, seed.

    Output of a tile is its z x L x L interior; the input is z x (L+2 halo)^2.
    """
    rng = np.random.default_rng([int(seed), 0xB47C])
    lo, hi = np.log(side[0]), np.log(side[1])
    out = []
    for t in range(n):
        L = int(round(float(np.exp(rng.uniform(lo, hi)))))
        z = int(rng.integers(slices[0], slices[1] + 1))
        out.append({"z": z, "h": L + 2 * halo, "w": L + 2 * halo, "halo": halo,
                    "seed": int(seed) * 100000 + t})
    return out


def student_patch_origins(rng: np.random.Generator, batch: int, n_volumes: int, Z: int,
                          H: int, W: int, patch: int = 128, margin: int = 3):
    """Uniform (volume, slice, y, x) draws; y, x in [margin, H - patch - margin]."""
    v = rng.integers(0, n_volumes, size=batch)
    z = rng.integers(0, Z, size=batch)
    y = rng.integers(margin, H - patch - margin + 1, size=batch)
    x = rng.integers(margin, W - patch - margin + 1, size=batch)
    return np.stack([v, z, y, x], axis=1)


def mixed_difficulty_volume(seed: int, Z: int, H: int, W: int, tile: int = 512,
                            hard_frac: float = 0.25):
    """Volume whose tiles are drawn from two generators: the default one, and a
    harder one (noise sigma 24, cell spacing 16) on a seeded subset of tiles.

    Returns (volume, hard_mask[z, ty, tx]).
    """
    rng = np.random.default_rng([int(seed), 0x4D49])
    ty, tx = (H + tile - 1) // tile, (W + tile - 1) // tile
    hard = rng.random((Z, ty, tx)) < hard_frac
    vol = np.empty((Z, H, W), dtype=np.uint8)
    for z in range(Z):
        easy = em_slice(seed, z, H, W)
        if hard[z].any():
            hardimg = em_slice(seed + 7919, z, H, W, noise=24.0, spacing=16.0)
            m = np.kron(hard[z], np.ones((tile, tile), dtype=bool))[:H, :W]
            vol[z] = np.where(m, hardimg, easy)
        else:
            vol[z] = easy
    return vol, hard


def maskextend_maps(seed: int, Z: int, H: int, W: int) -> np.ndarray:
    """Synthetic input of MaskExtend (Section 3): for each of Z output sections
    the twelve maps the paper stacks, as float32 Z x H x W x 12 (channel
    fastest). The paper's EM, object masks and membrane maps are not available;
    the stand-ins come from an EM-like stack E of Z + 6 sections (em_slice with
    this seed), section s = z + 4 for output z:

    * channels 0-2: E[s-1], E[s], E[s+1] / 255 (the three EM sections);
    * channels 3-6: object masks of sections s-4 .. s-1, 1 where the section
      blurred with sigma 2 exceeds 150 (bright cell interiors), else 0;
    * channels 7-11: membrane probabilities of sections s-2 .. s+2, a logistic
      of the section blurred with sigma 1: 1 / (1 + exp((b - 120) / 15)).
    """
    from scipy.ndimage import gaussian_filter
    E = np.stack([em_slice(seed, k, H, W) for k in range(Z + 6)]).astype(np.float64)
    mask = np.stack([(gaussian_filter(e, 2.0) > 150.0) for e in E]).astype(np.float64)
    prob = np.stack([1.0 / (1.0 + np.exp((gaussian_filter(e, 1.0) - 120.0) / 15.0)) for e in E])
    out = np.empty((Z, H, W, 12), dtype=np.float32)
    for z in range(Z):
        s = z + 4
        chans = [E[s - 1] / 255.0, E[s] / 255.0, E[s + 1] / 255.0]
        chans += [mask[k] for k in range(s - 4, s)]
        chans += [prob[k] for k in range(s - 2, s + 3)]
        out[z] = np.stack(chans, axis=-1)
    return out
