"""Distillation of the student from the plain net's probability maps.

The multi-pass idea of the paper (Section 1: a fast pass over everything, and
extra effort only where errors are likely) applied to the membrane stage: a
thinner student net is trained on the GPU (student_train_step: own forward and
backward kernels, FP64 loss and gradient-norm sums, Adam) to reproduce the
plain net's maps, and at inference tiles whose sampled disagreement is high fall
back to the plain net (student_infer_with_fallback).

Recipe: BCE on soft teacher probabilities, Adam (lr 1e-3, betas 0.9 / 0.999,
eps 1e-8), batches of 16 patches of 128 x 128 drawn uniformly over (volume,
slice, origin) with origins in [3, side - 131], targets = the teacher map
cropped to the student's centred 122 x 122 output (the teacher's receptive
radius is 12, the student's 6). Only argument marshalling and the seeded draw
of patch origins happen here; the gather and every arithmetic step run in the
library's kernels.
"""
from __future__ import annotations

import time

import numpy as np

from . import (STUDENT_R, Net, Student, cnn_infer, student_create, student_gather, student_infer,
               student_infer_with_fallback, student_train_step)


def teacher_maps(teacher: Net, volumes, stream=None):
    """Dense teacher probabilities for every volume (device tensors)."""
    return [cnn_infer(teacher, v, stream=stream) for v in volumes]


def sample_batch(rng: np.random.Generator, volumes, maps, teacher_R: int, batch: int = 16,
                 patch: int = 128, out=None, stream=None):
    """Seeded patch draw: (patches uint8 B x P x P, targets float32 B x (P-6) x (P-6)),
    gathered on the device by the library (student_gather) into `out` if given."""
    import torch
    m = (teacher_R - STUDENT_R) // 2  # centring offset between the two output frames
    Z, H, W = volumes[0].shape
    v = rng.integers(0, len(volumes), size=batch)
    z = rng.integers(0, Z, size=batch)
    y = rng.integers(m, H - patch - m + 1, size=batch)
    x = rng.integers(m, W - patch - m + 1, size=batch)
    if out is None:
        dev = volumes[0].device
        out = (torch.empty((batch, patch, patch), dtype=torch.uint8, device=dev),
               torch.empty((batch, patch - STUDENT_R, patch - STUDENT_R), dtype=torch.float32, device=dev))
    srcs = [(volumes[a], maps[a], b, c, d) for a, b, c, d in zip(v, z, y, x)]
    return student_gather(srcs, patch, teacher_R, out[0], out[1], stream=stream)


def train(student: Student, volumes, maps, teacher_R: int, steps: int, *, batch: int = 16,
          patch: int = 128, lr: float = 1e-3, seed: int = 0, log_every: int = 0, log=None,
          stream=None):
    """Run `steps` Adam steps; returns the per-step loss tensor (device, FP64)."""
    import torch
    rng = np.random.default_rng(seed)
    dev = volumes[0].device
    losses = torch.empty(steps, dtype=torch.float64, device=dev)
    gnorms = torch.empty(steps, dtype=torch.float64, device=dev)
    t0 = time.perf_counter()
    bufs = None
    for it in range(steps):
        # two batch buffers in turn: the gather of step it+1 may run while step it reads its own
        if bufs is None:
            bufs = [(torch.empty((batch, patch, patch), dtype=torch.uint8, device=dev),
                     torch.empty((batch, patch - STUDENT_R, patch - STUDENT_R), dtype=torch.float32, device=dev))
                    for _ in range(2)]
        pt, tt = sample_batch(rng, volumes, maps, teacher_R, batch, patch, out=bufs[it % 2], stream=stream)
        student_train_step(student, pt, tt, lr=lr, loss_out=losses[it:it + 1],
                           gnorm_out=gnorms[it:it + 1], stream=stream)
        if log and log_every and (it + 1) % log_every == 0:
            torch.cuda.synchronize()
            log("step %d loss %.5f gnorm %.4g (%.1f s)" % (it + 1, losses[it - log_every + 1:it + 1].mean().item(),
                                                          gnorms[it].item(), time.perf_counter() - t0))
    return losses, gnorms


def agreement(a, b) -> float:
    """Fraction of voxels on which the 0.5-threshold decisions (p >= 0.5) agree."""
    return float(((a >= 0.5) == (b >= 0.5)).float().mean().item())


def evaluate(student: Student, teacher: Net, volume, teacher_map, *, tau: float = 0.01,
             tile: int = 512, n_samples: int = 4, seed: int = 0, stream=None):
    """Raw and post-fallback agreement with the teacher map, and the fallback rate."""
    import torch
    R = teacher.R
    m = (R - STUDENT_R) // 2
    raw = student_infer(student, volume, stream=stream)[:, m:raw_crop(volume.shape[1], R, m),
                                                        m:raw_crop(volume.shape[2], R, m)]
    out, stats = student_infer_with_fallback(student, teacher, volume, tau=tau, tile=tile,
                                             n_samples=n_samples, seed=seed, stream=stream)
    torch.cuda.synchronize()
    flagged, total = stats.tolist()
    return {"raw_agreement": agreement(raw, teacher_map), "agreement": agreement(out, teacher_map),
            "fallback_tiles": flagged, "tiles": total, "fallback_rate": flagged / max(1, total)}, out, stats


def raw_crop(side: int, R: int, m: int) -> int:
    # student output has side - 6 columns; the teacher frame keeps [m, m + side - R)
    return m + side - R
