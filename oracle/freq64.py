"""Frequency-based scheduling of the optimisation (Sec. 3.3, "Frequency-based
Scheduling", Eqs. 9-12), in FP64 NumPy (test infrastructure: only the tests,
the smoke check and the CPU baseline use it).

* Frequency significance (Eqs. 10-11): X(I) = sum over all frequency bins
  (i, j) of || DFT(I)(i, j) ||_2, the unnormalised 2D DFT of each colour
  channel, the 2-norm taken over the three channels' complex values at the
  bin.  np.fft.fft2 in FP64 is the DFT.
* Ratios (Eqs. 9 and 12): r = X(I) / X(I~) for the ground truth I and the
  render I~; r' = X(I^n) / X(I~) for the ground truth downsampled by the
  current factor n.
* Level of detail: I^n is the n x n box average of I (the remainder rows and
  columns dropped); if r' < tau_f the ground-truth resolution is raised by one
  level (level index - 1, index 0 being full resolution).
* Frame sampling: frames are drawn with probability proportional to r.  The
  random numbers are inputs: pick b is the first frame f whose inclusive
  prefix sum of the weights exceeds u_b times their total.  The weights are r
  capped at FLT_MAX / (2F) (so that F of them cannot overflow; NaN -> 0) and
  summed sequentially in float32, the precision the decision is taken in on
  both sides.

Parity status: X pinned by closed forms (constant image, a single pixel, a
pure cosine), by a brute-force O(N^2) DFT on small images, and by the
invariance under circular shifts; the downsampling by its definition on small
images and mean preservation; the schedule by hand-built cases.
"""
from __future__ import annotations

import numpy as np

TAU_F = 2.0  # Sec. 4 implementation details


def significance(img) -> float:
    """X(I) of one planar [3, H, W] image (Eq. 10)."""
    img = np.asarray(img, np.float64)
    F = np.fft.fft2(img, axes=(1, 2))
    return float(np.sqrt((F.real ** 2 + F.imag ** 2).sum(axis=0)).sum())


def downsample(img, n: int):
    """I^n: mean over n x n blocks of a planar [C, H, W] image, floor(H/n) x floor(W/n)."""
    img = np.asarray(img, np.float64)
    C, H, W = img.shape
    h, w = H // n, W // n
    return img[:, :h * n, :w * n].reshape(C, h, n, w, n).mean(axis=(2, 4))


def ratios(x_gt, x_gt_level, x_render):
    """(r, r') of Eqs. 9 and 12, in float32 like the inputs."""
    x_gt = np.asarray(x_gt, np.float32)
    x_gt_level = np.asarray(x_gt_level, np.float32)
    x_render = np.asarray(x_render, np.float32)
    with np.errstate(divide="ignore", invalid="ignore"):
        return x_gt / x_render, x_gt_level / x_render


def next_levels(levels, r_prime, tau_f=TAU_F):
    """One level finer (index - 1) where r' < tau_f and the level is not already 0."""
    levels = np.asarray(levels, np.int32).copy()
    raise_ = (np.asarray(r_prime, np.float32) < np.float32(tau_f)) & (levels > 0)
    levels[raise_] -= 1
    return levels


def sample_frames(r, uniforms):
    """Frame index per uniform u in [0, 1), drawn proportionally to r."""
    r = np.asarray(r, np.float32)
    F = len(r)
    cap = np.float32(np.finfo(np.float32).max / np.float32(2 * F))
    w = np.where(np.isnan(r), np.float32(0.0), np.minimum(r, cap)).astype(np.float32)
    w = np.maximum(w, np.float32(0.0))
    cdf = np.zeros(F, np.float32)
    acc = np.float32(0.0)
    for f in range(F):
        acc = np.float32(acc + w[f])
        cdf[f] = acc
    picks = np.zeros(len(uniforms), np.int32)
    for b, u in enumerate(np.asarray(uniforms, np.float32)):
        if not acc > 0:
            picks[b] = min(int(np.float32(u) * np.float32(F)), F - 1)  # no weight: uniform
            continue
        target = np.float32(u * acc)
        f = 0
        while f < F - 1 and not cdf[f] > target:
            f += 1
        picks[b] = f
    return picks
