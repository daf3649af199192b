"""LoG-based insertion of new Gaussians (Sec. 3.2, "Redundancy-free Gaussian
Sampling", Eqs. 4-6), in FP64 NumPy (test infrastructure: only the tests,
the smoke check and the CPU baseline use it).

* Kernel.  The Laplacian of a Gaussian of standard deviation sigma, sampled
  on offsets -R..R per axis, R = ceil(3 sigma), and written as the separable
  sum K(x, y) = h(x) g(y) + g(x) h(y) (the Laplacian of G(x) G(y)), with
  g = the sampled 1D Gaussian normalised to sum 1 and h = the sampled second
  derivative (x^2 - sigma^2) / sigma^4 g(x), shifted to sum 0 and scaled to
  second moment sum x^2 h(x) = 2, so that K of a linear image is 0 and of
  x^2 + y^2 is exactly 4 (as for the continuous operator).
* Response (Eq. 5).  L_c = K * I_c per colour channel, a plain 2D
  convolution with the image's border pixels replicated outward;
  P(I) = min(||(L_r, L_g, L_b)||_2, 1) per pixel.
* Insertion (Eq. 4).  P_a = max(P(I) - P(I~), 0) for the ground truth I and
  the render I~; a pixel inserts a Gaussian when P_a > tau_a (0.2, Sec. 4).
* Scale (Eq. 6).  S = d / (2 sqrt(P(I)) f) with f = fx and d the distance
  from the new Gaussian's centre to the camera: the centre is the pixel
  centre back-projected to the depth map's z-depth,
  x_c = z ((u + 0.5 - cx) / fx, (v + 0.5 - cy) / fy, 1), x_w = R^T (x_c - t),
  d = |x_c|.
* The inserted pixels are listed in ascending pixel index (row-major).

Parity status: pinned by closed forms of the operator (zero on constant and
linear images, 4 on x^2 + y^2, the kernel's sums and symmetry), by a
circular convolution through the FFT on periodic images, by the clamp and
threshold semantics on hand-built cases, and by projecting the back-projected
centres with the renderer's own projection.
"""
from __future__ import annotations

import math

import numpy as np

TAU_A = 0.2  # Sec. 4 implementation details
SIGMA = 1.0  # the paper leaves sigma open


def log_kernels(sigma=SIGMA):
    """(g, h, R): the normalised 1D Gaussian and second-derivative taps."""
    R = int(math.ceil(3.0 * sigma))
    x = np.arange(-R, R + 1, dtype=np.float64)
    g = np.exp(-x * x / (2.0 * sigma * sigma))
    g /= g.sum()
    h = (x * x - sigma * sigma) / sigma ** 4 * g
    h -= h.mean()
    h *= 2.0 / (x * x * h).sum()
    return g, h, R


def log_kernel_2d(sigma=SIGMA):
    g, h, R = log_kernels(sigma)
    return np.outer(h, g) + np.outer(g, h), R  # [y offset, x offset]


def log_response(img, sigma=SIGMA):
    """K * I for a planar [C, H, W] image, borders replicated."""
    img = np.asarray(img, np.float64)
    K, R = log_kernel_2d(sigma)
    C, H, W = img.shape
    pad = np.pad(img, ((0, 0), (R, R), (R, R)), mode="edge")
    out = np.zeros_like(img)
    for dy in range(-R, R + 1):
        for dx in range(-R, R + 1):
            # out(v, u) += K(dy, dx) I(v - dy, u - dx)
            out += K[dy + R, dx + R] * pad[:, R - dy:R - dy + H, R - dx:R - dx + W]
    return out


def probability(img, sigma=SIGMA):
    """P(I) per pixel [H, W] (Eq. 5)."""
    L = log_response(img, sigma)
    return np.minimum(np.sqrt((L * L).sum(axis=0)), 1.0)


def insert(gt, render, depth, cam, sigma=SIGMA, tau_a=TAU_A, amb_eps=1e-5):
    """One view: dict(p_gt, p_render, p_a [H, W], mask, ambiguous [H, W],
    pix (ascending flat indices), scale [n], mean [n, 3])."""
    p_gt = probability(gt, sigma)
    p_r = probability(render, sigma)
    p_a = np.maximum(p_gt - p_r, 0.0)
    mask = p_a > tau_a
    ambiguous = np.abs(p_a - tau_a) <= amb_eps
    H, W = p_gt.shape
    pix = np.nonzero(mask.reshape(-1))[0]
    v, u = pix // W, pix % W
    z = np.asarray(depth, np.float64).reshape(-1)[pix]
    fx, fy = float(np.float32(cam.fx)), float(np.float32(cam.fy))
    cx, cy = float(np.float32(cam.cx)), float(np.float32(cam.cy))
    xc = np.stack([z * (u + 0.5 - cx) / fx, z * (v + 0.5 - cy) / fy, z], axis=1)
    d = np.linalg.norm(xc, axis=1)
    scale = d / (2.0 * np.sqrt(p_gt.reshape(-1)[pix]) * fx)
    R = np.asarray(cam.R, np.float32).astype(np.float64).reshape(3, 3)
    t = np.asarray(cam.t, np.float32).astype(np.float64).reshape(3)
    mean = (xc - t) @ R  # R^T (x_c - t), row-wise
    return dict(p_gt=p_gt, p_render=p_r, p_a=p_a, mask=mask, ambiguous=ambiguous, pix=pix, scale=scale, mean=mean)
