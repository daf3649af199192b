"""Per-camera merging of existing Gaussians with the samples of a new camera
(Sec. 3.2, "Redundancy-free Gaussian Sampling", Eqs. 7-8), in FP64 NumPy
(test infrastructure: only the tests, the smoke check and the CPU baseline
use it).

The paper's prose leaves several points open; the reading taken here:
* Correspondence.  An existing Gaussian g corresponds to the sampled
  (inserting) pixel of camera i that contains its projection
  x' = (fx x/z + cx, fy y/z + cy) of x_c = R mu + t, if it lies in front of
  the near plane z > 0.2 and the distances to the camera agree:
  |d' - d| <= tau_d, d' = |x_c|, d = |x_c| of the sample's back-projected
  centre.  Every other existing Gaussian is left as it is.
* Image-space scales.  s' = kappa S_g fx / d' (Eq. 7) with S_g = exp(mean of
  g's three log-scales); the paper prints kappa = 2, which disagrees with
  Eq. 6 and Eq. 8 (they give S f / d = 1 / (2 sqrt(P))), so kappa is a
  parameter (1 by default).  The sample's own scale is s = 1 / (2 sqrt(P(I_i)))
  at its pixel (Eq. 8).
* Merge.  Of the group made of a sample and the existing Gaussians that
  correspond to it, only the primitive with the smallest image-space scale
  is kept (existing Gaussians win ties, and among them the lower index);
  its colour becomes the mean of the group's colours, the existing ones
  taken as their DC colour Y_0 sh_0 + 1/2, the sample's as its ground-truth
  pixel.  Positions are not re-aligned (the paper does not say how).

Parity status: pinned by hand-built groups (each rule on its own: winner by
scale, ties, depth rejection, near plane, non-inserting pixels, kappa) and
by a second, loop-per-Gaussian writing of the same rules on random scenes.
"""
from __future__ import annotations

import math

import numpy as np

Y0 = 0.28209479177387814  # 1 / (2 sqrt(pi)), the degree-0 SH basis value
NEAR = 0.2


def _cam(cam):
    R = np.asarray(cam.R, np.float32).astype(np.float64).reshape(3, 3)
    t = np.asarray(cam.t, np.float32).astype(np.float64).reshape(3)
    f = [float(np.float32(v)) for v in (cam.fx, cam.fy, cam.cx, cam.cy)]
    return R, t, f[0], f[1], f[2], f[3], int(cam.width), int(cam.height)


def merge(mean, log_scale, sh0, cam, samples, p_map, tau_d, kappa=1.0, amb_eps=1e-5):
    """mean, log_scale, sh0: [3, N] (sh0 = the degree-0 SH coefficients).
    samples: dict(pix [K] local pixel indices, ascending; centre [K, 3] world
    centres; colour [K, 3] ground-truth RGB).  p_map: [H, W] P(I_i).
    Returns dict(keep [N] bool, colour [N, 3], keep_new [K] bool,
    colour_new [K, 3], match [N] (sample index or -1), ambiguous_g [N],
    ambiguous_new [K])."""
    R, t, fx, fy, cx, cy, W, H = _cam(cam)
    mean = np.asarray(mean, np.float64)
    N = mean.shape[1]
    K = len(samples["pix"])
    xc = R @ mean + t[:, None]
    z = xc[2]
    front = z > NEAR
    zs = np.where(front, z, 1.0)
    u = fx * xc[0] / zs + cx
    v = fy * xc[1] / zs + cy
    iu, iv = np.floor(u), np.floor(v)
    inside = front & (iu >= 0) & (iu < W) & (iv >= 0) & (iv < H)
    pidx = np.where(inside, iv * W + iu, -1).astype(np.int64)
    slot = np.full(W * H, -1, np.int64)
    slot[np.asarray(samples["pix"], np.int64)] = np.arange(K)
    k_of = np.where(inside, slot[np.clip(pidx, 0, W * H - 1)], -1)
    d_g = np.linalg.norm(xc, axis=0)
    c_new = (R @ np.asarray(samples["centre"], np.float64).T + t[:, None])
    d_new = np.linalg.norm(c_new, axis=0)
    has = k_of >= 0
    dd = np.where(has, np.abs(d_g - d_new[np.clip(k_of, 0, max(K - 1, 0))] if K else 0.0), np.inf)
    match = np.where(has & (dd <= tau_d), k_of, -1)
    S = np.exp(np.asarray(log_scale, np.float64).mean(axis=0))
    s_g = kappa * S * fx / d_g
    s_new = 1.0 / (2.0 * np.sqrt(np.asarray(p_map, np.float64).reshape(-1)[np.asarray(samples["pix"], np.int64)]))
    col_g = (Y0 * np.asarray(sh0, np.float64) + 0.5).T  # [N, 3]
    col_new = np.asarray(samples["colour"], np.float64)

    keep = np.ones(N, bool)
    colour = col_g.copy()
    keep_new = np.ones(K, bool)
    colour_new = col_new.copy()
    order = np.lexsort((np.arange(N), s_g))  # by scale, then index
    members = [[] for _ in range(K)]
    for g in order:
        if match[g] >= 0:
            members[match[g]].append(g)
    for k in range(K):
        m = members[k]
        if not m:
            continue
        mean_col = (col_new[k] + col_g[m].sum(axis=0)) / (len(m) + 1)
        best = m[0]
        if s_g[best] <= s_new[k]:
            keep_new[k] = False
            keep[m] = False
            keep[best] = True
            colour[best] = mean_col
        else:
            keep[m] = False
            colour_new[k] = mean_col

    # decisions within amb_eps of their threshold
    amb_g = np.zeros(N, bool)
    frac_u, frac_v = u - iu, v - iv
    amb_g |= front & ((np.minimum(frac_u, 1 - frac_u) <= 1e-4) | (np.minimum(frac_v, 1 - frac_v) <= 1e-4))
    amb_g |= np.abs(z - NEAR) <= amb_eps
    amb_g |= has & (np.abs(dd - tau_d) <= amb_eps * np.maximum(1.0, tau_d))
    amb_new = np.zeros(K, bool)
    for k in range(K):
        m = members[k]
        if not m:
            continue
        near_tie = np.abs(s_g[m] - s_new[k]) <= amb_eps * s_new[k]
        if len(m) > 1:
            srt = np.sort(s_g[m])
            near_tie = near_tie | (np.abs(s_g[m] - srt[0]) <= amb_eps * srt[0]) & (s_g[m] != srt[0])
        if near_tie.any():
            amb_new[k] = True
    for k in np.nonzero(amb_new)[0]:
        amb_g[members[k]] = True
    for g in np.nonzero(amb_g & has)[0]:
        amb_new[k_of[g]] = True
    return dict(keep=keep, colour=colour, keep_new=keep_new, colour_new=colour_new, match=match,
                ambiguous_g=amb_g, ambiguous_new=amb_new)


def merge_loops(mean, log_scale, sh0, cam, samples, p_map, tau_d, kappa=1.0):
    """The same rules written one Gaussian and one sample at a time."""
    R, t, fx, fy, cx, cy, W, H = _cam(cam)
    mean = np.asarray(mean, np.float64)
    log_scale = np.asarray(log_scale, np.float64)
    sh0 = np.asarray(sh0, np.float64)
    N = mean.shape[1]
    pix = [int(p) for p in samples["pix"]]
    K = len(pix)
    where = {p: k for k, p in enumerate(pix)}
    groups = {k: [] for k in range(K)}
    for g in range(N):
        xc = R @ mean[:, g] + t
        if not xc[2] > NEAR:
            continue
        u = fx * xc[0] / xc[2] + cx
        v = fy * xc[1] / xc[2] + cy
        iu, iv = math.floor(u), math.floor(v)
        if not (0 <= iu < W and 0 <= iv < H):
            continue
        k = where.get(iv * W + iu)
        if k is None:
            continue
        cn = R @ np.asarray(samples["centre"][k], np.float64) + t
        if abs(math.sqrt(xc @ xc) - math.sqrt(cn @ cn)) > tau_d:
            continue
        s = kappa * math.exp(log_scale[:, g].mean()) * fx / math.sqrt(xc @ xc)
        groups[k].append((s, g))
    keep = [True] * N
    colour = [Y0 * sh0[:, g] + 0.5 for g in range(N)]
    keep_new = [True] * K
    colour_new = [np.asarray(samples["colour"][k], np.float64) for k in range(K)]
    for k, mem in groups.items():
        if not mem:
            continue
        mem.sort()
        total = colour_new[k] + sum(Y0 * sh0[:, g] + 0.5 for _, g in mem)
        avg = total / (len(mem) + 1)
        s_new = 1.0 / (2.0 * math.sqrt(float(np.asarray(p_map).reshape(-1)[pix[k]])))
        for _, g in mem:
            keep[g] = False
        if mem[0][0] <= s_new:
            keep_new[k] = False
            keep[mem[0][1]] = True
            colour[mem[0][1]] = avg
        else:
            colour_new[k] = avg
    return dict(keep=np.array(keep), colour=np.array(colour), keep_new=np.array(keep_new),
                colour_new=np.array(colour_new))
