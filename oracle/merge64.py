"""Per-camera merging of existing Gaussians with the samples of a new camera
(Sec. 3.2, "Redundancy-free Gaussian Sampling", Eqs. 7-8), in FP64 NumPy
(test infrastructure: only the tests, the smoke check and the CPU baseline
use it).

The paper's prose leaves several points open; the reading taken here:
* Reprojection.  An existing Gaussian g is reprojected into camera i:
  x_c = R mu + t, x' = (fx x/z + cx, fy y/z + cy), d' = |x_c|.  Only
  Gaussians in front of the near plane (z > 0.2) whose x' lies in the image
  ([0, W) x [0, H)) take part.
* Bilinear correspondence.  The paper matches the reprojected pixel x' and
  the sampled pixels by bilinear interpolation of P (its Eq. 5).  With pixel
  (i, j) centred at (i + 1/2, j + 1/2), x' has four neighbouring pixel
  centres (i0 + a, j0 + b), a, b in {0, 1}, i0 = floor(u - 1/2), with the
  bilinear weights w_ab = (a ? al : 1 - al) (b ? be : 1 - be),
  al = u - 1/2 - i0, be = v - 1/2 - j0.  g corresponds to the sampled
  (inserting) pixel among those in the image with the largest positive
  weight (the lowest pixel index on equal weights) -- the pixel containing
  x' when it is sampled, a neighbour otherwise -- if the distances agree:
  |d' - d_k| <= tau_d, d_k the distance of sample k's back-projected centre.
  Every other existing Gaussian is left as it is.
* Image-space scales.  s' = kappa S_g fx / d' (Eq. 7) with S_g = exp(mean of
  g's three log-scales); the paper prints kappa = 2, which disagrees with
  Eq. 6 and Eq. 8 (they give S f / d = 1 / (2 sqrt(P))), so kappa is a
  parameter (1 by default).  The new camera's scale at x' is Eq. 8 evaluated
  on P(I_i) interpolated bilinearly at x':  s_i(x') = 1 / (2 sqrt(P(x'))),
  P(x') = sum_ab w_ab P(I_i)(i0 + a, j0 + b), borders replicated.
* Merge.  A group is a sample and the existing Gaussians that correspond to
  it.  Each member is measured against the new camera's scale where it
  sits: rho_g = s'_g / s_i(x'_g) for an existing Gaussian, rho = 1 for the
  sample itself (s_i at its own pixel centre).  Only the member with the
  smallest rho is kept (existing Gaussians win ties, and among them the
  lower index); its colour becomes the mean of the group's colours (the
  existing ones taken as their DC colour Y_0 sh_0 + 1/2, the sample's as its
  ground-truth pixel).
* Depth re-alignment.  The paper re-aligns depths by the merged primitives
  without saying how; here the survivor of a group is moved along camera
  i's ray through its centre to the mean distance of the group's members
  (d' of the existing ones, d_k of the sample): mu <- C + (mu - C) dbar / d,
  C = -R^T t the camera centre.  Every other primitive keeps its centre.

Parity status: pinned by hand-built groups (each rule on its own: winner by
scale, ties, the bilinear neighbour choice and the interpolated scale on
both sides of a pixel border, depth rejection, near plane, non-inserting
pixels, kappa, the re-aligned depth) and by a second, loop-per-Gaussian
writing of the same rules on random scenes.
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


def _neighbours(u, v):
    """The four pixel centres around x' = (u, v): integer columns and rows
    [4, ...] in the order (i0, j0), (i0+1, j0), (i0, j0+1), (i0+1, j0+1)
    (ascending pixel index), and their bilinear weights."""
    a, b = u - 0.5, v - 0.5
    i0, j0 = np.floor(a), np.floor(b)
    al, be = a - i0, b - j0
    ii = np.stack([i0, i0 + 1, i0, i0 + 1]).astype(np.int64)
    jj = np.stack([j0, j0, j0 + 1, j0 + 1]).astype(np.int64)
    w = np.stack([(1 - al) * (1 - be), al * (1 - be), (1 - al) * be, al * be])
    return ii, jj, w, al, be


def merge(mean, log_scale, sh0, cam, samples, p_map, tau_d, kappa=1.0, amb_eps=1e-5):
    """mean, log_scale, sh0: [3, N] (sh0 = the degree-0 SH coefficients).
    samples: dict(pix [K] local pixel indices, ascending; centre [K, 3] world
    centres; colour [K, 3] ground-truth RGB).  p_map: [H, W] P(I_i).
    Returns dict(keep [N] bool, colour [N, 3], keep_new [K] bool,
    colour_new [K, 3], mean [3, N] and mean_new [K, 3] (centres after the
    depth re-alignment), match [N] (sample index or -1), ambiguous_g [N],
    ambiguous_new [K]): a decision within amb_eps (relative) of its
    threshold makes the Gaussian, and its group, ambiguous."""
    R, t, fx, fy, cx, cy, W, H = _cam(cam)
    mean = np.asarray(mean, np.float64)
    N = mean.shape[1]
    K = len(samples["pix"])
    spix = np.asarray(samples["pix"], np.int64)
    P = np.asarray(p_map, np.float64).reshape(H, W)
    xc = R @ mean + t[:, None]
    z = xc[2]
    front = z > NEAR
    zs = np.where(front, z, 1.0)
    u = fx * xc[0] / zs + cx
    v = fy * xc[1] / zs + cy
    inside = front & (u >= 0) & (u < W) & (v >= 0) & (v < H)
    us, vs = np.where(inside, u, 0.5), np.where(inside, v, 0.5)
    ii, jj, w, al, be = _neighbours(us, vs)

    # the sampled neighbour with the largest positive weight
    slot = np.full(W * H, -1, np.int64)
    slot[spix] = np.arange(K)
    in_img = (ii >= 0) & (ii < W) & (jj >= 0) & (jj < H)
    nb_slot = np.where(in_img, slot[np.clip(jj, 0, H - 1) * W + np.clip(ii, 0, W - 1)], -1)
    sampled = in_img & (nb_slot >= 0) & inside[None]
    w_s = np.where(sampled, w, -1.0)
    best = np.argmax(w_s, axis=0)  # the first (lowest pixel index) of equal weights
    w_best = np.take_along_axis(w_s, best[None], 0)[0]
    k_of = np.where(w_best > 0, np.take_along_axis(nb_slot, best[None], 0)[0], -1)

    d_g = np.linalg.norm(xc, axis=0)
    c_new = (R @ np.asarray(samples["centre"], np.float64).reshape(-1, 3).T + t[:, None])
    d_new = np.linalg.norm(c_new, axis=0)
    has = k_of >= 0
    dd = np.where(has, np.abs(d_g - d_new[np.clip(k_of, 0, max(K - 1, 0))] if K else 0.0), np.inf)
    match = np.where(has & (dd <= tau_d), k_of, -1)

    # interpolated P at x' (replicated borders) and the scale ratios
    pc = P[np.clip(jj, 0, H - 1), np.clip(ii, 0, W - 1)]
    p_at = (1 - be) * ((1 - al) * pc[0] + al * pc[1]) + be * ((1 - al) * pc[2] + al * pc[3])
    S = np.exp(np.asarray(log_scale, np.float64).mean(axis=0))
    s_g = kappa * S * fx / d_g
    with np.errstate(divide="ignore", invalid="ignore"):
        rho = s_g * 2.0 * np.sqrt(p_at)  # s'_g / s_i(x'_g)
    col_g = (Y0 * np.asarray(sh0, np.float64) + 0.5).T  # [N, 3]
    col_new = np.asarray(samples["colour"], np.float64).reshape(-1, 3)

    keep = np.ones(N, bool)
    colour = col_g.copy()
    keep_new = np.ones(K, bool)
    colour_new = col_new.copy()
    mean_out = mean.copy()
    mean_new = np.asarray(samples["centre"], np.float64).reshape(-1, 3).copy()
    centre = -(R.T @ t)
    order = np.lexsort((np.arange(N), rho))  # by ratio, then index
    members = [[] for _ in range(K)]
    for g in order:
        if match[g] >= 0:
            members[match[g]].append(g)
    for k in range(K):
        m = members[k]
        if not m:
            continue
        mean_col = (col_new[k] + col_g[m].sum(axis=0)) / (len(m) + 1)
        dbar = (d_new[k] + d_g[m].sum()) / (len(m) + 1)
        first = m[0]
        if rho[first] <= 1.0:
            keep_new[k] = False
            keep[m] = False
            keep[first] = True
            colour[first] = mean_col
            mean_out[:, first] = centre + (mean[:, first] - centre) * (dbar / d_g[first])
        else:
            keep[m] = False
            colour_new[k] = mean_col
            mean_new[k] = centre + (mean_new[k] - centre) * (dbar / d_new[k])

    # decisions within amb_eps of their threshold
    amb_g = np.zeros(N, bool)
    amb_g |= front & ((np.abs(u) <= amb_eps * W) | (np.abs(u - W) <= amb_eps * W) |
                      (np.abs(v) <= amb_eps * H) | (np.abs(v - H) <= amb_eps * H))
    srt = np.sort(np.where(in_img & (nb_slot >= 0), w, -1.0), axis=0)
    amb_g |= inside & has & ((srt[3] - srt[2] <= amb_eps) | (srt[3] <= amb_eps))
    amb_g |= inside & ~has & (srt[3] >= 0) & (srt[3] <= amb_eps)
    amb_g |= np.abs(z - NEAR) <= amb_eps
    amb_g |= has & (np.abs(dd - tau_d) <= amb_eps * np.maximum(1.0, tau_d))
    amb_new = np.zeros(K, bool)
    for k in range(K):
        m = members[k]
        if not m:
            continue
        near_tie = np.abs(rho[m] - 1.0) <= amb_eps
        if len(m) > 1:
            r0 = rho[m[0]]
            near_tie = near_tie | (np.abs(rho[m] - r0) <= amb_eps * r0) & (np.arange(len(m)) > 0)
        if near_tie.any():
            amb_new[k] = True
    for k in np.nonzero(amb_new)[0]:
        amb_g[members[k]] = True
    for g in np.nonzero(amb_g & has)[0]:
        amb_new[k_of[g]] = True
    return dict(keep=keep, colour=colour, keep_new=keep_new, colour_new=colour_new, mean=mean_out,
                mean_new=mean_new, match=match, ambiguous_g=amb_g, ambiguous_new=amb_new)


def merge_loops(mean, log_scale, sh0, cam, samples, p_map, tau_d, kappa=1.0):
    """The same rules written one Gaussian and one sample at a time."""
    R, t, fx, fy, cx, cy, W, H = _cam(cam)
    mean = np.asarray(mean, np.float64)
    log_scale = np.asarray(log_scale, np.float64)
    sh0 = np.asarray(sh0, np.float64)
    P = np.asarray(p_map, np.float64).reshape(H, W)
    N = mean.shape[1]
    pix = [int(p) for p in samples["pix"]]
    K = len(pix)
    where = {p: k for k, p in enumerate(pix)}
    centre = -(R.T @ t)
    groups = {k: [] for k in range(K)}
    for g in range(N):
        xc = R @ mean[:, g] + t
        if not xc[2] > NEAR:
            continue
        u = fx * xc[0] / xc[2] + cx
        v = fy * xc[1] / xc[2] + cy
        if not (0 <= u < W and 0 <= v < H):
            continue
        i0, j0 = math.floor(u - 0.5), math.floor(v - 0.5)
        al, be = u - 0.5 - i0, v - 0.5 - j0
        best, best_w = None, 0.0
        p_at = 0.0
        for b in (0, 1):
            for a in (0, 1):
                wt = (al if a else 1 - al) * (be if b else 1 - be)
                i, j = i0 + a, j0 + b
                p_at += wt * P[min(max(j, 0), H - 1), min(max(i, 0), W - 1)]
                if 0 <= i < W and 0 <= j < H and (j * W + i) in where and wt > best_w:
                    best, best_w = where[j * W + i], wt
        if best is None:
            continue
        d = math.sqrt(xc @ xc)
        cn = R @ np.asarray(samples["centre"][best], np.float64) + t
        if abs(d - math.sqrt(cn @ cn)) > tau_d:
            continue
        s = kappa * math.exp(log_scale[:, g].mean()) * fx / d
        groups[best].append((s / (1.0 / (2.0 * math.sqrt(p_at))), g, d))
    keep = [True] * N
    colour = [Y0 * sh0[:, g] + 0.5 for g in range(N)]
    mean_out = mean.copy()
    keep_new = [True] * K
    colour_new = [np.asarray(samples["colour"][k], np.float64) for k in range(K)]
    mean_new = [np.asarray(samples["centre"][k], np.float64).copy() for k in range(K)]
    for k, mem in groups.items():
        if not mem:
            continue
        mem.sort()
        total = colour_new[k] + sum(Y0 * sh0[:, g] + 0.5 for _, g, _ in mem)
        avg = total / (len(mem) + 1)
        cn = R @ mean_new[k] + t
        d_k = math.sqrt(cn @ cn)
        dbar = (d_k + sum(d for _, _, d in mem)) / (len(mem) + 1)
        for _, g, _ in mem:
            keep[g] = False
        rho, g, d = mem[0]
        if rho <= 1.0:
            keep_new[k] = False
            keep[g] = True
            colour[g] = avg
            mean_out[:, g] = centre + (mean[:, g] - centre) * (dbar / d)
        else:
            colour_new[k] = avg
            mean_new[k] = centre + (mean_new[k] - centre) * (dbar / d_k)
    return dict(keep=np.array(keep), colour=np.array(colour), keep_new=np.array(keep_new),
                colour_new=np.array(colour_new), mean=mean_out, mean_new=np.array(mean_new).reshape(-1, 3))
