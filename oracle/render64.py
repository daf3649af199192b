"""FP64 brute-force front-to-back compositing, one pixel at a time, no tiles.

The 3DGS image model the paper renders with (Sec. 3.3): for pixel p with
centre (i + 0.5, j + 0.5), the candidate list is every visible Gaussian whose
FP32 pixel box contains p, ordered by (depth bits, Gaussian index).  Walking
it front to back with transmittance T = 1 and colour C = 0:

    alpha = min(0.99, o * exp(-(a dx^2 + c dy^2)/2 - b dx dy)),  d = p - mu'
    alpha < 1/255                 -> skip this Gaussian
    T (1 - alpha) < 1e-4          -> stop before compositing it
    otherwise C += rgb alpha T,  T <- T (1 - alpha)

and the pixel's value is C + T bg.  Besides the image the oracle reports the
final transmittance, the number of composited Gaussians, the last one, and an
"ambiguous" flag for pixels where a discrete decision sits so close to its
threshold that FP32 and FP64 evaluations may legitimately disagree
(|alpha_raw - 1/255| <= 1e-5/255, |T(1-alpha) - 1e-4| <= 1e-8, or
|alpha_raw - 0.99| <= 0.99e-6).

``render_view`` evaluates the definition for all pixels of a window at once by
walking the (pixel-independent) sorted order and updating every pixel of each
Gaussian's box; this keeps each pixel's own sequence of operations exactly as
above.  ``render_pixel`` is the same definition written as a literal per-pixel
loop and pins the vectorised form.

Parity status: pinned (closed-form single and two-Gaussian images, the
three-layer alpha = 0.95 stack, the telescoping identity sum w + T = 1,
white-colour identity, permutation and projective-scale invariance).
"""
from __future__ import annotations

import numpy as np
import torch

from .project64 import project_view, to_params64
from .spec32 import spec32

ALPHA_MIN = 1.0 / 255.0
ALPHA_MAX = 0.99
T_MIN = 1e-4
AMB_ALPHA_MIN = 1e-5 * ALPHA_MIN
AMB_T = 1e-4 * T_MIN
AMB_CAP = 1e-6 * ALPHA_MAX


def _f32_arrays(p64):
    return {k: v.detach().numpy().astype(np.float32) for k, v in p64.items()}


def view_setup(scene_arrays, sh_degree, cam, p64=None, tile_size=16, index_filter=None, pose=None):
    """Spec decisions, sorted visible list and FP64 projection of one view.

    pose: optional FP64 (R, t) replacing the camera's in the projected values
    only; the FP32 decisions stay those of the camera itself."""
    if p64 is None:
        p64 = to_params64(scene_arrays)
    a32 = _f32_arrays(p64)
    spec = spec32(a32["mean"], a32["log_scale"], a32["quat"], cam, tile_size)
    vis = np.nonzero(spec["visible"])[0]
    if index_filter is not None:
        vis = vis[index_filter(spec, vis)]
    order = vis[np.lexsort((vis, spec["zbits"][vis]))]
    with torch.no_grad():
        proj = project_view(p64, sh_degree, cam, index=order, pose=pose) if len(order) else None
    pj = {k: v.numpy() for k, v in proj.items()} if proj is not None else None
    return spec, order, pj


def render_view(scene_arrays, sh_degree, cam, bg=(0.0, 0.0, 0.0), window=None, p64=None,
                record=False, pose=None):
    """Render one view (or the pixel window (x0, x1, y0, y1), half-open).

    Returns dict: image [3,h,w], T [h,w], count [h,w], last [h,w] (Gaussian
    index, -1 if none), ambiguous [h,w], wsum [h,w] (sum of alpha*T), capped
    [h,w] (composited entries whose o G exceeded the 0.99 cap), and with
    ``record`` the composited entries (pixel flat index, Gaussian) in order.
    """
    W, H = int(cam.width), int(cam.height)
    x0, x1, y0, y1 = window if window is not None else (0, W, 0, H)
    w, h = x1 - x0, y1 - y0

    def in_window(spec, vis):
        i0, i1, j0, j1 = (b[vis] for b in spec["box"])
        return (i1 >= x0) & (i0 < x1) & (j1 >= y0) & (j0 < y1)

    spec, order, pj = view_setup(scene_arrays, sh_degree, cam, p64=p64, index_filter=in_window, pose=pose)
    bg = np.asarray(bg, dtype=np.float64)
    C = np.zeros((3, h, w))
    T = np.ones((h, w))
    wsum = np.zeros((h, w))
    count = np.zeros((h, w), dtype=np.int64)
    capped = np.zeros((h, w), dtype=np.int64)
    last = np.full((h, w), -1, dtype=np.int64)
    done = np.zeros((h, w), dtype=bool)
    amb = np.zeros((h, w), dtype=bool)
    rec_pix, rec_g = [], []
    pix_index = np.arange(h * w).reshape(h, w)

    i0a, i1a, j0a, j1a = spec["box"]
    for k, g in enumerate(order):
        bi0, bi1 = max(int(i0a[g]), x0), min(int(i1a[g]), x1 - 1)
        bj0, bj1 = max(int(j0a[g]), y0), min(int(j1a[g]), y1 - 1)
        if bi0 > bi1 or bj0 > bj1:
            continue
        sl = (slice(bj0 - y0, bj1 - y0 + 1), slice(bi0 - x0, bi1 - x0 + 1))
        act = ~done[sl]
        if not act.any():
            continue
        mx, my = pj["mu2"][k]
        a, b, c = pj["conic"][k]
        dx = (np.arange(bi0, bi1 + 1) + 0.5 - mx)[None, :]
        dy = (np.arange(bj0, bj1 + 1) + 0.5 - my)[:, None]
        power = -0.5 * (a * dx * dx + c * dy * dy) - b * dx * dy
        raw = pj["opacity"][k] * np.exp(power)
        alpha = np.minimum(ALPHA_MAX, raw)
        contrib = act & (alpha >= ALPHA_MIN)
        Tp = T[sl]
        Tn = Tp * (1.0 - alpha)
        stop = contrib & (Tn < T_MIN)
        comp = contrib & ~stop
        amb[sl] |= act & ((np.abs(raw - ALPHA_MIN) <= AMB_ALPHA_MIN) | (np.abs(raw - ALPHA_MAX) <= AMB_CAP))
        amb[sl] |= contrib & (np.abs(Tn - T_MIN) <= AMB_T)
        wgt = np.where(comp, alpha * Tp, 0.0)
        C[:, sl[0], sl[1]] += wgt[None] * pj["rgb"][k][:, None, None]
        wsum[sl] += wgt
        T[sl] = np.where(comp, Tn, Tp)
        count[sl] += comp
        capped[sl] += comp & (raw > ALPHA_MAX)
        last[sl] = np.where(comp, g, last[sl])
        done[sl] |= stop
        if record and comp.any():
            rec_pix.append(pix_index[sl][comp])
            rec_g.append(np.full(int(comp.sum()), g, dtype=np.int64))

    out = dict(image=C + T[None] * bg[:, None, None], T=T, count=count, last=last,
               ambiguous=amb, wsum=wsum, capped=capped, window=(x0, x1, y0, y1))
    if record:
        if rec_pix:
            pix = np.concatenate(rec_pix)
            gg = np.concatenate(rec_g)
            srt = np.argsort(pix, kind="stable")
            out["entries"] = (pix[srt], gg[srt])
        else:
            out["entries"] = (np.zeros(0, np.int64), np.zeros(0, np.int64))
    return out


def render(scene, cams, bg=(0.0, 0.0, 0.0)):
    """All views of a scene (a workloads.Scene); list of render_view dicts."""
    arrays = scene.arrays()
    p64 = to_params64(arrays)
    return [render_view(arrays, scene.sh_degree, cam, bg=bg, p64=p64) for cam in cams]


def render_pixels(scene_arrays, sh_degree, cam, pixels, bg=(0.0, 0.0, 0.0), setup=None):
    """``render_pixel`` for a list of (i, j) pixels, sharing one setup."""
    setup = setup if setup is not None else view_setup(scene_arrays, sh_degree, cam)
    spec, order, _ = setup
    i0, i1, j0, j1 = (b[order] for b in spec["box"])
    out = []
    for (i, j) in pixels:
        ks = np.nonzero((i0 <= i) & (i <= i1) & (j0 <= j) & (j <= j1))[0]
        out.append(render_pixel(scene_arrays, sh_degree, cam, i, j, bg=bg, setup=setup, candidates=ks))
    return out


def render_pixel(scene_arrays, sh_degree, cam, i, j, bg=(0.0, 0.0, 0.0), setup=None, candidates=None):
    """The definition as a literal loop for the single pixel (i, j).
    ``candidates`` optionally restricts the walk to these positions of the
    sorted order (those whose box contains the pixel); the box test below
    still applies."""
    spec, order, pj = setup if setup is not None else view_setup(scene_arrays, sh_degree, cam)
    i0, i1, j0, j1 = spec["box"]
    T, C, count, last, amb = 1.0, np.zeros(3), 0, -1, False
    px, py = i + 0.5, j + 0.5
    walk = range(len(order)) if candidates is None else candidates
    for k in walk:
        g = order[k]
        if not (i0[g] <= i <= i1[g] and j0[g] <= j <= j1[g]):
            continue
        dx = px - pj["mu2"][k][0]
        dy = py - pj["mu2"][k][1]
        a, b, c = pj["conic"][k]
        raw = pj["opacity"][k] * np.exp(-0.5 * (a * dx * dx + c * dy * dy) - b * dx * dy)
        alpha = min(ALPHA_MAX, raw)
        if abs(raw - ALPHA_MIN) <= AMB_ALPHA_MIN or abs(raw - ALPHA_MAX) <= AMB_CAP:
            amb = True
        if alpha < ALPHA_MIN:
            continue
        Tn = T * (1.0 - alpha)
        if abs(Tn - T_MIN) <= AMB_T:
            amb = True
        if Tn < T_MIN:
            break
        C = C + (alpha * T) * pj["rgb"][k]
        T = Tn
        count += 1
        last = int(g)
    return dict(color=C + T * np.asarray(bg, dtype=np.float64), T=T, count=count, last=last, ambiguous=amb)
