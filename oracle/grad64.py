"""FP64 gradients of the rendered images by torch autograd.

The paper updates Gaussian parameters by gradients of the photometric loss
through the differentiable renderer (Sec. 3.3, "Optimization").  This module
re-expresses the compositing definition of ``render64`` as a differentiable
torch computation with every discrete decision (visibility, pixel box, depth
order, the 1/255 skip and the 1e-4 stop) held at the value the FP64 forward
pass took, and returns the vector-Jacobian product  sum_pixels dL/dC . C  with
respect to (mean, log_scale, quat, opacity_logit, sh), in the ABI layouts.
The cap alpha = min(0.99, o G) is a torch.clamp, so its gradient is zero where
it is active; the Jacobian guard clamp and the colour clamp likewise.

With ``cam_grads`` it also returns each view's pose gradient dL/d(R_v, t_v)
through the geometry (the SH colour detached from the pose, as the paper
updates cameras).

Parity status: pinned against FP64 central finite differences of ``render64``
(relative 1e-6) in the tests; the pose gradients also against the world
translation and rotation invariances of the image at SH degree 0.
"""
from __future__ import annotations

import numpy as np
import torch

from .project64 import camera64, project_view, to_params64
from .render64 import render_view


def _view_term(p64, scene_arrays, sh_degree, cam, cot, bg, window, pose=None):
    fwd = render_view(scene_arrays, sh_degree, cam, bg=bg, window=window, p64=p64, record=True)
    pix, gg = fwd["entries"]
    if len(pix) == 0:
        return None, fwd
    x0, x1, y0, y1 = fwd["window"]
    w = x1 - x0
    uniq, local = np.unique(gg, return_inverse=True)
    proj = project_view(p64, sh_degree, cam, index=uniq, pose=pose)
    li = torch.from_numpy(local)
    px = torch.from_numpy((pix % w + x0).astype(np.float64) + 0.5)
    py = torch.from_numpy((pix // w + y0).astype(np.float64) + 0.5)
    mu = proj["mu2"][li]
    con = proj["conic"][li]
    dx = px - mu[:, 0]
    dy = py - mu[:, 1]
    power = -0.5 * (con[:, 0] * dx * dx + con[:, 2] * dy * dy) - con[:, 1] * dx * dy
    alpha = torch.clamp(proj["opacity"][li] * torch.exp(power), max=0.99)
    rgb = proj["rgb"][li]

    # entries are grouped by pixel, in compositing order within a pixel
    upix, start, counts = np.unique(pix, return_index=True, return_counts=True)
    P, L = len(upix), int(counts.max())
    row = np.repeat(np.arange(P), counts)
    rank = np.arange(len(pix)) - np.repeat(start, counts)
    flat = torch.from_numpy(row * L + rank)
    one_minus = torch.ones(P * L, dtype=torch.float64).index_put((flat,), 1.0 - alpha).reshape(P, L)
    cp = torch.cumprod(one_minus, dim=1)
    t_excl = torch.cat([torch.ones(P, 1, dtype=torch.float64), cp[:, :-1]], dim=1)
    w_e = alpha * t_excl.reshape(-1)[flat]
    colour = torch.zeros(P, 3, dtype=torch.float64).index_add(0, torch.from_numpy(row), w_e[:, None] * rgb)
    colour = colour + cp[:, -1:] * torch.as_tensor(bg, dtype=torch.float64)[None, :]

    cot_w = np.asarray(cot, dtype=np.float64)[:, y0:y1, x0:x1].reshape(3, -1)[:, upix].T
    return (torch.from_numpy(np.ascontiguousarray(cot_w)) * colour).sum(), fwd


def grad64(scene, cams, cotangents, bg=(0.0, 0.0, 0.0), windows=None, p64=None, cam_grads=False):
    """Gradient of sum_v sum_p cot_v[p] . C_v[p] w.r.t. all Gaussian parameters.

    cotangents: list (per view) of [3,H,W] arrays, e.g. dL/dC of a loss.
    windows: optional list (per view) of (x0, x1, y0, y1) pixel windows outside
    which the cotangent is taken as zero.
    cam_grads: also differentiate with respect to each view's pose (the
    paper updates camera parameters jointly with the Gaussians, with the SH
    colour detached from that update, Sec. 3.3): grads["cam"] [V,12] holds
    dL/dR (row-major, R a general 3x3 matrix) then dL/dt of x_c = R mu + t,
    through the geometry only, with the decisions held as above.
    Returns dict of float64 numpy arrays in the ABI layouts.
    """
    arrays = scene.arrays()
    if p64 is None:
        p64 = to_params64(arrays, requires_grad=True)
    poses = []
    total = None
    for v, cam in enumerate(cams):
        win = windows[v] if windows is not None else None
        pose = None
        if cam_grads:
            R0, t0 = camera64(cam)[:2]
            pose = (R0.clone().requires_grad_(True), t0.clone().requires_grad_(True))
            poses.append(pose)
        term, _ = _view_term(p64, arrays, scene.sh_degree, cam, cotangents[v], bg, win, pose=pose)
        if term is not None:
            total = term if total is None else total + term
    grads = {}
    if total is not None:
        total.backward()
    for k, t in p64.items():
        grads[k] = t.grad.numpy().copy() if t.grad is not None else np.zeros(t.shape)
    if cam_grads:
        cg = np.zeros((len(cams), 12))
        for v, (R, t) in enumerate(poses):
            if R.grad is not None:
                cg[v, :9] = R.grad.numpy().reshape(-1)
            if t.grad is not None:
                cg[v, 9:] = t.grad.numpy()
        grads["cam"] = cg
    return grads


def vjp_value(scene_arrays, sh_degree, cams, cotangents, p64, bg=(0.0, 0.0, 0.0), windows=None, poses=None):
    """sum_v sum_p cot . C evaluated by the FP64 forward definition (no autograd).

    poses: optional per-view FP64 (R, t) (or None) replacing the camera's pose
    in the geometry (the SH direction keeps the camera's own)."""
    total = 0.0
    sig = []
    for v, cam in enumerate(cams):
        win = windows[v] if windows is not None else None
        pose = poses[v] if poses is not None else None
        fwd = render_view(scene_arrays, sh_degree, cam, bg=bg, window=win, p64=p64, record=True, pose=pose)
        x0, x1, y0, y1 = fwd["window"]
        total += float((np.asarray(cotangents[v], np.float64)[:, y0:y1, x0:x1] * fwd["image"]).sum())
        sig.append((fwd["entries"][0].tobytes(), fwd["entries"][1].tobytes()))
    return total, sig
