"""Central finite differences of the FP64 renderer.

Checks ``grad64`` (and through it the GPU adjoint) without trusting autograd:
for one scalar parameter theta of Gaussian g, the functional
Phi(theta) = sum_v sum_p cot_v[p] . C_v[p] is evaluated by the forward
definition at theta +- h, h = h_rel * max(1, |theta|), and
(Phi(theta + h) - Phi(theta - h)) / 2h is returned.  Only pixels in g's pixel
boxes can change, so Phi is evaluated on those windows.  If any discrete
decision (composited entries per pixel, including skips and stops, or g's
visibility) differs between theta - h, theta and theta + h, the difference
quotient is not a derivative and the parameter is reported invalid.
"""
from __future__ import annotations

import numpy as np
import torch

from .grad64 import vjp_value
from .project64 import to_params64
from .spec32 import spec32

PARAM_NAMES = ("mean", "log_scale", "quat", "opacity_logit", "sh")


def _box_of(p64, g, cam):
    a = {k: v.detach().numpy()[..., g:g + 1].astype(np.float32) for k, v in p64.items() if k != "sh"}
    s = spec32(a["mean"], a["log_scale"], a["quat"], cam, 16)
    if not s["visible"][0]:
        return None
    return tuple(int(b[0]) for b in s["box"])


def fd_gradient(scene, cams, cotangents, name, flat_index, h_rel=1e-6, bg=(0.0, 0.0, 0.0)):
    arrays = scene.arrays()
    n = scene.n
    g = int(flat_index) % n
    base = to_params64(arrays)
    theta0 = float(base[name].reshape(-1)[flat_index])
    h = h_rel * max(1.0, abs(theta0))
    states = []
    for delta in (-h, 0.0, h):
        p = {k: v.clone() for k, v in base.items()}
        p[name].reshape(-1)[flat_index] = theta0 + delta
        states.append(p)
    windows = []
    active = []
    for cam in cams:
        boxes = [_box_of(p, g, cam) for p in states]
        if all(b is None for b in boxes):
            windows.append(None)
            active.append(False)
            continue
        if any(b is None for b in boxes):
            return 0.0, False
        windows.append((min(b[0] for b in boxes), max(b[1] for b in boxes) + 1,
                        min(b[2] for b in boxes), max(b[3] for b in boxes) + 1))
        active.append(True)
    if not any(active):
        return 0.0, True
    cams_a = [c for c, a in zip(cams, active) if a]
    cots_a = [c for c, a in zip(cotangents, active) if a]
    wins_a = [w for w, a in zip(windows, active) if a]
    vals, sigs = [], []
    for p in states:
        v, s = vjp_value(arrays, scene.sh_degree, cams_a, cots_a, p, bg=bg, windows=wins_a)
        vals.append(v)
        sigs.append(s)
    valid = sigs[0] == sigs[1] == sigs[2]
    return (vals[2] - vals[0]) / (2.0 * h), valid


def fd_pose_gradient(scene, cams, cotangents, view, entry, h=1e-6, bg=(0.0, 0.0, 0.0)):
    """Central difference of Phi with respect to entry ``entry`` (0..8: R
    row-major, 9..11: t) of view ``view``'s pose, perturbed in FP64 in the
    geometry x_c = R mu + t only (the SH direction and the FP32 binning
    decisions stay those of the camera).  Returns (value, valid) as above."""
    arrays = scene.arrays()
    base = to_params64(arrays)
    cam = cams[view]
    R0 = torch.from_numpy(np.ascontiguousarray(np.asarray(cam.R, np.float32), np.float64).reshape(3, 3))
    t0 = torch.from_numpy(np.ascontiguousarray(np.asarray(cam.t, np.float32), np.float64).reshape(3))
    vals, sigs = [], []
    for delta in (-h, 0.0, h):
        R, t = R0.clone(), t0.clone()
        if entry < 9:
            R.reshape(-1)[entry] += delta
        else:
            t[entry - 9] += delta
        v, s = vjp_value(arrays, scene.sh_degree, [cam], [cotangents[view]], base, bg=bg, poses=[(R, t)])
        vals.append(v)
        sigs.append(s)
    valid = sigs[0] == sigs[1] == sigs[2]
    return (vals[2] - vals[0]) / (2.0 * h), valid
