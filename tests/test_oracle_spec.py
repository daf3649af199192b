"""Pins of the FP32 binning rules (oracle/spec32.py) against FP64 truth and
against the independent torch projection (oracle/project64.py)."""
import math

import numpy as np
import torch

from oracle.project64 import project_view, to_params64
from oracle.spec32 import bexp32, spec32
from workloads import make_config


def _ulp_err(y32, y64):
    y32 = np.asarray(y32, np.float64)
    ulp = np.spacing(np.abs(y64).astype(np.float32)).astype(np.float64)
    return np.abs(y32 - y64) / ulp


def test_bexp32_within_two_ulp():
    rng = np.random.default_rng(0)
    x = np.concatenate([np.linspace(-86.0, 88.0, 200001), rng.uniform(-10, 5, 100000)]).astype(np.float32)
    y = bexp32(x)
    ref = np.exp(x.astype(np.float64))
    assert _ulp_err(y, ref).max() <= 2.0
    assert bexp32(np.float32(0.0)) == np.float32(1.0)
    assert bexp32(np.float32(1.0)) == np.float32(math.e)  # e rounds to the float32 nearest e


def test_bexp32_special_values():
    x = np.array([np.nan, np.inf, -np.inf, 88.5, -86.5, 88.0, -86.0], np.float32)
    y = bexp32(x)
    assert np.isnan(y[0]) and y[1] == np.inf and y[2] == 0.0 and y[3] == np.inf and y[4] == 0.0
    assert np.isfinite(y[5]) and y[5] > 1e38 and y[6] > 0 and np.isfinite(y[6])


def test_bexp32_deterministic_bits():
    x = np.random.default_rng(1).uniform(-20, 20, 50000).astype(np.float32)
    assert np.array_equal(bexp32(x).view(np.uint32), bexp32(x.copy()).view(np.uint32))


def _truth64(scene, cam):
    """The spec's continuous quantities recomputed in float64 with numpy."""
    R = np.asarray(cam.R, np.float64)
    t = np.asarray(cam.t, np.float64)
    X = scene.mean.astype(np.float64)
    xc = R @ X + t[:, None]
    xz, yz = xc[0] / xc[2], xc[1] / xc[2]
    u = cam.fx * xz + cam.cx
    v = cam.fy * yz + cam.cy
    return xc[2], u, v


def test_spec_continuous_values_match_fp64():
    scene, cams = make_config(2, scale=0.02)
    cam = cams[0]
    s = spec32(scene.mean, scene.log_scale, scene.quat, cam, 16)
    z64, u64, v64 = _truth64(scene, cam)
    vis = s["visible"]
    assert vis.sum() > 1000
    assert np.abs(s["zc"][vis] - z64[vis]).max() <= 4e-7 * np.abs(z64[vis]).max()
    assert np.abs(s["u"][vis] - u64[vis]).max() < 2e-3
    assert np.abs(s["v"][vis] - v64[vis]).max() < 2e-3
    # diagonal of the dilated covariance: spec32 (float32, hand-ordered) vs the
    # torch float64 projection (matrix products) -- two independent codes.
    idx = np.nonzero(vis)[0]
    pr = project_view(to_params64(scene.arrays()), scene.sh_degree, cam, index=idx)
    cov = pr["cov2"].numpy()
    assert np.abs(s["sxx"][idx] / cov[:, 0] - 1).max() < 2e-5
    assert np.abs(s["syy"][idx] / cov[:, 2] - 1).max() < 2e-5
    hx64 = np.sqrt(11.0826 * cov[:, 0])
    # integer boxes agree with the FP64 ones wherever the FP64 value is not
    # within 1e-3 px of a rounding boundary
    lo64 = u64[idx] - hx64 - 0.5
    safe = np.abs(lo64 - np.round(lo64)) > 1e-3
    i0_64 = np.clip(np.ceil(lo64), 0, cam.width - 1)
    assert np.array_equal(s["box"][0][idx][safe], i0_64[safe].astype(np.int32))


def test_spec_culls_degenerate_inputs():
    scene, cams = make_config(1, scale=0.01)
    m, ls, q = scene.mean.copy(), scene.log_scale.copy(), scene.quat.copy()
    n = m.shape[1]
    assert n >= 12
    q[:, 0] = 0.0                      # zero quaternion
    m[2, 1] = 0.2                      # on the near plane
    m[2, 2] = -3.0                     # behind the camera
    m[0, 3] = np.nan                   # NaN position
    ls[1, 4] = np.inf                  # infinite scale
    q[2, 5] = np.nan                   # NaN rotation
    m[0, 6] = 1e6                      # far outside the image
    s = spec32(m, ls, q, cams[0], 16)
    assert not s["visible"][:7].any()
    assert s["zbits"][:7].max() == 0


def test_spec_box_contains_every_pixel_above_threshold():
    """No pixel outside the FP32 box can reach alpha >= 1/255 (K >= 2 ln 255),
    up to the rounding of the box itself."""
    scene, cams = make_config(1)
    cam = cams[0]
    s = spec32(scene.mean, scene.log_scale, scene.quat, cam, 16)
    idx = np.nonzero(s["visible"])[0]
    pr = project_view(to_params64(scene.arrays()), 0, cam, index=idx)
    mu, con = pr["mu2"].numpy(), pr["conic"].numpy()
    jj, ii = np.mgrid[0:cam.height, 0:cam.width]
    px, py = ii.ravel() + 0.5, jj.ravel() + 0.5
    worst = 0.0
    for k, g in enumerate(idx[:400]):
        dx, dy = px - mu[k, 0], py - mu[k, 1]
        G = np.exp(-0.5 * (con[k, 0] * dx * dx + con[k, 2] * dy * dy) - con[k, 1] * dx * dy)
        i0, i1, j0, j1 = (b[g] for b in s["box"])
        inside = (ii.ravel() >= i0) & (ii.ravel() <= i1) & (jj.ravel() >= j0) & (jj.ravel() <= j1)
        if (~inside).any():
            worst = max(worst, G[~inside].max())
    assert worst < (1.0 / 255.0) * (1 + 1e-4)


def test_spec_is_deterministic():
    scene, cams = make_config(3, scale=0.01)
    a = spec32(scene.mean, scene.log_scale, scene.quat, cams[2], 16)
    b = spec32(scene.mean.copy(), scene.log_scale.copy(), scene.quat.copy(), cams[2], 16)
    for k in ("visible", "zbits"):
        assert np.array_equal(a[k], b[k])
    for x, y in zip(a["box"], b["box"]):
        assert np.array_equal(x, y)
