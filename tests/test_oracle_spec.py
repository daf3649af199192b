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


def _box64(scene, cam):
    """The spec's pixel box recomputed in FP64: the bounding box of the
    support ellipse d^2 <= 11.0826 around the projected mean (pixel i centred
    at i + 1/2), with the dilated covariance from the torch projection.
    Returns (z, bounds before clamping, the value each bound rounds)."""
    z64, u64, v64 = _truth64(scene, cam)
    pr = project_view(to_params64(scene.arrays()), scene.sh_degree, cam)
    cov = pr["cov2"].numpy()
    with np.errstate(all="ignore"):
        hx = np.sqrt(11.0826 * cov[:, 0])
        hy = np.sqrt(11.0826 * cov[:, 2])
    raw = (u64 - hx - 0.5, u64 + hx - 0.5, v64 - hy - 0.5, v64 + hy - 0.5)
    b = (np.ceil(raw[0]), np.floor(raw[1]), np.ceil(raw[2]), np.floor(raw[3]))
    return z64, b, raw


def test_spec_box_all_bounds_and_tile_rect_match_fp64():
    """All four box bounds, the visibility decision and the tile rectangle at
    8, 16 and 32 px equal their FP64 values on every Gaussian whose FP64
    bounds are not within 1e-3 px of a rounding boundary (and whose depth is
    not within 1e-6 of the near plane), over posed rig views and a full-HD
    view.  A box one pixel too large (or too small) on either side, or a tile
    rectangle off by one, fails."""
    checked = 0
    for cfg, scale in ((3, 0.01), (2, 0.02)):
        scene, cams = make_config(cfg, scale=scale)
        for cam in cams[:3]:
            W, H = cam.width, cam.height
            z64, b, raw = _box64(scene, cam)
            near = np.abs(z64 - 0.2) <= 1e-6
            safe = ~near
            for r in raw:
                with np.errstate(invalid="ignore"):
                    safe &= np.isfinite(r) & (np.abs(r - np.round(r)) > 1e-3)
            vis64 = (z64 > 0.2) & (b[0] <= b[1]) & (b[2] <= b[3]) & (b[1] >= 0) & (b[0] <= W - 1) & \
                    (b[3] >= 0) & (b[2] <= H - 1)
            i0 = np.clip(b[0], 0, W - 1)
            i1 = np.clip(b[1], 0, W - 1)
            j0 = np.clip(b[2], 0, H - 1)
            j1 = np.clip(b[3], 0, H - 1)
            for ts in (8, 16, 32):
                s = spec32(scene.mean, scene.log_scale, scene.quat, cam, ts)
                assert np.array_equal(s["visible"][safe], vis64[safe])
                sv = safe & vis64
                assert sv.sum() > 100
                for got, want in zip(s["box"], (i0, i1, j0, j1)):
                    assert np.array_equal(got[sv], want[sv].astype(np.int32))
                for got, want in zip(s["rect"], (i0, i1, j0, j1)):
                    assert np.array_equal(got[sv], (want[sv] // ts).astype(np.int32))
                checked += int(sv.sum())
    assert checked > 10000


def test_spec_box_is_not_larger_than_needed():
    """The box is the tight bounding box of the support ellipse d^2 <= 11.0826
    (FP64): at a pixel-centre column x the least d^2 over all y is x^2/S_xx,
    so the box's outermost columns (rows) reach the ellipse and the next ones
    out do not, wherever the edge is not the image border."""
    scene, cams = make_config(1)
    cam = cams[0]
    s = spec32(scene.mean, scene.log_scale, scene.quat, cam, 16)
    idx = np.nonzero(s["visible"])[0]
    pr = project_view(to_params64(scene.arrays()), 0, cam, index=idx)
    mu, cov = pr["mu2"].numpy(), pr["cov2"].numpy()
    k_in, k_out = 11.0826 * (1 + 1e-5), 11.0826 * (1 - 1e-5)
    checked = 0
    for k, g in enumerate(idx[:500]):
        i0, i1, j0, j1 = (int(b[g]) for b in s["box"])
        sxx, syy = cov[k, 0], cov[k, 2]
        x0, x1 = i0 + 0.5 - mu[k, 0], i1 + 0.5 - mu[k, 0]
        y0, y1 = j0 + 0.5 - mu[k, 1], j1 + 0.5 - mu[k, 1]
        if i0 > 0:
            assert x0 * x0 / sxx <= k_in and (x0 - 1) ** 2 / sxx > k_out, (g, "i0")
            checked += 1
        if i1 < cam.width - 1:
            assert x1 * x1 / sxx <= k_in and (x1 + 1) ** 2 / sxx > k_out, (g, "i1")
            checked += 1
        if j0 > 0:
            assert y0 * y0 / syy <= k_in and (y0 - 1) ** 2 / syy > k_out, (g, "j0")
            checked += 1
        if j1 < cam.height - 1:
            assert y1 * y1 / syy <= k_in and (y1 + 1) ** 2 / syy > k_out, (g, "j1")
            checked += 1
    assert checked > 1000
