"""Pins of the per-camera merge oracle (oracle/merge64.py): hand-built groups
that exercise one rule each, and agreement with the loop-per-Gaussian
writing of the same rules on random scenes."""
import math

import numpy as np
import pytest

from oracle.merge64 import Y0, merge, merge_loops
from tiny_scenes import camera

F, W, H = 100.0, 20, 20


def _on_ray(px, py, z):
    """World point at depth z on the ray through pixel (px, py) of the identity camera."""
    return np.array([z * (px + 0.5 - W / 2) / F, z * (py + 0.5 - H / 2) / F, z])


def _case(existing, sample_pix=((10, 10),), sample_z=(5.0,), p=0.25):
    """existing: list of (centre, image-space scale at kappa 1, colour)."""
    cam = camera(f=F, w=W, h=H)
    mean = np.stack([e[0] for e in existing], 1)
    d = np.linalg.norm(mean, axis=0)
    S = np.array([e[1] for e in existing]) * d / F
    log_scale = np.tile(np.log(S), (3, 1))
    sh0 = (np.stack([e[2] for e in existing], 1) - 0.5) / Y0
    samples = dict(pix=np.array([py * W + px for px, py in sample_pix]),
                   centre=np.stack([_on_ray(px, py, z) for (px, py), z in zip(sample_pix, sample_z)]),
                   colour=np.array([[0.9, 0.1, 0.1]] * len(sample_pix)))
    p_map = np.full((H, W), p)
    return cam, mean, log_scale, sh0, samples, p_map


def test_smaller_existing_gaussian_wins_and_takes_the_mean_colour():
    c0 = np.array([0.1, 0.5, 0.3])
    cam, mean, ls, sh0, smp, pm = _case([(_on_ray(10, 10, 5.0), 0.5, c0)])
    out = merge(mean, ls, sh0, cam, smp, pm, tau_d=1.0)
    assert out["keep"][0] and not out["keep_new"][0]
    assert np.allclose(out["colour"][0], (c0 + [0.9, 0.1, 0.1]) / 2, atol=1e-14)


def test_smaller_sample_wins():
    cam, mean, ls, sh0, smp, pm = _case([(_on_ray(10, 10, 5.2), 2.0, np.array([0.2, 0.2, 0.2]))])
    out = merge(mean, ls, sh0, cam, smp, pm, tau_d=1.0)
    assert not out["keep"][0] and out["keep_new"][0]
    assert np.allclose(out["colour_new"][0], ([0.2, 0.2, 0.2] + np.array([0.9, 0.1, 0.1])) / 2, atol=1e-14)


def test_equal_scales_keep_the_existing_gaussian_with_the_lower_index():
    c = np.array([0.5, 0.5, 0.5])
    # s_new = 1 / (2 sqrt(0.25)) = 1: an existing Gaussian of scale exactly 1 ties and wins
    cam, mean, ls, sh0, smp, pm = _case([(_on_ray(10, 10, 5.0), 1.0, c), (_on_ray(10, 10, 5.0), 1.0, c),
                                         (_on_ray(10, 10, 4.9), 3.0, c)])
    out = merge(mean, ls, sh0, cam, smp, pm, tau_d=1.0)
    assert list(out["keep"]) == [True, False, False] and not out["keep_new"][0]
    assert np.allclose(out["colour"][0], (3 * c + [0.9, 0.1, 0.1]) / 4, atol=1e-14)


def test_depth_discrepancy_near_plane_and_empty_pixels_leave_gaussians_alone():
    c = np.array([0.3, 0.3, 0.3])
    behind = np.array([0.0, 0.0, -1.0])
    cam, mean, ls, sh0, smp, pm = _case([(_on_ray(10, 10, 8.0), 0.1, c),  # 3 m behind the sample: no match
                                         (behind, 0.1, c),                 # behind the camera
                                         (_on_ray(3, 3, 5.0), 0.1, c)])    # a pixel with no sample
    out = merge(mean, ls, sh0, cam, smp, pm, tau_d=1.0)
    assert out["keep"].all() and out["keep_new"][0]
    assert np.allclose(out["colour"], np.tile(c, (3, 1)), atol=1e-14)
    assert list(out["match"]) == [-1, -1, -1]
    # a looser depth bound admits the first one (and it wins by scale)
    out = merge(mean, ls, sh0, cam, smp, pm, tau_d=3.5)
    assert out["match"][0] == 0 and not out["keep_new"][0]


def test_kappa_scales_the_existing_image_space_scale():
    cam, mean, ls, sh0, smp, pm = _case([(_on_ray(10, 10, 5.0), 0.6, np.array([0.5, 0.5, 0.5]))])
    assert not merge(mean, ls, sh0, cam, smp, pm, tau_d=1.0, kappa=1.0)["keep_new"][0]
    assert merge(mean, ls, sh0, cam, smp, pm, tau_d=1.0, kappa=2.0)["keep_new"][0]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_vectorised_and_loop_writings_agree(seed):
    rng = np.random.default_rng(seed)
    R = np.array([[math.cos(0.2), 0, math.sin(0.2)], [0, 1, 0], [-math.sin(0.2), 0, math.cos(0.2)]])
    cam = camera(f=60.0, w=48, h=32, R=R, t=np.array([0.1, 0.0, -0.2]))
    Np, K = 400, 60
    mean = np.stack([rng.uniform(-2, 2, Np), rng.uniform(-1.5, 1.5, Np), rng.uniform(-1, 8, Np)])
    ls = rng.normal(-3.0, 0.5, (3, Np))
    sh0 = rng.normal(0, 1, (3, Np))
    pix = np.sort(rng.choice(48 * 32, K, replace=False))
    z = rng.uniform(2, 7, K)
    u, v = pix % 48 + 0.5, pix // 48 + 0.5
    xc = np.stack([z * (u - 24) / 60, z * (v - 16) / 60, z], 1)
    centre = (xc - np.asarray(cam.t, np.float32).astype(np.float64)) @ np.asarray(cam.R, np.float32).astype(np.float64)
    samples = dict(pix=pix, centre=centre, colour=rng.uniform(0, 1, (K, 3)))
    # place a third of the Gaussians on sampled rays, near the sample's depth
    for g in range(0, Np, 3):
        k = rng.integers(0, K)
        xg = xc[k] * rng.uniform(0.9, 1.1)
        mean[:, g] = (xg - np.asarray(cam.t, np.float32).astype(np.float64)) @ np.asarray(cam.R, np.float32).astype(np.float64)
    p_map = rng.uniform(0.05, 1.0, (32, 48))
    a = merge(mean, ls, sh0, cam, samples, p_map, tau_d=0.3)
    b = merge_loops(mean, ls, sh0, cam, samples, p_map, tau_d=0.3)
    assert (a["match"] >= 0).sum() > 20
    ok_g, ok_n = ~a["ambiguous_g"], ~a["ambiguous_new"]
    assert np.array_equal(a["keep"][ok_g], b["keep"][ok_g])
    assert np.array_equal(a["keep_new"][ok_n], b["keep_new"][ok_n])
    assert np.abs(a["colour"][ok_g] - b["colour"][ok_g]).max() < 1e-12
    assert np.abs(a["colour_new"][ok_n] - b["colour_new"][ok_n]).max() < 1e-12
    assert (~a["keep"]).sum() > 0 and (~a["keep_new"]).sum() > 0
