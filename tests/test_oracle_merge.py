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
    assert np.abs(a["mean"][:, ok_g] - b["mean"][:, ok_g]).max() < 1e-12
    assert np.abs(a["mean_new"][ok_n] - b["mean_new"][ok_n]).max() < 1e-12
    assert (~a["keep"]).sum() > 0 and (~a["keep_new"]).sum() > 0
    # survivors were moved (and only survivors of groups)
    moved = np.any(a["mean"] != mean, axis=0)
    assert moved.sum() > 0 and not moved[a["match"] < 0].any()


def _at(u, v, z):
    """World point at depth z projecting to the subpixel position (u, v) of the identity camera."""
    return np.array([z * (u - W / 2) / F, z * (v - H / 2) / F, z])


def _border_case(u, sampled, p_vals=None, s_exist=0.8, z_g=5.0, z_s=5.0, col=(0.2, 0.4, 0.6)):
    """One existing Gaussian projecting to (u, 10.5) on the identity camera,
    samples at the pixels (px, 10) for px in ``sampled``; P = 0.25 except
    p_vals {px: P} on row 10."""
    cam = camera(f=F, w=W, h=H)
    mean = _at(u, 10.5, z_g)[:, None]
    d = np.linalg.norm(mean[:, 0])
    log_scale = np.full((3, 1), math.log(s_exist * d / F))
    sh0 = ((np.asarray(col) - 0.5) / Y0)[:, None]
    pix = np.array(sorted(10 * W + px for px in sampled))
    samples = dict(pix=pix, centre=np.stack([_on_ray(p % W, p // W, z_s) for p in pix]),
                   colour=np.array([[0.9, 0.1, 0.1]] * len(pix)))
    p_map = np.full((H, W), 0.25)
    for px, pv in (p_vals or {}).items():
        p_map[10, px] = pv
    return cam, mean, log_scale, sh0, samples, p_map


def test_bilinear_match_takes_the_sampled_neighbour_across_a_pixel_border():
    """x' at u = 10.95 lies in pixel 10, 0.45 px from the centre of pixel 11:
    bilinear weights 0.55 (pixel 10) and 0.45 (pixel 11).  With only pixel 11
    sampled the Gaussian corresponds to it (a floor to the containing pixel
    would find no sample); with both sampled, the heavier pixel 10 wins; at
    u = 11.05 the containing pixel 11 wins; exactly at pixel 10's centre
    pixel 11 has weight 0 and no sample of it is matched (a weight that
    rounding could make positive, so the decision is flagged)."""
    for u, sampled, want in ((10.95, [11], 10 * W + 11), (10.95, [10, 11], 10 * W + 10),
                             (11.05, [10, 11], 10 * W + 11), (10.5, [11], None), (10.5, [9, 11], None)):
        cam, mean, ls, sh0, smp, pm = _border_case(u, sampled, s_exist=0.5)
        out = merge(mean, ls, sh0, cam, smp, pm, tau_d=1.0)
        got = None if out["match"][0] < 0 else int(smp["pix"][out["match"][0]])
        assert got == want, (u, sampled, got)
        assert out["ambiguous_g"][0] == (u == 10.5)


def test_neighbour_outside_the_image_is_not_matched_and_p_replicates_the_border():
    """x' at u = 0.3: the neighbours are column -1 (outside, weight 0.2) and
    column 0 (weight 0.8); P is replicated from column 0, so the interpolated
    scale is column 0's: P = 1 -> s_i = 0.5, and an existing scale of 0.45
    wins, 0.55 loses."""
    for s_exist, wins in ((0.45, True), (0.55, False)):
        cam, mean, ls, sh0, smp, pm = _border_case(0.3, [0], p_vals={0: 1.0}, s_exist=s_exist)
        out = merge(mean, ls, sh0, cam, smp, pm, tau_d=1.0)
        assert out["match"][0] == 0
        assert out["keep"][0] == wins and out["keep_new"][0] == (not wins)


def test_scale_is_compared_with_the_bilinearly_interpolated_p():
    """Pixel 10 has P = 0.25 (s = 1), pixel 11 has P = 1 (s = 1/2).  At
    u = 10.95 (weights 0.55, 0.45) P(x') = 0.55 * 0.25 + 0.45 = 0.5875 and
    s_i(x') = 1 / (2 sqrt(0.5875)) = 0.65233; an existing Gaussian of scale
    0.8 (smaller than pixel 10's own s = 1, the sample it corresponds to)
    loses, one of 0.6 wins."""
    s_i = 1.0 / (2.0 * math.sqrt(0.55 * 0.25 + 0.45 * 1.0))
    assert abs(s_i - 0.652328) < 1e-6
    for s_exist, wins in ((0.8, False), (0.6, True), (s_i * (1 - 1e-3), True), (s_i * (1 + 1e-3), False)):
        cam, mean, ls, sh0, smp, pm = _border_case(10.95, [10], p_vals={11: 1.0}, s_exist=s_exist)
        out = merge(mean, ls, sh0, cam, smp, pm, tau_d=1.0)
        assert out["match"][0] == 0
        assert out["keep"][0] == wins and out["keep_new"][0] == (not wins), s_exist
        assert not out["ambiguous_g"][0] and not out["ambiguous_new"][0]
    # a ratio within 1e-5 of 1 is flagged, not decided
    cam, mean, ls, sh0, smp, pm = _border_case(10.95, [10], p_vals={11: 1.0}, s_exist=s_i * (1 + 1e-7))
    assert merge(mean, ls, sh0, cam, smp, pm, tau_d=1.0)["ambiguous_new"][0]


def test_survivor_is_realigned_to_the_mean_distance_of_its_group():
    """The survivor moves along its own ray from the camera centre to the
    group's mean distance; the losers and unmatched primitives keep their
    centres.  Existing at distance d' (z 5.2) beats the sample at d_k (z 5.0):
    its new distance is (d' + d_k) / 2; the other way round the sample's."""
    cam = camera(f=F, w=W, h=H)
    for s_exist, existing_wins in ((0.5, True), (2.0, False)):
        mean = np.stack([_at(10.7, 10.2, 5.2), _at(3.5, 3.5, 4.0)], 1)
        d = np.linalg.norm(mean, axis=0)
        ls = np.tile(np.log(np.array([s_exist, 1.0]) * d / F), (3, 1))
        sh0 = np.zeros((3, 2))
        smp = dict(pix=np.array([10 * W + 10]), centre=_on_ray(10, 10, 5.0)[None],
                   colour=np.array([[0.9, 0.1, 0.1]]))
        out = merge(mean, ls, sh0, cam, smp, np.full((H, W), 0.25), tau_d=1.0)
        d_k = np.linalg.norm(smp["centre"][0])
        dbar = (d[0] + d_k) / 2
        assert np.array_equal(out["mean"][:, 1], mean[:, 1])
        if existing_wins:
            assert out["keep"][0] and not out["keep_new"][0]
            moved = out["mean"][:, 0]
            assert abs(np.linalg.norm(moved) - dbar) < 1e-12
            assert np.allclose(moved / np.linalg.norm(moved), mean[:, 0] / d[0], atol=1e-15)
            assert np.array_equal(out["mean_new"], smp["centre"])
        else:
            assert not out["keep"][0] and out["keep_new"][0]
            moved = out["mean_new"][0]
            assert abs(np.linalg.norm(moved) - dbar) < 1e-12
            assert np.allclose(moved / np.linalg.norm(moved), smp["centre"][0] / d_k, atol=1e-15)
            assert np.array_equal(out["mean"][:, 0], mean[:, 0])


def test_realignment_uses_the_camera_centre_of_a_posed_view():
    """With a posed camera the ray starts at C = -R^T t: the survivor's
    distance to C (not to the world origin) becomes the group's mean."""
    a = 0.3
    R = np.array([[math.cos(a), 0, math.sin(a)], [0, 1, 0], [-math.sin(a), 0, math.cos(a)]])
    t = np.array([0.4, -0.2, 1.0])
    cam = camera(f=F, w=W, h=H, R=R, t=t)
    Rf, tf = np.asarray(cam.R, np.float32).astype(np.float64), np.asarray(cam.t, np.float32).astype(np.float64)
    C = -Rf.T @ tf
    xg, xs = _at(10.6, 10.4, 6.1), _on_ray(10, 10, 6.0)
    mean = (Rf.T @ (xg - tf))[:, None]
    centre = (Rf.T @ (xs - tf))[None]
    dg, dk = np.linalg.norm(xg), np.linalg.norm(xs)
    ls = np.full((3, 1), math.log(0.5 * dg / F))
    out = merge(mean, ls, np.zeros((3, 1)), cam, dict(pix=np.array([10 * W + 10]), centre=centre,
                                                      colour=np.array([[0.5, 0.5, 0.5]])),
                np.full((H, W), 0.25), tau_d=1.0)
    assert out["keep"][0] and not out["keep_new"][0]
    # (the float32 rotation is orthonormal to ~1e-8 only)
    assert abs(np.linalg.norm(out["mean"][:, 0] - C) - (dg + dk) / 2) < 1e-6
