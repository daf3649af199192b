"""Pins of the FP64 compositing definition (oracle/render64.py), the
projection (oracle/project64.py), the SH basis and the tile lists."""
import math

import numpy as np
import torch

from oracle.binning import tile_grid, tile_lists
from oracle.project64 import project_view, to_params64
from oracle.render64 import render, render_pixel, render_view, view_setup
from oracle.sh64 import sh_basis
from oracle.spec32 import spec32
from tiny_scenes import Y0, camera, logit, scene
from workloads import make_config

ID_Q = [1.0, 0.0, 0.0, 0.0]


def _alpha(o, power):
    return min(0.99, o * math.exp(power))


def test_single_isotropic_gaussian_on_axis_closed_form():
    f, z, ls, p = 60.0, 4.0, -2.0, 0.8
    col = [0.9, 0.4, 0.2]
    sc = scene([[0.0, 0.0, z]], [[ls] * 3], [ID_Q], [logit(p)], colours=[col])
    cam = camera(f, 64, 48)
    out = render(sc, [cam])[0]
    s = math.exp(np.float32(ls))
    o = 1.0 / (1.0 + math.exp(-float(np.float32(logit(p)))))
    var = (f * s / z) ** 2 + 0.3
    col64 = Y0 * np.float32((np.array(col) - 0.5) / Y0).astype(np.float64) + 0.5
    box = spec32(sc.mean, sc.log_scale, sc.quat, cam, 16)["box"]
    for j in range(48):
        for i in range(64):
            r2 = (i + 0.5 - 32.0) ** 2 + (j + 0.5 - 24.0) ** 2
            a = _alpha(o, -0.5 * r2 / var)
            inbox = box[0][0] <= i <= box[1][0] and box[2][0] <= j <= box[3][0]
            a = a if (inbox and a >= 1 / 255) else 0.0
            assert abs(out["image"][0, j, i] - col64[0] * a) < 1e-12
            assert abs(out["T"][j, i] - (1.0 - a)) < 1e-12
            assert out["count"][j, i] == (1 if a > 0 else 0)


def test_off_axis_isotropic_covariance_closed_form():
    f, fy = 60.0, 70.0
    pts = [[0.7, -0.4, 3.0], [-1.1, 0.5, 2.5]]
    ls = -2.5
    sc = scene(pts, [[ls] * 3] * 2, [ID_Q] * 2, [0.0, 0.0], colours=[[0.5] * 3] * 2)
    cam = camera(f, 64, 48, fy=fy)
    pr = project_view(to_params64(sc.arrays()), 0, cam)
    s2 = math.exp(2 * float(np.float32(ls)))
    for k, (x, y, z) in enumerate(np.asarray(pts, np.float32).astype(np.float64)):
        jjt = np.array([[f * f * (1 + x * x / z / z), f * fy * x * y / z / z],
                        [f * fy * x * y / z / z, fy * fy * (1 + y * y / z / z)]]) / z / z
        S = s2 * jjt + 0.3 * np.eye(2)
        got = pr["cov2"][k].numpy()
        assert np.allclose(got, [S[0, 0], S[0, 1], S[1, 1]], rtol=1e-12, atol=0)
        assert np.allclose(pr["mu2"][k].numpy(), [f * x / z + 32, fy * y / z + 24], rtol=1e-13)


def test_rotated_anisotropic_covariance_sign():
    """+45 deg about the optical axis turns the long x axis towards +x+y, so the
    2D covariance has S_xy = (f/z)^2 (a - b)/2 > 0; a transposed rotation
    matrix would flip its sign."""
    f, z = 60.0, 5.0
    la, lb = -1.5, -2.5
    half = math.radians(22.5)
    sc = scene([[0, 0, z]], [[la, lb, -3.0]], [[math.cos(half), 0, 0, math.sin(half)]], [0.0], colours=[[0.5] * 3])
    pr = project_view(to_params64(sc.arrays()), 0, camera(f))
    a, b = math.exp(2 * float(np.float32(la))), math.exp(2 * float(np.float32(lb)))
    k = (f / z) ** 2
    q = np.asarray(sc.quat[:, 0], np.float64)
    c2 = (q[0] ** 2 - q[3] ** 2) / (q[0] ** 2 + q[3] ** 2)  # cos of the actual float32 angle
    s2 = 2 * q[0] * q[3] / (q[0] ** 2 + q[3] ** 2)
    exp = [k * (a * c2 * c2 + b * s2 * s2) + 0.3, k * (a - b) * c2 * s2, k * (a * s2 * s2 + b * c2 * c2) + 0.3]
    assert np.allclose(pr["cov2"][0].numpy(), exp, rtol=1e-12)
    assert pr["cov2"][0, 1] > 0
    # the image is brighter along +x+y than along +x-y
    out = render(sc, [camera(f)])[0]
    assert out["image"][0, 24 + 3, 32 + 3] > out["image"][0, 24 - 4, 32 + 3] * 1.5


def test_jacobian_guard_clamps_x_over_z():
    f, z, x = 60.0, 2.0, 5.0  # x/z = 2.5 > 1.3 * 32 / 60
    ls = -2.0
    sc = scene([[x, 0, z]], [[ls] * 3], [ID_Q], [0.0], colours=[[0.5] * 3])
    pr = project_view(to_params64(sc.arrays()), 0, camera(f))
    lim = 1.3 * 32.0 / 60.0
    s2 = math.exp(2 * float(np.float32(ls)))
    J = np.array([[f / z, 0, -f * lim / z], [0, f / z, 0]])
    S = s2 * J @ J.T + 0.3 * np.eye(2)
    assert np.allclose(pr["cov2"][0].numpy(), [S[0, 0], S[0, 1], S[1, 1]], rtol=1e-12)


def test_two_gaussians_composite_front_to_back():
    c1, c2 = [0.9, 0.1, 0.3], [0.2, 0.8, 0.6]
    # the front Gaussian has the larger index: order must follow depth
    sc = scene([[0, 0, 5.0], [0, 0, 3.0]], [[-2.2] * 3, [-2.4] * 3], [ID_Q] * 2, [0.5, -0.3], colours=[c2, c1])
    cam = camera(60.0, 64, 48, cx=32.5, cy=24.5)
    pr = project_view(to_params64(sc.arrays()), 0, cam)
    o = pr["opacity"].numpy()
    rgb = pr["rgb"].numpy()
    out = render(sc, [cam])[0]
    a_front, a_back = min(0.99, o[1]), min(0.99, o[0])  # pixel (32, 24) sits on both centres
    exp = rgb[1] * a_front + rgb[0] * a_back * (1 - a_front)
    assert np.allclose(out["image"][:, 24, 32], exp, rtol=0, atol=1e-14)
    assert out["last"][24, 32] == 0 and out["count"][24, 32] == 2


def test_alpha_095_stack_composites_exactly_three():
    n = 6
    col = [0.7, 0.5, 0.3]
    sc = scene([[0, 0, 4.0]] * n, [[-2.0] * 3] * n, [ID_Q] * n, [logit(0.95)] * n, colours=[col] * n)
    cam = camera(60.0, 64, 48, cx=32.5, cy=24.5)
    out = render(sc, [cam])[0]
    assert out["count"][24, 32] == 3
    assert abs(out["T"][24, 32] - 0.05 ** 3) < 1e-9
    rgb = project_view(to_params64(sc.arrays()), 0, cam)["rgb"][0].numpy()
    assert np.allclose(out["image"][:, 24, 32], rgb * (1 - 0.05 ** 3), atol=1e-8)
    assert out["last"][24, 32] == 2  # equal depths: ties broken by index


def test_telescoping_and_white_identities(cfg1):
    scene_, cams, _ = cfg1
    out = render(scene_, cams)[0]
    assert np.abs(out["wsum"] + out["T"] - 1.0).max() < 1e-12
    white = scene_.subset(np.arange(scene_.n))
    white.sh[0] = np.float32(0.5 / Y0)
    o2 = render(white, cams, bg=(0.0, 0.0, 0.0))[0]
    rgb = 0.5 + Y0 * float(np.float32(0.5 / Y0))
    assert np.abs(o2["image"][0] - rgb * (1.0 - o2["T"])).max() < 1e-12
    assert out["ambiguous"].mean() <= 1e-4


def test_sh_orthonormal_by_quadrature():
    xg, wg = np.polynomial.legendre.leggauss(24)
    phi = (np.arange(48) + 0.5) * 2 * math.pi / 48
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    d = torch.from_numpy(np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3))
    w = torch.from_numpy((wg[:, None] * np.full(48, 2 * math.pi / 48)[None, :]).reshape(-1))
    Y = sh_basis(d, 3)
    gram = (Y * w[:, None]).T @ Y
    assert torch.allclose(gram, torch.eye(16, dtype=torch.float64), atol=1e-10)


def test_sh_degree1_colour_direction_from_camera_centre():
    """Camera centre C = -R^T t at (1, 0, 0); Gaussian at (0, 0, 5): d points
    to -x, so Y_3 = -C1 d_x > 0."""
    k = 4
    sh = np.zeros((k, 3, 1))
    sh[3, :, 0] = [1.0, -1.0, 0.5]
    sc = scene([[0, 0, 5.0]], [[-2.0] * 3], [ID_Q], [0.0], sh=sh, degree=1)
    cam = camera(60.0, t=[-1.0, 0.0, 0.0])
    rgb = project_view(to_params64(sc.arrays()), 1, cam)["rgb"][0].numpy()
    c1 = math.sqrt(3 / (4 * math.pi))
    y3 = -c1 * (-1.0 / math.sqrt(26.0))
    assert np.allclose(rgb, np.maximum(0, np.array([1.0, -1.0, 0.5]) * y3 + 0.5), rtol=1e-14)


def test_vectorised_render_equals_per_pixel_loop(cfg1):
    scene_, cams, _ = cfg1
    out = render(scene_, cams)[0]
    setup = view_setup(scene_.arrays(), 0, cams[0])
    rng = np.random.default_rng(3)
    for _ in range(150):
        i, j = int(rng.integers(0, 64)), int(rng.integers(0, 48))
        r = render_pixel(scene_.arrays(), 0, cams[0], i, j, setup=setup)
        assert np.array_equal(r["color"], out["image"][:, j, i])
        assert r["T"] == out["T"][j, i] and r["count"] == out["count"][j, i] and r["last"] == out["last"][j, i]


def test_window_render_equals_full_render(cfg1):
    scene_, cams, _ = cfg1
    full = render(scene_, cams)[0]
    win = render_view(scene_.arrays(), 0, cams[0], window=(10, 37, 5, 29))
    assert np.array_equal(win["image"], full["image"][:, 5:29, 10:37])
    assert np.array_equal(win["count"], full["count"][5:29, 10:37])


def test_permutation_invariance(cfg1):
    scene_, cams, _ = cfg1
    base = render(scene_, cams)[0]
    zb = spec32(scene_.mean, scene_.log_scale, scene_.quat, cams[0], 16)["zbits"]
    assert len(np.unique(zb[zb > 0])) == (zb > 0).sum()  # distinct depths
    perm = np.random.default_rng(5).permutation(scene_.n)
    out = render(scene_.subset(perm), cams)[0]
    assert np.array_equal(out["image"], base["image"])
    assert np.array_equal(out["T"], base["T"])


def test_projective_scale_invariance(cfg1):
    scene_, cams, _ = cfg1
    base = render(scene_, cams)[0]
    big = scene_.subset(np.arange(scene_.n))
    big.mean = (scene_.mean * np.float32(2.0)).astype(np.float32)
    big.log_scale = (scene_.log_scale.astype(np.float64) + math.log(2.0)).astype(np.float32)
    out = render(big, cams)[0]
    ok = ~(base["ambiguous"] | out["ambiguous"])
    assert ok.mean() > 0.99
    assert np.abs(out["image"] - base["image"])[:, ok].max() < 1e-5


def test_tile_lists_restrict_to_pixel_candidate_lists():
    scene_, cams = make_config(1, scale=0.5)
    for ts in (8, 16, 32):
        keys, vals, csr = tile_lists(scene_, cams, ts)
        tx_n, ty_n, base = tile_grid(cams, ts)
        s = spec32(scene_.mean, scene_.log_scale, scene_.quat, cams[0], ts)
        i0, i1, j0, j1 = s["box"]
        vis = s["visible"]
        assert np.all(np.diff(keys.astype(np.float64)) >= 0)
        for tile in range(int(base[-1])):
            lst = vals[csr[tile]:csr[tile + 1]]
            ty, tx = divmod(tile, int(tx_n[0]))
            for (i, j) in [(tx * ts, ty * ts), (min(tx * ts + ts - 1, 63), min(ty * ts + ts // 2, 47))]:
                inb = vis & (i0 <= i) & (i <= i1) & (j0 <= j) & (j <= j1)
                cand = np.nonzero(inb)[0]
                cand = cand[np.lexsort((cand, s["zbits"][cand]))]
                filt = [g for g in lst if i0[g] <= i <= i1[g] and j0[g] <= j <= j1[g]]
                assert list(cand) == filt
