"""Pins of the LoG insertion oracle (oracle/insert64.py): the sampled
operator's closed forms (zero on constant and linear images, 4 on x^2 + y^2,
its sums and symmetry), a circular convolution through the FFT, the clamp and
threshold semantics, the scale formula, and the back-projected centres
projected again by the renderer's projection."""
import math

import numpy as np
import pytest
import torch

from oracle.insert64 import TAU_A, insert, log_kernel_2d, log_kernels, log_response, probability
from oracle.project64 import project_view, to_params64
from tiny_scenes import camera


@pytest.mark.parametrize("sigma", [0.8, 1.0, 1.7])
def test_kernel_moments_and_symmetry(sigma):
    g, h, R = log_kernels(sigma)
    x = np.arange(-R, R + 1)
    assert R == math.ceil(3 * sigma)
    assert abs(g.sum() - 1) < 1e-15 and abs(h.sum()) < 1e-15 and abs((x * x * h).sum() - 2) < 1e-14
    K, _ = log_kernel_2d(sigma)
    X, Y = np.meshgrid(x, x)
    assert abs(K.sum()) < 1e-14
    assert np.array_equal(K, K.T) and np.array_equal(K, K[::-1, :]) and np.array_equal(K, K[:, ::-1])
    assert abs((K * (X * X + Y * Y)).sum() - 4.0) < 1e-13
    # the centre tap is negative (a LoG dips at the centre)
    assert K[R, R] < 0


def test_constant_linear_and_quadratic_images():
    H, W = 30, 40
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    const = np.stack([np.full((H, W), c) for c in (0.1, 0.5, 0.9)])
    assert np.abs(log_response(const)).max() < 1e-14  # borders included (replicated constant)
    lin = np.stack([0.3 * xx - 0.2 * yy + 1.0, 0.01 * xx, -0.05 * yy])
    quad = np.stack([0.01 * (xx * xx + yy * yy), 0.02 * (xx * xx + yy * yy), 0 * xx])
    for sigma in (1.0, 1.5):
        R = math.ceil(3 * sigma)
        inner = (slice(None), slice(R, H - R), slice(R, W - R))
        assert np.abs(log_response(lin, sigma)[inner]).max() < 1e-12
        q = log_response(quad, sigma)[inner]
        assert np.abs(q[0] - 0.04).max() < 1e-12 and np.abs(q[1] - 0.08).max() < 1e-12


def test_interior_equals_circular_convolution_by_fft():
    rng = np.random.default_rng(9)
    H, W = 24, 36
    img = rng.uniform(0, 1, (3, H, W))
    sigma = 1.2
    K, R = log_kernel_2d(sigma)
    Kp = np.zeros((H, W))
    for dy in range(-R, R + 1):
        for dx in range(-R, R + 1):
            Kp[dy % H, dx % W] = K[dy + R, dx + R]
    circ = np.real(np.fft.ifft2(np.fft.fft2(img, axes=(1, 2)) * np.fft.fft2(Kp)[None], axes=(1, 2)))
    ref = log_response(img, sigma)
    inner = (slice(None), slice(R, H - R), slice(R, W - R))
    assert np.abs(ref[inner] - circ[inner]).max() < 1e-12


def test_probability_clamps_at_one_and_uses_the_channel_norm():
    H, W = 16, 16
    img = np.zeros((3, H, W))
    img[:, 8, 8] = (3.0, 4.0, 0.0)  # a strong point: response norm well above 1 at the centre
    p = probability(img)
    assert p[8, 8] == 1.0
    K, R = log_kernel_2d()
    # one tap away the response is K[R, R+2] * (3, 4, 0): its norm is 5 |K|
    assert abs(p[8, 10] - min(5 * abs(K[R, R + 2]), 1.0)) < 1e-15


def test_insertion_threshold_scale_and_centres():
    H, W = 20, 28
    cam = camera(f=50.0, w=W, h=H, R=np.eye(3), t=np.array([0.1, -0.2, 0.3]))
    gt = np.zeros((3, H, W))
    gt[:, 6, 9] = 0.4  # a faint point: P(I) < 1 around it
    gt[:, 13, 20] = 2.0
    render = np.zeros((3, H, W))
    render[:, 13, 20] = 2.0  # the second point is already rendered
    depth = np.full((H, W), 4.0)
    depth[6, 9] = 5.0
    out = insert(gt, render, depth, cam)
    p_a = np.maximum(out["p_gt"] - out["p_render"], 0.0)
    assert np.array_equal(out["mask"], p_a > TAU_A)
    assert np.array_equal(out["pix"], np.nonzero((p_a > TAU_A).reshape(-1))[0])
    assert 6 * W + 9 in out["pix"]  # the faint point's centre
    assert not out["mask"][13, 20]  # rendered already: P_a = 0
    k = list(out["pix"]).index(6 * W + 9)
    xc = np.array([5.0 * (9.5 - 14.0) / 50.0, 5.0 * (6.5 - 10.0) / 50.0, 5.0])
    S = np.linalg.norm(xc) / (2.0 * math.sqrt(out["p_gt"][6, 9]) * 50.0)
    assert abs(out["scale"][k] - S) < 1e-15
    # the centres project back onto their pixel centres at their depths
    n = len(out["pix"])
    p64 = to_params64(dict(mean=out["mean"].T.astype(np.float32), log_scale=np.full((3, n), -5.0, np.float32),
                           quat=np.tile(np.float32([1, 0, 0, 0])[:, None], (1, n)),
                           opacity_logit=np.zeros(n, np.float32), sh=np.zeros((1, 3, n), np.float32)))
    proj = project_view(p64, 0, cam)
    u = (out["pix"] % W) + 0.5
    v = (out["pix"] // W) + 0.5
    with torch.no_grad():
        assert np.abs(proj["mu2"][:, 0].numpy() - u).max() < 1e-4
        assert np.abs(proj["mu2"][:, 1].numpy() - v).max() < 1e-4
        assert np.abs(proj["depth"].numpy() - depth.reshape(-1)[out["pix"]]).max() < 1e-5


def test_ambiguity_flag():
    H, W = 12, 12
    gt = np.zeros((3, H, W))
    render = np.zeros((3, H, W))
    cam = camera(f=20.0, w=W, h=H)
    out = insert(gt, render, np.ones((H, W)), cam, tau_a=0.0)
    # P_a = 0 everywhere sits exactly on a zero threshold: every pixel is flagged
    assert out["ambiguous"].all() and not out["mask"].any()
