"""Pins of the FP64 gradients (oracle/grad64.py) against central finite
differences of the forward definition (oracle/fd.py), of the L1 loss and of
the Adam recurrence."""
import numpy as np
import torch

from oracle.adam64 import adam_step
from oracle.fd import fd_gradient
from oracle.grad64 import grad64
from oracle.loss64 import l1_loss
from oracle.render64 import render
from tiny_scenes import mini_rig


def _check_fd(scene, cams, cot, grads, picks, rel=1e-6, h_rel=1e-6):
    checked = 0
    for name, flat in picks:
        fd, valid = fd_gradient(scene, cams, cot, name, flat, h_rel=h_rel)
        if not valid:
            continue
        ad = grads[name].reshape(-1)[flat]
        scale = np.abs(grads[name]).max()
        assert abs(fd - ad) <= rel * max(abs(ad), 1e-3 * scale), (name, flat, fd, ad)
        checked += 1
    return checked


def _picks(scene, grads, rng, per_group):
    picks = []
    for name, g in grads.items():
        flat = np.nonzero(np.abs(g.reshape(-1)) > 0)[0]
        if len(flat):
            for f in rng.choice(flat, size=min(per_group, len(flat)), replace=False):
                picks.append((name, int(f)))
    return picks


def test_autograd_matches_finite_differences_cfg1(cfg1):
    scene, cams, _ = cfg1
    rng = np.random.default_rng(11)
    cot = [rng.standard_normal((3, c.height, c.width)) for c in cams]
    grads = grad64(scene, cams, cot)
    n = _check_fd(scene, cams, cot, grads, _picks(scene, grads, rng, 12))
    assert n >= 45


def test_autograd_matches_finite_differences_posed_sh3():
    scene, cams = mini_rig()
    rng = np.random.default_rng(12)
    cot = [rng.standard_normal((3, c.height, c.width)) for c in cams]
    grads = grad64(scene, cams, cot)
    # every SH coefficient index must get checked at least once
    picks = _picks(scene, grads, rng, 10)
    n = scene.n
    for k in range(16):
        flat = k * 3 * n + np.nonzero(np.abs(grads["sh"][k, 0]) > 0)[0][:1]
        picks += [("sh", int(f)) for f in flat]
    assert _check_fd(scene, cams, cot, grads, picks) >= 55


def test_windowed_gradient_equals_masked_full_gradient(cfg1):
    scene, cams, _ = cfg1
    rng = np.random.default_rng(13)
    cot = rng.standard_normal((3, 48, 64))
    win = (8, 40, 12, 36)
    masked = np.zeros_like(cot)
    masked[:, 12:36, 8:40] = cot[:, 12:36, 8:40]
    g_full = grad64(scene, cams, [masked])
    g_win = grad64(scene, cams, [cot], windows=[win])
    for k in g_full:
        assert np.allclose(g_full[k], g_win[k], rtol=1e-12, atol=1e-15)


def test_l1_loss_gradient_by_finite_differences(cfg1):
    scene, cams, targets = cfg1
    img = render(scene, cams)[0]["image"]
    loss, grads = l1_loss([img], targets)
    assert abs(loss - np.abs(img - targets[0]).mean()) < 1e-15
    rng = np.random.default_rng(2)
    for _ in range(50):
        c, j, i = int(rng.integers(0, 3)), int(rng.integers(0, 48)), int(rng.integers(0, 64))
        h = 1e-5
        if abs(img[c, j, i] - targets[0][c, j, i]) < 1e-4:
            continue  # the kink of |x| is not differentiable
        p, m = img.copy(), img.copy()
        p[c, j, i] += h
        m[c, j, i] -= h
        fd = (l1_loss([p], targets)[0] - l1_loss([m], targets)[0]) / (2 * h)
        assert abs(fd - grads[0][c, j, i]) < 1e-6 * abs(grads[0][c, j, i])


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(4)
    p, g = rng.standard_normal(1000), rng.standard_normal(1000)
    z = np.zeros(1000)
    p1, m1, v1 = adam_step(p, g, z, z, 0, 1e-2)
    assert np.allclose(p1, p - 1e-2 * g / (np.abs(g) + 1e-15), rtol=0, atol=1e-15)


def test_adam_matches_torch_adam_float64():
    rng = np.random.default_rng(5)
    p0 = rng.standard_normal(500)
    gs = [rng.standard_normal(500) for _ in range(6)]
    tp = torch.nn.Parameter(torch.from_numpy(p0.copy()))
    opt = torch.optim.Adam([tp], lr=3e-3, betas=(0.9, 0.999), eps=1e-15)
    p, m, v = p0.copy(), np.zeros(500), np.zeros(500)
    for step, g in enumerate(gs):
        tp.grad = torch.from_numpy(g.copy())
        opt.step()
        p, m, v = adam_step(p, g, m, v, step, 3e-3)
    assert np.allclose(p, tp.detach().numpy(), rtol=0, atol=1e-13)


def test_autograd_matches_finite_differences_at_the_alpha_cap():
    """alpha = min(0.99, o G) has zero derivative in o and G where the cap
    is active (reading of Sec. 3.3's gradients through the renderer).  The
    scene holds >= 100 capped composited entries; the cotangent weighs the
    pixels with a capped entry 30x, and the picks include the opacity,
    position, scale and rotation of every capped Gaussian, so a gradient
    passed through the cap (or dropped from uncapped pixels) fails."""
    from oracle.render64 import render_view
    from tiny_scenes import capped

    scene, cams = capped()
    o = render_view(scene.arrays(), scene.sh_degree, cams[0])
    n_cap = int(o["capped"].sum())
    assert n_cap >= 100 and not o["ambiguous"].any()
    rng = np.random.default_rng(31)
    cot = [rng.standard_normal((3, cams[0].height, cams[0].width)) * (1.0 + 30.0 * (o["capped"] > 0))[None]]
    grads = grad64(scene, cams, cot)
    opac = 1.0 / (1.0 + np.exp(-scene.opacity_logit.astype(np.float64)))
    ids = np.nonzero(opac > 0.99)[0]
    assert len(ids) >= 12
    n = scene.n
    picks = [("opacity_logit", int(g)) for g in ids]
    picks += [("mean", int(c * n + g)) for g in ids for c in (0, 1)]
    picks += [("log_scale", int(g)) for g in ids[::2]] + [("quat", int(n + g)) for g in ids[1::2]]
    picks += _picks(scene, grads, rng, 6)
    # opacity logits near 6 make dL/dtheta small (o (1 - o) ~ 3e-3): a step of
    # 1e-5 keeps the difference quotient's rounding below the 1e-6 bar
    assert _check_fd(scene, cams, cot, grads, picks, h_rel=1e-5) >= 60


def test_autograd_matches_finite_differences_beyond_the_jacobian_guard():
    """Where x/z (or y/z) lies beyond the guard, J is built from the clamped
    value, which has zero derivative in x_c.  Ten large Gaussians centred
    outside the guard on all sides of a posed view (SH degree 3) reach into
    the image; FD of their positions, scales, rotations and SH coefficients
    pins the clamp's derivative (and its absence from the unclamped
    coordinate)."""
    from oracle.render64 import render_view
    from tiny_scenes import guard_clamped, guard_clamped_ids

    scene, cams = guard_clamped()
    ids = guard_clamped_ids(scene, cams)[0]
    o = render_view(scene.arrays(), scene.sh_degree, cams[0], record=True)
    _, gg = o["entries"]
    reached = [int(g) for g in ids if (gg == g).sum() >= 50]
    assert len(reached) >= 8
    rng = np.random.default_rng(41)
    cot = [rng.standard_normal((3, cams[0].height, cams[0].width))]
    grads = grad64(scene, cams, cot)
    n = scene.n
    picks = []
    for g in reached:
        picks += [("mean", c * n + g) for c in range(3)]
        picks += [("log_scale", c * n + g) for c in range(3)]
        picks += [("quat", c * n + g) for c in (0, 2)]
        picks += [("opacity_logit", g), ("sh", (5 * 3 + 1) * n + g)]
    picks += _picks(scene, grads, rng, 4)
    assert _check_fd(scene, cams, cot, grads, picks) >= 80
