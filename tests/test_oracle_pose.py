"""Pins of the FP64 camera-pose gradients (oracle/grad64.py, cam_grads) and
of the rig parameterisation (oracle/rig64.py): central differences of the
forward definition with the pose perturbed in the geometry only, the world
translation and world rotation invariances of the image (SH degree 0, where
the colour does not depend on the viewing direction), the composition order
of Eq. 3, and central differences of the rig products."""
import numpy as np
import pytest
import torch

from oracle.fd import fd_pose_gradient
from oracle.grad64 import grad64
from oracle.rig64 import compose, perturbed, rig_vjp, to_mat
from tiny_scenes import mini_rig


def _cots(cams, seed):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((3, c.height, c.width)) for c in cams]


def _check_pose_fd(scene, cams, cots, grads, rel=1e-6):
    checked = 0
    G = grads["cam"]
    scale = np.abs(G).max()
    for v in range(len(cams)):
        for e in range(12):
            for h in (1e-6, 1e-7, 1e-8):  # a smaller step where a decision flips
                fd, valid = fd_pose_gradient(scene, cams, cots, v, e, h=h)
                if valid:
                    break
            if not valid:
                continue
            ad = G[v, e]
            assert abs(fd - ad) <= rel * max(abs(ad), 1e-3 * scale), (v, e, fd, ad)
            checked += 1
    return checked


def test_pose_gradient_matches_finite_differences_cfg1(cfg1):
    scene, cams, _ = cfg1
    cots = _cots(cams, 31)
    grads = grad64(scene, cams, cots, cam_grads=True)
    assert grads["cam"].shape == (1, 12)
    assert _check_pose_fd(scene, cams, cots, grads) >= 11


def test_pose_gradient_matches_finite_differences_posed_sh3():
    """Two posed views, SH degree 3: the difference quotient keeps the
    viewing direction of the unperturbed camera, so a pose gradient that
    leaked the SH path would fail here."""
    scene, cams = mini_rig()
    cots = _cots(cams, 32)
    grads = grad64(scene, cams, cots, cam_grads=True)
    assert _check_pose_fd(scene, cams, cots, grads) >= 22


def test_pose_gradient_leaves_gaussian_gradients_unchanged():
    scene, cams = mini_rig()
    cots = _cots(cams, 33)
    a = grad64(scene, cams, cots)
    b = grad64(scene, cams, cots, cam_grads=True)
    for k in a:
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("which", ["cfg1", "rig"])
def test_world_translation_invariance(which, cfg1):
    """Shifting every mean by delta and every t_v by -R_v delta leaves x_c,
    hence the image, unchanged (degree 0): sum_g dL/dmu_g = sum_v R_v^T dL/dt_v."""
    if which == "cfg1":
        scene, cams, _ = cfg1
    else:
        scene, cams = mini_rig(degree=0)
    assert scene.sh_degree == 0
    grads = grad64(scene, cams, _cots(cams, 34), cam_grads=True)
    lhs = grads["mean"].sum(axis=1)
    rhs = sum(np.asarray(c.R, np.float32).astype(np.float64).reshape(3, 3).T @ grads["cam"][v, 9:]
              for v, c in enumerate(cams))
    bound = np.abs(grads["mean"]).sum(axis=1).max()
    assert np.abs(lhs - rhs).max() <= 1e-10 * bound, (lhs, rhs)
    assert np.abs(rhs).max() > 1e-3 * bound


def test_world_rotation_invariance():
    """Rotating the world by Q (means Q mu, Gaussian rotations Q R(q), i.e.
    q <- q_Q (x) q) and every camera by R_v Q^T leaves the image unchanged
    (degree 0).  At Q = I + [w]x: sum_g dL/dmu_g . (w x mu_g) + sum_g dL/dq_g .
    (0, w/2) (x) q_g = sum_v <dL/dR_v, R_v [w]x>."""
    scene, cams = mini_rig(degree=0, seed=9)
    grads = grad64(scene, cams, _cots(cams, 35), cam_grads=True)
    mu = scene.mean.astype(np.float64)  # [3, n]
    q = scene.quat.astype(np.float64)  # [4, n] = (w, x, y, z)
    for w in np.eye(3):
        dmu = np.cross(w[:, None], mu, axis=0)
        h = 0.5 * w[:, None]
        dq = np.concatenate([-(h * q[1:]).sum(axis=0, keepdims=True),
                             q[0:1] * h + np.cross(h, q[1:], axis=0)], axis=0)
        t_mu = (grads["mean"] * dmu).sum()
        t_q = (grads["quat"] * dq).sum()
        wx = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
        rhs = 0.0
        for v, c in enumerate(cams):
            R = np.asarray(c.R, np.float32).astype(np.float64).reshape(3, 3)
            rhs += (grads["cam"][v, :9].reshape(3, 3) * (R @ wx)).sum()
        bound = np.abs(grads["mean"] * dmu).sum() + np.abs(grads["quat"] * dq).sum()
        assert abs(t_mu + t_q - rhs) <= 1e-10 * bound, (w, t_mu + t_q, rhs)
        assert abs(rhs) > 1e-4 * bound


def _random_pose(rng):
    a = rng.standard_normal(3)
    A = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    R = torch.linalg.matrix_exp(torch.tensor(A)).numpy()
    return np.concatenate([R.reshape(-1), rng.standard_normal(3)])


def test_rig_composition_order():
    """T_v = T_m T_{i->m}: a relative transform T_m^{-1} T recovers T, and a
    pure relative translation tau moves the view to t_m + R_m tau."""
    rng = np.random.default_rng(40)
    Tm = np.stack([_random_pose(rng) for _ in range(2)])
    T = _random_pose(rng)
    Minv = np.linalg.inv(to_mat(Tm[1]).numpy())
    rel_inv = (Minv @ to_mat(T).numpy())
    rel = np.concatenate([rel_inv[:3, :3].reshape(-1), rel_inv[:3, 3]])
    tau = rng.standard_normal(3)
    rel_t = np.concatenate([np.eye(3).reshape(-1), tau])
    out = compose(Tm, np.stack([rel, rel_t]), [1, 0], [0, 1]).numpy()
    assert np.abs(out[0] - T).max() < 1e-12
    R0 = Tm[0, :9].reshape(3, 3)
    assert np.abs(out[1, :9] - Tm[0, :9]).max() == 0.0
    assert np.abs(out[1, 9:] - (Tm[0, 9:] + R0 @ tau)).max() < 1e-14


def _rig_case(seed):
    rng = np.random.default_rng(seed)
    F, K = 3, 4
    central = np.stack([_random_pose(rng) for _ in range(F)])
    relative = np.stack([_random_pose(rng) for _ in range(K)])
    frame = np.repeat(np.arange(F), K)
    camera = np.tile(np.arange(K), F)
    G = rng.standard_normal((F * K, 12))
    return central, relative, frame, camera, G


def test_rig_matrix_gradients_by_finite_differences():
    central, relative, frame, camera, G = _rig_case(41)
    out = rig_vjp(central, relative, frame, camera, G)

    def phi(c, r):
        return float((G * compose(c, r, frame, camera).numpy()).sum())

    h = 1e-6
    for name, arr, grad in (("central", central, out["d_central"]), ("relative", relative, out["d_relative"])):
        for idx in np.ndindex(arr.shape):
            a, b = arr.copy(), arr.copy()
            a[idx] += h
            b[idx] -= h
            if name == "central":
                fd = (phi(a, relative) - phi(b, relative)) / (2 * h)
            else:
                fd = (phi(central, a) - phi(central, b)) / (2 * h)
            assert abs(fd - grad[idx]) <= 1e-7 * max(1.0, abs(grad[idx])), (name, idx, fd, grad[idx])


def test_rig_tangent_gradients_by_finite_differences():
    central, relative, frame, camera, G = _rig_case(42)
    out = rig_vjp(central, relative, frame, camera, G)

    def phi(c, r):
        return float((G * compose(c, r, frame, camera).numpy()).sum())

    h = 1e-6
    for f in range(central.shape[0]):
        for k in range(6):
            xi = np.zeros((central.shape[0], 6))
            xi[f, k] = h
            fp = phi(perturbed(central, xi).numpy(), relative)
            fm = phi(perturbed(central, -xi).numpy(), relative)
            assert abs((fp - fm) / (2 * h) - out["xi_central"][f, k]) <= 1e-7 * max(1.0, abs(out["xi_central"][f, k]))
    for c in range(relative.shape[0]):
        for k in range(6):
            xi = np.zeros((relative.shape[0], 6))
            xi[c, k] = h
            fp = phi(central, perturbed(relative, xi).numpy())
            fm = phi(central, perturbed(relative, -xi).numpy())
            assert abs((fp - fm) / (2 * h) - out["xi_relative"][c, k]) <= 1e-7 * max(1.0, abs(out["xi_relative"][c, k]))


def test_rig_tangent_pure_translation():
    """With dL/dR_v = 0 and a single view, a left perturbation moves t by
    rho + phi x t, so dL/drho = g and dL/dphi = t x g for g = dL/dt_v."""
    rng = np.random.default_rng(43)
    central = _random_pose(rng)[None]
    relative = np.concatenate([np.eye(3).reshape(-1), np.zeros(3)])[None]
    g = rng.standard_normal(3)
    G = np.concatenate([np.zeros(9), g])[None]
    out = rig_vjp(central, relative, [0], [0], G)
    assert np.abs(out["xi_central"][0, :3] - g).max() < 1e-12
    assert np.abs(out["xi_central"][0, 3:] - np.cross(central[0, 9:], g)).max() < 1e-12
