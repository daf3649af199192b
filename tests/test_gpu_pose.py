"""Camera-pose gradients and the rig parameterisation through the C ABI,
against the FP64 oracle: each view's dL/d(R, t) with the SH colour detached
(on the 1-view workload at every tile size, on posed SH-3 views and on every
backward work split), its independence from the Gaussian gradients, the
accumulate mode and the fused Adam path, and the rig composition T_m T_{i->m}
with its gradients, end to end on a rig of 2 frames x 3 cameras.  Bar: the
gradient bar of the parity tests (1e-4 of the largest entry, 1e-4 relative
on entries above 1e-2 of it)."""
import math

import numpy as np
import pytest
import torch

from gpu_helpers import device_params, grads_to_host, log, render_gpu
from oracle.grad64 import grad64
from oracle.render64 import render
from oracle.rig64 import compose, rig_vjp
from paper_2512_08498_amd import FusedAdam, Rasterizer
from paper_2512_08498_amd._lib import GsrError
from test_gpu_parity import GRAD_TOL, _compare_grads, _masked_cotangent
from tiny_scenes import camera, mini_rig

pytestmark = pytest.mark.gpu


def _dl(cots):
    return torch.from_numpy(np.concatenate([c.astype(np.float32).reshape(-1) for c in cots])).cuda()


def _targets(cams, seed):
    rng = np.random.default_rng(seed)
    return [rng.uniform(0, 1, (3, c.height, c.width)).astype(np.float32) for c in cams]


def _pose_case(scene, cams, targets, ts=16, long_list=1024):
    cots = _masked_cotangent(render(scene, cams), targets)
    rast, params, out = render_gpu(scene, cams, ts=ts, long_list=long_list)
    grads = rast.backward(params, out, _dl(cots), cam_grads=True)
    torch.cuda.synchronize()
    return rast, params, out, cots, grads


@pytest.mark.parametrize("ts", [8, 16, 32])
def test_pose_gradients_cfg1(cfg1, ts):
    scene, cams, targets = cfg1
    _, _, _, cots, grads = _pose_case(scene, cams, targets, ts=ts)
    log(f"tile {ts}")
    _compare_grads(grads_to_host(grads), grad64(scene, cams, cots, cam_grads=True))


def test_pose_gradients_posed_sh3():
    scene, cams = mini_rig()
    _, _, _, cots, grads = _pose_case(scene, cams, _targets(cams, 51))
    _compare_grads(grads_to_host(grads), grad64(scene, cams, cots, cam_grads=True))


@pytest.mark.parametrize("long_list", [0, 16, 0xFFFFFFFF])
def test_pose_gradients_split_variants(long_list):
    scene, cams = mini_rig(seed=3)
    _, _, _, cots, grads = _pose_case(scene, cams, _targets(cams, 52), long_list=long_list)
    ref = grad64(scene, cams, cots, cam_grads=True)
    log(f"long_list={long_list}")
    _compare_grads({"cam": grads["camera"].cpu().numpy().astype(np.float64)}, {"cam": ref["cam"]})


def test_pose_gradients_leave_gaussian_gradients_and_accumulate():
    """The Gaussian gradients are bit for bit those of a backward without the
    pose output; accumulate = 1 adds the pose gradient onto the array."""
    scene, cams = mini_rig()
    rast, params, out, cots, grads = _pose_case(scene, cams, _targets(cams, 53))
    plain = rast.backward(params, out, _dl(cots))
    for k in plain:
        assert torch.equal(plain[k], grads[k]), k
    first = grads["camera"].clone()
    again = rast.backward(params, out, _dl(cots), grads=dict(grads), accumulate=True, cam_grads=grads["camera"])
    torch.cuda.synchronize()
    assert torch.equal(again["camera"], 2.0 * first)


def test_fused_adam_path_gives_the_same_pose_gradients():
    scene, cams = mini_rig()
    rast, params, out, cots, grads = _pose_case(scene, cams, _targets(cams, 54))
    opt = FusedAdam(rast, {k: v.clone() for k, v in params.items()})
    cam = torch.full((len(cams), 12), float("nan"), dtype=torch.float32, device="cuda")
    rast.backward_adam(opt.params, out, _dl(cots), opt, cam_grads=cam)  # Gaussian outputs all NULL
    torch.cuda.synchronize()
    assert torch.equal(cam, grads["camera"])


def _rot(axis, deg):
    a = math.radians(deg)
    x, y, z = np.asarray(axis, np.float64) / np.linalg.norm(axis)
    K = np.array([[0, -z, y], [z, 0, -x], [-y, x, 0]])
    return np.eye(3) + math.sin(a) * K + (1 - math.cos(a)) * K @ K


def _rig_setup(n_frames=2, n_cams=3, w=96, h=64):
    """Central poses moving along z, relative transforms of a small fan of
    cameras; view v = frame v // n_cams, camera v % n_cams."""
    central = []
    for f in range(n_frames):
        R = _rot([0.1, 1.0, 0.05], 3.0 * f)
        centre = np.array([0.05 * f, -0.02 * f, 0.3 * f])
        central.append(np.concatenate([R.reshape(-1), -R @ centre]))
    relative = []
    for k in range(n_cams):
        R = _rot([0.0, 1.0, 0.0], 10.0 * (k - (n_cams - 1) / 2))
        relative.append(np.concatenate([R.reshape(-1), np.array([0.1 * k, 0.0, -0.05 * k])]))
    central = np.asarray(central, np.float32).astype(np.float64)
    relative = np.asarray(relative, np.float32).astype(np.float64)
    frame = np.repeat(np.arange(n_frames), n_cams).astype(np.int32)
    cam = np.tile(np.arange(n_cams), n_frames).astype(np.int32)
    poses = compose(central, relative, frame, cam).numpy()
    cams = [camera(80.0, w, h, R=p[:9].reshape(3, 3).astype(np.float32), t=p[9:].astype(np.float32))
            for p in poses]
    return central, relative, frame, cam, cams


def test_rig_compose_and_gradients_match_the_oracle():
    central, relative, frame, cam, cams = _rig_setup()
    rast = Rasterizer(cams, 1, 0)
    rast.set_rig(frame, cam, len(central), len(relative))
    c_dev = torch.from_numpy(central.astype(np.float32)).cuda()
    r_dev = torch.from_numpy(relative.astype(np.float32)).cuda()
    cams_dev = torch.zeros_like(rast.cams_dev)
    cams_dev[:, 12:] = rast.cams_dev[:, 12:]
    rast.rig_compose(c_dev, r_dev, cams_dev=cams_dev)
    torch.cuda.synchronize()
    ref = compose(central, relative, frame, cam).numpy()
    got = cams_dev[:, :12].cpu().numpy().astype(np.float64)
    assert np.abs(got - ref).max() <= 1e-6
    assert torch.equal(cams_dev[:, 12:], rast.cams_dev[:, 12:])  # intrinsics and sizes untouched
    rng = np.random.default_rng(55)
    G = rng.standard_normal((len(cams), 12)).astype(np.float32)
    out = rast.rig_gradients(c_dev, r_dev, torch.from_numpy(G).cuda())
    o = rig_vjp(central, relative, frame, cam, G.astype(np.float64))
    for k in ("d_central", "d_relative", "xi_central", "xi_relative"):
        g = out[k].cpu().numpy().astype(np.float64)
        scale = np.abs(o[k]).max()
        log(f"  {k}: {np.abs(g - o[k]).max() / scale:.2e} of max")
        assert np.abs(g - o[k]).max() <= 1e-5 * scale, k


def test_rig_end_to_end_pose_gradients():
    """Render the rig's six views, take each view's pose gradient under the
    masked L1 loss, and carry it to the central poses and relative
    transforms: against the oracle's own chain (grad64 then rig_vjp)."""
    central, relative, frame, cam, cams = _rig_setup()
    scene, _ = mini_rig(seed=11, n=400)
    _, _, _, cots, grads = _pose_case(scene, cams, _targets(cams, 56))
    ref = grad64(scene, cams, cots, cam_grads=True)
    _compare_grads({"cam": grads["camera"].cpu().numpy().astype(np.float64)}, {"cam": ref["cam"]})
    rast = Rasterizer(cams, scene.n, scene.sh_degree)
    rast.set_rig(frame, cam, len(central), len(relative))
    out = rast.rig_gradients(torch.from_numpy(central.astype(np.float32)).cuda(),
                             torch.from_numpy(relative.astype(np.float32)).cuda(), grads["camera"])
    o = rig_vjp(central, relative, frame, cam, ref["cam"])
    _compare_grads({k: out[k].cpu().numpy().astype(np.float64) for k in o}, o, tol=GRAD_TOL)


def test_rig_plan_rejects_bad_indices():
    central, relative, frame, cam, cams = _rig_setup()
    rast = Rasterizer(cams, 1, 0)
    with pytest.raises(RuntimeError):
        rast.rig_compose(torch.zeros(2, 12, device="cuda"), torch.zeros(3, 12, device="cuda"))
    bad = frame.copy()
    bad[2] = 2
    with pytest.raises(GsrError):
        rast.set_rig(bad, cam, 2, 3)
    bad = cam.copy()
    bad[0] = -1
    with pytest.raises(GsrError):
        rast.set_rig(frame, bad, 2, 3)
    rast.set_rig(frame, cam, 2, 3)
    with pytest.raises(ValueError):
        rast.rig_gradients(torch.zeros(2, 12, device="cuda"), torch.zeros(3, 12, device="cuda"),
                           torch.zeros(5, 12, device="cuda"))
