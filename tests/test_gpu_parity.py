"""GPU parity of the HIP path against the CPU oracle (through the C ABI).

Bars: tile keys/values/CSR bit-exact; images within 1e-5 absolute, final
transmittance within 1e-5, contributor counts and last contributor exact on
pixels the oracle does not flag as ambiguous; gradients within 1e-4 of the
FP64 oracle relative to each parameter group's largest entry, and 1e-4
relative elementwise for entries above 1e-2 of it, under a loss masked to
non-ambiguous pixels.
"""
import math

import numpy as np
import pytest
import torch

from gpu_helpers import compare_grads, device_params, grads_to_host, host_outputs, last_gaussian, log, \
    render_gpu
from oracle.binning import tile_lists
from oracle.grad64 import grad64
from oracle.render64 import render
from tiny_scenes import camera, logit, mini_rig, needles, scene
from workloads import make_config

pytestmark = pytest.mark.gpu

IMG_TOL = 1e-5
GRAD_TOL = 1e-4


def _check_forward(scene, cams, ts, oracle=None, max_ambiguous=1e-3, **kw):
    rast, params, out = render_gpu(scene, cams, ts=ts, **kw)
    keys, vals, csr = rast.debug_binning()
    okeys, ovals, ocsr = tile_lists(scene, cams, ts)
    assert len(keys) == len(okeys)
    assert np.array_equal(keys, okeys)
    assert np.array_equal(vals, ovals)
    assert np.array_equal(csr, ocsr)
    oracle = oracle if oracle is not None else render(scene, cams)
    imgs, T, cnt, last = host_outputs(rast, out)
    for v in range(len(cams)):
        o = oracle[v]
        ok = ~o["ambiguous"]
        assert ok.mean() >= 1 - max_ambiguous
        err = np.abs(imgs[v] - o["image"])[:, ok].max()
        log(f"view {v}: max image err {err:.3e}, ambiguous {(~ok).sum()}")
        assert err <= IMG_TOL
        assert np.abs(T[v] - o["T"])[ok].max() <= IMG_TOL
        assert np.array_equal(cnt[v][ok], o["count"][ok])
        lg = last_gaussian(rast, last[v], v, vals, csr)
        assert np.array_equal(lg[ok], o["last"][ok])
    return rast, params, out


@pytest.mark.parametrize("ts", [16, 8, 32])
def test_forward_cfg1(cfg1, ts):
    scene, cams, _ = cfg1
    log(f"forward cfg1 ts={ts}")
    _check_forward(scene, cams, ts)


def test_forward_posed_two_views_sh3():
    scene, cams = mini_rig()
    log("forward mini rig ts=16")
    _check_forward(scene, cams, 16)


def _masked_cotangent(oracle, targets):
    px = sum(t.shape[1] * t.shape[2] for t in targets)
    cots = []
    for o, t in zip(oracle, targets):
        g = np.sign(o["image"] - t) / (3.0 * px)
        g[:, o["ambiguous"]] = 0.0
        cots.append(g)
    return cots


def _compare_grads(gpu, ora, tol=GRAD_TOL):
    compare_grads(gpu, ora, tol)


def _check_backward(scene, cams, targets, ts=16, cots=None, cam_grads=False, oracle=None, **kw):
    """GPU gradients (and with cam_grads the views' pose gradients) against
    grad64 under the masked L1 cotangent of ``targets``, or under ``cots``
    (per-view [3, H, W], zeroed here on ambiguous pixels)."""
    oracle = oracle if oracle is not None else render(scene, cams)
    if cots is None:
        cots = _masked_cotangent(oracle, targets)
    else:
        cots = [np.where(o["ambiguous"][None], 0.0, c.astype(np.float32).astype(np.float64))
                for o, c in zip(oracle, cots)]
    rast, params, out = render_gpu(scene, cams, ts=ts, **kw)
    dl = torch.from_numpy(np.concatenate([c.astype(np.float32).reshape(-1) for c in cots])).cuda()
    grads = rast.backward(params, out, dl, cam_grads=True if cam_grads else None)
    torch.cuda.synchronize()
    _compare_grads(grads_to_host(grads), grad64(scene, cams, cots, cam_grads=cam_grads))


@pytest.mark.parametrize("ts", [16, 8, 32])
def test_backward_cfg1(cfg1, ts):
    scene, cams, targets = cfg1
    log(f"backward cfg1 ts={ts}")
    _check_backward(scene, cams, targets, ts)


def test_backward_posed_two_views_sh3():
    scene, cams = mini_rig()
    rng = np.random.default_rng(21)
    targets = [rng.uniform(0, 1, (3, c.height, c.width)).astype(np.float32) for c in cams]
    log("backward mini rig")
    _check_backward(scene, cams, targets)


@pytest.mark.parametrize("degree", [0, 1, 2])
def test_forward_and_backward_other_sh_degrees(degree):
    """The mini rig at SH degrees 0, 1 and 2 (degree 3 above): image and
    gradients against the oracle.  Every gradient array sits at the front of
    a buffer twice its size filled with a sentinel, which must survive: the
    per-Gaussian kernel updates the SH coefficients in groups, and degree 2
    has an odd count (nine) of them."""
    scene, cams = mini_rig(degree=degree)
    log(f"mini rig, SH degree {degree}")
    oracle = render(scene, cams)
    rast, params, out = _check_forward(scene, cams, 16, oracle=oracle)
    rng = np.random.default_rng(30 + degree)
    targets = [rng.uniform(0, 1, (3, c.height, c.width)).astype(np.float32) for c in cams]
    cots = _masked_cotangent(oracle, targets)
    dl = torch.from_numpy(np.concatenate([c.astype(np.float32).reshape(-1) for c in cots])).cuda()
    sentinel = -12345.5
    bufs = {k: torch.full((2 * v.numel(),), sentinel, dtype=torch.float32, device="cuda") for k, v in params.items()}
    grads = {k: bufs[k][:v.numel()].view(v.shape) for k, v in params.items()}
    rast.backward(params, out, dl, grads=grads)
    torch.cuda.synchronize()
    for k, b in bufs.items():
        assert bool((b[params[k].numel():] == sentinel).all()), k
    _compare_grads(grads_to_host(grads), grad64(scene, cams, cots))


def deep_stack(seed=12, n=2600, w=48, h=32):
    """About n entries in every 16 px tile of a 48 x 32 view: wide, faint
    Gaussians (opacity 1-4%), so most pixels composite on past list
    position 1024 (and many past 2048): the backward recovers T by division
    over more than a thousand entries."""
    rng = np.random.default_rng(seed)
    means = np.stack([rng.uniform(-0.25, 0.25, n), rng.uniform(-0.15, 0.15, n), rng.uniform(3.0, 6.0, n)], 1)
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    sc = scene(means, rng.normal(math.log(0.5), 0.2, (n, 3)), q,
               [logit(p) for p in rng.uniform(0.01, 0.04, n)], colours=rng.uniform(0.0, 1.0, (n, 3)))
    return sc, [camera(50.0, w, h)]


@pytest.mark.parametrize("ts,long_list", [(16, 0), (16, 1024), (16, 0xFFFFFFFF), (8, 1024), (32, 1024)])
def test_long_lists_forward_and_backward(ts, long_list):
    """Lists of about 2600 entries (at 16 px; 8 and 32 px bin them
    differently), walked at 16 px by the four waves of a workgroup
    (long_list 0 or 1024) or by one wave ('never'): image and gradients
    against the oracle."""
    sc, cams = deep_stack()
    oracle = render(sc, cams)
    # about 0.7% of the pixels decide a composite within the oracle's
    # ambiguity margin after a thousand entries; they are left out
    _check_forward(sc, cams, ts, oracle=oracle, max_ambiguous=0.01, long_list=long_list)
    rng = np.random.default_rng(13)
    targets = [rng.uniform(0, 1, (3, c.height, c.width)).astype(np.float32) for c in cams]
    log(f"deep stack, ts {ts}, long_list {long_list}")
    _check_backward(sc, cams, targets, ts, oracle=oracle, long_list=long_list)


@pytest.mark.parametrize("ts,long_list", [(16, 1024), (16, 0), (8, 1024), (32, 1024)])
def test_needles_forward_and_backward(ts, long_list):
    """Elongated footprints near the opacity threshold: the backward drops,
    per tile, the records whose alpha >= 1/255 ellipse misses it (about 40%
    of this scene's pairs), in the one-wave and the workgroup walks
    (long_list 0 sends every tile to the workgroup walk)."""
    scene, cams = needles()
    log(f"needles ts={ts} long_list={long_list}")
    _check_forward(scene, cams, ts)
    rng = np.random.default_rng(3)
    targets = [rng.uniform(0, 1, (3, c.height, c.width)).astype(np.float32) for c in cams]
    _check_backward(scene, cams, targets, ts, long_list=long_list)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_binning_extreme_scenes(seed):
    """Tile lists bit for bit on scenes far from the workloads: coordinates up
    to 1e4, scales from 1e-3 to 1e2 of the scene, rotated cameras with
    principal points outside the image and unequal focal lengths (the
    visibility of every (view, Gaussian) pair decides the lists)."""
    import math

    from tiny_scenes import camera
    from workloads.generators import Scene

    rng = np.random.default_rng(700 + seed)
    scale = 10.0 ** rng.uniform(-1, 4)
    n = 6000
    mean = rng.standard_normal((3, n)) * scale
    mean[2] += scale * rng.uniform(0, 2)
    q = rng.standard_normal((4, n))
    scene = Scene(mean=mean.astype(np.float32),
                  log_scale=(rng.normal(math.log(scale) - 5, 1.5, (3, n))).astype(np.float32),
                  quat=q.astype(np.float32), opacity_logit=rng.normal(0, 1, n).astype(np.float32),
                  sh=rng.normal(0, 0.5, (1, 3, n)).astype(np.float32), sh_degree=0)
    cams = []
    for _ in range(3):
        a, b = rng.uniform(-3, 3, 2)
        R = np.array([[math.cos(a), 0, math.sin(a)], [0, 1, 0], [-math.sin(a), 0, math.cos(a)]]) @ \
            np.array([[1, 0, 0], [0, math.cos(b), -math.sin(b)], [0, math.sin(b), math.cos(b)]])
        w, h = int(rng.integers(40, 200)), int(rng.integers(30, 150))
        f = float(rng.uniform(0.3, 3.0) * w)
        cams.append(camera(f=f, w=w, h=h, cx=float(rng.uniform(-0.2, 1.2) * w), cy=float(rng.uniform(-0.2, 1.2) * h),
                           R=R, t=rng.standard_normal(3) * scale, fy=f * float(rng.uniform(0.7, 1.4))))
    log(f"extreme binning seed={seed} scale={scale:.3g}")
    rast, params, out = render_gpu(scene, cams, ts=16)
    keys, vals, csr = rast.debug_binning()
    okeys, ovals, ocsr = tile_lists(scene, cams, 16)
    log(f"  {len(okeys)} pairs")
    assert len(keys) == len(okeys)
    assert np.array_equal(keys, okeys) and np.array_equal(vals, ovals) and np.array_equal(csr, ocsr)


def _oracle_evaluations(scene, cams, oracle):
    """Bounds (lo, hi) on the backward's evaluation count from the oracle:
    per pixel, the Gaussians whose pixel box holds it, up to and including
    its last composited one in depth order.  An ambiguous pixel may stop
    anywhere, so it adds 0 to lo and all its boxes to hi."""
    from oracle.render64 import view_setup

    arrays = scene.arrays()
    lo = hi = 0
    for v, cam in enumerate(cams):
        spec, order, _ = view_setup(arrays, scene.sh_degree, cam)
        i0, i1, j0, j1 = spec["box"]
        rank = np.full(scene.n, -1, np.int64)
        rank[order] = np.arange(len(order))
        last = oracle[v]["last"]
        last_rank = np.where(last >= 0, rank[np.maximum(last, 0)], -1)
        amb = oracle[v]["ambiguous"]
        for k, g in enumerate(order):
            sl = (slice(int(j0[g]), int(j1[g]) + 1), slice(int(i0[g]), int(i1[g]) + 1))
            lo += int(((last_rank[sl] >= k) & ~amb[sl]).sum())
            hi += int(((last_rank[sl] >= k) | amb[sl]).sum())
    return lo, hi


@pytest.mark.parametrize("ts", [16, 8, 32])
def test_evaluation_count(cfg1, ts):
    """The work counter behind the compositing roofline equals the oracle's
    count at every tile size (the count does not depend on the tiling)."""
    scene, cams, _ = cfg1
    oracle = render(scene, cams)
    rast, params, out = render_gpu(scene, cams, ts=ts)
    got = rast.count_evaluations(out)
    lo, hi = _oracle_evaluations(scene, cams, oracle)
    log(f"ts={ts}: evaluations {got}, oracle [{lo}, {hi}]")
    assert lo <= got <= hi
    assert got >= int(out["n_contrib"].sum().item())


def test_evaluation_count_rig():
    scene, cams = mini_rig()
    oracle = render(scene, cams)
    rast, params, out = render_gpu(scene, cams, ts=16)
    got = rast.count_evaluations(out)
    lo, hi = _oracle_evaluations(scene, cams, oracle)
    log(f"mini rig: evaluations {got}, oracle [{lo}, {hi}]")
    assert lo <= got <= hi


@pytest.mark.parametrize("ts,long_list", [(16, 1024), (16, 0), (16, 0xFFFFFFFF), (8, 1024), (32, 1024)])
def test_alpha_cap_scene(ts, long_list):
    """Opaque Gaussians whose o G exceeds 0.99 at >= 100 composited entries:
    alpha takes the cap there and its derivative in opacity and falloff is
    zero (the oracle's FP64 gradient, pinned by finite differences at these
    entries).  Forward and gradients at the usual bars, with a cotangent that
    weighs the capped pixels 30x, for both backward walks at 16 px."""
    from tiny_scenes import capped

    scene, cams = capped()
    oracle = render(scene, cams)
    n_cap = int(oracle[0]["capped"].sum())
    log(f"alpha cap ts={ts} long_list={long_list}: {n_cap} capped entries, "
        f"{int(oracle[0]['ambiguous'].sum())} ambiguous pixels")
    assert n_cap >= 100
    _check_forward(scene, cams, ts, oracle=oracle)
    rng = np.random.default_rng(31)
    cot = rng.standard_normal((3, cams[0].height, cams[0].width)) * 1e-3
    cot *= (1.0 + 30.0 * (oracle[0]["capped"] > 0))[None]
    _check_backward(scene, cams, None, ts, cots=[cot], oracle=oracle, long_list=long_list)


@pytest.mark.parametrize("ts,long_list", [(16, 1024), (16, 0), (16, 0xFFFFFFFF), (8, 1024), (32, 1024)])
def test_guard_clamp_scene(ts, long_list):
    """Large Gaussians centred beyond the Jacobian guard on every side of a
    posed view (SH degree 3) whose footprints reach the image: J is built
    from the clamped x/z and y/z, whose derivative is zero (pinned by finite
    differences).  Forward, Gaussian gradients and the view's pose gradient
    against the oracle."""
    from oracle.render64 import render_view
    from tiny_scenes import guard_clamped, guard_clamped_ids

    scene, cams = guard_clamped()
    oracle = render(scene, cams)
    ids = guard_clamped_ids(scene, cams)[0]
    _, gg = render_view(scene.arrays(), scene.sh_degree, cams[0], record=True)["entries"]
    reached = int(sum((gg == g).sum() >= 50 for g in ids))
    log(f"guard clamp ts={ts} long_list={long_list}: {len(ids)} clamped Gaussians, {reached} composited "
        f"at >= 50 pixels")
    assert reached >= 8
    _check_forward(scene, cams, ts, oracle=oracle)
    rng = np.random.default_rng(41)
    targets = [rng.uniform(0, 1, (3, c.height, c.width)).astype(np.float32) for c in cams]
    _check_backward(scene, cams, targets, ts, cam_grads=True, oracle=oracle, long_list=long_list)
