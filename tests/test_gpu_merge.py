"""Per-camera merging through the C ABI against the FP64 oracle
(oracle/merge64.py): keep flags of the existing Gaussians and of the view's
samples bit for bit, and the surviving colours within 1e-6, on groups whose
decisions are not within 1e-5 of a threshold; other views' samples are left
alone; on a small posed view with placed Gaussians and on the rig's 1600x900
views with the 1M-Gaussian scene as the existing set (the samples there are
the oracle's own insertion lists of seeded synthetic images)."""
import math

import numpy as np
import pytest
import torch

from gpu_helpers import log
from oracle.insert64 import insert
from oracle.merge64 import merge
from paper_2512_08498_amd import Rasterizer
from tiny_scenes import camera
from workloads import make_config, make_insert_inputs

pytestmark = pytest.mark.gpu


def _samples_for(rast, cams, view, pix_local, centres, gt_flat):
    """Device sample list (global pixel indices, centres) for one view, and the host dict."""
    off = rast.pix_off[view]
    cap = len(pix_local) + 5
    pix = np.zeros(cap, np.int32)
    pix[:len(pix_local)] = (pix_local + off).astype(np.int32)
    mean = np.zeros((cap, 3), np.float32)
    mean[:len(pix_local)] = centres
    w, h = rast.sizes[view]
    img = gt_flat[3 * off:3 * (off + w * h)].reshape(3, h * w)
    host = dict(pix=pix_local, centre=centres.astype(np.float32).astype(np.float64),
                colour=img[:, pix_local].T.astype(np.float64))
    dev = dict(pix=torch.from_numpy(pix).cuda(), mean=torch.from_numpy(mean).cuda(),
               scale=torch.zeros(cap, dtype=torch.float32, device="cuda"),
               count=torch.tensor([len(pix_local)], dtype=torch.int32, device="cuda"))
    return host, dev


def _compare(res, ref, n, k):
    keep = res["keep"][:n].cpu().numpy().astype(bool)
    colour = res["colour"][:, :n].cpu().numpy().astype(np.float64).T
    keep_new = res["keep_new"][:k].cpu().numpy().astype(bool)
    colour_new = res["colour_new"][:k].cpu().numpy().astype(np.float64)
    ok_g, ok_n = ~ref["ambiguous_g"], ~ref["ambiguous_new"]
    assert np.array_equal(keep[ok_g], ref["keep"][ok_g])
    assert np.array_equal(keep_new[ok_n], ref["keep_new"][ok_n])
    assert np.abs(colour[ok_g] - ref["colour"][ok_g]).max(initial=0.0) <= 1e-6
    assert np.abs(colour_new[ok_n] - ref["colour_new"][ok_n]).max(initial=0.0) <= 1e-6
    if "mean" in res:
        # re-aligned centres: the double-precision result rounded to float32
        mean = res["mean"][:, :n].cpu().numpy().astype(np.float64)
        mean_new = res["mean_new"][:k].cpu().numpy().astype(np.float64)
        rm, rmn = ref["mean"][:, ok_g], ref["mean_new"][ok_n]
        assert (np.abs(mean[:, ok_g] - rm) <= 1e-6 * np.maximum(1.0, np.abs(rm))).all()
        assert (np.abs(mean_new[ok_n] - rmn) <= 1e-6 * np.maximum(1.0, np.abs(rmn))).all()
    log(f"  {int((ref['match'] >= 0).sum())} matched Gaussians, {int((~ref['keep']).sum())} removed, "
        f"{int((~ref['keep_new']).sum())} of {k} samples dropped; ambiguous {int(ref['ambiguous_g'].sum())} "
        f"Gaussians, {int(ref['ambiguous_new'].sum())} samples")
    return int((ref["match"] >= 0).sum())


def _small_view_case(seed):
    """A 48x32 posed view (view 1 of two) with K samples at random pixels and
    N Gaussians, half of them placed near the samples' back-projections."""
    rng = np.random.default_rng(seed)
    a = 0.15
    R = np.array([[math.cos(a), 0, math.sin(a)], [0, 1, 0], [-math.sin(a), 0, math.cos(a)]])
    cams = [camera(f=50.0, w=40, h=30), camera(f=60.0, w=48, h=32, R=R, t=np.array([0.1, 0.0, -0.2]))]
    rast = Rasterizer(cams, 1, 0)
    W, H = 48, 32
    K, N = 80, 600
    pix = np.sort(rng.choice(W * H, K, replace=False))
    z = rng.uniform(2, 7, K)
    u, v = pix % W + 0.5, pix // W + 0.5
    xc = np.stack([z * (u - 24) / 60, z * (v - 16) / 60, z], 1)
    Rf = np.asarray(cams[1].R, np.float32).astype(np.float64)
    tf = np.asarray(cams[1].t, np.float32).astype(np.float64)
    centres = ((xc - tf) @ Rf).astype(np.float32)
    mean = np.stack([rng.uniform(-2, 2, N), rng.uniform(-1.5, 1.5, N), rng.uniform(-1, 8, N)])
    for g in range(0, N, 2):
        # near a sample's depth, projected within 0.7 px of its pixel centre
        # (so across pixel borders, where the bilinear match differs from the
        # containing pixel)
        k = rng.integers(0, K)
        zz = xc[k, 2] * rng.uniform(0.92, 1.08)
        uu, vv = u[k] + rng.uniform(-0.7, 0.7), v[k] + rng.uniform(-0.7, 0.7)
        mean[:, g] = (np.array([zz * (uu - 24) / 60, zz * (vv - 16) / 60, zz]) - tf) @ Rf
    mean = mean.astype(np.float32)
    ls = rng.normal(-3.0, 0.6, (3, N)).astype(np.float32)
    sh = rng.normal(0, 1, (1, 3, N)).astype(np.float32)
    gt = rng.uniform(0, 1, 3 * rast.total_px).astype(np.float32)
    p = rng.uniform(0.05, 1.0, rast.total_px).astype(np.float32)
    ex = {k_: torch.from_numpy(np.ascontiguousarray(v_)).cuda() for k_, v_ in
          (("mean", mean), ("log_scale", ls), ("sh", sh))}
    p_view = p[rast.pix_off[1]:rast.pix_off[2]].reshape(H, W)
    return rast, cams, pix, centres, (mean, ls, sh), ex, gt, p, p_view


def _merge_small(rast, cams, pix, centres, params, ex, gt, p, p_view, kappa):
    host, dev = _samples_for(rast, cams, 1, pix, centres, gt)
    dev["p_gt"] = torch.from_numpy(p).cuda()
    res = rast.merge(ex, 1, torch.from_numpy(gt).cuda(), dev, tau_d=0.4, kappa=kappa)
    torch.cuda.synchronize()
    mean, ls, sh = params
    ref = merge(mean, ls, sh[0], cams[1], host, p_view, tau_d=0.4, kappa=kappa)
    return res, ref


@pytest.mark.parametrize("kappa", [1.0, 2.0])
def test_merge_small_view(kappa):
    rast, cams, pix, centres, params, ex, gt, p, p_view = _small_view_case(60)
    res, ref = _merge_small(rast, cams, pix, centres, params, ex, gt, p, p_view, kappa)
    K, N = len(pix), params[0].shape[1]
    assert _compare(res, ref, N, K) > 50
    # the spare entries (and any other view's) are untouched
    assert not res["keep_new"][K:].any()
    # written in place into an earlier result: the same outputs, spare entries kept
    for v_ in res.values():
        v_.fill_(7)
    _, dev = _samples_for(rast, cams, 1, pix, centres, gt)
    dev["p_gt"] = torch.from_numpy(p).cuda()
    res2 = rast.merge(ex, 1, torch.from_numpy(gt).cuda(), dev, tau_d=0.4, kappa=kappa, out=res)
    torch.cuda.synchronize()
    assert res2 is res
    _compare(res, ref, N, K)
    assert (res["keep_new"][K:] == 7).all() and (res["colour_new"][K:] == 7).all()


def test_merge_twice_on_one_workspace():
    """The pixel -> sample map in the workspace is not cleared between calls:
    a second merge with a third of the samples, at other list positions, must
    ignore what the first left behind (pixels it sampled that the second does not, indices
    that now name other pixels or lie past the count)."""
    rast, cams, pix, centres, params, ex, gt, p, p_view = _small_view_case(63)
    N = params[0].shape[1]
    res, ref = _merge_small(rast, cams, pix, centres, params, ex, gt, p, p_view, 1.0)
    assert _compare(res, ref, N, len(pix)) > 50
    sel = np.sort(np.random.default_rng(64).permutation(len(pix))[:len(pix) // 3])
    ws = rast._merge_ws.data_ptr()
    res2, ref2 = _merge_small(rast, cams, pix[sel], centres[sel], params, ex, gt, p, p_view, 1.0)
    assert rast._merge_ws.data_ptr() == ws
    assert 10 < _compare(res2, ref2, N, len(sel)) < int((ref["match"] >= 0).sum())


def test_merge_rig_views_with_the_scene():
    scene, cams = make_config(3)
    rast = Rasterizer(cams, 1, 0)
    gts, rds, depths = make_insert_inputs(rast.sizes, 61)
    gt_flat = np.concatenate([g.reshape(-1) for g in gts])
    ex = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in scene.arrays().items()}
    sh0 = scene.sh[0]
    total = 0
    for view in (0, 3):
        o = insert(gts[view], rds[view], depths[view], cams[view])
        host, dev = _samples_for(rast, cams, view, o["pix"], o["mean"].astype(np.float32), gt_flat)
        p_full = np.zeros(rast.total_px, np.float32)
        p_full[rast.pix_off[view]:rast.pix_off[view + 1]] = o["p_gt"].reshape(-1)
        dev["p_gt"] = torch.from_numpy(p_full).cuda()
        res = rast.merge(ex, view, torch.from_numpy(gt_flat).cuda(), dev, tau_d=50.0)
        torch.cuda.synchronize()
        ref = merge(scene.mean, scene.log_scale, sh0, cams[view], host, o["p_gt"].astype(np.float32), tau_d=50.0)
        log(f"view {view}: {len(o['pix'])} samples")
        total += _compare(res, ref, scene.n, len(o["pix"]))
    assert total > 100


def test_merge_without_samples():
    """An empty sample list: every existing Gaussian is kept with its own DC
    colour and the spare sample entries are untouched."""
    rng = np.random.default_rng(62)
    cams = [camera(f=50.0, w=40, h=30)]
    rast = Rasterizer(cams, 1, 0)
    N = 200
    mean = np.stack([rng.uniform(-1, 1, N), rng.uniform(-1, 1, N), rng.uniform(2, 6, N)]).astype(np.float32)
    ls = rng.normal(-3.0, 0.5, (3, N)).astype(np.float32)
    sh = rng.normal(0, 1, (1, 3, N)).astype(np.float32)
    gt = rng.uniform(0, 1, 3 * rast.total_px).astype(np.float32)
    host, dev = _samples_for(rast, cams, 0, np.zeros(0, np.int64), np.zeros((0, 3), np.float32), gt)
    dev["p_gt"] = torch.full((rast.total_px,), 0.5, dtype=torch.float32, device="cuda")
    ex = {k_: torch.from_numpy(np.ascontiguousarray(v_)).cuda() for k_, v_ in
          (("mean", mean), ("log_scale", ls), ("sh", sh))}
    res = rast.merge(ex, 0, torch.from_numpy(gt).cuda(), dev, tau_d=1.0)
    torch.cuda.synchronize()
    ref = merge(mean, ls, sh[0], cams[0], host, np.full((30, 40), 0.5), tau_d=1.0)
    assert ref["keep"].all()
    assert res["keep"][:N].cpu().numpy().astype(bool).all()
    colour = res["colour"][:, :N].cpu().numpy().astype(np.float64).T
    assert np.abs(colour - ref["colour"]).max() <= 1e-6
    assert not res["keep_new"].any()


def test_merge_rig_view_with_a_tight_depth_bound():
    """The rig's 1600x900 view 0 with the 1M-Gaussian scene as the existing
    set and tau_d = 0.5 m: each sample's centre is placed on its pixel's ray
    at the distance of a scene Gaussian that projects near it, plus N(0, 0.4 m),
    so the depth bound accepts some correspondences and rejects others at
    full scale."""
    scene, cams = make_config(3)
    view = 0
    cam = cams[view]
    rast = Rasterizer(cams, 1, 0)
    gts, rds, depths = make_insert_inputs(rast.sizes, 61)
    gt_flat = np.concatenate([g.reshape(-1) for g in gts])
    o = insert(gts[view], rds[view], depths[view], cam)
    W, H = rast.sizes[view]
    # distances of scene Gaussians by the pixel their projection falls in
    R = np.asarray(cam.R, np.float64)
    xc = R @ scene.mean.astype(np.float64) + np.asarray(cam.t, np.float64)[:, None]
    front = xc[2] > 0.2
    u = cam.fx * xc[0] / np.where(front, xc[2], 1) + cam.cx
    v = cam.fy * xc[1] / np.where(front, xc[2], 1) + cam.cy
    ok = front & (u >= 0) & (u < W) & (v >= 0) & (v < H)
    pix_g = (np.floor(v[ok]).astype(np.int64) * W + np.floor(u[ok]).astype(np.int64))
    dist_at = np.full(W * H, np.nan)
    dist_at[pix_g] = np.linalg.norm(xc[:, ok], axis=0)
    rng = np.random.default_rng(65)
    pix = o["pix"]
    d = dist_at[pix]
    has = np.isfinite(d)
    assert has.sum() > 1000
    d = np.where(has, d + rng.normal(0, 0.4, len(pix)), rng.uniform(5, 40, len(pix)))
    ray = np.stack([(pix % W + 0.5 - cam.cx) / cam.fx, (pix // W + 0.5 - cam.cy) / cam.fy, np.ones(len(pix))], 1)
    xs = ray / np.linalg.norm(ray, axis=1, keepdims=True) * d[:, None]
    centres = ((xs - np.asarray(cam.t, np.float64)) @ R).astype(np.float32)
    host, dev = _samples_for(rast, cams, view, pix, centres, gt_flat)
    p_full = np.zeros(rast.total_px, np.float32)
    p_full[rast.pix_off[view]:rast.pix_off[view + 1]] = o["p_gt"].reshape(-1)
    dev["p_gt"] = torch.from_numpy(p_full).cuda()
    ex = {k: torch.from_numpy(np.ascontiguousarray(v_)).cuda() for k, v_ in scene.arrays().items()}
    res = rast.merge(ex, view, torch.from_numpy(gt_flat).cuda(), dev, tau_d=0.5)
    torch.cuda.synchronize()
    ref = merge(scene.mean, scene.log_scale, scene.sh[0], cam, host, o["p_gt"].astype(np.float32), tau_d=0.5)
    loose = merge(scene.mean, scene.log_scale, scene.sh[0], cam, host, o["p_gt"].astype(np.float32), tau_d=50.0)
    rejected = int(((loose["match"] >= 0) & (ref["match"] < 0)).sum())
    log(f"tight tau_d: {len(pix)} samples, {rejected} correspondences rejected by depth")
    assert rejected > 100
    assert _compare(res, ref, scene.n, len(pix)) > 100
