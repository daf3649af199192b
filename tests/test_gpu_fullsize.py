"""Parity at the benchmark's full size, in the launch configuration bench.py
times (all 6 views of the 1M-Gaussian rig in one batch, 16 px tiles):
the complete binning bit for bit, sampled pixels against the per-pixel
oracle, and gradients under a loss restricted to pixel windows."""
import numpy as np
import pytest
import torch

from gpu_helpers import grads_to_host, host_outputs, last_gaussian, log, render_gpu
from oracle.binning import tile_lists
from oracle.grad64 import grad64
from oracle.render64 import render_pixels, render_view, view_setup
from workloads import make_config, make_target

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rig():
    log("generating the 1M-Gaussian rig")
    scene, cams = make_config(3)
    rast, params, out = render_gpu(scene, cams, ts=16)
    return scene, cams, rast, params, out


def test_fullsize_binning_bit_exact(rig):
    scene, cams, rast, params, out = rig
    keys, vals, csr = rast.debug_binning()
    log(f"pairs {len(keys)}")
    okeys, ovals, ocsr = tile_lists(scene, cams, 16)
    assert np.array_equal(csr, ocsr)
    assert np.array_equal(keys, okeys)
    assert np.array_equal(vals, ovals)


def test_fullsize_sampled_pixels(rig):
    scene, cams, rast, params, out = rig
    keys, vals, csr = rast.debug_binning()
    imgs, T, cnt, last = host_outputs(rast, out)
    rng = np.random.default_rng(3003)
    arrays = scene.arrays()
    checked = 0
    for v, c in enumerate(cams):
        setup = view_setup(arrays, scene.sh_degree, c)
        pix = [(int(rng.integers(0, c.width)), int(rng.integers(0, c.height))) for _ in range(25)]
        # plus the ragged bottom-right corner tile
        pix += [(c.width - 1, c.height - 1), (c.width - 3, c.height - 2)]
        ref = render_pixels(arrays, scene.sh_degree, c, pix, setup=setup)
        lg = last_gaussian(rast, last[v], v, vals, csr)
        for (i, j), r in zip(pix, ref):
            if r["ambiguous"]:
                continue
            assert np.abs(imgs[v][:, j, i] - r["color"]).max() <= 1e-5, (v, i, j)
            assert abs(T[v][j, i] - r["T"]) <= 1e-5
            assert cnt[v][j, i] == r["count"] and lg[j, i] == r["last"], (v, i, j)
            checked += 1
    assert checked >= 150


def test_fullsize_window_gradients(rig):
    scene, cams, rast, params, out = rig
    targets = make_target(3, cams)
    arrays = scene.arrays()
    wins = {0: (700, 732, 430, 462), 3: (200, 232, 600, 632), 5: (1500, 1532, 100, 132)}
    cots = [np.zeros((3, c.height, c.width)) for c in cams]
    total_px = rast.total_px
    for v, (x0, x1, y0, y1) in wins.items():
        fwd = render_view(arrays, scene.sh_degree, cams[v], window=(x0, x1, y0, y1))
        g = np.sign(fwd["image"] - targets[v][:, y0:y1, x0:x1]) / (3.0 * total_px)
        g[:, fwd["ambiguous"]] = 0.0
        cots[v][:, y0:y1, x0:x1] = g
    dl = torch.from_numpy(np.concatenate([c.astype(np.float32).reshape(-1) for c in cots])).cuda()
    gpu = grads_to_host(rast.backward(params, out, dl, cam_grads=True))
    ref = grad64(scene, cams, cots, windows=[wins.get(v) or (0, 0, 0, 0) for v in range(len(cams))],
                 cam_grads=True)
    for k in ref:
        scale = np.abs(ref[k]).max()
        diff = np.abs(gpu[k] - ref[k])
        big = np.abs(ref[k]) >= 1e-2 * scale
        rel = (diff[big] / np.abs(ref[k][big])).max()
        log(f"  grad {k}: {diff.max() / scale:.2e} of max, rel {rel:.2e}")
        assert diff.max() <= 1e-4 * scale, k
        assert rel <= 1e-4, k


def test_fullsize_persistent_schedule_bitwise(rig):
    """The persistent compositing schedule at full size gives the grid
    schedule's images, stop positions, counts and gradients bit for bit."""
    from paper_2512_08498_amd import Rasterizer

    scene, cams, rast, params, out = rig
    rng = np.random.default_rng(77)
    dl = torch.from_numpy(rng.standard_normal(3 * rast.total_px).astype(np.float32) * 1e-6).cuda()
    res = []
    for pers in (False, True):
        r = Rasterizer(cams, scene.n, scene.sh_degree, tile_size=16, persistent=pers,
                       capacity_records=rast.capacity[0], capacity_pairs=rast.capacity[1])
        o = r.forward(params)
        g = r.backward(params, o, dl)
        torch.cuda.synchronize()
        res.append({**{k: o[k].cpu().numpy() for k in ("image", "t_final", "last_pos", "n_contrib")},
                    **{"g_" + k: v.cpu().numpy() for k, v in g.items()}})
        log(f"persistent={pers} done")
        del r, o, g
    for k in res[0]:
        assert np.array_equal(res[0][k], res[1][k]), k
