"""Shared helpers of the GPU tests: move a scene to the device, run the HIP
path through the binding, and map its per-pixel state back to Gaussians."""
import sys

import numpy as np
import torch

from paper_2512_08498_amd import PARAM_NAMES, Rasterizer


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def device_params(scene, device="cuda"):
    return {k: torch.from_numpy(np.ascontiguousarray(v)).to(device) for k, v in scene.arrays().items()}


def render_gpu(scene, cams, ts=16, bg=(0.0, 0.0, 0.0), **kw):
    rast = Rasterizer(cams, scene.n, scene.sh_degree, tile_size=ts, bg=bg, **kw)
    params = device_params(scene)
    out = rast.forward(params)
    torch.cuda.synchronize()
    return rast, params, out


def host_outputs(rast, out):
    imgs = [x.cpu().numpy().astype(np.float64) for x in rast.view_images(out["image"])]
    T = [x.cpu().numpy().astype(np.float64) for x in rast.view_maps(out["t_final"])]
    cnt = [x.cpu().numpy() for x in rast.view_maps(out["n_contrib"])]
    last = [x.cpu().numpy() for x in rast.view_maps(out["last_pos"])]
    return imgs, T, cnt, last


def last_gaussian(rast, last_pos_v, v, vals, csr):
    """Gaussian index of each pixel's last composited entry (-1 if none)."""
    ts = rast.tile_size
    w, h = rast.sizes[v]
    base = 0
    for u in range(v):
        wu, hu = rast.sizes[u]
        base += ((wu + ts - 1) // ts) * ((hu + ts - 1) // ts)
    tx_n = (w + ts - 1) // ts
    jj, ii = np.mgrid[0:h, 0:w]
    tile = base + (jj // ts) * tx_n + ii // ts
    lp = last_pos_v.astype(np.int64)
    idx = csr[tile] + lp - 1
    out = np.where(lp > 0, vals[np.clip(idx, 0, max(len(vals) - 1, 0))].astype(np.int64) if len(vals) else -1, -1)
    return out


def grads_to_host(grads):
    """Gaussian gradients, and the views' pose gradients as "cam" when present."""
    out = {k: grads[k].cpu().numpy().astype(np.float64) for k in PARAM_NAMES}
    if "camera" in grads:
        out["cam"] = grads["camera"].cpu().numpy().astype(np.float64)
    return out


def compare_grads(gpu, ora, tol=1e-4):
    """Gradient bar: per group, max |gpu - oracle| <= tol * max |oracle|, and
    tol relative elementwise on entries of at least 1e-2 of that maximum; a
    group that is zero in the oracle must be exactly zero."""
    for k in ora:
        scale = np.abs(ora[k]).max()
        if scale == 0:
            assert np.abs(gpu[k]).max() == 0, k
            continue
        diff = np.abs(gpu[k] - ora[k])
        big = np.abs(ora[k]) >= 1e-2 * scale
        rel = (diff[big] / np.abs(ora[k][big])).max() if big.any() else 0.0
        log(f"  grad {k}: max |diff|/max|g| {diff.max() / scale:.2e}, max rel (big) {rel:.2e}")
        assert diff.max() <= tol * scale, k
        assert rel <= tol, k
