"""Launch configuration and autotuner (through the C ABI): every work split
of the 16 px backward meets the oracle, the autotuner picks one of its
candidates, caches it by device and batch shape, and the tuned plan renders
the same images as the default one."""
import numpy as np
import pytest
import torch

from gpu_helpers import grads_to_host, log, render_gpu
from oracle.grad64 import grad64
from oracle.render64 import render
from paper_2512_08498_amd import Rasterizer
from test_gpu_parity import _compare_grads, _masked_cotangent
from tiny_scenes import mini_rig
from workloads import make_config, make_target

pytestmark = pytest.mark.gpu

CANDIDATES = {(16, 512), (16, 256), (16, 1024), (16, 0), (16, 0xFFFFFFFF), (8, 512), (32, 512)}


@pytest.mark.parametrize("long_list", [0, 64, 0xFFFFFFFF])
def test_backward_split_variants_cfg1(cfg1, long_list):
    """All tiles walked by four waves, a threshold inside the length range,
    and all tiles walked by one wave each: the same gradients to 1e-4."""
    scene, cams, targets = cfg1
    oracle = render(scene, cams)
    cots = _masked_cotangent(oracle, targets)
    rast, params, out = render_gpu(scene, cams, ts=16, long_list=long_list)
    assert rast.tuning()["long_list"] == long_list
    dl = torch.from_numpy(np.concatenate([c.astype(np.float32).reshape(-1) for c in cots])).cuda()
    grads = grads_to_host(rast.backward(params, out, dl))
    log(f"long_list={long_list}")
    _compare_grads(grads, grad64(scene, cams, cots))


def test_backward_split_variants_rig():
    scene, cams = mini_rig()
    rng = np.random.default_rng(21)
    targets = [rng.uniform(0, 1, (3, c.height, c.width)).astype(np.float32) for c in cams]
    oracle = render(scene, cams)
    cots = _masked_cotangent(oracle, targets)
    ref = grad64(scene, cams, cots)
    dl = torch.from_numpy(np.concatenate([c.astype(np.float32).reshape(-1) for c in cots])).cuda()
    for long_list in (0, 16, 0xFFFFFFFF):
        rast, params, out = render_gpu(scene, cams, ts=16, long_list=long_list)
        log(f"mini rig long_list={long_list}")
        _compare_grads(grads_to_host(rast.backward(params, out, dl)), ref)


def test_autotune_choice_cache_and_images(tmp_path):
    """A scaled-down keyframe window (40 views of mixed resolution)."""
    scene, cams = make_config(4, scale=0.01)
    ref_rast, params, ref_out = render_gpu(scene, cams, ts=16)
    ref_img = ref_out["image"].cpu().numpy()
    del ref_rast, ref_out
    cache = tmp_path / "tune.txt"
    rast = Rasterizer(cams, scene.n, scene.sh_degree, capacity_records=2_000_000, capacity_pairs=8_000_000)
    best = rast.autotune(params, repeats=2, cache=cache)
    log(f"autotune: {best}")
    assert (best["tile_size"], best["long_list"]) in CANDIDATES
    assert best["step_ms"] > 0
    assert rast.tile_size == best["tile_size"]
    assert rast.tuning() == {"tile_size": best["tile_size"], "long_list": best["long_list"]}
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and "views=" in lines[0] and f"tile_size={best['tile_size']}" in lines[0]
    out = rast.forward(params)
    torch.cuda.synchronize()
    assert np.array_equal(out["image"].cpu().numpy(), ref_img)
    # a second context finds the choice in the cache without measuring
    r2 = Rasterizer(cams, scene.n, scene.sh_degree, capacity_records=2_000_000, capacity_pairs=8_000_000)
    again = r2.autotune(params, repeats=2, cache=cache)
    assert (again["tile_size"], again["long_list"]) == (best["tile_size"], best["long_list"])
    assert abs(again["step_ms"] - best["step_ms"]) <= 1e-4  # stored with four decimals
    assert len(cache.read_text().splitlines()) == 1
    out2 = r2.forward(params)
    torch.cuda.synchronize()
    assert np.array_equal(out2["image"].cpu().numpy(), ref_img)


def test_autotune_rejects_bad_arguments(tmp_path):
    from paper_2512_08498_amd._lib import GsrError

    scene, cams = mini_rig()
    rast, params, out = render_gpu(scene, cams)
    with pytest.raises(GsrError):
        rast.autotune(params, repeats=0)
    # the context is planned again after the failed call
    rast.forward(params)
    bad = tmp_path / "bad.txt"
    r2 = Rasterizer(cams, scene.n, scene.sh_degree)
    r2.autotune(params, repeats=1, cache=bad)
    key = bad.read_text().split(" ")[0]
    bad.write_text(key + " tile_size=12 long_list=1 step_ms=1.0\n")
    with pytest.raises(GsrError):
        r2.autotune(params, repeats=1, cache=bad)
