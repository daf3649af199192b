"""Launch configuration and autotuner (through the C ABI): every work split
of the 16 px backward meets the oracle, the persistent schedule gives the
grid schedule's results bit for bit, the autotuner picks one of its
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

CANDIDATES = {(ts, ll, pers) for pers in (False, True)
              for ts, ll in [(16, 512), (16, 256), (16, 1024), (16, 0), (16, 0xFFFFFFFF), (8, 512), (32, 512)]}


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
    choice = (best["tile_size"], best["long_list"], best["persistent"])
    assert choice in CANDIDATES
    assert best["step_ms"] > 0
    assert rast.tile_size == best["tile_size"]
    assert rast.tuning() == {"tile_size": best["tile_size"], "long_list": best["long_list"],
                             "persistent": best["persistent"]}
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and "views=" in lines[0] and f"tile_size={best['tile_size']}" in lines[0]
    assert f"persistent={int(best['persistent'])}" in lines[0]
    out = rast.forward(params)
    torch.cuda.synchronize()
    assert np.array_equal(out["image"].cpu().numpy(), ref_img)
    # a second context finds the choice in the cache without measuring
    r2 = Rasterizer(cams, scene.n, scene.sh_degree, capacity_records=2_000_000, capacity_pairs=8_000_000)
    again = r2.autotune(params, repeats=2, cache=cache)
    assert (again["tile_size"], again["long_list"], again["persistent"]) == choice
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
    for line in ("tile_size=12 long_list=1 persistent=0 step_ms=1.0", "tile_size=16 long_list=1 persistent=2 "
                 "step_ms=1.0", "tile_size=16 long_list=1 step_ms=1.0"):
        bad.write_text(key + " " + line + "\n")
        with pytest.raises(GsrError):
            r2.autotune(params, repeats=1, cache=bad)


def _all_outputs(rast, params, dl, target):
    """Forward, forward with the fused L1 loss, and two backwards in a row
    (the second starts from the work queue the first left behind)."""
    out = rast.forward(params)
    res = {k: out[k].cpu().numpy() for k in ("image", "t_final", "last_pos", "n_contrib")}
    out_l1, loss, dl_dimage = rast.forward_l1(params, target)
    g1 = rast.backward(params, out_l1, dl)
    g2 = rast.backward(params, out_l1, dl)
    torch.cuda.synchronize()
    res["loss"] = loss.cpu().numpy()
    res["dl_dimage"] = dl_dimage.cpu().numpy()
    for k, v in g1.items():
        res["g_" + k] = v.cpu().numpy()
        assert torch.equal(v, g2[k]), k
    return res


@pytest.mark.parametrize("ts,long_list", [(16, 1024), (16, 0), (16, 64), (8, 512), (32, 512)])
def test_persistent_schedule_equals_grid_bitwise(ts, long_list):
    """Every tile is walked by the same code whichever workgroup takes it,
    the loss keeps one partial per tile and the gradients one slot per
    (record, tile), so the two schedules agree bit for bit."""
    from workloads import make_config as mk
    scene, cams = mk(3, scale=0.01)
    params = None
    res = []
    for pers in (False, True):
        rast = Rasterizer(cams, scene.n, scene.sh_degree, tile_size=ts, long_list=long_list, persistent=pers)
        assert rast.tuning()["persistent"] == pers
        if params is None:
            from gpu_helpers import device_params
            params = device_params(scene)
            rng = np.random.default_rng(5)
            dl = torch.from_numpy(rng.standard_normal(3 * rast.total_px).astype(np.float32) * 1e-4).cuda()
            target = torch.from_numpy(rng.uniform(0, 1, 3 * rast.total_px).astype(np.float32)).cuda()
        log(f"schedule ts={ts} long_list={long_list} persistent={pers}")
        res.append(_all_outputs(rast, params, dl, target))
    for k in res[0]:
        assert np.array_equal(res[0][k], res[1][k]), k


def test_persistent_schedule_meets_the_oracle(cfg1):
    scene, cams, targets = cfg1
    oracle = render(scene, cams)
    cots = _masked_cotangent(oracle, targets)
    rast, params, out = render_gpu(scene, cams, ts=16, long_list=64, persistent=True)
    for v in range(len(cams)):
        ok = ~oracle[v]["ambiguous"]
        img = rast.view_images(out["image"])[v].cpu().numpy().astype(np.float64)
        assert np.abs(img - oracle[v]["image"])[:, ok].max(initial=0.0) <= 1e-5
    dl = torch.from_numpy(np.concatenate([c.astype(np.float32).reshape(-1) for c in cots])).cuda()
    _compare_grads(grads_to_host(rast.backward(params, out, dl)), grad64(scene, cams, cots))
