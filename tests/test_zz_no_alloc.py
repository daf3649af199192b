"""gsr_render_forward_noalloc through the C ABI: the forward with its
workspace in the library's per-GPU device scratch reproduces
gsr_render_forward (caller workspace) bit for bit, on two calls in a row
(the second with a smaller input, over what the first left in the
scratch), reports a capacity overflow through gsr_check(ctx, NULL), and
rejects a plan larger than the scratch."""
import ctypes as C

import numpy as np
import pytest
import torch

from gpu_helpers import device_params, log
from oracle.render64 import render
from paper_2512_08498_amd import Rasterizer
from paper_2512_08498_amd import _lib as L
from tiny_scenes import camera, mini_rig
from workloads import make_config

pytestmark = pytest.mark.gpu

SCRATCH = 64 << 20


def _noalloc(rast, params):
    """The entry point called through ctypes on the rasterizer's context
    and plan, into freshly allocated outputs."""
    out = {k: torch.full_like(v, 7) for k, v in rast.new_fwd_out().items()}
    g = rast._gaussians(params)
    st = rast.lib.gsr_render_forward_noalloc(rast.ctx, C.byref(g), C.c_void_p(rast.cams_dev.data_ptr()), rast.views,
                                             C.byref(rast._fwd_struct(out)), rast.stream())
    assert st == L.GSR_OK, rast.lib.gsr_last_error(rast.ctx)
    return out


def _same(a, b):
    for k in ("image", "t_final", "last_pos", "n_contrib"):
        assert torch.equal(a[k], b[k]), k


def test_noalloc_forward_equals_the_workspace_forward_twice():
    scene1, cams1 = make_config(1)
    scene2, cams2 = mini_rig(seed=9, n=200, w=48, h=40)
    results = []
    for scene, cams in ((scene1, cams1), (scene2, cams2)):
        rast = Rasterizer(cams, scene.n, scene.sh_degree)
        assert rast.ws_bytes <= SCRATCH
        params = device_params(scene)
        got = _noalloc(rast, params)
        torch.cuda.synchronize()
        rast.check_noalloc()
        ref = rast.forward(params)
        torch.cuda.synchronize()
        _same(got, ref)
        results.append((rast, got))
        log(f"{scene.n} Gaussians, {len(cams)} views, plan workspace {rast.ws_bytes} bytes: bitwise equal")
    # the smaller second call is also right against the oracle
    rast, got = results[1]
    ora = render(scene2, cams2)
    for v, img in enumerate(rast.view_images(got["image"])):
        ok = ~ora[v]["ambiguous"]
        assert np.abs(img.cpu().numpy().astype(np.float64) - ora[v]["image"])[:, ok].max() <= 1e-5


def test_noalloc_capacity_overflow_is_reported_through_the_scratch():
    scene, cams = make_config(1)
    rast = Rasterizer(cams, scene.n, scene.sh_degree, capacity_records=10, capacity_pairs=10)
    _noalloc(rast, device_params(scene))
    with pytest.raises(L.GsrError) as e:
        rast.check_noalloc()
    assert e.value.status == L.GSR_ERR_CAPACITY
    rec, pairs, _ = (C.c_int64(), C.c_int64(), C.c_int64())
    assert rast.lib.gsr_required_capacity(rast.ctx, None, C.byref(rec), C.byref(pairs), None, rast.stream()) == 0
    assert rec.value > 10 and pairs.value > 10


def test_noalloc_rejects_a_plan_larger_than_the_scratch():
    n = 1000
    rng = np.random.default_rng(3)
    from tiny_scenes import scene as make_scene

    sc = make_scene(np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(2, 6, n)], 1),
                    rng.normal(-3, 0.3, (n, 3)), rng.standard_normal((n, 4)), rng.normal(0, 1, n),
                    colours=rng.uniform(0, 1, (n, 3)))
    rast = Rasterizer([camera(60.0)], n, 0, capacity_pairs=4_000_000)
    assert rast.ws_bytes > SCRATCH
    out = rast.new_fwd_out()
    g = rast._gaussians(device_params(sc))
    st = rast.lib.gsr_render_forward_noalloc(rast.ctx, C.byref(g), C.c_void_p(rast.cams_dev.data_ptr()), 1,
                                             C.byref(rast._fwd_struct(out)), rast.stream())
    assert st == L.GSR_ERR_CAPACITY
    assert b"no-alloc scratch" in rast.lib.gsr_last_error(rast.ctx)
