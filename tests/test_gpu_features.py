"""GPU tests of the loss, the optimiser, invariances, the sort size classes,
capacity handling and edge cases (all through the C ABI)."""
import ctypes as C
import math

import numpy as np
import pytest
import torch

from gpu_helpers import compare_grads, device_params, grads_to_host, host_outputs, log, render_gpu
from oracle.adam64 import adam_step
from oracle.binning import tile_lists
from oracle.grad64 import grad64
from oracle.render64 import render
from paper_2512_08498_amd import PARAM_NAMES, FusedAdam, Rasterizer
from paper_2512_08498_amd import _lib as L
from tiny_scenes import camera, logit, mini_rig, scene
from workloads import make_config

pytestmark = pytest.mark.gpu


def test_l1_loss_and_gradient(cfg1):
    scene_, cams, targets = cfg1
    rast, params, out = render_gpu(scene_, cams)
    tgt = torch.from_numpy(targets[0].reshape(-1)).cuda()
    loss, dl = rast.l1_loss(out["image"], tgt)
    img = out["image"].cpu().numpy().astype(np.float64)
    d = img - targets[0].reshape(-1)
    assert abs(loss.item() - np.abs(d).mean()) <= 1e-6 * np.abs(d).mean()
    assert np.array_equal(dl.cpu().numpy(), (np.sign(d) / d.size).astype(np.float32))
    loss2, _ = rast.l1_loss(out["image"], tgt)
    assert loss2.item() == loss.item()  # fixed-order reduction


def _rand_state(scene_, seed):
    rng = np.random.default_rng(seed)
    return {k: rng.standard_normal(v.shape).astype(np.float32) for k, v in scene_.arrays().items()}


def test_adam_matches_oracle_over_steps(cfg1):
    scene_, cams, _ = cfg1
    rast = Rasterizer(cams, scene_.n, scene_.sh_degree)
    params = device_params(scene_)
    lr = (1e-3, 2e-3, 3e-3, 4e-3, 5e-3, 6e-3)
    opt = FusedAdam(rast, params, lr=lr)
    p = {k: v.astype(np.float64) for k, v in scene_.arrays().items()}
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v_ = {k: np.zeros_like(v) for k, v in p.items()}
    groups = dict(mean=0, log_scale=1, quat=2, opacity_logit=3)
    for it in range(4):
        g = _rand_state(scene_, 100 + it)
        opt.apply({k: torch.from_numpy(x).cuda() for k, x in g.items()})
        for k in PARAM_NAMES:
            if k == "sh":
                n = scene_.n
                flat_p, flat_g = p[k].reshape(-1), g[k].astype(np.float64).reshape(-1)
                fm, fv = m[k].reshape(-1), v_[k].reshape(-1)
                a = adam_step(flat_p[:3 * n], flat_g[:3 * n], fm[:3 * n], fv[:3 * n], it, lr[4])
                b = adam_step(flat_p[3 * n:], flat_g[3 * n:], fm[3 * n:], fv[3 * n:], it, lr[5])
                p[k] = np.concatenate([a[0], b[0]]).reshape(p[k].shape)
                m[k] = np.concatenate([a[1], b[1]]).reshape(p[k].shape)
                v_[k] = np.concatenate([a[2], b[2]]).reshape(p[k].shape)
            else:
                p[k], m[k], v_[k] = adam_step(p[k], g[k].astype(np.float64), m[k], v_[k], it, lr[groups[k]])
    torch.cuda.synchronize()
    assert int(opt.step.item()) == 4
    for k in PARAM_NAMES:
        got = params[k].cpu().numpy().astype(np.float64)
        step_scale = max(lr)
        assert np.abs(got - p[k]).max() <= 1e-5 * step_scale + 1e-6 * np.abs(p[k]).max(), k


@pytest.mark.parametrize("degree", [3, 2, 1, 0])
def test_fused_backward_adam_equals_backward_then_adam(degree):
    """The fused step against the backward followed by the separate Adam
    kernel, at every SH degree (the fused kernel updates the coefficients in
    groups whose loads overlap the previous group's stores)."""
    scene_, cams = mini_rig(degree=degree)
    rng = np.random.default_rng(5)
    rast, params, out = render_gpu(scene_, cams)
    dl = torch.from_numpy(rng.standard_normal(3 * rast.total_px).astype(np.float32) * 1e-4).cuda()
    grads = rast.backward(params, out, dl)
    p1 = {k: v.clone() for k, v in params.items()}
    opt1 = FusedAdam(rast, p1)
    opt1.apply(grads)
    p2 = {k: v.clone() for k, v in params.items()}
    opt2 = FusedAdam(rast, p2)
    g_out = {k: torch.empty_like(v) for k, v in params.items()}
    rast.backward_adam(p2, out, dl, opt2, grads_out=g_out)
    torch.cuda.synchronize()
    for k in PARAM_NAMES:
        assert torch.equal(g_out[k], grads[k]), k
        assert torch.allclose(p1[k], p2[k], rtol=0, atol=1e-7), k
        assert torch.equal(opt1.m[k], opt2.m[k]), k


@pytest.mark.parametrize("degree", [3, 2])
def test_fused_adam_into_separate_parameter_arrays(degree):
    """The fused step may update parameter arrays other than the rendered
    Gaussians' own (holding the same values): the result equals the
    in-place update bit for bit, so the kernel's reuse of the values it has
    already loaded is only taken when the arrays are the same."""
    scene_, cams = mini_rig(degree=degree)
    rng = np.random.default_rng(6)
    rast, params, out = render_gpu(scene_, cams)
    dl = torch.from_numpy(rng.standard_normal(3 * rast.total_px).astype(np.float32) * 1e-4).cuda()
    p_in = {k: v.clone() for k, v in params.items()}
    opt_in = FusedAdam(rast, p_in)
    rast.backward_adam(p_in, out, dl, opt_in)
    p_sep = {k: v.clone() for k, v in params.items()}
    opt_sep = FusedAdam(rast, p_sep)
    lib = rast.lib
    st = lib.gsr_render_backward_adam(
        rast.ctx, C.byref(rast._gaussians(params)), C.c_void_p(rast.cams_dev.data_ptr()), rast.views,
        C.c_void_p(rast.workspace.data_ptr()), rast.ws_bytes, C.byref(rast._fwd_struct(out)),
        C.c_void_p(dl.data_ptr()), C.byref(opt_sep.param_struct(p_sep)), C.byref(opt_sep.m_struct()),
        C.byref(opt_sep.v_struct()), C.byref(opt_sep.config), C.c_void_p(opt_sep.step.data_ptr()), None,
        rast.stream())
    assert st == 0
    torch.cuda.synchronize()
    for k in PARAM_NAMES:
        assert torch.equal(p_in[k], p_sep[k]), k
        assert torch.equal(opt_in.m[k], opt_sep.m[k]) and torch.equal(opt_in.v[k], opt_sep.v[k]), k


def test_forward_bitwise_invariant_to_tile_size_and_repeatable(cfg1):
    scene_, cams, _ = cfg1
    ref = None
    for ts in (16, 8, 32, 16):
        rast, params, out = render_gpu(scene_, cams, ts=ts)
        cur = (out["image"].cpu().numpy(), out["t_final"].cpu().numpy(), out["n_contrib"].cpu().numpy())
        if ref is None:
            ref = cur
        for a, b in zip(ref, cur):
            assert np.array_equal(a, b), ts


def test_batched_equals_per_view_bitwise():
    scene_, cams = make_config(3, scale=0.01)
    rast, params, out = render_gpu(scene_, cams)
    imgs = [x.cpu().numpy() for x in rast.view_images(out["image"])]
    rng = np.random.default_rng(9)
    dl = torch.from_numpy(rng.standard_normal(3 * rast.total_px).astype(np.float32) * 1e-5).cuda()
    g_b = grads_to_host(rast.backward(params, out, dl))
    g_sum = {k: np.zeros_like(v) for k, v in g_b.items()}
    for v, c in enumerate(cams):
        r1, p1, o1 = render_gpu(scene_, [c])
        assert np.array_equal(r1.view_images(o1["image"])[0].cpu().numpy(), imgs[v]), v
        g1 = grads_to_host(r1.backward(p1, o1, dl[3 * rast.pix_off[v]:3 * rast.pix_off[v + 1]].contiguous()))
        for k in g_sum:
            g_sum[k] += g1[k]
    for k in g_b:
        scale = np.abs(g_b[k]).max()
        assert np.abs(g_b[k] - g_sum[k]).max() <= 1e-5 * scale, k


def test_backward_is_deterministic():
    scene_, cams = mini_rig()
    rast, params, out = render_gpu(scene_, cams)
    dl = torch.from_numpy(np.random.default_rng(1).standard_normal(3 * rast.total_px).astype(np.float32)).cuda()
    a = rast.backward(params, out, dl)
    b = rast.backward(params, out, dl)
    torch.cuda.synchronize()
    for k in PARAM_NAMES:
        assert torch.equal(a[k], b[k]), k


@pytest.mark.parametrize("persistent", [False, True])
def test_graph_replays_match_eager(persistent):
    scene_, cams = make_config(3, scale=0.005)
    rast, params, _ = render_gpu(scene_, cams, persistent=persistent)
    out = rast.new_fwd_out()
    dl = torch.from_numpy(np.random.default_rng(2).standard_normal(3 * rast.total_px).astype(np.float32)).cuda()
    grads = {k: torch.empty_like(v) for k, v in params.items()}

    def step():
        rast.forward(params, out=out, check=False)
        rast.backward(params, out, dl, grads=grads)

    step()
    torch.cuda.synchronize()
    ref_img = out["image"].clone()
    ref_g = {k: v.clone() for k, v in grads.items()}
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    for rep in range(4):
        out["image"].zero_()
        for v in grads.values():
            v.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out["image"], ref_img), rep
        for k in PARAM_NAMES:
            assert torch.equal(grads[k], ref_g[k]), (rep, k)
        step()  # eager work between replays
        torch.cuda.synchronize()


# (case, tile size, copies of the six 1600x900 cameras): the tile sort takes
# 8-bit passes up to 2^16 tiles, two 9- or 10-bit passes up to 2^20 tiles and
# 8-bit passes beyond.
PASS_CASES = {
    "one_8bit": (16, 0),        # 12 tiles, one camera
    "two_8bit": (16, 1),        # 34,200 tiles
    "two_9bit": (8, 1),         # 135,600 tiles
    "two_10bit": (8, 2),        # 271,200 tiles
    "three_8bit": (8, 8),       # 1,084,800 tiles
}


@pytest.mark.parametrize("case", list(PASS_CASES))
def test_tile_sort_pass_counts_bit_exact(case):
    """Tile lists bit-exact against the oracle at each digit plan of the tile
    sort, and the image equal to the one binned at 32 px."""
    ts, copies = PASS_CASES[case]
    if copies == 0:
        scene_, cams = make_config(1)
    else:
        scene_, cams = make_config(3, scale=0.01)
        cams = cams * copies
    rast, params, out = render_gpu(scene_, cams, ts=ts)
    log(f"{case}: {rast.required_capacity()[2]} tiles")
    keys, vals, csr = rast.debug_binning()
    okeys, ovals, ocsr = tile_lists(scene_, cams, ts)
    assert np.array_equal(keys, okeys) and np.array_equal(vals, ovals) and np.array_equal(csr, ocsr)
    ref, _, ref_out = render_gpu(scene_, cams, ts=32)
    assert torch.equal(out["image"], ref_out["image"])


def test_sort_orders_equal_depths_by_gaussian_index():
    # 40 Gaussians at identical depth: every list is one long tie
    n = 40
    rng = np.random.default_rng(4)
    means = np.stack([rng.uniform(-0.5, 0.5, n), rng.uniform(-0.4, 0.4, n), np.full(n, 3.0)], 1)
    sc = scene(means, np.full((n, 3), -2.0), [[1, 0, 0, 0]] * n, rng.normal(0, 1, n),
               colours=rng.uniform(0, 1, (n, 3)))
    cams = [camera(60.0)]
    for ts in (8, 16, 32):
        rast, params, out = render_gpu(sc, cams, ts=ts)
        keys, vals, csr = rast.debug_binning()
        okeys, ovals, ocsr = tile_lists(sc, cams, ts)
        assert np.array_equal(keys, okeys) and np.array_equal(vals, ovals)


def test_capacity_overflow_reports_and_retries(cfg1):
    scene_, cams, _ = cfg1
    rast = Rasterizer(cams, scene_.n, scene_.sh_degree, capacity_records=10, capacity_pairs=10)
    params = device_params(scene_)
    out = rast.new_fwd_out()
    rast.forward(params, out=out, check=False)
    with pytest.raises(L.GsrError) as e:
        rast.check()
    assert e.value.status == L.GSR_ERR_CAPACITY
    rec, pairs, _ = rast.required_capacity()
    assert rec > 10 and pairs > 10
    out2 = rast.forward(params)  # re-plans and renders again
    ref = render(scene_, cams)[0]
    img = rast.view_images(out2["image"])[0].cpu().numpy()
    ok = ~ref["ambiguous"]
    assert np.abs(img - ref["image"])[:, ok].max() <= 1e-5


def test_abi_rejects_invalid_arguments(cfg1):
    scene_, cams, _ = cfg1
    rast = Rasterizer(cams, scene_.n, scene_.sh_degree)
    lib = rast.lib
    import ctypes as C
    bad = (L.Camera * 1)()
    C.memmove(bad, np.zeros(18, np.float32).ctypes.data, 72)
    ws, pix = C.c_size_t(), (C.c_int64 * 2)()
    opts = L.PlanOptions(16, 0, 0, (C.c_float * 3)(0, 0, 0))
    assert lib.gsr_plan(rast.ctx, bad, 1, 10, 0, C.byref(opts), C.byref(ws), pix) == L.GSR_ERR_INVALID_ARG
    good = rast._cams_host
    assert lib.gsr_plan(rast.ctx, good, 0, 10, 0, C.byref(opts), C.byref(ws), pix) == L.GSR_ERR_INVALID_ARG
    assert lib.gsr_plan(rast.ctx, good, 1, 10, 4, C.byref(opts), C.byref(ws), pix) == L.GSR_ERR_UNSUPPORTED
    opts.tile_size = 12
    assert lib.gsr_plan(rast.ctx, good, 1, 10, 0, C.byref(opts), C.byref(ws), pix) == L.GSR_ERR_INVALID_ARG
    # a render against a stale plan and a short workspace
    rast2 = Rasterizer(cams, scene_.n, scene_.sh_degree)
    params = device_params(scene_)
    g = rast2._gaussians(params)
    out = rast2.new_fwd_out()
    fo = rast2._fwd_struct(out)
    st = lib.gsr_render_forward(rast2.ctx, C.byref(g), C.c_void_p(rast2.cams_dev.data_ptr()), 1,
                                C.c_void_p(rast2.workspace.data_ptr()), 16, C.byref(fo), rast2.stream())
    assert st == L.GSR_ERR_INVALID_ARG and b"workspace" in lib.gsr_last_error(rast2.ctx)
    g.n = scene_.n + 1
    st = lib.gsr_render_forward(rast2.ctx, C.byref(g), C.c_void_p(rast2.cams_dev.data_ptr()), 1,
                                C.c_void_p(rast2.workspace.data_ptr()), rast2.ws_bytes, C.byref(fo), rast2.stream())
    assert st == L.GSR_ERR_NOT_PLANNED
    assert lib.gsr_set_tuning(rast2.ctx, C.byref(L.Tuning(12, 512, 0, 0.0))) == L.GSR_ERR_INVALID_ARG


def _edge_check(sc, cams, ts=16):
    rast, params, out = render_gpu(sc, cams, ts=ts)
    ora = render(sc, cams)
    imgs, T, cnt, _ = host_outputs(rast, out)
    for v in range(len(cams)):
        ok = ~ora[v]["ambiguous"]
        assert np.abs(imgs[v] - ora[v]["image"])[:, ok].max(initial=0.0) <= 1e-5
        assert np.array_equal(cnt[v][ok], ora[v]["count"][ok])
    if sc.n:
        keys, vals, csr = rast.debug_binning()
        okeys, ovals, ocsr = tile_lists(sc, cams, ts)
        assert np.array_equal(keys, okeys) and np.array_equal(vals, ovals) and np.array_equal(csr, ocsr)
        # gradients against the oracle's, under a random cotangent masked to
        # the non-ambiguous pixels (all zero where nothing composites)
        rng = np.random.default_rng(sc.n + 7 * ts)
        cots = [np.where(o["ambiguous"][None], 0.0,
                         (rng.standard_normal((3, c.height, c.width)) * 1e-3).astype(np.float32).astype(np.float64))
                for o, c in zip(ora, cams)]
        dl = torch.from_numpy(np.concatenate([c.astype(np.float32).reshape(-1) for c in cots])).cuda()
        grads = grads_to_host(rast.backward(params, out, dl))
        compare_grads(grads, grad64(sc, cams, cots))
    return rast


def test_edge_empty_scene():
    sc = scene(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 4)), np.zeros(0), colours=np.zeros((0, 3)))
    rast = _edge_check(sc, [camera(60.0, 37, 29)])
    assert rast.required_capacity()[:2] == (0, 0)


def test_edge_all_culled_and_degenerate_inputs():
    sc = scene([[0, 0, -2.0], [0, 0, 0.1], [50, 0, 2.0], [0, 0, 3.0], [0.2, 0, 3.0], [0, 0.1, 4.0]],
               [[-2.0] * 3, [-2.0] * 3, [-2.0] * 3, [-2.0] * 3, [5.0, -20.0, -3.0], [-20.0] * 3],
               [[1, 0, 0, 0], [1, 0, 0, 0], [1, 0, 0, 0], [0, 0, 0, 0], [1, 0, 0, 0], [1, 0, 0, 0]],
               [0.0] * 6, colours=[[0.5] * 3] * 6)
    _edge_check(sc, [camera(60.0)])


@pytest.mark.parametrize("wh", [(1, 1), (37, 29), (17, 100)])
@pytest.mark.parametrize("ts", [8, 16, 32])
def test_edge_ragged_and_tiny_images(wh, ts):
    w, h = wh
    rng = np.random.default_rng(w * 131 + h)
    n = 150
    means = np.stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(2, 6, n)], 1)
    q = rng.standard_normal((n, 4))
    sc = scene(means, rng.normal(-2.5, 0.5, (n, 3)), q, rng.normal(0, 1.5, n), colours=rng.uniform(0, 1, (n, 3)))
    _edge_check(sc, [camera(40.0, w, h)], ts=ts)


def test_edge_screen_filling_gaussians_and_stack():
    n = 30
    sc = scene([[0, 0, 3.0 + 0.01 * i] for i in range(n)], [[0.5, 0.4, 0.3]] * n, [[1, 0, 0, 0]] * n,
               [logit(0.3)] * n, colours=[[0.2 + 0.02 * i, 0.5, 0.7] for i in range(n)])
    _edge_check(sc, [camera(60.0, 96, 64)])


@pytest.mark.parametrize("ts", [8, 16, 32])
def test_forward_with_fused_l1_loss(ts):
    """gsr_render_forward_l1: the same image and dL/dimage bit for bit as
    the forward followed by gsr_l1_loss, and the same loss up to the order of
    the float sums; against the oracle's loss on its own image."""
    from oracle.loss64 import l1_loss
    from oracle.render64 import render

    scene, cams = mini_rig()
    rng = np.random.default_rng(77)
    targets = [rng.uniform(0, 1, (3, c.height, c.width)).astype(np.float32) for c in cams]
    tgt = torch.from_numpy(np.concatenate([t.reshape(-1) for t in targets])).cuda()
    rast, params, out = render_gpu(scene, cams, ts=ts, bg=(0.1, 0.2, 0.3))
    loss_a, dl_a = rast.l1_loss(out["image"], tgt)
    out_b, loss_b, dl_b = rast.forward_l1(params, tgt)
    torch.cuda.synchronize()
    assert torch.equal(out_b["image"], out["image"])
    assert torch.equal(out_b["t_final"], out["t_final"])
    assert torch.equal(dl_b, dl_a)
    assert abs(loss_b.item() - loss_a.item()) <= 1e-6 * abs(loss_a.item())
    ref = render(scene, cams, bg=(0.1, 0.2, 0.3))
    ref_loss, _ = l1_loss([r["image"] for r in ref], targets)
    log(f"ts {ts}: fused {loss_b.item():.8f}, separate {loss_a.item():.8f}, oracle {ref_loss:.8f}")
    assert abs(loss_b.item() - ref_loss) <= 1e-5 * ref_loss


def test_streaming_copy():
    """The bandwidth reference copy moves every byte, tails included, and
    rejects sizes that are not a multiple of 16 bytes."""
    from paper_2512_08498_amd import device_copy
    from paper_2512_08498_amd._lib import GsrError

    for n in (4, 1028, 3 * 2**20 + 12):
        src = torch.randint(-2**31, 2**31 - 1, (n,), dtype=torch.int32, device="cuda")
        dst = torch.zeros_like(src)
        device_copy(dst, src)
        torch.cuda.synchronize()
        assert torch.equal(dst, src)
    with pytest.raises(GsrError):
        device_copy(torch.zeros(3, dtype=torch.int32, device="cuda"), torch.zeros(3, dtype=torch.int32, device="cuda"))


def test_overflowed_step_leaves_adam_state_untouched(cfg1):
    """A fused backward + Adam step after a forward that overflowed its
    capacity (as a graph replay with no check would run it) updates nothing:
    not the parameters, not the moments and not the step counter, so the
    bias correction stays in step with the moments."""
    scene_, cams, _ = cfg1
    rast = Rasterizer(cams, scene_.n, scene_.sh_degree, capacity_records=10, capacity_pairs=10)
    params = device_params(scene_)
    before = {k: v.clone() for k, v in params.items()}
    opt = FusedAdam(rast, params)
    out = rast.new_fwd_out()
    rast.forward(params, out=out, check=False)
    dl = torch.full((3 * rast.total_px,), 1e-3, device="cuda")
    rast.backward_adam(params, out, dl, opt)
    torch.cuda.synchronize()
    assert int(opt.step.item()) == 0
    for k in PARAM_NAMES:
        assert torch.equal(params[k], before[k]), k
        assert not opt.m[k].any() and not opt.v[k].any(), k
    with pytest.raises(L.GsrError):
        rast.check()
