"""LoG-based insertion through the C ABI against the FP64 oracle
(oracle/insert64.py): P(I) and P(I~) per pixel within 1e-5, the insertion
mask bit for bit on pixels whose P_a is not within 1e-5 of tau_a, the list of
inserting pixels in ascending order (the same list up to such pixels), and
their scales and centres within 1e-5 relative; on small views of mixed size,
for several sigma, at capacity overflow, and on the rig's six 1600x900 views.
Inputs are seeded synthetic images (workloads.make_insert_inputs)."""
import numpy as np
import pytest
import torch

from gpu_helpers import log
from oracle.insert64 import insert
from paper_2512_08498_amd import Rasterizer
from paper_2512_08498_amd._lib import GsrError
from tiny_scenes import camera
from workloads import make_config, make_insert_inputs

pytestmark = pytest.mark.gpu

P_TOL = 1e-5


def _cams(sizes, seed):
    rng = np.random.default_rng(seed)
    cams = []
    for w, h in sizes:
        a = rng.uniform(-0.3, 0.3)
        R = np.array([[np.cos(a), 0, np.sin(a)], [0, 1, 0], [-np.sin(a), 0, np.cos(a)]])
        cams.append(camera(f=0.8 * w, w=w, h=h, R=R, t=rng.uniform(-0.5, 0.5, 3), fy=0.8 * w + 1.5))
    return cams


def _run(cams, gts, rds, depths, sigma=1.0, tau=0.2, capacity=None):
    rast = Rasterizer(cams, 1, 0)
    cu = lambda arrs: torch.from_numpy(np.concatenate([a.reshape(-1) for a in arrs])).cuda()  # noqa: E731
    res = rast.log_insert(cu(gts), cu(rds), cu(depths), sigma=sigma, tau_a=tau, capacity=capacity, p_render=True)
    torch.cuda.synchronize()
    return rast, res


def _check(cams, gts, rds, depths, sigma=1.0, tau=0.2):
    rast, res = _run(cams, gts, rds, depths, sigma, tau)
    p_gt = res["p_gt"].cpu().numpy().astype(np.float64)
    p_rd = res["p_render"].cpu().numpy().astype(np.float64)
    n = int(res["count"].item())
    pix = res["pix"][:n].cpu().numpy().astype(np.int64)
    scale = res["scale"][:n].cpu().numpy().astype(np.float64)
    mean = res["mean"][:n].cpu().numpy().astype(np.float64)
    assert np.all(np.diff(pix) > 0)
    ref_pix, ref_scale, ref_mean, amb_pix = [], [], [], []
    for v, c in enumerate(cams):
        o = insert(gts[v], rds[v], depths[v], c, sigma=sigma, tau_a=tau)
        lo, hi = rast.pix_off[v], rast.pix_off[v + 1]
        assert np.abs(p_gt[lo:hi] - o["p_gt"].reshape(-1)).max() <= P_TOL
        assert np.abs(p_rd[lo:hi] - o["p_render"].reshape(-1)).max() <= P_TOL
        ref_pix.append(o["pix"] + lo)
        ref_scale.append(o["scale"])
        ref_mean.append(o["mean"])
        amb_pix.append(np.nonzero(o["ambiguous"].reshape(-1))[0] + lo)
    ref_pix = np.concatenate(ref_pix)
    ref_scale = np.concatenate(ref_scale)
    ref_mean = np.concatenate(ref_mean)
    amb = set(np.concatenate(amb_pix).tolist())
    gpu_set, ref_set = set(pix.tolist()), set(ref_pix.tolist())
    assert (gpu_set ^ ref_set) <= amb, sorted(gpu_set ^ ref_set)[:10]
    common = np.intersect1d(pix, ref_pix)
    gi = np.searchsorted(pix, common)
    ri = np.searchsorted(ref_pix, common)
    if len(common):
        assert np.abs(scale[gi] - ref_scale[ri]).max() <= 1e-5 * np.abs(ref_scale[ri]).max()
        assert np.abs(mean[gi] - ref_mean[ri]).max() <= 1e-5 * max(1.0, np.abs(ref_mean[ri]).max())
    log(f"{len(cams)} views: {n} inserting pixels (oracle {len(ref_pix)}, {len(amb)} ambiguous)")
    return n


@pytest.mark.parametrize("sigma,tau", [(0.7, 0.2), (1.0, 0.2), (1.0, 0.1), (5.0 / 3.0, 0.03)])
def test_insert_small_views(sigma, tau):
    """A wider Gaussian responds less to the same detail: its threshold is lowered so pixels still insert."""
    sizes = [(96, 64), (37, 23), (130, 70), (5, 3)]
    cams = _cams(sizes, 90)
    gts, rds, depths = make_insert_inputs(sizes, 91)
    assert _check(cams, gts, rds, depths, sigma=sigma, tau=tau) > 50


def test_insert_capacity_overflow_and_determinism():
    sizes = [(96, 64), (64, 48)]
    cams = _cams(sizes, 92)
    gts, rds, depths = make_insert_inputs(sizes, 93)
    _, full = _run(cams, gts, rds, depths)
    n = int(full["count"].item())
    assert n > 20
    _, part = _run(cams, gts, rds, depths, capacity=n // 3)
    assert int(part["count"].item()) == n
    k = n // 3
    assert torch.equal(part["pix"][:k], full["pix"][:k])
    assert torch.equal(part["scale"][:k], full["scale"][:k])
    assert torch.equal(part["mean"][:k], full["mean"][:k])
    _, again = _run(cams, gts, rds, depths)
    for key in ("p_gt", "p_render", "pix", "scale", "mean", "count"):
        assert torch.equal(again[key][:n] if key in ("pix", "scale", "mean") else again[key],
                           full[key][:n] if key in ("pix", "scale", "mean") else full[key]), key


def test_insert_nothing_to_insert_on_tiny_and_ragged_views():
    """Render equal to the ground truth (P_a = 0 everywhere) on views smaller
    than a tile and than the filter: P maps still match, the list is empty."""
    sizes = [(1, 1), (3, 2), (70, 17)]
    cams = _cams(sizes, 97)
    gts, _, depths = make_insert_inputs(sizes, 97)
    assert _check(cams, gts, gts, depths) == 0


def test_insert_rig_views():
    _, cams = make_config(3, scale=1e-5)
    sizes = [(c.width, c.height) for c in cams]
    gts, rds, depths = make_insert_inputs(sizes, 94)
    assert _check(cams, gts, rds, depths) > 1000


def test_insert_rejects_bad_sigma():
    sizes = [(32, 32)]
    cams = _cams(sizes, 95)
    gts, rds, depths = make_insert_inputs(sizes, 96)
    with pytest.raises(GsrError):
        _run(cams, gts, rds, depths, sigma=2.0)
    with pytest.raises(GsrError):
        _run(cams, gts, rds, depths, sigma=0.0)
