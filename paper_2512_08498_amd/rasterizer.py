"""Python binding over the C ABI: device memory and streams come from torch,
every step of the rasterizer runs in the HIP library.

``Rasterizer`` owns a context, a plan for one batch of views and the device
workspace; ``RasterizeFn`` is the torch.autograd.Function around
render_forward / render_backward; ``FusedAdam`` is the optimiser step.
"""
from __future__ import annotations

import ctypes as C
from typing import Dict, Sequence

import numpy as np
import torch

from . import _lib as L

PARAM_NAMES = ("mean", "log_scale", "quat", "opacity_logit", "sh")
DEFAULT_LR = (1.6e-4, 5e-3, 1e-3, 5e-2, 2.5e-3, 2.5e-3 / 20.0)


def _vp(t: torch.Tensor):
    return C.c_void_p(t.data_ptr())


def camera_rows(cams) -> np.ndarray:
    """[V, 18] float32 rows in the gsr_camera layout (width/height as int32 bits)."""
    rows = np.zeros((len(cams), 18), dtype=np.float32)
    for i, c in enumerate(cams):
        rows[i, 0:9] = np.asarray(c.R, np.float32).reshape(-1)
        rows[i, 9:12] = np.asarray(c.t, np.float32).reshape(-1)
        rows[i, 12:16] = (c.fx, c.fy, c.cx, c.cy)
        rows[i, 16:18] = np.array([c.width, c.height], np.int32).view(np.float32)
    return rows


def _check_flat(name, t: torch.Tensor, numel, device):
    """A contiguous float32 tensor of numel elements on device, any shape."""
    if t.dtype != torch.float32 or not t.is_contiguous() or t.device != device or t.numel() != numel:
        raise ValueError(f"{name}: expected contiguous float32 with {numel} elements on {device}, got "
                         f"{t.dtype} {tuple(t.shape)} on {t.device} (contiguous={t.is_contiguous()})")


def device_copy(dst: torch.Tensor, src: torch.Tensor):
    """Copy src into dst (contiguous device tensors of the same byte size, a
    multiple of 16) with the library's streaming copy kernel, on the current
    stream: the reference for achievable HBM bandwidth."""
    nbytes = src.numel() * src.element_size()
    if (not src.is_contiguous() or not dst.is_contiguous() or src.device.type != "cuda" or dst.device != src.device
            or dst.numel() * dst.element_size() != nbytes):
        raise ValueError("device_copy: contiguous device tensors of the same byte size expected")
    lib = L.load()
    L.check(None, lib.gsr_copy_bytes(_vp(dst), _vp(src), nbytes, torch.cuda.current_stream(src.device).cuda_stream))


def _check_param(name, t: torch.Tensor, shape, device):
    if t.dtype != torch.float32 or not t.is_contiguous() or t.device != device or tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected contiguous float32 {tuple(shape)} on {device}, got "
                         f"{t.dtype} {tuple(t.shape)} on {t.device} (contiguous={t.is_contiguous()})")


class Rasterizer:
    """One planned batch of views over n Gaussians of a fixed SH degree."""

    def __init__(self, cams: Sequence, n: int, sh_degree: int, tile_size: int = 16, bg=(0.0, 0.0, 0.0),
                 capacity_records: int = 0, capacity_pairs: int = 0, device="cuda", cams_device=None,
                 long_list: int = 1024, persistent: bool = False):
        self.lib = L.load()
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.n = int(n)
        self.sh_degree = int(sh_degree)
        self.tile_size = int(tile_size) or 16
        self.bg = tuple(float(b) for b in bg)
        self.views = len(cams)
        self.sizes = [(int(c.width), int(c.height)) for c in cams]
        rows = camera_rows(cams)
        self._cams_host = (L.Camera * self.views)()
        C.memmove(self._cams_host, rows.ctypes.data, rows.nbytes)
        self.cams_dev = cams_device if cams_device is not None else torch.from_numpy(rows).to(self.device)
        self.ctx = C.c_void_p()
        L.check(None, self.lib.gsr_create(C.byref(self.ctx)))
        self.workspace = None
        self.rig = None
        # bumped by every call that rewrites the workspace's binning state (a
        # plan or a forward), so a backward can tell that its state is gone
        self.generation = 0
        self._check(self.lib.gsr_set_tuning(
            self.ctx, C.byref(L.Tuning(self.tile_size or 16, int(long_list), int(bool(persistent)), 0.0))))
        self._plan(capacity_records, capacity_pairs)

    # -- plan / workspace ------------------------------------------------------------------
    def _plan(self, cap_rec, cap_pairs):
        opts = L.PlanOptions(self.tile_size, int(cap_rec), int(cap_pairs), (C.c_float * 3)(*self.bg))
        ws = C.c_size_t()
        pix = (C.c_int64 * (self.views + 1))()
        self._check(self.lib.gsr_plan(self.ctx, self._cams_host, self.views, self.n, self.sh_degree,
                                      C.byref(opts), C.byref(ws), pix))
        self.capacity = (int(cap_rec), int(cap_pairs))
        self.ws_bytes = int(ws.value)
        self.pix_off = [int(p) for p in pix]
        self.total_px = self.pix_off[-1]
        self.workspace = None
        self._ins_ws = None
        self._merge_ws = None
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.generation += 1

    def tuning(self):
        t = L.Tuning()
        self._check(self.lib.gsr_get_tuning(self.ctx, C.byref(t)))
        return {"tile_size": t.tile_size, "long_list": t.long_list, "persistent": bool(t.persistent)}

    def set_tuning(self, tile_size, long_list=1024, persistent=False):
        """Change the launch configuration and re-plan (same capacities)."""
        self._check(self.lib.gsr_set_tuning(
            self.ctx, C.byref(L.Tuning(int(tile_size), int(long_list), int(bool(persistent)), 0.0))))
        self.tile_size = int(tile_size)
        self._plan(*self.capacity)

    def autotune(self, params, repeats=3, cache=None):
        """Time the candidate launch configurations on this batch (see
        gsr_autotune), adopt the fastest and re-plan; returns the choice."""
        g = self._gaussians(params)
        opts = L.PlanOptions(0, int(self.capacity[0]), int(self.capacity[1]), (C.c_float * 3)(*self.bg))
        best = L.Tuning()
        path = None if cache is None else str(cache).encode()
        self.workspace = None  # the plan is dropped; return its workspace for the measurement
        torch.cuda.empty_cache()
        status = self.lib.gsr_autotune(self.ctx, C.byref(g), self._cams_host, self.views, C.byref(opts),
                                       int(repeats), path, C.byref(best), self.stream())
        self.tile_size = best.tile_size if status == 0 else self.tile_size
        self._plan(*self.capacity)
        self._check(status)
        return {"tile_size": best.tile_size, "long_list": best.long_list, "persistent": bool(best.persistent),
                "step_ms": best.step_ms}

    def _check(self, status):
        L.check(self.ctx, status)

    def stream(self):
        return C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            self.lib.gsr_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers ---------------------------------------------------------------------------
    def _gaussians(self, p: Dict[str, torch.Tensor]) -> L.Gaussians:
        n, k = self.n, (self.sh_degree + 1) ** 2
        shapes = dict(mean=(3, n), log_scale=(3, n), quat=(4, n), opacity_logit=(n,), sh=(k, 3, n))
        for name in PARAM_NAMES:
            _check_param(name, p[name], shapes[name], self.device)
        return L.Gaussians(n, self.sh_degree, *(p[name].data_ptr() for name in PARAM_NAMES))

    def new_fwd_out(self):
        px = self.total_px
        return dict(image=torch.empty(3 * px, dtype=torch.float32, device=self.device),
                    t_final=torch.empty(px, dtype=torch.float32, device=self.device),
                    last_pos=torch.empty(px, dtype=torch.int32, device=self.device),
                    n_contrib=torch.empty(px, dtype=torch.int32, device=self.device))

    @staticmethod
    def _fwd_struct(out) -> L.FwdOut:
        return L.FwdOut(out["image"].data_ptr(), out["t_final"].data_ptr(), out["last_pos"].data_ptr(),
                        out["n_contrib"].data_ptr())

    def view_images(self, flat: torch.Tensor):
        """Per-view [3, H, W] views of a flat image buffer."""
        return [flat[3 * self.pix_off[v]:3 * self.pix_off[v + 1]].view(3, h, w)
                for v, (w, h) in enumerate(self.sizes)]

    def view_maps(self, flat: torch.Tensor):
        """Per-view [H, W] views of a flat per-pixel buffer."""
        return [flat[self.pix_off[v]:self.pix_off[v + 1]].view(h, w) for v, (w, h) in enumerate(self.sizes)]

    # -- calls -----------------------------------------------------------------------------
    def forward(self, params, out=None, check=True, cams_dev=None):
        """Render all views.  With ``check`` the call synchronises, and on a
        capacity overflow re-plans with the sizes the forward reported and
        renders again."""
        out = out if out is not None else self.new_fwd_out()
        g = self._gaussians(params)
        cams = cams_dev if cams_dev is not None else self.cams_dev
        self.generation += 1
        self._check(self.lib.gsr_render_forward(self.ctx, C.byref(g), _vp(cams), self.views, _vp(self.workspace),
                                                self.ws_bytes, C.byref(self._fwd_struct(out)), self.stream()))
        if check:
            st = self.lib.gsr_check(self.ctx, _vp(self.workspace), self.stream())
            if st == L.GSR_ERR_CAPACITY:
                rec, pairs, _ = self.required_capacity()
                self._plan(max(int(rec * 1.25) + 1024, self.capacity[0]), max(int(pairs * 1.25) + 4096,
                                                                                self.capacity[1]))
                return self.forward(params, out=out, check=True, cams_dev=cams_dev)
            self._check(st)
        return out

    def forward_noalloc(self, params, out=None, cams_dev=None):
        """forward() through gsr_render_forward_noalloc: the workspace is the
        library's per-GPU device scratch (the plan must fit in
        GSR_NOALLOC_SCRATCH_BYTES), so the call allocates nothing given
        ``out``.  No capacity re-plan: check_noalloc() reports an overflow.
        The backward cannot follow it (its binning state is not in this
        rasterizer's workspace)."""
        out = out if out is not None else self.new_fwd_out()
        g = self._gaussians(params)
        cams = cams_dev if cams_dev is not None else self.cams_dev
        self.generation += 1
        self._check(self.lib.gsr_render_forward_noalloc(self.ctx, C.byref(g), _vp(cams), self.views,
                                                        C.byref(self._fwd_struct(out)), self.stream()))
        return out

    def check_noalloc(self):
        """gsr_check of the no-alloc scratch (synchronises)."""
        self._check(self.lib.gsr_check(self.ctx, None, self.stream()))

    def forward_l1(self, params, target, out=None, loss_out=None, dl_out=None, check=True, cams_dev=None):
        """forward() with the L1 loss against ``target`` fused in: returns
        (out, loss [1], dL/dimage)."""
        out = out if out is not None else self.new_fwd_out()
        _check_param("target", target, (3 * self.total_px,), self.device)
        loss_out = loss_out if loss_out is not None else torch.empty(1, dtype=torch.float32, device=self.device)
        dl_out = dl_out if dl_out is not None else torch.empty_like(out["image"])
        g = self._gaussians(params)
        cams = cams_dev if cams_dev is not None else self.cams_dev
        self.generation += 1
        self._check(self.lib.gsr_render_forward_l1(self.ctx, C.byref(g), _vp(cams), self.views, _vp(self.workspace),
                                                   self.ws_bytes, C.byref(self._fwd_struct(out)), _vp(target),
                                                   _vp(loss_out), _vp(dl_out), self.stream()))
        if check:
            st = self.lib.gsr_check(self.ctx, _vp(self.workspace), self.stream())
            if st == L.GSR_ERR_CAPACITY:
                rec, pairs, _ = self.required_capacity()
                self._plan(max(int(rec * 1.25) + 1024, self.capacity[0]), max(int(pairs * 1.25) + 4096,
                                                                                self.capacity[1]))
                return self.forward_l1(params, target, out, loss_out, dl_out, True, cams_dev)
            self._check(st)
        return out, loss_out, dl_out

    def required_capacity(self):
        r, p, t = C.c_int64(), C.c_int64(), C.c_int64()
        self._check(self.lib.gsr_required_capacity(self.ctx, _vp(self.workspace), C.byref(r), C.byref(p),
                                                   C.byref(t), self.stream()))
        return r.value, p.value, t.value

    def check(self):
        self._check(self.lib.gsr_check(self.ctx, _vp(self.workspace), self.stream()))

    def _cam_grad_ptr(self, cam_grads):
        if cam_grads is None:
            return None
        _check_param("cam_grads", cam_grads, (self.views, 12), self.device)
        return cam_grads.data_ptr()

    def backward(self, params, fwd, dL_dimage, grads=None, accumulate=False, cams_dev=None, cam_grads=None):
        """Gradients of every Gaussian parameter; with ``cam_grads`` (a
        [views, 12] float32 tensor, or True for a new one) also each view's
        pose gradient dL/d(R, t), SH detached, returned as grads["camera"]."""
        g = self._gaussians(params)
        if grads is None:
            grads = {k: torch.empty_like(params[k]) for k in PARAM_NAMES}
        for k in PARAM_NAMES:
            _check_param(f"grads[{k}]", grads[k], tuple(params[k].shape), self.device)
        if cam_grads is True:
            cam_grads = torch.empty(self.views, 12, dtype=torch.float32, device=self.device)
        if cam_grads is not None:
            grads["camera"] = cam_grads
        gr = L.Grads(*(grads[k].data_ptr() for k in PARAM_NAMES), self._cam_grad_ptr(cam_grads))
        cams = cams_dev if cams_dev is not None else self.cams_dev
        dl = dL_dimage.contiguous()
        _check_flat("dL_dimage", dl, 3 * self.total_px, self.device)
        self._check(self.lib.gsr_render_backward(self.ctx, C.byref(g), _vp(cams), self.views, _vp(self.workspace),
                                                 self.ws_bytes, C.byref(self._fwd_struct(fwd)), _vp(dl),
                                                 C.byref(gr), 1 if accumulate else 0, self.stream()))
        return grads

    def backward_adam(self, params, fwd, dL_dimage, opt: "FusedAdam", grads_out=None, cams_dev=None, cam_grads=None):
        """Backward with the Adam update fused in; ``grads_out`` (optional)
        receives the Gaussian gradients, ``cam_grads`` (optional [views, 12])
        the views' pose gradients."""
        g = self._gaussians(params)
        cams = cams_dev if cams_dev is not None else self.cams_dev
        _check_flat("dL_dimage", dL_dimage, 3 * self.total_px, self.device)
        if grads_out is not None:
            for k in PARAM_NAMES:
                _check_param(f"grads_out[{k}]", grads_out[k], tuple(params[k].shape), self.device)
        go = None
        if grads_out is not None or cam_grads is not None:
            ptrs = [grads_out[k].data_ptr() for k in PARAM_NAMES] if grads_out is not None else [None] * 5
            go = C.byref(L.Grads(*ptrs, self._cam_grad_ptr(cam_grads)))
        self._check(self.lib.gsr_render_backward_adam(
            self.ctx, C.byref(g), _vp(cams), self.views, _vp(self.workspace), self.ws_bytes,
            C.byref(self._fwd_struct(fwd)), _vp(dL_dimage), C.byref(opt.param_struct(params)),
            C.byref(opt.m_struct()), C.byref(opt.v_struct()), C.byref(opt.config), _vp(opt.step), go,
            self.stream()))

    def l1_loss(self, image, target, loss_out=None, dl_out=None):
        n = image.numel()
        _check_flat("image", image, n, self.device)
        _check_flat("target", target, n, self.device)
        loss_out = loss_out if loss_out is not None else torch.empty(1, dtype=torch.float32, device=self.device)
        dl_out = dl_out if dl_out is not None else torch.empty_like(image)
        _check_flat("loss_out", loss_out, 1, self.device)
        _check_flat("dl_out", dl_out, n, self.device)
        self._check(self.lib.gsr_l1_loss(self.ctx, _vp(image), _vp(target), image.numel(), _vp(loss_out),
                                         _vp(dl_out), self.stream()))
        return loss_out, dl_out

    def profile(self, enable=True):
        """Per-stage HIP-event timing of subsequent calls (synchronising)."""
        self._check(self.lib.gsr_profile(self.ctx, 1 if enable else 0))

    def profile_read(self, reset=True):
        """{stage: (total ms, calls)} accumulated since the last reset."""
        ms = (C.c_double * L.N_STAGES)()
        calls = (C.c_int64 * L.N_STAGES)()
        self._check(self.lib.gsr_profile_read(self.ctx, ms, calls, 1 if reset else 0))
        return {name: (ms[i], calls[i]) for i, name in enumerate(L.STAGE_NAMES)}

    # -- rig poses (T_v = T_m^frame T_camera->m) -------------------------------------------------
    def set_rig(self, view_frame, view_camera, n_frames, n_cams):
        """Rig structure of the batch: view v is camera view_camera[v] at frame view_frame[v]."""
        vf = np.ascontiguousarray(view_frame, dtype=np.int32)
        vc = np.ascontiguousarray(view_camera, dtype=np.int32)
        if vf.shape != (self.views,) or vc.shape != (self.views,):
            raise ValueError(f"rig index arrays must have {self.views} entries")
        self._check(self.lib.gsr_rig_plan(self.ctx, vf.ctypes.data, vc.ctypes.data, self.views, int(n_frames),
                                          int(n_cams)))
        self.rig = (int(n_frames), int(n_cams))

    def _rig_sizes(self):
        if self.rig is None:
            raise RuntimeError("set_rig has not been called")
        return self.rig

    def rig_compose(self, central, relative, cams_dev=None):
        """Write the composed view poses into the camera array (default: the
        rasterizer's own), intrinsics untouched; returns that array."""
        F, K = self._rig_sizes()
        _check_param("central", central, (F, 12), self.device)
        _check_param("relative", relative, (K, 12), self.device)
        cams = cams_dev if cams_dev is not None else self.cams_dev
        self._check(self.lib.gsr_rig_compose(self.ctx, _vp(central), _vp(relative), _vp(cams), self.stream()))
        return cams

    def rig_gradients(self, central, relative, view_grads, tangent=True, out=None):
        """dL/d(central) [F,12], dL/d(relative) [K,12] and, with ``tangent``,
        the left-perturbation tangent gradients [F,6], [K,6] (into ``out``,
        a dict of such tensors, if given)."""
        F, K = self._rig_sizes()
        _check_param("central", central, (F, 12), self.device)
        _check_param("relative", relative, (K, 12), self.device)
        _check_param("view_grads", view_grads, (self.views, 12), self.device)
        if out is None:
            f32 = dict(dtype=torch.float32, device=self.device)
            out = dict(d_central=torch.empty(F, 12, **f32), d_relative=torch.empty(K, 12, **f32))
            if tangent:
                out.update(xi_central=torch.empty(F, 6, **f32), xi_relative=torch.empty(K, 6, **f32))
        shapes = dict(d_central=(F, 12), d_relative=(K, 12), xi_central=(F, 6), xi_relative=(K, 6))
        for k in (shapes if tangent else ("d_central", "d_relative")):
            _check_param(k, out[k], shapes[k], self.device)
        xc = _vp(out["xi_central"]) if tangent else None
        xr = _vp(out["xi_relative"]) if tangent else None
        self._check(self.lib.gsr_rig_gradients(self.ctx, _vp(central), _vp(relative), _vp(view_grads),
                                               _vp(out["d_central"]), _vp(out["d_relative"]), xc, xr,
                                               self.stream()))
        return out

    # -- LoG-based insertion of new Gaussians -------------------------------------------------
    def log_insert(self, gt, render, depth, sigma=1.0, tau_a=0.2, capacity=None, cams_dev=None, p_render=False):
        """Insertion probabilities of all views and the list of inserting
        pixels with the new Gaussians' scale and world centre (see
        gsr_log_insert).  Returns dict(p_gt, p_render, pix, scale, mean, count)."""
        px = self.total_px
        _check_param("gt", gt, (3 * px,), self.device)
        _check_param("render", render, (3 * px,), self.device)
        _check_param("depth", depth, (px,), self.device)
        if getattr(self, "_ins_ws", None) is None:
            nb = C.c_size_t()
            self._check(self.lib.gsr_insert_workspace(self.ctx, C.byref(nb)))
            self._ins_ws = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        cap = px if capacity is None else int(capacity)
        f32 = dict(dtype=torch.float32, device=self.device)
        res = dict(p_gt=torch.empty(px, **f32), p_render=torch.empty(px, **f32) if p_render else None,
                   pix=torch.empty(max(cap, 1), dtype=torch.int32, device=self.device),
                   scale=torch.empty(max(cap, 1), **f32), mean=torch.empty(max(cap, 1), 3, **f32),
                   count=torch.empty(1, dtype=torch.int32, device=self.device))
        out = L.InsertOut(res["pix"].data_ptr(), res["scale"].data_ptr(), res["mean"].data_ptr(),
                          res["count"].data_ptr(), cap)
        cams = cams_dev if cams_dev is not None else self.cams_dev
        self._check(self.lib.gsr_log_insert(self.ctx, _vp(cams), _vp(gt), _vp(render), _vp(depth),
                                            C.byref(L.InsertConfig(float(sigma), float(tau_a))), _vp(res["p_gt"]),
                                            _vp(res["p_render"]) if p_render else None, C.byref(out),
                                            _vp(self._ins_ws), self._ins_ws.numel(), self.stream()))
        return res

    def merge(self, existing, view, gt, ins, tau_d, kappa=1.0, cams_dev=None, out=None):
        """Merge the existing Gaussians (dict with mean [3, n], log_scale
        [3, n], sh [K, 3, n]) with the samples of ``view`` from ``ins`` (a
        log_insert result): returns dict(keep [n] uint8, colour [3, n],
        mean [3, n], keep_new [capacity] uint8, colour_new [capacity, 3],
        mean_new [capacity, 3]) (see gsr_merge; the means are the centres
        after the depth re-alignment).  New result tensors have keep_new,
        colour_new and mean_new zeroed; ``out`` (a dict of that form, e.g. an
        earlier result; "mean" and "mean_new" may be left out) is written in
        place instead, where the entries of other views' samples keep their
        values."""
        n = existing["mean"].shape[1]
        k = existing["sh"].shape[0]
        deg = int(round(k ** 0.5)) - 1
        for name, shape in (("mean", (3, n)), ("log_scale", (3, n)), ("sh", (k, 3, n))):
            _check_param(name, existing[name], shape, self.device)
        _check_param("gt", gt, (3 * self.total_px,), self.device)
        cap = ins["pix"].numel()
        for name, dtype, shape in (("pix", torch.int32, (cap,)), ("count", torch.int32, (1,)),
                                   ("mean", torch.float32, (cap, 3)), ("scale", torch.float32, (cap,)),
                                   ("p_gt", torch.float32, (self.total_px,))):
            t = ins[name]
            if t.dtype != dtype or not t.is_contiguous() or t.device != self.device or tuple(t.shape) != shape:
                raise ValueError(f"ins[{name}]: expected contiguous {dtype} {shape} on {self.device}, got "
                                 f"{t.dtype} {tuple(t.shape)} on {t.device}")
        nb = C.c_size_t()
        self._check(self.lib.gsr_merge_workspace(self.ctx, n, C.byref(nb)))
        ws = getattr(self, "_merge_ws", None)
        if ws is None or ws.numel() < int(nb.value):
            ws = self._merge_ws = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        shapes = (("keep", torch.uint8, (max(n, 1),)), ("colour", torch.float32, (3, max(n, 1))),
                  ("mean", torch.float32, (3, max(n, 1))), ("keep_new", torch.uint8, (cap,)),
                  ("colour_new", torch.float32, (cap, 3)), ("mean_new", torch.float32, (cap, 3)))
        if out is None:
            res = {name: (torch.zeros if name.endswith("_new") else torch.empty)(shape, dtype=dtype,
                                                                                 device=self.device)
                   for name, dtype, shape in shapes}
        else:
            res = out
            for name, dtype, shape in shapes:
                if name not in res and name in ("mean", "mean_new"):
                    continue
                t = res[name]
                if t.dtype != dtype or not t.is_contiguous() or t.device != self.device or tuple(t.shape) != shape:
                    raise ValueError(f"out[{name}]: expected contiguous {dtype} {shape} on {self.device}, got "
                                     f"{t.dtype} {tuple(t.shape)} on {t.device}")
        g = L.Gaussians(n, deg, existing["mean"].data_ptr(), existing["log_scale"].data_ptr(), None, None,
                        existing["sh"].data_ptr())
        so = L.InsertOut(ins["pix"].data_ptr(), ins["scale"].data_ptr(), ins["mean"].data_ptr(),
                         ins["count"].data_ptr(), cap)
        mo = L.MergeOut(res["keep"].data_ptr(), res["colour"].data_ptr(), res["keep_new"].data_ptr(),
                        res["colour_new"].data_ptr(), res["mean"].data_ptr() if "mean" in res else None,
                        res["mean_new"].data_ptr() if "mean_new" in res else None)
        cams = cams_dev if cams_dev is not None else self.cams_dev
        self._check(self.lib.gsr_merge(self.ctx, C.byref(g), int(view), _vp(cams), _vp(gt), _vp(ins["p_gt"]),
                                       C.byref(so), C.byref(L.MergeConfig(float(tau_d), float(kappa))), C.byref(mo),
                                       _vp(ws), ws.numel(), self.stream()))
        return res

    def count_evaluations(self, out):
        """(pixel, list entry) evaluations the last forward's backward walks
        over (pixel inside the entry's box, entry before the pixel's stop)."""
        ev = torch.zeros(1, dtype=torch.int64, device=self.device)
        fo = self._fwd_struct(out)
        self._check(self.lib.gsr_count_evaluations(self.ctx, _vp(self.workspace), C.byref(fo), _vp(ev),
                                                   self.stream()))
        return int(ev.item())

    def debug_binning(self):
        """(keys uint64, values uint32, tile CSR) of the last forward, as numpy."""
        _, pairs, tiles = self.required_capacity()
        keys = torch.empty(max(pairs, 1), dtype=torch.int64, device=self.device)
        vals = torch.empty(max(pairs, 1), dtype=torch.int32, device=self.device)
        csr = torch.empty(tiles + 1, dtype=torch.int32, device=self.device)
        self._check(self.lib.gsr_debug_binning(self.ctx, _vp(self.workspace), _vp(keys), _vp(vals), _vp(csr),
                                               self.stream()))
        torch.cuda.synchronize(self.device)
        return (keys.cpu().numpy().view(np.uint64)[:pairs], vals.cpu().numpy().view(np.uint32)[:pairs],
                csr.cpu().numpy().view(np.uint32).astype(np.int64))


class FusedAdam:
    """Dense Adam over the five parameter tensors (six learning-rate groups:
    mean, log_scale, quat, opacity_logit, SH degree 0, higher SH)."""

    def __init__(self, rast: Rasterizer, params, lr=DEFAULT_LR, betas=(0.9, 0.999), eps=1e-15):
        self.rast = rast
        self.params = params
        self.m = {k: torch.zeros_like(params[k]) for k in PARAM_NAMES}
        self.v = {k: torch.zeros_like(params[k]) for k in PARAM_NAMES}
        self.step = torch.zeros(1, dtype=torch.int32, device=rast.device)
        self.config = L.AdamConfig((C.c_float * 6)(*lr), betas[0], betas[1], eps)

    def param_struct(self, params=None):
        p = params if params is not None else self.params
        return L.Grads(*(p[k].data_ptr() for k in PARAM_NAMES))

    def m_struct(self):
        return L.Moments(*(self.m[k].data_ptr() for k in PARAM_NAMES))

    def v_struct(self):
        return L.Moments(*(self.v[k].data_ptr() for k in PARAM_NAMES))

    def apply(self, grads):
        r = self.rast
        r._check(r.lib.gsr_adam_step(r.ctx, C.byref(self.param_struct()),
                                     C.byref(L.Grads(*(grads[k].data_ptr() for k in PARAM_NAMES))),
                                     C.byref(self.m_struct()), C.byref(self.v_struct()), C.byref(self.config),
                                     _vp(self.step), r.n, r.sh_degree, r.stream()))


class RasterizeFn(torch.autograd.Function):
    """image = render(Gaussians) with the hand-written adjoint as backward.

    The workspace of ``rast`` carries the binning state (records, tile lists)
    from the forward to the backward.  A later forward or re-plan of the same
    rasterizer overwrites it; the backward then raises rather than return
    gradients of another state (each forward is stamped with the
    rasterizer's generation).  The forward's per-pixel outputs (final
    transmittance, last position, contributor count) stay available as
    ``rast.last_forward``.
    """

    @staticmethod
    def forward(ctx, rast: Rasterizer, mean, log_scale, quat, opacity_logit, sh):
        params = dict(mean=mean.contiguous(), log_scale=log_scale.contiguous(), quat=quat.contiguous(),
                      opacity_logit=opacity_logit.contiguous(), sh=sh.contiguous())
        out = rast.forward(params)
        rast.last_forward = out
        ctx.rast = rast
        ctx.fwd = out
        ctx.generation = rast.generation
        ctx.save_for_backward(*(params[k] for k in PARAM_NAMES))
        return out["image"]

    @staticmethod
    def backward(ctx, d_image):
        if ctx.rast.generation != ctx.generation:
            raise RuntimeError("RasterizeFn.backward: the rasterizer ran another forward or re-planned after this "
                               "forward, so its workspace no longer holds this forward's binning state; call "
                               "backward before the next forward of the same Rasterizer (or use one per graph)")
        params = dict(zip(PARAM_NAMES, ctx.saved_tensors))
        grads = ctx.rast.backward(params, ctx.fwd, d_image.contiguous())
        return (None,) + tuple(grads[k] for k in PARAM_NAMES)


def rasterize(rast: Rasterizer, params):
    """Differentiable flat image of all views (see Rasterizer.view_images)."""
    return RasterizeFn.apply(rast, *(params[k] for k in PARAM_NAMES))
