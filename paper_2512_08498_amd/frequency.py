"""Binding of the frequency-based scheduling entry points (gsr_freq_plan,
gsr_freq_significance, gsr_downsample, gsr_freq_schedule): argument
marshalling only, every step runs in the HIP library."""
from __future__ import annotations

import ctypes as C
from typing import Sequence, Tuple

import numpy as np
import torch

from . import _lib as L

TAU_F = 2.0  # the paper's threshold on r'


def _vp(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _check(t, name, dtype, shape, device):
    if t.dtype != dtype or not t.is_contiguous() or t.device != device or tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected contiguous {dtype} {tuple(shape)} on {device}, got {t.dtype} "
                         f"{tuple(t.shape)} on {t.device}")


class Frequency:
    """Frequency significance X of a fixed batch of image sizes, box
    downsampling and the scheduling step, on one device."""

    def __init__(self, sizes: Sequence[Tuple[int, int]] = (), device="cuda"):
        self.lib = L.load()
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.ctx = C.c_void_p()
        L.check(None, self.lib.gsr_create(C.byref(self.ctx)))
        self.sizes = []
        self.workspace = None
        self.plan(sizes)

    def _check(self, status):
        L.check(self.ctx, status)

    def stream(self):
        return C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def plan(self, sizes: Sequence[Tuple[int, int]]):
        """Fix the batch: a list of (width, height)."""
        w = np.ascontiguousarray([s[0] for s in sizes], dtype=np.int32)
        h = np.ascontiguousarray([s[1] for s in sizes], dtype=np.int32)
        ws = C.c_size_t()
        self._check(self.lib.gsr_freq_plan(self.ctx, w.ctypes.data if len(w) else None,
                                           h.ctypes.data if len(h) else None, len(w), C.byref(ws)))
        self.sizes = [(int(a), int(b)) for a, b in zip(w, h)]
        self.pix_off = np.concatenate([[0], np.cumsum([a * b for a, b in self.sizes])]).astype(np.int64)
        self.workspace = None
        self.workspace = torch.empty(max(int(ws.value), 1), dtype=torch.uint8, device=self.device)

    def significance(self, images: torch.Tensor, out=None) -> torch.Tensor:
        """X of every planned image; ``images`` flat, planar [3][h][w] per image in plan order."""
        _check(images, "images", torch.float32, (3 * int(self.pix_off[-1]),), self.device)
        out = out if out is not None else torch.empty(len(self.sizes), dtype=torch.float32, device=self.device)
        _check(out, "out", torch.float32, (len(self.sizes),), self.device)
        self._check(self.lib.gsr_freq_significance(self.ctx, _vp(images), _vp(self.workspace),
                                                   self.workspace.numel(), _vp(out), self.stream()))
        return out

    def downsample(self, image: torch.Tensor, width: int, height: int, factor: int, out=None) -> torch.Tensor:
        """n x n box average of one planar [3][height][width] image."""
        _check(image, "image", torch.float32, (3 * height * width,), self.device)
        shape = (3 * (height // factor) * (width // factor),)
        out = out if out is not None else torch.empty(shape, dtype=torch.float32, device=self.device)
        _check(out, "out", torch.float32, shape, self.device)
        self._check(self.lib.gsr_downsample(self.ctx, _vp(image), int(width), int(height), int(factor), _vp(out),
                                            self.stream()))
        return out

    def schedule(self, x_gt, x_render, x_gt_level=None, levels=None, uniforms=None, tau_f=TAU_F):
        """One scheduling step: returns dict(r, r_prime, picks); ``levels``
        (int32 tensor) is updated in place when given."""
        F = x_gt.numel()
        f32 = dict(dtype=torch.float32, device=self.device)
        for name, t in (("x_gt", x_gt), ("x_render", x_render), ("x_gt_level", x_gt_level)):
            if t is not None:
                _check(t, name, torch.float32, (F,), self.device)
        if levels is not None:
            _check(levels, "levels", torch.int32, (F,), self.device)
        n_picks = 0
        picks = None
        if uniforms is not None:
            n_picks = uniforms.numel()
            _check(uniforms, "uniforms", torch.float32, (n_picks,), self.device)
            picks = torch.empty(n_picks, dtype=torch.int32, device=self.device)
        r = torch.empty(F, **f32)
        rp = torch.empty(F, **f32) if x_gt_level is not None else None
        self._check(self.lib.gsr_freq_schedule(self.ctx, _vp(x_gt), _vp(x_gt_level), _vp(x_render), F,
                                               float(tau_f), _vp(levels), _vp(uniforms), n_picks, _vp(r), _vp(rp),
                                               _vp(picks), self.stream()))
        return dict(r=r, r_prime=rp, picks=picks)

    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            self.lib.gsr_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
