"""L1 photometric loss over a batch of views (FP64).

The paper names no loss; the rasterizer workloads train against a target image
with the mean absolute error over every view, pixel and channel:

    L = (1 / (3 Px)) sum_{v,p,ch} |C - C_target|,   Px = total pixel count
    dL/dC = sign(C - C_target) / (3 Px),  sign(0) = 0

Parity status: pinned against finite differences of the loss itself.
"""
from __future__ import annotations

import numpy as np


def l1_loss(images, targets):
    px = sum(int(np.asarray(t).shape[1] * np.asarray(t).shape[2]) for t in targets)
    total = 0.0
    grads = []
    for img, tgt in zip(images, targets):
        d = np.asarray(img, np.float64) - np.asarray(tgt, np.float64)
        total += float(np.abs(d).sum())
        grads.append(np.sign(d) / (3.0 * px))
    return total / (3.0 * px), grads
