"""FP64 Adam step (Kingma & Ba, with bias correction).

The paper updates Gaussian parameters jointly by gradients (Sec. 3.3) without
naming the optimiser; the rasterizer workloads take a dense Adam step over
every parameter each iteration:

    t <- t + 1
    m <- b1 m + (1 - b1) g
    v <- b2 v + (1 - b2) g^2
    p <- p - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)

with b1 = 0.9, b2 = 0.999, eps = 1e-15 and one learning rate per parameter
group (mean, log_scale, quat, opacity_logit, sh degree 0, sh higher degrees).

Parity status: pinned by the first-step closed form p - lr g / (|g| + eps) and
by torch.optim.Adam in float64.
"""
from __future__ import annotations

import numpy as np

BETA1 = 0.9
BETA2 = 0.999
EPS = 1e-15


def adam_step(p, g, m, v, step, lr, beta1=BETA1, beta2=BETA2, eps=EPS):
    """One step on float64 arrays; ``step`` is the count before this step.
    Returns (p, m, v)."""
    p = np.asarray(p, np.float64)
    g = np.asarray(g, np.float64)
    t = step + 1
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def group_slices(n, sh_k):
    """Flat (start, stop) ranges of the six groups inside each tensor:
    sh degree 0 is the first 3n entries of the [K][3][n] SH array."""
    return {
        "mean": ("mean", 0, 3 * n),
        "log_scale": ("log_scale", 0, 3 * n),
        "quat": ("quat", 0, 4 * n),
        "opacity_logit": ("opacity_logit", 0, n),
        "sh_dc": ("sh", 0, 3 * n),
        "sh_rest": ("sh", 3 * n, sh_k * 3 * n),
    }
