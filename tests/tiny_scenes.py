"""Hand-built tiny scenes for closed-form checks (inputs only, no rasterizer
arithmetic)."""
import math

import numpy as np

from workloads.generators import Camera, Scene

Y0 = 1.0 / (2.0 * math.sqrt(math.pi))


def camera(f=60.0, w=64, h=48, cx=None, cy=None, R=None, t=None, fy=None):
    return Camera(np.asarray(np.eye(3) if R is None else R, np.float32),
                  np.asarray(np.zeros(3) if t is None else t, np.float32),
                  float(np.float32(f)), float(np.float32(f if fy is None else fy)),
                  float(np.float32(w / 2 if cx is None else cx)),
                  float(np.float32(h / 2 if cy is None else cy)), w, h)


def scene(means, log_scales, quats, opacity_logits, colours=None, sh=None, degree=0):
    means = np.asarray(means, np.float64).T
    n = means.shape[1]
    if sh is None:
        col = np.asarray(colours, np.float64).T  # [3, n]
        k = (degree + 1) ** 2
        sh = np.zeros((k, 3, n))
        sh[0] = (col - 0.5) / Y0
    return Scene(mean=np.ascontiguousarray(means.astype(np.float32)),
                 log_scale=np.ascontiguousarray(np.asarray(log_scales, np.float64).T.astype(np.float32)),
                 quat=np.ascontiguousarray(np.asarray(quats, np.float64).T.astype(np.float32)),
                 opacity_logit=np.asarray(opacity_logits, np.float64).astype(np.float32).reshape(n),
                 sh=np.ascontiguousarray(np.asarray(sh, np.float64).astype(np.float32)),
                 sh_degree=degree)


def logit(p):
    return math.log(p / (1.0 - p))


def mini_rig(seed=7, n=300, degree=3, w=96, h=64):
    """Two posed views of a small random cloud, SH degree 3."""
    rng = np.random.default_rng(seed)
    means = np.stack([rng.uniform(-1.5, 1.5, n), rng.uniform(-1.0, 1.0, n), rng.uniform(3.0, 7.0, n)], 1)
    k = (degree + 1) ** 2
    sh = np.zeros((k, 3, n))
    sh[0] = rng.uniform(0.0, 1.0, (3, n))
    sh[1:] = rng.normal(0.0, 0.2, (k - 1, 3, n))
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    sc = scene(means, rng.normal(-2.6, 0.4, (n, 3)), q, rng.normal(0.0, 1.5, n), sh=sh, degree=degree)
    a = math.radians(8.0)
    R1 = np.array([[math.cos(a), 0, math.sin(a)], [0, 1, 0], [-math.sin(a), 0, math.cos(a)]]).T
    c1 = np.array([0.3, -0.1, 0.2])
    cams = [camera(80.0, w, h), camera(80.0, w, h, cx=w / 2 + 3.25, cy=h / 2 - 1.5, R=R1, t=-R1 @ c1, fy=84.0)]
    return sc, cams


def needles(seed=5, n=400, w=96, h=64):
    """Needle-like footprints (about 50:1 axes, every orientation), half of
    them with opacities just above 1/255: most tiles of their binning
    rectangles lie outside the alpha >= 1/255 ellipse, and many ellipses end
    close to a tile edge."""
    rng = np.random.default_rng(seed)
    means = np.stack([rng.uniform(-2.0, 2.0, n), rng.uniform(-1.4, 1.4, n), rng.uniform(3.0, 6.0, n)], 1)
    ls = np.stack([rng.uniform(-1.6, -0.9, n), rng.normal(-5.0, 0.2, n), rng.normal(-5.0, 0.2, n)], 1)
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    op = np.where(rng.random(n) < 0.5, rng.uniform(1.05 / 255, 4.0 / 255, n), rng.uniform(0.05, 0.9, n))
    col = rng.uniform(0.0, 1.0, (n, 3))
    return scene(means, ls, q, [logit(p) for p in op], colours=col), [camera(80.0, w, h)]
