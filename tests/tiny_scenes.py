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


def _pixel_ray(cam_f, cx, cy, i, j, z):
    """Camera-space point at depth z whose projection is the centre of pixel (i, j)."""
    return np.array([(i + 0.5 - cx) * z / cam_f, (j + 0.5 - cy) * z / cam_f, z])


def capped(seed=31, w=96, h=64, f=80.0):
    """Opaque Gaussians (opacity 0.996..0.9995, footprint sigma 8..13 px) centred on pixel centres in
    front, so o G > 0.99 at their central pixels and alpha takes the 0.99 cap,
    next to 0.98-opacity ones and a random layer behind.  The capped ones sit
    at least 14 px apart, so no pixel composites two capped entries (whose
    T (1 - alpha) would sit exactly at the 1e-4 stop)."""
    rng = np.random.default_rng(seed)
    cx, cy = w / 2, h / 2
    means, ls, op, col = [], [], [], []
    grid = [(i, j) for i in range(8, w - 8, 14) for j in range(8, h - 8, 14)]
    for k, (i, j) in enumerate(grid):
        z = float(rng.uniform(2.5, 3.5))
        means.append(_pixel_ray(f, cx, cy, i, j, z))
        sig = float(rng.uniform(8.0, 13.0))  # footprint sigma in pixels
        ls.append(np.log(np.full(3, sig * z / f)) + rng.normal(0, 0.1, 3))
        op.append(float(rng.uniform(0.996, 0.9995)) if k % 3 else 0.98)
        col.append(rng.uniform(0, 1, 3))
    m = 150
    means += list(np.stack([rng.uniform(-1.5, 1.5, m), rng.uniform(-1.0, 1.0, m), rng.uniform(4.0, 8.0, m)], 1))
    ls += list(rng.normal(-2.4, 0.4, (m, 3)))
    op += list(rng.uniform(0.05, 0.9, m))
    col += list(rng.uniform(0, 1, (m, 3)))
    n = len(means)
    q = rng.standard_normal((n, 4))
    return scene(np.array(means), np.array(ls), q, [logit(p) for p in op], colours=np.array(col)), \
        [camera(f, w, h)]


def guard_clamped(seed=41, w=96, h=64, f=80.0):
    """Large Gaussians centred outside the Jacobian guard (|x/z| above
    1.3 max(cx, W - cx)/fx, or the same in y), whose footprints still reach
    into the image, in a posed view with an off-centre principal point, plus
    a random layer of small Gaussians inside the image."""
    rng = np.random.default_rng(seed)
    a = math.radians(10.0)
    b = math.radians(-6.0)
    R = np.array([[math.cos(a), 0, math.sin(a)], [0, 1, 0], [-math.sin(a), 0, math.cos(a)]]) @ \
        np.array([[1, 0, 0], [0, math.cos(b), -math.sin(b)], [0, math.sin(b), math.cos(b)]])
    centre = np.array([0.2, -0.1, -0.3])
    t = -R @ centre
    cx, cy = w / 2 + 5.0, h / 2 - 3.0
    cam = camera(f, w, h, cx=cx, cy=cy, R=R, t=t, fy=f * 1.05)
    lim_x = 1.3 * max(cx, w - cx) / f
    lim_y = 1.3 * max(cy, h - cy) / (f * 1.05)
    means, ls, op, col = [], [], [], []
    # (x/z, y/z) directions beyond the guard on every side and at corners
    dirs = [(1.15, 0.1), (-1.15, -0.2), (0.2, 1.2), (-0.3, -1.2), (1.1, 1.1), (-1.1, 1.15), (1.2, -0.5),
            (0.0, 1.3), (1.3, 0.3), (-1.25, 0.4)]
    for (sx, sy) in dirs:
        z = float(rng.uniform(3.0, 5.0))
        xc = np.array([sx * lim_x * z, sy * lim_y * z, z])
        means.append(R.T @ (xc - t))
        # footprint sigma of 9..14 px: the box reaches 10+ px into the image
        sig = float(rng.uniform(9.0, 14.0))
        ls.append(np.log(sig * z / f) + np.array([0.3, -0.1, -0.4]) * rng.uniform(0.5, 1.0))
        op.append(float(rng.uniform(0.4, 0.9)))
        col.append(rng.uniform(0, 1, 3))
    m = 120
    means += list(np.stack([rng.uniform(-1.2, 1.2, m), rng.uniform(-0.8, 0.8, m), rng.uniform(3.0, 6.0, m)], 1))
    ls += list(rng.normal(-2.6, 0.4, (m, 3)))
    op += list(rng.uniform(0.05, 0.9, m))
    col += list(rng.uniform(0, 1, (m, 3)))
    n = len(means)
    q = rng.standard_normal((n, 4))
    sh = np.zeros((16, 3, n))
    sh[0] = (np.array(col).T - 0.5) / Y0
    sh[1:] = rng.normal(0.0, 0.15, (15, 3, n))
    return scene(np.array(means), np.array(ls), q, [logit(p) for p in op], sh=sh, degree=3), [cam]


def guard_clamped_ids(sc, cams):
    """Per view, the Gaussians whose x/z or y/z (FP64) lies beyond the
    Jacobian guard."""
    out = []
    for c in cams:
        R = np.asarray(c.R, np.float64)
        xc = R @ sc.mean.astype(np.float64) + np.asarray(c.t, np.float64)[:, None]
        lim_x = 1.3 * max(c.cx, c.width - c.cx) / c.fx
        lim_y = 1.3 * max(c.cy, c.height - c.cy) / c.fy
        out.append(np.nonzero((xc[2] > 0.2) & ((np.abs(xc[0] / xc[2]) > lim_x) | (np.abs(xc[1] / xc[2]) > lim_y)))[0])
    return out
