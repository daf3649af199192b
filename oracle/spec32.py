"""FP32 binning rules: visibility, depth bits and pixel box of each Gaussian.

The paper keeps the 3DGS rasterizer (Sec. 3.3, "Optimization") and so its
tile binning: every Gaussian is culled or given a screen-space footprint, and
(view, tile, depth) keys order the per-tile lists.  These decisions are
discrete, so they are specified here in IEEE binary32 with every operation
rounded once in the written order (no fused multiply-add), correctly rounded
division and square root, and a project-written exponential.  Evaluated in
NumPy float32 (each ufunc rounds once), they are reproducible bit for bit by
any implementation that follows the same sequence.

Parity status: pinned.  ``bexp32`` is checked against the FP64 exponential
within 2 ulp; every spec output is checked against the same quantity computed
in FP64 (within a few ulp for the continuous values, and exactly for the
integer boxes away from rounding boundaries).
"""
from __future__ import annotations

import math

import numpy as np

F = np.float32

# Cody-Waite reduction constants for exp(x) = 2^k * exp(r), r = x - k ln 2.
# ln 2 is split into a short high part (9 significant bits, so k * LN2_HI is
# exact for |k| < 2^15) and the float32 rounding of the remainder.
LOG2E = F(1.0 / math.log(2.0))
LN2_HI = F(0.693359375)
LN2_LO = F(math.log(2.0) - 0.693359375)
# 1.5 * 2^23: adding and subtracting it rounds a float32 of magnitude < 2^22
# to the nearest integer (ties to even).
ROUND_SHIFTER = F(12582912.0)
# Taylor coefficients 1/k!, k = 0..7, rounded to float32.  On |r| <= ln2/2 the
# truncation error r^8/8! is below 6e-9, under half an ulp.
INV_FACT = [F(1.0 / math.factorial(k)) for k in range(8)]
EXP_HI = F(88.0)    # above: +inf
EXP_LO = F(-86.0)   # below: 0 (keeps every finite result a normal number)

NEAR_Z = F(0.2)         # cull when the view-space depth is not above this
DILATION = F(0.3)       # low-pass dilation added to the 2D covariance diagonal
SUPPORT_K = F(11.0826)  # box half-extent sqrt(K * var), K >= 2 ln 255
CLAMP_FOV = F(1.3)      # Jacobian guard: |x/z| <= 1.3 * max(cx, W - cx) / fx
HALF = F(0.5)
ONE = F(1.0)
TWO = F(2.0)


def bexp32(x):
    """exp(x) in float32 from basic operations only (Cody-Waite range
    reduction, degree-7 Horner polynomial, exponent-field scaling)."""
    x = np.asarray(x, dtype=np.float32)
    nan = np.isnan(x)
    hi = x > EXP_HI
    lo = x < EXP_LO
    xs = np.where(nan | hi | lo, F(0.0), x).astype(np.float32)
    t = xs * LOG2E
    k = (t + ROUND_SHIFTER) - ROUND_SHIFTER
    r = (xs - k * LN2_HI) - k * LN2_LO
    p = INV_FACT[7]
    for c in INV_FACT[6::-1]:
        p = p * r + c
    ki = k.astype(np.int32)
    scale = ((ki + 127).astype(np.uint32) << np.uint32(23)).view(np.float32)
    y = (p * scale).astype(np.float32)
    y = np.where(hi, F(np.inf), y)
    y = np.where(lo, F(0.0), y)
    y = np.where(nan, F(np.nan), y)
    return y.astype(np.float32)


def camera_f32(cam):
    """Camera fields as float32 scalars plus integer width/height."""
    R = np.asarray(cam.R, dtype=np.float32).reshape(3, 3)
    t = np.asarray(cam.t, dtype=np.float32).reshape(3)
    return R, t, F(cam.fx), F(cam.fy), F(cam.cx), F(cam.cy), int(cam.width), int(cam.height)


def spec32(mean, log_scale, quat, cam, tile_size):
    """Binning decisions of every Gaussian in one view.

    mean, log_scale: (3, N); quat: (4, N) as (w, x, y, z).  All float32.
    Returns a dict with ``visible`` (bool), ``zbits`` (uint32 bit pattern of
    the view-space depth), ``box`` = (i0, i1, j0, j1) inclusive pixel bounds
    clamped to the image, and ``rect`` = (tx0, tx1, ty0, ty1) inclusive tile
    bounds.  Entries of culled Gaussians are zero.
    """
    with np.errstate(all="ignore"):
        return _spec32(np.asarray(mean, np.float32), np.asarray(log_scale, np.float32),
                       np.asarray(quat, np.float32), cam, int(tile_size))


def _spec32(mean, log_scale, quat, cam, ts):
    R, t, fx, fy, cx, cy, W, H = camera_f32(cam)
    X, Y, Z = mean[0], mean[1], mean[2]
    w, x, y, z = quat[0], quat[1], quat[2], quat[3]

    # 1. normalise the quaternion
    n2 = ((w * w + x * x) + y * y) + z * z
    q_ok = n2 > F(0.0)
    n = np.sqrt(np.where(q_ok, n2, ONE))
    qw, qx, qy, qz = w / n, x / n, y / n, z / n

    # 2. rotation matrix of the unit quaternion
    r00 = ONE - TWO * (qy * qy + qz * qz)
    r01 = TWO * (qx * qy - qw * qz)
    r02 = TWO * (qx * qz + qw * qy)
    r10 = TWO * (qx * qy + qw * qz)
    r11 = ONE - TWO * (qx * qx + qz * qz)
    r12 = TWO * (qy * qz - qw * qx)
    r20 = TWO * (qx * qz - qw * qy)
    r21 = TWO * (qy * qz + qw * qx)
    r22 = ONE - TWO * (qx * qx + qy * qy)
    rq = ((r00, r01, r02), (r10, r11, r12), (r20, r21, r22))

    # 3-4. scales and M = R_q diag(s)
    s = [bexp32(log_scale[j]) for j in range(3)]
    m = [[rq[i][j] * s[j] for j in range(3)] for i in range(3)]

    # 5. view-space centre
    xc = ((R[0, 0] * X + R[0, 1] * Y) + R[0, 2] * Z) + t[0]
    yc = ((R[1, 0] * X + R[1, 1] * Y) + R[1, 2] * Z) + t[1]
    zc = ((R[2, 0] * X + R[2, 1] * Y) + R[2, 2] * Z) + t[2]
    z_ok = zc > NEAR_Z

    # 6. projected centre
    xz = xc / zc
    yz = yc / zc
    u = fx * xz + cx
    v = fy * yz + cy

    # 7. Jacobian guard
    lim_x = CLAMP_FOV * (np.maximum(cx, F(W) - cx) / fx)
    lim_y = CLAMP_FOV * (np.maximum(cy, F(H) - cy) / fy)
    xt = np.minimum(np.maximum(xz, -lim_x), lim_x)
    yt = np.minimum(np.maximum(yz, -lim_y), lim_y)

    # 8. projection Jacobian
    j00 = fx / zc
    j02 = -((fx * xt) / zc)
    j11 = fy / zc
    j12 = -((fy * yt) / zc)

    # 9. T = J R_view (2 x 3)
    t0 = [j00 * R[0, k] + j02 * R[2, k] for k in range(3)]
    t1 = [j11 * R[1, k] + j12 * R[2, k] for k in range(3)]

    # 10. A = T M
    a0 = [(t0[0] * m[0][k] + t0[1] * m[1][k]) + t0[2] * m[2][k] for k in range(3)]
    a1 = [(t1[0] * m[0][k] + t1[1] * m[1][k]) + t1[2] * m[2][k] for k in range(3)]

    # 11. diagonal of the dilated 2D covariance
    sxx = ((a0[0] * a0[0] + a0[1] * a0[1]) + a0[2] * a0[2]) + DILATION
    syy = ((a1[0] * a1[0] + a1[1] * a1[1]) + a1[2] * a1[2]) + DILATION

    # 12. half extents of the support ellipse's bounding box
    hx = np.sqrt(SUPPORT_K * sxx)
    hy = np.sqrt(SUPPORT_K * syy)

    # 13. pixel box (pixel i has its centre at i + 0.5)
    finite = np.isfinite(u) & np.isfinite(v) & np.isfinite(hx) & np.isfinite(hy)
    Wf, Hf = F(W), F(H)
    i0f = np.minimum(np.maximum(np.ceil((u - hx) - HALF), F(-1.0)), Wf)
    i1f = np.minimum(np.maximum(np.floor((u + hx) - HALF), F(-1.0)), Wf)
    j0f = np.minimum(np.maximum(np.ceil((v - hy) - HALF), F(-1.0)), Hf)
    j1f = np.minimum(np.maximum(np.floor((v + hy) - HALF), F(-1.0)), Hf)
    good = q_ok & z_ok & finite
    zero = F(0.0)
    i0 = np.where(good, i0f, zero).astype(np.int32)
    i1 = np.where(good, i1f, zero).astype(np.int32)
    j0 = np.where(good, j0f, zero).astype(np.int32)
    j1 = np.where(good, j1f, zero).astype(np.int32)

    # 14. visibility, then clamp to the image
    visible = good & (i0 <= i1) & (j0 <= j1) & (i1 >= 0) & (i0 <= W - 1) & (j1 >= 0) & (j0 <= H - 1)
    i0 = np.where(visible, np.clip(i0, 0, W - 1), 0).astype(np.int32)
    i1 = np.where(visible, np.clip(i1, 0, W - 1), 0).astype(np.int32)
    j0 = np.where(visible, np.clip(j0, 0, H - 1), 0).astype(np.int32)
    j1 = np.where(visible, np.clip(j1, 0, H - 1), 0).astype(np.int32)

    # 15-16. tile rectangle and depth bits
    zbits = np.where(visible, np.asarray(zc, np.float32).view(np.uint32), np.uint32(0)).astype(np.uint32)
    return dict(
        visible=visible,
        zbits=zbits,
        box=(i0, i1, j0, j1),
        rect=(i0 // ts, i1 // ts, j0 // ts, j1 // ts),
        # intermediate values, exposed for the FP64 cross-checks
        u=u, v=v, hx=hx, hy=hy, zc=zc, sxx=sxx, syy=syy,
    )
