"""FP64 EWA projection of 3D Gaussians into one pinhole view (torch, autograd).

The paper renders with the 3DGS image model (Sec. 3.3) and optimises Gaussian
position, scale, rotation, opacity and SH colour by gradients.  Per view v and
Gaussian g this module computes, in float64 from the float32 parameters:

* opacity o = sigmoid(theta), scale s = exp(l), unit quaternion q / |q|
* covariance Sigma = M M^T with M = R(q) diag(s)
* camera-space centre x_c = R_v mu + t_v and 2D mean
  mu' = (fx x/z + cx, fy y/z + cy)
* local affine Jacobian J of the perspective map at x_c, its x/z and y/z
  entries clamped to 1.3 max(cx, W - cx)/fx (resp. y) so that Gaussians far
  outside the frustum do not blow up
* 2D covariance Sigma' = J R_v Sigma R_v^T J^T + 0.3 I (low-pass dilation)
  and its inverse, the conic (a, b, c) = (S_yy, -S_xy, S_xx) / det
* colour = max(0, sum_k sh_k Y_k(d) + 0.5), d the unit direction from the
  camera centre C_v = -R_v^T t_v to mu (C_v held constant under pose
  gradients).

Every operation is a differentiable torch op, so ``grad64`` differentiates the
same code.  Parity status: pinned by closed forms (isotropic on-axis and
off-axis projections, a 45-degree rotated anisotropic Gaussian, the clamped
Jacobian, degree-0/1 colours) and by FP64 finite differences.
"""
from __future__ import annotations

import numpy as np
import torch

from .sh64 import sh_basis

DILATION = 0.3
CLAMP_FOV = 1.3


def to_params64(scene_arrays, requires_grad=False):
    """float32 ABI-layout arrays -> dict of float64 torch tensors (same layout)."""
    out = {}
    for k in ("mean", "log_scale", "quat", "opacity_logit", "sh"):
        t = torch.from_numpy(np.asarray(scene_arrays[k], dtype=np.float64).copy())
        t.requires_grad_(requires_grad)
        out[k] = t
    return out


def quat_to_rot(q: torch.Tensor) -> torch.Tensor:
    """Rotation matrices [N,3,3] of quaternions q [N,4] = (w, x, y, z),
    normalised first."""
    q = q / torch.linalg.vector_norm(q, dim=1, keepdim=True)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    r = torch.stack([
        1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
        2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
        2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y),
    ], dim=1)
    return r.reshape(-1, 3, 3)


def camera64(cam):
    R = torch.tensor(np.asarray(cam.R, dtype=np.float32).astype(np.float64)).reshape(3, 3)
    t = torch.tensor(np.asarray(cam.t, dtype=np.float32).astype(np.float64)).reshape(3)
    f = [float(np.float32(v)) for v in (cam.fx, cam.fy, cam.cx, cam.cy)]
    return R, t, f[0], f[1], f[2], f[3], int(cam.width), int(cam.height)


def project_view(p64, sh_degree, cam, index=None, pose=None):
    """Project (a subset ``index`` of) the Gaussians into view ``cam``.

    p64: dict of float64 tensors in the ABI layouts (mean [3,N], log_scale
    [3,N], quat [4,N], opacity_logit [N], sh [K,3,N]).
    pose: optional (R [3,3], t [3]) float64 tensors used in place of the
    camera's rotation and translation in the geometry x_c = R mu + t (R a
    general 3x3 matrix there).  The SH viewing direction always comes from
    the camera's own pose, a constant: the paper detaches the SH colour from
    the camera update (Sec. 3.3, "Optimization"), so pose gradients carry
    only the geometric path.
    Returns dict with mu2 [n,2], conic [n,3] = (a, b, c), opacity [n],
    rgb [n,3], cov2 [n,3] = (S_xx, S_xy, S_yy), depth [n].
    """
    R, t, fx, fy, cx, cy, W, H = camera64(cam)
    if pose is not None:
        R, t = pose
    mean = p64["mean"].T
    ls = p64["log_scale"].T
    quat = p64["quat"].T
    opl = p64["opacity_logit"]
    sh = p64["sh"].permute(2, 0, 1)  # [N, K, 3]
    if index is not None:
        idx = torch.as_tensor(index, dtype=torch.long)
        mean, ls, quat, opl, sh = mean[idx], ls[idx], quat[idx], opl[idx], sh[idx]

    rq = quat_to_rot(quat)
    s = torch.exp(ls)
    M = rq * s[:, None, :]

    xc = mean @ R.T + t
    x, y, z = xc[:, 0], xc[:, 1], xc[:, 2]
    mu2 = torch.stack([fx * x / z + cx, fy * y / z + cy], dim=1)

    lim_x = CLAMP_FOV * max(cx, W - cx) / fx
    lim_y = CLAMP_FOV * max(cy, H - cy) / fy
    xt = torch.clamp(x / z, -lim_x, lim_x)
    yt = torch.clamp(y / z, -lim_y, lim_y)
    zeros = torch.zeros_like(z)
    J = torch.stack([
        torch.stack([fx / z, zeros, -fx * xt / z], dim=1),
        torch.stack([zeros, fy / z, -fy * yt / z], dim=1),
    ], dim=1)  # [n,2,3]

    A = J @ R @ M  # [n,2,3]
    S = A @ A.transpose(1, 2)
    sxx = S[:, 0, 0] + DILATION
    sxy = S[:, 0, 1]
    syy = S[:, 1, 1] + DILATION
    det = sxx * syy - sxy * sxy
    conic = torch.stack([syy / det, -sxy / det, sxx / det], dim=1)

    opacity = torch.sigmoid(opl)

    Rc, tc = camera64(cam)[:2]
    centre = -(Rc.T @ tc)
    dvec = mean - centre
    d = dvec / torch.linalg.vector_norm(dvec, dim=1, keepdim=True)
    basis = sh_basis(d, sh_degree)  # [n,K]
    rgb = torch.clamp_min((basis[:, :, None] * sh).sum(dim=1) + 0.5, 0.0)

    return dict(mu2=mu2, conic=conic, opacity=opacity, rgb=rgb,
                cov2=torch.stack([sxx, sxy, syy], dim=1), depth=z)
