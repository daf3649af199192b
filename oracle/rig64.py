"""FP64 rig parameterisation of the camera poses and its gradients (test
infrastructure: only the tests, the smoke check and the CPU baseline use it).

The paper links the cameras of the rig rigidly (Sec. 3.1, Eq. 3): the
extrinsics of camera i at time t are the product T_i^t = T_m^t T_{i->m} of the
central camera's pose at that time and the fixed relative transform of camera
i, and it optimises the central poses and, for the other cameras, the
relative transforms (Sec. 3.3, "Optimization").  A pose is stored as 12
numbers, R row-major (9) then t (3), of the 4x4 matrix [[R, t], [0, 1]] that
maps world points to camera coordinates, x_c = R x + t; the product is taken
in the order the paper prints it.

Given per-view pose gradients G_v = dL/d(R_v, t_v) (as ``grad64`` returns
them), ``rig_vjp`` returns dL/dT_m per frame and dL/dT_{i->m} per camera,
by torch autograd through ``compose``, and the gradients in the tangent of a
left perturbation T <- exp(xi^) T, xi = (rho, phi) (translation first), by
autograd through torch.linalg.matrix_exp at xi = 0.

Parity status: pinned in the tests by central differences of ``compose``
and of the perturbed products, by the composition of a pose with its own
inverse, and by the pure-translation case of the tangent.
"""
from __future__ import annotations

import numpy as np
import torch


def to_mat(p):
    """[..., 12] poses -> [..., 4, 4] homogeneous matrices."""
    p = torch.as_tensor(p, dtype=torch.float64)
    top = torch.cat([p[..., :9].reshape(*p.shape[:-1], 3, 3), p[..., 9:].reshape(*p.shape[:-1], 3, 1)], dim=-1)
    bottom = torch.zeros(*p.shape[:-1], 1, 4, dtype=torch.float64)
    bottom[..., 0, 3] = 1.0
    return torch.cat([top, bottom], dim=-2)


def from_mat(m):
    """[..., 4, 4] -> [..., 12]."""
    return torch.cat([m[..., :3, :3].reshape(*m.shape[:-2], 9), m[..., :3, 3]], dim=-1)


def compose(central, relative, view_frame, view_camera):
    """Per-view poses T_v = T_m^{f(v)} T_{c(v)->m} (Eq. 3), [V, 12]."""
    Tm = to_mat(central)[torch.as_tensor(np.asarray(view_frame, np.int64))]
    Tr = to_mat(relative)[torch.as_tensor(np.asarray(view_camera, np.int64))]
    return from_mat(Tm @ Tr)


def hat(xi):
    """Twist xi = (rho, phi) [..., 6] -> 4x4 matrix [[phi]x, rho; 0, 0]."""
    xi = torch.as_tensor(xi, dtype=torch.float64)
    rho, phi = xi[..., :3], xi[..., 3:]
    z = torch.zeros_like(phi[..., 0])
    row0 = torch.stack([z, -phi[..., 2], phi[..., 1], rho[..., 0]], dim=-1)
    row1 = torch.stack([phi[..., 2], z, -phi[..., 0], rho[..., 1]], dim=-1)
    row2 = torch.stack([-phi[..., 1], phi[..., 0], z, rho[..., 2]], dim=-1)
    row3 = torch.stack([z, z, z, z], dim=-1)
    return torch.stack([row0, row1, row2, row3], dim=-2)


def perturbed(p, xi):
    """exp(xi^) T for pose(s) p [..., 12] and twist(s) xi [..., 6], [..., 12]."""
    return from_mat(torch.linalg.matrix_exp(hat(xi)) @ to_mat(p))


def rig_vjp(central, relative, view_frame, view_camera, view_grads):
    """Returns dict of numpy arrays: d_central [F,12], d_relative [K,12],
    xi_central [F,6], xi_relative [K,6] for L with dL/dT_v = view_grads."""
    c = torch.tensor(np.asarray(central, np.float64))
    r = torch.tensor(np.asarray(relative, np.float64))
    G = torch.tensor(np.asarray(view_grads, np.float64))
    xc = torch.zeros(c.shape[0], 6, dtype=torch.float64, requires_grad=True)
    xr = torch.zeros(r.shape[0], 6, dtype=torch.float64, requires_grad=True)
    cm = c.clone().requires_grad_(True)
    rm = r.clone().requires_grad_(True)
    (G * compose(cm, rm, view_frame, view_camera)).sum().backward()
    (G * compose(perturbed(c, xc), perturbed(r, xr), view_frame, view_camera)).sum().backward()
    return dict(d_central=cm.grad.numpy(), d_relative=rm.grad.numpy(), xi_central=xc.grad.numpy(),
                xi_relative=xr.grad.numpy())
