"""Real orthonormal spherical harmonics up to degree 3 (FP64, torch).

The paper carries each Gaussian's colour in spherical harmonics (Sec. 3.3,
"Optimization": SH gradients are detached for the camera update) without
fixing a basis.  This is the real orthonormal basis with the sign pattern
common in graphics, ordered k = l^2 + l + m, m = -l..l, evaluated at a unit
direction d = (x, y, z).  Each constant is sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!)
times the usual factor of the Cartesian polynomial.

Parity status: pinned by orthonormality (quadrature over the sphere) and by
the degree-0/degree-1 closed forms in the tests.
"""
from __future__ import annotations

import math

import torch

C0 = 1.0 / (2.0 * math.sqrt(math.pi))
C1 = math.sqrt(3.0 / (4.0 * math.pi))
C2 = (0.5 * math.sqrt(15.0 / math.pi),
      0.25 * math.sqrt(5.0 / math.pi),
      0.25 * math.sqrt(15.0 / math.pi))
C3 = (0.25 * math.sqrt(35.0 / (2.0 * math.pi)),
      0.5 * math.sqrt(105.0 / math.pi),
      0.25 * math.sqrt(21.0 / (2.0 * math.pi)),
      0.25 * math.sqrt(7.0 / math.pi),
      0.25 * math.sqrt(105.0 / math.pi))


def sh_basis(d: torch.Tensor, degree: int) -> torch.Tensor:
    """Basis values [..., (degree+1)^2] at unit directions d [..., 3]."""
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    out = [torch.full_like(x, C0)]
    if degree >= 1:
        out += [-C1 * y, C1 * z, -C1 * x]
    if degree >= 2:
        xx, yy, zz = x * x, y * y, z * z
        out += [C2[0] * x * y,
                -C2[0] * y * z,
                C2[1] * (2.0 * zz - xx - yy),
                -C2[0] * x * z,
                C2[2] * (xx - yy)]
    if degree >= 3:
        out += [-C3[0] * y * (3.0 * xx - yy),
                C3[1] * x * y * z,
                -C3[2] * y * (4.0 * zz - xx - yy),
                C3[3] * z * (2.0 * zz - 3.0 * xx - 3.0 * yy),
                -C3[2] * x * (4.0 * zz - xx - yy),
                C3[4] * z * (xx - yy),
                -C3[0] * x * (xx - 3.0 * yy)]
    return torch.stack(out, dim=-1)
