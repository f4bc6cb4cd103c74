"""The FV step written in plain PyTorch CPU float64 ops, for reference gradients.

TEST INFRASTRUCTURE ONLY (like the rest of oracle/).  It follows the same
equations in the same order as fv_oracle.c (section 6.2.2: primitives,
rotation into the face frame, x-flux tensor, Lax-Friedrichs average minus
dissipation, rotation back, times |n_f|; forward Euler with dt / V_T), so
torch.autograd yields the exact derivative of that computation.  A test pins
it to the C oracle.
"""

from __future__ import annotations

import numpy as np
import torch


def _prims(U, gamma):
    rho = U[..., 0]
    u = U[..., 1] / rho
    v = U[..., 2] / rho
    p = (gamma - 1.0) * (U[..., 3] - 0.5 * rho * (u * u + v * v))
    c = torch.sqrt(gamma * p / rho)
    return rho, u, v, p, c


def face_flux(UL, UR, nx, ny, gamma=1.4):
    """R_n F |n| for arrays of faces (leading dimensions broadcast)."""
    ln = torch.sqrt(nx * nx + ny * ny)
    ex, ey = nx / ln, ny / ln
    tx, ty = -ey, ex
    rL, uL, vL, pL, cL = _prims(UL, gamma)
    rR, uR, vR, pR, cR = _prims(UR, gamma)
    unL, vtL = uL * ex + vL * ey, uL * tx + vL * ty
    unR, vtR = uR * ex + vR * ey, uR * tx + vR * ty
    QL = torch.stack([rL, rL * unL, rL * vtL, UL[..., 3]], -1)
    QR = torch.stack([rR, rR * unR, rR * vtR, UR[..., 3]], -1)
    GL = torch.stack([rL * unL, rL * unL * unL + pL, rL * unL * vtL, (UL[..., 3] + pL) * unL], -1)
    GR = torch.stack([rR * unR, rR * unR * unR + pR, rR * unR * vtR, (UR[..., 3] + pR) * unR], -1)
    alpha = torch.abs(0.5 * (unL + unR)) + 0.5 * (cL + cR)
    Fp = 0.5 * (GL + GR) - alpha[..., None] * 0.5 * (QR - QL)
    return torch.stack([ln * Fp[..., 0],
                        ln * (Fp[..., 1] * ex + Fp[..., 2] * tx),
                        ln * (Fp[..., 1] * ey + Fp[..., 2] * ty),
                        ln * Fp[..., 3]], -1)


class Mesh:
    def __init__(self, nbr, nrm, area):
        self.nbr = torch.as_tensor(np.asarray(nbr, dtype=np.int64))
        nrm = torch.as_tensor(np.asarray(nrm, dtype=np.float64))
        self.nx, self.ny = nrm[..., 0], nrm[..., 1]
        self.area = torch.as_tensor(np.asarray(area, dtype=np.float64))


def step(mesh: Mesh, U, dt, gamma=1.4):
    """One forward-Euler step; U is a float64 tensor [n, 4]."""
    R = None
    for f in range(3):
        F = face_flux(U, U[mesh.nbr[:, f]], mesh.nx[:, f], mesh.ny[:, f], gamma)
        R = F if R is None else R + F
    coef = dt / mesh.area
    return U - coef[:, None] * R


def rollout(mesh: Mesh, U, dt, n_steps, gamma=1.4):
    for _ in range(n_steps):
        U = step(mesh, U, dt, gamma)
    return U
