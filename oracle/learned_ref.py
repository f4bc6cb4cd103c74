"""Reference of the learned face-flux correction (plain PyTorch CPU).

TEST INFRASTRUCTURE ONLY.  The correction is not in the paper: it is an
addition to its Lax-Friedrichs flux (section 6.2.2).  Definition:

For a face with left state U_L (the cell being updated), right state U_R,
length-scaled outward normal n (length l, unit normal e, tangent t = (-e_y,
e_x)), inverse areas a_L, a_R and c = dt * (1 / V) on both sides:

  features x(L, R, n) = [rho_L - 1, un_L, ut_L, p_L - 1,
                         rho_R - 1, un_R, ut_R, p_R - 1,
                         e_x, e_y, l^2 (a_L + a_R) / 2, l (c_L + c_R) / 2]
  (un, ut: velocity along e and t), computed in float64, then rounded to
  float32 and to bfloat16 (round to nearest even);
  MLP y(x) = W3^T h2 + b3, h2 = bf16(relu(W2^T h1 + b2)),
  h1 = bf16(relu(W1^T x + bf16(b1))), weights rounded to bfloat16 (the first
  layer's bias too), products summed in float32;
  rotated back: R(e) y = (y0, y1 e_x + y2 t_x, y1 e_y + y2 t_y, y3);
  correction = l * (R(e) y(x(L, R, n)) - R(-e) y(x(R, L, -n))),
so the face flux stays exactly antisymmetric (conservation is unchanged).

Parameters: a flat float32 vector W1 [12][64], b1 [64], W2 [64][64],
b2 [64], W3 [64][4], b3 [4] (5252 values, [in][out] row-major).
"""

from __future__ import annotations

import numpy as np
import torch

from . import torch_ref

N_IN, N_HID, N_OUT = 12, 64, 4
N_PARAMS = N_IN * N_HID + N_HID + N_HID * N_HID + N_HID + N_HID * N_OUT + N_OUT


def unpack(params):
    p = torch.as_tensor(params)
    if not p.is_floating_point():
        p = p.float()
    sizes = [N_IN * N_HID, N_HID, N_HID * N_HID, N_HID, N_HID * N_OUT, N_OUT]
    parts = torch.split(p, sizes)
    return (parts[0].reshape(N_IN, N_HID), parts[1], parts[2].reshape(N_HID, N_HID), parts[3],
            parts[4].reshape(N_HID, N_OUT), parts[5])


def bf16(x):
    """Round float32 values to bfloat16 (nearest even) and back to float32.
    Differentiated as the identity (straight through): the value is the
    rounded one, the derivative that of x."""
    x = x.float()
    r = x.detach().to(torch.bfloat16).float()
    return x + (r - x.detach())


def features(UL, UR, nx, ny, aL, aR, cL, cR, gamma=1.4):
    ln = torch.sqrt(nx * nx + ny * ny)
    ex, ey = nx / ln, ny / ln
    tx, ty = -ey, ex

    def side(U):
        rho = U[..., 0]
        u = U[..., 1] / rho
        v = U[..., 2] / rho
        p = (gamma - 1.0) * (U[..., 3] - 0.5 * rho * (u * u + v * v))
        return rho - 1.0, u * ex + v * ey, u * tx + v * ty, p - 1.0

    return torch.stack([*side(UL), *side(UR), ex, ey, 0.5 * ln * ln * (aL + aR),
                        0.5 * ln * (cL + cR)], -1)


def mlp(x64, params, exact=False):
    """exact=True: the same network in float64 without any rounding (a smooth
    function almost everywhere, for finite-difference checks)."""
    W1, b1, W2, b2, W3, b3 = unpack(params)
    if exact:
        W1, b1, W2, b2, W3, b3 = (w.double() for w in (W1, b1, W2, b2, W3, b3))
        h1 = torch.relu(x64 @ W1 + b1)
        h2 = torch.relu(h1 @ W2 + b2)
        return h2 @ W3 + b3
    x = bf16(x64.float())
    h1 = bf16(torch.relu(x @ bf16(W1) + bf16(b1)))
    h2 = bf16(torch.relu(h1 @ bf16(W2) + b2))
    return h2 @ bf16(W3) + b3


def rotate(y, ex, ey):
    tx, ty = -ey, ex
    y = y.double()
    return torch.stack([y[..., 0], y[..., 1] * ex + y[..., 2] * tx,
                        y[..., 1] * ey + y[..., 2] * ty, y[..., 3]], -1)


def face_correction(UL, UR, nx, ny, aL, aR, cL, cR, params, gamma=1.4, exact=False):
    ln = torch.sqrt(nx * nx + ny * ny)
    ex, ey = nx / ln, ny / ln
    yA = mlp(features(UL, UR, nx, ny, aL, aR, cL, cR, gamma), params, exact)
    yB = mlp(features(UR, UL, -nx, -ny, aR, aL, cR, cL, gamma), params, exact)
    return ln[..., None] * (rotate(yA, ex, ey) - rotate(yB, -ex, -ey))


def corrected_step(mesh: torch_ref.Mesh, U, dt, params, gamma=1.4, exact=False):
    """One forward-Euler step with the corrected face flux (differentiable
    in U and params with torch autograd)."""
    inv = 1.0 / mesh.area
    c = dt * inv
    R = None
    for f in range(3):
        j = mesh.nbr[:, f]
        nx, ny = mesh.nx[:, f], mesh.ny[:, f]
        F = torch_ref.face_flux(U, U[j], nx, ny, gamma)
        F = F + face_correction(U, U[j], nx, ny, inv, inv[j], c, c[j], params, gamma, exact)
        R = F if R is None else R + F
    return U - c[:, None] * R


def random_params(seed=0, scale=0.5, out_scale=0.02):
    """Random parameters (test inputs): moderate hidden weights, small output."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((N_IN, N_HID)) * scale
    b1 = rng.standard_normal(N_HID) * 0.1
    W2 = rng.standard_normal((N_HID, N_HID)) * scale / 4
    b2 = rng.standard_normal(N_HID) * 0.1
    W3 = rng.standard_normal((N_HID, N_OUT)) * out_scale
    b3 = rng.standard_normal(N_OUT) * out_scale
    return np.concatenate([a.ravel() for a in (W1, b1, W2, b2, W3, b3)]).astype(np.float32)
