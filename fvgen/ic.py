"""Initial states and time steps for the periodic Euler workloads.

States are built in primitive form (rho, u, v, p) and converted to the
conserved vector U = (rho, rho u, rho v, E) with the ideal-gas energy of the
paper's section 6.1, E = p / (gamma - 1) + rho (u^2 + v^2) / 2, gamma = 1.4.
Point values are sampled at cell centroids using the nearest periodic image
of each feature centre.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

GAMMA = 1.4


@dataclass
class Primitive:
    rho: np.ndarray
    u: np.ndarray
    v: np.ndarray
    p: np.ndarray


def _nearest_image(d: np.ndarray, L: float) -> np.ndarray:
    return d - L * np.round(d / L)


def vortex_primitive(centroid: np.ndarray, L: float = 10.0, beta: float = 5.0,
                     center=(5.0, 5.0), u_inf: float = 1.0, v_inf: float = 0.0,
                     gamma: float = GAMMA) -> Primitive:
    """Isentropic vortex of strength beta on a uniform stream rho = p = 1.

    du = -beta/(2 pi) dy e^{(1-r^2)/2}, dv = beta/(2 pi) dx e^{(1-r^2)/2},
    T = 1 - (gamma-1) beta^2 / (8 gamma pi^2) e^{1-r^2}, rho = T^{1/(gamma-1)},
    p = rho T.  It is an exact steady solution of the Euler equations in the
    frame moving with the stream.
    """
    dx = _nearest_image(centroid[:, 0] - center[0], L)
    dy = _nearest_image(centroid[:, 1] - center[1], L)
    r2 = dx * dx + dy * dy
    f = np.exp(0.5 * (1.0 - r2))
    k = beta / (2.0 * math.pi)
    u = u_inf - k * dy * f
    v = v_inf + k * dx * f
    T = 1.0 - (gamma - 1.0) * beta * beta / (8.0 * gamma * math.pi * math.pi) * np.exp(1.0 - r2)
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho * T
    return Primitive(rho, u, v, p)


def vortex_exact_primitive(centroid: np.ndarray, t: float, L: float = 10.0, beta: float = 5.0,
                           center=(5.0, 5.0), u_inf: float = 1.0, v_inf: float = 0.0,
                           gamma: float = GAMMA) -> Primitive:
    """The vortex advected by the free stream for time t (periodic wrap)."""
    c = ((center[0] + u_inf * t) % L, (center[1] + v_inf * t) % L)
    return vortex_primitive(centroid, L, beta, c, u_inf, v_inf, gamma)


def bumps_primitive(centroid: np.ndarray, L: float = 10.0, n_bumps: int = 32, seed: int = 3,
                    mach: float = 0.5, gamma: float = GAMMA) -> Primitive:
    """Free stream at the given Mach number along +x plus Gaussian bumps.

    rho = p = 1 + sum_k a_k g_k with g_k = exp(-d_k^2 / (2 w_k^2)), centres
    U[0, L)^2, a_k ~ U[0.01, 0.1], w_k ~ U[0.1, 0.5]; u = mach * sqrt(gamma),
    the free-stream sound speed at rho = p = 1.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    cx = rng.uniform(0.0, L, size=n_bumps)
    cy = rng.uniform(0.0, L, size=n_bumps)
    a = rng.uniform(0.01, 0.1, size=n_bumps)
    w = rng.uniform(0.1, 0.5, size=n_bumps)
    s = np.zeros(centroid.shape[0])
    for k in range(n_bumps):
        dx = _nearest_image(centroid[:, 0] - cx[k], L)
        dy = _nearest_image(centroid[:, 1] - cy[k], L)
        s += a[k] * np.exp(-(dx * dx + dy * dy) / (2.0 * w[k] * w[k]))
    rho = 1.0 + s
    p = 1.0 + s
    u = np.full_like(rho, mach * math.sqrt(gamma))
    v = np.zeros_like(rho)
    return Primitive(rho, u, v, p)


def uniform_primitive(n: int, rho=1.0, u=0.3, v=-0.2, p=1.0) -> Primitive:
    return Primitive(np.full(n, float(rho)), np.full(n, float(u)), np.full(n, float(v)),
                     np.full(n, float(p)))


def to_conserved(P: Primitive, gamma: float = GAMMA) -> np.ndarray:
    """[n, 4] array of (rho, rho u, rho v, E)."""
    U = np.empty((P.rho.shape[0], 4), dtype=np.float64)
    U[:, 0] = P.rho
    U[:, 1] = P.rho * P.u
    U[:, 2] = P.rho * P.v
    U[:, 3] = P.p / (gamma - 1.0) + 0.5 * P.rho * (P.u * P.u + P.v * P.v)
    return U


def cfl_dt(P: Primitive, area: np.ndarray, perimeter: np.ndarray, cfl: float = 0.4,
           gamma: float = GAMMA) -> float:
    """dt = cfl * min_i area_i / (perimeter_i * (|v_i| + c_i)), from the initial state."""
    c = np.sqrt(gamma * P.p / P.rho)
    speed = np.sqrt(P.u * P.u + P.v * P.v) + c
    return float(cfl * np.min(area / (perimeter * speed)))


def _buckets(centroid: np.ndarray, L: float, reach: float):
    """Cells grouped by square buckets of side >= reach (for local sums)."""
    nb = int(L // reach)
    if nb < 3:
        return None
    b = L / nb
    bx = np.floor(centroid[:, 0] / b).astype(np.int64) % nb
    by = np.floor(centroid[:, 1] / b).astype(np.int64) % nb
    key = bx * nb + by
    order = np.argsort(key, kind="stable")
    start = np.searchsorted(key[order], np.arange(nb * nb + 1))
    return nb, b, order, start


def _near(bk, n: int, x: float, y: float) -> np.ndarray:
    """Indices of the cells in the 3 x 3 buckets around (x, y)."""
    if bk is None:
        return np.arange(n)
    nb, b, order, start = bk
    ix, iy = int(x // b) % nb, int(y // b) % nb
    parts = [order[start[((ix + a) % nb) * nb + (iy + c) % nb]:
                   start[((ix + a) % nb) * nb + (iy + c) % nb + 1]]
             for a in (-1, 0, 1) for c in (-1, 0, 1)]
    return np.concatenate(parts)


def flow_primitive(centroid: np.ndarray, h: float, seed: int, L: float = 10.0,
                   gamma: float = GAMMA) -> Primitive:
    """A seeded flow whose features are sized in mesh cells (h = quad side),
    so that meshes of different resolution see the same local structure:

    a uniform stream (rho = p = 1, speed U[0.2, 0.6] sqrt(gamma), direction
    U[0, 2 pi)) carrying isentropic vortices (core radius R ~ h U[4, 8],
    strength beta ~ U[2, 4], random sign) and Gaussian density/pressure bumps
    (amplitude U[0.01, 0.1], width h U[2, 6]), 3 vortices and 12 bumps per
    128 x 128 quads of area.  Vortex velocities and temperature deficits
    superpose: u = u_inf + sum du_k, T = 1 - sum dT_k, rho = T^(1/(gamma-1))
    + sum bumps, p = rho_v T + sum bumps (rho_v = T^(1/(gamma-1))).  Each
    feature is truncated beyond 6 of its radii (relative size < 2e-8)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = centroid.shape[0]
    quads = (L / h) ** 2
    n_vort = max(1, int(round(3 * quads / 128 ** 2)))
    n_bump = max(1, int(round(12 * quads / 128 ** 2)))
    speed = rng.uniform(0.2, 0.6) * math.sqrt(gamma)
    ang = rng.uniform(0.0, 2.0 * math.pi)
    vc = rng.uniform(0.0, L, size=(n_vort, 2))
    vR = h * rng.uniform(4.0, 8.0, size=n_vort)
    vb = rng.uniform(2.0, 4.0, size=n_vort) * rng.choice([-1.0, 1.0], size=n_vort)
    bc = rng.uniform(0.0, L, size=(n_bump, 2))
    ba = rng.uniform(0.01, 0.1, size=n_bump)
    bw = h * rng.uniform(2.0, 6.0, size=n_bump)

    du = np.zeros(n)
    dv = np.zeros(n)
    dT = np.zeros(n)
    s = np.zeros(n)
    bk = _buckets(centroid, L, 6.0 * 8.0 * h)
    for k in range(n_vort):
        idx = _near(bk, n, vc[k, 0], vc[k, 1])
        dx = _nearest_image(centroid[idx, 0] - vc[k, 0], L) / vR[k]
        dy = _nearest_image(centroid[idx, 1] - vc[k, 1], L) / vR[k]
        r2 = dx * dx + dy * dy
        f = np.where(r2 < 36.0, np.exp(0.5 * (1.0 - r2)), 0.0)
        c = vb[k] / (2.0 * math.pi)
        du[idx] -= c * dy * f
        dv[idx] += c * dx * f
        dT[idx] += (gamma - 1.0) * vb[k] ** 2 / (8.0 * gamma * math.pi ** 2) * f * f
    for k in range(n_bump):
        idx = _near(bk, n, bc[k, 0], bc[k, 1])
        dx = _nearest_image(centroid[idx, 0] - bc[k, 0], L) / bw[k]
        dy = _nearest_image(centroid[idx, 1] - bc[k, 1], L) / bw[k]
        r2 = dx * dx + dy * dy
        s[idx] += ba[k] * np.where(r2 < 36.0, np.exp(-0.5 * r2), 0.0)
    T = 1.0 - dT
    if np.min(T) <= 0.05:
        raise ValueError("vortices overlap too strongly for this seed")
    rv = T ** (1.0 / (gamma - 1.0))
    return Primitive(rv + s, speed * math.cos(ang) + du, speed * math.sin(ang) + dv, rv * T + s)
