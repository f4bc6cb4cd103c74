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
