"""Shared set-up for the GPU tests: workloads and comparison helpers."""

from __future__ import annotations

import math

import numpy as np

from fvgen import ic
from fvgen.mesh import periodic_mesh, permute_mesh, random_permutation

# Agreement bar with the FP64 oracle: per component k,
# max_i |U_gpu - U_oracle|_{i,k} / max_i |U_oracle|_{i,k} <= 1e-12.
TOL = 1e-12


def rel_err(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    scale = np.max(np.abs(b), axis=0)
    return np.max(np.abs(a - b), axis=0) / scale


def vortex_case(N: int, perm_seed: int = 2, mesh_seed: int = 1, cfl: float = 0.4):
    """Jittered periodic mesh with cells randomly permuted and the isentropic vortex."""
    m = permute_mesh(periodic_mesh(N, seed=mesh_seed), random_permutation(2 * N * N, perm_seed))
    P = ic.vortex_primitive(m.centroid)
    return m, ic.to_conserved(P), ic.cfl_dt(P, m.area, m.perimeter, cfl)


def bumps_case(N: int, perm_seed: int = 2, mesh_seed: int = 1, ic_seed: int = 3, cfl: float = 0.4):
    """Free stream at Mach 0.5 with 32 Gaussian density/pressure bumps."""
    m = permute_mesh(periodic_mesh(N, seed=mesh_seed), random_permutation(2 * N * N, perm_seed))
    P = ic.bumps_primitive(m.centroid, seed=ic_seed)
    return m, ic.to_conserved(P), ic.cfl_dt(P, m.area, m.perimeter, cfl)


def conserved_totals(m, U):
    return np.sum(m.area[:, None] * U, axis=0)


def log(msg: str) -> None:
    print(msg, flush=True)
