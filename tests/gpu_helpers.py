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


def bumps_case(N: int, perm_seed: int = 2, mesh_seed: int = 1, ic_seed: int = 3, cfl: float = 0.4,
               snap_bits: int = 32):
    """Free stream at Mach 0.5 with 32 Gaussian density/pressure bumps."""
    m = permute_mesh(periodic_mesh(N, seed=mesh_seed, snap_bits=snap_bits),
                     random_permutation(2 * N * N, perm_seed))
    P = ic.bumps_primitive(m.centroid, seed=ic_seed)
    return m, ic.to_conserved(P), ic.cfl_dt(P, m.area, m.perimeter, cfl)


def conserved_totals(m, U):
    return np.sum(m.area[:, None] * U, axis=0)


def log(msg: str) -> None:
    print(msg, flush=True)


def ladder_graph(length: int):
    """A ladder of `length` rungs (cell 2 i + s on rail s), every cell of
    degree 3 through a doubled rung at both ends: from a cell in the middle
    the pseudo-peripheral search moves to an end (the eccentricity grows), so
    the search takes the path beyond its first confirmation pass."""
    edges = []
    for i in range(length):
        edges.append((2 * i, 2 * i + 1))
        if i + 1 < length:
            edges += [(2 * i, 2 * i + 2), (2 * i + 1, 2 * i + 3)]
    edges += [(0, 1), (2 * length - 2, 2 * length - 1)]
    n = 2 * length
    adj = [[] for _ in range(n)]
    for u, v in edges:
        adj[u].append(v)
        adj[v].append(u)
    assert all(len(a) == 3 for a in adj)
    nbr = np.array(adj, dtype=np.int32)
    nrm = np.empty((n, 3, 2))
    for u in range(n):
        for f, v in enumerate(adj[u]):
            sgn = 1.0 if u < v else -1.0
            nrm[u, f] = (sgn * 1.0, sgn * 0.5)
    return nbr, nrm, np.ones(n)


def george_liu_passes(nbr) -> int:
    """Breadth-first passes the pseudo-peripheral search of the oracle's
    Cuthill-McKee takes on a connected graph whose lowest id is the start."""
    def levels(r):
        dist = -np.ones(nbr.shape[0], dtype=np.int64)
        dist[r] = 0
        q, h = [r], 0
        while h < len(q):
            v = q[h]
            h += 1
            for w in nbr[v]:
                if dist[w] < 0:
                    dist[w] = dist[v] + 1
                    q.append(int(w))
        return dist

    def degree(v):
        return len(set(int(x) for x in nbr[v]) - {v})

    d = levels(0)
    ecc, passes = int(d.max()), 1
    while True:
        last = np.flatnonzero(d == ecc)
        pick = min(last, key=lambda v: (degree(v), v))
        d2 = levels(pick)
        passes += 1
        if int(d2.max()) <= ecc:
            return passes
        d, ecc = d2, int(d2.max())
