"""The batched workload: many independent periodic meshes of uneven size."""

from __future__ import annotations

import numpy as np

from . import ic
from .mesh import periodic_mesh, permute_mesh, random_permutation


def batch_workload(n_meshes: int = 64, lo: int = 100, hi: int = 500, seed: int = 4):
    """n_meshes periodic jittered meshes with quads per side log-uniform in
    [lo, hi] (20k-500k cells each for the defaults), each randomly permuted,
    alternating isentropic-vortex (random centre) and bump states, each with
    its own CFL-0.4 time step.

    Returns (meshes, begin offsets [n_meshes + 1], sizes, states, dts)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = np.round(np.exp(rng.uniform(np.log(lo), np.log(hi), n_meshes))).astype(int)
    parts, Us, dts = [], [], []
    for k, N in enumerate(sizes):
        N = int(N)
        m = permute_mesh(periodic_mesh(N, seed=1000 + k), random_permutation(2 * N * N, 2000 + k))
        if k % 2 == 0:
            P = ic.vortex_primitive(m.centroid, center=tuple(rng.uniform(2.0, 8.0, 2)))
        else:
            P = ic.bumps_primitive(m.centroid, seed=3000 + k)
        parts.append(m)
        Us.append(ic.to_conserved(P))
        dts.append(ic.cfl_dt(P, m.area, m.perimeter, 0.4))
    begin = np.concatenate([[0], np.cumsum([m.n for m in parts])]).astype(np.int64)
    return parts, begin, sizes, Us, np.array(dts)


def concat(parts):
    """Concatenated nbr (offset per mesh), nrm and area of a batch."""
    begin = np.concatenate([[0], np.cumsum([m.n for m in parts])]).astype(np.int64)
    nbr = np.concatenate([m.nbr + b for m, b in zip(parts, begin)]).astype(np.int32)
    nrm = np.concatenate([m.nrm for m in parts])
    area = np.concatenate([m.area for m in parts])
    return nbr, nrm, area
