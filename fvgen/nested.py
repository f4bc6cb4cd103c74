"""Nested pairs of unjittered periodic meshes and the restriction between them.

With no jitter, the N x N-quad mesh and the rN x rN-quad mesh nest exactly:
coarse quad (I, J) is covered by fine quads (rI + a, rJ + b), 0 <= a, b < r,
and the quad diagonals lie on one line, so coarse triangle T0 (below the
diagonal, vertices (0,0), (1,0), (1,1) of its quad) holds the fine quads with
a > b whole and the T0 halves of those with a = b; T1 the rest.  Each coarse
cell covers r^2 fine cells.  The restriction of a fine state is the
area-weighted mean over them.
"""

from __future__ import annotations

import numpy as np

from .mesh import Mesh, periodic_mesh


def nested_pair(N: int, r: int, L: float = 10.0):
    """(coarse, fine, idx, w): idx int32 [n_coarse, r^2] fine cells in each
    coarse cell, w float64 [n_coarse, r^2] their area fractions (rows sum to
    1 up to rounding)."""
    coarse: Mesh = periodic_mesh(N, L, jitter=0.0)
    fine: Mesh = periodic_mesh(N * r, L, jitter=0.0)
    Nf = N * r
    a, b = np.meshgrid(np.arange(r), np.arange(r), indexing="ij")
    a, b = a.ravel(), b.ravel()
    # fine (quad offset, triangle) lists for coarse triangles k = 0 and 1
    lists = []
    for k in (0, 1):
        sel = []
        for aa, bb in zip(a, b):
            if (k == 0 and aa > bb) or (k == 1 and aa < bb):
                sel += [(aa, bb, 0), (aa, bb, 1)]
            elif aa == bb:
                sel.append((aa, bb, k))
        lists.append(np.array(sel, dtype=np.int64))
    I, J = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    I, J = I.ravel(), J.ravel()
    idx = np.empty((2 * N * N, r * r), dtype=np.int64)
    for k in (0, 1):
        sel = lists[k]
        fi = r * I[:, None] + sel[None, :, 0]
        fj = r * J[:, None] + sel[None, :, 1]
        idx[2 * (J * N + I) + k] = 2 * (fj * Nf + fi) + sel[None, :, 2]
    w = fine.area[idx] / coarse.area[:, None]
    return coarse, fine, idx.astype(np.int32), w
