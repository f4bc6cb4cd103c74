"""Doubly periodic jittered triangle meshes on [0, L]^2.

Geometry conventions (the cell-centred layout of the paper's section 6.2.1):
every cell is a triangle with counter-clockwise vertices P0, P1, P2.  Face f
is the edge P_f -> P_{f+1}; its stored normal is (y_{f+1} - y_f,
-(x_{f+1} - x_f)), i.e. the outward normal scaled by the face length.  The
cell's "volume" is its area.

Recipe: an N x N grid of quads with spacing h = L / N.  Vertices (i, j) with
1 <= i, j <= N - 1 move by independent U(-jitter*h, jitter*h) offsets in x
and y; the seam lines i = 0 and j = 0 stay fixed.  Every coordinate is then
snapped to a multiple of 2^-SNAP_BITS, so that coordinate differences, the
periodic shift by L, and the sum of a cell's three normals are all exact in
binary64.  Consequence: the two sides of a face carry normals that are exact
negatives of each other, and each cell's normals sum to exactly zero.

Quad (i, j) splits into T0 = (v_ij, v_{i+1,j}, v_{i+1,j+1}) and
T1 = (v_ij, v_{i+1,j+1}, v_{i,j+1}); cell id 2 * (j * N + i) + k.
A jitter of 0.2 h keeps every triangle positively oriented.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SNAP_BITS = 32


@dataclass
class Mesh:
    """Per-cell arrays of a closed triangle mesh (every cell has 3 neighbours)."""

    N: int
    L: float
    nbr: np.ndarray  # int32 [n, 3]: neighbour across face f
    nrm: np.ndarray  # float64 [n, 3, 2]: outward normal of face f, |nrm| = face length
    area: np.ndarray  # float64 [n]
    centroid: np.ndarray  # float64 [n, 2], wrapped into [0, L)
    perimeter: np.ndarray  # float64 [n]
    ijk: np.ndarray  # int32 [n, 3]: (i, j, k) of the quad and triangle a cell came from
    # verts: float64 [n, 3, 2] unwrapped vertex coordinates of each cell
    verts: np.ndarray = field(repr=False, default=None)

    @property
    def n(self) -> int:
        return int(self.nbr.shape[0])


def _snap(x: np.ndarray) -> np.ndarray:
    s = float(2**SNAP_BITS)
    return np.round(x * s) / s


def periodic_mesh(N: int, L: float = 10.0, jitter: float = 0.2, seed: int = 1) -> Mesh:
    """Build the N x N-quad periodic mesh (2 N^2 cells) in structured cell order."""
    if N < 2:
        raise ValueError("N must be >= 2 (N = 1 would give repeated neighbours)")
    h = L / N
    ii, jj = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    X = ii * h
    Y = jj * h
    if jitter > 0.0:
        rng = np.random.Generator(np.random.PCG64(seed))
        dx = rng.uniform(-jitter * h, jitter * h, size=(N - 1, N - 1))
        dy = rng.uniform(-jitter * h, jitter * h, size=(N - 1, N - 1))
        X = X.copy()
        Y = Y.copy()
        X[1:, 1:] += dx
        Y[1:, 1:] += dy
    X = _snap(X)
    Y = _snap(Y)
    Ls = float(L)

    # corner (di, dj) of quad (i, j) in unwrapped coordinates
    def corner(di: int, dj: int):
        i2 = ii + di
        j2 = jj + dj
        cx = X[i2 % N, j2 % N] + np.where(i2 >= N, Ls, 0.0)
        cy = Y[i2 % N, j2 % N] + np.where(j2 >= N, Ls, 0.0)
        return cx, cy

    c00 = corner(0, 0)
    c10 = corner(1, 0)
    c11 = corner(1, 1)
    c01 = corner(0, 1)

    # arrays indexed [j, i] so that the flat index is j * N + i
    def flat(a):
        return a.T.reshape(-1)

    n = 2 * N * N
    verts = np.empty((n, 3, 2), dtype=np.float64)
    tri = {0: (c00, c10, c11), 1: (c00, c11, c01)}
    for k in (0, 1):
        for v, (cx, cy) in enumerate(tri[k]):
            verts[k::2, v, 0] = flat(cx)
            verts[k::2, v, 1] = flat(cy)

    x = verts[:, :, 0]
    y = verts[:, :, 1]
    xn = np.roll(x, -1, axis=1)  # P_{f+1}
    yn = np.roll(y, -1, axis=1)
    nrm = np.empty((n, 3, 2), dtype=np.float64)
    nrm[:, :, 0] = yn - y
    nrm[:, :, 1] = -(xn - x)
    area = 0.5 * ((x[:, 1] - x[:, 0]) * (y[:, 2] - y[:, 0]) - (x[:, 2] - x[:, 0]) * (y[:, 1] - y[:, 0]))
    perimeter = np.sqrt(nrm[:, :, 0] ** 2 + nrm[:, :, 1] ** 2).sum(axis=1)
    centroid = np.stack([x.mean(axis=1) % Ls, y.mean(axis=1) % Ls], axis=1)

    # neighbours from the structured layout (checked by tests: reciprocity and
    # exact normal antisymmetry)
    I = flat(ii)
    J = flat(jj)

    def cid(i, j, k):
        return 2 * ((j % N) * N + (i % N)) + k

    nbr = np.empty((n, 3), dtype=np.int64)
    # T0 faces: bottom edge, right edge, diagonal
    nbr[0::2, 0] = cid(I, J - 1, 1)
    nbr[0::2, 1] = cid(I + 1, J, 1)
    nbr[0::2, 2] = cid(I, J, 1)
    # T1 faces: diagonal, top edge, left edge
    nbr[1::2, 0] = cid(I, J, 0)
    nbr[1::2, 1] = cid(I, J + 1, 0)
    nbr[1::2, 2] = cid(I - 1, J, 0)

    ijk = np.empty((n, 3), dtype=np.int32)
    ijk[0::2, 0] = I
    ijk[1::2, 0] = I
    ijk[0::2, 1] = J
    ijk[1::2, 1] = J
    ijk[0::2, 2] = 0
    ijk[1::2, 2] = 1

    return Mesh(
        N=N,
        L=Ls,
        nbr=nbr.astype(np.int32),
        nrm=nrm,
        area=area,
        centroid=centroid,
        perimeter=perimeter,
        ijk=ijk,
        verts=verts,
    )


def random_permutation(n: int, seed: int = 2) -> np.ndarray:
    """Fisher-Yates permutation (new -> old) from numpy's PCG64."""
    return np.random.Generator(np.random.PCG64(seed)).permutation(n).astype(np.int64)


def permute_mesh(mesh: Mesh, perm: np.ndarray) -> Mesh:
    """Relabel cells: new cell k is old cell perm[k].  Local face order is kept."""
    perm = np.asarray(perm, dtype=np.int64)
    n = mesh.n
    if perm.shape != (n,) or not np.array_equal(np.sort(perm), np.arange(n)):
        raise ValueError("perm must be a permutation of range(n)")
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n)
    return Mesh(
        N=mesh.N,
        L=mesh.L,
        nbr=inv[mesh.nbr[perm]].astype(np.int32),
        nrm=mesh.nrm[perm].copy(),
        area=mesh.area[perm].copy(),
        centroid=mesh.centroid[perm].copy(),
        perimeter=mesh.perimeter[perm].copy(),
        ijk=mesh.ijk[perm].copy(),
        verts=None if mesh.verts is None else mesh.verts[perm].copy(),
    )


def shuffled_periodic_mesh(N: int, L: float = 10.0, jitter: float = 0.2, mesh_seed: int = 1,
                           perm_seed: int = 2) -> Mesh:
    """The workload mesh: jittered periodic mesh with cells randomly permuted."""
    m = periodic_mesh(N, L, jitter, mesh_seed)
    return permute_mesh(m, random_permutation(m.n, perm_seed))
