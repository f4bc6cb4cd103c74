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


def _snap(x: np.ndarray, bits: int = SNAP_BITS) -> np.ndarray:
    s = float(2**bits)
    return np.round(x * s) / s


def periodic_mesh(N: int, L: float = 10.0, jitter: float = 0.2, seed: int = 1,
                  snap_bits: int = SNAP_BITS) -> Mesh:
    """Build the N x N-quad periodic mesh (2 N^2 cells) in structured cell order.
    snap_bits: coordinates are multiples of 2^-snap_bits (up to 45 keeps every
    difference and periodic shift exact; above 32 the normals are no longer
    multiples of 2^-32, as on a mesh that was not snapped to that grid)."""
    if not 1 <= snap_bits <= 45:
        raise ValueError("snap_bits must be in [1, 45]")
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
    X = _snap(X, snap_bits)
    Y = _snap(Y, snap_bits)
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


def irregular_periodic_mesh(N: int, L: float = 10.0, jitter: float = 0.2, seed: int = 1,
                            flip_fraction: float = 0.35, passes: int = 3,
                            refine: tuple | None = None) -> Mesh:
    """A doubly periodic triangle mesh of irregular topology (2 N^2 cells):
    the jittered, snapped vertex grid of periodic_mesh, each quad split along
    a random diagonal, then random edge flips (passes x flip_fraction of the
    candidate edges per pass) between triangles that do not touch the
    periodic seam, each flip kept only if the two new triangles have area
    at least 0.05 h^2.  Vertex degrees then range over 3-10 and breadth-first
    levels lose the grid's regularity, as on unstructured (Delaunay-type)
    meshes.  Conventions as for periodic_mesh: counter-clockwise vertices,
    face f = edge P_f -> P_{f+1}, normal (dy, -dx); snapped coordinates, so
    a face's normal is the exact negative of its twin's and a cell's normals
    sum to exactly zero.  Cells in construction order (permute them with
    random_permutation for a random order).

    refine = (cx, cy, radius, levels): local refinement, like a mesh graded
    towards a point: `levels` times, every triangle whose centroid lies
    within `radius` of (cx, cy) (no periodic wrap) is split into three at its
    snapped centroid (its outer edges are kept, so its neighbours are
    untouched), followed by Delaunay edge flips (an edge flips when the
    opposite vertex of one triangle lies inside the other's circumcircle)
    among triangles away from the seam."""
    if N < 4:
        raise ValueError("N must be >= 4")
    h = L / N
    rng = np.random.Generator(np.random.PCG64(seed))
    X = np.add.outer(np.arange(N) * h, np.zeros(N))
    Y = np.add.outer(np.zeros(N), np.arange(N) * h)
    if jitter > 0.0:
        X[1:, 1:] += rng.uniform(-jitter * h, jitter * h, size=(N - 1, N - 1))
        Y[1:, 1:] += rng.uniform(-jitter * h, jitter * h, size=(N - 1, N - 1))
    X = _snap(X)
    Y = _snap(Y)
    Ls = float(L)

    # corners as (vertex id, periodic shift x, periodic shift y); vid = i * N + j
    def corner(i, j):
        return ((i % N) * N + (j % N), int(i >= N), int(j >= N))

    tris = []
    diag = rng.integers(0, 2, size=(N, N))
    for i in range(N):
        for j in range(N):
            a, b, c, d = corner(i, j), corner(i + 1, j), corner(i + 1, j + 1), corner(i, j + 1)
            if diag[i, j] == 0:
                tris += [[a, b, c], [a, c, d]]
            else:
                tris += [[a, b, d], [b, c, d]]

    def xy(cn):
        v, sx, sy = cn
        return X.flat[v] + Ls * sx, Y.flat[v] + Ls * sy

    def area2(t):
        (x0, y0), (x1, y1), (x2, y2) = (xy(c) for c in t)
        return (x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0)

    min_area2 = 2 * 0.05 * h * h
    for _ in range(passes):
        # interior edges: both triangles unshifted (away from the seam)
        owner = {}
        for t, tri in enumerate(tris):
            if any(c[1] or c[2] for c in tri):
                continue
            for f in range(3):
                owner[(tri[f][0], tri[(f + 1) % 3][0])] = (t, f)
        edges = [e for e in owner if e[0] < e[1] and (e[1], e[0]) in owner]
        rng.shuffle(edges)
        busy = set()
        for e in edges[: int(flip_fraction * len(edges))]:
            t1, f1 = owner[e]
            t2, f2 = owner[(e[1], e[0])]
            if t1 in busy or t2 in busy:
                continue
            A, B = tris[t1][f1], tris[t1][(f1 + 1) % 3]
            C = tris[t1][(f1 + 2) % 3]  # t1 = (A, B, C)
            D = tris[t2][(f2 + 2) % 3]  # t2 = (B, A, D)
            n1, n2 = [C, A, D], [D, B, C]
            if area2(n1) < min_area2 or area2(n2) < min_area2:
                continue
            tris[t1], tris[t2] = n1, n2
            busy.update((t1, t2))

    if refine is not None:
        cx, cy, radius, levels = refine
        extra_x, extra_y = [], []  # coordinates of inserted vertices (ids N*N + k)

        def xy(cn):  # noqa: F811 - also knows the inserted vertices
            v, sx, sy = cn
            if v < N * N:
                return X.flat[v] + Ls * sx, Y.flat[v] + Ls * sy
            return extra_x[v - N * N] + Ls * sx, extra_y[v - N * N] + Ls * sy

        def incircle(a, b, c, d):
            # > 0 when d lies inside the circumcircle of the counter-clockwise a, b, c
            (ax, ay), (bx, by), (cx_, cy_), (dx, dy) = (xy(q) for q in (a, b, c, d))
            m = np.array([[ax - dx, ay - dy, (ax - dx) ** 2 + (ay - dy) ** 2],
                          [bx - dx, by - dy, (bx - dx) ** 2 + (by - dy) ** 2],
                          [cx_ - dx, cy_ - dy, (cx_ - dx) ** 2 + (cy_ - dy) ** 2]])
            return float(np.linalg.det(m))

        for _ in range(levels):
            out = []
            for tri in tris:
                pts = [xy(c) for c in tri]
                gx = sum(p[0] for p in pts) / 3.0
                gy = sum(p[1] for p in pts) / 3.0
                if (gx - cx) ** 2 + (gy - cy) ** 2 > radius * radius:
                    out.append(tri)
                    continue
                extra_x.append(float(_snap(np.array(gx))))
                extra_y.append(float(_snap(np.array(gy))))
                g = (N * N + len(extra_x) - 1, 0, 0)
                a, b, c = tri
                out += [[a, b, g], [b, c, g], [c, a, g]]
            tris = out
            for _ in range(4):  # Delaunay flips among unshifted triangles
                owner = {}
                for t, tri in enumerate(tris):
                    if any(c[1] or c[2] for c in tri):
                        continue
                    for f in range(3):
                        owner[(tri[f][0], tri[(f + 1) % 3][0])] = (t, f)
                busy, flipped = set(), 0
                for e in [e for e in owner if e[0] < e[1] and (e[1], e[0]) in owner]:
                    t1, f1 = owner[e]
                    t2, f2 = owner[(e[1], e[0])]
                    if t1 in busy or t2 in busy:
                        continue
                    A, B, C = tris[t1][f1], tris[t1][(f1 + 1) % 3], tris[t1][(f1 + 2) % 3]
                    D = tris[t2][(f2 + 2) % 3]
                    if incircle(A, B, C, D) <= 0:
                        continue
                    n1, n2 = [C, A, D], [D, B, C]
                    if area2(n1) <= 0 or area2(n2) <= 0:
                        continue
                    tris[t1], tris[t2] = n1, n2
                    busy.update((t1, t2))
                    flipped += 1
                if not flipped:
                    break

    n = len(tris)
    verts = np.empty((n, 3, 2), dtype=np.float64)
    for t, tri in enumerate(tris):
        for f, cn in enumerate(tri):
            verts[t, f] = xy(cn)
    x, y = verts[:, :, 0], verts[:, :, 1]
    xn, yn = np.roll(x, -1, axis=1), np.roll(y, -1, axis=1)
    nrm = np.empty((n, 3, 2), dtype=np.float64)
    nrm[:, :, 0] = yn - y
    nrm[:, :, 1] = -(xn - x)
    area = 0.5 * ((x[:, 1] - x[:, 0]) * (y[:, 2] - y[:, 0]) - (x[:, 2] - x[:, 0]) * (y[:, 1] - y[:, 0]))
    if np.any(area <= 0):
        raise RuntimeError("non-positive triangle area")
    perimeter = np.sqrt(nrm[:, :, 0] ** 2 + nrm[:, :, 1] ** 2).sum(axis=1)
    centroid = np.stack([x.mean(axis=1) % Ls, y.mean(axis=1) % Ls], axis=1)
    # neighbours: face (P_f -> P_f+1) meets the face (P_f+1 -> P_f) with the
    # opposite relative periodic shift
    face = {}
    for t, tri in enumerate(tris):
        for f in range(3):
            a, b = tri[f], tri[(f + 1) % 3]
            face[(a[0], b[0], b[1] - a[1], b[2] - a[2])] = (t, f)
    nbr = np.empty((n, 3), dtype=np.int32)
    for (va, vb, dx, dy), (t, f) in face.items():
        nbr[t, f] = face[(vb, va, -dx, -dy)][0]
    return Mesh(N=N, L=Ls, nbr=nbr, nrm=nrm, area=area, centroid=centroid, perimeter=perimeter,
                ijk=np.full((n, 3), -1, dtype=np.int32), verts=verts)
