"""The seeded input generators: mesh validity and the exactness the step relies on."""

import numpy as np
import pytest

from fvgen import ic
from fvgen.mesh import (irregular_periodic_mesh, periodic_mesh, permute_mesh, random_permutation,
                        shuffled_periodic_mesh)


@pytest.mark.parametrize("N", [2, 3, 8, 37])
def test_mesh_reciprocal_and_exact(N):
    m = shuffled_periodic_mesh(N)
    assert m.n == 2 * N * N
    assert np.all(m.area > 0)
    assert m.area.sum() == pytest.approx(m.L * m.L, rel=1e-13)
    # every face has exactly one partner face with the bitwise-negated normal
    for i in range(m.n):
        for f in range(3):
            j = m.nbr[i, f]
            assert j != i
            hits = [g for g in range(3) if m.nbr[j, g] == i and np.all(m.nrm[j, g] == -m.nrm[i, f])]
            assert len(hits) >= 1
    # normals of each cell close exactly
    assert np.all(m.nrm.sum(axis=1) == 0.0)
    # coordinates snapped to the 2^-32 grid
    assert np.all(m.verts * 2.0**32 == np.round(m.verts * 2.0**32))


@pytest.mark.parametrize("N,seed,refine", [(4, 1, None), (12, 2, None), (33, 3, None),
                                           (16, 4, (3.0, 7.0, 2.0, 2))])
def test_irregular_mesh_reciprocal_exact_and_irregular(N, seed, refine):
    """The irregular-topology mesh keeps every exactness property of the
    structured one, while its vertex degrees vary (the structured split has
    degree 6 at every vertex)."""
    m = irregular_periodic_mesh(N, seed=seed, refine=refine)
    h = m.L / N
    if refine is None:
        assert m.n == 2 * N * N
        assert np.all(m.area >= 0.05 * h * h * (1 - 1e-12))
    else:
        # each split turns one cell into three: refined cells are far smaller
        assert m.n > 2 * N * N and (m.n - 2 * N * N) % 2 == 0
        assert np.all(m.area > 0) and m.area.max() / m.area.min() > 50
    assert m.area.sum() == pytest.approx(m.L * m.L, rel=1e-13)
    for i in range(m.n):
        for f in range(3):
            j = m.nbr[i, f]
            assert j != i
            hits = [g for g in range(3) if m.nbr[j, g] == i and np.all(m.nrm[j, g] == -m.nrm[i, f])]
            assert len(hits) >= 1
    assert np.all(m.nrm.sum(axis=1) == 0.0)
    assert np.all(m.verts * 2.0**32 == np.round(m.verts * 2.0**32))
    # vertex degree = number of triangles around a vertex (each corner of a
    # cell is a vertex; wrap coordinates to identify periodic copies)
    key = np.round((m.verts % m.L) * 2.0**32).astype(np.int64).reshape(-1, 2)
    _, counts = np.unique(key, axis=0, return_counts=True)
    assert counts.sum() == 3 * m.n
    if N >= 12:
        assert counts.min() <= 4 and counts.max() >= 8, (counts.min(), counts.max())
    again = irregular_periodic_mesh(N, seed=seed, refine=refine)
    assert np.array_equal(again.nbr, m.nbr) and np.array_equal(again.nrm, m.nrm)


def test_jitter_bounds_and_seed():
    a = periodic_mesh(16, seed=1)
    b = periodic_mesh(16, seed=1)
    c = periodic_mesh(16, seed=7)
    assert np.array_equal(a.nrm, b.nrm)
    assert not np.array_equal(a.nrm, c.nrm)
    flat = periodic_mesh(16, jitter=0.0)
    h = 10.0 / 16
    assert np.max(np.abs(a.verts - flat.verts)) <= 0.2 * h + 2.0**-32


def test_permutation_relabels_consistently():
    m = periodic_mesh(6)
    perm = random_permutation(m.n, 2)
    mp = permute_mesh(m, perm)
    inv = np.empty(m.n, dtype=np.int64)
    inv[perm] = np.arange(m.n)
    assert np.array_equal(mp.nbr, inv[m.nbr[perm]])
    assert np.array_equal(mp.nrm, m.nrm[perm])


def test_initial_states():
    m = periodic_mesh(32)
    P = ic.vortex_primitive(m.centroid)
    # T_min = 1 - 0.4 * 25 / (8 * 1.4 * pi^2) * e = 0.754, rho_min = T_min^2.5 = 0.494
    assert 0.49 < P.rho.min() < 0.51 and P.rho.max() <= 1.0
    U = ic.to_conserved(P)
    assert U.shape == (m.n, 4)
    B = ic.bumps_primitive(m.centroid)
    assert np.all(B.rho >= 1.0) and np.all(B.p == B.rho)
    dt = ic.cfl_dt(P, m.area, m.perimeter)
    assert 0 < dt < 0.01


def test_nested_restriction_covers_each_fine_cell_once():
    """Every fine cell lies inside the coarse cell it is restricted to (its
    centroid, barycentric test on the coarse triangle's unwrapped vertices),
    each fine cell is used once, and the weights are area fractions."""
    from fvgen.nested import nested_pair

    for N, r in ((3, 2), (4, 4)):
        c, f, idx, w = nested_pair(N, r)
        assert idx.shape == (c.n, r * r)
        assert np.array_equal(np.sort(idx.ravel()), np.arange(f.n))
        assert np.allclose(w.sum(1), 1.0, rtol=0, atol=1e-9)  # coordinates snapped to 2^-32
        v = c.verts  # [n, 3, 2]
        p = f.centroid[idx]  # [n, r^2, 2]
        p = v[:, None, 0] + np.mod(p - v[:, None, 0] + 5.0, 10.0) - 5.0
        e1, e2 = v[:, 1] - v[:, 0], v[:, 2] - v[:, 0]
        d = e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]
        q = p - v[:, None, 0]
        l1 = (q[..., 0] * e2[:, None, 1] - q[..., 1] * e2[:, None, 0]) / d[:, None]
        l2 = (e1[:, None, 0] * q[..., 1] - e1[:, None, 1] * q[..., 0]) / d[:, None]
        assert np.all(l1 > 0) and np.all(l2 > 0) and np.all(l1 + l2 < 1)


def test_flow_features_scale_with_the_given_cell_size():
    """flow_primitive sizes its features by h: the same seed and h give the
    same flow on nested meshes (the coarse state is close to the restricted
    fine one), and the state is physical."""
    from fvgen.nested import nested_pair

    c, f, idx, w = nested_pair(32, 2)
    h = 10.0 / 32
    Pc = ic.flow_primitive(c.centroid, h, 5)
    Pf = ic.flow_primitive(f.centroid, h, 5)
    rf = np.sum(w * Pf.rho[idx], 1)
    assert np.all(Pc.rho > 0) and np.all(Pc.p > 0) and np.all(Pf.p > 0)
    assert np.max(np.abs(rf - Pc.rho)) < 0.05 * np.max(np.abs(Pc.rho - 1.0))


def test_finer_snapping_keeps_exactness_but_not_fixed_point():
    """Coordinates on a 2^-40 grid: twin normals are still exact negations and
    every cell's normals sum to zero (exact differences), but the normals are
    no longer multiples of 2^-32, so the step reads them as float64."""
    m = periodic_mesh(24, snap_bits=40)
    assert np.all(m.nrm.sum(axis=1) == 0.0)
    for i in range(m.n):
        for f in range(3):
            j = m.nbr[i, f]
            assert any(np.all(m.nrm[j, g] == -m.nrm[i, f]) for g in range(3))
    assert np.all(m.verts * 2.0**40 == np.round(m.verts * 2.0**40))
    assert not np.all(m.nrm * 2.0**32 == np.round(m.nrm * 2.0**32))
    with pytest.raises(ValueError):
        periodic_mesh(8, snap_bits=46)
