"""The seeded input generators: mesh validity and the exactness the step relies on."""

import numpy as np
import pytest

from fvgen import ic
from fvgen.mesh import periodic_mesh, permute_mesh, random_permutation, shuffled_periodic_mesh


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
