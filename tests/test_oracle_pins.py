"""Pins of the CPU oracle (no GPU): each checks the oracle against something
the paper or mathematics fixes, not against itself."""

import math

import mpmath
import numpy as np
import pytest

import oracle
import pins
from fvgen import ic
from fvgen.mesh import periodic_mesh, permute_mesh, random_permutation


@pytest.fixture(scope="module")
def o():
    return oracle.default()


@pytest.mark.parametrize("pin", pins.QUICK_PINS + [pins.pin_positivity, pins.pin_cm_is_bfs],
                         ids=lambda f: f.__name__)
def test_pin(o, pin):
    ok, detail = pin(o)
    assert ok, detail


@pytest.mark.slow
def test_vortex_convergence(o):
    """Isentropic vortex closed form: L2 density error falls under refinement
    with an observed order near 1 (the scheme is first order in space and time)."""
    ok, detail = pins.pin_vortex_convergence(o)
    assert ok, detail


def test_brute_force_50_digits(o):
    """One step on the 8-cell mesh, evaluated in 50-digit arithmetic from the
    frame-free form of the flux, agrees with the FP64 oracle to 1e-14."""
    mpmath.mp.dps = 50
    m = permute_mesh(periodic_mesh(2), random_permutation(8, 4))
    P = ic.vortex_primitive(m.centroid)
    U0 = ic.to_conserved(P)
    dt = ic.cfl_dt(P, m.area, m.perimeter)
    got = o.step(m.nbr, m.nrm, m.area, U0, dt, 1)

    gd = mpmath.mpf(1.4)  # the binary64 gamma the oracle uses

    def F(U, nx, ny, gam):
        rho, mx, my, E = U
        u, v = mx / rho, my / rho
        p = (gam - 1) * (E - rho * (u * u + v * v) / 2)
        V = u * nx + v * ny
        return [rho * V, mx * V + p * nx, my * V + p * ny, (E + p) * V], V, mpmath.sqrt(gam * p / rho)

    want = np.zeros_like(U0)
    for i in range(m.n):
        Ui = [mpmath.mpf(float(x)) for x in U0[i]]
        R = [mpmath.mpf(0)] * 4
        for f in range(3):
            j = int(m.nbr[i, f])
            Uj = [mpmath.mpf(float(x)) for x in U0[j]]
            nx, ny = mpmath.mpf(float(m.nrm[i, f, 0])), mpmath.mpf(float(m.nrm[i, f, 1]))
            FL, VL, cL = F(Ui, nx, ny, gd)
            FR, VR, cR = F(Uj, nx, ny, gd)
            s = abs(VL + VR) / 2 + mpmath.sqrt(nx * nx + ny * ny) * (cL + cR) / 2
            for k in range(4):
                R[k] += (FL[k] + FR[k]) / 2 - s * (Uj[k] - Ui[k]) / 2
        for k in range(4):
            want[i, k] = float(Ui[k] - mpmath.mpf(float(dt)) / mpmath.mpf(float(m.area[i])) * R[k])
    scale = np.max(np.abs(want), axis=0)
    err = np.max(np.abs(got - want), axis=0) / scale
    assert np.all(err <= 1e-14), err


def test_renumbering_invariance(o):
    """Stepping a renumbered mesh and undoing the renumbering is bitwise equal
    to stepping the original: the update of a cell reads only its own faces in
    their stored order."""
    N = 16
    m = permute_mesh(periodic_mesh(N), random_permutation(2 * N * N, 2))
    P = ic.vortex_primitive(m.centroid)
    U0 = ic.to_conserved(P)
    dt = ic.cfl_dt(P, m.area, m.perimeter)
    ref = o.step(m.nbr, m.nrm, m.area, U0, dt, 30)
    perm = o.cm_order(m.nbr)
    mc = permute_mesh(m, perm)
    got = o.step(mc.nbr, mc.nrm, mc.area, U0[perm], dt, 30)
    back = np.empty_like(got)
    back[perm] = got
    assert np.array_equal(back, ref)


def test_zero_steps_is_identity(o):
    m, U0, dt = pins.c1_like(4)
    assert np.array_equal(o.step(m.nbr, m.nrm, m.area, U0, dt, 0), U0)


def test_step_composes(o):
    """step(a) then step(b) is bitwise step(a + b)."""
    m, U0, dt = pins.c1_like(8)
    a = o.step(m.nbr, m.nrm, m.area, U0, dt, 7)
    b = o.step(m.nbr, m.nrm, m.area, a, dt, 5)
    assert np.array_equal(b, o.step(m.nbr, m.nrm, m.area, U0, dt, 12))


def test_threaded_steps_equal_sequential(o):
    """The all-core timing variant shares the cells of each step among
    threads; every update reads only the previous state, so it is bitwise the
    sequential oracle."""
    m, U0, dt = pins.c1_like(16)
    ref = o.step(m.nbr, m.nrm, m.area, U0, dt, 9)
    got, used = o.step_threads(m.nbr, m.nrm, m.area, U0, dt, 9, 4)
    assert 1 <= used <= 4
    assert np.array_equal(got, ref)
    with pytest.raises(RuntimeError):
        o.step_threads(m.nbr, m.nrm, m.area, U0, dt, 1, 0)


def test_bad_arguments(o):
    m, U0, dt = pins.c1_like(4)
    with pytest.raises(RuntimeError):
        o.step(m.nbr, m.nrm, m.area, U0, dt, -1)


def test_am1_order_is_valid(o):
    """AM1 on a shuffled 32 x 32 mesh: a permutation in which every cell after
    the first is adjacent to an earlier one (the part grows by neighbours),
    with the band of the structured order."""
    from fvgen.mesh import shuffled_periodic_mesh

    m = shuffled_periodic_mesh(32)
    perm = o.am1_order(m.nbr)
    assert np.array_equal(np.sort(perm), np.arange(m.n))
    lab = np.empty(m.n, dtype=np.int64)
    lab[perm] = np.arange(m.n)
    assert all(np.min(lab[m.nbr[v]]) < lab[v] for v in perm[1:])
    assert o.bandwidth(m.nbr, lab)["B"] <= 3 * 32


def test_torch_reference_matches_oracle(o):
    """The PyTorch CPU transcription of the step (used for reference
    gradients) agrees with the C oracle to round-off."""
    import torch

    from oracle import torch_ref

    m, U0, dt = pins.c1_like(8)
    ref = o.step(m.nbr, m.nrm, m.area, U0, dt, 10)
    got = torch_ref.rollout(torch_ref.Mesh(m.nbr, m.nrm, m.area), torch.from_numpy(U0), dt, 10)
    err = np.max(np.abs(got.numpy() - ref), axis=0) / np.max(np.abs(ref), axis=0)
    assert np.all(err <= 1e-14), err


def test_ladder_search_moves_as_the_helper_counts():
    """The ladder graph of the GPU test of a moving pseudo-peripheral search:
    the helper's George-Liu pass count is 3 (the eccentricity grows once) and
    its final root is the oracle's Cuthill-McKee root."""
    from gpu_helpers import george_liu_passes, ladder_graph

    nbr, _, _ = ladder_graph(40)
    rng = np.random.default_rng(1)
    p0 = rng.permutation(nbr.shape[0])
    inv0 = np.empty_like(p0)
    inv0[p0] = np.arange(p0.size)
    nbr = inv0[nbr[p0]].astype(np.int32)
    assert george_liu_passes(nbr) == 3
    root = int(oracle.cm_order(nbr)[0])
    # an end cell of the ladder (degree 2 through the doubled rung)
    assert len(set(int(x) for x in nbr[root])) == 2
