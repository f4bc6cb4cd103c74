"""Checks that pin the CPU oracle to facts fixed by the paper and by mathematics.

Every function takes an oracle.Oracle (the real build, or a copy with a
planted mistake) and returns (ok: bool, detail: str).  test_oracle_pins
asserts all of them on the real oracle; test_oracle_mutations asserts that
each planted mistake fails at least one.
"""

from __future__ import annotations

import json
import math
import os

import numpy as np

from fvgen import ic
from fvgen.mesh import irregular_periodic_mesh, periodic_mesh, permute_mesh, random_permutation

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
G = 1.4


def _load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# --- independent x-y forms, written from the flux tensor (eqFlux) -------------

def physical_flux_dot_n(U, nx, ny, gamma=G):
    """F(U) . n for the flux tensor of section 6.1 (no numerical flux involved)."""
    rho, mx, my, E = U
    u, v = mx / rho, my / rho
    p = (gamma - 1.0) * (E - 0.5 * rho * (u * u + v * v))
    V = u * nx + v * ny
    return np.array([rho * V, mx * V + p * nx, my * V + p * ny, (E + p) * V])


def lf_xy_form(UL, UR, nx, ny, gamma=G):
    """The Lax-Friedrichs flux written without a face frame.

    With n the length-scaled normal and V = u . n, rotating the face-frame
    flux back and scaling by |n| gives
    (F(U_L) + F(U_R)) . n / 2 - (|V_L + V_R| / 2 + |n| (c_L + c_R) / 2) (U_R - U_L) / 2.
    """
    def prim(U):
        rho, mx, my, E = U
        u, v = mx / rho, my / rho
        p = (gamma - 1.0) * (E - 0.5 * rho * (u * u + v * v))
        return u * nx + v * ny, math.sqrt(gamma * p / rho)

    VL, cL = prim(UL)
    VR, cR = prim(UR)
    ln = math.hypot(nx, ny)
    s = abs(0.5 * (VL + VR)) + 0.5 * ln * (cL + cR)
    return 0.5 * (physical_flux_dot_n(UL, nx, ny, gamma) + physical_flux_dot_n(UR, nx, ny, gamma)) \
        - 0.5 * s * (np.asarray(UR) - np.asarray(UL))


def random_state(rng, n=None):
    rho = rng.uniform(0.3, 3.0, n)
    u = rng.uniform(-2.0, 2.0, n)
    v = rng.uniform(-2.0, 2.0, n)
    p = rng.uniform(0.2, 4.0, n)
    return ic.to_conserved(ic.Primitive(np.atleast_1d(rho), np.atleast_1d(u), np.atleast_1d(v),
                                        np.atleast_1d(p)))


# --- pins ----------------------------------------------------------------------

def pin_golden_faces(o):
    d = _load("lf_face_cases.json")
    worst = 0.0
    for c in d["cases"]:
        F = o.face_flux(c["UL"], c["UR"], c["n"][0], c["n"][1], d["gamma"])
        ref = np.array(c["F"])
        scale = max(1.0, float(np.max(np.abs(ref))))
        err = float(np.max(np.abs(F - ref))) / scale
        worst = max(worst, err)
        if not err <= 4e-15:
            return False, f"{c['name']}: got {F.tolist()} want {c['F']}"
    return True, f"worst {worst:.2e}"


def pin_consistency(o, count=200, seed=11):
    """F^N(U, U, n) equals the physical flux F(U) . n."""
    rng = np.random.default_rng(seed)
    Us = random_state(rng, count)
    worst = 0.0
    for k in range(count):
        th = rng.uniform(0, 2 * math.pi)
        ln = rng.uniform(0.01, 3.0)
        nx, ny = ln * math.cos(th), ln * math.sin(th)
        F = o.face_flux(Us[k], Us[k], nx, ny)
        ref = physical_flux_dot_n(Us[k], nx, ny)
        err = float(np.max(np.abs(F - ref)) / np.max(np.abs(ref)))
        worst = max(worst, err)
    return worst <= 1e-14, f"worst relative {worst:.2e}"


def pin_xy_form(o, count=200, seed=12):
    """The face-frame (rotated) flux equals the frame-free form to round-off."""
    rng = np.random.default_rng(seed)
    UL = random_state(rng, count)
    UR = random_state(rng, count)
    worst = 0.0
    for k in range(count):
        th = rng.uniform(0, 2 * math.pi)
        ln = rng.uniform(0.01, 3.0)
        nx, ny = ln * math.cos(th), ln * math.sin(th)
        F = o.face_flux(UL[k], UR[k], nx, ny)
        ref = lf_xy_form(UL[k], UR[k], nx, ny)
        err = float(np.max(np.abs(F - ref)) / np.max(np.abs(ref)))
        worst = max(worst, err)
    return worst <= 1e-13, f"worst relative {worst:.2e}"


def pin_antisymmetry(o, N=8):
    """flux(i -> j) == -flux(j -> i) bitwise on every face of a jittered mesh."""
    m = permute_mesh(periodic_mesh(N), random_permutation(2 * N * N, 5))
    P = ic.vortex_primitive(m.centroid)
    U = ic.to_conserved(P)
    for i in range(m.n):
        for f in range(3):
            j = int(m.nbr[i, f])
            g = [g for g in range(3) if m.nbr[j, g] == i and np.all(m.nrm[j, g] == -m.nrm[i, f])][0]
            a = o.face_flux(U[i], U[j], *m.nrm[i, f])
            b = o.face_flux(U[j], U[i], *m.nrm[j, g])
            if not np.all(a == -b):
                return False, f"face ({i},{f}) vs ({j},{g}): {a} {b}"
    return True, "bitwise"


def c1_like(N=16, seed_perm=2):
    m = permute_mesh(periodic_mesh(N), random_permutation(2 * N * N, seed_perm))
    P = ic.vortex_primitive(m.centroid)
    return m, ic.to_conserved(P), ic.cfl_dt(P, m.area, m.perimeter)


def pin_conservation(o, N=16, steps=200):
    m, U0, dt = c1_like(N)
    U = o.step(m.nbr, m.nrm, m.area, U0, dt, steps)
    w = m.area[:, None]
    drift = np.abs(np.sum(w * U, 0) - np.sum(w * U0, 0)) / np.sum(w * np.abs(U0), 0)
    return bool(np.all(drift <= 1e-13)), f"drift {drift.tolist()}"


def pin_freestream(o, N=16, steps=200):
    m = permute_mesh(periodic_mesh(N), random_permutation(2 * N * N, 7))
    P = ic.uniform_primitive(m.n, 1.2, 0.7, -0.4, 0.9)
    U0 = ic.to_conserved(P)
    dt = ic.cfl_dt(P, m.area, m.perimeter)
    U = o.step(m.nbr, m.nrm, m.area, U0, dt, steps)
    err = float(np.max(np.abs(U - U0)))
    return err <= 1e-13, f"max |U - U_inf| {err:.2e}"


def pin_translation(o, N=16, steps=50):
    """Unjittered dyadic mesh, y-independent state: rows stay bitwise equal."""
    m = periodic_mesh(N, jitter=0.0)
    L = m.L
    x = m.centroid[:, 0]
    P = ic.Primitive(1.0 + 0.3 * np.sin(2 * math.pi * x / L), 0.6 + 0.1 * np.cos(2 * math.pi * x / L),
                     np.full(m.n, 0.2), 1.0 + 0.2 * np.cos(2 * math.pi * x / L))
    U0 = ic.to_conserved(P)
    dt = ic.cfl_dt(P, m.area, m.perimeter)
    perm = random_permutation(m.n, 9)
    mp = permute_mesh(m, perm)
    U = o.step(mp.nbr, mp.nrm, mp.area, U0[perm], dt, steps)
    # cell (i, j, k) -> row of the permuted mesh
    pos = np.empty((N, N, 2), dtype=np.int64)
    pos[mp.ijk[:, 0], mp.ijk[:, 1], mp.ijk[:, 2]] = np.arange(m.n)
    A = U[pos]  # [i, j, k, 4]
    same = np.all(A == A[:, :1], axis=(1, 2, 3)).all()
    moved = float(np.max(np.abs(U - U0[perm])))
    return bool(same) and moved > 1e-6, f"rows equal: {same}, change {moved:.2e}"


def pin_stability(o, N=8, steps=500, seed=13):
    """A small perturbation of a uniform stream decays (L2, area-weighted)."""
    m = permute_mesh(periodic_mesh(N), random_permutation(2 * N * N, 3))
    rng = np.random.default_rng(seed)
    P = ic.uniform_primitive(m.n, 1.0, 0.5, 0.25, 1.0)
    U0 = ic.to_conserved(P)
    dt = ic.cfl_dt(P, m.area, m.perimeter)
    dU = 1e-6 * rng.standard_normal(U0.shape)
    U = o.step(m.nbr, m.nrm, m.area, U0 + dU, dt, steps)
    w = m.area[:, None]
    n0 = math.sqrt(np.sum(w * dU * dU))
    n1 = math.sqrt(np.sum(w * (U - U0) ** 2))
    return (np.isfinite(n1) and n1 < n0), f"norm {n0:.3e} -> {n1:.3e}"


def pin_positivity(o, N=64, steps=200):
    m, U0, dt = c1_like(N)
    U = o.step(m.nbr, m.nrm, m.area, U0, dt, steps)
    rho = U[:, 0]
    p = 0.4 * (U[:, 3] - 0.5 * (U[:, 1] ** 2 + U[:, 2] ** 2) / rho)
    return bool(np.all(rho > 0) and np.all(p > 0)), f"min rho {rho.min():.4f} min p {p.min():.4f}"


def pin_cm_golden(o):
    d = _load("bandwidth_cases.json")
    for c in d["cases"]:
        if "cm_perm" in c:
            got = o.cm_order(np.array(c["nbr"], dtype=np.int32)).tolist()
            if got != c["cm_perm"]:
                return False, f"{c['name']}: {got} != {c['cm_perm']}"
    return True, "all cases"


def pin_am1_golden(o):
    d = _load("bandwidth_cases.json")
    for c in d["cases"]:
        if "am1_perm" in c:
            got = o.am1_order(np.array(c["nbr"], dtype=np.int32)).tolist()
            if got != c["am1_perm"]:
                return False, f"{c['name']}: {got} != {c['am1_perm']}"
    return True, "all cases"


def pin_bandwidth_golden(o):
    d = _load("bandwidth_cases.json")
    for c in d["cases"]:
        got = o.bandwidth(np.array(c["nbr"], dtype=np.int32), np.array(c["label"], dtype=np.int32))
        want = {"B": c["B"], "C_BW": c["C_BW"], "S_BW": c["S_BW"]}
        if got != want:
            return False, f"{c['name']}: {got} != {want}"
    return True, "all cases"


def pin_cm_is_bfs(o, N=16):
    """The CM labelling is a permutation whose labels never decrease along BFS levels."""
    m = permute_mesh(periodic_mesh(N), random_permutation(2 * N * N, 2))
    perm = o.cm_order(m.nbr)
    if not np.array_equal(np.sort(perm), np.arange(m.n)):
        return False, "not a permutation"
    lab = np.empty(m.n, dtype=np.int64)
    lab[perm] = np.arange(m.n)
    # distance from the root by plain BFS
    dist = np.full(m.n, -1)
    root = perm[0]
    dist[root] = 0
    q = [root]
    for v in q:
        for w in m.nbr[v]:
            if dist[w] < 0:
                dist[w] = dist[v] + 1
                q.append(w)
    if not np.all(np.diff(dist[perm]) >= 0):
        return False, "labels not in BFS level order"
    bw = o.bandwidth(m.nbr, lab)
    return bw["B"] < m.n // 4, f"B after CM {bw['B']}"


def vortex_errors(o, sizes=(16, 32, 64, 128), tf=1.0):
    errs = []
    for N in sizes:
        m = periodic_mesh(N)
        P = ic.vortex_primitive(m.centroid)
        U0 = ic.to_conserved(P)
        ns = math.ceil(tf / ic.cfl_dt(P, m.area, m.perimeter))
        U = o.step(m.nbr, m.nrm, m.area, U0, tf / ns, ns)
        Pe = ic.vortex_exact_primitive(m.centroid, tf)
        errs.append(math.sqrt(np.sum(m.area * (U[:, 0] - Pe.rho) ** 2) / np.sum(m.area)))
    return errs


def pin_vortex_convergence(o, sizes=(16, 32, 64, 128)):
    errs = vortex_errors(o, sizes)
    if not all(np.isfinite(errs)):
        return False, f"errors {errs}"
    dec = all(a > b for a, b in zip(errs, errs[1:]))
    order = math.log2(errs[-2] / errs[-1])
    return dec and 0.7 <= order <= 1.3, f"errors {errs}, finest order {order:.3f}"


def pin_contact_advection(o, N=16, tf=1.0, u=0.6, v=0.8):
    """Density wave at constant velocity and pressure: an exact Euler solution
    that translates by (u, v) t.  The wave varies along x only, so its phase
    moves by k u t; the discrete velocity and pressure stay constant to
    round-off, the phase shift matches to 3 % (the first-order scheme's
    dispersion at 32 cells per wavelength) and the amplitude decays."""
    m = permute_mesh(periodic_mesh(N), random_permutation(2 * N * N, 6))
    k = 2 * math.pi / m.L
    ph = k * m.centroid[:, 0]
    P = ic.Primitive(1.0 + 0.2 * np.sin(ph), np.full(m.n, u), np.full(m.n, v), np.full(m.n, 1.0))
    U0 = ic.to_conserved(P)
    ns = math.ceil(tf / ic.cfl_dt(P, m.area, m.perimeter))
    U = o.step(m.nbr, m.nrm, m.area, U0, tf / ns, ns)
    z0 = np.sum(m.area * (U0[:, 0] - 1.0) * np.exp(-1j * ph))
    z1 = np.sum(m.area * (U[:, 0] - 1.0) * np.exp(-1j * ph))
    shift = float(-np.angle(z1 / z0))
    exact = k * u * tf
    amp = float(abs(z1 / z0))
    uu = U[:, 1] / U[:, 0]
    vv = U[:, 2] / U[:, 0]
    p = 0.4 * (U[:, 3] - 0.5 * U[:, 0] * (uu * uu + vv * vv))
    dev = max(float(np.max(np.abs(uu - u))), float(np.max(np.abs(vv - v))),
              float(np.max(np.abs(p - 1.0))))
    ok = abs(shift - exact) <= 0.03 * exact and 0.3 < amp < 1.0 and dev <= 1e-13
    return ok, f"phase {shift:.4f} vs {exact:.4f}, amplitude {amp:.3f}, u/v/p deviation {dev:.1e}"


def pattern_sbw(nbr, pat):
    """Serial bandwidth of an access pattern (section 4.3), with validity
    checks: every vertex executed by exactly one load; an executed vertex's
    neighbours all loaded in its part; per part, s/e = first/last position of
    an executed vertex's closed neighbourhood (the load itself for a load
    that only brings a ghost), S suffix minimum of s, E prefix maximum of e,
    bandwidth max(E - S) (the section 4.1 definition).  Raises
    AssertionError on an invalid pattern."""
    n = nbr.shape[0]
    idx, ex, pb = pat["idx"], pat["ex"], pat["part_begin"]
    assert pb[0] == 0 and pb[-1] == len(idx), "part offsets"
    counts = np.bincount(idx[ex == 1], minlength=n)
    assert np.all(counts == 1), "every vertex executed exactly once"
    sbw = 0
    for p in range(len(pb) - 1):
        a, b = int(pb[p]), int(pb[p + 1])
        part = idx[a:b]
        local = {int(v): t for t, v in enumerate(part)}
        assert len(local) == b - a, "a vertex loaded twice in one part"
        s = np.arange(b - a)
        e = np.arange(b - a)
        for t in range(b - a):
            if ex[a + t]:
                v = int(part[t])
                ps = [t]
                for w in {int(w) for w in nbr[v] if w != v}:
                    assert w in local, f"neighbour {w} of executed {v} not in part {p}"
                    ps.append(local[w])
                s[t], e[t] = min(ps), max(ps)
        S = np.minimum.accumulate(s[::-1])[::-1]
        E = np.maximum.accumulate(e)
        sbw = max(sbw, int(np.max(E - S)))
    return sbw


def pin_bounded_pattern(o, N=16):
    """Section 4.3 on a shuffled mesh: at AM1's own bandwidth the pattern is
    the AM1 order in one part; at half of it and at 6 the pattern is valid,
    within the bound, and reloads some vertices."""
    m = permute_mesh(periodic_mesh(N), random_permutation(2 * N * N, 2))
    perm = o.am1_order(m.nbr)
    lab = np.empty(m.n, dtype=np.int32)
    lab[perm] = np.arange(m.n, dtype=np.int32)
    full = o.bandwidth(m.nbr, lab)["S_BW"]
    pat = o.am1_bounded(m.nbr, full)
    if len(pat["part_begin"]) != 2 or not np.array_equal(pat["idx"], perm):
        return False, "bound = AM1 bandwidth is not the AM1 order"
    for bound in (full // 2, 6):
        pat = o.am1_bounded(m.nbr, bound)
        try:
            got = pattern_sbw(m.nbr, pat)
        except AssertionError as e:
            return False, f"bound {bound}: {e}"
        if got > bound or len(pat["idx"]) <= m.n:
            return False, f"bound {bound}: bandwidth {got}, length {len(pat['idx'])}"
    return True, f"AM1 bandwidth {full}"


def section41_windows(nbr, perm):
    """Per label i of the labelling perm (new -> old): e(i), s(i) over the
    closed neighbourhood, E(i) = max e(1..i), S(i) = min s(i..n) (section 4.1),
    written here from the definitions."""
    n = len(perm)
    lab = np.empty(n, dtype=np.int64)
    lab[np.asarray(perm)] = np.arange(n)
    s = np.empty(n, dtype=np.int64)
    e = np.empty(n, dtype=np.int64)
    for i, v in enumerate(perm):
        ls = [i] + [int(lab[w]) for w in nbr[v]]
        s[i], e[i] = min(ls), max(ls)
    E = np.maximum.accumulate(e)
    S = np.minimum.accumulate(s[::-1])[::-1]
    return s, e, S, E


def pin_exact_sbw_golden(o):
    """Eq. exact-sbw (section 4.3.1) on the hand-worked AM1 runs."""
    d = _load("bandwidth_cases.json")
    for c in d["cases"]:
        if "am1_exact_sbw" in c:
            _, ex = o.am1_exact_sbw(np.array(c["nbr"], dtype=np.int32))
            if ex.tolist() != c["am1_exact_sbw"]:
                return False, f"{c['name']}: {ex.tolist()} != {c['am1_exact_sbw']}"
    return True, "hand-worked cases"


def pin_exact_sbw_is_the_definition(o):
    """The paper states that Eq. exact-sbw equals the serial bandwidth of
    section 4.1: AM1 always takes a node of u(I), so the union of u(k),
    I <= k <= i, receives the next labels and node(i)'s window ends at
    E(i); hence exact(i) = E(i) - s(i) of the final labelling wherever it is
    defined, and the largest E(i) - s(i) is S_BW = max E(i) - S(i)."""
    graphs = []
    for N, seed in ((6, 2), (9, 3)):
        m = periodic_mesh(N)
        graphs.append(permute_mesh(m, random_permutation(m.n, seed)).nbr)
    for N, seed in ((8, 4), (12, 5)):
        m = irregular_periodic_mesh(N, seed=seed)
        graphs.append(permute_mesh(m, random_permutation(m.n, seed)).nbr)
    for nbr in graphs:
        perm, ex = o.am1_exact_sbw(nbr)
        s, e, S, E = section41_windows(nbr, perm)
        own = E - s
        defined = ex >= 0
        if not np.array_equal(ex[defined], own[defined]):
            k = int(np.flatnonzero(ex[defined] != own[defined])[0])
            return False, f"n={len(perm)}: exact {ex[defined][k]} vs E - s {own[defined][k]}"
        lab = np.empty(len(perm), dtype=np.int32)
        lab[perm] = np.arange(len(perm), dtype=np.int32)
        sbw = o.bandwidth(nbr, lab)["S_BW"]
        if not (int(own.max()) == int(np.max(E - S)) == sbw and int(ex.max()) <= sbw):
            return False, f"n={len(perm)}: max E - s {own.max()}, S_BW {sbw}, max exact {ex.max()}"
    return True, f"{len(graphs)} graphs"


QUICK_PINS = [pin_golden_faces, pin_consistency, pin_xy_form, pin_antisymmetry, pin_conservation,
              pin_freestream, pin_translation, pin_stability, pin_contact_advection, pin_cm_golden,
              pin_am1_golden, pin_bandwidth_golden, pin_bounded_pattern, pin_exact_sbw_golden,
              pin_exact_sbw_is_the_definition]
