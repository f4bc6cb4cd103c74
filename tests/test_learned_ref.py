"""Pins of the learned-correction reference (oracle/learned_ref.py), on the
CPU.  The reference is what the GPU correction and its adjoint are compared
with, so it is checked against things other than itself: finite differences
of its own float64 form, exact conservation (antisymmetry of the added
flux), the plain step at zero parameters, and the bfloat16 rounding rule."""

import json
import os

import numpy as np
import pytest
import torch

from fvgen import ic
from fvgen.mesh import periodic_mesh, permute_mesh, random_permutation
from oracle import learned_ref as LR
from oracle import torch_ref


def small_case(N=4, seed=5):
    m = permute_mesh(periodic_mesh(N, seed=1), random_permutation(2 * N * N, seed))
    P = ic.vortex_primitive(m.centroid)
    U0 = ic.to_conserved(P)
    dt = ic.cfl_dt(P, m.area, m.perimeter, 0.4)
    return m, torch_ref.Mesh(m.nbr, m.nrm, m.area), torch.from_numpy(U0), dt


def rollout(M, U, dt, p, steps, exact):
    for _ in range(steps):
        U = LR.corrected_step(M, U, dt, p, exact=exact)
    return U


def test_zero_parameters_give_the_plain_step():
    m, M, U0, dt = small_case()
    zero = np.zeros(LR.N_PARAMS, np.float32)
    assert torch.equal(LR.corrected_step(M, U0, dt, zero), torch_ref.step(M, U0, dt))


def test_correction_is_conservative():
    """The added face flux is antisymmetric, so sum_i V_i U_i is unchanged
    to round-off while the state itself does change."""
    m, M, U0, dt = small_case(6)
    p = LR.random_params(4, out_scale=0.2)
    U = rollout(M, U0, dt, p, 10, exact=False)
    A = torch.from_numpy(m.area)[:, None]
    drift = (A * U).sum(0) - (A * U0).sum(0)
    scale = (A * U0.abs()).sum(0)
    assert torch.all(drift.abs() <= 1e-13 * scale), drift
    plain = U0
    for _ in range(10):
        plain = torch_ref.step(M, plain, dt)
    assert (U - plain).abs().max() > 1e-4


def test_bf16_rounds_to_nearest_even_and_passes_gradients_through():
    x = torch.tensor([1.0 + 2**-8, 1.0 + 3 * 2**-8, 1.0 + 2**-9, -3.0 - 2**-7 - 2**-8],
                     dtype=torch.float32, requires_grad=True)
    r = LR.bf16(x)
    # ties go to the even mantissa; the bf16 spacing at 1 is 2^-7
    assert r.tolist() == [1.0, 1.0 + 2**-6, 1.0, -3.0 - 2**-6]
    r.sum().backward()
    assert x.grad.tolist() == [1.0, 1.0, 1.0, 1.0]


def test_exact_gradient_matches_finite_differences():
    """Autograd through two corrected steps (float64, no rounding) against
    central differences along random directions in the parameters and in
    the initial state."""
    m, M, U0, dt = small_case(3)
    rng = np.random.default_rng(7)
    p0 = torch.from_numpy(LR.random_params(8, out_scale=0.3).astype(np.float64))
    w = torch.from_numpy(rng.standard_normal((m.n, 4)))

    def loss(p, U):
        return (w * rollout(M, U, dt, p, 2, exact=True)).sum()

    p = p0.clone().requires_grad_(True)
    U = U0.clone().requires_grad_(True)
    loss(p, U).backward()
    for k in range(3):
        dp = torch.from_numpy(rng.standard_normal(LR.N_PARAMS))
        h = 1e-5
        fd = (loss(p0 + h * dp, U0) - loss(p0 - h * dp, U0)) / (2 * h)
        ad = (p.grad * dp).sum()
        assert abs(fd - ad) <= 1e-6 * abs(ad) + 1e-12, (k, fd, ad)
        dU = torch.from_numpy(rng.standard_normal((m.n, 4))) * 1e-2
        fd = (loss(p0, U0 + h * dU) - loss(p0, U0 - h * dU)) / (2 * h)
        ad = (U.grad * dU).sum()
        assert abs(fd - ad) <= 1e-6 * abs(ad) + 1e-12, (k, fd, ad)


def test_rounded_and_exact_forms_agree_to_bfloat16_precision():
    """The rounded network is the exact one up to bfloat16 rounding of its
    inputs, weights and activations (relative 2^-8 each)."""
    m, M, U0, dt = small_case(5)
    p = LR.random_params(9, out_scale=0.2)
    pe = torch.from_numpy(p.astype(np.float64))
    plain = torch_ref.step(M, U0, dt)
    d_r = LR.corrected_step(M, U0, dt, p) - plain
    d_e = LR.corrected_step(M, U0, dt, pe, exact=True) - plain
    err = (d_r - d_e).abs().max() / d_e.abs().max()
    assert 1e-5 < err < 5e-2, err


# ---- hand-worked values (tests/golden/learned_cases.json) --------------------
#
# The pins above fix properties of the reference, not its values.  These fix
# the values: one face whose twelve features are exact, and a sparse network
# whose every sum is exact except at the rounding sites (b1 rounded to
# bfloat16, b2 and b3 kept in float32, a weight that bfloat16 rounds), each
# worked by hand.

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "learned_cases.json")


def golden():
    return json.load(open(GOLDEN))


def golden_params(net):
    """The flat parameter vector (W1 [12][64], b1, W2 [64][64], b2, W3 [64][4],
    b3, [in][out] row-major) of the sparse hand-picked network."""
    W1, b1 = np.zeros((12, 64)), np.zeros(64)
    W2, b2 = np.zeros((64, 64)), np.zeros(64)
    W3, b3 = np.zeros((64, 4)), np.zeros(4)
    for W, key in ((W1, "W1"), (W2, "W2"), (W3, "W3")):
        for i, o, v in net[key]:
            W[i, o] = v
    for b, key in ((b1, "b1"), (b2, "b2"), (b3, "b3")):
        for o, v in net[key]:
            b[o] = v
    return np.concatenate([a.ravel() for a in (W1, b1, W2, b2, W3, b3)]).astype(np.float32)


def face_args(f, reverse=False):
    t = lambda v: torch.tensor([v], dtype=torch.float64)  # noqa: E731
    UL, UR = torch.tensor([f["UL"]], dtype=torch.float64), torch.tensor([f["UR"]], dtype=torch.float64)
    nx, ny = t(f["n"][0]), t(f["n"][1])
    if reverse:
        return UR, UL, -nx, -ny, t(f["aR"]), t(f["aL"]), t(f["cR"]), t(f["cL"])
    return UL, UR, nx, ny, t(f["aL"]), t(f["aR"]), t(f["cL"]), t(f["cR"])


def check_features(L, g):
    f = g["face"]
    for rev, key in ((False, "x_LR"), (True, "x_RL")):
        got = L.features(*face_args(f, rev), gamma=f["gamma"])[0].tolist()
        if got != g["face"][key]:
            return False, f"{key}: {got}"
    return True, "features exact"


def check_mlp(L, g):
    p = golden_params(g["net"])
    for key_x, key_y in (("x_LR", "y_LR"), ("x_RL", "y_RL")):
        x = torch.tensor([g["face"][key_x]], dtype=torch.float64)
        got = L.mlp(x, p)[0]
        want = torch.tensor(g[key_y], dtype=torch.float32)
        if got.dtype != torch.float32 or not torch.equal(got, want):
            return False, f"{key_y}: {got.tolist()}"
    return True, "network outputs exact"


def check_correction(L, g):
    f = g["face"]
    got = L.face_correction(*face_args(f), golden_params(g["net"]), gamma=f["gamma"])[0]
    if got.tolist() != g["correction"]:
        return False, f"correction {got.tolist()}"
    return True, "correction exact"


LEARNED_PINS = (check_features, check_mlp, check_correction)


def test_learned_reference_matches_hand_worked_values():
    g = golden()
    for pin in LEARNED_PINS:
        ok, msg = pin(LR, g)
        assert ok, msg


LEARNED_MUTATIONS = {
    "normal and tangential velocity swapped": (
        "return rho - 1.0, u * ex + v * ey, u * tx + v * ty, p - 1.0",
        "return rho - 1.0, u * tx + v * ty, u * ex + v * ey, p - 1.0"),
    "tangent of the other orientation": ("    tx, ty = -ey, ex\n\n    def side", "    tx, ty = ey, -ex\n\n    def side"),
    "length instead of its square in the area term": ("0.5 * ln * ln * (aL + aR)", "0.5 * ln * (aL + aR)"),
    "pressure without the kinetic energy": ("(U[..., 3] - 0.5 * rho * (u * u + v * v))", "U[..., 3]"),
    "first-layer bias not rounded": ("x @ bf16(W1) + bf16(b1)", "x @ bf16(W1) + b1"),
    "second-layer bias rounded": ("h1 @ bf16(W2) + b2", "h1 @ bf16(W2) + bf16(b2)"),
    "output bias rounded": ("h2 @ bf16(W3) + b3", "h2 @ bf16(W3) + bf16(b3)"),
    "weights not rounded": ("h2 @ bf16(W3) + b3", "h2 @ W3.float() + b3"),
    "hidden activations not rounded": ("h2 = bf16(torch.relu(h1 @ bf16(W2) + b2))",
                                       "h2 = torch.relu(h1 @ bf16(W2) + b2)"),
    "rotation back with the wrong tangent component": (
        "y[..., 1] * ex + y[..., 2] * tx", "y[..., 1] * ex + y[..., 2] * ty"),
    "reversed row keeps the normal": ("features(UR, UL, -nx, -ny, aR, aL, cR, cL, gamma)",
                                      "features(UR, UL, nx, ny, aR, aL, cR, cL, gamma)"),
    "reversed row added instead of subtracted": (
        "(rotate(yA, ex, ey) - rotate(yB, -ex, -ey))", "(rotate(yA, ex, ey) + rotate(yB, -ex, -ey))"),
}


@pytest.mark.parametrize("name", sorted(LEARNED_MUTATIONS))
def test_learned_mutant_is_caught(name):
    """Each planted mistake in a copy of the reference fails a hand-worked pin."""
    import types

    src = open(LR.__file__).read()
    old, new = LEARNED_MUTATIONS[name]
    assert src.count(old) == 1, f"mutation site for '{name}' must occur exactly once"
    mod = types.ModuleType("learned_ref_mutant")
    code = src.replace(old, new).replace("from . import torch_ref", "from oracle import torch_ref")
    exec(compile(code, "learned_ref_mutant.py", "exec"), mod.__dict__)
    g = golden()
    failed = []
    for pin in LEARNED_PINS:
        try:
            ok, _ = pin(mod, g)
        except Exception:
            ok = False
        if not ok:
            failed.append(pin.__name__)
    assert failed, f"mutation '{name}' passed every pin"
