"""Pins of the learned-correction reference (oracle/learned_ref.py), on the
CPU.  The reference is what the GPU correction and its adjoint are compared
with, so it is checked against things other than itself: finite differences
of its own float64 form, exact conservation (antisymmetry of the added
flux), the plain step at zero parameters, and the bfloat16 rounding rule."""

import numpy as np
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
