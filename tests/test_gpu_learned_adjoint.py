"""The adjoint of the corrected step (fv_step_adjoint_grad): cotangents of
the state and gradients of the correction's parameters, through the C ABI
and the autograd rollout, against the CPU reference (autograd through
oracle/learned_ref.py with bfloat16 rounding differentiated as the identity,
the rule the kernel implements).

Bar: the kernel rounds the output and pre-activation cotangents to bfloat16
before the MFMA products (relative error at most 2^-9 each, so at most
2^-8 on a product of two rounded factors) and sums in float32 in another
order than the reference.  An entry of the correction's part of the state
cotangent, or of the parameter gradient, is a sum of such products, so it
carries at most 2^-8 of the sum of its terms' magnitudes; terms of mixed
sign can cancel, so the bar is twice that against the largest entry,
2 * 2^-8 ~ 7.8e-3 (measured 0.9-3.6e-3).  The plain part of the adjoint is
unchanged and exact (tests/test_gpu_adjoint.py)."""

import numpy as np
import pytest
import torch as _torch

import paper_1408_5715_amd as fv
from gpu_helpers import log, vortex_case
from oracle import learned_ref, torch_ref

pytestmark = pytest.mark.gpu

TOL = 2 * 2.0**-8


@pytest.fixture(scope="module")
def torch():
    assert _torch.cuda.is_available(), "GPU tests need a GPU"
    return _torch


def case(N, seed=0):
    m, U0, dt = vortex_case(N)
    rng = np.random.default_rng(seed)
    U0 = U0 * (1.0 + 0.02 * rng.standard_normal(U0.shape))
    w = rng.standard_normal(U0.shape)
    return m, U0, dt, w


def gpu_one_step(torch, m, U0, dt, lam, params):
    s = fv.Solver(m.nbr, m.nrm, m.area)
    try:
        s.set_correction(params)
        U = torch.tensor(U0, device="cuda")
        L = torch.tensor(lam, device="cuda")
        g = None
        if params is not None:
            g = torch.zeros(fv.FV_CORRECTION_PARAMS, dtype=torch.float64, device="cuda")
        fv.fvgpu.fv_step_adjoint_grad(s.ctx, U, L, dt, g)
        torch.cuda.synchronize()
        return L.cpu().numpy(), None if g is None else g.cpu().numpy()
    finally:
        s.close()


def ref_one_step(m, U0, dt, lam, params):
    M = torch_ref.Mesh(m.nbr, m.nrm, m.area)
    U = _torch.tensor(U0, requires_grad=True)
    p = _torch.tensor(params, requires_grad=True)
    out = learned_ref.corrected_step(M, U, dt, p)
    (out * _torch.from_numpy(lam)).sum().backward()
    U2 = _torch.tensor(U0, requires_grad=True)
    (torch_ref.step(M, U2, dt) * _torch.from_numpy(lam)).sum().backward()
    return U.grad.numpy(), U2.grad.numpy(), p.grad.numpy().astype(np.float64)


def rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("N,seed", [(8, 1), (20, 2)])
def test_one_step_matches_reference(torch, N, seed):
    m, U0, dt, lam = case(N, seed)
    p = learned_ref.random_params(seed + 10, out_scale=0.1)
    lam_g, g_g = gpu_one_step(torch, m, U0, dt, lam, p)
    lam_plain, _ = gpu_one_step(torch, m, U0, dt, lam, None)
    lam_r, lam_r_plain, g_r = ref_one_step(m, U0, dt, lam, p)
    assert rel(lam_plain, lam_r_plain) <= 1e-12
    e_lam = rel(lam_g - lam_plain, lam_r - lam_r_plain)
    e_g = rel(g_g, g_r)
    e_g2 = float(np.linalg.norm(g_g - g_r) / np.linalg.norm(g_r))
    log(f"N={N}: correction part of lambda rel {e_lam:.2e} (size "
        f"{np.max(np.abs(lam_r - lam_r_plain)):.2e}); parameter gradient max rel {e_g:.2e}, "
        f"norm rel {e_g2:.2e}")
    assert e_lam <= TOL
    assert e_g <= TOL
    # every parameter block receives gradient
    for a, b in ((0, 768), (768, 832), (832, 4928), (4928, 4992), (4992, 5248), (5248, 5252)):
        assert np.max(np.abs(g_g[a:b])) > 0


def test_repeatable_bits(torch):
    m, U0, dt, lam = case(16, 3)
    p = learned_ref.random_params(5, out_scale=0.1)
    a = gpu_one_step(torch, m, U0, dt, lam, p)
    b = gpu_one_step(torch, m, U0, dt, lam, p)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_gradient_without_correction_is_an_error(torch):
    m, U0, dt, lam = case(4)
    with pytest.raises(fv.FVError):
        s = fv.Solver(m.nbr, m.nrm, m.area)
        try:
            g = torch.zeros(fv.FV_CORRECTION_PARAMS, dtype=torch.float64, device="cuda")
            fv.fvgpu.fv_step_adjoint_grad(s.ctx, torch.tensor(U0, device="cuda"),
                                          torch.tensor(lam, device="cuda"), dt, g)
        finally:
            s.close()


def test_rollout_gradients_match_reference(torch):
    """Six corrected steps with checkpoints every 2, loss on the states after
    steps 3 and 6: gradients in U0 and in the parameters."""
    from paper_1408_5715_amd.autograd import rollout

    m, U0, dt, w = case(10, 4)
    p = learned_ref.random_params(6, out_scale=0.1)
    w2 = np.stack([w, np.roll(w, 7, axis=0)])
    s = fv.Solver(m.nbr, m.nrm, m.area)
    try:
        x = torch.tensor(U0, device="cuda", requires_grad=True)
        P = torch.tensor(p, requires_grad=True)
        out = rollout(x, s, 6, dt, checkpoint=2, params=P, every=3)
        (out * torch.tensor(w2, device="cuda")).sum().backward()
        gx, gp = x.grad.cpu().numpy(), P.grad.numpy()
    finally:
        s.close()
    M = torch_ref.Mesh(m.nbr, m.nrm, m.area)
    xr = _torch.tensor(U0, requires_grad=True)
    pr = _torch.tensor(p, requires_grad=True)
    U, loss = xr, 0.0
    for k in range(6):
        U = learned_ref.corrected_step(M, U, dt, pr)
        if (k + 1) % 3 == 0:
            loss = loss + (U * _torch.from_numpy(w2[(k + 1) // 3 - 1])).sum()
    loss.backward()
    # plain part, for the size of the correction's share of dL/dU0
    xp = _torch.tensor(U0, requires_grad=True)
    U, lp = xp, 0.0
    for k in range(6):
        U = torch_ref.step(M, U, dt)
        if (k + 1) % 3 == 0:
            lp = lp + (U * _torch.from_numpy(w2[(k + 1) // 3 - 1])).sum()
    lp.backward()
    e_x = rel(gx - xp.grad.numpy(), xr.grad.numpy() - xp.grad.numpy())
    e_p = rel(gp, pr.grad.numpy())
    log(f"rollout: correction part of dL/dU0 rel {e_x:.2e}, parameter gradient rel {e_p:.2e}")
    assert e_x <= TOL and e_p <= TOL
