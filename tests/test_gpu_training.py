"""The training pipeline of the learned correction on the GPU: the
restriction (fv_restrict) against a numpy evaluation, target trajectories
of the batched fine solver against single-mesh runs, a short training run,
and the committed trained parameters on a long rollout."""

import numpy as np
import pytest
import torch as _torch

import paper_1408_5715_amd as fv
from fvgen import ic
from fvgen.nested import nested_pair
from gpu_helpers import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    assert _torch.cuda.is_available(), "GPU tests need a GPU"
    return _torch


def test_restrict_matches_numpy(torch):
    rng = np.random.default_rng(0)
    src = rng.standard_normal((1000, 4))
    idx = rng.integers(0, 1000, size=(300, 7)).astype(np.int32)
    w = rng.random((300, 7))
    out = torch.empty((300, 4), dtype=torch.float64, device="cuda")
    fv.fvgpu.fv_restrict(torch.tensor(src, device="cuda"), torch.tensor(idx, device="cuda"),
                         torch.tensor(w, device="cuda"), out)
    ref = np.einsum("ik,ikc->ic", w, src[idx])
    assert np.max(np.abs(out.cpu().numpy() - ref)) <= 1e-14 * np.max(np.abs(ref))
    idx[5, 3] = 1000  # out of range: that row becomes NaN, the others are unchanged
    fv.fvgpu.fv_restrict(torch.tensor(src, device="cuda"), torch.tensor(idx, device="cuda"),
                         torch.tensor(w, device="cuda"), out)
    o = out.cpu().numpy()
    assert np.all(np.isnan(o[5])) and np.all(np.isfinite(np.delete(o, 5, axis=0)))


def test_targets_match_single_mesh_runs(torch):
    """Batched fine flows, restricted after every r fine steps, equal the
    restriction of each flow advanced alone (same bits)."""
    from paper_1408_5715_amd import learned

    N, r, seeds, steps = 8, 2, [11, 12], 3
    T, coarse, dt_c = learned.make_targets(N, r, seeds, steps, 0.8, torch)
    c, f, idx, w = nested_pair(N, r)
    dt_f = learned.mesh_dt(f, 0.8)
    assert dt_c == r * dt_f
    R = learned.Restriction(idx, w, f.n, 1, torch)
    for b, s in enumerate(seeds):
        sol = fv.Solver(f.nbr, f.nrm, f.area)
        try:
            sol.upload_state(learned.flows(f, 10.0 / N, [s])[0])
            for t in range(steps + 1):
                if t:
                    sol.step(r, dt_f)
                got = T[t, b * c.n:(b + 1) * c.n]
                assert torch.equal(got, R(sol.download_device())), (s, t)
        finally:
            sol.close()


def test_short_training_run(torch):
    """The untrained correction (zero output layer) is the plain solver, so
    the first loss is exactly 1; training then changes the parameters and
    stays finite."""
    from paper_1408_5715_amd import learned

    p0 = learned.init_params(3)
    p, hist = learned.train(N=16, r=2, n_flows=4, window=4, checkpoint=2, horizon=12, iters=12,
                            lr=1e-3, max_lead=4, params0=p0)
    log(f"short training: {[round(h, 4) for h in hist]}")
    assert hist[0] == pytest.approx(1.0, abs=1e-12)
    assert np.all(np.isfinite(hist))
    assert np.max(np.abs(p - p0)) > 0


def test_committed_parameters_long_rollout(torch):
    """The trained correction on a held-out flow: 500 steps stay physical
    (positive density and pressure), conserve mass, momentum and energy to
    round-off, and beat the plain coarse solver against the restricted fine
    solution over 64 steps."""
    from paper_1408_5715_amd import learned

    p = learned.load_params()
    c, f, idx, w = nested_pair(64, 4)
    h = 10.0 / 64
    U0f = learned.flows(f, h, [3001])[0]
    dt_c = 4 * learned.mesh_dt(f, 0.8)
    R = learned.Restriction(idx, w, f.n, 1, torch)
    U0c = R(torch.tensor(U0f, device="cuda")).cpu().numpy()
    s = fv.Solver(c.nbr, c.nrm, c.area)
    try:
        s.set_correction(p)
        s.upload_state(U0c)
        s.step(500, dt_c)
        s.check_state()
        U = s.download()
    finally:
        s.close()
    tot0, tot = (c.area[:, None] * U0c).sum(0), (c.area[:, None] * U).sum(0)
    scale = (c.area[:, None] * np.abs(U0c)).sum(0)
    assert np.all(np.abs(tot - tot0) <= 1e-13 * scale)
    res = learned.compare(p, 64, 4, [3001], 64)
    ratio = res["flows"][0]["ratio"]
    log(f"64 steps at 64x64 quads vs 256x256 restricted: corrected / plain L2 density error {ratio:.3f}")
    assert ratio < 0.9
