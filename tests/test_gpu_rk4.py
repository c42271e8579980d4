"""GPU parity of the fourth-order Runge-Kutta integrator (integrator 3: the whole
forward pass at four stages) against the FP64 reference.

* a smooth 4-link chain: one step and 40 steps from the same state (no contacts), the
  GPU's state against the reference's at FP32 accuracy;
* the quadruped from contact-rich states at 32- and 16-lane teams: the reported qacc
  (the first stage's) is the Euler step's from the same state bit for bit, and the
  step's average acceleration (qdot' - qdot) / h is within 1e-3 of max(|a|, g) per
  world with a median below 1e-5 (as for the implicit integrators: the later stages
  carry the solve's FP32 differences through the stage states).  The first stage
  against the reference is printed; its gate is that of the Euler parity tests;
* rollouts reject the integrator.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2502_08844_amd.synth import robots
from tests.gpu_util import G, compare_step, gpu_ctx, run_gpu, workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    return gpu_ctx()


def test_rk4_smooth_chain(lib):
    mjh, ctx = lib
    m = robots.hinge_chain(n=4, link=0.3)
    m.opt.integrator, m.opt.timestep = 3, 2e-3
    rng = np.random.default_rng(1)
    nw = 64
    qp = rng.uniform(-0.5, 0.5, size=(nw, 4)).astype(np.float32).astype(np.float64)
    qv = rng.normal(size=(nw, 4)).astype(np.float32).astype(np.float64)
    o = oracle.Oracle(m)
    for n, tol in ((1, 2e-6), (40, 2e-5)):
        g = run_gpu(ctx, mjh, m, qp, qv, None, None, n, contacts=False)
        r = o.step(qp.copy(), qv.copy(), nstep=n)
        eq = np.abs(g["qpos"] - r["qpos"]).max()
        ev = np.abs(g["qvel"] - r["qvel"]).max() / np.abs(r["qvel"]).max()
        print(f"[gpu] rk4 chain {n} steps: |d q| {eq:.1e} |d v|/max {ev:.1e}", flush=True)
        assert eq <= tol and ev <= tol


@pytest.mark.parametrize("team,block", [(32, 128), (16, 64)])
def test_rk4_quadruped_parity(lib, team, block):
    mjh, ctx = lib
    m, qp, qv, u = workload("quadruped_rk4", 203, 31, seed=6)
    r = run_gpu(ctx, mjh, m, qp, qv, None, u[:30], 30, team, block, contacts=False)
    qp, qv, ws = r["qpos"], r["qvel"], r["qacc"]
    g = run_gpu(ctx, mjh, m, qp, qv, ws, u[30:31], 1, team, block, contacts=True)
    ge = run_gpu(ctx, mjh, robots.quadruped(), qp, qv, ws, u[30:31], 1, team, block,
                 contacts=True)
    np.testing.assert_array_equal(g["qacc"], ge["qacc"])
    np.testing.assert_array_equal(g["contacts"], ge["contacts"])
    o = oracle.Oracle(m)
    cmp = compare_step(m, o, (qp, qv, ws), u[30:31], g)
    flag = cmp["flag"]
    ref = cmp["ref"]
    h = m.opt.timestep
    a_g, a_r = (g["qvel"] - qv) / h, (ref["qvel"] - qv) / h
    err = np.abs(a_g - a_r).max(1) / np.maximum(np.abs(a_r).max(1), G)
    ea = cmp["err_a"]
    print(f"[parity] quadruped_rk4-T{team}: stage-1 qacc max {ea[~flag].max():.2e} "
          f"(world {int(np.argmax(np.where(flag, 0, ea)))}, median {np.median(ea):.2e}); "
          f"step acceleration max {err[~flag].max():.2e} median {np.median(err):.2e}; "
          f"near-switch {flag.sum()}/{len(flag)}", flush=True)
    assert np.all(g["status"] & 1 == 0)
    assert err[~flag].max() <= 1e-3 and np.median(err) <= 1e-5
    assert flag.sum() <= 0.25 * len(flag)


def test_rollout_rejects_rk4(lib):
    mjh, ctx = lib
    m = robots.quadruped_rk4()
    w = mjh.World(ctx, m, 2)
    u = torch.zeros(4, 2, m.nu, device="cuda")
    loss = torch.zeros(2, device="cuda")
    with pytest.raises(mjh.MjhError):
        w.batch.rollout_fwd(4, 2, u, 2, 0.3, 1e-3, loss)
