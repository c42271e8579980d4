"""GPU parity of the fourth-order Runge-Kutta integrator (integrator 3: the whole
forward pass at four stages) against the FP64 reference.

* a smooth 4-link chain: one step and 40 steps from the same state (no contacts), the
  GPU's state against the reference's at FP32 accuracy;
* the quadruped from contact-rich states at 32- and 16-lane teams: the reported qacc
  (the first stage's) is the Euler step's from the same state bit for bit, and the
  step's average acceleration (qdot' - qdot) / h is within 1e-4 of max(|a|, g) per
  world with a median below 1e-5, and the first stage's qacc within 1e-4;
* (its rollouts' gradients: tests/test_gpu_adjoint_self.py);
* the Runge-Kutta instantiations of the env kernel and of a batch mixing Euler and
  Runge-Kutta groups reproduce the separate launches.
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
    assert ea[~flag].max() <= 1e-4
    assert err[~flag].max() <= 1e-4 and np.median(err) <= 1e-5
    assert flag.sum() <= max(1, 0.02 * len(flag))


def test_env_step_with_rk4_physics(lib):
    """The env kernel's Runge-Kutta instantiation: its physics equals the plain RK4
    step's with the action held for the substeps."""
    mjh, ctx = lib
    m, qp, qv, u = workload("quadruped_rk4", 64, 21, seed=3)
    r = run_gpu(ctx, mjh, m, qp, qv, None, u[:20], 20, contacts=False)
    qp, qv, ws = r["qpos"], r["qvel"], r["qacc"]
    nw, nsub = 64, 3
    act = u[20:21]
    dev = lambda x: torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float32,
                                    device="cuda").contiguous()
    w = mjh.World(ctx, m, nw, qpos=qp, qvel=qv)
    w.qacc_ws.copy_(dev(ws))
    obs = torch.zeros(1, nw, 12 + 3 * m.nu, device="cuda")
    rew = torch.zeros(1, nw, device="cuda")
    done = torch.zeros(1, nw, dtype=torch.int32, device="cuda")
    w.batch.env_step(nsub, dev(act), torch.zeros(nw, 3, device="cuda"), dev(qp), dev(qv),
                     torch.zeros(nw, m.nu, device="cuda"), obs, rew, done)
    torch.cuda.synchronize()
    p = run_gpu(ctx, mjh, m, qp, qv, ws, np.repeat(act, nsub, 0), nsub, contacts=False)
    keep = done.cpu().numpy()[0] == 0
    assert keep.all()
    np.testing.assert_allclose(w.qpos.cpu().double().numpy()[keep], p["qpos"][keep],
                               rtol=0, atol=1e-6)
    np.testing.assert_allclose(w.qvel.cpu().double().numpy()[keep], p["qvel"][keep],
                               rtol=1e-5, atol=1e-5)


def test_mixed_batch_euler_and_rk4(lib):
    """One launch over an Euler group and a Runge-Kutta group (the RK instantiation
    serves both) equals the two groups' own launches."""
    mjh, ctx = lib
    kinds = ("quadruped", "quadruped_rk4")
    ms, states, ctrls = [], [], []
    for k, kind in enumerate(kinds):
        m, qp, qv, u = workload(kind, 40, 10, seed=5 + k)
        ms.append(m); states.append((qp, qv)); ctrls.append(u)
    sep = [run_gpu(ctx, mjh, m, qp, qv, None, u, 10, contacts=False)
           for m, (qp, qv), u in zip(ms, states, ctrls)]
    gms = [ctx.model_upload(m) for m in ms]
    b = ctx.world_alloc(gms, [40, 40])
    held = []
    for g, (m, (qp, qv), u) in enumerate(zip(ms, states, ctrls)):
        q = torch.as_tensor(qp, dtype=torch.float32, device="cuda").contiguous()
        v = torch.as_tensor(qv, dtype=torch.float32, device="cuda").contiguous()
        a = torch.zeros(40, m.nv, device="cuda")
        st = torch.zeros(40, dtype=torch.int32, device="cuda")
        c = torch.as_tensor(u, dtype=torch.float32, device="cuda").contiguous()
        b.bind_state(g, q, v, a, st)
        b.bind_io(g, c)
        held.append((q, v, a, st, c))
    b.step(10)
    torch.cuda.synchronize()
    for g in range(2):
        np.testing.assert_allclose(held[g][0].cpu().double().numpy(), sep[g]["qpos"],
                                   rtol=0, atol=1e-6)
        np.testing.assert_allclose(held[g][1].cpu().double().numpy(), sep[g]["qvel"],
                                   rtol=1e-5, atol=1e-5)
