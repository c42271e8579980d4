"""GPU parity of the joint-limit rows against the FP64 reference.

Workloads: the quadruped with every hinge limited to its default angle +- 0.15 rad
(limit rows switch on and off all through a rollout, beside the foot contacts) and a
5-link chain on a slide with limited joints (limit rows only, 16-lane teams).  Same
tolerances as the other parity tests: qacc <= 1e-4 and contact forces <= 1e-3 per
world, states at a switch (a joint within 1e-5 of a range end, a row at its activation
threshold) counted and reported.  The adjoint's gradient through limit rows is checked
against forward-mode dual numbers of the reference rollout.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2502_08844_amd.synth import inputs, robots
from tests.gpu_util import (compare_step, directional_check, gpu_ctx, run_gpu, summarize,
                             teacher_forced)

pytestmark = pytest.mark.gpu

QACC_TOL = 1e-4
FORCE_TOL = 1e-3


@pytest.fixture(scope="module")
def lib():
    return gpu_ctx()


def _check(kind, stats):
    ea, ef, nflag, ntot = summarize(kind, stats)
    assert ea.max() <= QACC_TOL
    if ef.size:
        assert ef.max() <= FORCE_TOL
    assert nflag <= max(1, 0.02 * ntot)


def test_limit_invweight_matches_reference(lib):
    mjh, ctx = lib
    for m in (robots.quadruped_limits(), robots.hinge_chain(n=5, slide_root=True, limit=0.3)):
        gm = ctx.model_upload(m)
        assert gm.nlimit == m.nlimit and gm.nrowmax == 4 * m.opt.nconmax + m.nlimit
        o = oracle.Oracle(m)
        dadr = [k for k, j in zip(m.jnt_dofadr(), m.joints) if j.limited]
        ref = o.dof_invweight()[dadr]
        assert np.allclose(gm.limit_invweight(), ref, rtol=2e-5, atol=0)


def test_single_step_parity_quadruped_limits(lib):
    mjh, ctx = lib
    print("[gpu] parity quadruped_limits nw=203", flush=True)
    m, stats = teacher_forced(ctx, mjh, "quadruped_limits", 203, [0, 5, 50, 150])
    nlim = []
    o = oracle.Oracle(m)
    for s in stats[:2]:
        q, v, ws = s["state"]
        for w in range(0, len(q), 20):
            f = o.forward(q[w], v[w], ws[w], s["ctrl"][0, w])
            nlim.append(f["nrow"] - 4 * f["ncon"])
    print(f"[gpu] active limit rows in sampled states: mean {np.mean(nlim):.2f} "
          f"max {max(nlim)}", flush=True)
    assert max(nlim) >= 2
    _check("quadruped_limits", stats)


@pytest.mark.parametrize("team,block", [(32, 128), (64, 64), (16, 64)])
def test_limits_parity_launch_shapes(lib, team, block):
    mjh, ctx = lib
    print(f"[gpu] parity quadruped_limits team={team} block={block}", flush=True)
    m, stats = teacher_forced(ctx, mjh, "quadruped_limits", 77, [0, 3, 40], seed=2,
                              team=team, block=block)
    _check(f"quadruped_limits-T{team}", stats)


def test_limited_chain_without_contacts(lib):
    """Limit rows alone (no contacts), nv 6 so 16-lane teams, four worlds a wavefront."""
    mjh, ctx = lib
    m = robots.hinge_chain(n=5, slide_root=True, damping=0.05, limit=0.3)
    m.opt.iterations = 4
    nw = 96
    rng = np.random.default_rng(11)
    qp = inputs.f32(rng.uniform(-0.5, 0.5, size=(nw, m.nq)))
    qv = inputs.f32(rng.normal(scale=0.5, size=(nw, m.nv)))
    o = oracle.Oracle(m)
    stats = []
    ws = np.zeros((nw, m.nv))
    for t in range(3):
        g1 = run_gpu(ctx, mjh, m, qp, qv, ws, None, 1, contacts=True)
        cmp = compare_step(m, o, (qp, qv, ws), None, g1)
        cmp["t"], cmp["ncon"] = t, g1["ncon"]
        stats.append(cmp)
        r = run_gpu(ctx, mjh, m, qp, qv, ws, None, 25, contacts=False)
        qp, qv, ws = r["qpos"], r["qvel"], r["qacc"]
    nrows = [o.forward(s["state"][0][w], s["state"][1][w])["nrow"] for s in stats
             for w in range(0, nw, 8)]
    print(f"[gpu] chain limit rows in sampled states: mean {np.mean(nrows):.2f}", flush=True)
    assert np.mean(nrows) >= 1
    _check("chain_limits", stats)


def test_full_size_quadruped_limits(lib):
    mjh, ctx = lib
    from tests.test_gpu_fullsize import _check as full_check, _one_step, _sample, _state
    from tests.gpu_util import workload
    nw, nstep = 8192, 60
    print(f"[gpu] full-size parity quadruped_limits nw={nw} steps={nstep}", flush=True)
    m, qp, qv, u = workload("quadruped_limits", nw, nstep + 1, seed=7)
    w = mjh.World(ctx, m, nw, qpos=qp, qvel=qv)
    w.batch.set_launch(0, 32, 128)
    ut = torch.tensor(u, dtype=torch.float32, device="cuda")
    w.step(ut[:nstep])
    torch.cuda.synchronize()
    assert np.all(w.status.cpu().numpy() & 1 == 0)
    state = _state(w)
    u1 = ut[nstep:nstep + 1].contiguous()
    gpu1 = _one_step(w, mjh, u1)
    full_check("quadruped_limits-full", m, state, u[nstep:nstep + 1], gpu1, _sample(nw))


def test_adjoint_through_limit_rows_vs_dual_numbers(lib):
    mjh, ctx = lib
    H, K, nw = 32, 8, 64
    m = robots.quadruped_limits()
    qp, qv = inputs.initial_state("quadruped_limits", m, nw, seed=4)
    rng = inputs.rng(4, 7)
    qv = inputs.f32(qv + rng.normal(scale=0.1, size=qv.shape))
    u = inputs.f32(rng.uniform(-0.5, 0.5, size=(H, nw, m.nu)))
    print(f"[gpu] adjoint with limits nw={nw} horizon={H}", flush=True)
    w = mjh.World(ctx, m, nw, qpos=qp)
    qv0 = torch.tensor(qv, dtype=torch.float32, device="cuda", requires_grad=True)
    ut = torch.tensor(u, dtype=torch.float32, device="cuda", requires_grad=True)
    loss = mjh.Rollout.apply(qv0, ut, w, H, K)
    loss.sum().backward()
    torch.cuda.synchronize()
    L = loss.detach().cpu().double().numpy()
    gq, gu = qv0.grad.cpu().double().numpy(), ut.grad.cpu().double().numpy()
    o = oracle.Oracle(m)
    dv = np.random.default_rng(6).normal(size=(nw, m.nv))
    du = np.random.default_rng(7).normal(size=(H, nw, m.nu))
    Lr, dL = o.rollout_jvp(qp, qv, u, dv, du, mode=oracle.MODE_CONVERGED, nthreads=16)
    rel_loss = np.abs(L - Lr) / np.abs(Lr)
    rel, smooth = directional_check(o, qp, qv, u, gq, gu, dv, du, dL)
    print(f"[adjoint-limits] loss rel err max {rel_loss.max():.2e}; <grad, d> vs dual JVP, error / "
          f"(|grad| |d|): max {rel[smooth].max():.2e} median {np.median(rel[smooth]):.2e} over "
          f"{smooth.sum()}/{nw} smooth worlds; non-smooth worlds' err "
          f"{np.round(rel[~smooth], 5).tolist()}", flush=True)
    assert rel_loss.max() < 1e-3
    assert smooth.sum() >= 0.9 * nw
    assert rel[smooth].max() < 1e-3


def test_rollout_backward_is_deterministic(lib):
    """Two identical fwd+bwd rollouts with limit rows give bit-identical gradients, also
    with another model's kernels run in between (the reverse pass reads the violated-limit
    list the recomputed step wrote in the adjoint layout, never stale on-chip words)."""
    mjh, ctx = lib
    H, K, nw = 16, 4, 64
    m = robots.quadruped_limits()
    qp, qv = inputs.initial_state("quadruped_limits", m, nw, seed=4)
    u = inputs.controls("quadruped_limits", m, nw, H, seed=4)

    def run(junk):
        if junk:
            wj = mjh.World(ctx, robots.humanoid(), 256)
            wj.step(None, nstep=2)
        w = mjh.World(ctx, m, nw, qpos=qp)
        qv0 = torch.tensor(qv, dtype=torch.float32, device="cuda", requires_grad=True)
        ut = torch.tensor(u, dtype=torch.float32, device="cuda", requires_grad=True)
        mjh.Rollout.apply(qv0, ut, w, H, K).sum().backward()
        torch.cuda.synchronize()
        return qv0.grad.cpu().numpy(), ut.grad.cpu().numpy()

    a, b = run(False), run(True)
    for x, y in zip(a, b):
        assert np.all(np.isfinite(x)) and np.array_equal(x, y)
