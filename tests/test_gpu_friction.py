"""GPU parity of the friction-loss rows (dry joint friction) against the FP64 reference.

Workloads: the quadruped with friction loss 3 N m on every hinge (about a fifth of the
hinges stick at a time, the rest slip, so rows sit on all three pieces of their cost),
and a 4-link chain on a slide with friction loss and limits on every joint (16-lane
teams, no contacts).  Same tolerances as the other parity tests: qacc <= 1e-4 and contact
forces <= 1e-3 per world, switch states counted and reported.  The adjoint's gradient
through friction rows is checked against forward-mode dual numbers of the reference.
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


def test_friction_model_dims(lib):
    mjh, ctx = lib
    m = robots.quadruped_friction()
    gm = ctx.model_upload(m)
    assert gm.nfric == 12 and gm.nrowmax == 4 * m.opt.nconmax + 12


def test_single_step_parity_quadruped_friction(lib):
    mjh, ctx = lib
    print("[gpu] parity quadruped_friction nw=203", flush=True)
    m, stats = teacher_forced(ctx, mjh, "quadruped_friction", 203, [0, 5, 50, 150])
    o = oracle.Oracle(m)
    F = robots.QUAD_FRICTIONLOSS
    stick = slip = 0
    for s in stats[1:3]:
        q, v, ws = s["state"]
        for w in range(0, len(q), 20):
            f = o.forward(q[w], v[w], ws[w], s["ctrl"][0, w])
            fr = f["efc_force"][f["nrow"] - 12:]
            slip += int(np.sum(np.abs(np.abs(fr) - F) < 1e-9))
            stick += int(np.sum(np.abs(fr) < F * (1 - 1e-6)))
    print(f"[gpu] friction rows in sampled states: sticking {stick}, slipping {slip}", flush=True)
    assert stick >= 5 and slip >= 5
    _check("quadruped_friction", stats)


@pytest.mark.parametrize("team,block", [(32, 128), (64, 64), (16, 64)])
def test_friction_parity_launch_shapes(lib, team, block):
    mjh, ctx = lib
    print(f"[gpu] parity quadruped_friction team={team} block={block}", flush=True)
    m, stats = teacher_forced(ctx, mjh, "quadruped_friction", 77, [0, 3, 40], seed=2,
                              team=team, block=block)
    _check(f"quadruped_friction-T{team}", stats)


def test_chain_with_friction_and_limits(lib):
    mjh, ctx = lib
    m = robots.hinge_chain(n=4, slide_root=True, damping=0.05, limit=0.3, frictionloss=0.4)
    m.opt.iterations = 6
    nw = 96
    rng = np.random.default_rng(12)
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
    _check("chain_friction_limits", stats)


def test_full_size_quadruped_friction(lib):
    mjh, ctx = lib
    from tests.gpu_util import workload
    from tests.test_gpu_fullsize import _check as full_check, _one_step, _sample, _state
    nw, nstep = 8192, 60
    print(f"[gpu] full-size parity quadruped_friction nw={nw} steps={nstep}", flush=True)
    m, qp, qv, u = workload("quadruped_friction", nw, nstep + 1, seed=7)
    w = mjh.World(ctx, m, nw, qpos=qp, qvel=qv)
    w.batch.set_launch(0, 32, 128)
    ut = torch.tensor(u, dtype=torch.float32, device="cuda")
    w.step(ut[:nstep])
    torch.cuda.synchronize()
    assert np.all(w.status.cpu().numpy() & 1 == 0)
    state = _state(w)
    gpu1 = _one_step(w, mjh, ut[nstep:nstep + 1].contiguous())
    full_check("quadruped_friction-full", m, state, u[nstep:nstep + 1], gpu1, _sample(nw))


def test_adjoint_through_friction_rows_vs_dual_numbers(lib):
    mjh, ctx = lib
    H, K, nw = 32, 8, 64
    m = robots.quadruped_friction()
    qp, qv = inputs.initial_state("quadruped_friction", m, nw, seed=4)
    rng = inputs.rng(4, 7)
    qv = inputs.f32(qv + rng.normal(scale=0.1, size=qv.shape))
    u = inputs.f32(rng.uniform(-0.5, 0.5, size=(H, nw, m.nu)))
    print(f"[gpu] adjoint with friction loss nw={nw} horizon={H}", flush=True)
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
    print(f"[adjoint-friction] loss rel err max {rel_loss.max():.2e}; <grad, d> vs dual JVP, error / "
          f"(|grad| |d|): max {rel[smooth].max():.2e} median {np.median(rel[smooth]):.2e} over "
          f"{smooth.sum()}/{nw} smooth worlds; non-smooth worlds' err "
          f"{np.round(rel[~smooth], 5).tolist()}", flush=True)
    assert np.all(np.isfinite(gq)) and np.all(np.isfinite(gu))
    assert rel_loss.max() < 1e-3
    assert smooth.sum() >= 0.9 * nw
    assert rel[smooth].max() < 1e-3
