"""GPU adjoint of the checkpointed rollout for a model with self-contacts.

Workload: the humanoid (capsule-capsule and sphere-capsule pairs between its own limbs,
plus capsule and sphere feet on the floor), horizon 64, checkpoints every 8 steps, the
loss of the quadruped test (root z against 0.3, plus 1e-3 |u|^2).  Reference: the FP64
rollout's exact directional derivatives (forward-mode dual numbers, solver iterated to
convergence) along random directions of the initial qvel and the controls.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2502_08844_amd.synth import inputs, robots
from tests.gpu_util import directional_check

pytestmark = pytest.mark.gpu

H, K = 64, 8
GRAD_TOL = 1e-3


def _setup(nw, seed):
    m = robots.humanoid()
    qp, qv = inputs.initial_state("humanoid", m, nw, seed=seed)
    rng = inputs.rng(seed, 7)
    qv = inputs.f32(qv + rng.normal(scale=0.1, size=qv.shape))
    u = inputs.f32(rng.uniform(-0.5, 0.5, size=(H, nw, m.nu)))
    return m, qp, qv, u


def _self_contacts(o, m, qp, qv, u):
    """Self-contacts per world over the rollout (FP64 reference, converged solver)."""
    selfp = np.array([0 not in (m.geoms[p[0]].body, m.geoms[p[1]].body) for p in m.pairs])
    q, v, ws = qp.astype(float), qv.astype(float), np.zeros((qp.shape[0], m.nv))
    n = np.zeros(qp.shape[0], dtype=int)
    for s in range(u.shape[0]):
        out = o.step(q, v, ws, u[s][None], nstep=1, mode=oracle.MODE_CONVERGED, nthreads=16)
        for w in range(qp.shape[0]):
            k = out["ncon"][w]
            n[w] += selfp[out["contacts"][w, :k, 16].astype(int)].sum()
        q, v, ws = out["qpos"], out["qvel"], out["qacc"]
    return n


def test_humanoid_gradient_directional_vs_dual_numbers():
    from paper_2502_08844_amd import mjh
    nw = 64
    m, qp, qv, u = _setup(nw, seed=0)
    print(f"[gpu] adjoint rollout humanoid nw={nw} horizon={H} ckpt={K}", flush=True)
    ctx = mjh.Context(0)
    w = mjh.World(ctx, m, nw, qpos=qp)
    qv0 = torch.tensor(qv, dtype=torch.float32, device="cuda", requires_grad=True)
    ut = torch.tensor(u, dtype=torch.float32, device="cuda", requires_grad=True)
    loss = mjh.Rollout.apply(qv0, ut, w, H, K)
    loss.sum().backward()
    torch.cuda.synchronize()
    L = loss.detach().cpu().double().numpy()
    gq, gu = qv0.grad.cpu().double().numpy(), ut.grad.cpu().double().numpy()
    assert np.all(np.isfinite(gq)) and np.all(np.isfinite(gu))
    o = oracle.Oracle(m)
    rng = np.random.default_rng(11)
    dv = rng.normal(size=(nw, m.nv))
    du = rng.normal(size=(H, nw, m.nu))
    Lr, dL = o.rollout_jvp(qp, qv, u, dv, du, mode=oracle.MODE_CONVERGED, nthreads=16)
    rel_loss = np.abs(L - Lr) / np.abs(Lr)
    rel, smooth = directional_check(o, qp, qv, u, gq, gu, dv, du, dL)
    nself = _self_contacts(o, m, qp, qv, u)
    hit = nself > 0
    print(f"[adjoint-self] loss rel err max {rel_loss.max():.2e}; worlds with self-contacts "
          f"{hit.sum()}/{nw} (smooth {(hit & smooth).sum()})", flush=True)
    print(f"[adjoint-self] <grad, d> vs dual JVP, error / (|grad| |d|): smooth worlds with "
          f"self-contacts max {rel[hit & smooth].max():.2e} median "
          f"{np.median(rel[hit & smooth]):.2e}; without max {rel[~hit & smooth].max():.2e}; "
          f"non-smooth worlds' err {np.round(rel[~smooth], 5).tolist()}", flush=True)
    assert rel_loss.max() < 1e-3
    assert (hit & smooth).sum() >= 8  # the self-contact geometry is exercised
    assert smooth.sum() >= 0.75 * nw
    assert rel[smooth].max() < GRAD_TOL
