"""GPU adjoint of the checkpointed rollout against the FP64 reference.

Workload: the quadruped, horizon 64, checkpoints every 8 steps, loss
sum_t (torso z_t - 0.3)^2 + 1e-3 |u_t|^2; gradients with respect to the initial qvel
and the 64 x 12 controls.  References: central differences (h = 1e-6) of the FP64
reference rollout (solver iterated to convergence) on 16 worlds, and forward-mode dual
numbers of the same rollout (directional derivatives) on more worlds.
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


def _setup(nw, seed=0):
    m = robots.quadruped()
    qp, qv = inputs.initial_state("quadruped", m, nw, seed=seed)
    rng = inputs.rng(seed, 7)
    qv = inputs.f32(qv + rng.normal(scale=0.1, size=qv.shape))
    u = inputs.f32(rng.uniform(-0.5, 0.5, size=(H, nw, m.nu)))
    return m, qp, qv, u


def _gpu_grads(m, qp, qv, u):
    from paper_2502_08844_amd import mjh
    ctx = mjh.Context(0)
    nw = qp.shape[0]
    w = mjh.World(ctx, m, nw, qpos=qp)
    qv0 = torch.tensor(qv, dtype=torch.float32, device="cuda", requires_grad=True)
    ut = torch.tensor(u, dtype=torch.float32, device="cuda", requires_grad=True)
    loss = mjh.Rollout.apply(qv0, ut, w, H, K)
    loss.sum().backward()
    torch.cuda.synchronize()
    return (loss.detach().cpu().double().numpy(), qv0.grad.cpu().double().numpy(),
            ut.grad.cpu().double().numpy())


def test_rollout_loss_and_gradient_vs_finite_differences():
    nw_gpu, nw = 1024, 16
    m, qp, qv, u = _setup(nw_gpu)
    print(f"[gpu] adjoint rollout nw={nw_gpu} horizon={H} ckpt={K}", flush=True)
    L, gq, gu = _gpu_grads(m, qp, qv, u)
    o = oracle.Oracle(m)
    Lr = o.rollout_loss(qp[:nw], qv[:nw], u[:, :nw], mode=oracle.MODE_CONVERGED, nthreads=16)
    rel_loss = np.abs(L[:nw] - Lr) / np.abs(Lr)
    print(f"[adjoint] loss rel err max {rel_loss.max():.2e}", flush=True)
    assert rel_loss.max() < 1e-3
    # central differences of every input coordinate, all in one batched reference call
    h = 1e-6
    nd = m.nv + H * m.nu
    nb = nw * nd * 2
    QP = np.repeat(qp[:nw], nd * 2, axis=0)
    QV = np.repeat(qv[:nw], nd * 2, axis=0)
    U = np.repeat(u[:, :nw], nd * 2, axis=1)
    for w in range(nw):
        for d in range(nd):
            for sgn, off in ((1, 0), (-1, 1)):
                row = (w * nd + d) * 2 + off
                if d < m.nv:
                    QV[row, d] += sgn * h
                else:
                    t, a = divmod(d - m.nv, m.nu)
                    U[t, row, a] += sgn * h
    Lfd = o.rollout_loss(QP, QV, U, mode=oracle.MODE_CONVERGED, nthreads=16).reshape(nw, nd, 2)
    gfd = (Lfd[:, :, 0] - Lfd[:, :, 1]) / (2 * h)
    ggpu = np.concatenate([gq[:nw], gu[:, :nw].transpose(1, 0, 2).reshape(nw, -1)], axis=1)
    # worlds whose difference quotient crosses a contact switch disagree with the exact
    # directional derivative (dual numbers) of the same reference; they are reported
    rng = np.random.default_rng(3)
    dv = rng.normal(size=(nw, m.nv))
    du = rng.normal(size=(H, nw, m.nu))
    _, dL = o.rollout_jvp(qp[:nw], qv[:nw], u[:, :nw], dv, du, mode=oracle.MODE_CONVERGED,
                          nthreads=16)
    dirs = np.concatenate([dv, du.transpose(1, 0, 2).reshape(nw, -1)], axis=1)
    fd_dir = np.sum(gfd * dirs, axis=1)
    smooth = np.abs(fd_dir - dL) <= 1e-5 * np.maximum(1.0, np.abs(dL))
    err = np.linalg.norm(ggpu - gfd, axis=1) / np.linalg.norm(gfd, axis=1)
    cos = np.sum(ggpu * gfd, axis=1) / (np.linalg.norm(ggpu, axis=1) * np.linalg.norm(gfd, axis=1))
    print(f"[adjoint] grad normwise rel err vs FD (smooth worlds {smooth.sum()}/{nw}): "
          f"max {err[smooth].max():.2e} median {np.median(err[smooth]):.2e}; "
          f"cosine min {cos[smooth].min():.6f}; non-smooth worlds' err "
          f"{np.round(err[~smooth], 4).tolist()}", flush=True)
    assert smooth.sum() >= nw // 2
    assert err[smooth].max() < GRAD_TOL


def test_gradient_directional_vs_dual_numbers():
    nw = 64
    m, qp, qv, u = _setup(nw, seed=1)
    L, gq, gu = _gpu_grads(m, qp, qv, u)
    o = oracle.Oracle(m)
    rng = np.random.default_rng(5)
    dv = rng.normal(size=(nw, m.nv))
    du = rng.normal(size=(H, nw, m.nu))
    Lr, dL = o.rollout_jvp(qp, qv, u, dv, du, mode=oracle.MODE_CONVERGED, nthreads=16)
    rel, smooth = directional_check(o, qp, qv, u, gq, gu, dv, du, dL)
    print(f"[adjoint] <grad, d> vs dual JVP, error / (|grad| |d|): max {rel[smooth].max():.2e} "
          f"median {np.median(rel[smooth]):.2e} over {smooth.sum()}/{nw} smooth worlds; "
          f"non-smooth worlds' err {np.round(rel[~smooth], 5).tolist()}", flush=True)
    assert smooth.sum() >= 0.9 * nw
    assert rel[smooth].max() < GRAD_TOL


def test_rollout_rejects_unsupported_contacts():
    from paper_2502_08844_amd import mjh
    ctx = mjh.Context(0)
    m = robots.hand()  # capsule-box pairs: contact geometry not differentiated
    w = mjh.World(ctx, m, 2)
    u = torch.zeros(4, 2, m.nu, device="cuda")
    loss = torch.zeros(2, device="cuda")
    with pytest.raises(mjh.MjhError):
        w.batch.rollout_fwd(4, 2, u, 2, 0.3, 1e-3, loss)


def test_backward_of_a_replaced_rollout_is_refused():
    """Two forward rollouts of one world share its tapes: the first one's backward is
    refused (MJH_ESTATE), the second one's gradient equals a fresh single rollout's."""
    from paper_2502_08844_amd import mjh
    nw = 32
    m, qp, qv, u = _setup(nw, seed=2)
    ctx = mjh.Context(0)
    w = mjh.World(ctx, m, nw, qpos=qp)
    qv0 = torch.tensor(qv, dtype=torch.float32, device="cuda", requires_grad=True)
    ut = torch.tensor(u, dtype=torch.float32, device="cuda", requires_grad=True)
    loss1 = mjh.Rollout.apply(qv0, ut, w, H, K)
    w.qpos.copy_(torch.tensor(qp, dtype=torch.float32, device="cuda"))
    w.qacc_ws.zero_()
    loss2 = mjh.Rollout.apply(qv0, ut, w, H, K)
    with pytest.raises(mjh.MjhError) as e:
        loss1.sum().backward(retain_graph=True)
    assert e.value.code == mjh.ESTATE
    qv0.grad = None
    ut.grad = None
    loss2.sum().backward()
    torch.cuda.synchronize()
    L, gq, gu = _gpu_grads(m, qp, qv, u)
    assert np.array_equal(loss2.detach().cpu().double().numpy(), L)
    assert np.array_equal(qv0.grad.cpu().double().numpy(), gq)
    assert np.array_equal(ut.grad.cpu().double().numpy(), gu)
