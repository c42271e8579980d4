"""Reference derivatives of the rollout loss: forward-mode dual numbers through the FP64
reference agree with central finite differences.  No GPU."""
import numpy as np
import pytest

from oracle import MODE_CONVERGED, MODE_FIXED, Oracle
from paper_2502_08844_amd.synth import inputs, robots


def _setup(nw=3, horizon=16, seed=0):
    m = robots.quadruped()
    o = Oracle(m)
    qp, qv = inputs.initial_state("quadruped", m, nw, seed=seed)
    rng = np.random.default_rng(seed)
    u = inputs.f32(rng.uniform(-0.5, 0.5, size=(horizon, nw, m.nu)))
    qv = qv + inputs.f32(rng.normal(scale=0.1, size=qv.shape))
    return m, o, qp, qv, u


@pytest.mark.parametrize("mode", [MODE_FIXED, MODE_CONVERGED])
def test_dual_jvp_matches_central_differences(mode):
    m, o, qp, qv, u = _setup()
    rng = np.random.default_rng(1)
    nw = qp.shape[0]
    agree = 0
    for trial in range(3):
        dv = rng.normal(size=qv.shape)
        du = rng.normal(size=u.shape)
        L, dL = o.rollout_jvp(qp, qv, u, dv, du, mode=mode)
        h = 1e-6
        Lp = o.rollout_loss(qp, qv + h * dv, u + h * du, mode=mode)
        Lm = o.rollout_loss(qp, qv - h * dv, u - h * du, mode=mode)
        fd = (Lp - Lm) / (2 * h)
        assert np.allclose(L, o.rollout_loss(qp, qv, u, mode=mode), rtol=0, atol=1e-12)
        rel = np.abs(fd - dL) / (1e-3 + np.abs(dL))
        agree += int(np.sum(rel < 1e-5))
    # an active-set switch inside +-h can spoil a world's difference quotient; the rest
    # agree closely
    assert agree >= 3 * nw - 1


def test_loss_definition():
    m, o, qp, qv, u = _setup(nw=2, horizon=5)
    L = o.rollout_loss(qp, qv, u, ztarget=0.3, wctrl=1e-3)
    # recompute the sum from a recorded trajectory
    for w in range(2):
        tq, _, _ = o.trajectory(qp[w], qv[w], 5, ctrl=u[:, w, :])
        ref = np.sum((tq[:, 2] - 0.3) ** 2) + 1e-3 * np.sum(u[:, w, :] ** 2)
        assert L[w] == pytest.approx(ref, rel=1e-12)


def test_step_jvp_matches_central_differences():
    m, o, qp, qv, u = _setup(nw=1)
    rng = np.random.default_rng(4)
    ws = np.zeros(m.nv)
    dq = np.zeros(m.nq)
    dq[7:] = rng.normal(size=12)
    dq[:3] = rng.normal(size=3)
    dv = rng.normal(size=m.nv)
    du = rng.normal(size=m.nu)
    q1, v1, dq1, dv1 = o.step_jvp(qp[0], qv[0], ws, u[0, 0], dq, dv, du, mode=MODE_CONVERGED)
    h = 1e-7

    def run(s):
        r = o.step(qp[0] + s * dq, qv[0] + s * dv, ws[None], (u[0, 0] + s * du)[None, None],
                   mode=MODE_CONVERGED)
        return r["qpos"][0], r["qvel"][0]
    qp_, vp_ = run(h)
    qm_, vm_ = run(-h)
    assert np.allclose((qp_ - qm_) / (2 * h), dq1, rtol=1e-5, atol=1e-6)
    assert np.allclose((vp_ - vm_) / (2 * h), dv1, rtol=1e-5, atol=1e-5)
