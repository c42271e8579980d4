"""GPU parity of the implicit integrators against the FP64 reference: integrator 1
(joint damping and PD velocity gains taken at the end-of-step velocity) and integrator 2
(also the PD position gains at the end-of-step position).

The compared quantity is the integrator's acceleration a_int = (qvel' - qvel) / h of
one step from the same float32 state (the reported qacc is the solve's a*, covered by
the other parity tests), per world ||a_int,gpu - a_int,ref||_inf / max(||a_int,ref||_inf,
9.81), on worlds not at a contact or activation switch (those are counted and reported).

Tolerance 1e-4, the qacc tolerance, in every world not at a switch, with a median
below 1e-5: a_int = (M + h B)^-1 (qfrc_smooth + J^T f) takes the row forces f of the
fixed-iteration solve.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2502_08844_amd.synth import inputs, robots
from tests.gpu_util import G, compare_step, gpu_ctx, run_gpu, workload

pytestmark = pytest.mark.gpu

TOL = 1e-4
TOL_MEDIAN = 1e-5


@pytest.fixture(scope="module")
def lib():
    return gpu_ctx()


def _a_int_errors(ctx, mjh, m, qp, qv, ws, u1, team=None, block=None):
    """Errors of a_int per world, and the flags of worlds at a switch (as in the other
    parity tests: reported, not gated)."""
    g = run_gpu(ctx, mjh, m, qp, qv, ws, u1, 1, team, block, contacts=True)
    o = oracle.Oracle(m)
    cmp = compare_step(m, o, (qp, qv, ws), u1, g)
    r = o.step(qp.copy(), qv.copy(), ws.copy(), u1, nstep=1, mode=oracle.MODE_FIXED, nthreads=8)
    h = m.opt.timestep
    a_gpu = (g["qvel"] - qv) / h
    a_ref = (r["qvel"] - qv) / h
    err = np.abs(a_gpu - a_ref).max(1) / np.maximum(np.abs(a_ref).max(1), G)
    return err, cmp["flag"], g


@pytest.mark.parametrize("kind,team,block", [("quadruped_implicit", 32, 128),
                                             ("quadruped_implicit", 64, 64),
                                             ("quadruped_implicit", 16, 64),
                                             ("quadruped_implicit_pd", 32, 128),
                                             ("quadruped_implicit_pd", 16, 64)])
def test_quadruped_implicit_velocity_update(lib, kind, team, block):
    mjh, ctx = lib
    m, qp, qv, u = workload(kind, 203, 51, seed=4)
    # advance on the GPU to a contact-rich state, then compare one step
    r = run_gpu(ctx, mjh, m, qp, qv, None, u[:50], 50, team, block, contacts=False)
    err, flag, g = _a_int_errors(ctx, mjh, m, r["qpos"], r["qvel"], r["qacc"], u[50:51], team,
                                 block)
    print(f"[parity] {kind}-T{team}: a_int rel err max {err[~flag].max():.2e} "
          f"median {np.median(err):.2e}; near-switch states {flag.sum()}/{len(flag)}"
          + (f" (their err max {err[flag].max():.2e})" if flag.any() else ""), flush=True)
    assert np.all(g["status"] & 1 == 0)
    assert err[~flag].max() <= TOL
    assert np.median(err) <= TOL_MEDIAN
    assert flag.sum() <= max(1, 0.02 * len(flag))


def test_stiff_damping_decays_on_gpu(lib):
    """h b / m = 5: the explicit update would grow 4x per step; implicitly the velocity
    shrinks by 1/6 per step."""
    mjh, ctx = lib
    m = robots.slider(mass=1.0, range=None, damping=500.0, gravity=(0, 0, 0), timestep=0.01,
                      integrator=1)
    qv = np.full((64, 1), 1.0)
    r = run_gpu(ctx, mjh, m, np.zeros((64, 1)), qv, None, None, 10, contacts=False)
    np.testing.assert_allclose(r["qvel"][:, 0], (1 / 6) ** 10, rtol=1e-5)


def test_stiff_pd_decays_on_gpu(lib):
    """Integrator 2 on a PD slider with h^2 kp / m = 9: backward Euler of the spring,
    x_{n+1} = (I - h A)^-1 x_n, where semi-implicit Euler would grow sevenfold a step."""
    mjh, ctx = lib
    from paper_2502_08844_amd.synth.model import ACT_PD, Actuator
    mass, kp, h = 1.0, 90000.0, 0.01
    m = robots.slider(mass=mass, range=None, gravity=(0, 0, 0), timestep=h, integrator=2)
    m.actuators.append(Actuator(type=ACT_PD, joint=0, kp=kp, kd=0.0, ctrlrange=(-1, 1)))
    r = run_gpu(ctx, mjh, m, np.full((64, 1), 0.1), np.zeros((64, 1)), None,
                np.zeros((10, 64, 1)), 10, contacts=False)
    A = np.array([[0.0, 1.0], [-kp / mass, 0.0]])
    x = np.array([0.1, 0.0])
    for _ in range(10):
        x = np.linalg.solve(np.eye(2) - h * A, x)
    np.testing.assert_allclose(r["qpos"][:, 0], x[0], rtol=1e-4, atol=1e-9)
    np.testing.assert_allclose(r["qvel"][:, 0], x[1], rtol=1e-4, atol=1e-7)


def test_rollout_rejects_implicit_beyond_one_dof_per_lane(lib):
    """The implicit integrators' reverse sweep takes the dense factor (nv <= team)."""
    mjh, ctx = lib
    m = robots.quadruped_implicit()  # nv 18
    w = mjh.World(ctx, m, 2)
    w.batch.set_launch(0, 16, 64)
    u = torch.zeros(4, 2, m.nu, device="cuda")
    loss = torch.zeros(2, device="cuda")
    with pytest.raises(mjh.MjhError):
        w.batch.rollout_fwd(4, 2, u, 2, 0.3, 1e-3, loss)
