"""Pins of the joystick environment reference (observation, reward, termination, reset).
No GPU.  Each check builds a state whose outputs are known in closed form."""
import numpy as np
import pytest

from oracle import Oracle
from oracle import env
from paper_2502_08844_amd.synth import inputs, robots


def _standing(m):
    q = robots.quadruped_standing_qpos(m)
    return q, np.zeros(m.nv)


def test_standing_still_earns_the_tracking_maximum():
    m = robots.quadruped()
    q, v = _standing(m)
    a = np.zeros(m.nu)
    obs = env.observe(m, q, v, a, np.zeros(3))
    assert obs.shape == (48,)
    np.testing.assert_allclose(obs[:3], [0, 0, -1], atol=1e-15)
    assert np.abs(obs[3:]).max() == 0.0
    r, done = env.reward_done(m, q, v, a, a, np.zeros(3))
    assert r == pytest.approx(env.K_V + env.K_W + env.K_POSE, abs=1e-15) and not done


def test_tracking_terms_and_body_frame_velocity():
    m = robots.quadruped()
    q, v = _standing(m)
    yaw = robots.axis_angle_quat((0, 0, 1), np.pi / 2)
    q[3:7] = yaw
    v[0:3] = [1.0, 0.0, 0.0]  # world +x is the body's -y after a quarter turn
    v[5] = 0.3                # yaw rate (body frame)
    a = np.zeros(m.nu)
    obs = env.observe(m, q, v, a, np.array([0.0, -1.0, 0.3]))
    np.testing.assert_allclose(obs[3:6], [0, -1, 0], atol=1e-15)
    np.testing.assert_allclose(obs[6:9], [0, 0, 0.3], atol=1e-15)
    r, _ = env.reward_done(m, q, v, a, a, np.array([0.0, -1.0, 0.3]))
    # both commands tracked exactly, in the default pose; the yaw rate is a body-frame
    # angular velocity about z, which none of the penalties counts
    assert r == pytest.approx(1.5 + env.K_POSE, abs=1e-12)
    r2, _ = env.reward_done(m, q, v, a, a, np.array([0.5, -1.0, -0.2]))
    assert r2 == pytest.approx(np.exp(-0.25 / 0.25) + 0.5 * np.exp(-0.25 / 0.25) + env.K_POSE,
                               abs=1e-12)


def test_orientation_termination_and_clipping():
    m = robots.quadruped()
    q, v = _standing(m)
    a = np.zeros(m.nu)
    q[3:7] = robots.axis_angle_quat((1, 0, 0), np.pi / 2)  # on its side
    obs = env.observe(m, q, v, a, np.zeros(3))
    np.testing.assert_allclose(obs[:3], [0, -1, 0], atol=1e-15)
    r, done = env.reward_done(m, q, v, a, a, np.zeros(3))
    assert r == 0.0 and not done  # 1.5 + 0.5 - 5 |g_xy|^2 clipped at zero
    q[3:7] = robots.axis_angle_quat((1, 0, 0), 0.55 * np.pi)  # past the side: inverted
    assert env.reward_done(m, q, v, a, a, np.zeros(3))[1]


def test_penalty_terms_one_at_a_time():
    m = robots.quadruped()
    q, v = _standing(m)
    a0 = np.zeros(m.nu)
    base = env.K_V + env.K_W + env.K_POSE
    v2 = v.copy(); v2[2] = 0.2  # vertical velocity (world z = body z here)
    assert env.reward_done(m, q, v2, a0, a0, np.zeros(3))[0] == pytest.approx(
        base + env.K_LINZ * 0.04, abs=1e-12)
    v3 = v.copy(); v3[3:5] = [0.1, 0.2]
    assert env.reward_done(m, q, v3, a0, a0, np.zeros(3))[0] == pytest.approx(
        base + env.K_ANGXY * 0.05, abs=1e-12)
    a1 = np.zeros(m.nu); a1[0] = 0.1  # PD torque kp * 0.1 on one hinge, action rate 0.01
    kp = m.actuators[0].kp
    assert env.reward_done(m, q, v, a1, a0, np.zeros(3))[0] == pytest.approx(
        base + env.K_TAU * (kp * 0.1) ** 2 + env.K_RATE * 0.01, abs=1e-12)
    q4 = q.copy(); q4[7] += 0.2  # joint offset with the matching action: no torque
    a4 = np.zeros(m.nu); a4[0] = 0.2
    assert env.reward_done(m, q4, v, a4, a4, np.zeros(3))[0] == pytest.approx(
        base + env.K_Q * 0.04 + env.K_POSE * (np.exp(-0.04) - 1), abs=1e-12)
    # a joint velocity: PD damping torque -kd qdot, its square and the power |qdot tau|
    v5 = v.copy(); v5[6] = 0.5
    kd = m.actuators[0].kd
    assert env.reward_done(m, q, v5, a0, a0, np.zeros(3))[0] == pytest.approx(
        base + env.K_TAU * (kd * 0.5) ** 2 + env.K_ENERGY * (kd * 0.25), abs=1e-12)


def test_env_step_resets_inverted_worlds():
    m = robots.quadruped()
    o = Oracle(m)
    nw = 4
    qp, qv = inputs.initial_state("quadruped", m, nw, seed=2)
    qp[1, 3:7] = robots.axis_angle_quat((1, 0, 0), np.pi)  # world 1 starts upside down
    qp[1, 2] = 0.5
    reset_q, reset_v = inputs.initial_state("quadruped", m, nw, seed=9)
    prev = np.full((nw, m.nu), 0.3)
    act = inputs.controls("quadruped", m, nw, 1, seed=2)[0]
    cmd = np.tile([0.5, 0.0, 0.1], (nw, 1))
    obs, rew, done, (q, v, ws, nprev) = env.env_step(o, m, qp, qv, np.zeros((nw, m.nv)), prev,
                                                     act, cmd, reset_q, reset_v, nsub=5)
    assert done.tolist() == [False, True, False, False]
    np.testing.assert_array_equal(q[1], reset_q[1])
    np.testing.assert_array_equal(v[1], reset_v[1])
    assert np.all(ws[1] == 0) and np.all(nprev[1] == 0)
    np.testing.assert_array_equal(nprev[0], act[0])
    assert rew[1] == 0.0
    np.testing.assert_array_equal(obs[:, 33:45], prev)  # the previous action in the obs
    np.testing.assert_array_equal(obs[:, 45:48], cmd)


# ------------------------------------------------------------------ domain randomisation
def _record(m, fric=1.0, payload=0.0, com=(0, 0, 0), kp=1.0, kd=1.0, calib=None, arm=None):
    rec = env.dr_identity(m)
    rec[0], rec[1], rec[2:5], rec[5], rec[6] = fric, payload, com, kp, kd
    if calib is not None:
        rec[8:8 + m.nu] = calib
    if arm is not None:
        rec[8 + m.nu:] = arm
    return rec


def test_identity_record_changes_nothing():
    m = robots.quadruped()
    assert env.randomized_model(m, env.dr_identity(m)).to_blob() == m.to_blob()
    o = Oracle(m)
    nw = 3
    qp, qv = inputs.initial_state("quadruped", m, nw, seed=2)
    a = np.random.default_rng(1).uniform(-0.5, 0.5, size=(nw, m.nu))
    args = (qp, qv, np.zeros((nw, m.nv)), np.zeros((nw, m.nu)), a, np.zeros((nw, 3)), qp, qv, 3)
    ref = env.env_step(o, m, *args)
    dr = np.stack([env.dr_identity(m)] * nw)
    noise = np.random.default_rng(2).normal(size=(nw, 48))
    got = env.env_step(o, m, *args, dr=dr, noise=noise)
    np.testing.assert_array_equal(got[0], ref[0] + noise)
    np.testing.assert_array_equal(got[1], ref[1])
    np.testing.assert_array_equal(got[3][0], ref[3][0])


def test_payload_and_com_shift_closed_form():
    """At qpos0 (root frame = world frame): the translational mass block gains the
    payload, and the gravity bias on the root's rotational dofs gains the moment of the
    root body's shifted, heavier centre of mass about the root origin."""
    m = robots.quadruped()
    dm, dc = 1.5, np.array([0.02, -0.01, 0.005])
    o0 = Oracle(m)
    ow = env.randomized_oracle(o0, m, _record(m, payload=dm, com=dc))
    q, v = m.qpos0.copy(), np.zeros(m.nv)
    f0, fw = o0.forward(q, v), ow.forward(q, v)
    mtot = sum(b.mass for b in m.bodies)
    np.testing.assert_allclose(np.diag(f0["M"])[:3], mtot, rtol=1e-14)
    np.testing.assert_allclose(np.diag(fw["M"])[:3], mtot + dm, rtol=1e-14)
    s = np.sign(f0["bias"][2])  # the bias holds the force against gravity, up to sign
    assert f0["bias"][2] == pytest.approx(s * mtot * 9.81, rel=1e-12)
    mroot = m.bodies[m.joints[0].body].mass
    c0 = np.asarray(m.bodies[m.joints[0].body].ipos)
    gz = np.array([0.0, 0.0, 9.81])
    expect = s * (np.cross((mroot + dm) * (c0 + dc), gz) - np.cross(mroot * c0, gz))
    np.testing.assert_allclose(fw["bias"][:3] - f0["bias"][:3], s * dm * gz, atol=1e-12)
    np.testing.assert_allclose(fw["bias"][3:6] - f0["bias"][3:6], expect, atol=1e-12)
    np.testing.assert_allclose(fw["bias"][6:], f0["bias"][6:], atol=1e-12)


def test_armature_gains_and_calibration_closed_form():
    m = robots.quadruped()
    rng = np.random.default_rng(5)
    arm = rng.uniform(0.005, 0.02, m.nu)
    calib = rng.uniform(-0.05, 0.05, m.nu)
    skp, skd = 0.8, 1.3
    o0 = Oracle(m)
    ow = env.randomized_oracle(o0, m, _record(m, kp=skp, kd=skd, calib=calib, arm=arm))
    qp, qv = inputs.initial_state("quadruped", m, 1, seed=4)
    qv = rng.normal(size=(1, m.nv))
    u = rng.uniform(-0.5, 0.5, m.nu)
    f0, fw = o0.forward(qp[0], qv[0], ctrl=u), ow.forward(qp[0], qv[0], ctrl=u)
    np.testing.assert_allclose(fw["M"] - f0["M"], np.diag(np.r_[np.zeros(6), arm]), atol=1e-14)
    for k, a in enumerate(m.actuators):
        tau = skp * a.kp * (a.qdefault + u[k] - (qp[0, 7 + k] + calib[k])) \
            - skd * a.kd * qv[0, 6 + k]
        assert fw["act"][6 + k] == pytest.approx(tau, rel=1e-12, abs=1e-12)
    # the observation reports the encoder reading q + delta
    obs = env.observe(env.randomized_model(m, _record(m, calib=calib)), qp[0], qv[0],
                      np.zeros(m.nu), np.zeros(3))
    qdef = np.array([a.qdefault for a in m.actuators])
    np.testing.assert_allclose(obs[9:21], qp[0, 7:] + calib - qdef, atol=1e-15)
    # the regularisers keep the nominal inverse weights
    np.testing.assert_array_equal(ow.body_invweight(), o0.body_invweight())
    np.testing.assert_array_equal(ow.dof_invweight(), o0.dof_invweight())
    assert not np.allclose(Oracle(env.randomized_model(m, _record(m, arm=arm))).dof_invweight(),
                           o0.dof_invweight())


def test_friction_scale_on_an_incline():
    """Gravity tilted by atan(0.5): with mu = 1 a box sticks; with the coefficient
    scaled to f < 0.5 it slides, and the friction it feels, (g sin - a) / (g cos), is f
    (Coulomb along a pyramid edge) within 2 % (the soft contact's regulariser lets a
    sliding contact transmit slightly less than mu N)."""
    th = np.arctan(0.5)
    grav = (9.81 * np.sin(th), 0.0, -9.81 * np.cos(th))
    m = robots.free_body("box", mass=1.0, half=(0.1, 0.2, 0.05), plane=True, mu=1.0,
                         gravity=grav, timestep=0.002)
    q0 = m.qpos0.copy()
    q0[2] = 0.05
    for f in (1.0, 0.4, 0.3, 0.2):
        o = env.randomized_oracle(Oracle(m), m, _record(m, fric=f))
        r1 = o.step(q0[None].copy(), np.zeros((1, 6)), nstep=300, mode=1)
        r2 = o.step(r1["qpos"], r1["qvel"], r1["qacc_ws"], nstep=200, mode=1)
        acc = (r2["qvel"][0, 0] - r1["qvel"][0, 0]) / (200 * m.opt.timestep)
        if f == 1.0:
            assert abs(acc) < 1e-3
        else:
            mu_eff = (9.81 * np.sin(th) - acc) / (9.81 * np.cos(th))
            assert mu_eff == pytest.approx(f, rel=2e-2)


def test_nonfinite_state_terminates_with_zero_reward():
    m = robots.quadruped()
    q, v = _standing(m)
    v = v.copy()
    v[7] = np.nan
    r, done = env.reward_done(m, q, v, np.zeros(m.nu), np.zeros(m.nu), np.zeros(3))
    assert done and r == 0.0
