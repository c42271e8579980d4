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
    fs = np.tile(np.r_[[0.05, 0.0, 0.3, 0.1], [0, 1, 1, 0], 1.0], (nw, 1))
    obs, rew, done, (q, v, ws, nprev, nfs), term = env.env_step(
        o, m, qp, qv, np.zeros((nw, m.nv)), prev, act, cmd, reset_q, reset_v, nsub=5,
        feet_state=fs)
    assert done.tolist() == [False, True, False, False]
    np.testing.assert_array_equal(q[1], reset_q[1])
    np.testing.assert_array_equal(v[1], reset_v[1])
    assert np.all(ws[1] == 0) and np.all(nprev[1] == 0)
    np.testing.assert_array_equal(nprev[0], act[0])
    assert rew[1] == 0.0
    # the terminal observation holds the previous action; the inverted world's
    # observation is its reset state's, with a zero previous action
    np.testing.assert_array_equal(term[:, 33:45], prev)
    np.testing.assert_array_equal(obs[[0, 2, 3]], term[[0, 2, 3]])
    np.testing.assert_array_equal(obs[1], env.observe(m, reset_q[1], reset_v[1], np.zeros(m.nu),
                                                      cmd[1]))
    assert not np.array_equal(obs[1], term[1])
    np.testing.assert_array_equal(obs[:, 45:48], cmd)
    np.testing.assert_array_equal(nfs[1], env.feet_state0(m))
    # the gait clock of the others advanced by 2 pi 2 Hz 0.02 s
    np.testing.assert_allclose(nfs[[0, 2, 3], 8], 1.0 + 2 * np.pi * 2.0 * 0.02, rtol=1e-15)


# ------------------------------------------------------------------ domain randomisation
def _record(m, fric=1.0, payload=0.0, com=(0, 0, 0), kp=1.0, kd=1.0, calib=None, arm=None):
    rec = env.dr_identity(m)
    rec[0], rec[1], rec[2:5], rec[5], rec[6] = fric, payload, com, kp, kd
    if calib is not None:
        rec[8:8 + m.nu] = calib
    if arm is not None:
        rec[8 + m.nu:8 + 2 * m.nu] = arm
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
    np.testing.assert_array_equal(got[3][4], ref[3][4])
    np.testing.assert_array_equal(got[4], ref[4] + noise)


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


def test_link_com_shift_closed_form():
    """Shifting one link's centre of mass by delta, at qpos0 (legs straight down, every
    frame aligned with the world's): the gravity bias changes by the moment of
    m_link delta x g on every dof the link hangs from (the root's rotation, and each
    hinge about its own axis), and nowhere else."""
    m = robots.quadruped()
    o0 = Oracle(m)
    q, v = m.qpos0.copy(), np.zeros(m.nv)
    f0 = o0.forward(q, v)
    s = np.sign(f0["bias"][2])
    gz = np.array([0.0, 0.0, 9.81])
    # leg 0: hip body 2 (abduction about x, dof 6), thigh 3 (pitch about y, dof 7),
    # shin 4 (knee about y, dof 8); the dofs a body hangs from
    hang = {2: [6], 3: [6, 7], 4: [6, 7, 8]}
    axes = {6: 0, 7: 1, 8: 1}
    for b, delta in ((4, np.array([0.01, -0.02, 0.03])), (2, np.array([-0.004, 0.03, 0.0])),
                     (3, np.array([0.0, 0.0, -0.05]))):
        rec = env.dr_identity(m)
        off = env.DR_HEAD + 2 * m.nu + 3 * (b - 2)
        rec[off:off + 3] = delta
        fw = env.randomized_oracle(o0, m, rec).forward(q, v)
        mom = s * np.cross(delta, m.bodies[b].mass * gz)
        expect = np.zeros(m.nv)
        expect[3:6] = mom
        for d in hang[b]:
            expect[d] = mom[axes[d]]
        np.testing.assert_allclose(fw["bias"] - f0["bias"], expect, atol=1e-12)
        np.testing.assert_allclose(np.diag(fw["M"])[:3], np.diag(f0["M"])[:3], rtol=1e-14)


# ------------------------------------------------------------------ feet terms
def _pose(m, z0=robots.QUAD_STAND_Z, yaw=0.0, th1=np.pi / 4, th2=-np.pi / 2, xy=(0.3, -0.2)):
    q = m.qpos0.copy()
    q[0:3] = [xy[0], xy[1], z0]
    q[3:7] = robots.axis_angle_quat((0, 0, 1), yaw)
    q[7:] = np.tile([0.0, th1, th2], 4)
    return q


def test_feet_heights_closed_form():
    """Foot k's centre sits at the torso's origin plus R_z(yaw) (0.15 sx - 0.2 sin th1 -
    0.2 sin(th1 + th2), 0.25 sy, -0.2 cos th1 - 0.2 cos(th1 + th2)) (leg geometry, thigh
    and knee about y); its lowest point is the radius 0.025 below.  In the standing pose
    every foot touches z = 0."""
    m = robots.quadruped()
    o = Oracle(m)
    pz, _ = env.feet_kinematics(m, o, _pose(m), np.zeros(m.nv))
    np.testing.assert_allclose(pz, 0.0, atol=1e-15)
    for yaw, th1, th2, z0 in ((0.4, 0.3, -1.1, 0.5), (-2.0, 0.9, -0.2, 0.41)):
        pz, _ = env.feet_kinematics(m, o, _pose(m, z0, yaw, th1, th2), np.zeros(m.nv))
        np.testing.assert_allclose(
            pz, z0 - 0.2 * np.cos(th1) - 0.2 * np.cos(th1 + th2) - 0.025, atol=1e-14)


def _quat_mul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def _advance(q, v, h):
    """The configuration after time h at constant velocity: the free joint's position
    moves with its world linear velocity, its orientation turns by the body-frame angular
    velocity (q <- q exp(w h / 2)), the hinges move linearly."""
    q = q.copy()
    q[0:3] += h * v[0:3]
    w = v[3:6]
    a = np.linalg.norm(w) * h  # signed with h
    dq = np.r_[np.cos(a / 2), np.sin(a / 2) * w / np.linalg.norm(w)] if a != 0 else np.r_[1, 0, 0, 0]
    q[3:7] = _quat_mul(q[3:7], dq)
    q[7:] += h * v[6:]
    return q


def _foot_centres(m, o, q):
    f = o.forward(q, np.zeros(m.nv))
    return np.array([f["xpos"][b] + f["xmat"][b] @ np.asarray(m.geoms[g].pos)
                     for g, b, _ in env.feet(m)])


def test_feet_velocity_is_the_derivative_of_their_position():
    """Horizontal foot speed against a central difference of the feet's positions
    along the motion (h = 1e-5: error O(h^2))."""
    m = robots.quadruped()
    o = Oracle(m)
    rng = np.random.default_rng(3)
    for _ in range(3):
        q = _pose(m, 0.45, rng.uniform(-3, 3), 0.7, -1.2)
        q[3:7] = _quat_mul(q[3:7], robots.axis_angle_quat(rng.normal(size=3), 0.4))
        v = rng.normal(size=m.nv)
        _, vxy = env.feet_kinematics(m, o, q, v)
        h = 1e-5
        d = (_foot_centres(m, o, _advance(q, v, h)) - _foot_centres(m, o, _advance(q, v, -h))) / (2 * h)
        np.testing.assert_allclose(vxy, np.hypot(d[:, 0], d[:, 1]), rtol=1e-7, atol=1e-9)


def test_airtime_is_paid_on_landing_and_clipped():
    """Foot 0 leaves the ground for k env steps of dt = 0.02 s and lands: on landing it
    earns clip((k + 1) dt - 0.1, 0, 0.4), nothing before and nothing for a foot that
    stayed down; its timer restarts."""
    m = robots.quadruped()
    o = Oracle(m)
    q, v = _pose(m), np.zeros(m.nv)
    dt = 0.02
    for k, expect in ((3, 0.0), (10, 0.12), (30, 0.4), (0, 0.0)):
        st = env.feet_state0(m)
        st[2 * 4] = 0.0
        for step in range(k):
            t, st = env.feet_terms(m, o, q, v, {1, 2, 3}, st, np.zeros(3), dt)
            assert t["air"] == 0.0
            assert st[0] == pytest.approx((step + 1) * dt, rel=1e-15) and st[4] == 0.0
        t, st = env.feet_terms(m, o, q, v, {0, 1, 2, 3}, st, np.zeros(3), dt)
        assert t["air"] == pytest.approx(expect, abs=1e-15)
        np.testing.assert_array_equal(st[:8], [0, 0, 0, 0, 1, 1, 1, 1])


def test_phase_term_closed_form():
    """Feet on the ground (p_z = 0) with the gait clock at pi/2 after its advance: feet
    0 and 3 should be at the swing height 0.08, feet 1 and 2 (half a cycle later) on the
    ground: 2 exp(-0.08^2 / 0.01) + 2.  A quarter cycle later (clock at pi) all four
    reference heights are 0: 4."""
    m = robots.quadruped()
    o = Oracle(m)
    q, v = _pose(m), np.zeros(m.nv)
    dt = 0.02
    st = env.feet_state0(m)
    st[8] = np.pi / 2 - 2 * np.pi * 2.0 * dt
    t, st = env.feet_terms(m, o, q, v, {0, 1, 2, 3}, st, np.zeros(3), dt)
    assert t["phase"] == pytest.approx(2 * np.exp(-0.0064 / 0.01) + 2, rel=1e-12)
    assert st[8] == pytest.approx(np.pi / 2, rel=1e-15)
    st[8] = np.pi - 2 * np.pi * 2.0 * dt
    t, st = env.feet_terms(m, o, q, v, {0, 1, 2, 3}, st, np.zeros(3), dt)
    assert t["phase"] == pytest.approx(4.0, rel=1e-12)
    assert abs(st[8]) == pytest.approx(np.pi, rel=1e-15)  # wrapped to (-pi, pi]


def test_clearance_slip_and_stand_still_closed_form():
    """The robot lifted by h with its torso translating at (0.3, 0.4, 0) m/s: every foot
    is h above the ground moving at 0.5 m/s, so the clearance term is
    -2 * 4 (h - 0.075)^2 0.5^0.5 and, with feet 0 and 2 in contact, the slip term
    -0.1 * 2 * 0.25; the stand-still term is -0.5 |cmd_xy|."""
    m = robots.quadruped()
    o = Oracle(m)
    for h in (0.0, 0.03, 0.2):
        q = _pose(m, robots.QUAD_STAND_Z + h, yaw=0.7)
        v = np.zeros(m.nv)
        v[0:2] = [0.3, 0.4]
        t, _ = env.feet_terms(m, o, q, v, {0, 2}, env.feet_state0(m), np.array([0.3, -0.4, 0.7]),
                              0.02)
        assert t["clear"] == pytest.approx(-2.0 * 4 * (h - 0.075) ** 2 * np.sqrt(0.5), rel=1e-12)
        assert t["slip"] == pytest.approx(-0.1 * 2 * 0.25, rel=1e-12)
        assert t["stand"] == pytest.approx(-0.5 * 0.5, rel=1e-15)


def test_contact_flags_come_from_the_last_physics_step():
    """A standing robot has all four feet down after an env step; one lifted 0.1 m has
    none, and its feet's timers run."""
    m = robots.quadruped()
    o = Oracle(m)
    q = np.stack([_pose(m, robots.QUAD_STAND_Z - 1e-3), _pose(m, robots.QUAD_STAND_Z + 0.1)])
    v = np.zeros((2, m.nv))
    z = np.zeros((2, m.nu))
    out = env.env_step(o, m, q, v, np.zeros((2, m.nv)), z, z, np.zeros((2, 3)), q, v, nsub=5)
    nfs = out[3][4]
    np.testing.assert_array_equal(nfs[0, :8], [0, 0, 0, 0, 1, 1, 1, 1])
    np.testing.assert_allclose(nfs[1, :4], 0.02, rtol=1e-15)
    np.testing.assert_array_equal(nfs[1, 4:8], 0)
