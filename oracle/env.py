"""Reference of the joystick locomotion environment step (TEST INFRASTRUCTURE ONLY, like
the rest of this package): observation, reward terms, termination and reset around
the FP64 physics step, written out plainly in numpy.

Task (the paper's locomotion appendix: observation list, absolute joint-position
actions through the PD mapping of eq. pd_mapping, the reward table, termination when
the robot inverts):
* one env step = ``nsub`` physics steps with the action held as the PD targets'
  offsets (the model's position actuators: q_des = q_default + gear * a);
* observation, from the state after those steps (body frame = the root body's):
  gravity direction in the body frame (3), base linear velocity in the body frame (3),
  base angular velocity (3), joint positions minus their defaults (n), joint
  velocities (n), the previous action (n), the command (3): 12 + 3 n values;
* reward, the clipped-at-zero weighted sum of these terms of the reward table:
  linear-velocity tracking  1.0 * exp(-|cmd_xy - v_xy|^2 / 0.25)
  yaw-rate tracking         0.5 * exp(-(cmd_wz - w_z)^2 / 0.25)
  linear velocity in z     -2.0 * v_z^2
  angular velocity in xy   -0.05 * |w_xy|^2
  orientation              -5.0 * |g_xy|^2          (g: gravity in the body frame)
  joint torque             -2e-4 * |tau|^2          (PD torques at the new state)
  joint position           -0.1 * |q - q_default|^2
  action rate              -0.01 * |a_t - a_{t-1}|^2
  energy                   -1e-3 * sum_k |qdot_k tau_k|
  pose                      0.5 * exp(-|q - q_default|^2)
  termination              -1.0 * done
  feet airtime              1.0 * sum_f clip((T_air,f - 0.1) C_first,f, 0, 0.5 - 0.1)
  feet clearance           -2.0 * sum_f (p_f,z - 0.075)^2 |v_f,xy|^0.5
  feet phase                1.0 * sum_f exp(-(p_f,z - r_z(phi_f))^2 / 0.01)
  feet slip                -0.1 * sum_f C_f |v_f,xy|^2
  stand still              -0.5 * |cmd_xy|          (as printed)
  A foot is the moving geom of a contact pair (every pair is a foot against the ground):
  C_f = 1 when the pair had a contact in the env step's last physics step; p_f,z is the
  height of the foot's lowest point (centre z minus radius) above z = 0 and v_f,xy its
  centre's horizontal velocity, at the new state.  T_air,f is the time since the foot
  last left the ground, counted in env steps of nsub dt and paid when it lands
  (C_first,f = C_f and not C_f at the previous env step), then zeroed.  A gait clock
  phi_0 advances 2 pi 2 Hz per second of env time; foot f is at phi_f = phi_0 +
  pi ((f xor floor(f / 2)) mod 2) (a trot for legs ordered front-left, front-right,
  rear-left, rear-right), wrapped to (-pi, pi], and its reference height is
  r_z(phi) = 0.08 max(0, sin phi).
* termination: the root body's z axis points downwards (the robot has inverted), or
  the state is no longer finite (then the reward is 0);
* reset: a terminated world restarts from its reset state (given by the caller) with a
  zero warm start, a zero previous action and fresh feet state (timers 0, feet in
  contact, gait phase 0); its observation is the reset state's (with the zero previous
  action), and the terminal observation, of the state it ended in, is returned beside;
  its reward and done are those of the state it ended in.
* feet state, per world: [T_air (nf), C_f of the previous env step (nf), phi_0].
* the model's root is a free joint and actuator k drives dof 6 + k.

Domain randomisation (the paper's locomotion appendix: sensor noise; link centre of
mass, reflected inertia and joint calibration offsets; ground friction and payload
mass; the PD gains), one record of 8 + 2 n + 3 (nbody - 2) values per world:
  [0] friction scale: every contact pair's coefficient times this;
  [1] payload mass added to the root body at its centre of mass (its rotational
      inertia about the centre of mass is unchanged);
  [2:5] shift of the root body's centre of mass, in the root body's frame;
  [8+2n+3(b-2) : +3] shift of body b's centre of mass, in its frame (b >= 2, every
      link after the root);
  [5], [6] scales of the position actuators' kp and kd;  [7] unused;
  [8:8+n] joint calibration offsets: the encoder reads q + delta, so the PD law and
      the observation see q + delta (equivalently q_default - delta);
  [8+n:8+2n] the reflected inertia (armature) of dof 6 + k, replacing the model's.
The rows' regularisers keep the nominal model's inverse weights (computed once at
qpos0), as a compiled model's constants are not recomputed when its parameters are
varied.  Sensor noise is added to the observation as given (one value per entry).
"""
from __future__ import annotations

import copy

import numpy as np

K_V, SIG_V = 1.0, 0.25
K_W, SIG_W = 0.5, 0.25
K_LINZ, K_ANGXY, K_ORI, K_TAU, K_Q, K_RATE, K_TERM = -2.0, -0.05, -5.0, -2e-4, -0.1, -0.01, -1.0
K_ENERGY, K_POSE = -1e-3, 0.5
K_AIR, T_MIN, T_MAX = 1.0, 0.1, 0.5
K_CLEAR, P_DES = -2.0, 0.075
K_PHASE, SIG_PHASE, GAIT_HZ, H_SWING = 1.0, 0.01, 2.0, 0.08
K_SLIP, K_STAND = -0.1, -0.5


def quat_mat(q):
    """Rotation matrix of the unit quaternion (w, x, y, z)."""
    w, x, y, z = np.asarray(q, dtype=np.float64) / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def pd_torques(m, qpos, qvel, action):
    """tau_k = kp (q_default + gear clamp(a) - q) - kd qdot for each position actuator."""
    qadr, dadr = m.jnt_qposadr(), m.jnt_dofadr()
    tau = np.zeros(m.nu)
    for k, a in enumerate(m.actuators):
        u = min(max(action[k], a.ctrlrange[0]), a.ctrlrange[1])
        q, qd = qpos[qadr[a.joint]], qvel[dadr[a.joint]]
        tau[k] = a.kp * (a.qdefault + a.gear * u - q) - a.kd * qd
    return tau


def observe(m, qpos, qvel, prev_action, cmd, noise=None):
    R = quat_mat(qpos[3:7])
    g = R.T @ np.array([0.0, 0.0, -1.0])
    v = R.T @ qvel[0:3]  # free-joint qvel: world linear velocity of the body origin
    w = qvel[3:6]        # and the body-frame angular velocity
    qdef = np.array([a.qdefault for a in m.actuators])
    obs = np.concatenate([g, v, w, qpos[7:] - qdef, qvel[6:], prev_action, cmd])
    return obs if noise is None else obs + noise


def feet(m):
    """(geom, body, radius) of each contact pair's moving geom: the feet."""
    out = []
    for g1, g2, *_ in m.pairs:
        g = g2 if m.geoms[g1].body == 0 else g1
        assert (m.geoms[g1].body == 0) != (m.geoms[g2].body == 0), "a foot against the ground"
        out.append((g, m.geoms[g].body, m.geoms[g].size[0]))
    return out


def feet_state0(m):
    """The feet state of a fresh world: timers 0, every foot in contact, phase 0."""
    nf = len(m.pairs)
    return np.concatenate([np.zeros(nf), np.ones(nf), [0.0]])


def wrap(phi):
    return phi - 2 * np.pi * np.round(phi / (2 * np.pi))


def feet_kinematics(m, o, qpos, qvel):
    """Height of each foot's lowest point above z = 0 and its centre's horizontal speed."""
    f = o.forward(qpos, qvel)
    pz, vxy = [], []
    for g, b, rad in feet(m):
        p = f["xpos"][b] + f["xmat"][b] @ np.asarray(m.geoms[g].pos, dtype=np.float64)
        w, vo = f["cvel"][b][:3], f["cvel"][b][3:]   # velocity of the point at the origin
        vel = vo + np.cross(w, p)
        pz.append(p[2] - rad)
        vxy.append(np.hypot(vel[0], vel[1]))
    return np.array(pz), np.array(vxy)


def foot_phase_offset(k):
    """Gait phase offset of foot k: feet 0 and 3 in phase, 1 and 2 half a cycle apart."""
    return np.pi * ((k ^ (k // 2)) & 1)


def feet_terms(m, o, qpos, qvel, contact_pairs, state, cmd, dt_env):
    """The weighted feet terms and the stand-still term at the new state (qpos, qvel),
    given the set of pairs in contact in the last physics step and the world's feet
    state; returns {term: value} and the next feet state."""
    nf = len(m.pairs)
    pz, vxy = feet_kinematics(m, o, qpos, qvel)
    air, cprev, phi0 = state[:nf].copy(), state[nf:2 * nf], state[2 * nf]
    phi0 = wrap(phi0 + 2 * np.pi * GAIT_HZ * dt_env)
    c = np.array([1.0 if k in contact_pairs else 0.0 for k in range(nf)])
    t_air = air + dt_env
    first = (c > 0) & (cprev == 0)
    r_air = K_AIR * np.sum(np.where(first, np.clip(t_air - T_MIN, 0.0, T_MAX - T_MIN), 0.0))
    air = np.where(c > 0, 0.0, t_air)
    phi = wrap(phi0 + foot_phase_offset(np.arange(nf)))
    rz = H_SWING * np.maximum(0.0, np.sin(phi))
    terms = dict(air=r_air,
                 clear=K_CLEAR * np.sum((pz - P_DES) ** 2 * np.sqrt(vxy)),
                 phase=K_PHASE * np.sum(np.exp(-(pz - rz) ** 2 / SIG_PHASE)),
                 slip=K_SLIP * np.sum(c * vxy ** 2),
                 stand=K_STAND * np.linalg.norm(cmd[:2]))
    return terms, np.concatenate([air, c, [phi0]])


def reward_done(m, qpos, qvel, action, prev_action, cmd, extra=0.0):
    """Reward (the table's other terms plus `extra`, clipped at zero) and done."""
    if not (np.all(np.isfinite(qpos)) and np.all(np.isfinite(qvel))):
        return 0.0, True
    R = quat_mat(qpos[3:7])
    done = R[2, 2] < 0.0
    g = R.T @ np.array([0.0, 0.0, -1.0])
    v = R.T @ qvel[0:3]
    w = qvel[3:6]
    qdef = np.array([a.qdefault for a in m.actuators])
    tau = pd_torques(m, qpos, qvel, action)
    r = (K_V * np.exp(-np.sum((cmd[:2] - v[:2]) ** 2) / SIG_V)
         + K_W * np.exp(-(cmd[2] - w[2]) ** 2 / SIG_W)
         + K_LINZ * v[2] ** 2 + K_ANGXY * np.sum(w[:2] ** 2) + K_ORI * np.sum(g[:2] ** 2)
         + K_TAU * np.sum(tau ** 2) + K_Q * np.sum((qpos[7:] - qdef) ** 2)
         + K_RATE * np.sum((action - prev_action) ** 2)
         + K_ENERGY * np.sum(np.abs(qvel[6:] * tau))
         + K_POSE * np.exp(-np.sum((qpos[7:] - qdef) ** 2)) + K_TERM * float(done))
    return max(r + extra, 0.0), bool(done)


def env_step(o, m, qpos, qvel, qacc_ws, prev_action, action, cmd, reset_qpos, reset_qvel,
             nsub, mode=0, dr=None, noise=None, feet_state=None):
    """One env step of every world (arrays [nworld, ...]); returns the outputs and the
    next (qpos, qvel, qacc_ws, prev_action, feet_state) after resets, and the terminal
    observations.  dr: per-world randomisation records [nworld, 8 + 2 nu + 3 (nbody - 2)]
    or None; noise: observation noise [nworld, nobs] or None (added to both
    observations); feet_state [nworld, 2 nf + 1] or None (fresh worlds)."""
    nw = qpos.shape[0]
    if feet_state is None:
        feet_state = np.tile(feet_state0(m), (nw, 1))
    u = np.repeat(np.asarray(action, dtype=np.float64)[None], nsub, axis=0)
    if dr is None:
        ms, os_ = [m] * nw, [o] * nw
        r = o.step(qpos.copy(), qvel.copy(), qacc_ws.copy(), u, nstep=nsub, mode=mode,
                   nthreads=8)
        q, v, ws = r["qpos"], r["qvel"], r["qacc_ws"]
        pairs = [set(r["contacts"][w, :r["ncon"][w], 16].astype(int).tolist()) for w in range(nw)]
    else:
        ms = [randomized_model(m, dr[w]) for w in range(nw)]
        os_ = [randomized_oracle(o, m, dr[w]) for w in range(nw)]
        q, v, ws = np.zeros_like(qpos), np.zeros_like(qvel), np.zeros_like(qacc_ws)
        pairs = []
        for w in range(nw):
            r = os_[w].step(qpos[w:w + 1].copy(), qvel[w:w + 1].copy(), qacc_ws[w:w + 1].copy(),
                            u[:, w:w + 1], nstep=nsub, mode=mode)
            q[w], v[w], ws[w] = r["qpos"][0], r["qvel"][0], r["qacc_ws"][0]
            pairs.append(set(r["contacts"][0, :r["ncon"][0], 16].astype(int).tolist()))
    dt_env = nsub * m.opt.timestep
    nz = lambda w: None if noise is None else noise[w]
    term = np.stack([observe(ms[w], q[w], v[w], prev_action[w], cmd[w], nz(w)) for w in range(nw)])
    rew, done, nfs = np.zeros(nw), np.zeros(nw, dtype=bool), np.zeros_like(feet_state)
    for w in range(nw):
        finite = np.all(np.isfinite(q[w])) and np.all(np.isfinite(v[w]))
        if finite:
            terms, nfs[w] = feet_terms(ms[w], os_[w], q[w], v[w], pairs[w], feet_state[w],
                                       cmd[w], dt_env)
            extra = sum(terms.values())
        else:
            extra, nfs[w] = 0.0, feet_state[w]
        rew[w], done[w] = reward_done(ms[w], q[w], v[w], action[w], prev_action[w], cmd[w],
                                      extra)
    nxt_prev = np.where(done[:, None], 0.0, action)
    q = np.where(done[:, None], reset_qpos, q)
    v = np.where(done[:, None], reset_qvel, v)
    ws = np.where(done[:, None], 0.0, ws)
    nfs = np.where(done[:, None], feet_state0(m)[None], nfs)
    obs = np.stack([observe(ms[w], q[w], v[w], nxt_prev[w], cmd[w], nz(w)) if done[w]
                    else term[w] for w in range(nw)])
    return obs, rew, done, (q, v, ws, nxt_prev, nfs), term


DR_HEAD = 8


def dr_size(m):
    return DR_HEAD + 2 * m.nu + 3 * (m.nbody - 2)


def dr_identity(m):
    """The record that leaves the model as it is."""
    rec = np.zeros(dr_size(m))
    rec[0] = rec[5] = rec[6] = 1.0
    dadr = m.jnt_dofadr()
    for k, a in enumerate(m.actuators):
        j = a.joint
        rec[DR_HEAD + m.nu + k] = m.joints[j].armature
        assert dadr[j] == 6 + k
    return rec


def randomized_model(m, rec):
    """A copy of the model with one world's randomised parameters (record above)."""
    rec = np.asarray(rec, dtype=np.float64)
    n = m.nu
    assert rec.shape == (dr_size(m),)
    r = copy.deepcopy(m)
    r.pairs = [(p[0], p[1], p[2] * rec[0], *p[3:]) for p in r.pairs]
    root = r.bodies[r.joints[0].body]
    root.mass = root.mass + rec[1]
    root.ipos = tuple(np.asarray(root.ipos, dtype=np.float64) + rec[2:5])
    for b in range(2, r.nbody):
        o = DR_HEAD + 2 * n + 3 * (b - 2)
        r.bodies[b].ipos = tuple(np.asarray(r.bodies[b].ipos, dtype=np.float64) + rec[o:o + 3])
    for k, a in enumerate(r.actuators):
        a.kp, a.kd = a.kp * rec[5], a.kd * rec[6]
        a.qdefault = a.qdefault - rec[DR_HEAD + k]
        r.joints[a.joint].armature = rec[DR_HEAD + n + k]
    return r


def randomized_oracle(o_nominal, m, rec):
    """The reference for one world's randomised model, with the nominal inverse weights."""
    from oracle import Oracle
    o = Oracle(randomized_model(m, rec))
    o.set_invweight(o_nominal.body_invweight(), o_nominal.dof_invweight())
    return o
