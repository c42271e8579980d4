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
  termination              -1.0 * done
* termination: the root body's z axis points downwards (the robot has inverted);
* reset: a terminated world restarts from its reset state (given by the caller) with a
  zero warm start and a zero previous action; the outputs of that env step are those
  of the state it terminated in.
* the model's root is a free joint and actuator k drives dof 6 + k.
"""
from __future__ import annotations

import numpy as np

K_V, SIG_V = 1.0, 0.25
K_W, SIG_W = 0.5, 0.25
K_LINZ, K_ANGXY, K_ORI, K_TAU, K_Q, K_RATE, K_TERM = -2.0, -0.05, -5.0, -2e-4, -0.1, -0.01, -1.0


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


def observe(m, qpos, qvel, prev_action, cmd):
    R = quat_mat(qpos[3:7])
    g = R.T @ np.array([0.0, 0.0, -1.0])
    v = R.T @ qvel[0:3]  # free-joint qvel: world linear velocity of the body origin
    w = qvel[3:6]        # and the body-frame angular velocity
    qdef = np.array([a.qdefault for a in m.actuators])
    return np.concatenate([g, v, w, qpos[7:] - qdef, qvel[6:], prev_action, cmd])


def reward_done(m, qpos, qvel, action, prev_action, cmd):
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
         + K_RATE * np.sum((action - prev_action) ** 2) + K_TERM * float(done))
    return max(r, 0.0), bool(done)


def env_step(o, m, qpos, qvel, qacc_ws, prev_action, action, cmd, reset_qpos, reset_qvel,
             nsub, mode=0):
    """One env step of every world (arrays [nworld, ...]); returns the outputs and the
    next (qpos, qvel, qacc_ws, prev_action) after resets."""
    nw = qpos.shape[0]
    u = np.repeat(np.asarray(action, dtype=np.float64)[None], nsub, axis=0)
    r = o.step(qpos.copy(), qvel.copy(), qacc_ws.copy(), u, nstep=nsub, mode=mode, nthreads=8)
    q, v, ws = r["qpos"], r["qvel"], r["qacc_ws"]
    obs = np.stack([observe(m, q[w], v[w], prev_action[w], cmd[w]) for w in range(nw)])
    rd = [reward_done(m, q[w], v[w], action[w], prev_action[w], cmd[w]) for w in range(nw)]
    rew = np.array([x[0] for x in rd])
    done = np.array([x[1] for x in rd])
    nxt_prev = np.where(done[:, None], 0.0, action)
    q = np.where(done[:, None], reset_qpos, q)
    v = np.where(done[:, None], reset_qvel, v)
    ws = np.where(done[:, None], 0.0, ws)
    return obs, rew, done, (q, v, ws, nxt_prev)
