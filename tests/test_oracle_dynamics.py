"""Pins of the FP64 reference's smooth dynamics (kinematics, CRBA, RNE, LTDL, Euler).

Each check compares the reference with something other than itself: a closed form, a
conservation law, a brute-force construction from finite differences, or a library
routine.  No GPU.
"""
import math
import os

import numpy as np
import pytest

from oracle import Oracle
from paper_2502_08844_amd.synth import model as mdl
from paper_2502_08844_amd.synth import robots

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
G = 9.81


# ------------------------------------------------------------------ helpers
def quat_mul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2,
                     w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2,
                     w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def quat_exp(w):
    a = np.linalg.norm(w)
    if a < 1e-300:
        return np.array([1.0, 0, 0, 0])
    return np.concatenate([[math.cos(a / 2)], math.sin(a / 2) * w / a])


def tangent_perturb(m, qpos, k, eps):
    """qpos moved by eps along dof k (free rotations: body-frame exponential map)."""
    q = np.array(qpos, dtype=np.float64)
    for j, qa, da in zip(m.joints, m.jnt_qposadr(), m.jnt_dofadr()):
        nv = mdl.JNT_NV[j.type]
        if not (da <= k < da + nv):
            continue
        if j.type == mdl.JNT_FREE:
            i = k - da
            if i < 3:
                q[qa + i] += eps
            else:
                e = np.zeros(3)
                e[i - 3] = eps
                q[qa + 3:qa + 7] = quat_mul(q[qa + 3:qa + 7], quat_exp(e))
        else:
            q[qa] += eps
    return q


def body_inertia_world(m, xmat, b):
    Ib = m.bodies[b].inertia
    I = np.array([[Ib[0], Ib[3], Ib[4]], [Ib[3], Ib[1], Ib[5]], [Ib[4], Ib[5], Ib[2]]])
    return xmat[b] @ I @ xmat[b].T


def fd_jacobians(o, m, qpos, eps=1e-6):
    """Per-body COM (Jv) and angular (Jw) Jacobians by central differences of FK."""
    nb, nv = m.nbody, m.nv
    Jv = np.zeros((nb, 3, nv))
    Jw = np.zeros((nb, 3, nv))
    for k in range(nv):
        fp = o.forward(tangent_perturb(m, qpos, k, eps))
        fm = o.forward(tangent_perturb(m, qpos, k, -eps))
        Jv[:, :, k] = (fp["xipos"] - fm["xipos"]) / (2 * eps)
        for b in range(nb):
            Rdot = (fp["xmat"][b] - fm["xmat"][b]) / (2 * eps)
            R = 0.5 * (fp["xmat"][b] + fm["xmat"][b])
            W = Rdot @ R.T
            W = 0.5 * (W - W.T)
            Jw[b, :, k] = (W[2, 1], W[0, 2], W[1, 0])
    return Jv, Jw


def brute_mass_matrix(o, m, qpos):
    Jv, Jw = fd_jacobians(o, m, qpos)
    xmat = o.forward(qpos)["xmat"]
    M = np.zeros((m.nv, m.nv))
    for b in range(1, m.nbody):
        Iw = body_inertia_world(m, xmat, b)
        M += m.bodies[b].mass * Jv[b].T @ Jv[b] + Jw[b].T @ Iw @ Jw[b]
    arm = np.concatenate([[j.armature] * mdl.JNT_NV[j.type] for j in m.joints])
    return M + np.diag(arm)


def potential(o, m, qpos):
    xipos = o.forward(qpos)["xipos"]
    return sum(m.bodies[b].mass * G * xipos[b, 2] for b in range(1, m.nbody))


def random_pose(m, rng, scale=0.5):
    q = np.array(m.qpos0, dtype=np.float64)
    for j, qa in zip(m.joints, m.jnt_qposadr()):
        if j.type == mdl.JNT_FREE:
            q[qa:qa + 3] += rng.uniform(-0.2, 0.2, 3)
            quat = rng.normal(size=4)
            q[qa + 3:qa + 7] = quat / np.linalg.norm(quat)
        else:
            q[qa] += rng.uniform(-scale, scale)
    return q


# ------------------------------------------------------------------ P1 pendulum
def _period(t, theta, center):
    s = theta - center
    idx = np.where((s[:-1] > 0) & (s[1:] <= 0))[0]
    # linear interpolation of the downward crossings
    tc = t[idx] + (t[idx + 1] - t[idx]) * s[idx] / (s[idx] - s[idx + 1])
    return (tc[-1] - tc[0]) / (len(tc) - 1)


def test_pendulum_period_fixed_pivot():
    m = robots.hinge_chain(n=1, link=0.6, mass=0.1, damping=0.0)
    m.opt.timestep = 1e-4
    o = Oracle(m)
    r, hl, mass, d = 0.03, 0.3, 0.1, 0.3
    Ip = robots.capsule_inertia(mass, r, hl)[0, 0] + mass * d * d
    T = 2 * math.pi * math.sqrt(Ip / (mass * G * d))
    th0 = 0.01
    nstep = int(20.5 * T / 1e-4)
    tq, _, _ = o.trajectory([math.pi / 2 + th0], [0.0], nstep)
    t = 1e-4 * np.arange(1, nstep + 1)
    Tm = _period(t, tq[:, 0], math.pi / 2)
    assert abs(Tm / (T * (1 + th0 ** 2 / 16)) - 1) < 2e-5


def test_pendulum_period_cart_free():
    m = robots.cartpole(hanging=True, damping=0.0, timestep=1e-4)
    o = Oracle(m)
    Mc, mp, d = 1.0, 0.1, 0.3
    Ip = robots.capsule_inertia(mp, 0.045, 0.3)[0, 0] + mp * d * d
    w2 = (Mc + mp) * mp * G * d / ((Mc + mp) * Ip - mp * mp * d * d)
    T = 2 * math.pi / math.sqrt(w2)
    th0 = 0.01
    nstep = int(20.5 * T / 1e-4)
    tq, _, _ = o.trajectory([0.0, th0], [0.0, 0.0], nstep, ctrl=np.zeros(nstep))
    t = 1e-4 * np.arange(1, nstep + 1)
    Tm = _period(t, tq[:, 1], 0.0)
    assert abs(Tm / T - 1) < 3e-5
    # horizontal momentum is conserved: the system's COM never moves sideways
    f = o.forward(tq[-1])
    com_x = (Mc * f["xipos"][1, 0] + mp * f["xipos"][2, 0]) / (Mc + mp)
    f0 = o.forward([0.0, th0])
    com0 = (Mc * f0["xipos"][1, 0] + mp * f0["xipos"][2, 0]) / (Mc + mp)
    assert abs(com_x - com0) < 1e-9


# ------------------------------------------------------------------ P2 energy
def _energy(o, m, q, v):
    f = o.forward(q, v)
    return 0.5 * v @ f["M"] @ v + sum(m.bodies[b].mass * G * f["xipos"][b, 2]
                                      for b in range(1, m.nbody))


def _rk4(o, q, v, h, nstep):
    def acc(q, v):
        return o.forward(q, v)["qacc_smooth"]
    for _ in range(nstep):
        k1q, k1v = v, acc(q, v)
        k2q, k2v = v + 0.5 * h * k1v, acc(q + 0.5 * h * k1q, v + 0.5 * h * k1v)
        k3q, k3v = v + 0.5 * h * k2v, acc(q + 0.5 * h * k2q, v + 0.5 * h * k2v)
        k4q, k4v = v + h * k3v, acc(q + h * k3q, v + h * k3v)
        q = q + h / 6 * (k1q + 2 * k2q + 2 * k3q + k4q)
        v = v + h / 6 * (k1v + 2 * k2v + 2 * k3v + k4v)
    return q, v


@pytest.mark.parametrize("axes", [None, [(0, 1, 0), (1, 0, 0), (0, 0, 1), (0, 1, 1)]])
def test_energy_conserved_rk4(axes):
    m = robots.hinge_chain(n=4, link=0.3, axes=axes)
    o = Oracle(m)
    q0 = np.array([0.3, -0.2, 0.4, 0.1])
    v0 = np.array([0.5, -1.0, 0.7, 0.2])
    E0 = _energy(o, m, q0, v0)
    q, v = _rk4(o, q0, v0, 1e-4, 10000)
    E1 = _energy(o, m, q, v)
    scale = abs(E0) + 0.5 * v0 @ o.forward(q0)["M"] @ v0
    assert abs(E1 - E0) / scale < 1e-9


def test_semi_implicit_euler_energy_error_is_first_order():
    errs = []
    for h in (1e-3, 5e-4):
        m = robots.hinge_chain(n=3, link=0.3)
        m.opt.timestep = h
        o = Oracle(m)
        q0 = np.array([0.3, -0.2, 0.4])
        v0 = np.zeros(3)
        E0 = _energy(o, m, q0, v0)
        n = int(round(1.0 / h))
        tq, tv, _ = o.trajectory(q0, v0, n)
        E = np.array([_energy(o, m, tq[i], tv[i]) for i in range(0, n, 10)])
        errs.append(np.max(np.abs(E - E0)))
    ratio = errs[0] / errs[1]
    assert 1.6 < ratio < 2.5


# ------------------------------------------------------------------ P3 CRBA
@pytest.mark.parametrize("kind", ["quadruped", "humanoid", "hand", "chain_slide"])
def test_mass_matrix_equals_bruteforce_and_is_spd(kind):
    rng = np.random.default_rng(7)
    if kind == "chain_slide":
        m = robots.hinge_chain(n=3, axes=[(0, 1, 0), (1, 0, 0), (0, 0, 1)], slide_root=True)
    else:
        m = robots.WORKLOADS[kind]()
    o = Oracle(m)
    q = random_pose(m, rng)
    M = o.forward(q)["M"]
    Mb = brute_mass_matrix(o, m, q)
    assert np.max(np.abs(M - Mb)) < 1e-7 * np.max(np.abs(M))
    assert np.max(np.abs(M - M.T)) <= 1e-14 * np.max(np.abs(M))
    np.linalg.cholesky(M)
    assert np.linalg.eigvalsh(M).min() > 0


# ------------------------------------------------------------------ P4 RNE
@pytest.mark.parametrize("seed", [0, 1])
def test_bias_equals_lagrangian_derivative(seed):
    rng = np.random.default_rng(seed)
    m = robots.hinge_chain(n=4, axes=[(0, 1, 0), (1, 0, 0), (0, 0, 1), (1, 1, 0)],
                           slide_root=True)
    o = Oracle(m)
    q = rng.uniform(-1, 1, m.nq)
    v = rng.uniform(-2, 2, m.nv)
    eps = 1e-5
    n = m.nv
    dM = np.zeros((n, n, n))  # dM[k] = dM/dq_k
    dV = np.zeros(n)
    for k in range(n):
        e = np.zeros(n)
        e[k] = eps
        dM[k] = (o.forward(q + e)["M"] - o.forward(q - e)["M"]) / (2 * eps)
        dV[k] = (potential(o, m, q + e) - potential(o, m, q - e)) / (2 * eps)
    Mdot = np.einsum("kij,k->ij", dM, v)
    c_lag = Mdot @ v - 0.5 * np.einsum("kij,i,j->k", dM, v, v) + dV
    c = o.forward(q, v)["bias"]
    assert np.max(np.abs(c - c_lag)) < 1e-7 * (1 + np.max(np.abs(c)))


def test_inverse_dynamics_is_mass_times_acc_plus_bias():
    rng = np.random.default_rng(3)
    m = robots.humanoid()
    o = Oracle(m)
    q = random_pose(m, rng)
    v = rng.normal(size=m.nv)
    a = rng.normal(size=m.nv)
    f = o.forward(q, v)
    tau = o.inverse(q, v, a)
    # RNEA covers the rigid bodies only; the rotor armature sits on M's diagonal
    arm = np.array([j.armature for j in m.joints for _ in range(mdl.JNT_NV[j.type])])
    assert np.allclose(tau, (f["M"] - np.diag(arm)) @ a + f["bias"], atol=1e-10)


# ------------------------------------------------------------------ P9 free fall
def test_free_fall_closed_form():
    m = robots.free_body("box", mass=2.0, z0=1.0)
    m.opt.timestep = 0.01
    o = Oracle(m)
    q0 = m.qpos0.copy()
    v0 = np.array([0.1, -0.2, 0.5, 0, 0, 0])
    f = o.forward(q0, v0)
    assert np.allclose(f["qacc"], [0, 0, -G, 0, 0, 0], atol=1e-14, rtol=0)
    n = 50
    tq, tv, _ = o.trajectory(q0, v0, n)
    h = 0.01
    k = np.arange(1, n + 1)
    z = 1.0 + k * h * 0.5 - G * h * h * k * (k + 1) / 2
    assert np.max(np.abs(tq[:, 2] - z)) < 1e-12
    assert np.max(np.abs(tq[:, 0] - k * h * 0.1)) < 1e-12
    assert np.allclose(tq[:, 3], 1.0) and np.allclose(tq[:, 4:7], 0.0)


# ------------------------------------------------------------------ P10 rigid body
def test_torque_free_body_gyroscopic_bias():
    m = robots.free_body("box", mass=1.5, gravity=(0, 0, 0), half=(0.1, 0.2, 0.3))
    o = Oracle(m)
    rng = np.random.default_rng(11)
    q = m.qpos0.copy()
    quat = rng.normal(size=4)
    q[3:7] = quat / np.linalg.norm(quat)
    w = rng.normal(size=3)
    v = np.concatenate([rng.normal(size=3), w])
    f = o.forward(q, v)
    I = np.diag(m.bodies[1].inertia[:3])
    assert np.allclose(f["bias"][3:], np.cross(w, I @ w), atol=1e-13)
    assert np.allclose(f["bias"][:3], 0.0, atol=1e-13)
    assert np.allclose(f["qacc"][3:], -np.linalg.solve(I, np.cross(w, I @ w)), atol=1e-12)


def _rk4_free(o, m, q, v, h, nstep):
    """RK4 for a model whose only non-scalar joint is one free joint at qpos[0:7]."""
    def deriv(q, v):
        qd = np.zeros_like(q)
        qd[0:3] = v[0:3]
        qd[3:7] = 0.5 * quat_mul(q[3:7], np.concatenate([[0.0], v[3:6]]))
        qd[7:] = v[6:]
        return qd, o.forward(q, v)["qacc_smooth"]
    for _ in range(nstep):
        a1, b1 = deriv(q, v)
        a2, b2 = deriv(q + 0.5 * h * a1, v + 0.5 * h * b1)
        a3, b3 = deriv(q + 0.5 * h * a2, v + 0.5 * h * b2)
        a4, b4 = deriv(q + h * a3, v + h * b3)
        q = q + h / 6 * (a1 + 2 * a2 + 2 * a3 + a4)
        v = v + h / 6 * (b1 + 2 * b2 + 2 * b3 + b4)
    return q, v


def _momentum(o, m, q, v):
    """World linear and angular momentum (about the origin) from FD Jacobians."""
    Jv, Jw = fd_jacobians(o, m, q)
    f = o.forward(q)
    P = np.zeros(3)
    L = np.zeros(3)
    for b in range(1, m.nbody):
        vc = Jv[b] @ v
        w = Jw[b] @ v
        P += m.bodies[b].mass * vc
        L += body_inertia_world(m, f["xmat"], b) @ w + np.cross(f["xipos"][b],
                                                                m.bodies[b].mass * vc)
    return P, L


@pytest.mark.slow
def test_floating_humanoid_conserves_momentum_and_energy():
    m = robots.humanoid()
    m.opt.gravity = (0.0, 0.0, 0.0)
    for j in m.joints:
        j.damping = 0.0
    m.pairs = []
    m.opt.nconmax = 0
    o = Oracle(m)
    rng = np.random.default_rng(5)
    q0 = random_pose(m, rng, scale=0.3)
    v0 = rng.normal(scale=0.5, size=m.nv)
    P0, L0 = _momentum(o, m, q0, v0)
    E0 = 0.5 * v0 @ o.forward(q0)["M"] @ v0
    q, v = _rk4_free(o, m, q0, v0, 2e-3, 100)
    P1, L1 = _momentum(o, m, q, v)
    E1 = 0.5 * v @ o.forward(q)["M"] @ v
    assert np.max(np.abs(P1 - P0)) < 1e-6 * (1 + np.abs(P0).max())
    assert np.max(np.abs(L1 - L0)) < 1e-6 * (1 + np.abs(L0).max())
    assert abs(E1 - E0) < 1e-6 * E0


def test_torque_free_body_conserves_angular_momentum():
    m = robots.free_body("box", mass=1.0, gravity=(0, 0, 0), half=(0.05, 0.15, 0.3))
    o = Oracle(m)
    q0 = m.qpos0.copy()
    v0 = np.array([0.0, 0.0, 0.0, 0.3, 2.0, 0.1])  # near the unstable middle axis
    I = np.diag(m.bodies[1].inertia[:3])

    def Lw(q, v):
        R = o.forward(q)["xmat"][1]
        return R @ I @ v[3:]
    L0 = Lw(q0, v0)
    q, v = _rk4_free(o, m, q0, v0, 1e-3, 1000)
    assert np.max(np.abs(Lw(q, v) - L0)) < 1e-10 * np.linalg.norm(L0)


# ------------------------------------------------------------------ P11 LTDL
@pytest.mark.parametrize("kind", ["quadruped", "humanoid", "hand"])
def test_ltdl_solve_matches_dense_solve(kind):
    rng = np.random.default_rng(2)
    m = robots.WORKLOADS[kind]()
    o = Oracle(m)
    q = random_pose(m, rng)
    b = rng.normal(size=m.nv)
    x, LD = o.ltdl_solve(q, b)
    M = o.forward(q)["M"]
    xr = np.linalg.solve(M, b)
    assert np.max(np.abs(x - xr)) < 1e-13 * np.max(np.abs(xr)) * np.linalg.cond(M) ** 0.5
    # factor reproduces M as L^T D L with no fill-in outside the dof-ancestor pattern
    L = np.tril(LD, -1) + np.eye(m.nv)
    D = np.diag(np.diag(LD))
    assert np.allclose(L.T @ D @ L, M, atol=1e-13 * np.abs(M).max())
    parent = o.dof_parent()
    for i in range(m.nv):
        anc = set()
        j = parent[i]
        while j >= 0:
            anc.add(j)
            j = parent[j]
        for j in range(i):
            if j not in anc:
                assert LD[i, j] == 0.0


# ------------------------------------------------------------------ actuation
def test_pd_mapping_matches_worked_cases():
    rows = []
    with open(os.path.join(GOLDEN, "pd_mapping.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([float(x) for x in line.split()])
    for kp, kd, ka, qdef, a, q, qd, tau in rows:
        m = robots.hinge_chain(n=1)
        m.actuators = [mdl.Actuator(type=mdl.ACT_PD, joint=0, gear=ka, kp=kp, kd=kd,
                                    ctrlrange=(-1, 1), qdefault=qdef)]
        o = Oracle(m)
        f = o.forward([q], [qd], ctrl=[a])
        assert f["act"][0] == pytest.approx(tau, abs=1e-12)


def test_motor_gear_clamp_and_damping():
    m = robots.cartpole()
    o = Oracle(m)
    f = o.forward([0.1, 0.2], [0.3, -0.4], ctrl=[2.5])  # clamped to 1
    assert f["act"][0] == pytest.approx(10.0) and f["act"][1] == 0.0
    assert np.allclose(f["passive"], [-0.05 * 0.3, 0.05 * 0.4])


# ------------------------------------------------------------------ offset anchors
def test_hinge_about_offset_anchor():
    """A body hinged about an anchor away from its origin swings about the anchor."""
    bld = robots._Builder("offset")
    b = bld.body(0, pos=(0.2, 0.0, 0.5))
    bld.joint(b, mdl.JNT_HINGE, axis=(0, 0, 1), pos=(-0.2, 0.0, 0.0))
    bld.geom(b, mdl.GEOM_SPHERE, (0.05,), pos=(0.1, 0, 0), mass=1.0)
    m = bld.finish()
    m.opt.nconmax = 0
    m.qpos0 = np.zeros(1)
    o = Oracle(m)
    th = 0.7
    f = o.forward([th])
    # origin rotates about the anchor (0, 0, 0.5): offset (0.2, 0, 0) -> rotated
    assert np.allclose(f["xpos"][1], [0.2 * math.cos(th), 0.2 * math.sin(th), 0.5], atol=1e-15)
    assert np.allclose(f["xipos"][1], [0.3 * math.cos(th), 0.3 * math.sin(th), 0.5], atol=1e-15)
    # a brute-force mass matrix with offset anchors on a spatial chain
    bld = robots._Builder("offset_chain")
    parent = 0
    for i, ax in enumerate([(0, 1, 0), (1, 0, 0), (0, 0, 1)]):
        b = bld.body(parent, pos=(0.25, 0.05 * i, 0.0))
        bld.joint(b, mdl.JNT_HINGE, axis=ax, pos=(-0.1, 0.02, 0.03))
        bld.capsule_fromto(b, (0, 0, 0), (0.25, 0, 0), 0.03, mass=1.0)
        parent = b
    m = bld.finish()
    m.qpos0 = np.zeros(3)
    o = Oracle(m)
    q = np.array([0.4, -0.3, 0.9])
    M = o.forward(q)["M"]
    assert np.max(np.abs(M - brute_mass_matrix(o, m, q))) < 1e-7 * np.max(np.abs(M))


# ------------------------------------------------------------------ orientation update
def test_free_sphere_spin_composes_in_body_frame():
    """An isotropic body spinning torque-free keeps its body-frame angular velocity, and
    the semi-implicit step with the exponential map gives R_n = R_0 exp(n h [w])."""
    m = robots.free_body("sphere", mass=1.0, gravity=(0, 0, 0), half=(0.1, 0, 0))
    h = 0.01
    m.opt.timestep = h
    o = Oracle(m)
    rng = np.random.default_rng(9)
    q0 = m.qpos0.copy()
    quat = rng.normal(size=4)
    q0[3:7] = quat / np.linalg.norm(quat)
    w = rng.normal(size=3)
    v0 = np.concatenate([[0, 0, 0], w])
    n = 37
    tq, tv, _ = o.trajectory(q0, v0, n)
    assert np.allclose(tv[-1, 3:], w, atol=1e-14)
    R0 = robots.quat_to_mat(q0[3:7])
    ang = n * h * np.linalg.norm(w)
    Rw = robots.quat_to_mat(robots.axis_angle_quat(w, ang))
    Rn = o.forward(tq[-1])["xmat"][1]
    assert np.allclose(Rn, R0 @ Rw, atol=1e-12)
