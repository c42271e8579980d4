"""Pins of the FP64 reference's connect-equality rows (a point of one body held on a
point of another, or of the world: three two-sided soft-constraint rows).  No GPU.

What fixes the answers here, independently of the reference's arithmetic:
* a sphere pinned at its centre decouples into three one-dof problems with a
  closed-form minimiser;
* with only two-sided rows the Newton solution is the solution of one linear system;
* a parallelogram linkage closed by a connect keeps its coupler from turning and its
  cranks parallel (q_coupler = -q_crank1, q_crank2 = q_crank1);
* a capsule pinned at one end swings with the compound-pendulum period
  2 pi sqrt(I_pin / (m g d)) and, at rest, the rows carry its weight;
* two free spheres held centre to centre move relative to each other as one body of
  the reduced mass, and their centre of mass does not accelerate.
"""
import math

import numpy as np
import pytest

from oracle import MODE_CONVERGED, MODE_FIXED, Oracle
from paper_2502_08844_amd.synth import robots

from tests.test_oracle_contacts import SOLIMP, SOLREF, impedance

G = 9.81


def _KB(m):
    tc = max(SOLREF[0], 2 * m.opt.timestep)
    return 1 / (SOLIMP[1] ** 2 * tc ** 2 * SOLREF[1] ** 2), 2 / (SOLIMP[1] * tc)


@pytest.mark.parametrize("mode", [MODE_FIXED, MODE_CONVERGED])
def test_pinned_sphere_closed_form(mode):
    mass = 2.0
    m = robots.pinned_body("sphere", mass=mass, z0=1.0)
    o = Oracle(m)
    K, B = _KB(m)
    assert o.body_invweight()[1] == pytest.approx(1 / mass, rel=1e-12)
    rng = np.random.default_rng(0)
    for _ in range(4):
        dx = rng.normal(scale=4e-4, size=3)
        q = np.r_[np.array([0, 0, 1.0]) + dx, 1, 0, 0, 0]
        v = np.r_[rng.normal(scale=0.3, size=3), rng.normal(size=3)]
        f = o.forward(q, v, mode=mode)
        assert f["nrow"] == 3
        a0 = np.array([0, 0, -G])
        for k in range(3):
            d = impedance(dx[k])
            D = d / ((1 - d) * (1 / mass))
            aref = -B * v[k] - K * d * dx[k]
            assert f["D"][k] == pytest.approx(D, rel=1e-12)
            assert f["aref"][k] == pytest.approx(aref, rel=1e-12, abs=1e-12)
            a = (mass * a0[k] + D * aref) / (mass + D)
            assert f["qacc"][k] == pytest.approx(a, rel=1e-12, abs=1e-12)
            assert f["efc_force"][k] == pytest.approx(D * (aref - a), rel=1e-10, abs=1e-12)
        # the centre carries no angular coupling: angular accelerations are the smooth ones
        np.testing.assert_allclose(f["qacc"][3:], f["qacc_smooth"][3:], atol=1e-12)


@pytest.mark.parametrize("mode", [MODE_FIXED, MODE_CONVERGED])
def test_two_sided_rows_solve_one_linear_system(mode):
    rng = np.random.default_rng(1)
    for m in (robots.four_bar(damping=0.05), robots.pinned_body("capsule", anchor=(0, 0, 0.2))):
        o = Oracle(m)
        for _ in range(4):
            if m.name == "four_bar":
                q = rng.uniform(-0.4, 0.4, size=3)
            else:
                q = m.qpos0 + np.r_[rng.normal(scale=1e-3, size=3), 0, 0, 0, 0]
                q[3:7] = robots.axis_angle_quat(rng.normal(size=3), 0.2)
            v = rng.normal(size=m.nv)
            f = o.forward(q, v, mode=mode)
            M, a0, J, aref, D = f["M"], f["qacc_smooth"], f["J"], f["aref"], f["D"]
            a = np.linalg.solve(M + (J.T * D) @ J, M @ a0 + J.T @ (D * aref))
            assert np.max(np.abs(f["qacc"] - a)) < 1e-10 * (1 + np.abs(a).max())


def test_parallelogram_linkage_kinematics():
    m = robots.four_bar()
    o = Oracle(m)
    tq, tv, _ = o.trajectory(np.array([0.3, -0.3, 0.3]), np.zeros(3), 2500,
                             mode=MODE_FIXED)
    assert np.abs(tq[:, 0] + tq[:, 1]).max() < 1e-3
    assert np.abs(tq[:, 2] - tq[:, 0]).max() < 1e-3
    assert tq[:, 0].min() < -0.25  # it swings through


def test_pinned_capsule_compound_pendulum():
    mass, d = 1.0, 0.2
    m = robots.pinned_body("capsule", mass=mass, anchor=(0, 0, d), z0=1.0, timestep=0.0005)
    o = Oracle(m)
    b = m.bodies[1]
    I_pin = b.inertia[1] + mass * d * d
    T = 2 * math.pi * math.sqrt(I_pin / (mass * G * d))
    th = 0.03
    pin = np.array([0, 0, 1.0 + d])
    R = robots.quat_to_mat(robots.axis_angle_quat((0, 1, 0), th))
    q = np.r_[pin - R @ np.array([0, 0, d]), robots.axis_angle_quat((0, 1, 0), th)]
    n = int(2.2 * T / m.opt.timestep)
    tq, _, _ = o.trajectory(q, np.zeros(6), n, mode=MODE_FIXED)
    x = tq[:, 0]  # the centre's horizontal offset changes sign twice a period
    ups = [i for i in range(1, n) if x[i - 1] < 0 <= x[i]]
    assert len(ups) >= 2
    period = (ups[1] - ups[0]) * m.opt.timestep
    assert period == pytest.approx(T, rel=5e-3)


def test_pinned_capsule_at_rest_rows_carry_weight():
    mass = 1.3
    m = robots.pinned_body("capsule", mass=mass, anchor=(0, 0, 0.2))
    o = Oracle(m)
    r = o.step(m.qpos0[None], np.zeros((1, 6)), nstep=4000, mode=MODE_CONVERGED)
    f = o.forward(r["qpos"][0], r["qvel"][0], mode=MODE_CONVERGED)
    np.testing.assert_allclose(f["efc_force"], [0, 0, mass * G], atol=1e-8 * mass * G)
    assert np.abs(f["qacc"]).max() < 1e-8


@pytest.mark.parametrize("mode", [MODE_FIXED, MODE_CONVERGED])
def test_connected_spheres_reduced_mass(mode):
    """Two free spheres held centre to centre: the relative motion is a one-body problem
    with the reduced mass mu = m1 m2 / (m1 + m2), whose inverse 1/m1 + 1/m2 is the
    regulariser's A."""
    m1, m2 = 1.0, 3.0
    m = robots.connected_spheres(m1, m2, gravity=(0.0, 0.0, 0.0))
    o = Oracle(m)
    K, B = _KB(m)
    mu = m1 * m2 / (m1 + m2)
    rng = np.random.default_rng(5)
    for _ in range(3):
        q = m.qpos0.copy()
        sep = rng.normal(scale=3e-4, size=3)
        q[7:10] = q[0:3] - sep  # p1 - p2 = sep
        v = rng.normal(size=12)
        f = o.forward(q, v, mode=mode)
        for k in range(3):
            d = impedance(sep[k])
            D = d / ((1 - d) * (1 / m1 + 1 / m2))
            vrel = v[k] - v[6 + k]
            aref = -B * vrel - K * d * sep[k]
            arel = D * aref / (mu + D)  # smooth relative acceleration is 0 here
            assert f["D"][k] == pytest.approx(D, rel=1e-12)
            assert f["qacc"][k] - f["qacc"][6 + k] == pytest.approx(arel, rel=1e-10, abs=1e-12)
            # momentum: the pair's centre of mass does not accelerate
            assert m1 * f["qacc"][k] + m2 * f["qacc"][6 + k] == pytest.approx(0, abs=1e-9)
