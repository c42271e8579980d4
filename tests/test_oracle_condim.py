"""Pins of the FP64 reference's frictionless contacts (pair condim 1: one row along the
normal, J = J_n, R = (1-d)/d (w1 + w2)).  No GPU.

What fixes the answers, independently of the reference's arithmetic:
* a sphere resting on a plane carries m g with no tangential force, at the penetration
  p solving the scalar soft-contact balance m g = m K d(p)^2 p / (1 - d(p)) of a
  single row (the friction pyramid's four rows give (1 + mu^2) / 4 times it);
* on a plane tilted by theta (gravity tilted instead) a frictionless box accelerates
  down the slope at exactly g sin(theta), whatever its contacts do along the normal;
* each frictionless contact takes one row.
"""
import math

import numpy as np
import pytest
from scipy.optimize import brentq

from oracle import MODE_CONVERGED, Oracle
from paper_2502_08844_amd.synth import robots

from tests.test_oracle_contacts import SOLIMP, SOLREF, impedance

G = 9.81


def test_frictionless_sphere_rest_penetration():
    r, mass = 0.1, 3.0
    m = robots.free_body("sphere", mass=mass, half=(r, 0, 0), plane=True, condim=1,
                         timestep=0.002)
    o = Oracle(m)
    tc = max(SOLREF[0], 2 * m.opt.timestep)
    K = 1 / (SOLIMP[1] ** 2 * tc ** 2 * SOLREF[1] ** 2)
    p = brentq(lambda p: p - G * (1 - impedance(-p)) / (K * impedance(-p) ** 2), 1e-9, 0.05)
    q0 = m.qpos0.copy()
    q0[2] = r
    res = o.step(q0[None], np.zeros((1, 6)), nstep=3000, mode=MODE_CONVERGED)
    c = res["contacts"][0, 0]
    assert res["ncon"][0] == 1
    assert -c[0] == pytest.approx(p, rel=1e-6)
    assert c[13] == pytest.approx(mass * G, rel=1e-9)
    assert c[14] == 0 and c[15] == 0
    f = o.forward(res["qpos"][0], res["qvel"][0], res["qacc_ws"][0], mode=MODE_CONVERGED)
    assert f["nrow"] == 1


@pytest.mark.parametrize("theta", [0.2, 0.6])
def test_frictionless_box_slides_at_g_sin_theta(theta):
    grav = (G * math.sin(theta), 0.0, -G * math.cos(theta))
    m = robots.free_body("box", mass=1.0, half=(0.1, 0.2, 0.05), plane=True, condim=1,
                         gravity=grav, timestep=0.002)
    o = Oracle(m)
    q0 = m.qpos0.copy()
    q0[2] = 0.05
    q, v, ws = q0[None], np.zeros((1, 6)), None
    for _ in range(3):
        res = o.step(q, v, ws, nstep=100, mode=MODE_CONVERGED)
        q, v, ws = res["qpos"], res["qvel"], res["qacc_ws"]
        assert res["ncon"][0] == 4
        assert res["qacc"][0, 0] == pytest.approx(G * math.sin(theta), rel=1e-12)
        assert np.abs(res["contacts"][0, :4, 14:16]).max() == 0
    f = o.forward(q[0], v[0], ws[0], mode=MODE_CONVERGED)
    assert f["nrow"] == 4


# ------------------------------------------------------------------ condim 4 and 6
def _settled_sphere(condim, mu_t=0.0, mu_r=0.0, r=0.1, mass=3.0):
    m = robots.free_body("sphere", mass=mass, half=(r, 0, 0), plane=True, condim=condim,
                         mu_torsion=mu_t, mu_rolling=mu_r, timestep=0.002)
    o = Oracle(m)
    q0 = m.qpos0.copy()
    q0[2] = r
    res = o.step(q0[None], np.zeros((1, 6)), nstep=1500, mode=MODE_CONVERGED)
    return m, o, res


def _trace(o, res, v, nstep):
    """Per step: contact count, velocity, acceleration and the rows' total force."""
    q, vv, ws = res["qpos"], v, res["qacc_ws"]
    out = []
    for _ in range(nstep):
        f = o.forward(q[0], vv[0], ws[0], mode=MODE_CONVERGED)
        r = o.step(q, vv, ws, nstep=1, mode=MODE_CONVERGED)
        out.append((int(r["ncon"][0]), vv[0].copy(), f["qacc"].copy(), f["efc_force"].sum(),
                    f["nrow"]))
        q, vv, ws = r["qpos"], r["qvel"], r["qacc_ws"]
    return out


@pytest.mark.parametrize("condim,mu_t", [(3, 0.0), (4, 0.01), (4, 0.02)])
def test_torsional_friction_opposes_spin_within_its_bound(condim, mu_t):
    """Spin about the vertical.  A point contact with sliding friction only exerts no
    torque about the normal: the spin is kept exactly.  Torsional friction (two more
    pyramid edges J_n -+ mu_t J_spin with forces f+, f- >= 0) exerts the torque
    mu_t (f+ - f-), so |I_z dw/dt| <= mu_t sum(f) at every step, and the spin falls
    monotonically.  (The soft contact makes the torque approach that bound only where
    the edges' slip mu_t w is large against its regularisation: at these rates it is
    velocity dependent, not Coulomb's.)  The spin stays below g / (B mu_t):
    an edge reads it as a normal approach speed mu_t w, and its reference acceleration
    B mu_t w would lift the ball off the plane above that."""
    r, mass, w0 = 0.1, 3.0, 1.5
    m, o, res = _settled_sphere(condim, mu_t, r=r, mass=mass)
    v = res["qvel"].copy()
    v[0, 5] = w0
    tr = _trace(o, res, v, 25)
    assert all(n == 1 for n, *_ in tr)
    w = np.array([x[1][5] for x in tr])
    if condim == 3:
        np.testing.assert_allclose(w, w0, rtol=1e-10)
        assert tr[-1][4] == 4
        return
    assert tr[-1][4] == 6
    assert np.all(np.diff(w) < 0)
    Iz = 0.4 * mass * r * r
    torque = np.array([-Iz * x[2][5] for x in tr])
    bound = np.array([mu_t * x[3] for x in tr])
    assert np.all(torque > 0) and np.all(torque <= bound * (1 + 1e-9))


@pytest.mark.parametrize("condim,mu_r", [(4, 0.0), (6, 0.002)])
def test_rolling_friction_opposes_rolling_within_its_bound(condim, mu_r):
    """A ball rolling without slipping keeps rolling under sliding and torsional
    friction alone (to 1e-3 over 60 steps, the soft contact's own loss; rolling
    friction takes 17 times that here).  Rolling friction (edges J_n -+ mu_r J_roll about the tangents)
    resists it: the speed falls monotonically, and the resisting torque, (I/r + m r)
    |dv/dt| (m a = f, I alpha = -f r - tau, a = alpha r), never exceeds mu_r sum(f)."""
    r, mass, v0 = 0.1, 3.0, 1.0
    m, o, res = _settled_sphere(condim, 0.01, mu_r, r=r, mass=mass)
    v = res["qvel"].copy()
    v[0, 0], v[0, 4] = v0, v0 / r  # x velocity with the spin about +y of rolling
    tr = _trace(o, res, v, 60)
    assert all(n == 1 for n, *_ in tr)
    vx = np.array([x[1][0] for x in tr])
    if condim == 4:
        np.testing.assert_allclose(vx, v0, rtol=1e-3)
        return
    assert tr[-1][4] == 10
    assert np.all(np.diff(vx[5:]) < 0)
    I = 0.4 * mass * r * r
    tau = np.array([-(I / r + mass * r) * x[2][0] for x in tr])[5:]
    bound = np.array([mu_r * x[3] for x in tr])[5:]
    assert np.all(tau > 0) and np.all(tau <= bound * (1 + 1e-6))


@pytest.mark.parametrize("condim", [4, 6])
def test_resting_ball_normal_force_sums_every_edge(condim):
    """At rest the torsional and rolling edges carry part of the load like the sliding
    ones (every edge has unit normal component): the exported normal force, the sum
    over all edges, is m g."""
    mass = 3.0
    m, o, res = _settled_sphere(condim, 0.02, 0.002, mass=mass)
    assert res["contacts"][0, 0, 13] == pytest.approx(mass * G, rel=1e-9)
