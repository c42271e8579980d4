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
