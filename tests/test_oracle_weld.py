"""Pins of the FP64 reference's weld equality (a body's pose held relative to another
body or the world: the three translational rows of a connect, then three rotational
rows on the error rotation E = R1 Q R2^T, residual vee(E - E^T)/2, J = J_w1 - J_w2).
No GPU.

What fixes the answers, independently of the reference's arithmetic:
* a box welded to the world at its centre and at its reference orientation decouples
  into six one-dof problems with a closed-form minimiser (the rotational ones act on
  the body-frame angular velocity through its principal inertias);
* a box welded to the world off its centre hangs as a cantilever: at rest the rows
  carry its weight and the moment m g L of its weight about the anchor;
* the first three rows of a weld are the connect rows of the same anchors;
* two free boxes welded together exchange only internal forces and torques: their
  total linear momentum is constant, and their relative pose stays at the reference.
"""
import numpy as np
import pytest

from oracle import MODE_CONVERGED, MODE_FIXED, Oracle
from paper_2502_08844_amd.synth import robots
from paper_2502_08844_amd.synth.model import EQ_CONNECT, Equality

from tests.test_oracle_contacts import SOLIMP, SOLREF, impedance

G = 9.81


def _KB(m):
    tc = max(SOLREF[0], 2 * m.opt.timestep)
    return 1 / (SOLIMP[1] ** 2 * tc ** 2 * SOLREF[1] ** 2), 2 / (SOLIMP[1] * tc)


@pytest.mark.parametrize("mode", [MODE_FIXED, MODE_CONVERGED])
def test_welded_box_six_one_dof_problems(mode):
    mass, half, z0 = 1.5, (0.1, 0.05, 0.03), 0.3
    m = robots.welded_box(mass=mass, half=half, z0=z0)
    o = Oracle(m)
    K, B = _KB(m)
    Ib = robots.box_inertia(mass, half)
    rng = np.random.default_rng(3)
    for _ in range(4):
        dx = rng.normal(scale=4e-4, size=3)
        q = np.r_[np.array([0, 0, z0]) + dx, 1, 0, 0, 0]
        v = rng.normal(scale=0.5, size=6)
        f = o.forward(q, v, mode=mode)
        assert f["nrow"] == 6
        a0 = f["qacc_smooth"]
        inert = np.r_[mass, mass, mass, np.diag(Ib)]
        for k in range(6):
            r = dx[k] if k < 3 else 0.0
            d = impedance(r)
            D = d / ((1 - d) * (1 / mass))
            aref = -B * v[k] - K * d * r
            assert f["D"][k] == pytest.approx(D, rel=1e-12)
            assert f["aref"][k] == pytest.approx(aref, rel=1e-12, abs=1e-12)
            a = (inert[k] * a0[k] + D * aref) / (inert[k] + D)
            assert f["qacc"][k] == pytest.approx(a, rel=1e-10, abs=1e-12)


def test_cantilever_carries_weight_and_moment():
    mass, L, z0 = 2.0, 0.08, 0.3
    m = robots.welded_box(mass=mass, z0=z0, anchor=(-L, 0, z0))
    o = Oracle(m)
    r = o.step(m.qpos0[None].copy(), np.zeros((1, 6)), nstep=2000, mode=MODE_CONVERGED)
    f = o.forward(r["qpos"][0], r["qvel"][0], r["qacc_ws"][0], mode=MODE_CONVERGED)
    F = f["efc_force"]
    # translational rows: the weight, upwards; rotational rows: the moment about the
    # centre of the anchor force, cancelled: (c - a) x (m g z) = (L, 0, 0) x (0, 0, m g)
    np.testing.assert_allclose(F[:3], [0, 0, mass * G], rtol=1e-6, atol=1e-8)
    np.testing.assert_allclose(F[3:], [0, -L * mass * G, 0], rtol=1e-6, atol=1e-8)
    assert np.abs(r["qvel"]).max() < 1e-9


def test_weld_translational_rows_are_connect_rows():
    mw = robots.welded_pair()
    mc = robots.welded_pair()
    e = mc.equalities[0]
    mc.equalities = [Equality(type=EQ_CONNECT, body1=e.body1, body2=e.body2,
                              anchor1=e.anchor1, anchor2=e.anchor2)]
    rng = np.random.default_rng(5)
    q = mw.qpos0 + np.r_[rng.normal(scale=1e-3, size=3), 0, 0, 0, 0,
                         rng.normal(scale=1e-3, size=3), 0, 0, 0, 0]
    v = rng.normal(size=12)
    fw, fc = Oracle(mw).forward(q, v), Oracle(mc).forward(q, v)
    assert fw["nrow"] == 6 and fc["nrow"] == 3
    for k in ("J", "aref", "D"):
        np.testing.assert_array_equal(fw[k][:3], fc[k])


def test_welded_pair_internal_forces_and_relative_pose():
    m = robots.welded_pair()
    o = Oracle(m)
    rng = np.random.default_rng(7)
    q0 = m.qpos0.copy()
    v0 = rng.normal(scale=0.5, size=12)
    masses = [m.bodies[1].mass, m.bodies[2].mass]
    p0 = masses[0] * v0[0:3] + masses[1] * v0[6:9]
    q, v, ws = q0[None].copy(), v0[None].copy(), None
    R_ref = robots.quat_to_mat(q0[3:7]).T @ robots.quat_to_mat(q0[10:14])
    for _ in range(5):
        r = o.step(q, v, ws, nstep=100, mode=MODE_CONVERGED)
        q, v, ws = r["qpos"], r["qvel"], r["qacc_ws"]
        p = masses[0] * v[0, 0:3] + masses[1] * v[0, 6:9]
        np.testing.assert_allclose(p, p0, atol=1e-12)
    R_rel = robots.quat_to_mat(q[0, 3:7]).T @ robots.quat_to_mat(q[0, 10:14])
    assert np.abs(R_rel - R_ref).max() < 2e-3
