"""Pins of the reference's elliptic friction cone (model option cone = 1), no GPU.

Each check compares the reference with something other than itself:
* rotating a sliding sphere's velocity about the contact normal rotates its friction
  force with it, magnitude unchanged (a round cone; the pyramid fails this);
* a box sliding down an incline steeper than its friction angle, in any direction:
  every contact's friction force has magnitude mu f_n exactly and opposes the slip, and
  along the slope the box accelerates at g sin(theta) - mu (sum of f_n) / m;
* a box on an incline below its friction angle is held: in its steady state friction
  balances gravity's pull along the slope, every contact strictly inside the cone;
* one contact: the converged force equals the minimiser of the dual problem
  min over f in the cone of 1/2 f^T (A + R) f + f^T (J a0 - aref), A = J M^-1 J^T,
  found by brute force (zones enumerated, the cone's surface searched directly);
* the solver's Hessian is exact: one Newton iteration from a point eps away from the
  solution lands O(eps^2) away;
* frictionless contacts (condim 1) are the pyramid's.
"""
import math

import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import MODE_CONVERGED, MODE_FIXED, Oracle
from paper_2502_08844_amd.synth import robots

G = 9.81


def _elliptic(m):
    m.opt.cone = 1
    return m


def _sliding_sphere(angle, cone, v=0.8, mu=0.5):
    m = robots.free_body("sphere", mass=2.0, half=(0.1, 0, 0), z0=0.1, plane=True, mu=mu,
                         timestep=0.002)
    m.opt.cone = cone
    q = m.qpos0.copy()
    q[2] = 0.1 - 1e-3   # 1 mm into the plane
    qv = np.zeros(6)
    qv[0:2] = v * np.array([math.cos(angle), math.sin(angle)])
    return m, q, qv


def _world_friction(c):
    """World friction force of exported contact rows c (frame rows 4:13, forces 13:16)."""
    fr = c[:, 4:13].reshape(-1, 3, 3)
    return np.einsum("k,kj->j", c[:, 14], fr[:, 1]) + np.einsum("k,kj->j", c[:, 15], fr[:, 2])


def test_friction_turns_with_the_slip_direction():
    mags, pyr = [], []
    for ang in np.linspace(0.0, math.pi / 2, 7):
        m, q, v = _sliding_sphere(ang, 1)
        f = Oracle(m).forward(q, v, mode=MODE_CONVERGED)
        c = f["contacts"]
        assert len(c) == 1
        ft = _world_friction(c)
        mags.append(np.linalg.norm(ft))
        vdir = np.array([math.cos(ang), math.sin(ang), 0.0])
        np.testing.assert_allclose(ft / np.linalg.norm(ft), -vdir, atol=1e-12)
        # sliding: the force sits on the cone's surface
        assert np.linalg.norm(ft) == pytest.approx(0.5 * c[0, 13], rel=1e-12)
        mp, qp_, vp = _sliding_sphere(ang, 0)
        pyr.append(np.linalg.norm(_world_friction(Oracle(mp).forward(qp_, vp, mode=MODE_CONVERGED)["contacts"])))
    assert np.ptp(mags) <= 1e-12 * max(mags)
    assert np.ptp(pyr) > 1e-3 * max(pyr)  # the pyramid's friction depends on the direction


def _incline_box(theta, mu, v0, dirn=(1.0, 0.0)):
    """A box on a plane under gravity tilted by theta towards dirn (the incline), moving
    at v0 down the slope."""
    dirn = np.asarray(dirn) / np.linalg.norm(dirn)
    grav = (G * math.sin(theta) * dirn[0], G * math.sin(theta) * dirn[1], -G * math.cos(theta))
    m = _elliptic(robots.free_body("box", mass=1.5, half=(0.15, 0.15, 0.02), plane=True, mu=mu,
                                   gravity=grav, timestep=0.002, iterations=30))
    q = m.qpos0.copy()
    q[2] = 0.02 - 2e-4
    v = np.zeros(6)
    v[0:2] = v0 * dirn
    return m, q, v


@pytest.mark.parametrize("dirn", [(1.0, 0.0), (1.0, 1.0), (-0.3, 1.0)])
def test_box_sliding_down_an_incline(dirn):
    """A box sliding down the slope (not yet rotating): every contact's friction has
    magnitude mu f_n exactly and opposes the slip, and along the slope its centre of
    mass accelerates at g sin(theta) - mu (sum of f_n) / m (Newton's law with Coulomb's
    sliding friction at every contact; the friction's moment about the centre of mass
    pitches the box, which changes neither).  The incline's direction is immaterial."""
    theta, mu = 0.5, 0.3
    m, q, v = _incline_box(theta, mu, 0.3, dirn)
    f = Oracle(m).forward(q, v, mode=MODE_CONVERGED)
    c = f["contacts"]
    assert len(c) == 4
    fn, ft = c[:, 13], np.hypot(c[:, 14], c[:, 15])
    assert np.all(fn > 0)
    np.testing.assert_allclose(ft, mu * fn, rtol=1e-12)
    u = np.array([*np.asarray(dirn) / np.linalg.norm(dirn), 0.0])
    for k in range(4):
        fw = c[k, 14] * c[k, 7:10] + c[k, 15] * c[k, 10:13]
        np.testing.assert_allclose(fw / np.linalg.norm(fw), -u, atol=1e-12)
    along = f["qacc"][:3] @ u  # the centre of mass's acceleration along the slope
    assert along == pytest.approx(G * math.sin(theta) - mu * fn.sum() / 1.5, rel=1e-10)


def test_box_held_on_an_incline_below_the_friction_angle():
    """Below the friction angle the box is held: it settles to a steady state (the soft
    model's sticking friction acts like a stiff damper, so a slow creep carries the
    load) in which friction balances gravity's pull along the slope exactly, every
    contact strictly inside the cone."""
    theta, mu = 0.3, 0.6     # tan(0.3) = 0.31 < 0.6
    m, q, v = _incline_box(theta, mu, 0.2)
    o = Oracle(m)
    r = o.step(q, v, None, None, nstep=1500, mode=MODE_CONVERGED)
    assert np.abs(r["qacc"][0]).max() < 1e-9
    assert np.abs(r["qvel"][0]).max() < 2e-3
    c = r["contacts"][0, :int(r["ncon"][0])]
    assert len(c) == 4
    fw = _world_friction(c)
    assert fw[0] == pytest.approx(-1.5 * G * math.sin(theta), rel=1e-9)
    assert c[:, 13].sum() == pytest.approx(1.5 * G * math.cos(theta), rel=1e-9)
    assert np.all(np.hypot(c[:, 14], c[:, 15]) < 0.9 * mu * c[:, 13])


def _dual_bruteforce(A, R, b, mu):
    """argmin over f with |f_t| <= mu f_n of 1/2 f^T (A + R) f + f^T b (3 x 3): the
    unconstrained minimiser if it lies in the cone, else the best of f = 0 and the
    minimiser over the cone's surface f = f_n (1, mu cos p, mu sin p), f_n >= 0, searched
    over a fine grid of p and refined."""
    Q = A + R
    obj = lambda f: 0.5 * f @ Q @ f + f @ b
    cand = [np.zeros(3)]
    f0 = np.linalg.solve(Q, -b)
    if f0[0] >= 0 and np.hypot(f0[1], f0[2]) <= mu * f0[0]:
        return f0
    def surf(p):
        u = np.array([1.0, mu * math.cos(p), mu * math.sin(p)])
        fn = max(0.0, -(u @ b) / (u @ Q @ u))
        return fn * u
    ps = np.linspace(0.0, 2 * math.pi, 20001)
    best = min(ps, key=lambda p: obj(surf(p)))
    res = minimize(lambda x: obj(surf(x[0])), [best], method="Nelder-Mead",
                   options={"xatol": 1e-14, "fatol": 1e-18, "maxiter": 2000})
    cand.append(surf(res.x[0]))
    return min(cand, key=obj)


@pytest.mark.parametrize("seed", range(4))
def test_one_contact_equals_the_dual_bruteforce(seed):
    rng = np.random.default_rng(seed)
    m = _elliptic(robots.free_body("sphere", mass=1.3, half=(0.08, 0, 0), z0=0.08, plane=True,
                                   mu=0.7, timestep=0.002, iterations=60))
    o = Oracle(m)
    q = m.qpos0.copy()
    q[2] = 0.08 - rng.uniform(2e-4, 2e-3)
    v = np.zeros(6)
    v[0:3] = rng.normal(scale=[0.5, 0.5, 0.2])
    v[3:6] = rng.normal(scale=3.0, size=3)
    f = o.forward(q, v, mode=MODE_CONVERGED)
    assert f["nrow"] == 3
    J, aref, D, M, a0 = f["J"], f["aref"], f["D"], f["M"], f["qacc_smooth"]
    A = J @ np.linalg.solve(M, J.T)
    fb = _dual_bruteforce(A, np.diag(1.0 / D), J @ a0 - aref, 0.7)
    scale = max(np.abs(fb).max(), 1.3 * G)
    np.testing.assert_allclose(f["efc_force"], fb, atol=1e-8 * scale)
    np.testing.assert_allclose(f["qacc"], a0 + np.linalg.solve(M, J.T @ fb), atol=1e-8 * (1 + np.abs(f["qacc"]).max()))


def test_newton_converges_quadratically():
    """One Newton iteration from the solution plus eps * r: the error falls with eps^2
    where the cost is smooth (a sliding contact), which needs the exact cone Hessian."""
    m, q, v = _sliding_sphere(0.4, 1)
    o = Oracle(m)
    a = o.forward(q, v, mode=MODE_CONVERGED)["qacc"]
    m1 = _sliding_sphere(0.4, 1)[0]
    m1.opt.iterations = 1
    o1 = Oracle(m1)
    r = np.random.default_rng(1).normal(size=6)
    err = []
    for eps in (1e-2, 1e-3):
        a1 = o1.forward(q, v, a + eps * r, mode=MODE_FIXED)["qacc"]
        err.append(np.abs(a1 - a).max())
    assert err[1] < 2e-2 * err[0] or err[1] < 1e-12 * np.abs(a).max()


def test_frictionless_contacts_are_the_pyramids():
    for cone in (0, 1):
        m = robots.free_body("box", mass=1.0, half=(0.1, 0.2, 0.05), plane=True, condim=1,
                             gravity=(2.0, 0.0, -G), timestep=0.002)
        m.opt.cone = cone
        q = m.qpos0.copy()
        q[2] = 0.049
        f = Oracle(m).forward(q, np.zeros(6), mode=MODE_CONVERGED)
        if cone == 0:
            ref = f
        else:
            np.testing.assert_array_equal(f["qacc"], ref["qacc"])
            np.testing.assert_array_equal(f["efc_force"], ref["efc_force"])
