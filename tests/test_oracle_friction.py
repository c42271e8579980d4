"""Pins of the FP64 reference's friction-loss rows (dry joint friction: a row on the dof
whose force is confined to [-F, F], in the same convex soft-constraint model as the
contacts).  No GPU.

What fixes the answers here, independently of the reference's arithmetic:
* one dof, one row: the minimiser of a scalar quadratic plus a Huber term in closed
  form, on both linear pieces and on the quadratic one;
* Coulomb sliding: a block sliding under gravity accelerates at exactly -g + F/m;
* soft sticking: a block held by friction stronger than its weight creeps at the
  constant velocity where the row's damping force b D |v| balances m g;
* the Newton solution equals the one found by enumerating every row's piece;
* the exact line search equals a dense 1-D search of the cost along the direction;
* mirror symmetry of a planar chain with friction on every joint;
* the cost of each row is the largest admissible row work, max over forces f of
  -f e - f^2 / (2 D), found by a dense search over f.
"""
import itertools

import numpy as np
import pytest

from oracle import MODE_CONVERGED, MODE_FIXED, Oracle
from paper_2502_08844_amd.synth import inputs, robots

from tests.test_oracle_contacts import SOLIMP, SOLREF, impedance

G = 9.81


def _B(m):
    tc = max(SOLREF[0], 2 * m.opt.timestep)
    return 2 / (SOLIMP[1] * tc)


def _huber(e, D, F):
    return np.where(np.abs(D * e) <= F, 0.5 * D * e * e, F * np.abs(e) - F * F / (2 * D))


@pytest.mark.parametrize("mode", [MODE_FIXED, MODE_CONVERGED])
def test_one_dof_friction_closed_form(mode):
    mass, arm = 2.0, 0.1
    Mtot = mass + arm
    B = _B(robots.slider())
    d = impedance(0.0)
    D = d / ((1 - d) * (1 / Mtot))  # A = (M^-1)_kk = 1 / (m + armature)
    a0 = -G * mass / Mtot
    for F in (0.5, 5.0, 50.0):  # slipping down, slipping, sticking
        m = robots.slider(mass=mass, armature=arm, range=None, frictionloss=F)
        o = Oracle(m)
        for v in (-0.4, 0.0, 0.3):
            f = o.forward([0.2], [v], mode=mode)
            assert f["nrow"] == 1 and f["J"][0, 0] == 1.0
            aref = -B * v
            assert f["D"][0] == pytest.approx(D, rel=1e-12)
            assert f["aref"][0] == pytest.approx(aref, rel=1e-12, abs=1e-15)
            # stationarity of Mtot (a - a0) + s'(a - aref) = 0 on each piece
            a_quad = (Mtot * a0 + D * aref) / (Mtot + D)
            if abs(D * (a_quad - aref)) <= F:
                a = a_quad
            elif a_quad > aref:
                a = a0 - F / Mtot
            else:
                a = a0 + F / Mtot
            assert f["qacc"][0] == pytest.approx(a, rel=1e-12, abs=1e-12)
            force = np.clip(D * (aref - a), -F, F)
            assert f["efc_force"][0] == pytest.approx(force, rel=1e-10, abs=1e-12)


def test_coulomb_sliding_acceleration():
    mass, F = 1.5, 4.0  # F < m g: slides
    m = robots.slider(mass=mass, range=None, frictionloss=F, timestep=0.001)
    o = Oracle(m)
    q, v = np.array([[0.0]]), np.array([[-1.0]])  # moving down: friction pushes up
    for _ in range(50):
        f = o.forward(q[0], v[0], mode=MODE_CONVERGED)
        assert f["qacc"][0] == pytest.approx(-G + F / mass, rel=1e-12)
        assert f["efc_force"][0] == pytest.approx(F, rel=1e-12)
        r = o.step(q, v, nstep=1, mode=MODE_CONVERGED)
        q, v = r["qpos"], r["qvel"]
    assert v[0, 0] == pytest.approx(-1.0 + 50 * 0.001 * (-G + F / mass), rel=1e-12)


def test_soft_sticking_creeps_at_balance_velocity():
    mass, F = 1.0, 30.0  # F > m g: held, up to the soft constraint's creep
    m = robots.slider(mass=mass, range=None, frictionloss=F, timestep=0.002)
    o = Oracle(m)
    B = _B(m)
    d = impedance(0.0)
    D = d / ((1 - d) * (1 / mass))
    vstar = -mass * G / (B * D)
    r = o.step(np.array([[0.0]]), np.zeros((1, 1)), nstep=4000, mode=MODE_CONVERGED)
    assert r["qvel"][0, 0] == pytest.approx(vstar, rel=1e-9)
    f = o.forward(r["qpos"][0], r["qvel"][0], mode=MODE_CONVERGED)
    assert abs(f["qacc"][0]) < 1e-9
    assert f["efc_force"][0] == pytest.approx(mass * G, rel=1e-9)


def _pieces_solution(M, a0, J, aref, D, fl):
    """Enumerate every row's piece (one-sided: inactive/active; friction: -F, quadratic,
    +F), solve each linear system, keep the consistent assignments."""
    nr = len(aref)
    choices = [(0, 1) if fl[r] == 0 else (-1, 0, 1) for r in range(nr)]
    sols = []
    for pick in itertools.product(*choices):
        H, rhs = M.copy(), M @ a0
        for r, c in enumerate(pick):
            if fl[r] == 0:
                if c == 1:
                    H += D[r] * np.outer(J[r], J[r]); rhs += D[r] * aref[r] * J[r]
            elif c == 0:
                H += D[r] * np.outer(J[r], J[r]); rhs += D[r] * aref[r] * J[r]
            else:
                rhs -= c * fl[r] * J[r]  # s' = +-F on a linear piece
        a = np.linalg.solve(H, rhs)
        e = J @ a - aref
        ok = True
        for r, c in enumerate(pick):
            tol = 1e-10 * (1 + abs(aref[r]))
            if fl[r] == 0:
                ok &= (e[r] <= tol) if c == 1 else (e[r] >= -tol)
            elif c == 0:
                ok &= abs(D[r] * e[r]) <= fl[r] * (1 + 1e-10)
            else:
                ok &= c * D[r] * e[r] >= fl[r] * (1 - 1e-10)
        if ok:
            sols.append(a)
    return sols


@pytest.mark.parametrize("seed", range(3))
def test_newton_equals_piece_enumeration(seed):
    m = robots.hinge_chain(n=3, slide_root=True, damping=0.1, limit=0.25, frictionloss=0.8)
    o = Oracle(m)
    rng = np.random.default_rng(seed)
    q = rng.uniform(-0.35, 0.35, size=m.nq)
    v = rng.normal(size=m.nv)
    f = o.forward(q, v, mode=MODE_CONVERGED)
    nl = f["nrow"] - m.nfric
    assert m.nfric == 4 and nl >= 1
    fl = np.r_[np.zeros(nl), np.full(m.nfric, 0.8)]
    sols = _pieces_solution(f["M"], f["qacc_smooth"], f["J"], f["aref"], f["D"], fl)
    assert len(sols) >= 1
    for s in sols[1:]:
        assert np.allclose(s, sols[0], atol=1e-9)
    assert np.max(np.abs(f["qacc"] - sols[0])) < 1e-10 * (1 + np.abs(sols[0]).max())
    # friction rows: J = e_k, forces inside their bounds
    Jf = f["J"][nl:]
    assert np.array_equal(Jf, np.eye(m.nv))
    assert np.all(np.abs(f["efc_force"][nl:]) <= 0.8 * (1 + 1e-12))


def test_line_search_exact_with_friction_rows():
    """One Newton iteration lands on the exact minimiser of the cost along the Newton
    direction (dense 1-D search), with friction rows on both linear pieces."""
    for seed in (1, 2, 3):
        rng = np.random.default_rng(seed)
        m = robots.hinge_chain(n=3, slide_root=True, limit=0.25, frictionloss=0.5)
        m.opt.iterations = 1
        o = Oracle(m)
        q = rng.uniform(-0.35, 0.35, size=m.nq)
        v = rng.normal(size=m.nv)
        ws = rng.normal(scale=5.0, size=m.nv)
        f0 = o.forward(q, v, qacc_ws=ws)
        M, a0, J, aref, D = f0["M"], f0["qacc_smooth"], f0["J"], f0["aref"], f0["D"]
        nl = f0["nrow"] - m.nfric
        fl = np.r_[np.zeros(nl), np.full(m.nfric, 0.5)]

        def cost(a):
            e = J @ a - aref
            one = np.where(fl == 0, 0.5 * D * np.minimum(e, 0) ** 2, 0.0)
            return (0.5 * (a - a0) @ M @ (a - a0) + one.sum()
                    + np.sum(np.where(fl > 0, _huber(e, D, np.maximum(fl, 1e-300)), 0.0)))
        start = ws if cost(ws) <= cost(a0) else a0
        e = J @ start - aref
        quad = np.where(fl == 0, e < 0, np.abs(D * e) < fl)
        ds = np.where(fl == 0, D * np.minimum(e, 0), np.clip(D * e, -fl, fl))
        g = M @ (start - a0) + J.T @ ds
        H = M + (J[quad].T * D[quad]) @ J[quad]
        delta = -np.linalg.solve(H, g)
        al = np.linspace(0, 3, 30001)
        vals = np.array([cost(start + x * delta) for x in al])
        k = int(np.argmin(vals))
        lo, hi = al[max(k - 1, 0)], al[min(k + 1, len(al) - 1)]
        for _ in range(100):
            x1, x2 = lo + 0.382 * (hi - lo), lo + 0.618 * (hi - lo)
            if cost(start + x1 * delta) < cost(start + x2 * delta):
                hi = x2
            else:
                lo = x1
        a_ref = start + 0.5 * (lo + hi) * delta
        assert np.max(np.abs(f0["qacc"] - a_ref)) < 1e-6 * (1 + np.abs(a_ref).max())


def test_mirror_symmetry_with_friction():
    m = robots.hinge_chain(n=4, damping=0.1, limit=0.3, frictionloss=0.4)
    m.opt.gravity = (0.0, 0.0, 0.0)
    o = Oracle(m)
    rng = np.random.default_rng(8)
    for _ in range(5):
        q = rng.uniform(-0.4, 0.4, size=m.nq)
        v = rng.normal(size=m.nv)
        f1 = o.forward(q, v, mode=MODE_CONVERGED)
        f2 = o.forward(-q, -v, mode=MODE_CONVERGED)
        np.testing.assert_allclose(f2["qacc"], -f1["qacc"], rtol=1e-10, atol=1e-10)
        nr = f1["nrow"]
        np.testing.assert_allclose(f2["efc_force"][nr - m.nfric:],
                                   -f1["efc_force"][nr - m.nfric:], rtol=1e-9, atol=1e-9)


def test_friction_workload_sticks_and_slips():
    """The quadruped_friction inputs put rows on every piece."""
    m = robots.quadruped_friction()
    o = Oracle(m)
    qp, qv = inputs.initial_state("quadruped_friction", m, 8, seed=0)
    u = inputs.controls("quadruped_friction", m, 8, 30, seed=0)
    r = o.step(qp, qv, None, u[:29], nstep=29)
    F = robots.QUAD_FRICTIONLOSS
    stick = slip = 0
    for w in range(8):
        f = o.forward(r["qpos"][w], r["qvel"][w], r["qacc_ws"][w], u[29, w])
        fr = f["efc_force"][f["nrow"] - 12:]
        slip += int(np.sum(np.abs(np.abs(fr) - F) < 1e-9))
        stick += int(np.sum(np.abs(fr) < F * (1 - 1e-6)))
    assert stick >= 4 and slip >= 4


def test_cost_is_the_largest_admissible_row_work():
    """Each row's cost term is max over its admissible forces f of -f e - f^2 / (2 D)
    (f >= 0 one-sided, |f| <= F friction), evaluated here by a dense search over f."""
    m = robots.hinge_chain(n=3, slide_root=True, limit=0.25, frictionloss=0.6)
    o = Oracle(m)
    rng = np.random.default_rng(4)
    q = rng.uniform(-0.35, 0.35, size=m.nq)
    v = rng.normal(size=m.nv)
    f = o.forward(q, v)
    M, a0, J, aref, D = f["M"], f["qacc_smooth"], f["J"], f["aref"], f["D"]
    nl = f["nrow"] - m.nfric
    for _ in range(5):
        a = a0 + rng.normal(scale=30.0, size=m.nv)
        e = J @ a - aref
        tot = 0.5 * (a - a0) @ M @ (a - a0)
        for r in range(f["nrow"]):
            fs = np.linspace(0.0, 50.0 * (1 + abs(D[r] * e[r])), 200001) if r < nl else \
                np.linspace(-0.6, 0.6, 200001)
            w = -fs * e[r] - fs * fs / (2 * D[r])
            k = int(np.argmax(w))
            tot += w[k]
        assert o.cost(q, v, None, a) == pytest.approx(tot, rel=1e-8, abs=1e-9)
