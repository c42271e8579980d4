"""The reference's capsule-box contacts are exact: they do not depend on its two
tolerances, and they match closed forms (no GPU).

Along the capsule's segment p(t) = a + t u the box's signed distance f(t) is convex and
piecewise smooth.  The reference takes the minimiser set of f from the exact piecewise
analysis (breakpoints where a box-frame coordinate crosses -h, 0 or h or, inside the
box, where two face distances are equal; closed-form minimisers of the outside pieces,
where f^2 is quadratic).  Its two tolerances only absorb rounding: the allowance within
which two values of f count as equal (relative to the segment's scale) and the distance
within which two candidates count as one.  Checked:
* contacts under allowances 1e-10 and 1e-14 and de-duplication distances 1e-7 and 1e-5
  equal the defaults' (1e-12, 1e-6) on the configurations of the capsule-box sampling
  tests, the capsules lying on and overhanging a face, and passes beside an edge;
* a capsule crossing a box edge outside the box touches it where the segment is closest
  to the edge line (closed form);
* a capsule lying on a face and overhanging it: the flat stretch ends exactly at the
  edge, where the normal is still the face's.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2502_08844_amd.synth import robots
from tests.test_oracle_contacts import _contacts, quat_axis, two_body_qpos

DEFAULT = (1e-12, 1e-6)
VARIANTS = [(1e-10, 1e-6), (1e-14, 1e-6), (1e-12, 1e-7), (1e-12, 1e-5)]


@pytest.fixture
def tolerances():
    prev = oracle.set_capsule_box_tolerances(*DEFAULT)
    assert prev == DEFAULT
    yield
    oracle.set_capsule_box_tolerances(*DEFAULT)


def _configs():
    """(model, qpos) of the sampling tests' capsule-box configurations, the lying and
    edge-overhanging capsules and the rounded-edge passes."""
    out = []
    half = (0.05, 0.07, 0.03)
    m = robots.two_bodies("capsule", "box", (0.02, 0.06), half)
    for seed in range(3):
        rng = np.random.default_rng(100 + seed)
        qb = rng.normal(size=4)
        qb /= np.linalg.norm(qb)
        for _ in range(3):  # the sphere trials' draws come first in the sampling test
            rng.normal(size=3), rng.uniform(0.02, 0.09)
        for _ in range(3):
            qc = rng.normal(size=4)
            qc /= np.linalg.norm(qc)
            pc = rng.normal(size=3)
            pc *= rng.uniform(0.02, 0.08) / np.linalg.norm(pc)
            out.append((m, two_body_qpos(pc, qc, np.zeros(3), qb)))
    m2 = robots.two_bodies("capsule", "box", (0.01, 0.04), (0.1, 0.1, 0.03))
    q = quat_axis((0, 1, 0), math.pi / 2)
    out.append((m2, two_body_qpos([0.0, 0.0, 0.039], q, [0, 0, 0], [1, 0, 0, 0])))
    out.append((m2, two_body_qpos([0.1, 0.0, 0.039], q, [0, 0, 0], [1, 0, 0, 0])))
    m3 = robots.two_bodies("capsule", "box", (0.01, 0.04), (0.05, 0.05, 0.05))
    rng = np.random.default_rng(9)
    for _ in range(20):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        q3 = np.array(robots.quat_z_to(d))
        corner = np.array([0.05, 0.05, rng.uniform(-0.03, 0.03)])
        center = corner + np.array([1.0, 1.0, 0.0]) / np.sqrt(2) * 0.008 + \
            d * rng.uniform(-0.02, 0.02)
        out.append((m3, two_body_qpos(center, q3, [0, 0, 0], [1, 0, 0, 0])))
    return out


def test_contacts_do_not_depend_on_the_tolerances(tolerances):
    configs = _configs()
    base = [_contacts(m, q) for m, q in configs]
    assert sum(len(c) for c in base) >= 20  # penetrating cases are among them
    worst = 0.0
    for eq, dup in VARIANTS:
        oracle.set_capsule_box_tolerances(eq, dup)
        for (m, q), c0 in zip(configs, base):
            c = _contacts(m, q)
            assert c.shape == c0.shape
            # depth, point and normal; the candidate index may not change either
            np.testing.assert_array_equal(c[:, 17], c0[:, 17])
            dev = np.abs(c[:, :7] - c0[:, :7]).max() if len(c) else 0.0
            worst = max(worst, dev)
            assert dev <= 1e-15, (eq, dup, dev)
    oracle.set_capsule_box_tolerances(*DEFAULT)
    print(f"[oracle] capsule-box contacts across tolerance variants: max deviation {worst:.1e}")


@pytest.mark.parametrize("eq,dup", [DEFAULT] + VARIANTS)
def test_capsule_across_a_box_edge_closed_form(tolerances, eq, dup):
    """A capsule in the xz-plane passing over the box's edge x = z = 0.05 (along y),
    outside the box, 2 mm into its rounded surface: the contact is at the segment's
    closest point to the edge line."""
    oracle.set_capsule_box_tolerances(eq, dup)
    half, r, hl = (0.05, 0.05, 0.05), 0.01, 0.04
    m = robots.two_bodies("capsule", "box", (r, hl), half)
    edge = np.array([0.05, 0.0, 0.05])
    for ang in (0.3, 0.7, 1.1):
        d = np.array([math.cos(ang), 0.0, -math.sin(ang)])      # the capsule's axis
        nrm = np.array([math.sin(ang), 0.0, math.cos(ang)])     # unit, normal to d in xz
        closest = edge + (r - 0.002) * nrm                      # 2 mm inside the surface
        center = closest + 0.01 * d                             # off the capsule's centre
        q = np.array(robots.quat_z_to(d))
        c = _contacts(m, two_body_qpos(center, q, [0, 0, 0], [1, 0, 0, 0]))
        assert len(c) == 1
        assert c[0, 0] == pytest.approx(-0.002, abs=1e-12)
        np.testing.assert_allclose(c[0, 4:7], -nrm, atol=1e-9)
        # midway between the box's surface (the edge) and the capsule's (2 mm past it)
        np.testing.assert_allclose(c[0, 1:4], edge - 0.5 * 0.002 * nrm, atol=1e-9)


def test_flat_stretch_ends_at_the_edge(tolerances):
    """A capsule along x lying 1 mm into the top face and reaching past its edge at
    x = 0.1: its contacts are the inner end (x = 0.06) and the edge itself, both with the
    face's normal and 1 mm deep."""
    m = robots.two_bodies("capsule", "box", (0.01, 0.04), (0.1, 0.1, 0.03))
    q = quat_axis((0, 1, 0), math.pi / 2)
    c = _contacts(m, two_body_qpos([0.1, 0.0, 0.039], q, [0, 0, 0], [1, 0, 0, 0]))
    assert len(c) == 2
    c = c[np.argsort(c[:, 1])]
    np.testing.assert_allclose(c[:, 1], [0.06, 0.1], atol=1e-15)
    np.testing.assert_allclose(c[:, 0], [-0.001, -0.001], atol=1e-15)
    np.testing.assert_array_equal(c[:, 4:7], [[0.0, 0.0, -1.0]] * 2)
