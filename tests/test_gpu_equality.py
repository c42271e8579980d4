"""GPU parity of equality rows against the FP64 reference: connect (three two-sided rows
holding a point of one body on a point of another body or of the world) and weld (those
three plus three rotational rows holding the relative orientation).

Workloads: the parallelogram linkage (a closed loop of hinges, 16-lane teams), a capsule
pinned at one end (a free body), two free spheres held centre to centre, and the
quadruped with its torso tethered to its standing position beside the foot contacts;
welds: a box welded to the world off its centre (a cantilever), two free boxes welded
to each other, and the quadruped with its torso welded to the world (a fixed base).
Same tolerances as the other parity tests.  The rollouts' gradients with equalities are
in `tests/test_gpu_adjoint_self.py`.
"""
import numpy as np
import pytest

import oracle
from paper_2502_08844_amd.synth import inputs, robots
from tests.gpu_util import compare_step, gpu_ctx, run_gpu, summarize, teacher_forced

pytestmark = pytest.mark.gpu

QACC_TOL = 1e-4
FORCE_TOL = 1e-3


@pytest.fixture(scope="module")
def lib():
    return gpu_ctx()


def _check(kind, stats):
    ea, ef, nflag, ntot = summarize(kind, stats)
    assert ea.max() <= QACC_TOL
    if ef.size:
        assert ef.max() <= FORCE_TOL
    assert nflag <= max(1, 0.02 * ntot)


def _states(m, nw, rng):
    if m.name.startswith("welded"):  # near the welded pose: 1 mm and 0.05 rad off
        q = np.tile(m.qpos0, (nw, 1))
        for b in range(m.nq // 7):
            q[:, 7 * b:7 * b + 3] += rng.normal(scale=1e-3, size=(nw, 3))
            for w in range(nw):
                dq = robots.axis_angle_quat(rng.normal(size=3), rng.uniform(0, 0.05))
                R = robots.quat_to_mat(m.qpos0[7 * b + 3:7 * b + 7]) @ robots.quat_to_mat(dq)
                q[w, 7 * b + 3:7 * b + 7] = robots.mat_to_quat(R)
        return inputs.f32(q), inputs.f32(rng.normal(scale=0.5, size=(nw, m.nv)))
    if m.name == "four_bar":
        q = rng.uniform(-0.5, 0.5, size=(nw, 3))
        q[:, 1] = -q[:, 0] + rng.normal(scale=1e-3, size=nw)  # near the closed loop
        q[:, 2] = q[:, 0] + rng.normal(scale=1e-3, size=nw)
        return inputs.f32(q), inputs.f32(rng.normal(scale=0.5, size=(nw, m.nv)))
    q = np.tile(m.qpos0, (nw, 1))
    nfree = m.nq // 7
    for b in range(nfree):
        q[:, 7 * b:7 * b + 3] += rng.normal(scale=1e-3, size=(nw, 3))
        for w in range(nw):
            q[w, 7 * b + 3:7 * b + 7] = robots.axis_angle_quat(rng.normal(size=3),
                                                               rng.uniform(0, 0.5))
    return inputs.f32(q), inputs.f32(rng.normal(scale=0.5, size=(nw, m.nv)))


@pytest.mark.parametrize("name", ["four_bar", "pinned_sphere", "pinned_capsule",
                                  "connected_spheres", "four_bar_friction", "welded_box",
                                  "welded_pair"])
def test_equality_parity_small_models(lib, name):
    """The pinned bodies hang 0.3 m above the origin, the quadruped torso's height.
    Spatial inertias and motion subspaces are kept at the world origin, so FP32 rounds
    a body's rotational inertia at the scale m |x|^2: a capsule's axial inertia (500
    times below its transverse one) pinned 1.2 m up has 2e-4 relative error, beyond
    the tolerance."""
    mjh, ctx = lib
    m = {"four_bar": lambda: robots.four_bar(damping=0.02),
         "pinned_sphere": lambda: robots.pinned_body("sphere", anchor=(0, 0, 0.15), z0=0.3),
         "pinned_capsule": lambda: robots.pinned_body("capsule", anchor=(0, 0, 0.2), z0=0.3),
         "connected_spheres": lambda: robots.connected_spheres(1.0, 3.0),
         "four_bar_friction": lambda: robots.four_bar(frictionloss=0.05),
         "welded_box": lambda: robots.welded_box(anchor=(-0.08, 0.02, 0.3)),
         "welded_pair": lambda: robots.welded_pair(gravity=(0, 0, -9.81))}[name]()
    gm = ctx.model_upload(m)
    assert gm.neq == 1 and gm.nrowmax == m.nrowmax
    nw = 96
    rng = np.random.default_rng(3)
    qp, qv = _states(m, nw, rng)
    o = oracle.Oracle(m)
    stats = []
    ws = np.zeros((nw, m.nv))
    print(f"[gpu] parity {name} nw={nw}", flush=True)
    for t in range(3):
        g1 = run_gpu(ctx, mjh, m, qp, qv, ws, None, 1, contacts=True)
        cmp = compare_step(m, o, (qp, qv, ws), None, g1)
        cmp["t"], cmp["ncon"] = t, g1["ncon"]
        stats.append(cmp)
        r = run_gpu(ctx, mjh, m, qp, qv, ws, None, 40, contacts=False)
        qp, qv, ws = r["qpos"], r["qvel"], r["qacc"]
    assert np.all(r["status"] & 1 == 0)
    _check(name, stats)


def test_parallelogram_stays_closed_on_gpu(lib):
    mjh, ctx = lib
    m = robots.four_bar()
    qp = np.tile(np.array([0.3, -0.3, 0.3]), (64, 1))
    r = run_gpu(ctx, mjh, m, qp, np.zeros((64, 3)), None, None, 2000, contacts=False)
    q = r["qpos"]
    assert np.abs(q[:, 0] + q[:, 1]).max() < 2e-3
    assert np.abs(q[:, 2] - q[:, 0]).max() < 2e-3


def test_single_step_parity_quadruped_tethered(lib):
    mjh, ctx = lib
    print("[gpu] parity quadruped_tethered nw=203", flush=True)
    m, stats = teacher_forced(ctx, mjh, "quadruped_tethered", 203, [0, 5, 50, 150])
    _check("quadruped_tethered", stats)


def test_single_step_parity_quadruped_welded(lib):
    mjh, ctx = lib
    print("[gpu] parity quadruped_welded nw=203", flush=True)
    m, stats = teacher_forced(ctx, mjh, "quadruped_welded", 203, [0, 5, 50, 150])
    _check("quadruped_welded", stats)


@pytest.mark.parametrize("team,block", [(16, 64), (64, 64)])
def test_welded_parity_launch_shapes(lib, team, block):
    mjh, ctx = lib
    m, stats = teacher_forced(ctx, mjh, "quadruped_welded", 77, [0, 3, 40], seed=2,
                              team=team, block=block)
    _check(f"quadruped_welded-T{team}", stats)


@pytest.mark.parametrize("team,block", [(16, 64), (64, 64)])
def test_tethered_parity_launch_shapes(lib, team, block):
    mjh, ctx = lib
    m, stats = teacher_forced(ctx, mjh, "quadruped_tethered", 77, [0, 3, 40], seed=2,
                              team=team, block=block)
    _check(f"quadruped_tethered-T{team}", stats)

