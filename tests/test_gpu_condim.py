"""GPU parity of the contact dimensions against the FP64 reference: frictionless
contacts (condim 1, one row), torsional friction (condim 4, six pyramid edges) and
rolling friction (condim 6, ten edges).

* the quadruped on frictionless ground at 32-, 16- and 64-lane teams (tolerances of the
  other parity tests);
* a box on a plane tilted by 0.4 rad accelerates down the slope at g sin(theta), with
  no tangential contact force;
* the quadruped with torsional / rolling friction at the feet (condim 4 / 6) at the
  usual tolerances (qacc 1e-4, contact force 1e-3 relative to m g) in every world not
  at a switch;
* spinning spheres on a plane with torsional friction (one step from many states);
* the rollouts' gradients for every contact dimension are in
  `tests/test_gpu_adjoint_self.py`.
"""
import math

import numpy as np
import pytest
import torch

from paper_2502_08844_amd.synth import robots
from tests.gpu_util import gpu_ctx, run_gpu, summarize, teacher_forced

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    return gpu_ctx()


@pytest.mark.parametrize("team,block", [(None, None), (16, 64), (64, 64)])
def test_frictionless_quadruped_parity(lib, team, block):
    mjh, ctx = lib
    print(f"[gpu] parity quadruped_frictionless team={team}", flush=True)
    m, stats = teacher_forced(ctx, mjh, "quadruped_frictionless", 203 if team is None else 77,
                              [0, 5, 50], seed=3, team=team, block=block)
    ea, ef, nflag, ntot = summarize(f"quadruped_frictionless-T{team}", stats)
    assert ea.max() <= 1e-4 and ef.size > 0 and ef.max() <= 1e-3
    assert nflag <= max(1, 0.02 * ntot)
    for s in stats:
        gc = s["gpu_contacts"]
        assert np.abs(gc[:, :, 14:16]).max() == 0


@pytest.mark.parametrize("kind,team,block", [("quadruped_torsion", None, None),
                                             ("quadruped_torsion", 16, 64),
                                             ("quadruped_rolling", None, None),
                                             ("quadruped_rolling", 64, 64)])
def test_torsion_rolling_quadruped_parity(lib, kind, team, block):
    mjh, ctx = lib
    print(f"[gpu] parity {kind} team={team}", flush=True)
    m, stats = teacher_forced(ctx, mjh, kind, 203 if team is None else 77, [0, 5, 50],
                              seed=4, team=team, block=block)
    ea, ef, nflag, ntot = summarize(f"{kind}-T{team}", stats)
    assert ea.max() <= 1e-4
    assert ef.size > 0 and ef.max() <= 1e-3
    assert nflag <= max(1, 0.02 * ntot)


def test_spinning_spheres_torsion(lib):
    import oracle
    from tests.gpu_util import compare_step
    mjh, ctx = lib
    m = robots.free_body("sphere", mass=3.0, half=(0.1, 0, 0), plane=True, condim=6,
                         mu_torsion=0.02, mu_rolling=0.002, timestep=0.002)
    nw = 64
    rng = np.random.default_rng(2)
    qp = np.tile(m.qpos0, (nw, 1))
    qp[:, 2] = 0.1 - rng.uniform(0, 2e-3, nw)
    qv = np.zeros((nw, 6))
    qv[:, 5] = rng.uniform(-3, 3, nw)
    qv[:, 0:2] = rng.normal(scale=0.3, size=(nw, 2))
    qv[:, 3:5] = rng.normal(scale=3.0, size=(nw, 2))
    from paper_2502_08844_amd.synth import inputs
    qp, qv = inputs.f32(qp), inputs.f32(qv)
    g1 = run_gpu(ctx, mjh, m, qp, qv, np.zeros((nw, 6)), None, 1, contacts=True)
    cmp = compare_step(m, oracle.Oracle(m), (qp, qv, np.zeros((nw, 6))), None, g1)
    ok = ~cmp["flag"]
    print(f"[gpu] spinning spheres condim 6: qacc max {cmp['err_a'][ok].max():.2e} "
          f"force max {cmp['err_f'][ok].max():.2e}, flagged {int(cmp['flag'].sum())}",
          flush=True)
    assert cmp["err_a"][ok].max() <= 1e-4 and cmp["err_f"][ok].max() <= 1e-3
    assert cmp["flag"].sum() <= 0.02 * nw


def test_frictionless_box_on_incline(lib):
    mjh, ctx = lib
    th = 0.4
    grav = (9.81 * math.sin(th), 0.0, -9.81 * math.cos(th))
    m = robots.free_body("box", mass=1.0, half=(0.1, 0.2, 0.05), plane=True, condim=1,
                         gravity=grav, timestep=0.002)
    q0 = np.tile(m.qpos0, (32, 1))
    q0[:, 2] = 0.05
    r = run_gpu(ctx, mjh, m, q0, np.zeros((32, 6)), None, None, 200, contacts=True)
    assert np.all(r["ncon"] == 4)
    np.testing.assert_allclose(r["qacc"][:, 0], 9.81 * math.sin(th), rtol=1e-6)
    assert np.abs(r["contacts"][:, :4, 14:16]).max() == 0
    np.testing.assert_allclose(r["contacts"][:, :4, 13].sum(1), 9.81 * math.cos(th), rtol=1e-3)

