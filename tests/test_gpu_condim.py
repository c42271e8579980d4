"""GPU parity of frictionless contacts (pair condim 1) against the FP64 reference.

The GPU keeps four rows per contact: a frictionless contact's are four identical normal
rows with four times the single row's regulariser each, whose costs sum to the
reference's single row; accelerations and the total normal force are compared.

* the quadruped on frictionless ground at 32-, 16- and 64-lane teams (tolerances of the
  other parity tests);
* a box on a plane tilted by 0.4 rad accelerates down the slope at g sin(theta), with
  no tangential contact force;
* rollouts reject frictionless pairs.
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
    assert nflag <= 0.25 * ntot
    for s in stats:
        gc = s["gpu_contacts"]
        assert np.abs(gc[:, :, 14:16]).max() == 0


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


def test_rollout_rejects_frictionless(lib):
    mjh, ctx = lib
    m = robots.quadruped_frictionless()
    w = mjh.World(ctx, m, 2)
    u = torch.zeros(4, 2, m.nu, device="cuda")
    loss = torch.zeros(2, device="cuda")
    with pytest.raises(mjh.MjhError):
        w.batch.rollout_fwd(4, 2, u, 2, 0.3, 1e-3, loss)
