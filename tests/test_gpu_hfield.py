"""GPU parity of sphere-heightfield contacts against the FP64 reference.

Workloads: the quadruped on Perlin-noise rough terrain (feet against a 128 x 128
heightfield) at 16/32/64-lane teams and at full size, and free spheres dropped on a
rotated, shifted Perlin heightfield.  Same tolerances as the other parity tests:
qacc <= 1e-4 and contact forces <= 1e-3 per world, states at a switch reported.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2502_08844_amd.synth import inputs, robots
from tests.gpu_util import compare_step, gpu_ctx, run_gpu, summarize, teacher_forced

pytestmark = pytest.mark.gpu

QACC_TOL = 1e-4
FORCE_TOL = 1e-3


@pytest.fixture(scope="module")
def lib():
    return gpu_ctx()


def _check(kind, stats, min_contacts=1):
    ea, ef, nflag, ntot = summarize(kind, stats)
    assert ea.max() <= QACC_TOL
    assert ef.size >= min_contacts
    assert ef.max() <= FORCE_TOL
    assert nflag <= max(1, 0.02 * ntot)


def test_single_step_parity_quadruped_rough(lib):
    mjh, ctx = lib
    print("[gpu] parity quadruped_rough nw=203", flush=True)
    m, stats = teacher_forced(ctx, mjh, "quadruped_rough", 203, [0, 5, 50, 150])
    geo = np.concatenate([s["err_geo"] for s in stats])
    print(f"[gpu] rough-terrain contact geometry: |d dist| max {geo[:, 0].max():.1e} "
          f"|d pos| max {geo[:, 1].max():.1e} |d normal| max {geo[:, 2].max():.1e}", flush=True)
    assert geo[:, 0].max() < 1e-5 and geo[:, 2].max() < 5e-4
    _check("quadruped_rough", stats, min_contacts=100)


@pytest.mark.parametrize("team,block", [(16, 64), (64, 64)])
def test_rough_parity_launch_shapes(lib, team, block):
    mjh, ctx = lib
    m, stats = teacher_forced(ctx, mjh, "quadruped_rough", 77, [0, 3, 40], seed=2,
                              team=team, block=block)
    _check(f"quadruped_rough-T{team}", stats)


def test_spheres_on_rotated_terrain(lib):
    """Spheres within 0.4 m of the origin: spatial inertias are kept at the world
    origin, so FP32 rounds a small sphere's rotational inertia (0.002 kg m^2 here) at
    the scale m |x|^2, which at |x| ~ 1 m costs it about 5e-5 of its value."""
    mjh, ctx = lib
    data = robots.perlin_terrain(32, cells=4, seed=9)
    m = robots.sphere_on_hfield(data, size=(1.0, 1.0, 0.15), radius=0.07,
                                hpos=(0.2, -0.1, 0.05),
                                hquat=robots.axis_angle_quat((0.2, 0.1, 1.0), 0.4))
    o = oracle.Oracle(m)
    nw = 128
    rng = np.random.default_rng(4)
    qp = np.tile(m.qpos0, (nw, 1))
    Rg = robots.quat_to_mat(robots.axis_angle_quat((0.2, 0.1, 1.0), 0.4))
    for w in range(nw):
        xy = rng.uniform(-0.4, 0.4, size=2)
        j = int((xy[0] + 1) / (2 / 31)); i = int((xy[1] + 1) / (2 / 31))
        loc = np.r_[xy, 0.15 * data[i, j] + rng.uniform(0.0, 0.1)]
        qp[w, :3] = Rg @ loc + np.array([0.2, -0.1, 0.05])
    qp, qv = inputs.f32(qp), inputs.f32(rng.normal(scale=0.3, size=(nw, 6)))
    stats = []
    ws = np.zeros((nw, 6))
    for t in range(3):
        g1 = run_gpu(ctx, mjh, m, qp, qv, ws, None, 1, contacts=True)
        cmp = compare_step(m, o, (qp, qv, ws), None, g1)
        cmp["t"], cmp["ncon"] = t, g1["ncon"]
        stats.append(cmp)
        r = run_gpu(ctx, mjh, m, qp, qv, ws, None, 30, contacts=False)
        qp, qv, ws = r["qpos"], r["qvel"], r["qacc"]
    geo = np.concatenate([s["err_geo"] for s in stats])
    print(f"[gpu] terrain contact geometry: |d dist| max {geo[:, 0].max():.1e} "
          f"|d pos| max {geo[:, 1].max():.1e} |d normal| max {geo[:, 2].max():.1e}", flush=True)
    assert geo[:, 0].max() < 1e-5 and geo[:, 2].max() < 5e-4
    _check("spheres_on_terrain", stats, min_contacts=50)


def test_full_size_quadruped_rough(lib):
    mjh, ctx = lib
    from tests.gpu_util import workload
    from tests.test_gpu_fullsize import _check as full_check, _one_step, _sample, _state
    nw, nstep = 8192, 60
    print(f"[gpu] full-size parity quadruped_rough nw={nw} steps={nstep}", flush=True)
    m, qp, qv, u = workload("quadruped_rough", nw, nstep + 1, seed=7)
    w = mjh.World(ctx, m, nw, qpos=qp, qvel=qv)
    w.batch.set_launch(0, 32, 128)
    ut = torch.tensor(u, dtype=torch.float32, device="cuda")
    w.step(ut[:nstep])
    torch.cuda.synchronize()
    assert np.all(w.status.cpu().numpy() & 1 == 0)
    state = _state(w)
    gpu1 = _one_step(w, mjh, ut[nstep:nstep + 1].contiguous())
    full_check("quadruped_rough-full", m, state, u[nstep:nstep + 1], gpu1, _sample(nw))
