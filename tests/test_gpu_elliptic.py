"""GPU parity of elliptic friction cones (model option cone = 1) against the FP64
reference, at the tolerances of the other parity tests (qacc 1e-4, contact forces 1e-3
of the total weight, in every world not at a switch; a cone at the border of its zones
counts as one):

* the quadruped (condim 3) at 32-, 16- and 64-lane teams, and with sliding, torsional
  and rolling friction (condim 6: six frame rows a contact);
* the humanoid and the hand with elliptic cones;
* 8192 elliptic quadrupeds in the benchmark's launch (sampled worlds);
* a sphere sliding in seven directions: its friction turns with the slip at constant
  magnitude, on the cone's surface (|f_t| = mu f_n);
* a batch mixing pyramid and elliptic models matches the models stepped alone;
* rollouts and env steps reject elliptic models.
"""
import math

import numpy as np
import pytest
import torch

from paper_2502_08844_amd.synth import inputs, robots
from tests.gpu_util import gpu_ctx, run_gpu, summarize, teacher_forced

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    return gpu_ctx()


def _gate(kind, stats):
    ea, ef, nflag, ntot = summarize(kind, stats)
    assert ea.max() <= 1e-4
    assert ef.size == 0 or ef.max() <= 1e-3
    assert nflag <= max(1, 0.02 * ntot)


@pytest.mark.parametrize("kind,team,block,nw", [("quadruped_elliptic", None, None, 203),
                                                ("quadruped_elliptic", 16, 64, 77),
                                                ("quadruped_elliptic", 64, 64, 77),
                                                ("quadruped_elliptic_rolling", None, None, 203),
                                                ("humanoid_elliptic", None, None, 67),
                                                ("hand_elliptic", None, None, 67)])
def test_elliptic_parity(lib, kind, team, block, nw):
    mjh, ctx = lib
    print(f"[gpu] parity {kind} team={team} nw={nw}", flush=True)
    m, stats = teacher_forced(ctx, mjh, kind, nw, [0, 5, 50], seed=6, team=team, block=block)
    for s in stats:
        assert np.all(s["status"] & 1 == 0)
    _gate(f"{kind}-T{team}", stats)


def test_full_size_quadruped_elliptic(lib):
    mjh, ctx = lib
    from tests.gpu_util import workload
    from tests.test_gpu_fullsize import _check, _one_step, _sample, _state
    nw, nstep = 8192, 60
    print(f"[gpu] full-size parity quadruped_elliptic nw={nw} steps={nstep}", flush=True)
    m, qp, qv, u = workload("quadruped_elliptic", nw, nstep + 1, seed=2)
    w = mjh.World(ctx, m, nw, qpos=qp, qvel=qv)
    w.batch.set_launch(0, 32, 128)
    ut = torch.tensor(u, dtype=torch.float32, device="cuda")
    w.step(ut[:nstep])
    torch.cuda.synchronize()
    state = _state(w)
    g1 = _one_step(w, mjh, ut[nstep:nstep + 1].contiguous())
    assert np.all(w.status.cpu().numpy() & 1 == 0)
    _check("quadruped_elliptic-full", m, state, u[nstep:nstep + 1], g1, _sample(nw))


def test_friction_turns_with_the_slip(lib):
    mjh, ctx = lib
    m = robots.free_body("sphere", mass=2.0, half=(0.1, 0, 0), z0=0.1, plane=True, mu=0.5,
                         timestep=0.002)
    m.opt.cone = 1
    angles = np.linspace(0.0, math.pi / 2, 7)
    qp = np.tile(m.qpos0, (len(angles), 1))
    qp[:, 2] = 0.1 - 1e-3
    qv = np.zeros((len(angles), 6))
    qv[:, 0], qv[:, 1] = 0.8 * np.cos(angles), 0.8 * np.sin(angles)
    qp, qv = inputs.f32(qp), inputs.f32(qv)
    r = run_gpu(ctx, mjh, m, qp, qv, np.zeros_like(qv), None, 1, contacts=True)
    assert np.all(r["ncon"] == 1)
    c = r["contacts"][:, 0]
    ft = c[:, 14:15] * c[:, 7:10] + c[:, 15:16] * c[:, 10:13]
    mag = np.linalg.norm(ft, axis=1)
    print(f"[gpu] elliptic friction over slip directions: |f_t| {mag.min():.6f}..{mag.max():.6f}",
          flush=True)
    np.testing.assert_allclose(mag, 0.5 * c[:, 13], rtol=1e-5)
    assert np.ptp(mag) <= 1e-5 * mag.max()
    vdir = np.stack([np.cos(angles), np.sin(angles), 0 * angles], 1)
    np.testing.assert_allclose(ft / mag[:, None], -vdir, atol=1e-5)


def test_mixed_pyramid_and_elliptic_batch(lib):
    """One launch over quadruped worlds with pyramids and with elliptic cones (the
    elliptic instantiation runs both) against each model stepped in its own batch."""
    mjh, ctx = lib
    nw, ns = 96, 20
    models = [robots.quadruped(), robots.quadruped_elliptic()]
    gms = [ctx.model_upload(mm) for mm in models]
    sep, held = [], []
    het = ctx.world_alloc(gms, [nw, nw])
    for g, (mm, gm) in enumerate(zip(models, gms)):
        qp, qv = inputs.initial_state("quadruped", mm, nw, seed=g)
        u = torch.tensor(inputs.controls("quadruped", mm, nw, ns, seed=g), dtype=torch.float32,
                         device="cuda").contiguous()
        w = mjh.World(ctx, gm, nw, qpos=qp, qvel=qv)
        w.batch.bind_io(0, u)
        w.batch.step(ns)
        sep.append(w)
        st = (torch.tensor(inputs.f32(qp), dtype=torch.float32, device="cuda"),
              torch.tensor(inputs.f32(qv), dtype=torch.float32, device="cuda"),
              torch.zeros(nw, mm.nv, device="cuda"),
              torch.zeros(nw, dtype=torch.int32, device="cuda"))
        het.bind_state(g, *st)
        het.bind_io(g, u)
        held.append((st, u))
    het.step(ns)
    torch.cuda.synchronize()
    for g in range(2):
        dq = (held[g][0][0] - sep[g].qpos).abs().max().item()
        dv = (held[g][0][1] - sep[g].qvel).abs().max().item() / max(
            sep[g].qvel.abs().max().item(), 1.0)
        print(f"[gpu] mixed batch group {g}: |d qpos| {dq:.1e} |d qvel|/max {dv:.1e}", flush=True)
        assert dq <= 1e-4 and dv <= 1e-3


def test_rollouts_and_env_reject_elliptic(lib):
    mjh, ctx = lib
    m = robots.quadruped_elliptic()
    w = mjh.World(ctx, m, 2)
    u = torch.zeros(4, 2, m.nu, device="cuda")
    loss = torch.zeros(2, device="cuda")
    with pytest.raises(mjh.MjhError):
        w.batch.rollout_fwd(4, 2, u, 2, 0.3, 1e-3, loss)
    f = dict(device="cuda", dtype=torch.float32)
    with pytest.raises(mjh.MjhError):
        w.batch.env_step(5, torch.zeros(1, 2, m.nu, **f), torch.zeros(2, 3, **f),
                         w.qpos.clone(), w.qvel.clone(), torch.zeros(2, m.nu, **f),
                         torch.zeros(1, 2, 12 + 3 * m.nu, **f), torch.zeros(1, 2, **f),
                         torch.zeros(1, 2, dtype=torch.int32, device="cuda"))
