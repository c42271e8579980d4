"""Heterogeneous batches, HIP-graph replay and the launch-shape autotuner on the GPU."""
import numpy as np
import pytest
import torch

from paper_2502_08844_amd.synth import inputs, robots

pytestmark = pytest.mark.gpu

KINDS = ("quadruped", "humanoid", "hand")


@pytest.fixture(scope="module")
def lib():
    from paper_2502_08844_amd import mjh
    return mjh, mjh.Context(0)


def _states(kind, nw, nstep, seed):
    m = robots.WORKLOADS[kind]()
    qp, qv = inputs.initial_state(kind, m, nw, seed=seed)
    u = inputs.controls(kind, m, nw, nstep, seed=seed)
    t = lambda x: torch.tensor(x, dtype=torch.float32, device="cuda").contiguous()
    return m, t(qp), t(qv), t(u)


def test_heterogeneous_batch_equals_per_model_launches(lib):
    mjh, ctx = lib
    counts = {"quadruped": 70, "humanoid": 33, "hand": 29}
    ns = 12
    data = {k: _states(k, counts[k], ns, seed=11) for k in KINDS}
    models = {k: ctx.model_upload(data[k][0]) for k in KINDS}
    # one launch for all three models
    b = ctx.world_alloc([models[k] for k in KINDS], [counts[k] for k in KINDS])
    het = {}
    for g, k in enumerate(KINDS):
        _, qp, qv, u = data[k]
        st = (qp.clone(), qv.clone(), torch.zeros_like(qv), torch.zeros(counts[k], dtype=torch.int32, device="cuda"))
        b.bind_state(g, *st)
        b.bind_io(g, u)
        het[k] = st
    b.step(ns)
    # each model alone, same launch shape
    for g, k in enumerate(KINDS):
        _, qp, qv, u = data[k]
        w = mjh.World(ctx, models[k], counts[k], qpos=qp.cpu().numpy(), qvel=qv.cpu().numpy())
        team, block = b.get_launch(g)
        w.batch.set_launch(0, team, block)
        w.step(u)
        torch.cuda.synchronize()
        assert torch.equal(w.qpos, het[k][0]), k
        assert torch.equal(w.qvel, het[k][1]), k
        assert torch.equal(w.qacc_ws, het[k][2]), k


def test_graph_replay_matches_eager(lib):
    mjh, ctx = lib
    m, qp, qv, u = _states("quadruped", 96, 5, seed=2)
    gm = ctx.model_upload(m)
    ref = mjh.World(ctx, gm, 96, qpos=qp.cpu().numpy(), qvel=qv.cpu().numpy())
    g = mjh.World(ctx, gm, 96, qpos=qp.cpu().numpy(), qvel=qv.cpu().numpy())
    g.batch.bind_io(0, u)
    s = torch.cuda.Stream()
    g.batch.graph_capture(5, s)
    for rep in range(3):
        ref.step(u)
        g.batch.graph_launch(s)
        s.synchronize()
        # eager work of the program between replays
        junk = torch.randn(1000, device="cuda").sum().item()
        assert np.isfinite(junk)
        torch.cuda.synchronize()
        assert torch.equal(ref.qpos, g.qpos), rep
        assert torch.equal(ref.qacc_ws, g.qacc_ws), rep
    # rebinding new buffers needs no recapture: the replay steps the new state and
    # leaves the old buffers alone
    old = (g.qpos.clone(), g.qvel.clone(), g.qacc_ws.clone())
    g2 = (g.qpos.clone(), g.qvel.clone(), g.qacc_ws.clone(),
          torch.zeros(96, dtype=torch.int32, device="cuda"))
    u2 = u.flip(0).contiguous()
    g.batch.bind_state(0, *g2)
    g.batch.bind_io(0, u2)
    for rep in range(2):
        ref.step(u2)
        g.batch.graph_launch(s)
        s.synchronize()
        junk = torch.randn(1000, device="cuda").sum().item()
        assert np.isfinite(junk)
        torch.cuda.synchronize()
        assert torch.equal(ref.qpos, g2[0]), rep
        assert torch.equal(ref.qvel, g2[1]), rep
        assert torch.equal(ref.qacc_ws, g2[2]), rep
    assert torch.equal(old[0], g.qpos) and torch.equal(old[1], g.qvel)
    # a new launch shape drops the graph: replaying it is refused until a new capture
    g.batch.set_launch(0, 64, 64)
    with pytest.raises(mjh.MjhError) as e:
        g.batch.graph_launch(s)
    assert e.value.code == mjh.ESTATE
    g.batch.graph_capture(5, s)
    ref.batch.set_launch(0, 64, 64)
    ref.step(u2)
    g.batch.graph_launch(s)
    torch.cuda.synchronize()
    assert torch.equal(ref.qpos, g2[0])


def test_autotune_keeps_state_and_results(lib):
    mjh, ctx = lib
    m, qp, qv, u = _states("quadruped", 300, 8, seed=4)
    gm = ctx.model_upload(m)
    w = mjh.World(ctx, gm, 300, qpos=qp.cpu().numpy(), qvel=qv.cpu().numpy())
    w.batch.bind_io(0, u)
    before = w.qpos.clone()
    w.batch.autotune(4)
    torch.cuda.synchronize()
    assert torch.equal(before, w.qpos)
    team, block = w.batch.get_launch(0)
    assert team in (16, 32, 64) and block % team == 0
    ref = mjh.World(ctx, gm, 300, qpos=qp.cpu().numpy(), qvel=qv.cpu().numpy())
    ref.step(u)
    w.step(u)
    torch.cuda.synchronize()
    assert (w.qpos - ref.qpos).abs().max().item() < 1e-3


def test_autotune_cache_round_trip(lib, tmp_path):
    """A tuned shape is written to the cache file; a fresh batch of the same model and
    world count takes the cached choice without probing, and another world count is a
    new entry."""
    mjh, ctx = lib
    m, qp, qv, u = _states("quadruped", 300, 8, seed=4)
    gm = ctx.model_upload(m)
    path = str(tmp_path / "tune.txt")
    w = mjh.World(ctx, gm, 300, qpos=qp.cpu().numpy(), qvel=qv.cpu().numpy())
    w.batch.bind_io(0, u)
    w.batch.autotune(4, cache_path=path)
    team, block = w.batch.get_launch(0)
    lines = open(path).read().splitlines()
    assert len(lines) == 1 and lines[0].endswith(f" : {team} {block}"), lines
    # plant a shape the probes never choose (16-lane teams for an 18-dof world run the
    # serial solves) and expect it back: the lookup, not a probe, decided
    key = lines[0].split(" : ")[0]
    with open(path, "w") as f:
        f.write(f"{key} : 16 64\n")
    w2 = mjh.World(ctx, gm, 300, qpos=qp.cpu().numpy(), qvel=qv.cpu().numpy())
    w2.batch.bind_io(0, u)
    before = w2.qpos.clone()
    w2.batch.autotune(4, cache_path=path)
    assert w2.batch.get_launch(0) == (16, 64)
    torch.cuda.synchronize()
    assert torch.equal(before, w2.qpos)
    # malformed lines and invalid shapes are ignored
    with open(path, "a") as f:
        f.write("garbage line\n1 2 3 : 17 64\n")
    w3 = mjh.World(ctx, gm, 150, qpos=qp[:150].cpu().numpy(), qvel=qv[:150].cpu().numpy())
    w3.batch.bind_io(0, u[:, :150].contiguous())
    w3.batch.autotune(4, cache_path=path)
    lines = open(path).read().splitlines()
    assert len(lines) == 2 and any(l.startswith(key + " : 16 64") for l in lines), lines
    t3, b3 = w3.batch.get_launch(0)
    assert any(l.endswith(f" 150 : {t3} {b3}") for l in lines), lines
