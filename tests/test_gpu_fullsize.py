"""Parity at the full workload sizes, in the launch configurations the benchmark uses.

All worlds of each workload advance on the GPU; then one more step is compared with the
FP64 reference for a sample of worlds (evenly spaced, plus the last world of each
group), from the GPU's own float32 states:

* 8192 quadrupeds, team 32 / block 128 (the benchmark's launch), 60 steps;
* 8192 humanoids and 8192 hands, each model's default launch, 30 steps;
* the heterogeneous batch (4096 quadruped + 2048 humanoid + 2048 hand worlds), one
  autotuned launch replayed from a HIP graph, 30 steps, the compared step also replayed
  from a graph.

Tolerances as in the small parity tests: qacc <= 1e-4, contact forces <= 1e-3, with
states at a contact switch counted and reported.
"""
import numpy as np
import pytest
import torch

import oracle
from tests.gpu_util import compare_step, gpu_ctx, summarize, workload

pytestmark = pytest.mark.gpu

QACC_TOL = 1e-4
FORCE_TOL = 1e-3
NSAMPLE = 40


@pytest.fixture(scope="module")
def lib():
    return gpu_ctx()


def _sample(nw, k=NSAMPLE):
    idx = np.unique(np.linspace(0, nw - 1, k).round().astype(int))
    return np.union1d(idx, [nw - 1])


def _state(w):
    return (w.qpos.cpu().double().numpy(), w.qvel.cpu().double().numpy(),
            w.qacc_ws.cpu().double().numpy())


def _check(kind, m, state, u1, gpu1, idx):
    q, v, ws = state
    sub = (q[idx], v[idx], ws[idx])
    g1 = {k: gpu1[k][idx] for k in ("qacc", "contacts", "ncon")}
    cmp = compare_step(m, oracle.Oracle(m), sub, u1[:, idx], g1)
    cmp["t"], cmp["ncon"] = -1, g1["ncon"]
    print(f"[parity] {kind}: {len(idx)} sampled worlds", flush=True)
    ea, ef, nflag, ntot = summarize(kind, [cmp])
    assert ea.max() <= QACC_TOL
    if ef.size:
        assert ef.max() <= FORCE_TOL
    assert nflag <= max(1, 0.02 * ntot)


def _one_step(w, mjh, u1):
    """One more step of every world, exporting its contacts."""
    m = w.model
    con = torch.zeros(w.nworld, max(m.nconmax, 1), mjh.CON_SIZE, device="cuda")
    ncon = torch.zeros(w.nworld, dtype=torch.int32, device="cuda")
    w.batch.bind_io(0, u1, con, ncon)
    w.batch.step(1)
    torch.cuda.synchronize()
    return dict(qacc=w.qacc_ws.cpu().double().numpy(), contacts=con.cpu().double().numpy(),
                ncon=ncon.cpu().numpy())


@pytest.mark.parametrize("kind,nw,nstep,launch", [
    ("quadruped", 8192, 60, (32, 128)),
    ("humanoid", 8192, 30, None),
    ("hand", 8192, 30, None),
])
def test_full_size_single_model(lib, kind, nw, nstep, launch):
    mjh, ctx = lib
    print(f"[gpu] full-size parity {kind} nw={nw} steps={nstep} launch={launch}", flush=True)
    m, qp, qv, u = workload(kind, nw, nstep + 1, seed=7)
    w = mjh.World(ctx, m, nw, qpos=qp, qvel=qv)
    if launch is not None:
        w.batch.set_launch(0, *launch)
    ut = torch.tensor(u, dtype=torch.float32, device="cuda")
    w.step(ut[:nstep])
    torch.cuda.synchronize()
    assert np.all(w.status.cpu().numpy() & 1 == 0)
    state = _state(w)
    u1 = ut[nstep:nstep + 1].contiguous()
    gpu1 = _one_step(w, mjh, u1)
    _check(f"{kind}-full", m, state, u[nstep:nstep + 1], gpu1, _sample(nw))


def test_full_size_heterogeneous_graph(lib):
    mjh, ctx = lib
    spec = [("quadruped", 4096), ("humanoid", 2048), ("hand", 2048)]
    nstep = 30
    print(f"[gpu] full-size parity heterogeneous {spec} steps={nstep}", flush=True)
    data = [workload(kind, nw, nstep + 1, seed=11 + g) for g, (kind, nw) in enumerate(spec)]
    models = [ctx.model_upload(d[0]) for d in data]
    b = ctx.world_alloc(models, [nw for _, nw in spec])
    st, ctrl, ctrl1, cons = [], [], [], []
    for g, ((kind, nw), (m, qp, qv, u)) in enumerate(zip(spec, data)):
        s = (torch.tensor(qp, dtype=torch.float32, device="cuda"),
             torch.tensor(qv, dtype=torch.float32, device="cuda"),
             torch.zeros(nw, m.nv, device="cuda"),
             torch.zeros(nw, dtype=torch.int32, device="cuda"))
        b.bind_state(g, *s)
        ut = torch.tensor(u, dtype=torch.float32, device="cuda")
        ctrl.append(ut[:nstep].contiguous())
        ctrl1.append(ut[nstep:nstep + 1].contiguous())
        b.bind_io(g, ctrl[g])
        st.append(s)
    b.autotune(4)
    stream = torch.cuda.Stream()
    b.graph_capture(nstep, stream)
    b.graph_launch(stream)
    stream.synchronize()
    states = [(s[0].cpu().double().numpy(), s[1].cpu().double().numpy(),
               s[2].cpu().double().numpy()) for s in st]
    for g, (kind, nw) in enumerate(spec):
        assert np.all(st[g][3].cpu().numpy() & 1 == 0), kind
        con = torch.zeros(nw, max(models[g].nconmax, 1), mjh.CON_SIZE, device="cuda")
        ncon = torch.zeros(nw, dtype=torch.int32, device="cuda")
        b.bind_io(g, ctrl1[g], con, ncon)
        cons.append((con, ncon))
    b.graph_capture(1, stream)  # the compared step, replayed from a graph as well
    b.graph_launch(stream)
    stream.synchronize()
    for g, (kind, nw) in enumerate(spec):
        m, u = data[g][0], data[g][3]
        gpu1 = dict(qacc=st[g][2].cpu().double().numpy(),
                    contacts=cons[g][0].cpu().double().numpy(), ncon=cons[g][1].cpu().numpy())
        print(f"[gpu] group {kind} launch {b.get_launch(g)}", flush=True)
        _check(f"hetero-{kind}", m, states[g], u[nstep:nstep + 1], gpu1, _sample(nw, 24))
