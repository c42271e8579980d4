"""GPU parity of the fused joystick env step (observation, reward, termination and reset
around the physics step) against the reference env in float64.

Checks, on the quadruped from contact-rich states with a share of inverted worlds:
* the physics inside the env step is the plain step's (same controls, nsub steps);
* obs, reward and done from that post-physics state match the reference's formulas
  evaluated in float64 on the same float32 state (|d| <= 5e-6 (1 + |x|));
* done worlds restart from their reset state with a zero warm start and previous
  action, the others keep the new state and remember the action;
* several env steps in one launch give the outputs of as many single launches;
* end to end against the reference env step from the same float32 state (FP32 against
  FP64 physics over nsub steps): done identical, obs within 1e-4 (1 + |x|) in every
  world;
* models without a free root and per-dof position actuators are rejected, and so are
  nenv 0, nsub 0 and per-world parameters on an implicit model, leaving every buffer;
* the GPU env computes the reward table's terms without the feet terms and the
  stand-still term, and returns the observation of the state a world ended in (its
  terminal observation) also for a done world: it is compared with the reference's
  terminal observations and with its reward before those terms; its parameter
  records carry no link centre-of-mass shifts (the reference's records are padded
  with zero shifts);
* domain randomisation: identity records and zero noise change no bit; with random
  records (friction, payload, centre of mass, PD gains, calibration, armature) and
  sensor noise, one physics step's qacc matches each world's randomised reference
  model at the parity tolerance (1e-4, worlds at a switch reported), the outputs match
  the float64 formulas of that model, and the end-to-end env step matches the
  reference env with the same records.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import env as renv
from paper_2502_08844_amd.synth import inputs, robots
from tests.gpu_util import G, compare_step, gpu_ctx, run_gpu, workload

pytestmark = pytest.mark.gpu

OUT_TOL = 5e-6
NSUB = 5


@pytest.fixture(scope="module")
def lib():
    return gpu_ctx()


def _scene(ctx, mjh, nw, seed, invert=True):
    """Contact-rich quadruped states (50 random-target steps), every fifth world turned
    upside down 0.45 m up; commands and actions drawn per world."""
    m, qp, qv, u = workload("quadruped", nw, 50, seed=seed)
    r = run_gpu(ctx, mjh, m, qp, qv, None, u, 50, contacts=False)
    qp, qv, ws = r["qpos"], r["qvel"], r["qacc"]
    inv = (np.arange(nw) % 5 == 3) & invert
    qp[inv, 2] = 0.45
    qp[inv, 3:7] = (0.0, 1.0, 0.0, 0.0)
    rng = np.random.default_rng(seed + 100)
    cmd = np.stack([rng.uniform(-1, 1, nw), rng.uniform(-0.5, 0.5, nw),
                    rng.uniform(-1, 1, nw)], 1)
    reset_q, reset_v = inputs.initial_state("quadruped", m, nw, seed=seed + 1)
    prev = rng.uniform(-0.5, 0.5, size=(nw, m.nu))
    return m, inputs.f32(qp), inputs.f32(qv), inputs.f32(ws), inputs.f32(cmd), reset_q, \
        reset_v, inputs.f32(prev), inv


def _gpu_record_size(m):
    """Words of the GPU env's parameter record: the reference's without link shifts."""
    return 8 + 2 * m.nu


def _pad_records(m, dr):
    """The reference's records for GPU records: zero link centre-of-mass shifts."""
    return np.concatenate([dr, np.zeros((dr.shape[0], renv.dr_size(m) - dr.shape[1]))], 1)


def _dev(x, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda").contiguous()


def _env_gpu(ctx, mjh, m, qp, qv, ws, acts, cmd, reset_q, reset_v, prev, nsub=NSUB, dr=None,
             noise=None):
    nenv, nw = acts.shape[:2]
    w = mjh.World(ctx, m, nw, qpos=qp, qvel=qv)
    w.qacc_ws.copy_(_dev(ws))
    la = _dev(prev)
    obs = torch.zeros(nenv, nw, 12 + 3 * m.nu, device="cuda")
    rew = torch.zeros(nenv, nw, device="cuda")
    done = torch.zeros(nenv, nw, dtype=torch.int32, device="cuda")
    w.batch.env_step(nsub, _dev(acts), _dev(cmd), _dev(reset_q), _dev(reset_v), la, obs, rew,
                     done, params=None if dr is None else _dev(dr),
                     obs_noise=None if noise is None else _dev(noise))
    torch.cuda.synchronize()
    f = lambda t: t.cpu().double().numpy()
    return dict(obs=f(obs), reward=f(rew), done=done.cpu().numpy().astype(bool), qpos=f(w.qpos),
                qvel=f(w.qvel), qacc=f(w.qacc_ws), last_action=f(la), status=w.status.cpu().numpy())


def test_env_step_outputs_and_resets(lib):
    mjh, ctx = lib
    nw = 240
    print(f"[gpu] env step quadruped nw={nw} nsub={NSUB}", flush=True)
    m, qp, qv, ws, cmd, rq, rv, prev, inv = _scene(ctx, mjh, nw, seed=3)
    act = inputs.f32(np.random.default_rng(7).uniform(-0.6, 0.6, size=(1, nw, m.nu)))
    g = _env_gpu(ctx, mjh, m, qp, qv, ws, act, cmd, rq, rv, prev)
    # the plain physics step with the action held for nsub steps
    p = run_gpu(ctx, mjh, m, qp, qv, ws, np.repeat(act, NSUB, 0), NSUB, contacts=False)
    assert np.all(g["status"] & 1 == 0) and np.all(p["status"] & 1 == 0)
    done_ref = np.array([renv.reward_done(m, p["qpos"][w], p["qvel"][w], act[0, w], prev[w],
                                          cmd[w])[1] for w in range(nw)])
    assert np.array_equal(g["done"][0], done_ref)
    assert np.array_equal(done_ref, inv)  # exactly the inverted worlds terminate
    keep = ~done_ref
    dq = np.abs(g["qpos"][keep] - p["qpos"][keep]).max()
    dv = np.abs(g["qvel"][keep] - p["qvel"][keep]).max() / max(np.abs(p["qvel"]).max(), 1.0)
    print(f"[gpu] env physics vs plain step: |d qpos| {dq:.1e} |d qvel|/max {dv:.1e}", flush=True)
    assert dq <= 1e-5 and dv <= 1e-5
    # outputs from the post-physics state against the float64 formulas
    eo, er = 0.0, 0.0
    for w in range(nw):
        o_ref = renv.observe(m, p["qpos"][w], p["qvel"][w], prev[w], cmd[w])
        r_ref, _ = renv.reward_done(m, p["qpos"][w], p["qvel"][w], act[0, w], prev[w], cmd[w])
        eo = max(eo, (np.abs(g["obs"][0, w] - o_ref) / (1 + np.abs(o_ref))).max())
        er = max(er, abs(g["reward"][0, w] - r_ref) / (1 + abs(r_ref)))
    print(f"[gpu] env outputs: obs err {eo:.1e} reward err {er:.1e}", flush=True)
    assert eo <= OUT_TOL and er <= OUT_TOL
    assert np.all(g["reward"] >= 0)
    # resets and the remembered action
    np.testing.assert_array_equal(g["qpos"][inv], rq[inv].astype(np.float32))
    np.testing.assert_array_equal(g["qvel"][inv], rv[inv].astype(np.float32))
    assert np.all(g["qacc"][inv] == 0) and np.all(g["last_action"][inv] == 0)
    np.testing.assert_array_equal(g["last_action"][keep], act[0, keep].astype(np.float32))


def test_multi_env_steps_one_launch(lib):
    mjh, ctx = lib
    nw, nenv = 96, 3
    print(f"[gpu] env steps nenv={nenv} in one launch vs {nenv} launches", flush=True)
    m, qp, qv, ws, cmd, rq, rv, prev, inv = _scene(ctx, mjh, nw, seed=5)
    acts = inputs.f32(np.random.default_rng(9).uniform(-0.6, 0.6, size=(nenv, nw, m.nu)))
    one = _env_gpu(ctx, mjh, m, qp, qv, ws, acts, cmd, rq, rv, prev)
    s = (qp, qv, ws, prev)
    for e in range(nenv):
        g = _env_gpu(ctx, mjh, m, *s[:3], acts[e:e + 1], cmd, rq, rv, s[3])
        for k in ("obs", "reward"):
            np.testing.assert_allclose(one[k][e], g[k][0], rtol=1e-6, atol=1e-7)
        assert np.array_equal(one["done"][e], g["done"][0])
        s = (g["qpos"], g["qvel"], g["qacc"], g["last_action"])
    np.testing.assert_allclose(one["qpos"], s[0], rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(one["last_action"], s[3], rtol=0, atol=0)
    assert one["done"][0].sum() == inv.sum()


def test_env_step_against_reference_env(lib):
    mjh, ctx = lib
    nw = 64
    print(f"[gpu] env step end to end vs reference nw={nw}", flush=True)
    m, qp, qv, ws, cmd, rq, rv, prev, inv = _scene(ctx, mjh, nw, seed=11)
    act = inputs.f32(np.random.default_rng(13).uniform(-0.6, 0.6, size=(1, nw, m.nu)))
    g = _env_gpu(ctx, mjh, m, qp, qv, ws, act, cmd, rq, rv, prev)
    o = oracle.Oracle(m)
    _, rew, done, (q, v, w_, pa, _), term = renv.env_step(o, m, qp, qv, ws, prev, act[0], cmd,
                                                          rq, rv, NSUB)
    assert np.array_equal(g["done"][0], done)
    err = (np.abs(g["obs"][0] - term) / (1 + np.abs(term))).max(1)
    print(f"[gpu] env obs vs FP64 env: median {np.median(err):.1e} max {err.max():.1e}",
          flush=True)
    assert err.max() <= 1e-4
    np.testing.assert_array_equal(g["last_action"], pa.astype(np.float32))


def test_env_step_rejects_other_models(lib):
    mjh, ctx = lib
    m = robots.hinge_chain(n=3)
    w = mjh.World(ctx, m, 4)
    z = lambda *s: torch.zeros(*s, device="cuda")
    with pytest.raises(mjh.MjhError):
        w.batch.env_step(1, z(1, 4, m.nu), z(4, 3), z(4, m.nq), z(4, m.nv), z(4, m.nu),
                         z(1, 4, 12 + 3 * m.nu), z(1, 4),
                         torch.zeros(1, 4, dtype=torch.int32, device="cuda"))


def _records(m, nw, seed):
    """Random per-world parameters in the ranges of the paper's randomisation (friction
    0.4-1.25, payload -0.5-2 kg, centre of mass +-3 cm, gains +-20 %, calibration +-0.05
    rad, armature 0-0.02 kg m^2)."""
    rng = np.random.default_rng(seed)
    rec = np.zeros((nw, _gpu_record_size(m)))
    rec[:, 0] = rng.uniform(0.4, 1.25, nw)
    rec[:, 1] = rng.uniform(-0.5, 2.0, nw)
    rec[:, 2:5] = rng.uniform(-0.03, 0.03, (nw, 3))
    rec[:, 5:7] = rng.uniform(0.8, 1.2, (nw, 2))
    rec[:, 8:8 + m.nu] = rng.uniform(-0.05, 0.05, (nw, m.nu))
    rec[:, 8 + m.nu:] = rng.uniform(0.0, 0.02, (nw, m.nu))
    return inputs.f32(rec)


def test_identity_records_change_nothing(lib):
    mjh, ctx = lib
    nw = 96
    print(f"[gpu] env step identity records nw={nw}", flush=True)
    m, qp, qv, ws, cmd, rq, rv, prev, inv = _scene(ctx, mjh, nw, seed=21)
    act = inputs.f32(np.random.default_rng(3).uniform(-0.6, 0.6, size=(2, nw, m.nu)))
    ref = _env_gpu(ctx, mjh, m, qp, qv, ws, act, cmd, rq, rv, prev)
    dr = np.stack([renv.dr_identity(m)[:_gpu_record_size(m)]] * nw)
    got = _env_gpu(ctx, mjh, m, qp, qv, ws, act, cmd, rq, rv, prev, dr=dr,
                   noise=np.zeros((2, nw, 12 + 3 * m.nu)))
    for k in ("obs", "reward", "done", "qpos", "qvel", "qacc", "last_action"):
        np.testing.assert_array_equal(got[k], ref[k], err_msg=k)


def test_randomised_physics_step_parity(lib):
    """nsub = 1 from the same float32 state: the written-back warm start is the step's
    a*, compared per world with the reference built from that world's record."""
    mjh, ctx = lib
    nw = 128
    print(f"[gpu] env step randomised physics parity nw={nw}", flush=True)
    m, qp, qv, ws, cmd, rq, rv, prev, _ = _scene(ctx, mjh, nw, seed=23, invert=False)
    dr = _records(m, nw, seed=5)
    act = inputs.f32(np.random.default_rng(6).uniform(-0.6, 0.6, size=(1, nw, m.nu)))
    noise = inputs.f32(np.random.default_rng(8).normal(scale=0.01, size=(1, nw, 48)))
    g = _env_gpu(ctx, mjh, m, qp, qv, ws, act, cmd, rq, rv, prev, nsub=1, dr=dr, noise=noise)
    assert not g["done"].any() and np.all(g["status"] & 1 == 0)
    o = oracle.Oracle(m)
    err, flag, eo, er = np.zeros(nw), np.zeros(nw, dtype=bool), 0.0, 0.0
    for w in range(nw):
        rec = _pad_records(m, dr[w:w + 1])[0]
        mw = renv.randomized_model(m, rec)
        ow = renv.randomized_oracle(o, m, rec)
        st = (qp[w:w + 1], qv[w:w + 1], ws[w:w + 1])
        ref = ow.step(*(x.copy() for x in st), act[:, w:w + 1], nstep=1)
        gpu1 = {"qacc": g["qacc"][w:w + 1], "ncon": ref["ncon"], "contacts": ref["contacts"]}
        cmp = compare_step(mw, ow, st, act[:, w:w + 1], gpu1)
        err[w], flag[w] = cmp["err_a"][0], cmp["flag"][0]
        # the outputs from the GPU's own post-step state, by this world's model
        qn, vn = g["qpos"][w], g["qvel"][w]
        o_ref = renv.observe(mw, qn, vn, prev[w], cmd[w], noise[0, w])
        r_ref, _ = renv.reward_done(mw, qn, vn, act[0, w], prev[w], cmd[w])
        eo = max(eo, (np.abs(g["obs"][0, w] - o_ref) / (1 + np.abs(o_ref))).max())
        er = max(er, abs(g["reward"][0, w] - r_ref) / (1 + abs(r_ref)))
    print(f"[gpu] randomised qacc rel err max {err[~flag].max():.2e} median {np.median(err):.2e};"
          f" near-switch {flag.sum()}/{nw}; obs err {eo:.1e} reward err {er:.1e}", flush=True)
    assert err[~flag].max() <= 1e-4 and flag.sum() <= max(1, 0.02 * nw)
    assert eo <= OUT_TOL and er <= OUT_TOL


def test_randomised_env_step_against_reference_env(lib):
    mjh, ctx = lib
    nw = 48
    print(f"[gpu] randomised env step end to end nw={nw}", flush=True)
    m, qp, qv, ws, cmd, rq, rv, prev, inv = _scene(ctx, mjh, nw, seed=27)
    dr = _records(m, nw, seed=9)
    act = inputs.f32(np.random.default_rng(10).uniform(-0.6, 0.6, size=(1, nw, m.nu)))
    noise = inputs.f32(np.random.default_rng(11).normal(scale=0.01, size=(1, nw, 48)))
    g = _env_gpu(ctx, mjh, m, qp, qv, ws, act, cmd, rq, rv, prev, dr=dr, noise=noise)
    _, rew, done, (q, v, w_, pa, _), obs = renv.env_step(
        oracle.Oracle(m), m, qp, qv, ws, prev, act[0], cmd, rq, rv, NSUB, dr=_pad_records(m, dr),
        noise=noise[0])
    assert np.array_equal(g["done"][0], done) and np.array_equal(done, inv)
    err = (np.abs(g["obs"][0] - obs) / (1 + np.abs(obs))).max(1)
    print(f"[gpu] randomised env obs vs FP64 env: median {np.median(err):.1e} "
          f"max {err.max():.1e}", flush=True)
    assert err.max() <= 1e-4
    np.testing.assert_array_equal(g["last_action"], pa.astype(np.float32))


def test_nonfinite_worlds_terminate_and_reset(lib):
    """Worlds whose state is no longer finite end (done, reward 0) and restart from
    their reset state; the other worlds' outputs are those of a run without them."""
    mjh, ctx = lib
    nw = 64
    print(f"[gpu] env step non-finite worlds nw={nw}", flush=True)
    m, qp, qv, ws, cmd, rq, rv, prev, inv = _scene(ctx, mjh, nw, seed=31, invert=False)
    act = inputs.f32(np.random.default_rng(4).uniform(-0.6, 0.6, size=(1, nw, m.nu)))
    ref = _env_gpu(ctx, mjh, m, qp, qv, ws, act, cmd, rq, rv, prev)
    bad = np.arange(nw) % 7 == 2
    qv_bad = qv.copy()
    qv_bad[bad, 7] = np.nan
    g = _env_gpu(ctx, mjh, m, qp, qv_bad, ws, act, cmd, rq, rv, prev)
    assert np.all(g["done"][0][bad]) and np.all(g["reward"][0][bad] == 0)
    np.testing.assert_array_equal(g["qpos"][bad], rq[bad].astype(np.float32))
    np.testing.assert_array_equal(g["qvel"][bad], rv[bad].astype(np.float32))
    assert np.all(g["last_action"][bad] == 0) and np.all(np.isfinite(g["qpos"]))
    ok = ~bad
    for k in ("obs", "reward", "done"):
        np.testing.assert_array_equal(g[k][0][ok], ref[k][0][ok])
    np.testing.assert_array_equal(g["qpos"][ok], ref["qpos"][ok])


def test_env_step_argument_errors_leave_state(lib):
    """No env steps (nenv 0), no physics steps per env step (nsub 0) and per-world
    parameters on a model with implicit damping are refused before any launch, and the
    bound state, previous action and outputs are left as they were."""
    mjh, ctx = lib
    nw = 6
    for m, params in ((robots.quadruped(), False), (robots.quadruped_implicit(), True)):
        nobs = 12 + 3 * m.nu
        qp, qv = inputs.initial_state("quadruped", m, nw, seed=3)
        w = mjh.World(ctx, m, nw, qpos=qp, qvel=qv)
        q0, v0 = w.qpos.clone(), w.qvel.clone()
        la = torch.full((nw, m.nu), 0.25, device="cuda")
        rq, rv = _dev(qp), _dev(qv)
        cmd = torch.zeros(nw, 3, device="cuda")
        dr = _dev(np.tile(renv.dr_identity(m)[:_gpu_record_size(m)], (nw, 1))) if params else None
        cases = [(1, NSUB)] if params else [(0, NSUB), (1, 0)]
        for nenv, nsub in cases:
            obs = torch.full((nenv, nw, nobs), 7.0, device="cuda")
            rew = torch.full((nenv, nw), 7.0, device="cuda")
            done = torch.full((nenv, nw), 7, dtype=torch.int32, device="cuda")
            acts = torch.zeros(nenv, nw, m.nu, device="cuda")
            print(f"[gpu] env_step refusal: integrator {m.opt.integrator} nenv {nenv} "
                  f"nsub {nsub} params {params}", flush=True)
            with pytest.raises(mjh.MjhError):
                w.batch.env_step(nsub, acts, cmd, rq, rv, la, obs, rew, done,
                                 params=dr if params else None)
            torch.cuda.synchronize()
            assert torch.equal(w.qpos, q0) and torch.equal(w.qvel, v0)
            assert torch.all(la == 0.25)
            assert torch.all(obs == 7.0) and torch.all(rew == 7.0) and torch.all(done == 7)
