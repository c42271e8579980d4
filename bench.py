"""Benchmark: world-steps/s of the batched physics step at 8192 quadruped worlds.

One bench "step" is one launch of the whole hot path (actuation, kinematics, CRBA,
LTDL, RNE, collision, constraint rows, Newton solve, Euler) advancing 8192 quadruped
worlds by 1000 physics steps (the 8192 x 1000 quadruped workload) on one GPU, with
per-step random PD targets resident in HBM.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--nworld 8192] [--nstep 1000]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X's published FP32 vector peak (it counts packed FP32, two FMAs per lane and
# cycle) is the roofline's peak.  This build disables packed FP32, so its own ceiling is
# 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz = 78.6 TFLOP/s, reported beside.
FP32_PUBLISHED_PEAK_TFLOPS = 157.3
FP32_NONPACKED_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12   # 78.6
QACC_TOL, FORCE_TOL, GRAD_TOL = 1e-4, 1e-3, 1e-3
HBM_PEAK_GBS = 8000.0             # MI355X published HBM3E bandwidth
PROFILE = os.path.join(ROOT, "profiles", "mjh_step_kernel_quadruped_8192x1000.txt")
PROFILED = (8192, 1000)           # nworld, nstep of the committed counter profile


def algo_bytes(nu, nq, nv, nstep):
    """Algorithmic HBM bytes per world-step: the controls of the step, plus qpos, qvel
    and the warm start read and written once per launch."""
    return 4.0 * nu + 4.0 * 2 * (nq + 2 * nv) / nstep


ALGO_BYTES_PER_WORLD_STEP_AT_1000 = algo_bytes(12, 19, 18, 1000)  # quadruped


def kernel_digest():
    """Digest of the library's sources and compile flags: a counter profile applies to
    the current kernel only if it was taken with the same digest.  (The built file
    itself is not hashed: it records the directory it was built in.)"""
    import hashlib
    from paper_2502_08844_amd import build
    h = hashlib.sha256()
    for name in sorted(os.listdir(build.CSRC)):
        if name.endswith((".hip", ".h", ".cpp")):
            with open(os.path.join(build.CSRC, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    h.update(" ".join(build.FLAGS).encode())
    return h.hexdigest()[:16]


def profiled_traffic(kind, nw, ns):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE profile,
    when it was taken on this kernel and this workload; otherwise None."""
    if kind != "quadruped" or (nw, ns) != PROFILED or not os.path.exists(PROFILE):
        return None
    digest, traffic = None, None
    with open(PROFILE) as f:
        for line in f:
            if line.startswith("kernel source digest:"):
                digest = line.split(":", 1)[1].strip()
            elif line.strip().startswith("traffic_bytes_per_launch:"):
                traffic = float(line.split(":", 1)[1])
    return traffic if digest == kernel_digest() else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--model", default="quadruped",
                    choices=["quadruped", "quadruped_limits", "quadruped_friction",
                             "quadruped_tethered", "quadruped_welded", "quadruped_frictionless",
                             "quadruped_implicit", "quadruped_implicit_pd", "quadruped_rk4",
                             "quadruped_rough", "quadruped_elliptic", "humanoid", "hand",
                             "cartpole"],
                    help="robot of the timed batch (the headline metric is the quadruped)")
    ap.add_argument("--nworld", type=int, default=8192)
    ap.add_argument("--nstep", type=int, default=1000)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the host leg (FP64 reference: parity, FLOP count, CPU rate)")
    ap.add_argument("--cpu-sample-worlds", type=int, default=8192)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="run the reference on the host in chunks of 40 steps until this "
                         "much time has been spent")
    ap.add_argument("--no-rollout", action="store_true",
                    help="skip the adjoint-rollout comparison (1024 worlds, horizon 64)")
    ap.add_argument("--no-hetero", action="store_true",
                    help="skip the heterogeneous-batch comparison")
    ap.add_argument("--no-limits", action="store_true",
                    help="skip the quadruped variants (limits, friction loss, equalities, "
                         "contact dimensions, integrators, rough terrain)")
    ap.add_argument("--no-env", action="store_true",
                    help="skip the fused joystick env step measurement")
    ap.add_argument("--graph", action="store_true", help="replay a captured HIP graph")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run a plain device copy of this many MiB (a reference "
                         "kernel for calibrating hardware byte counters)")
    return ap.parse_args()


def host_cpu():
    """(CPU model, CPUs the host reports, threads the reference may use).  The threads
    are the CPUs this process may run on, capped by OMP_NUM_THREADS when it is set (a
    GPU machine's share of its host's cores)."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    avail = len(os.sched_getaffinity(0))
    share = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    return name, os.cpu_count(), min(avail, share) if share > 0 else avail


def gpu_states(ctx, kind, nw, warm, seed):
    """nw worlds of `kind` advanced `warm` steps on the GPU from the seeded initial state
    with random controls; returns the model, the float32 state (as float64) and the
    control of the next step."""
    import torch
    from paper_2502_08844_amd import mjh
    from paper_2502_08844_amd.synth import inputs, robots
    m = robots.WORKLOADS[kind]()
    qp, qv = inputs.initial_state(kind, m, nw, seed=seed)
    u = inputs.controls(kind, m, nw, warm + 1, seed=seed)
    w = mjh.World(ctx, m, nw, qpos=qp, qvel=qv)
    w.step(torch.tensor(u[:warm], dtype=torch.float32, device="cuda"), nstep=warm)
    torch.cuda.synchronize()
    st = [x.cpu().double().numpy() for x in (w.qpos, w.qvel, w.qacc_ws)]
    return m, w, st, u[warm:warm + 1]


def step_parity(ctx, o, kind, nw=64, warm=50, seed=0):
    """One GPU step against one reference step (fixed iteration count) from the same
    float32 states after `warm` GPU steps: per world ||qacc_gpu - qacc_ref||_inf /
    max(||qacc_ref||_inf, 9.81), and each contact's frame force error / (total mass *
    9.81).  Worlds whose contact sets differ, or with a contact within 1e-5 of its
    emission distance, sit at a switch: they are counted, not included."""
    import numpy as np
    import torch
    m, w, (q, v, a), u1 = gpu_states(ctx, kind, nw, warm, seed)
    con, ncon = w.step(torch.tensor(u1, dtype=torch.float32, device="cuda"), nstep=1,
                       contacts=True)
    torch.cuda.synchronize()
    ga, gc, gn = (w.qacc_ws.cpu().double().numpy(), con.cpu().double().numpy(),
                  ncon.cpu().numpy())
    ref = o.step(q, v, a, u1, nstep=1, nthreads=8)
    mass = sum(b.mass for b in m.bodies)
    ea, ef, nsw = [], [], 0
    for k in range(nw):
        nr = int(ref["ncon"][k])
        cr, cg = ref["contacts"][k, :nr], gc[k, :int(gn[k])]
        if int(gn[k]) != nr or not np.array_equal(cr[:, 16:18], cg[:, 16:18]) or \
                (nr and np.abs(cr[:, 0]).min() < 1e-5):
            nsw += 1
            continue
        ea.append(np.abs(ga[k] - ref["qacc"][k]).max() / max(np.abs(ref["qacc"][k]).max(), 9.81))
        if nr:
            ef.append(np.abs(cg[:, 13:16] - cr[:, 13:16]).max() / (mass * 9.81))
    return ({"qacc_max": float(f"{max(ea):.3g}"), "force_max": float(f"{max(ef):.3g}") if ef else 0.0,
             "worlds": nw, "at_switch": nsw, "step": warm + 1},
            (q, v, a, u1[0]))


def adjoint_parity(ctx, o, nw=16, horizon=64, ckpt=8, seed=0):
    """The GPU rollout gradient (wrt qvel0 and the 64 x 12 controls) along one random
    direction per world against the reference's exact directional derivative (dual
    numbers, solver converged): |<g, d> - dL| / (|g| |d|)."""
    import numpy as np
    import torch
    from paper_2502_08844_amd import mjh
    from paper_2502_08844_amd.synth import inputs, robots
    m = robots.quadruped()
    qp, qv = inputs.initial_state("quadruped", m, nw, seed=seed)
    rng = inputs.rng(seed, 7)
    qv = inputs.f32(qv + rng.normal(scale=0.1, size=qv.shape))
    u = inputs.f32(rng.uniform(-0.5, 0.5, size=(horizon, nw, m.nu)))
    w = mjh.World(ctx, m, nw, qpos=qp)
    qv0 = torch.tensor(qv, dtype=torch.float32, device="cuda", requires_grad=True)
    ut = torch.tensor(u, dtype=torch.float32, device="cuda", requires_grad=True)
    mjh.Rollout.apply(qv0, ut, w, horizon, ckpt).sum().backward()
    torch.cuda.synchronize()
    gq, gu = qv0.grad.cpu().double().numpy(), ut.grad.cpu().double().numpy()
    dv = rng.normal(size=(nw, m.nv))
    du = rng.normal(size=(horizon, nw, m.nu))
    import oracle
    _, dL = o.rollout_jvp(qp, qv, u, dv, du, mode=oracle.MODE_CONVERGED, nthreads=8)
    g_dot = np.sum(gq * dv, axis=1) + np.einsum("twa,twa->w", gu, du)
    gn = np.sqrt(np.sum(gq * gq, 1) + np.einsum("twa,twa->w", gu, gu))
    dn = np.sqrt(np.sum(dv * dv, 1) + np.einsum("twa,twa->w", du, du))
    rel = np.abs(g_dot - dL) / (gn * dn)
    return {"directional_max": float(f"{rel.max():.3g}"), "worlds": nw, "horizon": horizon,
            "ckpt_every": ckpt}


def host_leg(ctx, kind, m, qp, qv, seconds, seed, single_seconds=4.0, chunk=40,
             max_chunks=200):
    """Everything that runs the FP64 reference (the oracle), on the host, outside the
    timed GPU region:
    * parity: one GPU step against one reference step for every workload's model
      (cartpole, quadruped, humanoid, hand: the heterogeneous batch runs the same
      per-world kernels) and the adjoint rollout's gradient against dual numbers;
    * the algorithmic FLOP count per world-step on the quadruped's sampled states;
    * the reference's own rate on a bounded sample of the benched workload: chunks of
      `chunk` steps with fresh controls until `seconds` are spent, at the threads the
      host grants, and on one thread for `single_seconds`."""
    import oracle
    from paper_2502_08844_amd.synth import inputs, robots
    parity = {"tolerance": {"qacc": QACC_TOL, "force": FORCE_TOL, "gradient": GRAD_TOL}}
    flops = None
    for k in ("cartpole", "quadruped", "humanoid", "hand"):
        o = oracle.Oracle(robots.WORKLOADS[k]())
        parity[k], (q, v, a, u1) = step_parity(ctx, o, k, seed=seed)
        if k == kind or (flops is None and k == "quadruped"):
            flops = {"nonzero": o.count_flops(q, v, a, u1, nonzero=True),
                     "dense": o.count_flops(q, v, a, u1)}
    parity["adjoint"] = adjoint_parity(ctx, oracle.Oracle(robots.quadruped()), seed=seed)
    name, ncpu, nthreads = host_cpu()
    o = oracle.Oracle(m)
    rates = {}
    for threads, budget, nw in ((nthreads, seconds, qp.shape[0]),
                                (1, single_seconds, min(qp.shape[0], 1024))):
        q, v, ws = qp[:nw].copy(), qv[:nw].copy(), None
        spent, steps = 0.0, 0
        for c in range(max_chunks):
            u = inputs.controls(kind, m, nw, chunk, seed=seed + 1000 + c)
            t0 = time.perf_counter()
            out = o.step(q, v, ws, u, nstep=chunk, nthreads=threads)
            spent += time.perf_counter() - t0
            steps += chunk
            q, v, ws = out["qpos"], out["qvel"], out["qacc_ws"]
            if spent >= budget:
                break
        rates[threads] = (nw * steps / spent, spent, steps, nw)
    r, r1 = rates[nthreads], rates[1]
    cpu = {"value": round(r[0], 1), "unit": "world-steps/s", "cores": nthreads, "kind": "oracle",
           "sample": f"{r[3]} {kind} worlds x {r[2]} steps (chunks of {chunk}, fresh random "
                     f"controls), FP64, {r[1]:.1f} s on {nthreads} threads",
           "single_thread_value": round(r1[0], 1),
           "single_thread_sample": f"{r1[3]} worlds x {r1[2]} steps, {r1[1]:.1f} s",
           "cpu_model": name, "host_cpus": ncpu}
    return cpu, parity, flops


def timed(fn, stream, reps):
    """Median event-timed duration (ms) of fn() on `stream` over reps runs."""
    import torch
    ms = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b))
    return sorted(ms)[len(ms) // 2]


def rollout_compare(ctx, seed, nw=1024, horizon=64, ckpt=8, reps=3):
    """Adjoint rollout (forward with checkpoints + reverse sweep) against the plain step
    on the same worlds: 1024 quadrupeds, horizon 64, checkpoints every 8 steps.  Both
    use the launch shape the autotuner picks for the plain step at this world count."""
    import torch
    from paper_2502_08844_amd import mjh
    from paper_2502_08844_amd.synth import inputs, robots
    m = robots.quadruped()
    gm = ctx.model_upload(m)
    qp, qv = inputs.initial_state("quadruped", m, nw, seed=seed)
    rng = inputs.rng(seed, 7)
    u = torch.tensor(inputs.f32(rng.uniform(-0.5, 0.5, size=(horizon, nw, m.nu))),
                     dtype=torch.float32, device="cuda").contiguous()
    stream = torch.cuda.current_stream()
    plain = mjh.World(ctx, gm, nw, qpos=qp, qvel=qv)
    q0, v0 = plain.qpos.clone(), plain.qvel.clone()
    plain.batch.bind_io(0, u)
    plain.batch.autotune(8)
    team, block = plain.batch.get_launch(0)

    def run_plain():
        plain.qpos.copy_(q0); plain.qvel.copy_(v0); plain.qacc_ws.zero_()
        plain.batch.step(horizon, stream)
    run_plain()
    t_plain = timed(run_plain, stream, reps)
    w = mjh.World(ctx, gm, nw, qpos=qp, qvel=qv)
    w.batch.set_launch(0, team, block)
    loss = torch.empty(nw, device="cuda")
    dloss = torch.ones(nw, device="cuda")
    gq = torch.empty(nw, m.nv, device="cuda")
    gu = torch.empty_like(u)

    def run_fwd():
        w.qpos.copy_(q0); w.qvel.copy_(v0); w.qacc_ws.zero_()
        w.batch.rollout_fwd(horizon, ckpt, u, 2, 0.3, 1e-3, loss, stream)

    def run_bwd():
        w.batch.rollout_bwd(dloss, gq, gu, stream)
    run_fwd(); run_bwd()
    t_fwd = timed(run_fwd, stream, reps)
    t_bwd = timed(run_bwd, stream, reps)
    ws = nw * horizon
    return {"workload": f"quadruped {nw} worlds, horizon {horizon}, checkpoints every {ckpt}",
            "plain_world_steps_per_s": round(ws / (t_plain * 1e-3), 1),
            "fwd_bwd_rollout_steps_per_s": round(ws / ((t_fwd + t_bwd) * 1e-3), 1),
            "fwd_ms": round(t_fwd, 3), "bwd_ms": round(t_bwd, 3), "plain_ms": round(t_plain, 3),
            "fwd_bwd_over_plain_time": round((t_fwd + t_bwd) / t_plain, 2),
            "launch": [team, block]}


def constraint_compare(ctx, seed, kind, what, nw=8192, nstep=1000, reps=3):
    """A quadruped variant with more constraint rows beside the contacts (limited
    hinges, dry joint friction, or a tether equality), 8192 worlds x 1000 steps in its
    default launch."""
    import torch
    from paper_2502_08844_amd import mjh
    from paper_2502_08844_amd.synth import inputs, robots
    stream = torch.cuda.current_stream()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    m = robots.WORKLOADS[kind]()
    qp, qv = inputs.initial_state(kind, m, nw, seed=seed)
    w = mjh.World(ctx, ctx.model_upload(m), nw, qpos=qp, qvel=qv)
    u = (torch.rand((nstep, nw, m.nu), device="cuda", generator=gen) - 0.5).contiguous()
    w.batch.bind_io(0, u)
    q0, v0 = w.qpos.clone(), w.qvel.clone()

    def run():
        w.qpos.copy_(q0); w.qvel.copy_(v0); w.qacc_ws.zero_()
        w.batch.step(nstep, stream)
    run()
    ms = timed(run, stream, reps)
    status = w.status.cpu()
    return {"workload": f"quadruped with {what}, {nw} worlds x {nstep} steps",
            "world_steps_per_s": round(nw * nstep / (ms * 1e-3), 1),
            "nrowmax": m.nrowmax,
            "launch": list(w.batch.get_launch(0)),
            "status_nonzero_worlds": int((status != 0).sum())}


def env_compare(ctx, seed, nw=8192, nenv=200, nsub=5, reps=3):
    """The joystick env step fused around the physics (observation, reward, termination
    and reset in the same kernel): 8192 quadruped worlds x 200 env steps of 5 physics
    steps (a 0.02 s control period at dt 0.004), one launch, actions U(-0.5, 0.5) drawn
    per env step and resident in HBM with the outputs."""
    import torch
    from paper_2502_08844_amd import mjh
    from paper_2502_08844_amd.synth import inputs, robots
    stream = torch.cuda.current_stream()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    m = robots.WORKLOADS["quadruped"]()
    qp, qv = inputs.initial_state("quadruped", m, nw, seed=seed)
    w = mjh.World(ctx, ctx.model_upload(m), nw, qpos=qp, qvel=qv)
    f = dict(device="cuda", dtype=torch.float32)
    act = (torch.rand((nenv, nw, m.nu), device="cuda", generator=gen) - 0.5).contiguous()
    cmd = torch.stack([2 * torch.rand(nw, device="cuda", generator=gen) - 1,
                       torch.rand(nw, device="cuda", generator=gen) - 0.5,
                       2 * torch.rand(nw, device="cuda", generator=gen) - 1], 1).contiguous()
    q0, v0 = w.qpos.clone(), w.qvel.clone()
    last = torch.zeros(nw, m.nu, **f)
    obs = torch.zeros(nenv, nw, 12 + 3 * m.nu, **f)
    rew = torch.zeros(nenv, nw, **f)
    done = torch.zeros(nenv, nw, dtype=torch.int32, device="cuda")

    # per-world randomised parameters in the ranges of the paper's randomisation, and
    # sensor noise N(0, 0.01) on every observation entry
    u = lambda lo, hi, *shape: lo + (hi - lo) * torch.rand(shape, device="cuda", generator=gen)
    params = torch.cat([u(0.4, 1.25, nw, 1), u(-0.5, 2.0, nw, 1), u(-0.03, 0.03, nw, 3),
                        u(0.8, 1.2, nw, 2), torch.zeros(nw, 1, device="cuda"),
                        u(-0.05, 0.05, nw, m.nu), u(0.0, 0.02, nw, m.nu)], 1).contiguous()
    noise = (0.01 * torch.randn(obs.shape, device="cuda", generator=gen)).contiguous()

    def run(dr=False):
        w.qpos.copy_(q0); w.qvel.copy_(v0); w.qacc_ws.zero_(); last.zero_()
        w.batch.env_step(nsub, act, cmd, q0, v0, last, obs, rew, done,
                         params if dr else None, noise if dr else None, stream)
    run()
    ms = timed(run, stream, reps)
    run(True)
    ms_dr = timed(lambda: run(True), stream, reps)
    return {"workload": f"quadruped joystick env, {nw} worlds x {nenv} env steps of {nsub} "
                        "physics steps, one launch",
            "env_steps_per_s": round(nw * nenv / (ms * 1e-3), 1),
            "world_steps_per_s": round(nw * nenv * nsub / (ms * 1e-3), 1),
            "randomised_env_steps_per_s": round(nw * nenv / (ms_dr * 1e-3), 1),
            "nobs": 12 + 3 * m.nu, "launch": list(w.batch.get_launch(0)),
            "terminations": int(done.sum().item()),
            "mean_reward": round(float(rew.mean().item()), 4),
            "status_nonzero_worlds": int((w.status != 0).sum().item())}


def hetero_compare(ctx, seed, nstep=500, reps=3):
    """4096 quadruped + 2048 humanoid + 2048 hand worlds in one autotuned launch replayed
    from a HIP graph, against the three models stepped by their own default launches."""
    import torch
    from paper_2502_08844_amd import mjh
    from paper_2502_08844_amd.synth import inputs, robots
    spec = [("quadruped", 4096), ("humanoid", 2048), ("hand", 2048)]
    stream = torch.cuda.current_stream()
    worlds, ctrls, init = [], [], []
    for k, (kind, nw) in enumerate(spec):
        m = robots.WORKLOADS[kind]()
        qp, qv = inputs.initial_state(kind, m, nw, seed=seed + k)
        u = torch.tensor(inputs.controls(kind, m, nw, nstep, seed=seed + k),
                         dtype=torch.float32, device="cuda")
        w = mjh.World(ctx, ctx.model_upload(m), nw, qpos=qp, qvel=qv)
        w.batch.bind_io(0, u.contiguous())
        worlds.append(w); ctrls.append(u.contiguous()); init.append((w.qpos.clone(), w.qvel.clone()))
    total = sum(nw for _, nw in spec) * nstep

    def reset(ws):
        for w, (q, v) in zip(ws, init):
            w.qpos.copy_(q); w.qvel.copy_(v); w.qacc_ws.zero_()

    def run_plain():
        reset(worlds)
        for w in worlds:
            w.batch.step(nstep, stream)
    run_plain()
    t_plain = timed(run_plain, stream, reps)
    het = ctx.world_alloc([w.model for w in worlds], [nw for _, nw in spec])
    states = []
    for g, w in enumerate(worlds):
        st = (w.qpos.clone(), w.qvel.clone(), torch.zeros_like(w.qvel),
              torch.zeros(w.nworld, dtype=torch.int32, device="cuda"))
        het.bind_state(g, *st)
        het.bind_io(g, ctrls[g])
        states.append(st)
    t0 = time.perf_counter()
    het.autotune(20)
    torch.cuda.synchronize()
    t_tune = time.perf_counter() - t0
    gs = torch.cuda.Stream()
    het.graph_capture(nstep, gs)

    def run_graph():
        for (q, v, a, _), (q0, v0) in zip(states, init):
            q.copy_(q0); v.copy_(v0); a.zero_()
        het.graph_launch(stream)
    run_graph()
    t_graph = timed(run_graph, stream, reps)
    return {"workload": "4096 quadruped + 2048 humanoid + 2048 hand worlds x "
                        f"{nstep} steps",
            "graph_autotuned_world_steps_per_s": round(total / (t_graph * 1e-3), 1),
            "per_model_default_world_steps_per_s": round(total / (t_plain * 1e-3), 1),
            "speedup": round(t_plain / t_graph, 3),
            "launch": {kind: list(het.get_launch(g)) for g, (kind, _) in enumerate(spec)},
            "autotune_s": round(t_tune, 2)}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: measures one GPU only (--gpus 1); worlds are independent, so a "
              "multi-GPU run would split nworld across GPUs with no exchange", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2502_08844_amd import mjh
    from paper_2502_08844_amd.synth import inputs, robots

    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    kind = args.model
    m = robots.WORKLOADS[kind]()
    nw, ns = args.nworld, args.nstep
    ctx = mjh.Context(0)
    gm = ctx.model_upload(m)
    qp, qv = inputs.initial_state(kind, m, nw, seed=args.seed)
    dev = "cuda"
    world = mjh.World(ctx, gm, nw, qpos=qp, qvel=qv)
    q0, v0 = world.qpos.clone(), world.qvel.clone()
    gen = torch.Generator(device=dev)
    gen.manual_seed(args.seed)
    # controls resampled every step, resident in HBM, drawn on the device with the
    # distributions of the synthetic workloads
    shape = (ns, nw, m.nu)
    if kind.startswith("quadruped"):  # PD target offsets U(-0.5, 0.5)
        ctrl = torch.rand(shape, device=dev, generator=gen) - 0.5
    elif kind == "humanoid":   # torques N(0, 0.3) clipped to [-1, 1]
        ctrl = (0.3 * torch.randn(shape, device=dev, generator=gen)).clamp_(-1.0, 1.0)
    elif kind == "hand":       # PD target offsets U(-0.3, 0.3)
        ctrl = 0.6 * torch.rand(shape, device=dev, generator=gen) - 0.3
    else:                      # cart force U(-1, 1)
        ctrl = 2.0 * torch.rand(shape, device=dev, generator=gen) - 1.0
    ctrl = ctrl.contiguous()
    world.batch.bind_io(0, ctrl)
    stream = torch.cuda.current_stream()

    def reset():
        world.qpos.copy_(q0)
        world.qvel.copy_(v0)
        world.qacc_ws.zero_()

    if args.graph:
        gs = torch.cuda.Stream()
        world.batch.graph_capture(ns, gs)

    def launch():
        if args.graph:
            world.batch.graph_launch(stream)
        else:
            world.batch.step(ns, stream)

    for _ in range(args.warmup):
        reset()
        launch()
    torch.cuda.synchronize()
    # kernel-only timing with events on the launch stream, per launch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        reset()
        ev[k][0].record(stream)
        launch()
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [a.elapsed_time(b) for a, b in ev]
    status = world.status.cpu().numpy()
    world_steps = nw * ns * args.steps
    value = world_steps / wall
    ms_per_step = 1000.0 * wall / args.steps
    kavg = float(np.mean(kern_ms))

    # roofline of the step kernel: plain FP32 ALU work (no MFMA, not HBM bound); the
    # algorithmic FLOP count comes from the host leg below
    bytes_ws = algo_bytes(m.nu, m.nq, m.nv, ns)
    roof = {"bound": "alu", "achieved": None, "peak": FP32_PUBLISHED_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": None, "traffic": profiled_traffic(kind, nw, ns),
            "peak_nonpacked": round(FP32_NONPACKED_PEAK_TFLOPS, 1), "frac_nonpacked": None,
            "kernel": "mjh_step_kernel", "kernel_ms": round(kavg, 3),
            "flops_per_world_step": None, "flops_per_world_step_dense": None,
            "hbm_bytes_per_world_step": round(bytes_ws, 2),
            "hbm_frac": round(bytes_ws * nw * ns / (kavg * 1e-3) / 1e9 / HBM_PEAK_GBS, 8)}
    metric = ("world-steps/sec at 8192 quadruped worlds; fwd+bwd rollout steps/sec vs plain"
              if kind == "quadruped" else f"world-steps/sec at {nw} {kind} worlds")
    out = {"metric": metric,
           "value": round(value, 1),
           "unit": "world-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": f"synthetic (seeded {kind} states, random controls every step)",
           "config": {"workload": f"{kind} {nw} worlds x {ns} physics steps per launch",
                      "nworld": nw, "nstep_per_launch": ns, "dt": m.opt.timestep,
                      "newton_iterations": m.opt.iterations, "graph": bool(args.graph),
                      "launch": list(world.batch.get_launch(0)),
                      "status_nonzero_worlds": int(np.count_nonzero(status))},
           "roofline": roof}
    del world, ctrl
    if not args.no_rollout:
        out["rollout"] = rollout_compare(ctx, args.seed)
    if not args.no_hetero:
        out["hetero"] = hetero_compare(ctx, args.seed)
    if not args.no_env:
        out["env_step"] = env_compare(ctx, args.seed)
    if not args.no_limits:
        out["limits"] = constraint_compare(ctx, args.seed, "quadruped_limits",
                                           "limited hinges (default angle +- 0.15 rad)")
        out["friction_loss"] = constraint_compare(
            ctx, args.seed, "quadruped_friction",
            f"dry joint friction {robots.QUAD_FRICTIONLOSS} N m on every hinge")
        out["equality"] = constraint_compare(
            ctx, args.seed, "quadruped_tethered",
            "its torso centre held on its standing position by a connect equality")
        out["weld"] = constraint_compare(
            ctx, args.seed, "quadruped_welded",
            "its torso welded to the world at its standing pose (a fixed base)")
        out["frictionless"] = constraint_compare(
            ctx, args.seed, "quadruped_frictionless",
            "frictionless feet (condim 1: one row a contact)")
        out["torsion"] = constraint_compare(
            ctx, args.seed, "quadruped_torsion",
            "torsional friction at the feet (condim 4: six pyramid edges a contact)")
        out["rolling"] = constraint_compare(
            ctx, args.seed, "quadruped_rolling",
            "torsional and rolling friction at the feet (condim 6: ten edges a contact)")
        out["elliptic"] = constraint_compare(
            ctx, args.seed, "quadruped_elliptic",
            "elliptic friction cones at the feet (three frame rows a contact)")
        out["elliptic_rolling"] = constraint_compare(
            ctx, args.seed, "quadruped_elliptic_rolling",
            "elliptic cones over sliding, torsional and rolling friction (six rows a contact)")
        out["implicit_damping"] = constraint_compare(
            ctx, args.seed, "quadruped_implicit",
            "its PD velocity gains integrated implicitly")
        out["implicit_pd"] = constraint_compare(
            ctx, args.seed, "quadruped_implicit_pd",
            "its PD velocity and position gains integrated implicitly")
        out["rk4"] = constraint_compare(
            ctx, args.seed, "quadruped_rk4",
            "fourth-order Runge-Kutta (four forward passes a step)")
        out["rough_terrain"] = constraint_compare(
            ctx, args.seed, "quadruped_rough",
            "its feet on 8 m x 8 m Perlin-noise terrain (128 x 128 heightfield, 6 cm relief)")
    if not args.no_cpu_baseline:
        cpu, parity, flops = host_leg(ctx, kind, m, qp[:min(args.cpu_sample_worlds, nw)],
                                      qv[:min(args.cpu_sample_worlds, nw)], args.cpu_seconds,
                                      args.seed)
        achieved = flops["nonzero"] * nw * ns / (kavg * 1e-3) / 1e12
        roof.update({"achieved": round(achieved, 4),
                     "frac": round(achieved / FP32_PUBLISHED_PEAK_TFLOPS, 6),
                     "frac_nonpacked": round(achieved / FP32_NONPACKED_PEAK_TFLOPS, 6),
                     "flops_per_world_step": round(flops["nonzero"], 1),
                     "flops_per_world_step_dense": round(flops["dense"], 1)})
        out["parity"] = parity
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
