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

FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X published FP32 vector peak
HBM_PEAK_GBS = 8000.0             # MI355X published HBM3E bandwidth


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nworld", type=int, default=8192)
    ap.add_argument("--nstep", type=int, default=1000)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-worlds", type=int, default=8192)
    ap.add_argument("--cpu-sample-steps", type=int, default=40)
    ap.add_argument("--graph", action="store_true", help="replay a captured HIP graph")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run a plain device copy of this many MiB (a reference "
                         "kernel for calibrating hardware byte counters)")
    return ap.parse_args()


def algorithmic_flops_per_world_step(model, qpos, qvel, ctrl):
    """Floating-point operations of the reference algorithm per world-step, counted by
    running the FP64 reference with an operation-counting scalar on sampled states."""
    import oracle
    o = oracle.Oracle(model)
    return o.count_flops(qpos, qvel, None, ctrl)


def cpu_baseline(model, qpos, qvel, ctrl, nthreads):
    import oracle
    o = oracle.Oracle(model)
    nw, ns = qpos.shape[0], ctrl.shape[0]
    t0 = time.perf_counter()
    o.step(qpos.copy(), qvel.copy(), None, ctrl, nstep=ns, nthreads=nthreads)
    dt = time.perf_counter() - t0
    return nw * ns / dt, dt


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build measures one GPU only; worlds are independent and "
              "would shard across GPUs with no exchange (see DESIGN.md)", file=sys.stderr)
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
    kind = "quadruped"
    m = robots.quadruped()
    nw, ns = args.nworld, args.nstep
    ctx = mjh.Context(0)
    gm = ctx.model_upload(m)
    qp, qv = inputs.initial_state(kind, m, nw, seed=args.seed)
    dev = "cuda"
    world = mjh.World(ctx, gm, nw, qpos=qp, qvel=qv)
    q0, v0 = world.qpos.clone(), world.qvel.clone()
    gen = torch.Generator(device=dev)
    gen.manual_seed(args.seed)
    # PD target offsets U(-0.5, 0.5), resampled every step, resident in HBM
    ctrl = (torch.rand(ns, nw, m.nu, device=dev, generator=gen) - 0.5).contiguous()
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

    # roofline of the step kernel: plain FP32 ALU work (no MFMA, not HBM bound)
    sample = min(nw, 64)
    flops_ws = algorithmic_flops_per_world_step(m, qp[:sample], qv[:sample],
                                                inputs.controls(kind, m, sample, 1, seed=1))
    achieved_tf = flops_ws * nw * ns / (kavg * 1e-3) / 1e12
    bytes_ws = 4.0 * m.nu + 4.0 * 2 * (m.nq + 2 * m.nv) / ns
    roof = {"bound": "alu", "achieved": round(achieved_tf, 4), "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved_tf / FP32_VECTOR_PEAK_TFLOPS, 6),
            "traffic": None,
            "kernel": "mjh_step_kernel", "kernel_ms": round(kavg, 3),
            "flops_per_world_step": round(flops_ws, 1),
            "hbm_bytes_per_world_step": round(bytes_ws, 2),
            "hbm_frac": round(bytes_ws * nw * ns / (kavg * 1e-3) / 1e9 / HBM_PEAK_GBS, 8)}
    out = {"metric": "world-steps/sec at 8192 quadruped worlds", "value": round(value, 1),
           "unit": "world-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic (seeded quadruped states, uniform random PD targets)",
           "config": {"workload": f"quadruped {nw} worlds x {ns} physics steps per launch",
                      "nworld": nw, "nstep_per_launch": ns, "dt": m.opt.timestep,
                      "newton_iterations": m.opt.iterations, "graph": bool(args.graph),
                      "launch": list(world.batch.get_launch(0)),
                      "status_nonzero_worlds": int(np.count_nonzero(status))},
           "roofline": roof}
    if not args.no_cpu_baseline:
        nthreads = min(os.cpu_count() or 1, 16)
        cw, cs = args.cpu_sample_worlds, args.cpu_sample_steps
        u = inputs.controls(kind, m, cw, cs, seed=args.seed)
        rate, secs = cpu_baseline(m, qp[:cw], qv[:cw], u, nthreads)
        out["cpu_baseline"] = {"value": round(rate, 1), "unit": "world-steps/s",
                               "cores": nthreads, "kind": "oracle",
                               "sample": f"{cw} quadruped worlds x {cs} steps, FP64, "
                                         f"{secs:.1f} s"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
