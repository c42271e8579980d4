"""Seeded synthetic inputs: initial states and control sequences.

Every array is drawn in float64 from numpy's counter-based Philox bit generator keyed by
(seed, stream) and then rounded to float32, so that the GPU library and the FP64
reference receive bit-identical starting values.  Random actions follow the paper's
raw-throughput benchmark (physics stepped with random actions); 8192 parallel worlds is
the environment count of its locomotion and manipulation PPO runs.

Streams: 1 initial qpos noise, 2 initial qvel, 3 controls.
"""
from __future__ import annotations

import numpy as np

from .model import Model
from . import robots

STREAM_QPOS, STREAM_QVEL, STREAM_CTRL = 1, 2, 3


def rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=[int(seed), int(stream)]))


def f32(x: np.ndarray) -> np.ndarray:
    """Round to float32 and return as float64 (the exact values both sides see)."""
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def initial_state(kind: str, m: Model, nworld: int, seed: int = 0):
    """(qpos [nworld, nq], qvel [nworld, nv]) for the named workload."""
    nq, nv = m.nq, m.nv
    qpos = np.tile(m.qpos0, (nworld, 1)).astype(np.float64)
    qvel = np.zeros((nworld, nv))
    r_q, r_v = rng(seed, STREAM_QPOS), rng(seed, STREAM_QVEL)
    if kind == "cartpole":
        qpos[:] = r_q.uniform(-0.1, 0.1, size=(nworld, nq))
        qvel[:] = r_v.uniform(-0.05, 0.05, size=(nworld, nv))
    elif kind.startswith("quadruped"):
        qpos[:, 7:] = np.tile(robots.QUAD_Q_DEFAULT, 4) + r_q.uniform(-0.2, 0.2,
                                                                        size=(nworld, 12))
    elif kind.startswith("humanoid"):
        qpos[:, 7:] += r_q.uniform(-0.1, 0.1, size=(nworld, nq - 7))
    elif kind.startswith("hand"):
        qpos[:, :16] += r_q.uniform(-0.1, 0.1, size=(nworld, 16))
    else:
        raise ValueError(kind)
    return f32(qpos), f32(qvel)


def controls(kind: str, m: Model, nworld: int, nstep: int, seed: int = 0) -> np.ndarray:
    """ctrl [nstep, nworld, nu], resampled every step."""
    r = rng(seed, STREAM_CTRL)
    shape = (nstep, nworld, m.nu)
    if kind == "cartpole":
        u = r.uniform(-1.0, 1.0, size=shape)
    elif kind.startswith("quadruped"):
        u = r.uniform(-0.5, 0.5, size=shape)
    elif kind.startswith("humanoid"):
        u = np.clip(r.normal(0.0, 0.3, size=shape), -1.0, 1.0)
    elif kind.startswith("hand"):
        u = r.uniform(-0.3, 0.3, size=shape)
    else:
        raise ValueError(kind)
    return f32(u)


def model(kind: str) -> Model:
    return robots.WORKLOADS[kind]()
