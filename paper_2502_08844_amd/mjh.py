"""Python binding of the mjh C ABI (ctypes; argument marshalling only).

Every numerical step runs in the HIP kernels of ``libmjh.so``.  PyTorch supplies device
memory and streams: state, controls and outputs are CUDA(HIP) float32 / int32 tensors
whose data pointers are passed straight through.  Importing this module loads the
library and raises if it has not been built; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# MJH_LIB_PATH selects another build of the same sources (e.g. a phase-timing build)
LIB_PATH = os.environ.get("MJH_LIB_PATH", os.path.join(_HERE, "libmjh.so"))
CON_SIZE = 20

OK, EINVAL, ENOMEM, EHIP, EMODEL, EUNSUPPORTED, ESTATE = 0, -1, -2, -3, -4, -5, -6
WORLD_NONFINITE, WORLD_OVERFLOW, WORLD_NODESCENT = 1, 2, 4

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                      "(hipcc --offload-arch=gfx950)")
_lib = C.CDLL(LIB_PATH)

P = C.c_void_p
I32 = C.c_int32
F = C.c_float


class Dims(C.Structure):
    _fields_ = [("nq", I32), ("nv", I32), ("nu", I32), ("nbody", I32), ("ngeom", I32),
                ("npair", I32), ("ncand", I32), ("nconmax", I32), ("iterations", I32),
                ("lds_bytes", I32), ("timestep", F), ("nlimit", I32), ("nrowmax", I32),
                ("nfric", I32), ("neq", I32)]


def _sig(name, *args):
    fn = getattr(_lib, name)
    fn.argtypes = list(args)
    fn.restype = I32
    return fn


mjh_create = _sig("mjh_create", C.c_int, C.POINTER(P))
_lib.mjh_destroy.argtypes = [P]
_lib.mjh_destroy.restype = None
_lib.mjh_last_error.argtypes = [P]
_lib.mjh_last_error.restype = C.c_char_p
mjh_model_upload = _sig("mjh_model_upload", P, C.c_char_p, C.c_size_t, C.POINTER(I32))
mjh_model_info = _sig("mjh_model_info", P, I32, C.POINTER(Dims))
mjh_model_invweight = _sig("mjh_model_invweight", P, I32, C.POINTER(F))
mjh_model_limit_invweight = _sig("mjh_model_limit_invweight", P, I32, C.POINTER(F))
mjh_world_alloc = _sig("mjh_world_alloc", P, C.POINTER(I32), C.POINTER(I32), I32, C.POINTER(P))
_lib.mjh_world_free.argtypes = [P]
_lib.mjh_world_free.restype = None
mjh_bind_state = _sig("mjh_bind_state", P, I32, P, P, P, P)
mjh_bind_io = _sig("mjh_bind_io", P, I32, P, I32, P, P)
mjh_step = _sig("mjh_step", P, I32, P)
mjh_graph_capture = _sig("mjh_graph_capture", P, I32, P)
mjh_graph_launch = _sig("mjh_graph_launch", P, P)
mjh_autotune = _sig("mjh_autotune", P, I32, C.c_char_p)
mjh_set_launch = _sig("mjh_set_launch", P, I32, I32, I32)
mjh_get_launch = _sig("mjh_get_launch", P, I32, C.POINTER(I32), C.POINTER(I32))
I64 = C.c_int64
mjh_rollout_fwd = _sig("mjh_rollout_fwd", P, I32, I32, P, I32, F, F, P, C.POINTER(I64), P)
mjh_rollout_bwd = _sig("mjh_rollout_bwd", P, I64, P, P, P, P)
mjh_rollout_noalloc = _sig("mjh_rollout_noalloc", P, I32, I32, P, I32, F, F, P, P, P, P, P)
mjh_env_step = _sig("mjh_env_step", P, I32, I32, P, P, P, P, P, P, P, P, P, P, P)


class MjhError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mjh error {code}: {msg}")
        self.code = code


def _ptr(t: Optional[torch.Tensor], dtype=torch.float32):
    if t is None:
        return None
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"expected a contiguous {dtype} device tensor, got "
                         f"{t.dtype} on {t.device} (contiguous={t.is_contiguous()})")
    return C.c_void_p(t.data_ptr())


def _stream(stream: Optional[torch.cuda.Stream]):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Context:
    """One library context on a HIP device."""

    def __init__(self, device: int = 0):
        torch.cuda.init()
        h = P()
        rc = mjh_create(int(device), C.byref(h))
        if rc != OK:
            raise MjhError(rc, f"mjh_create({device}) failed")
        self._h = h
        self._free = _lib.mjh_destroy
        self.device = device

    def check(self, rc: int):
        if rc != OK:
            raise MjhError(rc, _lib.mjh_last_error(self._h).decode())

    def close(self):
        # the library handle is held by the instance: module globals may already be
        # cleared when this runs at interpreter exit
        if getattr(self, "_h", None):
            self._free(self._h)
            self._h = None

    def __del__(self):
        self.close()

    # ---------------------------------------------------------------- models
    def model_upload(self, model_or_blob) -> "Model":
        blob = model_or_blob if isinstance(model_or_blob, (bytes, bytearray)) \
            else model_or_blob.to_blob()
        mid = I32()
        self.check(mjh_model_upload(self._h, bytes(blob), len(blob), C.byref(mid)))
        return Model(self, mid.value)

    def world_alloc(self, models: Sequence["Model"], counts: Sequence[int]) -> "Batch":
        n = len(models)
        ids = (I32 * n)(*[m.id for m in models])
        cnt = (I32 * n)(*[int(c) for c in counts])
        b = P()
        self.check(mjh_world_alloc(self._h, ids, cnt, n, C.byref(b)))
        return Batch(self, list(models), list(counts), b)


class Model:
    def __init__(self, ctx: Context, mid: int):
        self.ctx = ctx
        self.id = mid
        d = Dims()
        ctx.check(mjh_model_info(ctx._h, mid, C.byref(d)))
        self.dims = d
        self.nq, self.nv, self.nu = d.nq, d.nv, d.nu
        self.nconmax = d.nconmax
        self.nlimit, self.nrowmax, self.nfric, self.neq = d.nlimit, d.nrowmax, d.nfric, d.neq
        self.timestep = d.timestep

    def invweight(self):
        import numpy as np
        out = (F * self.dims.nbody)()
        self.ctx.check(mjh_model_invweight(self.ctx._h, self.id, out))
        return np.array(out[:], dtype=np.float64)

    def limit_invweight(self):
        """(M^-1)_kk at qpos0 of each limited joint's dof, in joint order."""
        import numpy as np
        out = (F * max(self.dims.nlimit, 1))()
        self.ctx.check(mjh_model_limit_invweight(self.ctx._h, self.id, out))
        return np.array(out[:self.dims.nlimit], dtype=np.float64)


@dataclass
class GroupState:
    qpos: torch.Tensor
    qvel: torch.Tensor
    qacc_ws: torch.Tensor
    status: Optional[torch.Tensor] = None


class Batch:
    """A set of world groups (one per model) stepped together in one launch."""

    def __init__(self, ctx: Context, models, counts, handle):
        self.ctx = ctx
        self.models = models
        self.counts = counts
        self._h = handle
        self._free = _lib.mjh_world_free
        self._state = [None] * len(models)
        self._io = [None] * len(models)

    def close(self):
        if getattr(self, "_h", None):
            self._free(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def bind_state(self, group: int, qpos, qvel, qacc_ws, status=None):
        key = tuple(None if t is None else t.data_ptr() for t in (qpos, qvel, qacc_ws, status))
        if self._state[group] is not None and self._state[group][0] == key:
            return
        self.ctx.check(mjh_bind_state(self._h, group, _ptr(qpos), _ptr(qvel), _ptr(qacc_ws),
                                      _ptr(status, torch.int32)))
        self._state[group] = (key, (qpos, qvel, qacc_ws, status))

    def bind_io(self, group: int, ctrl=None, contact_out=None, ncon_out=None):
        nstep = 0 if ctrl is None else int(ctrl.shape[0])
        key = (None if ctrl is None else ctrl.data_ptr(), nstep,
               None if contact_out is None else contact_out.data_ptr(),
               None if ncon_out is None else ncon_out.data_ptr())
        if self._io[group] is not None and self._io[group][0] == key:
            return
        self.ctx.check(mjh_bind_io(self._h, group, _ptr(ctrl), nstep, _ptr(contact_out),
                                   _ptr(ncon_out, torch.int32)))
        self._io[group] = (key, (ctrl, contact_out, ncon_out))

    def step(self, nstep: int, stream=None):
        self.ctx.check(mjh_step(self._h, int(nstep), _stream(stream)))

    def graph_capture(self, nstep: int, stream: torch.cuda.Stream):
        self.ctx.check(mjh_graph_capture(self._h, int(nstep), _stream(stream)))

    def graph_launch(self, stream=None):
        self.ctx.check(mjh_graph_launch(self._h, _stream(stream)))

    def autotune(self, nstep_probe: int = 20, cache_path: Optional[str] = None):
        self.ctx.check(mjh_autotune(self._h, int(nstep_probe),
                                    None if cache_path is None else cache_path.encode()))

    def set_launch(self, group: int, team: int, block: int):
        self.ctx.check(mjh_set_launch(self._h, group, team, block))

    def get_launch(self, group: int):
        t, b = I32(), I32()
        self.ctx.check(mjh_get_launch(self._h, group, C.byref(t), C.byref(b)))
        return t.value, b.value

    def rollout_fwd(self, horizon: int, ckpt_every: int, ctrl, zidx: int, ztarget: float,
                    wctrl: float, loss, stream=None) -> int:
        """Forward rollout; returns its generation number (rollout_bwd's key)."""
        if len(self.models) != 1:
            raise ValueError("rollouts take a single-model batch")
        nw, nu = self.counts[0], self.models[0].nu
        if ctrl is None or ctrl.numel() != horizon * nw * nu or loss.numel() != nw:
            raise ValueError(f"ctrl must be [{horizon}, {nw}, {nu}] and loss [{nw}]")
        gen = I64(0)
        self.ctx.check(mjh_rollout_fwd(self._h, int(horizon), int(ckpt_every), _ptr(ctrl),
                                       int(zidx), float(ztarget), float(wctrl), _ptr(loss),
                                       C.byref(gen), _stream(stream)))
        self._rollout = (int(horizon), nw, self.models[0].nv, nu, gen.value)
        return gen.value

    def env_step(self, nsub: int, action, command, reset_qpos, reset_qvel, last_action, obs,
                 reward, done, params=None, obs_noise=None, stream=None):
        """Joystick env steps of a single-model batch: action [nenv, nworld, nu], command
        [nworld, 3], reset_qpos/reset_qvel [nworld, nq]/[nworld, nv], last_action
        [nworld, nu] (read and updated); writes obs [nenv, nworld, 12 + 3 nu], reward and
        done [nenv, nworld].  The bound state advances nenv * nsub physics steps.
        params: per-world randomised parameters [nworld, 8 + 2 nu] or None; obs_noise:
        [nenv, nworld, 12 + 3 nu] added to obs, or None."""
        if len(self.models) != 1:
            raise ValueError("env steps take a single-model batch")
        m, nw = self.models[0], self.counts[0]
        nenv = action.shape[0] if action.dim() == 3 else 0
        shapes = ((action, (nenv, nw, m.nu)), (command, (nw, 3)), (reset_qpos, (nw, m.nq)),
                  (reset_qvel, (nw, m.nv)), (last_action, (nw, m.nu)),
                  (obs, (nenv, nw, 12 + 3 * m.nu)), (reward, (nenv, nw)), (done, (nenv, nw)))
        if params is not None:
            shapes += ((params, (nw, 8 + 2 * m.nu)),)
        if obs_noise is not None:
            shapes += ((obs_noise, (nenv, nw, 12 + 3 * m.nu)),)
        for t, shp in shapes:
            if tuple(t.shape) != shp or not t.is_contiguous():
                raise ValueError(f"env_step: expected a contiguous {shp}, got {tuple(t.shape)}")
        self.ctx.check(mjh_env_step(self._h, nenv, int(nsub), _ptr(action), _ptr(command),
                                    _ptr(reset_qpos), _ptr(reset_qvel), _ptr(params),
                                    _ptr(obs_noise), _ptr(last_action),
                                    _ptr(obs), _ptr(reward), _ptr(done, torch.int32),
                                    _stream(stream)))

    def rollout_bwd(self, dloss, grad_qvel0, grad_ctrl, stream=None, generation=None):
        """Adjoint of the rollout `generation` (default: the last rollout_fwd).  The
        library refuses any rollout but the last one (its tapes were overwritten)."""
        shp = getattr(self, "_rollout", None)
        if shp is None:
            raise ValueError("rollout_bwd needs a preceding rollout_fwd")
        horizon, nw, nv, nu, last = shp
        if (dloss.numel() != nw or grad_qvel0.numel() != nw * nv
                or grad_ctrl.numel() != horizon * nw * nu):
            raise ValueError(f"dloss [{nw}], grad_qvel0 [{nw}, {nv}], "
                             f"grad_ctrl [{horizon}, {nw}, {nu}] expected")
        gen = last if generation is None else int(generation)
        self.ctx.check(mjh_rollout_bwd(self._h, gen, _ptr(dloss), _ptr(grad_qvel0),
                                       _ptr(grad_ctrl), _stream(stream)))

    def rollout_noalloc(self, horizon: int, ckpt_every: int, ctrl, zidx: int, ztarget: float,
                        wctrl: float, dloss, loss, grad_qvel0, grad_ctrl, stream=None):
        """rollout_fwd then rollout_bwd in one library call that allocates no device
        memory (its tapes live in the library's static scratch).  Every tensor is
        caller-owned: ctrl [horizon, nworld, nu] and dloss [nworld] in; loss [nworld],
        grad_qvel0 [nworld, nv] and grad_ctrl [horizon, nworld, nu] out."""
        if len(self.models) != 1:
            raise ValueError("rollouts take a single-model batch")
        nw, nv, nu = self.counts[0], self.models[0].nv, self.models[0].nu
        if (ctrl is None or ctrl.numel() != horizon * nw * nu or loss.numel() != nw
                or dloss.numel() != nw or grad_qvel0.numel() != nw * nv
                or grad_ctrl.numel() != horizon * nw * nu):
            raise ValueError(f"ctrl [{horizon}, {nw}, {nu}], dloss and loss [{nw}], "
                             f"grad_qvel0 [{nw}, {nv}], grad_ctrl [{horizon}, {nw}, {nu}] "
                             "expected")
        self.ctx.check(mjh_rollout_noalloc(self._h, int(horizon), int(ckpt_every), _ptr(ctrl),
                                           int(zidx), float(ztarget), float(wctrl),
                                           _ptr(dloss), _ptr(loss), _ptr(grad_qvel0),
                                           _ptr(grad_ctrl), _stream(stream)))


# ------------------------------------------------------------------ convenience
class World:
    """Single-model convenience wrapper: owns the state tensors of nworld worlds."""

    def __init__(self, ctx: Context, model, nworld: int, qpos=None, qvel=None,
                 device="cuda"):
        self.model = model if isinstance(model, Model) else ctx.model_upload(model)
        m = self.model
        self.nworld = nworld
        self.batch = ctx.world_alloc([m], [nworld])
        z = dict(dtype=torch.float32, device=device)
        self.qpos = torch.zeros(nworld, m.nq, **z) if qpos is None else \
            torch.as_tensor(qpos, **z).contiguous()
        self.qvel = torch.zeros(nworld, m.nv, **z) if qvel is None else \
            torch.as_tensor(qvel, **z).contiguous()
        self.qacc_ws = torch.zeros(nworld, m.nv, **z)
        self.status = torch.zeros(nworld, dtype=torch.int32, device=device)
        self.batch.bind_state(0, self.qpos, self.qvel, self.qacc_ws, self.status)

    def step(self, ctrl=None, nstep: Optional[int] = None, contacts: bool = False,
             stream=None):
        """Advance nstep steps; ctrl is [nstep, nworld, nu] (device) or None."""
        if ctrl is not None:
            ctrl = torch.as_tensor(ctrl, dtype=torch.float32,
                                   device=self.qpos.device).contiguous()
            nstep = ctrl.shape[0] if nstep is None else nstep
        nstep = 1 if nstep is None else nstep
        con = ncon = None
        if contacts:
            m = self.model
            con = torch.zeros(self.nworld, max(m.nconmax, 1), CON_SIZE, dtype=torch.float32,
                              device=self.qpos.device)
            ncon = torch.zeros(self.nworld, dtype=torch.int32, device=self.qpos.device)
        self.batch.bind_io(0, ctrl, con, ncon)
        self.batch.step(nstep, stream)
        return (con, ncon) if contacts else None


class Rollout(torch.autograd.Function):
    """Differentiable rollout loss of a single-model World.

    forward(ctx, qvel0, ctrl, world, horizon, ckpt_every, zidx, ztarget, wctrl)
      -> loss [nworld]: sum_t (qpos_t[zidx] - ztarget)^2 + wctrl |ctrl_t|^2, starting from
      world.qpos with initial velocity qvel0 [nworld, nv] and controls ctrl
      [horizon, nworld, nu].  backward returns d(loss)/d(qvel0) and d(loss)/d(ctrl) from
      the library's adjoint (checkpointed every ckpt_every steps).
    The world's state is advanced to the final step by forward.
    """

    @staticmethod
    def forward(ctx, qvel0, ctrl, world, horizon, ckpt_every, zidx=2, ztarget=0.3,
                wctrl=1e-3):
        world.qvel.copy_(qvel0)
        ctrl = ctrl.contiguous()
        loss = torch.empty(world.nworld, dtype=torch.float32, device=qvel0.device)
        ctx.generation = world.batch.rollout_fwd(horizon, ckpt_every, ctrl, zidx, ztarget,
                                                 wctrl, loss)
        ctx.world = world
        ctx.save_for_backward(ctrl)
        return loss

    @staticmethod
    def backward(ctx, dloss):
        (ctrl,) = ctx.saved_tensors
        w = ctx.world
        gq = torch.empty(w.nworld, w.model.nv, dtype=torch.float32, device=dloss.device)
        gu = torch.empty_like(ctrl)
        # a later forward rollout of the same world overwrote the tapes: the library
        # refuses this backward (MJH_ESTATE) rather than return another rollout's gradient
        w.batch.rollout_bwd(dloss.contiguous().float(), gq, gu, generation=ctx.generation)
        return gq, gu, None, None, None, None, None, None


def rollout_fwd(world: World, ctrl, horizon: int, ckpt_every: int, zidx: int = 2,
                ztarget: float = 0.3, wctrl: float = 1e-3, stream=None):
    loss = torch.empty(world.nworld, dtype=torch.float32, device=world.qpos.device)
    world.batch.rollout_fwd(horizon, ckpt_every, ctrl, zidx, ztarget, wctrl, loss, stream)
    return loss


def rollout_bwd(world: World, dloss, horizon: int, stream=None):
    """Gradients (d loss/d qvel0 [nworld, nv], d loss/d ctrl [horizon, nworld, nu]) of the
    last rollout_fwd of this world, weighted by dloss [nworld]."""
    dev = world.qpos.device
    gq = torch.empty(world.nworld, world.model.nv, dtype=torch.float32, device=dev)
    gu = torch.empty(horizon, world.nworld, world.model.nu, dtype=torch.float32, device=dev)
    world.batch.rollout_bwd(dloss.contiguous().float(), gq, gu, stream)
    return gq, gu
