"""ctypes wrapper of the FP64 reference library ``libmjo.so`` (built from mjo.cpp).

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the benchmark's
CPU-baseline leg; never by the GPU path.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
CON_SIZE = 20  # dist, pos[3], frame[9], f_n, f_t1, f_t2, pair, sub, geom1, geom2
MODE_FIXED, MODE_CONVERGED = 0, 1


def lib_path() -> str:
    return os.path.join(_HERE, "libmjo.so")


def build(verbose: bool = False) -> str:
    """Compile the reference library with g++ (FP64, -O2)."""
    src = os.path.join(_HERE, "mjo.cpp")
    out = lib_path()
    cmd = ["g++", "-O2", "-std=c++17", "-shared", "-fPIC", src, "-o", out + ".tmp",
           "-lpthread"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(lib_path()):
            build()
        lib = C.CDLL(lib_path())
        P = C.c_void_p
        D = C.POINTER(C.c_double)
        I = C.POINTER(C.c_int)
        lib.mjo_load.restype = P
        lib.mjo_load.argtypes = [C.c_char_p, C.c_long, C.c_char_p, C.c_int]
        lib.mjo_free.argtypes = [P]
        lib.mjo_dims.argtypes = [P, I]
        lib.mjo_body_invweight.argtypes = [P, D]
        lib.mjo_dof_invweight.argtypes = [P, D]
        lib.mjo_dof_parent.argtypes = [P, I]
        lib.mjo_set_invweight.argtypes = [P, D, D]
        lib.mjo_step.argtypes = [P, C.c_int, C.c_int, D, D, D, D, C.c_int, C.c_int, D, D, I,
                                 I, D]
        lib.mjo_forward.argtypes = [P, D, D, D, D, C.c_int] + [D] * 12 + [I, D, I, D, D, D,
                                                                         D, I]
        lib.mjo_inverse.argtypes = [P, D, D, D, D]
        lib.mjo_cost.argtypes = [P, D, D, D, D]
        lib.mjo_cost.restype = C.c_double
        lib.mjo_ltdl_solve.argtypes = [P, D, D, D, D]
        lib.mjo_point_jac.argtypes = [P, D, C.c_int, D, D]
        lib.mjo_rollout_loss.argtypes = [P, C.c_int, C.c_int, D, D, D, D, C.c_double,
                                         C.c_double, C.c_int, C.c_int, C.c_int, D]
        lib.mjo_rollout_jvp.argtypes = [P, C.c_int, C.c_int, D, D, D, D, D, D, C.c_double,
                                        C.c_double, C.c_int, C.c_int, C.c_int, D, D]
        lib.mjo_step_jvp.argtypes = [P, D, D, D, D, D, D, D, C.c_int, D, D, D, D]
        lib.mjo_trajectory.argtypes = [P, C.c_int, D, D, D, D, C.c_int, D, D, I]
        lib.mjo_count_flops.argtypes = [P, C.c_int, D, D, D, D]
        lib.mjo_count_flops.restype = C.c_double
        lib.mjo_set_capsule_box_tolerances.argtypes = [C.c_double, C.c_double, D]
        lib.mjo_set_capsule_box_tolerances.restype = None
        lib.mjo_count_flops2.argtypes = [P, C.c_int, D, D, D, D, D]
        lib.mjo_count_flops2.restype = C.c_double
        _lib = lib
    return _lib


def _d(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_int))


def _arr(x, n=None):
    if x is None:
        return None
    a = np.ascontiguousarray(x, dtype=np.float64)
    if n is not None:
        assert a.size == n, (a.shape, n)
    return a


def set_capsule_box_tolerances(tau: float, flat: float):
    """Set the capsule-box bracket tolerances (defaults 1e-5 and 1e-3); returns the
    previous pair.  For tests of the contacts' independence from them."""
    prev = np.zeros(2)
    _load().mjo_set_capsule_box_tolerances(float(tau), float(flat), _d(prev))
    return float(prev[0]), float(prev[1])


class Oracle:
    """One parsed model in the FP64 reference."""

    def __init__(self, model_or_blob):
        blob = model_or_blob if isinstance(model_or_blob, (bytes, bytearray)) \
            else model_or_blob.to_blob()
        self._lib = _load()
        err = C.create_string_buffer(256)
        self._h = self._lib.mjo_load(bytes(blob), len(blob), err, 256)
        if not self._h:
            raise ValueError("oracle rejected model: " + err.value.decode())
        dims = np.zeros(15, dtype=np.int32)
        self._lib.mjo_dims(self._h, _i(dims))
        (self.nq, self.nv, self.nu, self.nbody, self.njnt, self.ngeom, self.npair,
         self.nconmax, self.iterations, self.ls_iterations, self.nlimit, self.nfric,
         self.neq, self.neqrow, self.conrows) = (int(x) for x in dims)
        self.nrowmax = self.conrows * self.nconmax + self.nlimit + self.nfric + self.neqrow

    def __del__(self):
        if getattr(self, "_h", None):
            self._lib.mjo_free(self._h)
            self._h = None

    # ------------------------------------------------------------ model constants
    def body_invweight(self) -> np.ndarray:
        out = np.zeros(self.nbody)
        self._lib.mjo_body_invweight(self._h, _d(out))
        return out

    def dof_invweight(self) -> np.ndarray:
        """(M^-1)_kk at qpos0, the A of a joint-limit row on dof k."""
        out = np.zeros(self.nv)
        self._lib.mjo_dof_invweight(self._h, _d(out))
        return out

    def set_invweight(self, body, dof):
        """Use these inverse weights (e.g. a nominal model's) in every row's regulariser."""
        b, d = _arr(body, self.nbody), _arr(dof, self.nv)
        self._lib.mjo_set_invweight(self._h, _d(b), _d(d))

    def dof_parent(self) -> np.ndarray:
        out = np.zeros(self.nv, dtype=np.int32)
        self._lib.mjo_dof_parent(self._h, _i(out))
        return out

    # ------------------------------------------------------------------ stepping
    def step(self, qpos, qvel, qacc_ws=None, ctrl=None, nstep=1, mode=MODE_FIXED,
             nthreads=1):
        """Advance [nworld] worlds nstep steps.  ctrl is [nstep, nworld, nu] or None."""
        qpos = np.array(qpos, dtype=np.float64, order="C", ndmin=2)
        qvel = np.array(qvel, dtype=np.float64, order="C", ndmin=2)
        nw = qpos.shape[0]
        ws = np.zeros((nw, self.nv)) if qacc_ws is None else \
            np.array(qacc_ws, dtype=np.float64, order="C", ndmin=2)
        u = None if ctrl is None else _arr(ctrl, nstep * nw * self.nu)
        out = dict(qacc=np.zeros((nw, self.nv)), qacc_smooth=np.zeros((nw, self.nv)),
                   status=np.zeros(nw, dtype=np.int32), ncon=np.zeros(nw, dtype=np.int32),
                   contacts=np.zeros((nw, max(self.nconmax, 1), CON_SIZE)))
        self._lib.mjo_step(self._h, nw, nstep, _d(qpos), _d(qvel), _d(ws), _d(u), mode,
                           nthreads, _d(out["qacc"]), _d(out["qacc_smooth"]),
                           _i(out["status"]), _i(out["ncon"]), _d(out["contacts"]))
        out.update(qpos=qpos, qvel=qvel, qacc_ws=ws)
        return out

    def forward(self, qpos, qvel=None, qacc_ws=None, ctrl=None, mode=MODE_FIXED):
        """All intermediates of one forward evaluation of a single world."""
        nv, nb, nc = self.nv, self.nbody, max(self.nconmax, 1)
        nr = max(self.nrowmax, 1)
        qpos = _arr(qpos, self.nq)
        qvel = _arr(qvel, nv) if qvel is not None else np.zeros(nv)
        ws = _arr(qacc_ws, nv) if qacc_ws is not None else np.zeros(nv)
        u = _arr(ctrl, self.nu) if ctrl is not None else np.zeros(max(self.nu, 1))
        o = dict(xpos=np.zeros((nb, 3)), xmat=np.zeros((nb, 3, 3)), xipos=np.zeros((nb, 3)),
                 cdof=np.zeros((nv, 6)), cvel=np.zeros((nb, 6)), M=np.zeros((nv, nv)),
                 bias=np.zeros(nv), act=np.zeros(nv), passive=np.zeros(nv),
                 qacc_smooth=np.zeros(nv), qacc=np.zeros(nv), qfrc_con=np.zeros(nv),
                 contacts=np.zeros((nc, CON_SIZE)), J=np.zeros((nr, nv)),
                 aref=np.zeros(nr), D=np.zeros(nr), efc_force=np.zeros(nr))
        ncon = np.zeros(1, dtype=np.int32)
        nrow = np.zeros(1, dtype=np.int32)
        status = np.zeros(1, dtype=np.int32)
        self._lib.mjo_forward(self._h, _d(qpos), _d(qvel), _d(ws), _d(u), mode,
                              _d(o["xpos"]), _d(o["xmat"]), _d(o["xipos"]), _d(o["cdof"]),
                              _d(o["cvel"]), _d(o["M"]), _d(o["bias"]), _d(o["act"]),
                              _d(o["passive"]), _d(o["qacc_smooth"]), _d(o["qacc"]),
                              _d(o["qfrc_con"]), _i(ncon), _d(o["contacts"]), _i(nrow),
                              _d(o["J"]), _d(o["aref"]), _d(o["D"]), _d(o["efc_force"]),
                              _i(status))
        k, r = int(ncon[0]), int(nrow[0])
        o["ncon"], o["nrow"], o["status"] = k, r, int(status[0])
        o["contacts"] = o["contacts"][:k]
        for key in ("J", "aref", "D", "efc_force"):
            o[key] = o[key][:r]
        return o

    def cost(self, qpos, qvel, ctrl, a) -> float:
        """The Newton cost F(a) of one world's step from (qpos, qvel) under ctrl."""
        u = _arr(ctrl, self.nu) if ctrl is not None else np.zeros(max(self.nu, 1))
        return float(self._lib.mjo_cost(self._h, _d(_arr(qpos, self.nq)),
                                        _d(_arr(qvel, self.nv)), _d(u), _d(_arr(a, self.nv))))

    def inverse(self, qpos, qvel, qacc) -> np.ndarray:
        tau = np.zeros(self.nv)
        self._lib.mjo_inverse(self._h, _d(_arr(qpos, self.nq)), _d(_arr(qvel, self.nv)),
                              _d(_arr(qacc, self.nv)), _d(tau))
        return tau

    def ltdl_solve(self, qpos, b):
        x = np.zeros(self.nv)
        LD = np.zeros((self.nv, self.nv))
        self._lib.mjo_ltdl_solve(self._h, _d(_arr(qpos, self.nq)), _d(_arr(b, self.nv)),
                                 _d(x), _d(LD))
        return x, LD

    def point_jac(self, qpos, body, point) -> np.ndarray:
        J = np.zeros((3, self.nv))
        self._lib.mjo_point_jac(self._h, _d(_arr(qpos, self.nq)), int(body),
                                _d(_arr(point, 3)), _d(J))
        return J

    # ---------------------------------------------------------------- rollouts
    def rollout_loss(self, qpos, qvel, ctrl_seq, qacc_ws=None, ztarget=0.3, wctrl=1e-3,
                     mode=MODE_FIXED, zidx=2, nthreads=8):
        qpos = np.array(qpos, dtype=np.float64, order="C", ndmin=2)
        qvel = np.array(qvel, dtype=np.float64, order="C", ndmin=2)
        nw = qpos.shape[0]
        u = np.ascontiguousarray(ctrl_seq, dtype=np.float64)
        H = u.shape[0]
        ws = None if qacc_ws is None else np.ascontiguousarray(qacc_ws, dtype=np.float64)
        loss = np.zeros(nw)
        self._lib.mjo_rollout_loss(self._h, nw, H, _d(qpos), _d(qvel), _d(ws), _d(u),
                                   ztarget, wctrl, mode, zidx, nthreads, _d(loss))
        return loss

    def rollout_jvp(self, qpos, qvel, ctrl_seq, dqvel, dctrl, qacc_ws=None, ztarget=0.3,
                    wctrl=1e-3, mode=MODE_FIXED, zidx=2, nthreads=8):
        qpos = np.array(qpos, dtype=np.float64, order="C", ndmin=2)
        qvel = np.array(qvel, dtype=np.float64, order="C", ndmin=2)
        nw = qpos.shape[0]
        u = np.ascontiguousarray(ctrl_seq, dtype=np.float64)
        H = u.shape[0]
        ws = None if qacc_ws is None else np.ascontiguousarray(qacc_ws, dtype=np.float64)
        loss, dloss = np.zeros(nw), np.zeros(nw)
        self._lib.mjo_rollout_jvp(self._h, nw, H, _d(qpos), _d(qvel), _d(ws), _d(u),
                                  _d(_arr(dqvel, nw * self.nv)), _d(_arr(dctrl, u.size)),
                                  ztarget, wctrl, mode, zidx, nthreads, _d(loss), _d(dloss))
        return loss, dloss

    def step_jvp(self, qpos, qvel, qacc_ws, ctrl, dqpos, dqvel, dctrl, mode=MODE_FIXED):
        out = [np.zeros(self.nq), np.zeros(self.nv), np.zeros(self.nq), np.zeros(self.nv)]
        self._lib.mjo_step_jvp(self._h, _d(_arr(qpos, self.nq)), _d(_arr(qvel, self.nv)),
                               _d(_arr(qacc_ws, self.nv) if qacc_ws is not None else None),
                               _d(_arr(ctrl, self.nu) if ctrl is not None else None),
                               _d(_arr(dqpos, self.nq) if dqpos is not None else None),
                               _d(_arr(dqvel, self.nv) if dqvel is not None else None),
                               _d(_arr(dctrl, self.nu) if dctrl is not None else None),
                               mode, *(_d(a) for a in out))
        return tuple(out)

    def trajectory(self, qpos, qvel, nstep, qacc_ws=None, ctrl=None, mode=MODE_FIXED):
        """One world for nstep steps; returns (qpos [nstep, nq], qvel [nstep, nv], status)."""
        tq = np.zeros((nstep, self.nq))
        tv = np.zeros((nstep, self.nv))
        st = np.zeros(1, dtype=np.int32)
        self._lib.mjo_trajectory(self._h, int(nstep), _d(_arr(qpos, self.nq)),
                                 _d(_arr(qvel, self.nv)),
                                 _d(_arr(qacc_ws, self.nv) if qacc_ws is not None else None),
                                 _d(_arr(ctrl, nstep * self.nu) if ctrl is not None else None),
                                 mode, _d(tq), _d(tv), _i(st))
        return tq, tv, int(st[0])

    def count_flops(self, qpos, qvel, qacc_ws=None, ctrl=None, nonzero=False) -> float:
        """Average floating-point operations of one reference step from each state: every
        operation of the dense loops, or with nonzero=True those whose operands are all
        nonzero (products and sums with an exact zero are free to a sparse
        implementation).  ctrl is [nworld, nu] or [1, nworld, nu]."""
        qpos = np.array(qpos, dtype=np.float64, order="C", ndmin=2)
        qvel = np.array(qvel, dtype=np.float64, order="C", ndmin=2)
        nw = qpos.shape[0]
        ws = None if qacc_ws is None else np.ascontiguousarray(qacc_ws, dtype=np.float64)
        u = None if ctrl is None else np.ascontiguousarray(ctrl, dtype=np.float64).reshape(
            nw, self.nu)
        nz = np.zeros(1)
        dense = float(self._lib.mjo_count_flops2(self._h, nw, _d(qpos), _d(qvel), _d(ws), _d(u),
                                                 _d(nz)))
        return float(nz[0]) if nonzero else dense
