"""Model description and its flat binary form (the "model blob").

A model is a tree of rigid bodies with joints, collision geoms, an explicit list of
collision pairs and actuators, in the MJCF-like terms that the physics step of MuJoCo
Playground consumes (the paper's physics knobs are MJCF options: Table
``tab:dm_control_envs`` in the DM Control appendix, and the PD mapping of eq.
``pd_mapping``).  This module only stores and serialises the description; it holds none
of the step's arithmetic.  Both the FP64 reference and the GPU library parse the blob
with their own code.

Blob layout (little endian, version 3), every block 8-byte aligned:

  header   int32[16]  : magic 0x4D484A4D ('MJHM'), version, nbody, njnt, ngeom, npair,
                        nu, nq, nv, iterations, ls_iterations, nconmax, neq,
                        integrator (0 semi-implicit Euler, 1 with implicit damping, 2 also with
                        implicit PD position gains),
                        hfield (1 if the model has a heightfield),
                        cone (0 pyramidal, 1 elliptic friction cone)
           float64[16]: timestep, gravity[3], solref[2], solimp[5], tolerance, 0 x4
  body     int32 [nbody][2] : parent, 0
           f64   [nbody][19]: pos[3], quat[4] (w first), mass, ipos[3],
                              inertia[6] (Ixx Iyy Izz Ixy Ixz Iyz, body frame, about ipos),
                              0, 0
  joint    int32 [njnt][4]  : type (0 free, 1 slide, 2 hinge), body, limited (0/1), 0
           f64   [njnt][11] : pos[3], axis[3], damping, armature, range[2], frictionloss
  geom     int32 [ngeom][2] : type (0 plane, 1 sphere, 2 capsule, 3 box), body
           f64   [ngeom][11]: size[3], pos[3], quat[4], friction
  pair     int32 [npair][4] : geom1, geom2 (type(geom1) <= type(geom2)), condim (1, 3, 4, 6), 0
           f64   [npair][3] : friction coefficients: sliding mu, torsional, rolling
  actuator int32 [nu][2]    : type (0 motor, 1 position PD), joint
           f64   [nu][7]    : gear, kp, kd, ctrlrange[2], qdefault, 0
  equality int32 [neq][4]   : type (0 connect, 1 weld), body1, body2, 0
           f64   [neq][10]  : anchor in body1's frame[3], the same point in body2's frame[3],
                              body2's orientation in body1's frame when welded (quat[4])
  hfield   int32 [2]        : nrow, ncol (>= 2 each)            } only when header hfield = 1
           f64   [3]        : half extents sx, sy; height scale sz
           f64   [nrow][ncol] elevations in [0, 1] (row i at y = -sy + 2 sy i / (nrow - 1),
                             column j at x = -sx + 2 sx j / (ncol - 1), z = sz h)
  qpos0    f64   [nq]

A limited hinge or slide joint keeps its coordinate inside range[0] < q < range[1]
through a soft one-sided constraint (the joint-limit rows of the constraint set).  A
hinge or slide joint with frictionloss F > 0 gets a dry-friction row whose force is
bounded by F.

A connect equality holds a point of body1 on a point of body2 (a ball joint closing a
loop, or pinning a body to the world when body2 = 0): three always-present two-sided
rows.  A weld also holds body2's orientation relative to body1 at a reference
(three more rows).

A heightfield geom (type 4) is the model's heightfield surface, placed by the geom's
pose: each grid cell is split into the triangles (v_ij, v_i,j+1, v_i+1,j+1) and
(v_ij, v_i+1,j+1, v_i+1,j).  Only sphere-heightfield pairs are supported.

Geom sizes: sphere (r), capsule (r, half segment length; segment along local z),
box (half extents).  Plane normal is the geom's local +z.
"""
from __future__ import annotations

import struct
from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

MAGIC = 0x4D484A4D
VERSION = 3

JNT_FREE, JNT_SLIDE, JNT_HINGE = 0, 1, 2
GEOM_PLANE, GEOM_SPHERE, GEOM_CAPSULE, GEOM_BOX, GEOM_HFIELD = 0, 1, 2, 3, 4
ACT_MOTOR, ACT_PD = 0, 1
EQ_CONNECT, EQ_WELD = 0, 1

JNT_NQ = {JNT_FREE: 7, JNT_SLIDE: 1, JNT_HINGE: 1}
JNT_NV = {JNT_FREE: 6, JNT_SLIDE: 1, JNT_HINGE: 1}


@dataclass
class Body:
    parent: int
    pos: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    quat: Tuple[float, float, float, float] = (1.0, 0.0, 0.0, 0.0)
    mass: float = 0.0
    ipos: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    inertia: Tuple[float, ...] = (0.0, 0.0, 0.0, 0.0, 0.0, 0.0)
    name: str = ""


@dataclass
class Joint:
    type: int
    body: int
    pos: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    axis: Tuple[float, float, float] = (0.0, 0.0, 1.0)
    damping: float = 0.0
    armature: float = 0.0
    limited: bool = False
    range: Tuple[float, float] = (0.0, 0.0)
    frictionloss: float = 0.0
    name: str = ""


@dataclass
class Geom:
    type: int
    body: int
    size: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    pos: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    quat: Tuple[float, float, float, float] = (1.0, 0.0, 0.0, 0.0)
    friction: float = 1.0
    name: str = ""


@dataclass
class Actuator:
    type: int
    joint: int
    gear: float = 1.0
    kp: float = 0.0
    kd: float = 0.0
    ctrlrange: Tuple[float, float] = (-1.0, 1.0)
    qdefault: float = 0.0


@dataclass
class Equality:
    type: int
    body1: int
    body2: int
    anchor1: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    anchor2: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    relquat: Tuple[float, float, float, float] = (1.0, 0.0, 0.0, 0.0)  # weld only


@dataclass
class Heightfield:
    nrow: int
    ncol: int
    size: Tuple[float, float, float]  # half extents x, y and the height scale
    data: np.ndarray = None           # [nrow, ncol] elevations in [0, 1]


@dataclass
class Options:
    timestep: float = 0.002
    gravity: Tuple[float, float, float] = (0.0, 0.0, -9.81)
    solref: Tuple[float, float] = (0.02, 1.0)
    solimp: Tuple[float, float, float, float, float] = (0.9, 0.95, 0.001, 0.5, 2.0)
    tolerance: float = 1e-8
    iterations: int = 4
    ls_iterations: int = 8
    nconmax: int = 0
    integrator: int = 0  # 1: joint damping and PD velocity gains taken implicitly;
                         # 2: also the PD position gains (at the end-of-step position)
    cone: int = 0        # friction cone: 0 pyramidal (2 (condim - 1) edge rows a contact),
                         # 1 elliptic (the contact frame's condim rows)


@dataclass
class Model:
    name: str
    bodies: List[Body] = field(default_factory=list)
    joints: List[Joint] = field(default_factory=list)
    geoms: List[Geom] = field(default_factory=list)
    # (geom1, geom2, mu[, condim[, mu_torsion[, mu_rolling]]]): condim 3 (default) is
    # the sliding-friction pyramid, 1 a frictionless contact (one normal row), 4 adds
    # torsional friction about the normal and 6 rolling friction about the tangents
    pairs: List[tuple] = field(default_factory=list)
    actuators: List[Actuator] = field(default_factory=list)
    equalities: List[Equality] = field(default_factory=list)
    hfield: Heightfield = None
    opt: Options = field(default_factory=Options)
    qpos0: np.ndarray = None

    # ------------------------------------------------------------------ sizes
    @property
    def nbody(self) -> int:
        return len(self.bodies)

    @property
    def nq(self) -> int:
        return sum(JNT_NQ[j.type] for j in self.joints)

    @property
    def nv(self) -> int:
        return sum(JNT_NV[j.type] for j in self.joints)

    @property
    def nu(self) -> int:
        return len(self.actuators)

    @property
    def nfric(self) -> int:
        """Dofs with friction loss: one constraint row each, always present."""
        return sum(1 for j in self.joints if j.frictionloss > 0)

    @property
    def neq(self) -> int:
        return len(self.equalities)

    @property
    def neqrow(self) -> int:
        """Equality rows: three per connect, six per weld."""
        return sum(6 if e.type == EQ_WELD else 3 for e in self.equalities)

    @property
    def conrows(self) -> int:
        """Rows of the model's widest contact: 1 frictionless; 2 (condim - 1) pyramid
        edges, or condim frame rows with the elliptic cone."""
        cd = [p[3] if len(p) > 3 else 3 for p in self.pairs]
        if self.opt.cone == 1:
            return max(cd, default=3)
        return max([1 if c == 1 else 2 * (c - 1) for c in cd], default=4)

    @property
    def nrowmax(self) -> int:
        return self.conrows * self.opt.nconmax + self.nlimit + self.nfric + self.neqrow

    @property
    def nlimit(self) -> int:
        """Limited joints: each adds at most one constraint row (one side at a time)."""
        return sum(1 for j in self.joints if j.limited)

    def jnt_qposadr(self) -> List[int]:
        out, a = [], 0
        for j in self.joints:
            out.append(a)
            a += JNT_NQ[j.type]
        return out

    def jnt_dofadr(self) -> List[int]:
        out, a = [], 0
        for j in self.joints:
            out.append(a)
            a += JNT_NV[j.type]
        return out

    def total_mass(self) -> float:
        return float(sum(b.mass for b in self.bodies))

    # -------------------------------------------------------------- validity
    def validate(self) -> None:
        assert self.bodies and self.bodies[0].parent == -1, "body 0 must be the world"
        for i, b in enumerate(self.bodies[1:], start=1):
            assert 0 <= b.parent < i, f"body {i}: parent must precede child"
        last = 0
        for j in self.joints:
            assert j.body >= last, "joints must be grouped by body in body order"
            last = j.body
            if j.type == JNT_FREE:
                assert self.bodies[j.body].parent == 0, "free joints attach to the world"
                assert sum(1 for k in self.joints if k.body == j.body) == 1
                assert not j.limited, "free joints have no limits"
            if j.limited:
                assert j.range[0] < j.range[1], "limited joint needs range[0] < range[1]"
            assert j.frictionloss >= 0 and (j.type != JNT_FREE or j.frictionloss == 0), \
                "friction loss needs a hinge or slide joint"
        for e in self.equalities:
            assert e.type in (EQ_CONNECT, EQ_WELD), "connect and weld equalities only"
            assert 0 < e.body1 < self.nbody and 0 <= e.body2 < self.nbody
            assert e.body1 != e.body2
        assert self.opt.cone in (0, 1), "cone 0 (pyramidal) or 1 (elliptic)"
        for g1, g2, *rest in self.pairs:
            assert len(rest) == 1 or rest[1] in (1, 3, 4, 6), "pair condim 1, 3, 4 or 6"
            cd = rest[1] if len(rest) > 1 else 3
            if self.opt.cone == 1 and cd >= 3:
                assert rest[0] > 0 and all(mu > 0 for mu in rest[2:cd - 1]), \
                    "elliptic cones need positive friction coefficients"
            assert self.geoms[g1].type <= self.geoms[g2].type, "pair order by geom type"
            if self.geoms[g2].type == GEOM_HFIELD:
                assert self.geoms[g1].type == GEOM_SPHERE, "heightfields pair with spheres"
                assert self.hfield is not None
        if self.hfield is not None:
            hf = self.hfield
            assert hf.nrow >= 2 and hf.ncol >= 2 and hf.data.shape == (hf.nrow, hf.ncol)
        assert self.qpos0 is not None and len(self.qpos0) == self.nq

    # ---------------------------------------------------------------- to blob
    def to_blob(self) -> bytes:
        self.validate()
        o = self.opt
        hdr_i = [MAGIC, VERSION, self.nbody, len(self.joints), len(self.geoms),
                 len(self.pairs), self.nu, self.nq, self.nv, o.iterations,
                 o.ls_iterations, o.nconmax, self.neq, o.integrator,
                 int(self.hfield is not None), o.cone]
        hdr_f = [o.timestep, *o.gravity, *o.solref, *o.solimp, o.tolerance, 0, 0, 0, 0]
        assert len(hdr_f) == 16
        parts = [struct.pack("<16i", *hdr_i), struct.pack("<16d", *hdr_f)]

        def blk_i(rows):
            a = np.asarray(rows, dtype="<i4").reshape(-1)
            return a.tobytes()

        def blk_f(rows):
            a = np.asarray(rows, dtype="<f8").reshape(-1)
            return a.tobytes()

        parts.append(blk_i([[b.parent, 0] for b in self.bodies]))
        parts.append(blk_f([[*b.pos, *b.quat, b.mass, *b.ipos, *b.inertia, 0, 0]
                            for b in self.bodies]))
        parts.append(blk_i([[j.type, j.body, int(bool(j.limited)), 0] for j in self.joints]))
        parts.append(blk_f([[*j.pos, *j.axis, j.damping, j.armature, *j.range,
                             j.frictionloss] for j in self.joints]))
        parts.append(blk_i([[g.type, g.body] for g in self.geoms]))
        parts.append(blk_f([[*g.size, *g.pos, *g.quat, g.friction] for g in self.geoms]))
        parts.append(blk_i([[p[0], p[1], p[3] if len(p) > 3 else 3, 0] for p in self.pairs]))
        parts.append(blk_f([[p[2], p[4] if len(p) > 4 else 0.0, p[5] if len(p) > 5 else 0.0]
                            for p in self.pairs]))
        parts.append(blk_i([[a.type, a.joint] for a in self.actuators]))
        parts.append(blk_f([[a.gear, a.kp, a.kd, *a.ctrlrange, a.qdefault, 0]
                            for a in self.actuators]))
        parts.append(blk_i([[e.type, e.body1, e.body2, 0] for e in self.equalities]))
        parts.append(blk_f([[*e.anchor1, *e.anchor2, *e.relquat] for e in self.equalities]))
        if self.hfield is not None:
            hf = self.hfield
            parts.append(blk_i([hf.nrow, hf.ncol]))
            parts.append(blk_f(list(hf.size)))
            parts.append(blk_f(np.asarray(hf.data, dtype=np.float64)))
        parts.append(blk_f(np.asarray(self.qpos0, dtype=np.float64)))
        return b"".join(parts)
