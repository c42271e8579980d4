"""Synthetic robots shaped like the paper's workloads.

The paper trains on MuJoCo Menagerie robots and DM Control tasks (its sections on DM
Control, locomotion and manipulation environments).  Those asset files are not part of
this project, so these generic models stand in for them, with the shapes the workloads
need:

* ``cartpole``  -- slider cart plus hinged capsule pole (DM Control CartpoleBalance).
* ``quadruped`` -- free torso and 4 legs of 3 hinges with sphere feet; only the feet
  collide with the floor, the reduced collision model the paper uses for joystick
  policies (locomotion section, feet-only contacts).
* ``humanoid``  -- free torso plus 21 hinges over 13 capsule bodies, floor contacts and
  self-contacts between non-adjacent bodies, timestep 0.005 as in the DM Control
  humanoid edits (Table ``tab:dm_control_envs``).
* ``hand``      -- 4 fingers of 4 hinges above a palm (the floor) and a free cube; finger
  joints carry the gearbox armature I_a = k_g^2 I_r of the LEAP-hand system
  identification (manipulation appendix): k_g = 288.35, I_r = 1/2 m_r r_r^2 with
  m_r = 2.0e-3 kg and r_r = 4.12e-3 m.

Mass properties are uniform-density solids (standard closed forms; a capsule is a
cylinder plus two hemispheres).  Nothing here is the physics step.
"""
from __future__ import annotations

import math
from typing import List, Sequence, Tuple

import numpy as np

from .model import (EQ_WELD, ACT_MOTOR, ACT_PD, EQ_CONNECT, GEOM_BOX, GEOM_CAPSULE, GEOM_HFIELD,
                    GEOM_PLANE, GEOM_SPHERE, JNT_FREE, JNT_HINGE, JNT_SLIDE, Actuator, Body,
                    Equality, Geom, Heightfield, Joint, Model, Options)

# ----------------------------------------------------------------------------------
# closed-form mass properties (uniform density)


def capsule_volume(r: float, half_len: float) -> float:
    return math.pi * r * r * (2.0 * half_len) + 4.0 / 3.0 * math.pi * r ** 3


def sphere_volume(r: float) -> float:
    return 4.0 / 3.0 * math.pi * r ** 3


def box_volume(half: Sequence[float]) -> float:
    return 8.0 * half[0] * half[1] * half[2]


def capsule_inertia(mass: float, r: float, half_len: float) -> np.ndarray:
    """Principal inertia about the centre, segment along local z (cylinder + 2 caps)."""
    L = 2.0 * half_len
    vc = math.pi * r * r * L
    vs = 4.0 / 3.0 * math.pi * r ** 3
    mc = mass * vc / (vc + vs)
    ms = mass * vs / (vc + vs)
    h = half_len
    i_axis = mc * r * r / 2.0 + ms * 2.0 * r * r / 5.0
    i_perp = mc * (r * r / 4.0 + L * L / 12.0) + ms * (2.0 * r * r / 5.0 + h * h + 0.75 * h * r)
    return np.diag([i_perp, i_perp, i_axis])


def box_inertia(mass: float, half: Sequence[float]) -> np.ndarray:
    a, b, c = (2.0 * x for x in half)
    return np.diag([mass * (b * b + c * c) / 12.0, mass * (a * a + c * c) / 12.0,
                    mass * (a * a + b * b) / 12.0])


def sphere_inertia(mass: float, r: float) -> np.ndarray:
    return np.eye(3) * (0.4 * mass * r * r)


# ----------------------------------------------------------------------------------
# small rotation helpers for building models


def quat_to_mat(q: Sequence[float]) -> np.ndarray:
    w, x, y, z = np.asarray(q, dtype=np.float64) / np.linalg.norm(q)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def quat_z_to(u: Sequence[float]) -> Tuple[float, float, float, float]:
    """Unit quaternion rotating local +z onto direction u."""
    u = np.asarray(u, dtype=np.float64)
    u = u / np.linalg.norm(u)
    z = np.array([0.0, 0.0, 1.0])
    c = float(np.dot(z, u))
    if c > 1.0 - 1e-15:
        return (1.0, 0.0, 0.0, 0.0)
    if c < -1.0 + 1e-15:
        return (0.0, 1.0, 0.0, 0.0)
    ax = np.cross(z, u)
    ax /= np.linalg.norm(ax)
    ang = math.acos(c)
    s = math.sin(ang / 2)
    return (math.cos(ang / 2), ax[0] * s, ax[1] * s, ax[2] * s)


def axis_angle_quat(axis: Sequence[float], ang: float) -> Tuple[float, float, float, float]:
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    s = math.sin(ang / 2)
    return (math.cos(ang / 2), a[0] * s, a[1] * s, a[2] * s)


def mat_to_quat(R) -> Tuple[float, float, float, float]:
    """Unit quaternion (w, x, y, z), w >= 0, of a rotation matrix (largest-pivot form)."""
    R = np.asarray(R, dtype=np.float64)
    tr = R[0, 0] + R[1, 1] + R[2, 2]
    if tr > 0:
        w = math.sqrt(1.0 + tr) * 2
        q = (0.25 * w, (R[2, 1] - R[1, 2]) / w, (R[0, 2] - R[2, 0]) / w, (R[1, 0] - R[0, 1]) / w)
    else:
        i = int(np.argmax(np.diag(R)))
        j, k = (i + 1) % 3, (i + 2) % 3
        s = math.sqrt(1.0 + R[i, i] - R[j, j] - R[k, k]) * 2
        v = [0.0, 0.0, 0.0]
        v[i] = 0.25 * s
        v[j] = (R[j, i] + R[i, j]) / s
        v[k] = (R[k, i] + R[i, k]) / s
        q = ((R[k, j] - R[j, k]) / s, *v)
    q = np.asarray(q) / np.linalg.norm(q)
    return tuple(float(x) for x in (q if q[0] >= 0 else -q))


class _Builder:
    """Accumulates bodies/geoms and derives each body's mass properties from its geoms."""

    def __init__(self, name: str):
        self.m = Model(name=name)
        self.m.bodies.append(Body(parent=-1, name="world"))
        self._geom_mass: List[Tuple[int, float, np.ndarray, np.ndarray, np.ndarray]] = []

    def body(self, parent: int, pos=(0, 0, 0), quat=(1, 0, 0, 0), name="") -> int:
        self.m.bodies.append(Body(parent=parent, pos=tuple(map(float, pos)),
                                  quat=tuple(map(float, quat)), name=name))
        return len(self.m.bodies) - 1

    def joint(self, body: int, type: int, axis=(0, 0, 1), pos=(0, 0, 0), damping=0.0,
              armature=0.0, range=None, frictionloss=0.0, name="") -> int:
        self.m.joints.append(Joint(type=type, body=body, pos=tuple(map(float, pos)),
                                   axis=tuple(map(float, axis)), damping=float(damping),
                                   armature=float(armature), limited=range is not None,
                                   range=(0.0, 0.0) if range is None else
                                   (float(range[0]), float(range[1])),
                                   frictionloss=float(frictionloss), name=name))
        return len(self.m.joints) - 1

    def geom(self, body: int, type: int, size, pos=(0, 0, 0), quat=(1, 0, 0, 0),
             mass: float = 0.0, friction: float = 1.0, name="") -> int:
        size = tuple(float(s) for s in size) + (0.0,) * (3 - len(size))
        self.m.geoms.append(Geom(type=type, body=body, size=size,
                                 pos=tuple(map(float, pos)), quat=tuple(map(float, quat)),
                                 friction=float(friction), name=name))
        gid = len(self.m.geoms) - 1
        if mass > 0.0:
            if type == GEOM_SPHERE:
                ig = sphere_inertia(mass, size[0])
            elif type == GEOM_CAPSULE:
                ig = capsule_inertia(mass, size[0], size[1])
            elif type == GEOM_BOX:
                ig = box_inertia(mass, size)
            else:
                raise ValueError("massive plane")
            R = quat_to_mat(quat)
            self._geom_mass.append((body, mass, np.asarray(pos, float), R @ ig @ R.T, R))
        return gid

    def connect(self, body1: int, body2: int, anchor1, anchor2) -> int:
        """Hold anchor1 (body1's frame) on anchor2 (body2's frame; the world if 0)."""
        self.m.equalities.append(Equality(type=EQ_CONNECT, body1=body1, body2=body2,
                                          anchor1=tuple(map(float, anchor1)),
                                          anchor2=tuple(map(float, anchor2))))
        return len(self.m.equalities) - 1

    def frame(self, body: int):
        """World pose (R, p) of a body with every joint at zero (its built pose)."""
        R, p = np.eye(3), np.zeros(3)
        chain = []
        while body > 0:
            chain.append(body)
            body = self.m.bodies[body].parent
        for b in reversed(chain):
            bb = self.m.bodies[b]
            p = p + R @ np.asarray(bb.pos, float)
            R = R @ quat_to_mat(bb.quat)
        return R, p

    def weld(self, body1: int, body2: int, anchor=None) -> int:
        """Hold body1's pose relative to body2 (the world if 0) at their built poses; the
        translational rows hold the world point `anchor` (default body1's origin)."""
        R1, p1 = self.frame(body1)
        R2, p2 = self.frame(body2)
        a = p1 if anchor is None else np.asarray(anchor, float)
        self.m.equalities.append(Equality(
            type=EQ_WELD, body1=body1, body2=body2,
            anchor1=tuple(map(float, R1.T @ (a - p1))), anchor2=tuple(map(float, R2.T @ (a - p2))),
            relquat=mat_to_quat(R1.T @ R2)))
        return len(self.m.equalities) - 1

    def capsule_fromto(self, body, p0, p1, r, mass=0.0, friction=1.0, name="") -> int:
        p0 = np.asarray(p0, float)
        p1 = np.asarray(p1, float)
        d = p1 - p0
        return self.geom(body, GEOM_CAPSULE, (r, 0.5 * np.linalg.norm(d)),
                         pos=0.5 * (p0 + p1), quat=quat_z_to(d), mass=mass,
                         friction=friction, name=name)

    def finish(self) -> Model:
        # body mass, COM and inertia about the COM in the body frame
        for bi, b in enumerate(self.m.bodies):
            parts = [g for g in self._geom_mass if g[0] == bi]
            if not parts:
                continue
            mass = sum(p[1] for p in parts)
            com = sum(p[1] * p[2] for p in parts) / mass
            I = np.zeros((3, 3))
            for _, m_, c, Ic, _ in parts:
                d = c - com
                I += Ic + m_ * (np.dot(d, d) * np.eye(3) - np.outer(d, d))
            b.mass = float(mass)
            b.ipos = tuple(float(x) for x in com)
            b.inertia = (I[0, 0], I[1, 1], I[2, 2], I[0, 1], I[0, 2], I[1, 2])
        return self.m


def _set_point_mass_props(m: Model, bi: int, mass: float, ipos, inertia_diag) -> None:
    b = m.bodies[bi]
    b.mass = float(mass)
    b.ipos = tuple(map(float, ipos))
    b.inertia = (float(inertia_diag[0]), float(inertia_diag[1]), float(inertia_diag[2]),
                 0.0, 0.0, 0.0)


# ----------------------------------------------------------------------------------
# the four workload models


def cartpole(hanging: bool = False, damping: float = 0.05, timestep: float = 0.01) -> Model:
    """Slider cart (1 kg) + hinge pole (capsule r 0.045, length 0.6, 0.1 kg).

    nq = nv = 2.  Motor on the slider with gear 10, ctrl in [-1, 1]; joint damping 0.05.
    ``hanging`` points the pole down (for the small-angle pendulum check).
    """
    bld = _Builder("cartpole")
    cart = bld.body(0, name="cart")
    bld.joint(cart, JNT_SLIDE, axis=(1, 0, 0), damping=damping, name="slider")
    # the cart only translates; its rotational inertia never enters the dynamics
    bld.geom(cart, GEOM_BOX, (0.1, 0.075, 0.05), mass=1.0, name="cart")
    pole = bld.body(cart, name="pole")
    bld.joint(pole, JNT_HINGE, axis=(0, 1, 0), damping=damping, name="hinge")
    tip = (0.0, 0.0, -0.6) if hanging else (0.0, 0.0, 0.6)
    bld.capsule_fromto(pole, (0, 0, 0), tip, 0.045, mass=0.1, name="pole")
    m = bld.finish()
    m.actuators.append(Actuator(type=ACT_MOTOR, joint=0, gear=10.0, ctrlrange=(-1.0, 1.0)))
    m.opt = Options(timestep=timestep, iterations=1, ls_iterations=4, nconmax=0)
    m.qpos0 = np.zeros(2)
    return m


QUAD_Q_DEFAULT = (0.0, math.pi / 4, -math.pi / 2)
QUAD_STAND_Z = 0.2 * math.sqrt(2.0) + 0.025


# joint ranges of the limited quadruped: the default pose +- these half widths (rad)
QUAD_RANGE_HALF = (0.15, 0.15, 0.15)


# dry joint friction of the quadruped_friction workload (N m): large enough that with
# the random PD targets about a fifth of the hinges stick at a time, the rest slip
QUAD_FRICTIONLOSS = 3.0


def quadruped(mu: float = 1.0, timestep: float = 0.004, iterations: int = 4,
              limits: bool = False, frictionloss: float = 0.0, tether: bool = False,
              implicit: int = 0, weld_base: bool = False, condim: int = 3,
              mu_torsion: float = 0.0, mu_rolling: float = 0.0) -> Model:
    """Free torso (box 0.3x0.1x0.05 m, 5 kg) + 4 legs x 3 hinges (capsules r 0.02,
    length 0.2, 0.5 kg) with massless sphere feet (r 0.025).  nq 19, nv 18, nu 12.

    With ``limits`` every hinge is limited to its default angle +- 0.15 rad, narrower
    than the initial noise and the reach of the random PD targets, so that limit rows
    switch on and off all through a rollout (with the benchmark inputs about 2.3 of
    the 12 are active on average, up to 7).  With ``frictionloss`` every hinge carries
    that dry friction (one friction-loss row each).  With ``tether`` the torso's centre
    is held by a connect equality on its standing position (a gantry tether: three
    two-sided rows).  With ``condim`` = 1 the feet's contacts are frictionless; 4 adds
    torsional friction ``mu_torsion`` and 6 also rolling friction ``mu_rolling``.  With
    ``weld_base`` the torso is welded to the world at its standing
    pose (a fixed-base robot: six two-sided rows).  With ``implicit`` = 1 the PD velocity gains are integrated
    implicitly (integrator 1); with 2 the PD position gains as well (integrator 2).

    Each leg: hip link (hinge about x, capsule lateral 0.2 m), thigh (hinge about y,
    capsule down 0.2 m), shin (hinge about y, capsule down 0.2 m, foot sphere).
    Position (PD) actuators kp 35, kd 0.5 on every hinge; ctrl is the target offset from
    the default pose (0, pi/4, -pi/2) per leg.  Only the feet collide (plane x 4 feet).
    """
    bld = _Builder("quadruped" + ("_limits" if limits else "") +
                   ("_friction" if frictionloss > 0 else "") + ("_tethered" if tether else "") +
                   ("_implicit" if implicit == 1 else "") +
                   ("_implicit_pd" if implicit == 2 else "") + ("_welded" if weld_base else "") +
                   ("_frictionless" if condim == 1 else "") +
                   (f"_condim{condim}" if condim in (4, 6) else ""))

    def rng(k):
        if not limits:
            return None
        return (QUAD_Q_DEFAULT[k] - QUAD_RANGE_HALF[k], QUAD_Q_DEFAULT[k] + QUAD_RANGE_HALF[k])

    plane = bld.geom(0, GEOM_PLANE, (0, 0, 0), friction=mu, name="floor")
    torso = bld.body(0, pos=(0, 0, QUAD_STAND_Z), name="torso")
    bld.joint(torso, JNT_FREE, name="root")
    bld.geom(torso, GEOM_BOX, (0.15, 0.05, 0.025), mass=5.0, name="torso")
    feet = []
    hinge_ids = []
    for i, (sx, sy) in enumerate(((1, 1), (1, -1), (-1, 1), (-1, -1))):
        hip = bld.body(torso, pos=(0.15 * sx, 0.05 * sy, 0.0), name=f"hip{i}")
        hinge_ids.append(bld.joint(hip, JNT_HINGE, axis=(1, 0, 0), range=rng(0),
                                   frictionloss=frictionloss, name=f"abd{i}"))
        bld.capsule_fromto(hip, (0, 0, 0), (0, 0.2 * sy, 0), 0.02, mass=0.5)
        thigh = bld.body(hip, pos=(0, 0.2 * sy, 0), name=f"thigh{i}")
        hinge_ids.append(bld.joint(thigh, JNT_HINGE, axis=(0, 1, 0), range=rng(1),
                                   frictionloss=frictionloss, name=f"hip{i}"))
        bld.capsule_fromto(thigh, (0, 0, 0), (0, 0, -0.2), 0.02, mass=0.5)
        shin = bld.body(thigh, pos=(0, 0, -0.2), name=f"shin{i}")
        hinge_ids.append(bld.joint(shin, JNT_HINGE, axis=(0, 1, 0), range=rng(2),
                                   frictionloss=frictionloss, name=f"knee{i}"))
        bld.capsule_fromto(shin, (0, 0, 0), (0, 0, -0.2), 0.02, mass=0.5)
        feet.append(bld.geom(shin, GEOM_SPHERE, (0.025,), pos=(0, 0, -0.2), friction=mu,
                             name=f"foot{i}"))
    m = bld.finish()
    for k, j in enumerate(hinge_ids):
        m.actuators.append(Actuator(type=ACT_PD, joint=j, gear=1.0, kp=35.0, kd=0.5,
                                    ctrlrange=(-1.0, 1.0), qdefault=QUAD_Q_DEFAULT[k % 3]))
    m.pairs = [(plane, f, mu, condim, mu_torsion, mu_rolling) for f in feet]
    if tether:
        bld.connect(torso, 0, (0, 0, 0), (0, 0, QUAD_STAND_Z))
    if weld_base:
        bld.weld(torso, 0)
    m.opt = Options(timestep=timestep, iterations=iterations, ls_iterations=8,
                    nconmax=4, integrator=int(implicit))
    q0 = np.zeros(m.nq)
    q0[0:3] = (0, 0, QUAD_STAND_Z)
    q0[3] = 1.0
    m.qpos0 = q0
    return m


def quadruped_standing_qpos(m: Model) -> np.ndarray:
    q = m.qpos0.copy()
    q[7:] = np.tile(QUAD_Q_DEFAULT, 4)
    return q


HUMANOID_TOTAL_MASS = 35.0


def humanoid(mu: float = 0.8, timestep: float = 0.005, iterations: int = 6,
             nconmax: int = 32) -> Model:
    """Free torso plus 21 hinges over 13 capsule/sphere bodies (nq 28, nv 27, nu 21).

    Bodies: torso (free; capsule + head sphere), lower_waist (2 hinges), pelvis (1),
    thigh x2 (3), shin x2 (1), foot x2 (2), upper_arm x2 (2), lower_arm x2 (1).
    Radii 0.03-0.06 m, total mass 35 kg by uniform density.  Motors with gear 50 and
    ctrl in [-1, 1]; hinge damping 0.2 and armature 0.02.  Collisions: the floor with
    every geom, and every geom pair whose bodies are neither the same nor parent/child.
    """
    shapes = []  # (body, kind, args) collected first so density can be set for 35 kg
    bld = _Builder("humanoid")
    plane = bld.geom(0, GEOM_PLANE, (0, 0, 0), friction=mu, name="floor")
    z0 = 1.25
    torso = bld.body(0, pos=(0, 0, z0), name="torso")
    bld.joint(torso, JNT_FREE, name="root")
    shapes += [(torso, "cap", ((0, -0.07, 0), (0, 0.07, 0), 0.06)),
               (torso, "sph", ((0, 0, 0.19), 0.06))]
    hk = dict(damping=0.2, armature=0.02)
    hinges = []
    lw = bld.body(torso, pos=(0, 0, -0.26), name="lower_waist")
    hinges.append(bld.joint(lw, JNT_HINGE, axis=(0, 0, 1), **hk))
    hinges.append(bld.joint(lw, JNT_HINGE, axis=(0, 1, 0), **hk))
    shapes.append((lw, "cap", ((0, -0.06, 0), (0, 0.06, 0), 0.05)))
    pelvis = bld.body(lw, pos=(0, 0, -0.165), name="pelvis")
    hinges.append(bld.joint(pelvis, JNT_HINGE, axis=(1, 0, 0), **hk))
    shapes.append((pelvis, "cap", ((0, -0.07, 0), (0, 0.07, 0), 0.06)))
    for side, sy in (("r", -1.0), ("l", 1.0)):
        th = bld.body(pelvis, pos=(0, 0.1 * sy, -0.04), name=f"thigh_{side}")
        for ax in ((1, 0, 0), (0, 0, 1), (0, 1, 0)):
            hinges.append(bld.joint(th, JNT_HINGE, axis=ax, **hk))
        shapes.append((th, "cap", ((0, 0, 0), (0, 0.0, -0.35), 0.05)))
        sh = bld.body(th, pos=(0, 0, -0.4), name=f"shin_{side}")
        hinges.append(bld.joint(sh, JNT_HINGE, axis=(0, -1, 0), **hk))
        shapes.append((sh, "cap", ((0, 0, 0), (0, 0, -0.3), 0.04)))
        ft = bld.body(sh, pos=(0, 0, -0.35), name=f"foot_{side}")
        hinges.append(bld.joint(ft, JNT_HINGE, axis=(0, 1, 0), **hk))
        hinges.append(bld.joint(ft, JNT_HINGE, axis=(1, 0, 0), **hk))
        shapes.append((ft, "cap", ((-0.03, 0, 0), (0.12, 0, 0), 0.03)))
    for side, sy in (("r", -1.0), ("l", 1.0)):
        ua = bld.body(torso, pos=(0, 0.17 * sy, 0.06), name=f"upper_arm_{side}")
        hinges.append(bld.joint(ua, JNT_HINGE, axis=(1, 0, 0), **hk))
        hinges.append(bld.joint(ua, JNT_HINGE, axis=(0, 1, 0), **hk))
        shapes.append((ua, "cap", ((0, 0, 0), (0, 0.05 * sy, -0.24), 0.04)))
        la = bld.body(ua, pos=(0, 0.05 * sy, -0.26), name=f"lower_arm_{side}")
        hinges.append(bld.joint(la, JNT_HINGE, axis=(0, -1, 0), **hk))
        shapes.append((la, "cap", ((0, 0, 0), (0, 0.02 * sy, -0.23), 0.03)))

    vol = 0.0
    for _, kind, a in shapes:
        if kind == "cap":
            vol += capsule_volume(a[2], 0.5 * np.linalg.norm(np.subtract(a[1], a[0])))
        else:
            vol += sphere_volume(a[1])
    rho = HUMANOID_TOTAL_MASS / vol
    geom_ids = []
    for bi, kind, a in shapes:
        if kind == "cap":
            hl = 0.5 * np.linalg.norm(np.subtract(a[1], a[0]))
            geom_ids.append(bld.capsule_fromto(bi, a[0], a[1], a[2],
                                               mass=rho * capsule_volume(a[2], hl),
                                               friction=mu))
        else:
            geom_ids.append(bld.geom(bi, GEOM_SPHERE, (a[1],), pos=a[0],
                                     mass=rho * sphere_volume(a[1]), friction=mu))
    m = bld.finish()
    for j in hinges:
        m.actuators.append(Actuator(type=ACT_MOTOR, joint=j, gear=50.0,
                                    ctrlrange=(-1.0, 1.0)))
    pairs = [(plane, g, mu) for g in geom_ids]
    for i, gi in enumerate(geom_ids):
        for gj in geom_ids[i + 1:]:
            bi, bj = m.geoms[gi].body, m.geoms[gj].body
            if bi == bj or m.bodies[bi].parent == bj or m.bodies[bj].parent == bi:
                continue
            a, b = (gi, gj) if m.geoms[gi].type <= m.geoms[gj].type else (gj, gi)
            pairs.append((a, b, mu))
    m.pairs = pairs
    m.opt = Options(timestep=timestep, iterations=iterations, ls_iterations=8,
                    nconmax=nconmax)
    q0 = np.zeros(m.nq)
    q0[0:3] = (0, 0, z0)
    q0[3] = 1.0
    m.qpos0 = q0
    return m


LEAP_GEAR_RATIO = 288.35
LEAP_ROTOR_MASS = 2.0e-3
LEAP_ROTOR_RADIUS = 4.12e-3


def leap_rotor_inertia() -> float:
    """I_r = 1/2 m_r r_r^2 (uniform disc rotor)."""
    return 0.5 * LEAP_ROTOR_MASS * LEAP_ROTOR_RADIUS ** 2


def leap_armature() -> float:
    """Reflected rotor inertia I_a = k_g^2 I_r; the paper rounds I_r to 1.7e-8."""
    return LEAP_GEAR_RATIO ** 2 * 1.7e-8


HAND_LINKS = (0.02, 0.045, 0.035, 0.03)


def hand(mu: float = 1.0, timestep: float = 0.0025, iterations: int = 6) -> Model:
    """4 fingers x 4 hinges over a palm (the floor plane) and a free 0.06 m cube.

    Finger bases at x in {-0.045, -0.015, 0.015, 0.045}, y = -0.06, z = 0.075; links are
    capsules (r 0.01, density 1000) along +y of lengths 0.02/0.045/0.035/0.03; the first
    hinge abducts about z, the other three flex toward -z.  Armature k_g^2 I_r on every
    finger joint; PD actuators kp 0.5, kd 0.01.  Cube: edge 0.06, 0.1 kg, released 1 mm
    above the palm.  Collisions: cube x 16 capsules (capsule-box) and palm x cube (plane-box).
    nq 23, nv 22, nu 16, nconmax 36.
    """
    bld = _Builder("hand")
    plane = bld.geom(0, GEOM_PLANE, (0, 0, 0), friction=mu, name="palm")
    arm = leap_armature()
    rho = 1000.0
    r = 0.01
    caps = []
    joints = []
    for fx in (-0.045, -0.015, 0.015, 0.045):
        parent, pos = 0, (fx, -0.06, 0.075)
        for k, L in enumerate(HAND_LINKS):
            b = bld.body(parent, pos=pos)
            axis = (0, 0, 1) if k == 0 else (-1, 0, 0)
            joints.append(bld.joint(b, JNT_HINGE, axis=axis, armature=arm))
            caps.append(bld.capsule_fromto(b, (0, 0, 0), (0, L, 0), r,
                                           mass=rho * capsule_volume(r, 0.5 * L),
                                           friction=mu))
            parent, pos = b, (0, L, 0)
    cube = bld.body(0, pos=(0, 0, 0.031), name="cube")
    bld.joint(cube, JNT_FREE)
    cube_g = bld.geom(cube, GEOM_BOX, (0.03, 0.03, 0.03), mass=0.1, friction=mu)
    m = bld.finish()
    for j in joints:
        m.actuators.append(Actuator(type=ACT_PD, joint=j, gear=1.0, kp=0.5, kd=0.01,
                                    ctrlrange=(-1.0, 1.0), qdefault=0.0))
    # pair order follows geom type: capsule (2) before box (3), plane (0) before box
    m.pairs = [(c, cube_g, mu) for c in caps] + [(plane, cube_g, mu)]
    m.opt = Options(timestep=timestep, iterations=iterations, ls_iterations=8,
                    nconmax=36)
    q0 = np.zeros(m.nq)
    q0[16:19] = (0, 0, 0.031)  # 1 mm above the palm: no contact exactly at distance 0
    q0[19] = 1.0
    m.qpos0 = q0
    return m


# ----------------------------------------------------------------------------------
# small models used by the reference checks


def quadruped_limits() -> Model:
    """The quadruped with every hinge limited (see ``quadruped``)."""
    return quadruped(limits=True)


def quadruped_tethered() -> Model:
    """The quadruped with its torso centre tethered to its standing position."""
    return quadruped(tether=True)


def perlin_terrain(n: int = 64, cells: int = 8, octaves: int = 3, seed: int = 0) -> np.ndarray:
    """An n x n gradient-noise (Perlin) elevation map in [0, 1]: ``octaves`` layers of
    random unit gradients on lattices of cells, 2 cells, ... per side, blended with the
    quintic fade 6t^5 - 15t^4 + 10t^3, each octave at half the previous amplitude.
    Deterministic (numpy Philox keyed by ``seed``)."""
    rng = np.random.Generator(np.random.Philox(key=[int(seed), 17]))
    u = np.linspace(0.0, 1.0, n)
    out = np.zeros((n, n))
    amp = 1.0
    for o in range(octaves):
        k = cells * 2 ** o
        ang = rng.uniform(0.0, 2.0 * np.pi, size=(k + 1, k + 1))
        gx, gy = np.cos(ang), np.sin(ang)
        x = u * k
        i0 = np.minimum(np.floor(x).astype(int), k - 1)
        t = x - i0
        fade = t ** 3 * (t * (t * 6 - 15) + 10)
        # rows follow y, columns follow x
        Y, X = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        iy, ix, ty, tx = i0[Y], i0[X], t[Y], t[X]
        fy, fx = fade[Y], fade[X]

        def corner(dy, dx):
            return gx[iy + dy, ix + dx] * (tx - dx) + gy[iy + dy, ix + dx] * (ty - dy)
        top = corner(0, 0) * (1 - fx) + corner(0, 1) * fx
        bot = corner(1, 0) * (1 - fx) + corner(1, 1) * fx
        out += amp * (top * (1 - fy) + bot * fy)
        amp *= 0.5
    out -= out.min()
    return out / max(out.max(), 1e-12)


# rough terrain of the quadruped_rough workload: 8 m x 8 m, 128 x 128 samples (6.3 cm
# spacing), 16 noise cells a side (50 cm features), 6 cm from the lowest to the highest
# point.  Under random PD targets a quadruped wanders up to 2.8 m from the origin in
# 1000 steps (4 s), so every world stays on the terrain.
ROUGH_SIZE, ROUGH_N, ROUGH_CELLS, ROUGH_HEIGHT = 4.0, 128, 16, 0.06


def quadruped_rough(seed: int = 0) -> Model:
    """The quadruped on Perlin-noise rough terrain: the feet collide with a heightfield
    instead of the floor plane (the paper's rough-terrain locomotion setting)."""
    m = quadruped()
    m.name = "quadruped_rough"
    data = perlin_terrain(ROUGH_N, cells=ROUGH_CELLS, seed=seed)
    m.hfield = Heightfield(nrow=ROUGH_N, ncol=ROUGH_N,
                           size=(ROUGH_SIZE, ROUGH_SIZE, ROUGH_HEIGHT), data=data)
    floor = m.pairs[0][0]
    m.geoms[floor].type = GEOM_HFIELD
    m.pairs = [(p[1], floor, *p[2:]) for p in m.pairs]
    # stand on the terrain: lift the torso by the terrain height under the origin
    h0 = ROUGH_HEIGHT * data[ROUGH_N // 2, ROUGH_N // 2]
    m.qpos0 = m.qpos0.copy()
    m.qpos0[2] += h0 + 0.01
    return m


def sphere_on_hfield(data: np.ndarray, size=(1.0, 1.0, 0.2), radius: float = 0.1,
                     mass: float = 1.0, hpos=(0.0, 0.0, 0.0), hquat=(1.0, 0.0, 0.0, 0.0),
                     timestep: float = 0.002, mu: float = 1.0) -> Model:
    """A free sphere and a heightfield geom (elevations ``data``, placed at hpos/hquat)
    with one sphere-heightfield pair (collision and resting checks)."""
    bld = _Builder("sphere_hfield")
    hf = bld.geom(0, GEOM_HFIELD, (0.0, 0.0, 0.0), pos=hpos, quat=hquat, friction=mu)
    b = bld.body(0, pos=(0, 0, 1.0))
    bld.joint(b, JNT_FREE)
    g = bld.geom(b, GEOM_SPHERE, (radius,), mass=mass, friction=mu)
    m = bld.finish()
    data = np.asarray(data, dtype=np.float64)
    m.hfield = Heightfield(nrow=data.shape[0], ncol=data.shape[1], size=tuple(size), data=data)
    m.pairs = [(g, hf, mu)]
    m.opt = Options(timestep=timestep, iterations=20, ls_iterations=20, nconmax=1)
    q0 = np.zeros(7)
    q0[2], q0[3] = 1.0, 1.0
    m.qpos0 = q0
    return m


def quadruped_implicit() -> Model:
    """The quadruped with its PD velocity gains integrated implicitly."""
    return quadruped(implicit=1)


def quadruped_welded() -> Model:
    """The quadruped with its torso welded to the world at its standing pose."""
    return quadruped(weld_base=True)


def quadruped_frictionless() -> Model:
    """The quadruped on frictionless ground (condim 1 foot contacts)."""
    return quadruped(condim=1)


def quadruped_torsion() -> Model:
    """The quadruped with torsional friction at the feet (condim 4, mu_t 0.02 m)."""
    return quadruped(condim=4, mu_torsion=0.02)


def quadruped_rolling() -> Model:
    """The quadruped with torsional and rolling friction at the feet (condim 6)."""
    return quadruped(condim=6, mu_torsion=0.02, mu_rolling=0.001)


def elliptic(m: Model) -> Model:
    """The model with elliptic friction cones (the contact frame's rows) in place of the
    pyramid."""
    m.name = m.name + "_elliptic"
    m.opt.cone = 1
    return m


def quadruped_elliptic() -> Model:
    """The quadruped with elliptic friction cones at the feet."""
    return elliptic(quadruped())


def quadruped_elliptic_rolling() -> Model:
    """The quadruped with elliptic cones over sliding, torsional and rolling friction
    (condim 6: six frame rows a contact)."""
    return elliptic(quadruped_rolling())


def humanoid_elliptic() -> Model:
    return elliptic(humanoid())


def hand_elliptic() -> Model:
    return elliptic(hand())


def quadruped_rk4() -> Model:
    """The quadruped integrated by fourth-order Runge-Kutta (integrator 3)."""
    m = quadruped()
    m.name = "quadruped_rk4"
    m.opt.integrator = 3
    return m


def quadruped_implicit_pd() -> Model:
    """The quadruped with its PD velocity and position gains integrated implicitly."""
    return quadruped(implicit=2)


def quadruped_friction() -> Model:
    """The quadruped with dry friction QUAD_FRICTIONLOSS on every hinge."""
    return quadruped(frictionloss=QUAD_FRICTIONLOSS)


def slider(mass: float = 2.0, armature: float = 0.0, range=(0.0, 1.0), axis=(0, 0, 1),
           gravity=(0.0, 0.0, -9.81), timestep: float = 0.002,
           frictionloss: float = 0.0, damping: float = 0.0, integrator: int = 0) -> Model:
    """One sphere on a slide joint (nv 1), limited to ``range`` unless it is None: the
    one-dof limit and friction-loss problems."""
    bld = _Builder("slider")
    b = bld.body(0, name="slider")
    bld.joint(b, JNT_SLIDE, axis=axis, armature=armature, range=range,
              frictionloss=frictionloss, damping=damping)
    bld.geom(b, GEOM_SPHERE, (0.05,), mass=mass)
    m = bld.finish()
    m.opt = Options(timestep=timestep, gravity=tuple(gravity), iterations=8, nconmax=0,
                    integrator=integrator)
    m.qpos0 = np.zeros(1)
    return m


def pinned_body(shape: str = "sphere", mass: float = 1.0, anchor=(0.0, 0.0, 0.0),
                z0: float = 1.0, timestep: float = 0.002) -> Model:
    """A free sphere or capsule (half length 0.2 along z) whose point ``anchor`` (body
    frame) is pinned by a connect equality to where it sits at qpos0."""
    bld = _Builder(f"pinned_{shape}")
    b = bld.body(0, pos=(0, 0, z0))
    bld.joint(b, JNT_FREE)
    if shape == "sphere":
        bld.geom(b, GEOM_SPHERE, (0.1,), mass=mass)
    else:
        bld.geom(b, GEOM_CAPSULE, (0.03, 0.2), mass=mass)
    m = bld.finish()
    bld.connect(b, 0, anchor, (anchor[0], anchor[1], anchor[2] + z0))
    m.opt = Options(timestep=timestep, iterations=4, nconmax=0)
    q0 = np.zeros(7)
    q0[2] = z0
    q0[3] = 1.0
    m.qpos0 = q0
    return m


def welded_box(mass: float = 1.0, half=(0.1, 0.05, 0.03), z0: float = 0.3, anchor=None,
               gravity=(0.0, 0.0, -9.81), timestep: float = 0.002) -> Model:
    """A free box welded to the world at its built pose (centre at (0, 0, z0)); the
    translational rows hold the world point `anchor` (default the centre)."""
    bld = _Builder("welded_box")
    b = bld.body(0, pos=(0, 0, z0))
    bld.joint(b, JNT_FREE)
    bld.geom(b, GEOM_BOX, half, mass=mass)
    bld.weld(b, 0, anchor)
    m = bld.finish()
    m.opt = Options(timestep=timestep, gravity=tuple(gravity), iterations=50,
                    ls_iterations=50, nconmax=0)
    m.qpos0 = np.array([0, 0, z0, 1, 0, 0, 0], dtype=np.float64)
    return m


def welded_pair(m1: float = 1.0, m2: float = 2.0, gravity=(0.0, 0.0, 0.0),
                timestep: float = 0.002) -> Model:
    """Two free boxes side by side (centres 0.25 m apart along x, the second turned 30
    degrees about z) welded to each other at the midpoint."""
    bld = _Builder("welded_pair")
    b1 = bld.body(0, pos=(-0.1, 0, 0.3))
    bld.joint(b1, JNT_FREE)
    bld.geom(b1, GEOM_BOX, (0.1, 0.05, 0.04), mass=m1)
    b2 = bld.body(0, pos=(0.15, 0, 0.3), quat=axis_angle_quat((0, 0, 1), math.pi / 6))
    bld.joint(b2, JNT_FREE)
    bld.geom(b2, GEOM_BOX, (0.08, 0.06, 0.05), mass=m2)
    bld.weld(b1, b2, anchor=(0.0, 0.0, 0.3))
    m = bld.finish()
    m.opt = Options(timestep=timestep, gravity=tuple(gravity), iterations=50,
                    ls_iterations=50, nconmax=0)
    q = np.zeros(14)
    q[0:3], q[3:7] = (-0.1, 0, 0.3), (1, 0, 0, 0)
    q[7:10], q[10:14] = (0.15, 0, 0.3), axis_angle_quat((0, 0, 1), math.pi / 6)
    m.qpos0 = q
    return m


def connected_spheres(m1: float = 1.0, m2: float = 3.0, gap: float = 0.0,
                      gravity=(0.0, 0.0, -9.81), timestep: float = 0.002) -> Model:
    """Two free spheres whose centres are held together by a connect equality (the
    second sphere starts ``gap`` above the first)."""
    bld = _Builder("connected_spheres")
    b1 = bld.body(0, pos=(0, 0, 1.0))
    bld.joint(b1, JNT_FREE)
    bld.geom(b1, GEOM_SPHERE, (0.1,), mass=m1)
    b2 = bld.body(0, pos=(0, 0, 1.0 + gap))
    bld.joint(b2, JNT_FREE)
    bld.geom(b2, GEOM_SPHERE, (0.1,), mass=m2)
    m = bld.finish()
    bld.connect(b1, b2, (0, 0, 0), (0, 0, 0))
    m.opt = Options(timestep=timestep, gravity=tuple(gravity), iterations=4, nconmax=0)
    q0 = np.zeros(14)
    q0[2], q0[3], q0[9], q0[10] = 1.0, 1.0, 1.0 + gap, 1.0
    m.qpos0 = q0
    return m


def four_bar(link: float = 0.3, span: float = 0.4, mass: float = 0.5, damping: float = 0.0,
             frictionloss: float = 0.0, timestep: float = 0.002) -> Model:
    """A planar parallelogram linkage closed by a connect equality: two cranks of length
    ``link`` hang from world pivots ``span`` apart (hinges about y); a coupler rides on
    the first crank's tip and its far end is connected to the second crank's tip.  One
    degree of freedom: the coupler translates without turning (q_coupler = -q_crank1,
    q_crank2 = q_crank1)."""
    bld = _Builder("four_bar")
    c1 = bld.body(0, pos=(0, 0, 0), name="crank1")
    bld.joint(c1, JNT_HINGE, axis=(0, 1, 0), damping=damping, frictionloss=frictionloss)
    bld.capsule_fromto(c1, (0, 0, 0), (0, 0, -link), 0.02, mass=mass)
    cp = bld.body(c1, pos=(0, 0, -link), name="coupler")
    bld.joint(cp, JNT_HINGE, axis=(0, 1, 0), damping=damping, frictionloss=frictionloss)
    bld.capsule_fromto(cp, (0, 0, 0), (span, 0, 0), 0.02, mass=mass)
    c2 = bld.body(0, pos=(span, 0, 0), name="crank2")
    bld.joint(c2, JNT_HINGE, axis=(0, 1, 0), damping=damping, frictionloss=frictionloss)
    bld.capsule_fromto(c2, (0, 0, 0), (0, 0, -link), 0.02, mass=mass)
    m = bld.finish()
    bld.connect(cp, c2, (span, 0, 0), (0, 0, -link))
    m.opt = Options(timestep=timestep, iterations=4, nconmax=0)
    m.qpos0 = np.zeros(3)
    return m


def hinge_chain(n: int = 4, link: float = 0.3, mass: float = 1.0, damping: float = 0.0,
                axes=None, slide_root: bool = False, limit: float = None,
                frictionloss: float = 0.0) -> Model:
    """Planar/spatial chain of capsule links hanging from the world (no contacts).
    With ``limit`` every hinge is limited to [-limit, limit] (and the slide root to
    [-2 limit, 2 limit]).  Every joint gets dry friction ``frictionloss``."""
    bld = _Builder(f"chain{n}")
    parent, pos = 0, (0, 0, 0)
    if slide_root:
        cart = bld.body(0, name="cart")
        bld.joint(cart, JNT_SLIDE, axis=(1, 0, 0), damping=damping,
                  range=None if limit is None else (-2 * limit, 2 * limit),
                  frictionloss=frictionloss)
        bld.geom(cart, GEOM_BOX, (0.1, 0.1, 0.1), mass=2.0)
        parent = cart
    for i in range(n):
        b = bld.body(parent, pos=pos)
        ax = (0, 1, 0) if axes is None else axes[i % len(axes)]
        bld.joint(b, JNT_HINGE, axis=ax, damping=damping,
                  range=None if limit is None else (-limit, limit),
                  frictionloss=frictionloss)
        bld.capsule_fromto(b, (0, 0, 0), (link, 0, 0), 0.03, mass=mass)
        parent, pos = b, (link, 0, 0)
    m = bld.finish()
    m.opt = Options(timestep=1e-3, iterations=1, nconmax=0)
    m.qpos0 = np.zeros(m.nq)
    return m


def free_body(shape: str = "box", mass: float = 1.0, gravity=(0.0, 0.0, -9.81),
              half=(0.1, 0.2, 0.3), z0: float = 1.0, plane: bool = False,
              mu: float = 1.0, timestep: float = 0.002, iterations: int = 50,
              condim: int = 3, mu_torsion: float = 0.0, mu_rolling: float = 0.0) -> Model:
    """One free body (box or sphere), optionally resting on a plane (condim 1: the
    contacts are frictionless; 4: with torsional friction; 6: also rolling friction)."""
    bld = _Builder(f"free_{shape}")
    pl = bld.geom(0, GEOM_PLANE, (0, 0, 0), friction=mu) if plane else None
    b = bld.body(0, pos=(0, 0, z0))
    bld.joint(b, JNT_FREE)
    if shape == "box":
        g = bld.geom(b, GEOM_BOX, half, mass=mass, friction=mu)
        nc = 4
    elif shape == "sphere":
        g = bld.geom(b, GEOM_SPHERE, (half[0],), mass=mass, friction=mu)
        nc = 1
    elif shape == "capsule":
        g = bld.geom(b, GEOM_CAPSULE, (half[0], half[1]), mass=mass, friction=mu)
        nc = 2
    else:
        raise ValueError(shape)
    m = bld.finish()
    if plane:
        m.pairs = [(pl, g, mu, condim, mu_torsion, mu_rolling)]
    m.opt = Options(timestep=timestep, gravity=tuple(gravity), iterations=iterations,
                    ls_iterations=50, nconmax=nc if plane else 0)
    q0 = np.zeros(7)
    q0[2] = z0
    q0[3] = 1.0
    m.qpos0 = q0
    return m


def two_bodies(t1: str, t2: str, size1, size2, gravity=(0.0, 0.0, 0.0)) -> Model:
    """Two free bodies with one collision pair between them (collision unit checks)."""
    bld = _Builder(f"{t1}_{t2}")
    kinds = {"sphere": GEOM_SPHERE, "capsule": GEOM_CAPSULE, "box": GEOM_BOX}
    gs = []
    for t, s, z in ((t1, size1, 0.0), (t2, size2, 1.0)):
        b = bld.body(0, pos=(0, 0, z))
        bld.joint(b, JNT_FREE)
        gs.append(bld.geom(b, kinds[t], s, mass=1.0))
    m = bld.finish()
    g1, g2 = gs
    if m.geoms[g1].type > m.geoms[g2].type:
        g1, g2 = g2, g1
    m.pairs = [(g1, g2, 1.0)]
    m.opt = Options(timestep=0.002, gravity=tuple(gravity), iterations=20, nconmax=4)
    q0 = np.zeros(14)
    q0[3] = q0[10] = 1.0
    q0[9] = 1.0
    m.qpos0 = q0
    return m


WORKLOADS = {
    "cartpole": cartpole,
    "quadruped": quadruped,
    "quadruped_limits": quadruped_limits,
    "quadruped_friction": quadruped_friction,
    "quadruped_tethered": quadruped_tethered,
    "quadruped_implicit": quadruped_implicit,
    "quadruped_implicit_pd": quadruped_implicit_pd,
    "quadruped_rk4": quadruped_rk4,
    "quadruped_welded": quadruped_welded,
    "quadruped_frictionless": quadruped_frictionless,
    "quadruped_torsion": quadruped_torsion,
    "quadruped_rolling": quadruped_rolling,
    "quadruped_rough": quadruped_rough,
    "quadruped_elliptic": quadruped_elliptic,
    "quadruped_elliptic_rolling": quadruped_elliptic_rolling,
    "humanoid": humanoid,
    "humanoid_elliptic": humanoid_elliptic,
    "hand": hand,
    "hand_elliptic": hand_elliptic,
}
