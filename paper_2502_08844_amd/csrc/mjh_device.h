// Device phases of one physics step for one world, executed by a team of T lanes
// (T in {16, 32, 64}, always inside one wavefront).  The world's working set lives in
// LDS at `W` (layout in DevModel); loops are strided over the team's lanes and phases
// are separated by wavefront-level barriers.
//
// Phase order per step (the MuJoCo pipeline that the paper's environments step):
//   actuation -> kinematics + velocities + RNE forward sweep (by tree level)
//   -> backward sweep (composite inertia, RNE forces) -> mass matrix (CRBA)
//   -> sparse L^T D L factorisation and unconstrained acceleration
//   -> collision candidates, selection, contact records -> pyramidal constraint rows
//   -> Newton solve with exact line search -> semi-implicit Euler.
// The mathematics follows Featherstone, Rigid Body Dynamics Algorithms (spatial
// algebra ch. 2, RNEA Table 5.1, CRBA Table 6.2, LTDL sec. 6.5), Todorov (ICRA 2014)
// for the soft-constraint cost, and Ericson ch. 5 for closest points.
#pragma once
#include <hip/hip_runtime.h>

#include "mjh_model.h"

namespace mjh {

#define DEV __device__ __forceinline__

typedef float f32x16 __attribute__((ext_vector_type(16)));

// A zero the compiler cannot see through.  Adding it to the LDS base pointer and the
// lane index at the start of a phase keeps values derived from them (region pointers,
// lane masks) from being hoisted out of the step loop and held, or spilled, across
// phases; each phase recomputes them with a few adds.
DEV int opaque_zero() {
  int z = 0;
  asm volatile("" : "+v"(z));
  return z;
}


// ------------------------------------------------------------------- team helpers
struct Team {
  int lane;       // 0 .. T-1
  int T;          // lanes per world: 16, 32 or 64
  const unsigned char* tp;  // triangle table in LDS: tp[p] = b for p = b(b+1)/2 + a
  // packed index p -> (b, a) with 0 <= a <= b
  DEV void unrank(int p, int& b, int& a) const {
    b = tp[p];
    a = p - (__mul24(b, b + 1) >> 1);
  }
  // wavefront-level barrier: orders LDS traffic of all lanes of the wave
  DEV void sync() const {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  // All-reductions over the team's lanes.  Within a 16-lane row they use DPP lane
  // permutations (xor 1 and xor 2 by quad permutes, then the half-row and row mirrors);
  // wider teams then combine row pairs and wave halves with the gfx950 permlane swaps.
  // Every step combines a lane's value with its partner's by a commutative operation,
  // so all lanes of the team end with bitwise the same result.  Every lane of the team
  // must be active.
  template <class Op>
  DEV int allreduce(int v, Op op) const {
    v = op(v, __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
    v = op(v, __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
    v = op(v, __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, false));  // row_half_mirror
    v = op(v, __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, false));  // row_mirror
    if (T >= 32) {
      const auto r = __builtin_amdgcn_permlane16_swap((unsigned)v, (unsigned)v, false, false);
      v = op((int)r[0], (int)r[1]);
    }
    if (T == 64) {
      const auto r = __builtin_amdgcn_permlane32_swap((unsigned)v, (unsigned)v, false, false);
      v = op((int)r[0], (int)r[1]);
    }
    return v;
  }
  template <class Op>
  DEV float allreducef(float v, Op op) const {
    return __int_as_float(allreduce(__float_as_int(v), [&](int a, int b) {
      return __float_as_int(op(__int_as_float(a), __int_as_float(b)));
    }));
  }
  DEV float sum(float v) const { return allreducef(v, [](float a, float b) { return a + b; }); }
  DEV float max(float v) const { return allreducef(v, [](float a, float b) { return fmaxf(a, b); }); }
  DEV float min(float v) const { return allreducef(v, [](float a, float b) { return fminf(a, b); }); }
  DEV int isum(int v) const { return allreduce(v, [](int a, int b) { return a + b; }); }
  DEV int ior(int v) const { return allreduce(v, [](int a, int b) { return a | b; }); }
  // the value of `v` held by lane `i` of this team (i uniform), read with v_readlane:
  // one read per team of the wavefront, then each lane keeps its own team's
  DEV float bcast(float v, int i) const {
    const int base = (int)(threadIdx.x & 63) - lane;  // the team's first lane in the wave
    const int iv = __float_as_int(v);
    int r = __builtin_amdgcn_readlane(iv, i);
    if (T == 32) {
      const int r1 = __builtin_amdgcn_readlane(iv, i + 32);
      r = base ? r1 : r;
    } else if (T == 16) {
      const int r1 = __builtin_amdgcn_readlane(iv, i + 16);
      const int r2 = __builtin_amdgcn_readlane(iv, i + 32);
      const int r3 = __builtin_amdgcn_readlane(iv, i + 48);
      r = base == 0 ? r : base == 16 ? r1 : base == 32 ? r2 : r3;
    }
    return __int_as_float(r);
  }
  // exclusive prefix sum over the team's lanes
  DEV int exscan(int v) const {
    int x = v;
    for (int o = 1; o < T; o <<= 1) {
      int y = __shfl_up(x, o, T);
      if (lane >= o) x += y;
    }
    return x - v;
  }
};

// ------------------------------------------------------------------ small algebra
DEV float dot3(const float* a, const float* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
DEV void cross3(const float* a, const float* b, float* r) {
  float x = a[1] * b[2] - a[2] * b[1];
  float y = a[2] * b[0] - a[0] * b[2];
  float z = a[0] * b[1] - a[1] * b[0];
  r[0] = x; r[1] = y; r[2] = z;
}
DEV void mv3(const float* R, const float* v, float* r) {  // r = R v (row-major R)
  float x = R[0] * v[0] + R[1] * v[1] + R[2] * v[2];
  float y = R[3] * v[0] + R[4] * v[1] + R[5] * v[2];
  float z = R[6] * v[0] + R[7] * v[1] + R[8] * v[2];
  r[0] = x; r[1] = y; r[2] = z;
}
DEV void mtv3(const float* R, const float* v, float* r) {  // r = R^T v
  float x = R[0] * v[0] + R[3] * v[1] + R[6] * v[2];
  float y = R[1] * v[0] + R[4] * v[1] + R[7] * v[2];
  float z = R[2] * v[0] + R[5] * v[1] + R[8] * v[2];
  r[0] = x; r[1] = y; r[2] = z;
}
DEV void mm3(const float* A, const float* B, float* C) {  // C = A B (C may alias)
  float o[9];
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++)
      o[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
#pragma unroll
  for (int k = 0; k < 9; k++) C[k] = o[k];
}
DEV void quat_to_mat(const float* q, float* R) {
  float w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1.f - 2.f * (y * y + z * z); R[1] = 2.f * (x * y - w * z); R[2] = 2.f * (x * z + w * y);
  R[3] = 2.f * (x * y + w * z); R[4] = 1.f - 2.f * (x * x + z * z); R[5] = 2.f * (y * z - w * x);
  R[6] = 2.f * (x * z - w * y); R[7] = 2.f * (y * z + w * x); R[8] = 1.f - 2.f * (x * x + y * y);
}
// rotation by angle about unit axis a
DEV void axis_rot(const float* a, float ang, float* R) {
  float s, c;
  sincosf(ang, &s, &c);
  float t = 1.f - c;
  R[0] = c + t * a[0] * a[0];        R[1] = t * a[0] * a[1] - s * a[2]; R[2] = t * a[0] * a[2] + s * a[1];
  R[3] = t * a[0] * a[1] + s * a[2]; R[4] = c + t * a[1] * a[1];        R[5] = t * a[1] * a[2] - s * a[0];
  R[6] = t * a[0] * a[2] - s * a[1]; R[7] = t * a[1] * a[2] + s * a[0]; R[8] = c + t * a[2] * a[2];
}
// spatial motion cross product [w1; v1] x [w2; v2]
DEV void crossm(const float* m1, const float* m2, float* r) {
  float a[3], b[3], c[3];
  cross3(m1, m2, a);
  cross3(m1, m2 + 3, b);
  cross3(m1 + 3, m2, c);
  r[0] = a[0]; r[1] = a[1]; r[2] = a[2];
  r[3] = b[0] + c[0]; r[4] = b[1] + c[1]; r[5] = b[2] + c[2];
}
// spatial force cross product [w; v] x* [n; f]
DEV void crossf(const float* m, const float* f, float* r) {
  float a[3], b[3], c[3];
  cross3(m, f, a);
  cross3(m + 3, f + 3, b);
  cross3(m, f + 3, c);
  r[0] = a[0] + b[0]; r[1] = a[1] + b[1]; r[2] = a[2] + b[2];
  r[3] = c[0]; r[4] = c[1]; r[5] = c[2];
}
// spatial inertia (m, h = m c, I_O) applied to motion [w; v]
DEV void inertia_mul(const float* I, const float* mv, float* f) {
  const float* w = mv;
  const float* v = mv + 3;
  float hv[3], hw[3];
  cross3(I + 1, v, hv);
  cross3(I + 1, w, hw);
  f[0] = I[4] * w[0] + I[7] * w[1] + I[8] * w[2] + hv[0];
  f[1] = I[7] * w[0] + I[5] * w[1] + I[9] * w[2] + hv[1];
  f[2] = I[8] * w[0] + I[9] * w[1] + I[6] * w[2] + hv[2];
  f[3] = I[0] * v[0] - hw[0];
  f[4] = I[0] * v[1] - hw[1];
  f[5] = I[0] * v[2] - hw[2];
}
DEV float dot6(const float* a, const float* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + a[3] * b[3] + a[4] * b[4] + a[5] * b[5];
}
// packed lower-triangular index of a symmetric matrix (indices < 2^12, so the product
// fits the full-rate 24-bit multiplier)
DEV int tri(int i, int j) { return (__mul24(i, i + 1) >> 1) + j; }  // requires i >= j
DEV int sym(int i, int j) { return i >= j ? tri(i, j) : tri(j, i); }
// v0 plus row i of a packed symmetric matrix times x, summed in k order from v0: M_ik
// sits at tri(i, k) = tri(i, 0) + k for k <= i, then at tri(k, i), which grows by k + 1
// from one k to the next
DEV float sym_row_dot(const float* M, int i, const float* x, int n, float v0 = 0.f) {
  float v = v0;
  int at = tri(i, 0);
  for (int k = 0; k < n; k++) {
    v += M[at] * x[k];
    at += k < i ? 1 : k + 1;
  }
  return v;
}
// ------------------------------------------------------------ per-world parameters
// Optional per-world parameter record (domain randomisation, in LDS), 8 + 2 nu words:
// [0] contact friction scale, [1] payload mass added to body 1 at its centre of mass,
// [2..4] shift of body 1's centre of mass (body frame), [5] kp scale, [6] kd scale,
// [7] unused, [8 + k] calibration offset of actuator k (the PD law sees q + offset),
// [8 + nu + k] armature of dof 6 + k (replacing the model's).  The caller guarantees
// body 1 is the free root and actuator k drives dof 6 + k.  nullptr: the model as is.
constexpr int kDrFric = 0, kDrPayload = 1, kDrCom = 2, kDrKp = 5, kDrKd = 6, kDrHead = 8;

// ------------------------------------------------------------ A0: actuation
// per dof: motor tau = gear u; position actuator (eq. pd_mapping)
// tau = kp (q_default + gear u - q) - kd qdot; joint damping -b qdot.  Controls are
// clamped to their range.  Result: frc = act + passive (bias subtracted later).
DEV void actuation(const DevModel& m, float* W, const Team& t, const float* ctrl,
                   const float* dr = nullptr) {
  const float* qpos = W + m.o_qpos;
  const float* qvel = W + m.o_qvel;
  float* frc = W + m.o_frc;
  for (int i = t.lane; i < m.nv; i += t.T) {
    float f = -m.dof_damping[i] * qvel[i];
    int a = m.dof_act[i];
    if (a >= 0) {
      const float c = ctrl ? ctrl[a] : 0.f;
      float u = fminf(fmaxf(c, m.act_lo[a]), m.act_hi[a]);
      if (m.act_type[a] == ACT_MOTOR) {
        f += m.act_gear[a] * u;
      } else {
        float kp = m.act_kp[a], kd = m.act_kd[a], q0 = m.act_qdef[a];
        if (dr) {
          kp *= dr[kDrKp];
          kd *= dr[kDrKd];
          q0 -= dr[kDrHead + a];
        }
        f += kp * (q0 + m.act_gear[a] * u - qpos[m.act_qadr[a]]) - kd * qvel[i];
      }
    }
    frc[i] = f;
  }
}

// ----------------------------------- A1/A2/A5 forward sweep by tree level (RBDA 4, 5)
// For each body: place its frame on the parent, apply its joints in order (hinge:
// rotation about the world axis through the world anchor; slide: translation; free:
// absolute pose), record motion subspaces S (world origin) and their rates, the
// body velocity V, bias acceleration A (qacc = 0, world at -gravity), spatial
// inertia and the body force f = I A + V x* I V.
// still: velocities taken as zero and no gravity (then cfrc = the forces of M qacc alone)
DEV void forward_sweep(const DevModel& m, float* W, const Team& t, const float* qacc = nullptr,
                       const float* dr = nullptr, bool still = false) {
  const float* qpos = W + m.o_qpos;
  const float* qv0 = W + m.o_qvel;
  auto qvel = [&](int i) { return still ? 0.f : qv0[i]; };
  float* xpos = W + m.o_xpos;
  float* xmat = W + m.o_xmat;
  float* cvel = W + m.o_cvel;
  float* cacc = W + m.o_cacc;
  float* cfrc = W + m.o_cfrc;
  float* cinert = W + m.o_cinert;
  float* cdof = W + m.o_cdof;
  // the world body: at rest, accelerating at -gravity (this scratch is shared with the
  // contact phases, so it is set again every step)
  if (t.lane < 6) {
    cvel[t.lane] = 0.f;
    cacc[t.lane] = (still || t.lane < 3) ? 0.f : -m.grav[t.lane - 3];
  }
  // Positions are relative to the origin p0, the first joint's position when it is a
  // free joint (else the world origin): the world body sits at -p0.  The step is
  // translation invariant, and spatial inertias taken at an origin near the bodies keep
  // their rotational part, which FP32 rounds away against m |c|^2 far from the origin.
  if (t.lane < 3)
    xpos[t.lane] = (m.njnt > 0 && m.jnt_type[0] == JNT_FREE) ? -qpos[m.jnt_qposadr[0] + t.lane] : 0.f;
  t.sync();
  for (int lv = 1; lv < m.nlevel; lv++) {
    const int e = m.level_start[lv + 1];
    for (int ib = m.level_start[lv] + t.lane; ib < e; ib += t.T) {
      const int b = m.level_body[ib];
      const int p = m.body_parent[b];
      float pos[3], R[9], V[6], A[6];
      mv3(xmat + 9 * p, m.body_pos + 3 * b, pos);
      for (int k = 0; k < 3; k++) pos[k] += xpos[3 * p + k];
      mm3(xmat + 9 * p, m.body_rot + 9 * b, R);
      for (int k = 0; k < 6; k++) { V[k] = cvel[6 * p + k]; A[k] = cacc[6 * p + k]; }
      const int j0 = m.body_jntadr[b], nj = m.body_jntnum[b];
      for (int j = j0; j < j0 + nj; j++) {
        const int qa = m.jnt_qposadr[j], da = m.jnt_dofadr[j];
        float* S = cdof + 6 * da;
        float Sd[6];
        const int type = m.jnt_type[j];
        if (type == JNT_FREE) {
          float q[4] = {qpos[qa + 3], qpos[qa + 4], qpos[qa + 5], qpos[qa + 6]};
          float inv = 1.f / sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
          for (int k = 0; k < 4; k++) q[k] *= inv;
          quat_to_mat(q, R);
          for (int k = 0; k < 3; k++) pos[k] = qpos[qa + k] + xpos[k];  // relative to p0
          for (int i = 0; i < 3; i++) {
            float* s = S + 6 * i;
            s[0] = s[1] = s[2] = 0.f;
            s[3] = (i == 0) ? 1.f : 0.f; s[4] = (i == 1) ? 1.f : 0.f; s[5] = (i == 2) ? 1.f : 0.f;
            float* r = S + 6 * (3 + i);
            float col[3] = {R[i], R[3 + i], R[6 + i]};
            r[0] = col[0]; r[1] = col[1]; r[2] = col[2];
            cross3(pos, col, r + 3);
          }
          for (int i = 0; i < 6; i++)
            for (int k = 0; k < 6; k++) V[k] += S[6 * i + k] * qvel(da + i);
          // translation subspaces are fixed in the world (zero rate), rotation ones turn
          // with the body: rate V_body x S
          for (int i = 3; i < 6; i++) {
            crossm(V, S + 6 * i, Sd);
            for (int k = 0; k < 6; k++) A[k] += Sd[k] * qvel(da + i);
          }
          if (qacc)
            for (int i = 0; i < 6; i++)
              for (int k = 0; k < 6; k++) A[k] += S[6 * i + k] * qacc[da + i];
        } else if (type == JNT_SLIDE) {
          float ax[3];
          mv3(R, m.jnt_axis + 3 * j, ax);
          const float q = qpos[qa];
          for (int k = 0; k < 3; k++) pos[k] += ax[k] * q;
          S[0] = S[1] = S[2] = 0.f;
          S[3] = ax[0]; S[4] = ax[1]; S[5] = ax[2];
          for (int k = 0; k < 6; k++) V[k] += S[k] * qvel(da);
          crossm(V, S, Sd);
          for (int k = 0; k < 6; k++) A[k] += Sd[k] * qvel(da) + (qacc ? S[k] * qacc[da] : 0.f);
        } else {  // hinge
          // Rotation about the world axis R a equals R Rot(a, q) with the body-frame
          // axis a.  The second form builds the joint rotation from exact model data,
          // so FP32 rounding only adds along a chain; rotating about the rounded world
          // axis amplifies the frame error at every large-angle hinge.
          float ax[3], off[3], anc[3], Rj[9];
          mv3(R, m.jnt_pos + 3 * j, off);
          for (int k = 0; k < 3; k++) anc[k] = pos[k] + off[k];
          axis_rot(m.jnt_axis + 3 * j, qpos[qa], Rj);
          mm3(R, Rj, R);
          mv3(R, m.jnt_axis + 3 * j, ax);
          mv3(R, m.jnt_pos + 3 * j, off);
          for (int k = 0; k < 3; k++) pos[k] = anc[k] - off[k];
          S[0] = ax[0]; S[1] = ax[1]; S[2] = ax[2];
          cross3(anc, ax, S + 3);
          for (int k = 0; k < 6; k++) V[k] += S[k] * qvel(da);
          crossm(V, S, Sd);
          for (int k = 0; k < 6; k++) A[k] += Sd[k] * qvel(da) + (qacc ? S[k] * qacc[da] : 0.f);
        }
      }
      for (int k = 0; k < 3; k++) xpos[3 * b + k] = pos[k];
      for (int k = 0; k < 9; k++) xmat[9 * b + k] = R[k];
      for (int k = 0; k < 6; k++) { cvel[6 * b + k] = V[k]; cacc[6 * b + k] = A[k]; }
    }
    t.sync();
  }
  // Spatial inertias and bias forces need only each body's own pose, velocity and
  // acceleration: one pass over all bodies, not one per level.
  const int z = opaque_zero();  // (a context of its own: see opaque_zero)
  for (int b = 1 + t.lane + z; b < m.nbody; b += t.T) {
    {
      const float* pos = W + z + m.o_xpos + 3 * b;
      const float* R = W + z + m.o_xmat + 9 * b;
      const float* V = W + z + m.o_cvel + 6 * b;
      const float* A = W + z + m.o_cacc + 6 * b;
      // spatial inertia at the world origin: m, h = m c, I_O = R I R^T + m (|c|^2 1 - c c^T)
      float c[3], RI[9], ip[3] = {m.body_ipos[3 * b], m.body_ipos[3 * b + 1],
                                  m.body_ipos[3 * b + 2]};
      float mass = m.body_mass[b];
      if (dr && b == 1) {
        for (int k = 0; k < 3; k++) ip[k] += dr[kDrCom + k];
        mass += dr[kDrPayload];
      }
      mv3(R, ip, c);
      for (int k = 0; k < 3; k++) c[k] += pos[k];
      const float* bi = m.body_inertia + 6 * b;
      float Il[9] = {bi[0], bi[3], bi[4], bi[3], bi[1], bi[5], bi[4], bi[5], bi[2]};
      mm3(R, Il, RI);
      // the six entries of R I R^T the inertia keeps: (R I R^T)_ij = (R I)_i . R_j
      auto iw = [&](int i, int j) {
        return RI[3 * i] * R[3 * j] + RI[3 * i + 1] * R[3 * j + 1] + RI[3 * i + 2] * R[3 * j + 2];
      };
      const float Iw[9] = {iw(0, 0), iw(0, 1), iw(0, 2), 0.f, iw(1, 1), iw(1, 2), 0.f, 0.f,
                           iw(2, 2)};
      const float cc = dot3(c, c);
      float* ci = W + z + m.o_cinert + kCinert * b;
      ci[0] = mass;
      ci[1] = mass * c[0]; ci[2] = mass * c[1]; ci[3] = mass * c[2];
      ci[4] = Iw[0] + mass * (cc - c[0] * c[0]);
      ci[5] = Iw[4] + mass * (cc - c[1] * c[1]);
      ci[6] = Iw[8] + mass * (cc - c[2] * c[2]);
      ci[7] = Iw[1] - mass * c[0] * c[1];
      ci[8] = Iw[2] - mass * c[0] * c[2];
      ci[9] = Iw[5] - mass * c[1] * c[2];
      float IA[6], IV[6], VIV[6];
      inertia_mul(ci, A, IA);
      inertia_mul(ci, V, IV);
      crossf(V, IV, VIV);
      for (int k = 0; k < 6; k++) W[z + m.o_cfrc + 6 * b + k] = IA[k] + VIV[k];
    }
  }
  t.sync();
}

// ------------------------------- A3/A5 backward sweep, bias forces and CRBA (RBDA 6)
DEV void backward_and_mass(const DevModel& m, float* W, const Team& t,
                           const float* dr = nullptr) {
  float* cfrc = W + m.o_cfrc;
  float* Ic = W + m.o_cinert;  // body inertias become subtree (composite) inertias
  const float* cdof = W + m.o_cdof;
  float* F = W + m.o_F;
  float* M = W + m.o_M;
  float* frc = W + m.o_frc;
  for (int lv = m.nlevel - 1; lv >= 1; lv--) {
    const int e = m.level_start[lv + 1];
    for (int ib = m.level_start[lv] + t.lane; ib < e; ib += t.T) {
      const int b = m.level_body[ib];
      float ic[kCinert], f[6];
      for (int k = 0; k < kCinert; k++) ic[k] = Ic[kCinert * b + k];
      for (int k = 0; k < 6; k++) f[k] = cfrc[6 * b + k];
      for (int c = m.child_start[b]; c < m.child_start[b + 1]; c++) {
        const int ch = m.child_list[c];
        for (int k = 0; k < kCinert; k++) ic[k] += Ic[kCinert * ch + k];
        for (int k = 0; k < 6; k++) f[k] += cfrc[6 * ch + k];
      }
      for (int k = 0; k < kCinert; k++) Ic[kCinert * b + k] = ic[k];
      for (int k = 0; k < 6; k++) cfrc[6 * b + k] = f[k];
    }
    t.sync();
  }
  // bias force c_i = S_i . f_subtree; F_i = Ic S_i
  for (int i = t.lane; i < m.nv; i += t.T) {
    const int b = m.dof_body[i];
    frc[i] -= dot6(cdof + 6 * i, cfrc + 6 * b);
    inertia_mul(Ic + kCinert * b, cdof + 6 * i, F + 6 * i);
  }
  t.sync();
  // M_ij = S_j . F_i for j ancestor-or-self of i (other entries stay zero)
  for (int k = t.lane; k < m.nmpair; k += t.T) {
    const int pr = m.mpair[k];
    const int i = pr >> 16, j = pr & 0xffff;
    float v = dot6(cdof + 6 * j, F + 6 * i);
    if (i == j) v += (dr && i >= 6) ? dr[kDrHead + m.nu + i - 6] : m.dof_armature[i];
    M[tri(i, j)] = v;
  }
  t.sync();
}

// ------------------------------------------ A4/A6 sparse L^T D L and a0 = M^-1 frc
// Factor a copy of M in H (no fill-in outside the dof-ancestor pattern), leaves first.
// Eliminating dof k updates the entries among its ancestors with row k unscaled; the
// scaling of row k by 1/D_k waits one elimination (nothing reads it meanwhile), so each
// elimination costs one barrier.  When `rhs` is given, the first triangular solve
// L^T y = rhs rides along: once row k is final, y_i -= L_ki y_k for its ancestors.
// With `hgain` the factor is of M + h diag(dof_vgain) (implicit damping).
DEV void ltdl_factor(const DevModel& m, float* W, const Team& t, float* y = nullptr,
                     bool hgain = false) {
  const float* M = W + m.o_M;
  float* H = W + m.o_H;
  for (int k = t.lane; k < m.ntri; k += t.T) H[k] = M[k];
  t.sync();
  if (hgain) {
    for (int i = t.lane; i < m.nv; i += t.T) H[tri(i, i)] += m.dt * m.dof_vgain[i];
    t.sync();
  }
  for (int k = m.nv - 1; k >= -1; k--) {
    if (k >= 0) {
      const int a0 = m.anc_start[k], na = m.anc_start[k + 1] - a0;
      const float inv = 1.f / H[tri(k, k)];
      const int npr = na * (na + 1) / 2;
      for (int p = t.lane; p < npr; p += t.T) {
        int bi, ai;
        t.unrank(p, bi, ai);
        const int i = m.anc_list[a0 + ai];  // nearer ancestor (larger index)
        const int j = m.anc_list[a0 + bi];  // j ancestor-or-self of i
        H[tri(i, j)] -= H[tri(k, i)] * H[tri(k, j)] * inv;
      }
    }
    const int k1 = k + 1;  // deferred: scale row k1, then propagate y_k1
    if (k1 < m.nv) {
      const int a1 = m.anc_start[k1], n1 = m.anc_start[k1 + 1] - a1;
      const float inv1 = 1.f / H[tri(k1, k1)];
      const float yk = y ? y[k1] : 0.f;
      for (int q = t.lane; q < n1; q += t.T) {
        const int i = m.anc_list[a1 + q];
        const float l = H[tri(k1, i)] * inv1;
        H[tri(k1, i)] = l;
        if (y) y[i] -= l * yk;
      }
    }
    t.sync();
  }
}
// x = M^-1 rhs with the factors in H: L^T y = rhs, y /= D, L x = y (one lane; the
// other lanes wait at the barrier).  rhs and x may alias.  With `half` the first solve
// has already been done by ltdl_factor and x holds y.
DEV void ltdl_solve(const DevModel& m, float* W, const Team& t, const float* rhs, float* x,
                    bool half = false) {
  const float* H = W + m.o_H;
  const int nv = m.nv;
  if (nv <= t.T) {
    // lane k holds entry k; each column's finished entry is broadcast from its lane and
    // applied to the others.  Entries of H off the tree pattern are exact zeros, so
    // the dense column updates equal the ancestor-list ones.
    const int k = t.lane;
    float acc = k < nv ? (half ? x[k] : rhs[k]) : 0.f;
    if (!half) {
      for (int j = nv - 1; j > 0; j--) {  // L^T y = rhs
        const float yj = t.bcast(acc, j);
        if (k < j) acc -= H[tri(j, k)] * yj;
      }
    }
    if (k < nv) acc /= H[tri(k, k)];
    for (int j = 0; j < nv - 1; j++) {  // L x = y / D
      const float xj = t.bcast(acc, j);
      if (k > j && k < nv) acc -= H[tri(k, j)] * xj;
    }
    if (k < nv) x[k] = acc;
    t.sync();
    return;
  }
  if (t.lane == 0) {
    if (!half) {
      for (int i = 0; i < m.nv; i++) x[i] = rhs[i];
      for (int k = m.nv - 1; k >= 0; k--) {
        const float yk = x[k];
        for (int q = m.anc_start[k]; q < m.anc_start[k + 1]; q++) {
          const int i = m.anc_list[q];
          x[i] -= H[tri(k, i)] * yk;
        }
      }
    }
    for (int k = 0; k < m.nv; k++) {
      float s = x[k] / H[tri(k, k)];
      for (int q = m.anc_start[k]; q < m.anc_start[k + 1]; q++) {
        const int i = m.anc_list[q];
        s -= H[tri(k, i)] * x[i];
      }
      x[k] = s;
    }
  }
  t.sync();
}

// ------------------------------------------------------------------ A7: collision
// geom pose from its body's pose
DEV void geom_pose(const DevModel& m, const float* W, int g, float* pos, float* R) {
  const int b = m.geom_body[g];
  const float* xp = W + m.o_xpos + 3 * b;
  const float* xr = W + m.o_xmat + 9 * b;
  mv3(xr, m.geom_pos + 3 * g, pos);
  pos[0] += xp[0]; pos[1] += xp[1]; pos[2] += xp[2];
  mm3(xr, m.geom_rot + 9 * g, R);
}

// signed distance of a box-frame point to a box (half extents h) and the outward
// gradient (box frame)
DEV float box_sdf(const float* p, const float* h, float* grad) {
  float q[3], o[3];
  bool outside = false;
  for (int k = 0; k < 3; k++) {
    q[k] = fabsf(p[k]) - h[k];
    o[k] = fmaxf(q[k], 0.f);
    outside |= q[k] > 0.f;
  }
  if (outside) {
    float L = sqrtf(o[0] * o[0] + o[1] * o[1] + o[2] * o[2]);
    for (int k = 0; k < 3; k++) grad[k] = (p[k] < 0.f ? -1.f : 1.f) * o[k] / L;
    return L;
  }
  int ax = 0;
  if (q[1] > q[ax]) ax = 1;
  if (q[2] > q[ax]) ax = 2;
  grad[0] = grad[1] = grad[2] = 0.f;
  grad[ax] = p[ax] < 0.f ? -1.f : 1.f;
  return q[ax];
}
// box (centre c, rotation R, half extents h) at world point p: sdf and outward
// world normal
DEV float box_point(const float* c, const float* R, const float* h, const float* p, float* n) {
  float rel[3] = {p[0] - c[0], p[1] - c[1], p[2] - c[2]}, pl[3], g[3];
  mtv3(R, rel, pl);
  float s = box_sdf(pl, h, g);
  mv3(R, g, n);
  return s;
}
DEV float box_sdf_only(const float* c, const float* R, const float* h, const float* p) {
  float n[3];
  return box_point(c, R, h, p, n);
}

// capsule segment a + t u (radius r) against a box.  The box SDF f(t) along the
// segment is convex, so f'(t) = grad sdf(p(t)) . u is nondecreasing; the minimiser set
// is bracketed by t_lo = sup{f' < -tau} and t_hi = inf{f' > tau} (tau = 1e-5 |u|),
// found by bisection on the sign of f' -- derivative signs stay reliable in FP32 where
// differences of SDF values do not.  A bracket of length >= 1e-3 is a flat stretch
// (both ends are candidates), otherwise its midpoint is.  Candidates t = 0, t = 1 and
// the interior ones, de-duplicated within 1e-6; the two deepest penetrating ones are
// kept (others get +inf).
constexpr float kCapBoxTau = 1e-5f;
constexpr float kCapBoxFlat = 1e-3f;
constexpr float kCapBoxDup = 1e-6f;
// bisection steps: the bracket of [0, 1] halves to 2^-24, the FP32 spacing near t = 1
// and well inside kCapBoxDup (more steps move the point by less than 3e-9 |u|)
constexpr int kCapBoxBisect = 24;
DEV void capsule_box_cands(const float* a, const float* u, float r, const float* c,
                           const float* R, const float* h, float* dist, float* tpar) {
  auto fprime = [&](float t) {
    float p[3] = {a[0] + t * u[0], a[1] + t * u[1], a[2] + t * u[2]}, n[3];
    box_point(c, R, h, p, n);
    return dot3(n, u);
  };
  const float tau = kCapBoxTau * sqrtf(dot3(u, u));
  float tlo, thi;
  if (!(fprime(0.f) < -tau)) tlo = 0.f;
  else if (fprime(1.f) < -tau) tlo = 1.f;
  else {
    float l = 0.f, g = 1.f;
    for (int it = 0; it < kCapBoxBisect; it++) {
      const float md = 0.5f * (l + g);
      if (fprime(md) < -tau) l = md; else g = md;
    }
    tlo = 0.5f * (l + g);
  }
  if (!(fprime(1.f) > tau)) thi = 1.f;
  else if (fprime(0.f) > tau) thi = 0.f;
  else {
    float l = 0.f, g = 1.f;
    for (int it = 0; it < kCapBoxBisect; it++) {
      const float md = 0.5f * (l + g);
      if (fprime(md) > tau) g = md; else l = md;
    }
    thi = 0.5f * (l + g);
  }
  float ts[4] = {0.f, 1.f, tlo, thi};
  bool keep[4] = {true, true, true, true};
  if (thi - tlo < kCapBoxFlat) {
    ts[2] = 0.5f * (tlo + thi);
    keep[3] = false;
  }
  for (int k = 2; k < 4; k++)
    if (fabsf(ts[k]) < kCapBoxDup || fabsf(ts[k] - 1.f) < kCapBoxDup) keep[k] = false;
  if (keep[2] && keep[3] && fabsf(ts[3] - ts[2]) < kCapBoxDup) keep[3] = false;
  float dep[4];
  for (int k = 0; k < 4; k++) {
    float p[3] = {a[0] + ts[k] * u[0], a[1] + ts[k] * u[1], a[2] + ts[k] * u[2]};
    dep[k] = box_sdf_only(c, R, h, p) - r;
    if (!(dep[k] < 0.f)) keep[k] = false;
  }
  int s0 = -1, s1 = -1;
  for (int k = 0; k < 4; k++)
    if (keep[k] && (s0 < 0 || dep[k] < dep[s0])) s0 = k;
  for (int k = 0; k < 4; k++)
    if (keep[k] && k != s0 && (s1 < 0 || dep[k] < dep[s1])) s1 = k;
  for (int k = 0; k < 4; k++) {
    dist[k] = (k == s0 || k == s1) ? dep[k] : INFINITY;
    tpar[k] = ts[k];
  }
}

// closest points of segments p0 + s d1 and q0 + t d2; parallel ones take the middle
// of the overlap (same rule as the reference)
DEV void seg_seg(const float* p0, const float* d1, const float* q0, const float* d2, float& s,
                 float& t) {
  float r[3] = {p0[0] - q0[0], p0[1] - q0[1], p0[2] - q0[2]};
  float a = dot3(d1, d1), e = dot3(d2, d2), f = dot3(d2, r), c = dot3(d1, r), b = dot3(d1, d2);
  float den = a * e - b * b;
  if (den > 1e-6f * a * e) {
    s = fminf(fmaxf((b * f - c * e) / den, 0.f), 1.f);
    t = (b * s + f) / e;
    if (t < 0.f) { t = 0.f; s = fminf(fmaxf(-c / a, 0.f), 1.f); }
    else if (t > 1.f) { t = 1.f; s = fminf(fmaxf((b - c) / a, 0.f), 1.f); }
  } else {
    float s0 = fminf(fmaxf(-c / a, 0.f), 1.f);
    float s1 = fminf(fmaxf((b - c) / a, 0.f), 1.f);
    s = 0.5f * (s0 + s1);
    t = fminf(fmaxf((b * s + f) / e, 0.f), 1.f);
  }
}

// full contact of two spheres (centres c1, c2): dist, midpoint, normal 1 -> 2
DEV float sphere_sphere(const float* c1, float r1, const float* c2, float r2, float* pos, float* n) {
  float d[3] = {c2[0] - c1[0], c2[1] - c1[1], c2[2] - c1[2]};
  float L = sqrtf(dot3(d, d));
  if (L > 1e-12f) { n[0] = d[0] / L; n[1] = d[1] / L; n[2] = d[2] / L; }
  else { n[0] = 0.f; n[1] = 0.f; n[2] = 1.f; }
  float dist = L - r1 - r2;
  for (int k = 0; k < 3; k++) pos[k] = c1[k] + n[k] * (r1 + 0.5f * dist);
  return dist;
}

// Three-vectors by value: the heightfield test takes its triangle's corners as values,
// never as pointers into local arrays (which would move those arrays to scratch memory).
struct V3 { float x, y, z; };
DEV V3 v3sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
DEV float v3dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
DEV V3 v3cross(V3 a, V3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// nearest point x of segment (s0, s1) to p; keeps it in (best, q) when strictly nearer
DEV void seg_nearest(V3 s0, V3 s1, V3 p, float& best, V3& q) {
  const V3 u = v3sub(s1, s0), w = v3sub(p, s0);
  const float tt = fminf(fmaxf(v3dot(w, u) / v3dot(u, u), 0.f), 1.f);
  const V3 x = {s0.x + tt * u.x, s0.y + tt * u.y, s0.z + tt * u.z};
  const V3 dx = v3sub(p, x);
  const float dd = v3dot(dx, dx);
  if (dd < best) { best = dd; q = x; }
}

// Nearest point of triangle (a, b, c) to p: p's projection onto the triangle's plane
// when its barycentric weights are all >= 0, else the nearest edge point (edges ab, bc,
// ca, the first on ties).  nrm receives the (unnormalised) normal (b - a) x (c - a).
DEV V3 tri_nearest(V3 a, V3 b, V3 c, V3 p, V3& nrm) {
  nrm = v3cross(v3sub(b, a), v3sub(c, a));
  const float hgt = v3dot(v3sub(p, a), nrm) / v3dot(nrm, nrm);
  const V3 pp = {p.x - hgt * nrm.x, p.y - hgt * nrm.y, p.z - hgt * nrm.z};
  const bool in_a = v3dot(v3cross(v3sub(b, pp), v3sub(c, pp)), nrm) >= 0.f;
  const bool in_b = v3dot(v3cross(v3sub(c, pp), v3sub(a, pp)), nrm) >= 0.f;
  const bool in_c = v3dot(v3cross(v3sub(a, pp), v3sub(b, pp)), nrm) >= 0.f;
  if (in_a && in_b && in_c) return pp;
  float best = INFINITY;
  V3 q = a;
  seg_nearest(a, b, p, best, q);
  seg_nearest(b, c, p, best, q);
  seg_nearest(c, a, p, best, q);
  return q;
}

// Sphere (geom 1: centre c, radius r) against the heightfield (geom 2 at xg, Rg): the
// contact is the nearest point of the triangles of the grid cells under the sphere's
// footprint (the first in cell and triangle order on ties), signed by the side of that
// triangle's plane.  The search (hfield_nearest) runs once per candidate in the
// candidate phase and returns the winning triangle as ((i ncol + j) << 1 | k), -1 when
// the footprint misses the grid; sphere_hfield_tri evaluates that one triangle, so the
// inlined contact code holds no loops.

// the sphere centre in the heightfield's frame
DEV V3 hfield_local(const float* xg, const float* Rg, const float* c) {
  const float rx = c[0] - xg[0], ry = c[1] - xg[1], rz = c[2] - xg[2];
  return {Rg[0] * rx + Rg[3] * ry + Rg[6] * rz, Rg[1] * rx + Rg[4] * ry + Rg[7] * rz,
          Rg[2] * rx + Rg[5] * ry + Rg[8] * rz};
}

// triangle k (0: v00 v01 v11, 1: v00 v11 v10) of cell (i, j)
DEV void hfield_tri(const DevModel& m, int i, int j, int k, V3& a, V3& b, V3& c) {
  const int nc = m.hf_ncol;
  const float sx = m.hf_size[0], sy = m.hf_size[1], sz = m.hf_size[2];
  const float dx = 2.f * sx / (nc - 1), dy = 2.f * sy / (m.hf_nrow - 1);
  const float x0 = -sx + dx * j, x1 = x0 + dx, y0 = -sy + dy * i, y1 = y0 + dy;
  const float* hrow = m.hf_data + (size_t)i * nc + j;
  a = {x0, y0, sz * hrow[0]};
  if (k == 0) {
    b = {x1, y0, sz * hrow[1]};
    c = {x1, y1, sz * hrow[nc + 1]};
  } else {
    b = {x1, y1, sz * hrow[nc + 1]};
    c = {x0, y1, sz * hrow[nc]};
  }
}

DEV int hfield_nearest(const DevModel& m, const float* xg, const float* Rg, const float* c,
                       float r) {
  const int nr = m.hf_nrow, nc = m.hf_ncol;
  const float sx = m.hf_size[0], sy = m.hf_size[1];
  const float dx = 2.f * sx / (nc - 1), dy = 2.f * sy / (nr - 1);
  const V3 cl = hfield_local(xg, Rg, c);
  // cell range of the footprint, clamped before the conversion to int
  auto cell = [](float x, int hi) { return (int)floorf(fminf(fmaxf(x, -1.f), (float)hi)); };
  const int j0 = max(0, cell((cl.x - r + sx) / dx, nc));
  const int j1 = min(nc - 2, cell((cl.x + r + sx) / dx, nc));
  const int i0 = max(0, cell((cl.y - r + sy) / dy, nr));
  const int i1 = min(nr - 2, cell((cl.y + r + sy) / dy, nr));
  float best = INFINITY;
  int code = -1;
  for (int i = i0; i <= i1; i++)
    for (int j = j0; j <= j1; j++)
      for (int k = 0; k < 2; k++) {
        V3 a, b, cc, nt;
        hfield_tri(m, i, j, k, a, b, cc);
        const V3 d = v3sub(cl, tri_nearest(a, b, cc, cl, nt));
        const float dd = v3dot(d, d);
        if (dd < best) { best = dd; code = ((i * nc + j) << 1) | k; }
      }
  return code;
}

// The contact with triangle `code`: the normal points from the sphere into the surface
// and pos is midway between the surfaces; +inf for code < 0.
DEV float sphere_hfield_tri(const DevModel& m, const float* xg, const float* Rg, const float* c,
                            float r, int code, float* pos, float* n) {
  if (code < 0) return INFINITY;
  const int cellid = code >> 1, k = code & 1;
  const int i = cellid / m.hf_ncol, j = cellid - i * m.hf_ncol;
  const V3 cl = hfield_local(xg, Rg, c);
  V3 a, b, cc, bn;
  hfield_tri(m, i, j, k, a, b, cc);
  const V3 bq = tri_nearest(a, b, cc, cl, bn);
  const V3 d = v3sub(cl, bq);
  const float L = sqrtf(v3dot(d, d));
  const bool below = v3dot(bn, d) < 0.f;
  float nl[3];
  if (L > 1e-12f) {
    const float sg = (below ? 1.f : -1.f) / L;
    nl[0] = sg * d.x; nl[1] = sg * d.y; nl[2] = sg * d.z;
  } else {
    const float inv = -1.f / sqrtf(v3dot(bn, bn));
    nl[0] = inv * bn.x; nl[1] = inv * bn.y; nl[2] = inv * bn.z;
  }
  const float bqa[3] = {bq.x, bq.y, bq.z};
  float qw[3];
  mv3(Rg, nl, n);
  mv3(Rg, bqa, qw);
  for (int q = 0; q < 3; q++) pos[q] = 0.5f * (c[q] + r * n[q] + qw[q] + xg[q]);
  return (below ? -L : L) - r;
}

// Evaluate candidate `sub` of pair `p` (kind-specific); returns dist and fills pos and
// normal.  For capsule-box the parameter t selects the segment point.
DEV float pair_contact(const DevModel& m, const float* W, int p, int sub, float tpar, float* pos,
                       float* n) {
  const int g1 = m.pair_g1[p], g2 = m.pair_g2[p];
  float x1[3], R1[9], x2[3], R2[9];
  geom_pose(m, W, g1, x1, R1);
  geom_pose(m, W, g2, x2, R2);
  const float* s1 = m.geom_size + 3 * g1;
  const float* s2 = m.geom_size + 3 * g2;
  const float z1[3] = {R1[2], R1[5], R1[8]};
  const float z2[3] = {R2[2], R2[5], R2[8]};
  switch (m.pair_kind[p]) {
    case PK_PLANE_SPHERE:
    case PK_PLANE_CAPSULE: {
      float c[3] = {x2[0], x2[1], x2[2]};
      if (m.pair_kind[p] == PK_PLANE_CAPSULE) {
        const float sg = sub == 0 ? -s2[1] : s2[1];
        for (int k = 0; k < 3; k++) c[k] += sg * z2[k];
      }
      float rel[3] = {c[0] - x1[0], c[1] - x1[1], c[2] - x1[2]};
      float dist = dot3(z1, rel) - s2[0];
      for (int k = 0; k < 3; k++) { n[k] = z1[k]; pos[k] = c[k] - z1[k] * (s2[0] + 0.5f * dist); }
      return dist;
    }
    case PK_PLANE_BOX: {
      float loc[3] = {(sub & 1) ? s2[0] : -s2[0], (sub & 2) ? s2[1] : -s2[1],
                      (sub & 4) ? s2[2] : -s2[2]}, w[3], cor[3];
      mv3(R2, loc, w);
      for (int k = 0; k < 3; k++) cor[k] = x2[k] + w[k];
      float rel[3] = {cor[0] - x1[0], cor[1] - x1[1], cor[2] - x1[2]};
      float dist = dot3(z1, rel);
      for (int k = 0; k < 3; k++) { n[k] = z1[k]; pos[k] = cor[k] - 0.5f * dist * z1[k]; }
      return dist;
    }
    case PK_SPHERE_SPHERE:
      return sphere_sphere(x1, s1[0], x2, s2[0], pos, n);
    case PK_SPHERE_CAPSULE: {
      float a[3], u[3];
      for (int k = 0; k < 3; k++) { a[k] = x2[k] - s2[1] * z2[k]; u[k] = 2.f * s2[1] * z2[k]; }
      float uu = dot3(u, u);
      float ap[3] = {x1[0] - a[0], x1[1] - a[1], x1[2] - a[2]};
      float t = uu < 1e-30f ? 0.f : fminf(fmaxf(dot3(ap, u) / uu, 0.f), 1.f);
      float q[3] = {a[0] + t * u[0], a[1] + t * u[1], a[2] + t * u[2]};
      return sphere_sphere(x1, s1[0], q, s2[0], pos, n);
    }
    case PK_SPHERE_HFIELD:  // tpar: the winning triangle found in the candidate phase
      return sphere_hfield_tri(m, x2, R2, x1, s1[0], __float_as_int(tpar), pos, n);
    case PK_SPHERE_BOX: {
      float nb[3];
      float sd = box_point(x2, R2, s2, x1, nb);
      for (int k = 0; k < 3; k++) { n[k] = -nb[k]; pos[k] = x1[k] - 0.5f * (s1[0] + sd) * nb[k]; }
      return sd - s1[0];
    }
    case PK_CAPSULE_CAPSULE: {
      float a[3], u[3], b[3], w[3];
      for (int k = 0; k < 3; k++) {
        a[k] = x1[k] - s1[1] * z1[k]; u[k] = 2.f * s1[1] * z1[k];
        b[k] = x2[k] - s2[1] * z2[k]; w[k] = 2.f * s2[1] * z2[k];
      }
      float s, t;
      seg_seg(a, u, b, w, s, t);
      float pp[3] = {a[0] + s * u[0], a[1] + s * u[1], a[2] + s * u[2]};
      float qq[3] = {b[0] + t * w[0], b[1] + t * w[1], b[2] + t * w[2]};
      return sphere_sphere(pp, s1[0], qq, s2[0], pos, n);
    }
    case PK_CAPSULE_BOX: {
      float pt[3], nb[3];
      for (int k = 0; k < 3; k++) pt[k] = x1[k] + (2.f * tpar - 1.f) * s1[1] * z1[k];
      float sd = box_point(x2, R2, s2, pt, nb);
      for (int k = 0; k < 3; k++) { n[k] = -nb[k]; pos[k] = pt[k] - 0.5f * (s1[0] + sd) * nb[k]; }
      return sd - s1[0];
    }
  }
  return INFINITY;
}

// Phase 1: every pair writes its candidates' distances (and parameters) into the
// candidate slots; non-penetrating / not-kept candidates get +inf.
DEV void collide_candidates(const DevModel& m, float* W, const Team& t) {
  float* cd = W + m.o_cand;
  float* cp = cd + m.ncand;
  for (int p = t.lane; p < m.npair; p += t.T) {
    const int base = m.pair_candadr[p];
    const int kind = m.pair_kind[p];
    if (kind == PK_CAPSULE_BOX) {
      const int g1 = m.pair_g1[p], g2 = m.pair_g2[p];
      float x1[3], R1[9], x2[3], R2[9];
      geom_pose(m, W, g1, x1, R1);
      geom_pose(m, W, g2, x2, R2);
      const float* s1 = m.geom_size + 3 * g1;
      const float* h = m.geom_size + 3 * g2;
      // bounding spheres reject far pairs without changing any result
      float dc[3] = {x2[0] - x1[0], x2[1] - x1[1], x2[2] - x1[2]};
      float rb = sqrtf(h[0] * h[0] + h[1] * h[1] + h[2] * h[2]);
      if (sqrtf(dot3(dc, dc)) > rb + s1[1] + s1[0]) {
        for (int k = 0; k < 4; k++) { cd[base + k] = INFINITY; cp[base + k] = 0.f; }
        continue;
      }
      float a[3], u[3];
      for (int k = 0; k < 3; k++) { a[k] = x1[k] - s1[1] * R1[3 * k + 2]; u[k] = 2.f * s1[1] * R1[3 * k + 2]; }
      float dist[4], tp[4];
      capsule_box_cands(a, u, s1[0], x2, R2, h, dist, tp);
      for (int k = 0; k < 4; k++) { cd[base + k] = dist[k]; cp[base + k] = tp[k]; }
    } else if (kind == PK_PLANE_BOX) {
      float dist[8];
      float pos[3], n[3];
      for (int k = 0; k < 8; k++) {
        float d = pair_contact(m, W, p, k, 0.f, pos, n);
        dist[k] = d < 0.f ? d : INFINITY;
      }
      // keep the 4 deepest (ties to the lower corner)
      unsigned used = 0;
      for (int s = 0; s < 4; s++) {
        int best = -1;
        for (int k = 0; k < 8; k++)
          if (!(used >> k & 1) && dist[k] < INFINITY && (best < 0 || dist[k] < dist[best])) best = k;
        if (best < 0) break;
        used |= 1u << best;
      }
      for (int k = 0; k < 8; k++) { cd[base + k] = (used >> k & 1) ? dist[k] : INFINITY; cp[base + k] = 0.f; }
    } else if (kind == PK_SPHERE_HFIELD) {
      const int g1 = m.pair_g1[p], g2 = m.pair_g2[p];
      float x1[3], R1[9], x2[3], R2[9];
      geom_pose(m, W, g1, x1, R1);
      geom_pose(m, W, g2, x2, R2);
      const float r = m.geom_size[3 * g1];
      const int code = hfield_nearest(m, x2, R2, x1, r);
      float pos[3], n[3];
      const float d = sphere_hfield_tri(m, x2, R2, x1, r, code, pos, n);
      cd[base] = d < 0.f ? d : INFINITY;
      cp[base] = __int_as_float(code);
    } else {
      const int nc = kind == PK_PLANE_CAPSULE ? 2 : 1;
      float pos[3], n[3];
      for (int k = 0; k < nc; k++) {
        float d = pair_contact(m, W, p, k, 0.f, pos, n);
        cd[base + k] = d < 0.f ? d : INFINITY;
        cp[base + k] = 0.f;
      }
    }
  }
  t.sync();
}

// contact frame: tangent 1 from the world axis least aligned with the normal (lowest
// index on ties), tangent 2 = n x t1
DEV void contact_frame(const float* n, float* fr) {
  int ax = 0;
  if (fabsf(n[1]) < fabsf(n[ax])) ax = 1;
  if (fabsf(n[2]) < fabsf(n[ax])) ax = 2;
  float en = n[ax];
  float t1[3] = {-en * n[0], -en * n[1], -en * n[2]};
  t1[ax] += 1.f;
  float inv = 1.f / sqrtf(dot3(t1, t1));
  for (int k = 0; k < 3; k++) t1[k] *= inv;
  float t2[3];
  cross3(n, t1, t2);
  for (int k = 0; k < 3; k++) { fr[k] = n[k]; fr[3 + k] = t1[k]; fr[6 + k] = t2[k]; }
}

// Phase 2: select the contacts (all penetrating candidates in slot order, or on
// overflow the nconmax deepest, ties to the lower slot) and build their records.
DEV void select_contacts(const DevModel& m, float* W, const Team& t, int& status,
                         const float* dr = nullptr) {
  const float* cd = W + m.o_cand;
  const float* cp = cd + m.ncand;
  float* con = W + m.o_con;
  int* scal = (int*)(W + m.o_scal);
  // count penetrating candidates
  int cnt = 0;
  for (int c = t.lane; c < m.ncand; c += t.T) cnt += cd[c] < INFINITY;
  const int total = t.isum(cnt);
  const bool overflow = total > m.nconmax;
  if (overflow) status |= 2;
  int base = 0;
  for (int c0 = 0; c0 < m.ncand; c0 += t.T) {
    const int c = c0 + t.lane;
    bool sel = false;
    if (c < m.ncand && cd[c] < INFINITY) {
      sel = true;
      if (overflow) {
        int rank = 0;
        const float dc = cd[c];
        for (int q = 0; q < m.ncand; q++) {
          const float dq = cd[q];
          rank += (dq < dc) || (dq == dc && q < c);
        }
        sel = rank < m.nconmax;
      }
    }
    const int slot = base + t.exscan(sel ? 1 : 0);
    if (sel) {
      const int p = m.cand_pair[c];
      const int sub = c - m.pair_candadr[p];
      float pos[3], n[3];
      const float dist = pair_contact(m, W, p, sub, cp[c], pos, n);
      float* r = con + kConRec * slot;
      r[0] = dist;
      r[1] = pos[0]; r[2] = pos[1]; r[3] = pos[2];
      contact_frame(n, r + 4);
      // a frictionless pair keeps four rows, all along the normal (mu = 0)
      r[13] = m.pair_condim[p] == 1 ? 0.f : (dr ? m.pair_mu[p] * dr[kDrFric] : m.pair_mu[p]);
      r[14] = __int_as_float(m.geom_body[m.pair_g1[p]]);
      r[15] = __int_as_float(m.geom_body[m.pair_g2[p]]);
      r[16] = __int_as_float(p);
      r[17] = __int_as_float(sub);
    }
    base += t.isum(sel ? 1 : 0);
  }
  if (t.lane == 0) scal[SC_NCON] = base;
  t.sync();
}

// ------------------------------------------------------------- A8: constraint rows
// impedance d(r) of the soft-constraint model from solimp (dmin, dmax, width, mid, power)
DEV float impedance(const DevModel& m, float dist) {
  const float x = fminf(fabsf(dist) / m.width, 1.f);
  float y;
  if (x <= m.mid) y = powf(x, m.power) / powf(m.mid, m.power - 1.f);
  else y = 1.f - powf(1.f - x, m.power) / powf(1.f - m.mid, m.power - 1.f);
  return m.dmin + y * (m.dmax - m.dmin);
}

// rows with a per-row force bound (friction loss, equalities): the bound array exists
DEV bool has_bounds(const DevModel& m) { return m.nfric + m.neq > 0; }

// world positions of connect equality q's point through body1 (p1) and body2 (p2)
DEV void eq_points(const DevModel& m, const float* W, int q, float* p1, float* p2) {
  const int b1 = m.eq_body[2 * q], b2 = m.eq_body[2 * q + 1];
  const float* a = m.eq_anchor + 6 * q;
  mv3(W + m.o_xmat + 9 * b1, a, p1);
  mv3(W + m.o_xmat + 9 * b2, a + 3, p2);
  for (int k = 0; k < 3; k++) {
    p1[k] += W[m.o_xpos + 3 * b1 + k];
    p2[k] += W[m.o_xpos + 3 * b2 + k];
  }
}

// Weld rotational residual, component k: with E = R1 Q R2^T (identity while the weld
// holds), r = vee(E - E^T) / 2 = sin(angle) axis in the world frame, whose rate at E = I
// is w1 - w2.
DEV float weld_residual(const DevModel& m, const float* W, int q, int k) {
  const float* R1 = W + m.o_xmat + 9 * m.eq_body[2 * q];
  const float* R2 = W + m.o_xmat + 9 * m.eq_body[2 * q + 1];
  const float* Q = m.eq_relR + 9 * q;
  const int i = k == 0 ? 2 : (k == 1 ? 0 : 1), j = k == 0 ? 1 : (k == 1 ? 2 : 0);
  float eij = 0.f, eji = 0.f;  // E_ij and E_ji
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) {
      eij += R1[3 * i + a] * Q[3 * a + b] * R2[3 * j + b];
      eji += R1[3 * j + a] * Q[3 * a + b] * R2[3 * i + b];
    }
  return 0.5f * (eij - eji);
}

// violated joint limit k of a world (its o_lim entry): dof, sign of its row and distance
DEV void limit_row(const DevModel& m, const float* W, int code, int& dof, float& sg,
                   float& dist) {
  const int l = code & 0xffff;
  const bool upper = code >> 16;
  const float q = W[m.o_qpos + m.lim_qadr[l]];
  dof = m.lim_dadr[l];
  sg = upper ? -1.f : 1.f;
  dist = upper ? m.lim_hi[l] - q : q - m.lim_lo[l];
}

// Pyramid rows J_e = J_n +- mu J_tk (order +t1, -t1, +t2, -t2) from the point
// Jacobians of the two bodies at the contact point; impedance d(r), reference
// acceleration aref = -B (J_e qvel) - K d(r) r, regulariser R = (1-d)/d (1+mu^2)
// (w1 + w2), D = 1/R.  Then one row per joint outside its range, in joint order:
// J = +-e_dof, r the distance past the range end, R = (1-d)/d (M^-1)_kk at qpos0.
// Then one friction-loss row per dof with a bound F > 0, always: J = e_dof, r = 0,
// the same R, and the bound stored per row (0 marks a one-sided row).  Then three
// two-sided rows per connect equality (bound +inf): with p1, p2 the held point through
// body1 and body2, J = J_p(b1, p1) - J_p(b2, p2) per world axis, r = p1 - p2,
// R = (1-d)/d (w1 + w2); a weld adds three rotational rows, J = J_w(b1) - J_w(b2) per
// world axis with r its rotation residual (weld_residual) and the same R.  Writes the
// row count to the SC_NROW slot.
DEV void constraint_rows(const DevModel& m, float* W, const Team& t) {
  int* scal = (int*)(W + m.o_scal);
  const int ncon = scal[SC_NCON];
  const int nv = m.nv;
  float* con = W + m.o_con;
  // each contact's rows (1 frictionless; else two pyramid edges per friction direction,
  // 4, 6 or 10, or an elliptic cone's condim frame rows) and its first row.  With every
  // pair at condim 3 they are con_nr and con_nr c; otherwise a prefix sum in contact
  // order packs them into the record's slot word (candidate slot | rows << 4 | first
  // row << 8).
  int nrc = m.con_nr * ncon;
  if (!m.con_nr) {
    nrc = 0;
    for (int c0 = 0; c0 < ncon; c0 += t.T) {
      const int c = c0 + t.lane;
      int nr = 0;
      if (c < ncon) {
        const int cd = m.pair_condim[__float_as_int(con[kConRec * c + 16])];
        nr = (cd == 1 || m.cone) ? cd : 2 * (cd - 1);
      }
      const int first = nrc + t.exscan(nr);
      if (c < ncon) {
        const int sub = __float_as_int(con[kConRec * c + 17]) & 15;
        con[kConRec * c + 17] = __int_as_float(sub | (nr << 4) | (first << 8));
      }
      nrc += t.isum(nr);
    }
    t.sync();
  }
  const float* cdof = W + m.o_cdof;
  float* J = W + m.o_J;
  // violated limits, compacted in joint order
  int nl = 0;
  int* lim = (int*)(W + m.o_lim);
  for (int l0 = 0; l0 < m.nlim; l0 += t.T) {
    const int l = l0 + t.lane;
    int code = -1;
    if (l < m.nlim) {
      const float q = W[m.o_qpos + m.lim_qadr[l]];
      if (q < m.lim_lo[l]) code = l;
      else if (q > m.lim_hi[l]) code = l | 0x10000;
    }
    const int act = code >= 0 ? 1 : 0;
    const int slot = nl + t.exscan(act);
    if (act) lim[slot] = code;
    nl += t.isum(act);
  }
  const int nrf = nrc + nl;  // first friction-loss row
  const int nre = nrf + m.nfric;  // first equality row
  const int nrow = nre + m.neqrow;
  if (t.lane == 0) {
    scal[SC_NROW] = nrow;
    scal[SC_NRC] = nrc;
  }
  for (int idx = t.lane; idx < ncon * nv; idx += t.T) {
    const int c = idx / nv, i = idx - c * nv;
    const float* r = con + kConRec * c;
    const int b1 = __float_as_int(r[14]), b2 = __float_as_int(r[15]);
    const unsigned long long bit = 1ull << i;
    float jd[3] = {0.f, 0.f, 0.f}, jw[3] = {0.f, 0.f, 0.f};
    const bool in2 = (m.body_dofmask[b2] & bit) != 0;
    const bool in1 = (m.body_dofmask[b1] & bit) != 0;
    if (in1 != in2) {
      const float* S = cdof + 6 * i;
      float wx[3];
      cross3(S, r + 1, wx);
      const float sg = in2 ? 1.f : -1.f;
      for (int k = 0; k < 3; k++) {
        jd[k] = sg * (S[3 + k] + wx[k]);
        jw[k] = sg * S[k];  // relative angular velocity (torsion and rolling rows)
      }
    }
    const int slot = __float_as_int(r[17]);
    const int first = m.con_nr ? m.con_nr * c : slot >> 8, nr = m.con_nr ? m.con_nr : (slot >> 4) & 15;
    const float jn = dot3(r + 4, jd);
    float* Jr = J + (m.jframe ? 3 * c : first) * nv + i;
    if (nr == 1) {  // frictionless
      Jr[0] = jn;
    } else if (m.jframe) {  // the pyramid's frame: normal, tangents
      Jr[0] = jn;
      Jr[nv] = dot3(r + 7, jd);
      Jr[2 * nv] = dot3(r + 10, jd);
    } else if (m.cone) {  // elliptic: normal, tangents, spin (condim 4), rolling (6)
      Jr[0] = jn;
      Jr[nv] = dot3(r + 7, jd);
      Jr[2 * nv] = dot3(r + 10, jd);
      if (nr > 3) {
        Jr[3 * nv] = dot3(r + 4, jw);
        if (nr > 4) {
          Jr[4 * nv] = dot3(r + 7, jw);
          Jr[5 * nv] = dot3(r + 10, jw);
        }
      }
    } else {  // edges J_n +- mu J_dir: tangents, then spin (condim 4), then rolling (6)
      const float j1 = dot3(r + 7, jd), j2 = dot3(r + 10, jd);
      const float mu = r[13];
      Jr[0] = jn + mu * j1;
      Jr[nv] = jn - mu * j1;
      Jr[2 * nv] = jn + mu * j2;
      Jr[3 * nv] = jn - mu * j2;
      if (nr > 4) {
        const int p = __float_as_int(r[16]);
        const float mt = m.pair_mu_t[p], js = dot3(r + 4, jw);
        Jr[4 * nv] = jn + mt * js;
        Jr[5 * nv] = jn - mt * js;
        if (nr > 6) {
          const float mr = m.pair_mu_r[p], jr1 = dot3(r + 7, jw), jr2 = dot3(r + 10, jw);
          Jr[6 * nv] = jn + mr * jr1;
          Jr[7 * nv] = jn - mr * jr1;
          Jr[8 * nv] = jn + mr * jr2;
          Jr[9 * nv] = jn - mr * jr2;
        }
      }
    }
  }
  // J row of row nrc (the first non-contact row): frame-row contacts keep 3 of their 4
  float* Jo = J + (m.jframe ? 3 * ncon : nrc) * nv;
  for (int idx = t.lane; idx < nl * nv; idx += t.T) {
    const int k = idx / nv, i = idx - k * nv;
    int dof;
    float sg, dist;
    limit_row(m, W, lim[k], dof, sg, dist);
    Jo[k * nv + i] = i == dof ? sg : 0.f;
  }
  for (int idx = t.lane; idx < m.nfric * nv; idx += t.T) {
    const int k = idx / nv, i = idx - k * nv;
    Jo[(nl + k) * nv + i] = i == m.fric_dadr[k] ? 1.f : 0.f;
  }
  for (int idx = t.lane; idx < m.neqrow * nv; idx += t.T) {
    const int er = idx / nv, i = idx - er * nv;
    const int q = m.eq_row[er] & 0xffff, k = m.eq_row[er] >> 16;
    const unsigned long long bit = 1ull << i;
    const float* S = cdof + 6 * i;
    const bool in1 = (m.body_dofmask[m.eq_body[2 * q]] & bit) != 0;
    const bool in2 = (m.body_dofmask[m.eq_body[2 * q + 1]] & bit) != 0;
    float jv = 0.f;
    if (k < 3) {  // translational: J_p(b1, p1) - J_p(b2, p2), component k
      float p1[3], p2[3];
      eq_points(m, W, q, p1, p2);
      if (in1) {
        float wx[3];
        cross3(S, p1, wx);
        jv += S[3 + k] + wx[k];
      }
      if (in2) {
        float wx[3];
        cross3(S, p2, wx);
        jv -= S[3 + k] + wx[k];
      }
    } else {  // rotational: J_w(b1) - J_w(b2), component k - 3
      jv = (in1 ? S[k - 3] : 0.f) - (in2 ? S[k - 3] : 0.f);
    }
    Jo[(nl + m.nfric + er) * nv + i] = jv;
  }
  t.sync();
  const float* qvel = W + m.o_qvel;
  float* aref = W + m.o_aref;
  float* D = W + m.o_D;
  // frame-row contacts: the rows' J qvel from their frames' products, staged in o_fw
  float* pf = W + m.o_fw;
  if (m.jframe) {
    for (int f = t.lane; f < nrow - ncon; f += t.T) {
      float v = 0.f;
      for (int i = 0; i < nv; i++) v += J[f * nv + i] * qvel[i];
      pf[f] = v;
    }
    t.sync();
  }
  for (int row = t.lane; row < nrow; row += t.T) {
    float dist, jv = 0.f, A;
    if (row < nrc) {
      int c = m.con_nr ? row / m.con_nr : 0;  // con_nr rows a contact when uniform
      if (!m.con_nr)
        while (c + 1 < ncon && (__float_as_int(con[kConRec * (c + 1) + 17]) >> 8) <= row) c++;
      const float* r = con + kConRec * c;
      dist = r[0];
      if (m.jframe) {
        const int k = row & 3;
        jv = pf[3 * c] + ((k & 1) ? -r[13] : r[13]) * pf[3 * c + 1 + (k >> 1)];
      } else {
        for (int i = 0; i < nv; i++) jv += J[row * nv + i] * qvel[i];
      }
      const int b1 = __float_as_int(r[14]), b2 = __float_as_int(r[15]);
      const float mu = r[13];  // 0 for a frictionless contact: A = w1 + w2
      if (m.cone) {
        // elliptic: the normal row's impedance and A = w1 + w2 for every row; a friction
        // row has no distance term and D scaled by (mu_j / mu)^2
        const int first = m.con_nr ? m.con_nr * c : __float_as_int(r[17]) >> 8;
        const int k = row - first;
        A = m.body_invweight[b1] + m.body_invweight[b2];
        if (k > 0) {
          const int p = __float_as_int(r[16]);
          const float ratio = k < 3 ? 1.f : (k == 3 ? m.pair_mu_t[p] : m.pair_mu_r[p]) / mu;
          const float imp = impedance(m, dist);
          aref[row] = -m.B * jv;
          D[row] = ratio * ratio * imp / ((1.f - imp) * fmaxf(A, 1e-15f));
          if (has_bounds(m)) W[m.o_fl + row] = 0.f;
          continue;
        }
      } else {
        A = (1.f + mu * mu) * (m.body_invweight[b1] + m.body_invweight[b2]);
      }
    } else if (row < nrf) {
      const int code = lim[row - nrc];
      int dof;
      float sg;
      limit_row(m, W, code, dof, sg, dist);
      jv = sg * qvel[dof];
      A = m.dof_invweight[dof];
    } else if (row < nre) {
      const int dof = m.fric_dadr[row - nrf];
      dist = 0.f;
      jv = qvel[dof];
      A = m.dof_invweight[dof];
    } else {
      const int q = m.eq_row[row - nre] & 0xffff, k = m.eq_row[row - nre] >> 16;
      if (k < 3) {
        float p1[3], p2[3];
        eq_points(m, W, q, p1, p2);
        dist = p1[k] - p2[k];
      } else {
        dist = weld_residual(m, W, q, k - 3);
      }
      if (m.jframe) {
        jv = pf[row - ncon];
      } else {
        for (int i = 0; i < nv; i++) jv += J[row * nv + i] * qvel[i];
      }
      A = m.body_invweight[m.eq_body[2 * q]] + m.body_invweight[m.eq_body[2 * q + 1]];
    }
    const float imp = impedance(m, dist);
    aref[row] = -m.B * jv - m.K * imp * dist;
    D[row] = imp / ((1.f - imp) * fmaxf(A, 1e-15f));
    if (has_bounds(m))
      W[m.o_fl + row] = row < nrf ? 0.f : (row < nre ? m.fric_loss[row - nrf] : INFINITY);
  }
  t.sync();
}

// Pieces of a row's cost s(e) in the Newton solve: one-sided rows (bound F = 0)
// s = 1/2 D min(0, e)^2; friction-loss rows (F > 0) the Huber term, 1/2 D e^2 while
// |D e| <= F, else F |e| - F^2 / (2 D); two-sided rows (F = +inf) 1/2 D e^2.
DEV float row_cost(float D, float F, float e) {
  if (F == 0.f) return e < 0.f ? 0.5f * D * e * e : 0.f;
  return fabsf(D * e) <= F ? 0.5f * D * e * e : F * fabsf(e) - 0.5f * F * F / D;
}
DEV float row_slope(float D, float F, float e) {  // s'(e), D min(0, e) or clamp(D e, +-F)
  const float v = D * e;
  return F == 0.f ? fminf(v, 0.f) : fminf(fmaxf(v, -F), F);
}
DEV bool row_quad(float D, float F, float e) {  // on the quadratic piece: curvature D
  return F == 0.f ? e < 0.f : fabsf(D * e) < F;
}
// which piece of its cost a row is on: 1 quadratic; 0 inactive (one-sided row) or the
// friction bound -F; 2 the bound +F
DEV int row_piece(float D, float F, float e) {
  if (F == 0.f) return e < 0.f ? 1 : 0;
  const float v = D * e;
  return v >= F ? 2 : (v <= -F ? 0 : 1);
}

// --------------------------------------------------- A9: Newton solve (NW ch. 3, 6)
// Loops over all constraint rows run to a wave-uniform bound (the largest row count
// among the wavefront's worlds), which keeps them off the EXEC mask.  Every lane reads
// the row counts that the wavefront's teams stored in their own LDS (slot SC_NROW,
// written by constraint_rows before its last barrier), clamped to [0, nrowmax]: teams
// that left the kernel never wrote theirs, and cross-lane operations are not used here
// because teams may be inactive.  A world's rows from its own count up to the bound are
// zeroed (J, D, e, s), so they add nothing to gradients, Hessian or line search.
// With frame-row contacts (jframe) the non-contact rows follow a world's 4 ncon edge
// rows and 3 ncon frame rows; their loops run to nou, the largest non-contact row count
// in the wavefront, and the padding reaches edge row 4 ncon + nou and J row 3 ncon + nou.
struct RowBounds {
  int nru;  // rows
  int nou;  // non-contact rows (jframe only, else 0)
};
DEV RowBounds pad_rows(const DevModel& m, float* W, const Team& t, int nrow) {
  const int tw = 64 / t.T;                              // teams per wavefront
  const int my = (int)((threadIdx.x & 63) / t.T);      // this team's place in it
  // a team that left holds stale counts: clamping them to the model's maxima keeps every
  // padded index inside its region (non-contact rows: at most nrowmax - 4 nconmax)
  const int nomax = m.nrowmax - 4 * m.nconmax;
  int mx = 0, mo = 0;
  for (int k = 0; k < tw; k++) {
    const int* sk = (const int*)(W + (k - my) * m.lds_words + m.o_scal);
    const int nr = min(max(sk[SC_NROW], 0), m.nrowmax);
    mx = max(mx, nr);
    if (m.jframe)
      mo = max(mo, min(max(nr - 4 * min(max(sk[SC_NCON], 0), m.nconmax), 0), nomax));
  }
  // every active lane computed the same bounds, and this team's own counts are among them
  RowBounds rb;
  rb.nru = __builtin_amdgcn_readfirstlane(mx);
  rb.nou = __builtin_amdgcn_readfirstlane(mo);
  const int nv = m.nv;
  int rend = rb.nru, jfirst = nrow, jend = rb.nru;  // zeroed: rows [nrow, rend), J rows [jfirst, jend)
  if (m.jframe) {
    const int ncon = ((const int*)(W + m.o_scal))[SC_NCON];
    rend = max(rb.nru, 4 * ncon + rb.nou);
    jfirst = nrow - ncon;
    jend = 3 * ncon + rb.nou;
  }
  float* J = W + m.o_J;
  for (int k = jfirst * nv + t.lane; k < jend * nv; k += t.T) J[k] = 0.f;
  float* D = W + m.o_D;
  float* e = W + m.o_e;
  float* s = W + m.o_s;
  for (int r = nrow + t.lane; r < rend; r += t.T) { D[r] = 0.f; e[r] = 0.f; s[r] = 0.f; }
  if (has_bounds(m))
    for (int r = nrow + t.lane; r < rend; r += t.T) W[m.o_fl + r] = 0.f;
  t.sync();
  return rb;
}

// Entry i of row r's Jacobian (nrc = 4 ncon contact rows; frame-row contacts form the
// edge J_n +- mu J_tk from their frames).  For the few per-row reads of the adjoint.
DEV float row_entry(const DevModel& m, const float* W, int r, int i, int ncon) {
  const float* J = W + m.o_J;
  const int nv = m.nv;
  if (!m.jframe) return J[r * nv + i];
  if (r >= 4 * ncon) return J[(r - ncon) * nv + i];
  const int c = r >> 2, k = r & 3;
  const float mu = W[m.o_con + kConRec * c + 13];
  return J[3 * c * nv + i] + ((k & 1) ? -mu : mu) * J[(3 * c + 1 + (k >> 1)) * nv + i];
}

// Products with the constraint rows.  rows_times: out[r] = J_r x for r < max(nru, 4 ncon
// + nou) (0 past the world's rows).  rows_t_times: out_i = init_i + sum_r y(r) J_ri over
// the same rows, y a row functor (0 past the world's rows).  With frame-row contacts the
// frames' products (or weights) are staged in o_fw: a contact's edges J_n +- mu J_tk take
// J_n x +- mu J_tk x, and its frames' weights are sum_e y_e on J_n and mu (y_+ - y_-) on
// J_tk.  Both end with a barrier; out may alias init.
DEV void rows_times(const DevModel& m, float* W0, const Team& t0, int nrow, const RowBounds& rb,
                    const float* x, float* out) {
  float* W = W0 + opaque_zero();
  const Team t{t0.lane + opaque_zero(), t0.T, t0.tp};
  const int nv = m.nv;
  const float* J = W + m.o_J;
  if (!m.jframe) {
    for (int r = t.lane; r < rb.nru; r += t.T) {
      float v = 0.f;
      for (int i = 0; i < nv; i++) v += J[r * nv + i] * x[i];
      out[r] = v;
    }
    t.sync();
    return;
  }
  const int ncon = ((const int*)(W + m.o_scal))[SC_NCON];
  const float* con = W + m.o_con;
  float* pf = W + m.o_fw;
  const int nf = 3 * ncon + rb.nou;
  for (int f = t.lane; f < nf; f += t.T) {
    float v = 0.f;
    for (int i = 0; i < nv; i++) v += J[f * nv + i] * x[i];
    pf[f] = v;
  }
  t.sync();
  for (int c = t.lane; c < ncon; c += t.T) {
    const float mu = con[kConRec * c + 13];
    const float pn = pf[3 * c], p1 = mu * pf[3 * c + 1], p2 = mu * pf[3 * c + 2];
    out[4 * c] = pn + p1;
    out[4 * c + 1] = pn - p1;
    out[4 * c + 2] = pn + p2;
    out[4 * c + 3] = pn - p2;
  }
  const int r0 = 4 * ncon, rend = max(rb.nru, r0 + rb.nou);
  for (int r = r0 + t.lane; r < rend; r += t.T) {
    const int k = r - r0;
    out[r] = (k < rb.nou && r < nrow) ? pf[3 * ncon + k] : 0.f;
  }
  t.sync();
}

template <class Y>
DEV void rows_t_times(const DevModel& m, float* W0, const Team& t0, const RowBounds& rb, Y y,
                      const float* init, float* out) {
  float* W = W0 + opaque_zero();
  const Team t{t0.lane + opaque_zero(), t0.T, t0.tp};
  const int nv = m.nv;
  const float* J = W + m.o_J;
  if (!m.jframe) {
    for (int i = t.lane; i < nv; i += t.T) {
      float v = init ? init[i] : 0.f;
      for (int r = 0; r < rb.nru; r++) v += y(r) * J[r * nv + i];
      out[i] = v;
    }
    t.sync();
    return;
  }
  const int ncon = ((const int*)(W + m.o_scal))[SC_NCON];
  const float* con = W + m.o_con;
  float* fy = W + m.o_fw;
  for (int c = t.lane; c < ncon; c += t.T) {
    const float mu = con[kConRec * c + 13];
    const float y0 = y(4 * c), y1 = y(4 * c + 1), y2 = y(4 * c + 2), y3 = y(4 * c + 3);
    fy[3 * c] = (y0 + y1) + (y2 + y3);
    fy[3 * c + 1] = mu * (y0 - y1);
    fy[3 * c + 2] = mu * (y2 - y3);
  }
  for (int k = t.lane; k < rb.nou; k += t.T) fy[3 * ncon + k] = y(4 * ncon + k);
  t.sync();
  const int nf = 3 * ncon + rb.nou;
  for (int i = t.lane; i < nv; i += t.T) {
    float v = init ? init[i] : 0.f;
    for (int f = 0; f < nf; f++) v += fy[f] * J[f * nv + i];
    out[i] = v;
  }
  t.sync();
}

// H = M + sum_{rows with e < 0} D J^T J (packed lower), factorised in place as L L^T.
// nru is the padded row bound of pad_rows.
// Right-looking.  With nv <= T four columns share two barriers; otherwise each column
// costs one, used unscaled by its own trailing update and scaled in the next barrier
// interval.  When `y` is given the
// forward solve L y = b (b overwritten) rides along.  Returns false for a non-positive
// pivot.  `w` (nrow words) receives the rows' curvatures: D on the quadratic piece, else 0.
// Jh (default the constraint rows J) and w_given (the caller stored the weights in the
// o_s words) let the elliptic-cone solve pass its own Hessian rows and weights.
DEV bool hessian_cholesky(const DevModel& m, float* W0, const Team& t0, int nru,
                          float* b = nullptr, float* y = nullptr, bool rev = false,
                          bool hgain = false, const float* Jh = nullptr,
                          bool w_given = false, int nou = 0) {
  float* W = W0 + opaque_zero();
  const Team t{t0.lane + opaque_zero(), t0.T, t0.tp};
  const int nv = m.nv;
  const float* M = W + m.o_M;
  float* H = W + m.o_H;
  const float* J = Jh ? Jh : W + m.o_J;
  const float* D = W + m.o_D;
  const float* e = W + m.o_e;
  float* w = W + m.o_s;  // row weights; the line search rewrites this scratch later
  // frame-row contacts: the rows run to 4 ncon + nou (pad_rows), and each contact's four
  // edges J_n +- mu J_tk with weights w0..w3 add J3^T C J3 to H over its frames J3 =
  // (J_n, J_t1, J_t2), C = [[w0+w1+w2+w3, mu (w0-w1), mu (w2-w3)], [., mu^2 (w0+w1), 0],
  // [., 0, mu^2 (w2+w3)]]; o_fw holds C's five entries per contact
  const bool fr = m.jframe && !Jh && nru > 0;
  const int ncon = fr ? ((const int*)(W + m.o_scal))[SC_NCON] : 0;
  const int rend = fr ? max(nru, 4 * ncon + nou) : nru;
  if (w_given) {
  } else if (has_bounds(m)) {
    const float* fl = W + m.o_fl;
    for (int r = t.lane; r < rend; r += t.T) w[r] = row_quad(D[r], fl[r], e[r]) ? D[r] : 0.f;
  } else {
    for (int r = t.lane; r < rend; r += t.T) w[r] = e[r] < 0.f ? D[r] : 0.f;
  }
  const float* con = W + m.o_con;
  float* cf = W + m.o_fw;
  if (fr) {
    t.sync();
    for (int c = t.lane; c < ncon; c += t.T) {
      const float mu = con[kConRec * c + 13];
      const float w0 = w[4 * c], w1 = w[4 * c + 1], w2 = w[4 * c + 2], w3 = w[4 * c + 3];
      cf[5 * c] = (w0 + w1) + (w2 + w3);
      cf[5 * c + 1] = mu * (w0 - w1);
      cf[5 * c + 2] = mu * mu * (w0 + w1);
      cf[5 * c + 3] = mu * (w2 - w3);
      cf[5 * c + 4] = mu * mu * (w2 + w3);
    }
  }
  t.sync();
  if (t.T == 64 && nv <= 32) {
    // One world per wavefront: H = M + sum_r w_r J_r^T J_r as a dense contraction on
    // the matrix cores, two rows per v_mfma_f32_32x32x2_f32 (A = w J, B = J, the
    // 32 x 32 accumulator padded beyond nv).  Operand layout: lane l holds column
    // l % 32 of row r + l / 32.  Accumulator element v of lane l is entry
    // (8 (v / 4) + 4 (l / 32) + v % 4, l % 32).
    const int j = t.lane & 31, kh = t.lane >> 5;
    const int nr = nru;
    f32x16 C;
#pragma unroll
    for (int v = 0; v < 16; v++) {
      const int i = 8 * (v >> 2) + 4 * kh + (v & 3);
      C[v] = (i < nv && j <= i) ? (rev ? M[tri(nv - 1 - j, nv - 1 - i)] : M[tri(i, j)]) : 0.f;
      if (hgain && i < nv && j == i) C[v] += m.dt * m.dof_vgain[rev ? nv - 1 - i : i];
    }
    const int nrf = fr ? rend : nr;
    for (int r = 0; r < nrf; r += 2) {
      const int rr = r + kh;
      float a = 0.f, b = 0.f;
      if (rr < nrf && j < nv) {
        if (!fr) {
          b = J[rr * nv + j];
        } else if (rr < 4 * ncon) {  // edge rr & 3 of contact rr / 4 from its frames
          const int c = rr >> 2, k = rr & 3;
          const float mu = con[kConRec * c + 13];
          b = J[3 * c * nv + j] + ((k & 1) ? -mu : mu) * J[(3 * c + 1 + (k >> 1)) * nv + j];
        } else {
          b = J[(rr - ncon) * nv + j];
        }
        a = w[rr] * b;
      }
      C = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, C, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 16; v++) {
      const int i = 8 * (v >> 2) + 4 * kh + (v & 3);
      if (i < nv && j <= i) H[tri(i, j)] = C[v];
    }
  } else {
    for (int k = t.lane; k < m.ntri; k += t.T) {
      int i, j;
      t.unrank(k, i, j);
      float v = rev ? M[tri(nv - 1 - j, nv - 1 - i)] : M[k];
      if (hgain && i == j) v += m.dt * m.dof_vgain[rev ? nv - 1 - i : i];
      if (!fr) {
        for (int r = 0; r < nru; r++) v += w[r] * J[r * nv + i] * J[r * nv + j];
      } else {
        for (int c = 0; c < ncon; c++) {
          const float* q = cf + 5 * c;
          const float* Jn = J + 3 * c * nv;
          const float ni = Jn[i], nj = Jn[j], ai = Jn[nv + i], aj = Jn[nv + j];
          const float bi = Jn[2 * nv + i], bj = Jn[2 * nv + j];
          v += q[0] * ni * nj + q[2] * ai * aj + q[4] * bi * bj + q[1] * (ni * aj + ai * nj) +
               q[3] * (ni * bj + bi * nj);
        }
        const float* Jo = J + 3 * ncon * nv;
        const float* wo = w + 4 * ncon;
        for (int k2 = 0; k2 < nou; k2++) v += wo[k2] * Jo[k2 * nv + i] * Jo[k2 * nv + j];
      }
      H[k] = v;
    }
  }
  t.sync();
  bool ok = true;
  if (nv <= t.T) {
    // Blocks of four columns, two barriers each; lane r owns row r.
    //  A: every lane eliminates the 4 x 4 diagonal block in registers (the same values
    //     in all lanes; lane a stores row a of the factor after the barrier).  Lane i
    //     of a row below the block applies the block's columns, in order, to its four
    //     entries and stores them as L.  The forward solve takes the same columns.
    //  B: every trailing entry takes the block's four rank-1 updates in one pass.
    const int i = t.lane;
    for (int j = 0; j < nv; j += 4) {
      const int bw = min(4, nv - j);
      float P[4][4], in[4];
#pragma unroll
      for (int a = 0; a < 4; a++)
#pragma unroll
        for (int c = 0; c <= a; c++) P[a][c] = (a < bw) ? H[tri(j + a, j + c)] : 0.f;
#pragma unroll
      for (int c = 0; c < 4; c++) {
        const float pc = c < bw ? P[c][c] : 1.f;
        ok = ok && (pc > 0.f);
        in[c] = __builtin_amdgcn_rsqf(fmaxf(pc, 1e-30f));  // v_rsq: one instruction
        const float rc = in[c] * in[c];
#pragma unroll
        for (int a = c + 1; a < 4; a++)
#pragma unroll
          for (int a2 = c + 1; a2 <= a; a2++) P[a][a2] -= P[a][c] * P[a2][c] * rc;
      }
      float dr[4];  // row i of the block's factor, for lane i < bw (sqrt(p) = p / sqrt(p))
#pragma unroll
      for (int c = 0; c < 4; c++) {
        float v = 0.f;
#pragma unroll
        for (int a = c; a < 4; a++) v = (i == a) ? P[a][c] * in[c] : v;
        dr[c] = v;
      }
      const bool prow = i >= j + bw && i < nv;
      float u[4] = {0.f, 0.f, 0.f, 0.f};  // this row's L entries of the block
      if (prow) {
        const int ri = tri(i, j);
#pragma unroll
        for (int c = 0; c < 4; c++) {
          float v = c < bw ? H[ri + c] : 0.f;
#pragma unroll
          for (int c2 = 0; c2 < c; c2++) v -= u[c2] * P[c][c2] * in[c2];
          u[c] = v * in[c];
          if (c < bw) H[ri + c] = u[c];
        }
      }
      if (y) {  // L y = b for the block's columns; rows below take their updates
        float yv[4];
#pragma unroll
        for (int c = 0; c < 4; c++) {
          float v = c < bw ? b[j + c] : 0.f;
#pragma unroll
          for (int c2 = 0; c2 < c; c2++) v -= P[c][c2] * in[c2] * yv[c2];
          yv[c] = v * in[c];
        }
        if (prow) {
          float v = b[i];
#pragma unroll
          for (int c = 0; c < 4; c++) v -= u[c] * yv[c];
          b[i] = v;
        }
        if (t.lane == 0) {
#pragma unroll
          for (int c = 0; c < 4; c++)
            if (c < bw) y[j + c] = yv[c];
        }
      }
      t.sync();
      if (i < bw) {  // every lane has read the block: store row j + i of its factor
#pragma unroll
        for (int c = 0; c < 4; c++)
          if (c <= i) H[tri(j + i, j + c)] = dr[c];
      }
      const int c0 = j + bw, n2 = nv - c0, npr = n2 * (n2 + 1) / 2;
      for (int p = t.lane; p < npr; p += t.T) {
        int bi, ai;
        t.unrank(p, bi, ai);
        const int ri = tri(c0 + bi, 0), rk = tri(c0 + ai, 0);
        float v = H[ri + c0 + ai];
#pragma unroll
        for (int c = 0; c < 4; c++)
          if (c < bw) v -= H[ri + j + c] * H[rk + j + c];
        H[ri + c0 + ai] = v;
      }
      t.sync();
    }
    return ok;
  }
  float dlast = 1.f, invlast = 1.f;  // column j - 1, scaled during column j
  for (int j = 0; j <= nv; j++) {
    float dj = 1.f, inv = 1.f;
    if (j < nv) {
      const float piv = H[tri(j, j)];
      ok = ok && (piv > 0.f);
      dj = sqrtf(fmaxf(piv, 1e-30f));
      inv = 1.f / dj;
      const float inv2 = inv * inv;
      const int n2 = nv - j - 1;
      const int npr = n2 * (n2 + 1) / 2;
      for (int p = t.lane; p < npr; p += t.T) {
        int bi, ai;
        t.unrank(p, bi, ai);
        const int i = j + 1 + bi, k = j + 1 + ai;
        H[tri(i, k)] -= H[tri(i, j)] * H[tri(k, j)] * inv2;
      }
      if (y) {
        const float yj = b[j] * inv;
        for (int i = j + 1 + t.lane; i < nv; i += t.T) b[i] -= H[tri(i, j)] * inv * yj;
        if (t.lane == 0) y[j] = yj;
      }
    }
    if (j >= 1) {
      const int c = j - 1;
      for (int i = c + 1 + t.lane; i < nv; i += t.T) H[tri(i, c)] *= invlast;
      if (t.lane == 0) H[tri(c, c)] = dlast;
    }
    dlast = dj;
    invlast = inv;
    t.sync();
  }
  return ok;
}
// Triangular solves with the factor L in H (packed lower), lane i holding entry i of a
// team of TT lanes (nv <= TT); each finished entry is broadcast from its lane.  The team
// size is a template argument so that the loops carry no test of it.
template <int TT>
DEV float team_bcast(float v, int j, int base) {  // v of the team's lane j (j uniform)
  const int iv = __float_as_int(v);
  int r = __builtin_amdgcn_readlane(iv, j);
  if constexpr (TT == 32) {
    const int r1 = __builtin_amdgcn_readlane(iv, j + 32);
    r = base ? r1 : r;
  } else if constexpr (TT == 16) {
    const int r1 = __builtin_amdgcn_readlane(iv, j + 16);
    const int r2 = __builtin_amdgcn_readlane(iv, j + 32);
    const int r3 = __builtin_amdgcn_readlane(iv, j + 48);
    r = base == 0 ? r : base == 16 ? r1 : base == 32 ? r2 : r3;
  }
  return __int_as_float(r);
}
// acc: this lane's right-hand side entry; fwd: L y = acc first; then L^T x = y.  Returns
// x_i scaled by the pivot (the caller multiplies by rinv)
template <int TT>
DEV float tri_solves(const float* H0, int nv, int i0, float acc, float rinv, bool fwd) {
  const float* H = H0 + opaque_zero();  // (a context of its own: see opaque_zero)
  const int i = i0 + opaque_zero();
  const int base = (int)(threadIdx.x & 63) - i;  // the team's first lane in the wave
  // (the row tests select the factor entry or 0 from an address valid in every lane,
  // rather than branching around the update)
  if (fwd) {
    const int last = i < nv ? i : 0;  // the row takes columns j < last
    const float* Hi = H + tri(last, 0);  // row i of the factor (row 0 past nv)
    for (int j = 0; j < nv - 1; j++) {
      const float yj = team_bcast<TT>(acc * rinv, j, base);
      acc -= (j < last ? Hi[j] : 0.f) * yj;
    }
    acc *= rinv;
  }
  int at = tri(nv - 1, i);  // tri(j, i), one column down per step
  for (int j = nv - 1; j > 0; j--) {
    const float xj = team_bcast<TT>(acc * rinv, j, base);
    acc -= (i < j ? H[i < j ? at : 0] : 0.f) * xj;
    at -= j;
  }
  return acc;
}
DEV float tri_solves(const Team& t, const float* H, int nv, float acc, float rinv, bool fwd) {
  if (t.T == 32) return tri_solves<32>(H, nv, t.lane, acc, rinv, fwd);
  if (t.T == 64) return tri_solves<64>(H, nv, t.lane, acc, rinv, fwd);
  return tri_solves<16>(H, nv, t.lane, acc, rinv, fwd);
}
// x = sgn * (L L^T)^{-1} rhs with the factor in H (rhs and x may alias)
DEV void cholesky_solve(const DevModel& m, float* W, const Team& t, const float* rhs, float* x,
                        float sgn) {
  const float* H = W + m.o_H;
  const int nv = m.nv;
  if (nv <= t.T) {
    const int i = t.lane;
    const float rinv = i < nv ? 1.f / H[tri(i, i)] : 0.f;
    const float acc = tri_solves(t, H, nv, i < nv ? sgn * rhs[i] : 0.f, rinv, true);
    if (i < nv) x[i] = acc * rinv;
    t.sync();
    return;
  }
  if (t.lane == 0) {
    for (int i = 0; i < nv; i++) {
      float v = sgn * rhs[i];
      for (int k = 0; k < i; k++) v -= H[tri(i, k)] * x[k];
      x[i] = v / H[tri(i, i)];
    }
    for (int i = nv - 1; i >= 0; i--) {
      float v = x[i];
      for (int k = i + 1; k < nv; k++) v -= H[tri(k, i)] * x[k];
      x[i] = v / H[tri(i, i)];
    }
  }
  t.sync();
}
// back substitution L^T x = y (x and y may alias)
DEV void cholesky_back(const DevModel& m, float* W, const Team& t, const float* y, float* x) {
  const float* H = W + m.o_H;
  const int nv = m.nv;
  if (nv <= t.T) {
    const int i = t.lane;
    const float rinv = i < nv ? 1.f / H[tri(i, i)] : 0.f;
    const float acc = tri_solves(t, H, nv, i < nv ? y[i] : 0.f, rinv, false);
    if (i < nv) x[i] = acc * rinv;
    t.sync();
    return;
  }
  if (t.lane == 0) {
    for (int i = nv - 1; i >= 0; i--) {
      float v = y[i];
      for (int k = i + 1; k < nv; k++) v -= H[tri(k, i)] * x[k];
      x[i] = v / H[tri(i, i)];
    }
  }
  t.sync();
}

// F(a) = 1/2 (a - a0)^T M (a - a0) + sum_r s_r(J_r a - aref_r), with the row pieces of
// row_cost (1/2 D min(0, e)^2 for one-sided rows, the Huber term for friction loss).
// Start from the cheaper of the warm start and a0; each iteration: gradient and
// Hessian on the active set, dense Cholesky of H, Newton direction, exact line
// search (phi' evaluated at every breakpoint in parallel), update.  Stops early when
// the Newton direction is no longer a descent direction (converged to precision) or,
// with gtol > 0, when max |g| <= gtol * max(1, max |qfrc_smooth|).  FR: the model has
// friction-loss rows (two breakpoints each, Huber pieces) or two-sided equality rows
// (quadratic everywhere, no breakpoint); without them every row is one-sided and the
// loops keep their shorter form.
// Newton stops before its iteration count when the last step stayed on one piece of
// every row's cost and its refinement correction was below this fraction of max(1,
// max |a|): the iterate is then the minimiser up to FP32 rounding.
constexpr float kNewtonExitTol = 1e-6f;
template <bool FR>
DEV void newton_impl(const DevModel& m, float* W, const Team& t, int& status, int iters,
                     float gtol) {
  const float* fl = W + m.o_fl;  // per-row friction bound (FR only)
  const int* scal = (const int*)(W + m.o_scal);
  const int nv = m.nv, nrow = scal[SC_NROW];
  const float* M = W + m.o_M;
  const float* aref = W + m.o_aref;
  const float* D = W + m.o_D;
  float* e = W + m.o_e;     // J a - aref
  float* s = W + m.o_s;     // J delta
  const float* a0 = W + m.o_a0;
  float* a = W + m.o_qacc;  // iterate (warm start on entry)
  float* Mr = W + m.o_Mr;   // M (a - a0)
  float* g = W + m.o_g;
  float* d = W + m.o_d;
  float* Md = W + m.o_Md;
  float* tmp = W + m.o_tmp;
  if (nrow == 0) {
    for (int i = t.lane; i < nv; i += t.T) a[i] = a0[i];
    t.sync();
    return;
  }
  const RowBounds rb = pad_rows(m, W, t, nrow);
  const int nru = rb.nru;
  // rows the row products define (frame-row contacts: to 4 ncon + nou, see pad_rows)
  const int rend = m.jframe ? max(nru, 4 * scal[SC_NCON] + rb.nou) : nru;
  // ---- start point: cost of the warm start vs cost of a0
  for (int i = t.lane; i < nv; i += t.T) tmp[i] = a[i] - a0[i];
  t.sync();
  float qw = 0.f;
  for (int i = t.lane; i < nv; i += t.T) {
    float v = sym_row_dot(M, i, tmp, nv);
    Mr[i] = v;
    qw += 0.5f * tmp[i] * v;
  }
  rows_times(m, W, t, nrow, rb, a, e);
  rows_times(m, W, t, nrow, rb, a0, s);
  float cw = 0.f, c0 = 0.f;
  for (int r = t.lane; r < nrow; r += t.T) {
    const float ew = e[r] - aref[r], e0 = s[r] - aref[r];
    if (FR) {
      cw += row_cost(D[r], fl[r], ew);
      c0 += row_cost(D[r], fl[r], e0);
    } else {
      if (ew < 0.f) cw += 0.5f * D[r] * ew * ew;
      if (e0 < 0.f) c0 += 0.5f * D[r] * e0 * e0;
    }
    e[r] = ew;
    s[r] = e0;  // stash
  }
  cw = t.sum(cw + qw);
  c0 = t.sum(c0);
  t.sync();
  if (!(cw <= c0)) {
    for (int i = t.lane; i < nv; i += t.T) { a[i] = a0[i]; Mr[i] = 0.f; }
    for (int r = t.lane; r < nrow; r += t.T) e[r] = s[r];
    t.sync();
  }
  float gstop = 0.f;
  if (gtol > 0.f) {
    const float* frc = W + m.o_frc;
    float fm = 1.f;
    for (int i = t.lane; i < nv; i += t.T) fm = fmaxf(fm, fabsf(frc[i]));
    gstop = gtol * t.max(fm);
  }
  bool kept = false;  // o_H holds the factor of the Hessian at the current pieces
  for (int it = 0; it < iters; it++) {
    // ---- gradient g = M (a - a0) + sum_active D e J
    rows_t_times(m, W, t, rb, [&](int r) {
      const float er = e[r];
      return FR ? row_slope(D[r], fl[r], er) : (er < 0.f ? D[r] * er : 0.f);
    }, Mr, g);
    float gmax = 0.f;
    for (int i = t.lane; i < nv; i += t.T) gmax = fmaxf(gmax, fabsf(g[i]));
    if (gtol > 0.f && t.max(gmax) <= gstop) break;  // converged to FP32 precision
    // ---- delta = -H^-1 g.  H depends on the iterate only through the rows' pieces, so
    // after a step on which no row changed piece the factor left in o_H is this
    // iteration's: solve with it.  Otherwise assemble and factor, the forward solve
    // fused into the factorisation, then the back substitution.
    if (kept) {
      cholesky_solve(m, W, t, g, d, -1.f);
    } else {
      for (int i = t.lane; i < nv; i += t.T) d[i] = -g[i];
      if (!hessian_cholesky(m, W, t, nru, d, tmp, false, false, nullptr, false, rb.nou)) {
        status |= 4;
        break;
      }
      cholesky_back(m, W, t, tmp, d);
    }
    // ---- one step of iterative refinement: the FP32 factor of H carries a relative
    // error near cond(H) eps into d, and the fixed iteration count leaves the iterate
    // mid-path, where such errors compound.  The residual r = g + H d, with H applied
    // unassembled (M d + sum over rows on their quadratic piece of D J^T (J d)), is
    // accurate to the gradient's own rounding; d -= H^-1 r with the same factor.
    rows_times(m, W, t, nrow, rb, d, s);
    for (int r = t.lane; r < rend; r += t.T) {
      const bool q = FR ? row_quad(D[r], fl[r], e[r]) : e[r] < 0.f;
      s[r] = q ? D[r] * s[r] : 0.f;
    }
    for (int i = t.lane; i < nv; i += t.T) {
      float v = sym_row_dot(M, i, d, nv, g[i]);
      tmp[i] = v;
    }
    t.sync();
    rows_t_times(m, W, t, rb, [&](int r) { return s[r]; }, tmp, tmp);
    cholesky_solve(m, W, t, tmp, tmp, 1.f);
    float cmax = 0.f;  // size of the correction: the unrefined direction's error
    for (int i = t.lane; i < nv; i += t.T) {
      d[i] -= tmp[i];
      cmax = fmaxf(cmax, fabsf(tmp[i]));
    }
    t.sync();
    // ---- line search quantities
    float gd = 0.f, dMd = 0.f, dMr = 0.f;
    for (int i = t.lane; i < nv; i += t.T) {
      float v = sym_row_dot(M, i, d, nv);
      Md[i] = v;
      gd += g[i] * d[i];
      dMd += d[i] * v;
      dMr += d[i] * Mr[i];
    }
    rows_times(m, W, t, nrow, rb, d, s);
    gd = t.sum(gd);
    dMd = t.sum(dMd);
    dMr = t.sum(dMr);
    t.sync();
    if (!(gd < 0.f)) break;  // gradient already zero to working precision
    // phi'(al) = dMr + al dMd + sum_r D_r s_r min(0, e_r + al s_r), nondecreasing.
    // Evaluate it at every positive breakpoint; the root lies between the largest
    // breakpoint with phi' <= 0 and the smallest with phi' > 0, where phi' is linear.
    // Breakpoints: a one-sided row's e crosses 0; a friction row's D e crosses +F
    // (candidate r) and -F (candidate nrow + its index among the friction rows); a
    // two-sided row (bound +inf) has none.
    float lo = 0.f, hi = INFINITY;
    const int nbp = FR ? nrow + m.nfric : nrow;
    const int nfr0 = nrow - m.nfric - m.neqrow;  // first friction-loss row
    for (int c = t.lane; c < nbp; c += t.T) {
      const int r = c < nrow ? c : nfr0 + (c - nrow);
      const float sr = s[r];
      if (sr == 0.f) continue;
      float at = 0.f;
      if (FR && fl[r] > 0.f) {
        if (fl[r] == INFINITY) continue;
        at = (c < nrow ? fl[r] : -fl[r]) / D[r];
      }
      const float br = (at - e[r]) / sr;
      if (!(br > 0.f)) continue;
      float dp = dMr + br * dMd;
      for (int q = 0; q < nru; q++) {
        const float sq = s[q], v = e[q] + br * sq;
        dp += FR ? sq * row_slope(D[q], fl[q], v) : (v < 0.f ? D[q] * sq : 0.f) * v;
      }
      if (dp <= 0.f) lo = fmaxf(lo, br);
      else hi = fminf(hi, br);
    }
    lo = t.max(lo);
    hi = t.min(hi);
    const float probe = (hi < INFINITY) ? 0.5f * (lo + hi) : lo + 1.f;
    float Ac = 0.f, Bc = 0.f;
    for (int r = t.lane; r < nrow; r += t.T) {
      const float ep = e[r] + probe * s[r];
      if (FR ? row_quad(D[r], fl[r], ep) : ep < 0.f) {
        Ac += D[r] * s[r] * e[r];
        Bc += D[r] * s[r] * s[r];
      } else if (FR) {
        Ac += s[r] * row_slope(D[r], fl[r], ep);  // +-F on a friction row's linear piece
      }
    }
    Ac = t.sum(Ac) + dMr;
    Bc = t.sum(Bc) + dMd;
    float al = -Ac / Bc;
    al = fminf(fmaxf(al, lo), hi);
    // ---- update
    float amax = 1.f;
    for (int i = t.lane; i < nv; i += t.T) {
      a[i] += al * d[i];
      Mr[i] += al * Md[i];
      amax = fmaxf(amax, fabsf(a[i]));
    }
    int moved = 0;  // some row changed piece between 0 and al
    for (int r = t.lane; r < nrow; r += t.T) {
      const float e1 = e[r] + al * s[r];
      moved |= FR ? (row_piece(D[r], fl[r], e[r]) != row_piece(D[r], fl[r], e1))
                  : ((e[r] < 0.f) != (e1 < 0.f));
      e[r] = e1;
    }
    // Exact optimum: when no row changed piece, the step stayed on the piece the Hessian
    // was built for, where F is that quadratic; a + al d is its minimiser (al = 1 up to
    // rounding) and the gradient there vanishes, so further iterations only reduce the
    // FP32 error of this step, which is about cond(H) eps |d|.  Stop once that error is
    // known small: the refinement's correction, the unrefined direction's error, is
    // below kNewtonExitTol max(1, max |a|).
    moved = t.ior(moved);
    const float cm = t.max(cmax), am = t.max(amax);
    t.sync();
    if (!moved && cm <= kNewtonExitTol * am) break;
    kept = !moved;
  }
}
// ------------------------------------------------- A9 with elliptic friction cones
// One contact's cone at e (its nd rows' J a - aref): the cost, the rows' slopes ds/de
// (minus the row forces) and its zone, in the coordinates x_j = e_j r_j (r_j = mu_j / mu:
// 1 on the normal and the tangents) where the cone |g_t| <= mu g_n is round and the rows
// share D = D_n (the convex soft-constraint cost of the force set, maximised at the
// projection of -D x onto the cone):
//   separated (0)  x_0 >= mu |x_t|:        s = 0;
//   sliding   (1)  otherwise:              s = c psi^2 / 2, psi = mu |x_t| - x_0 > 0,
//                                          c = D / (1 + mu^2);
//   sticking  (2)  mu x_0 + |x_t| <= 0:    s = D |x|^2 / 2.
// With V (nd x nd) and w (nd) given, also the Hessian as weighted virtual rows,
// d2s/de2 = sum_k w_k V_k V_k^T: the rows themselves when sticking (w_k = D r_k^2); when
// sliding the direction a = (-1, mu t), t = x_t / |x_t|, with weight c, and a
// Householder basis of the friction coordinates orthogonal to t with weight
// c psi mu / |x_t|, both mapped back by r_j.
DEV int cone_eval(float mu, float D, const float* ratio, int nd, const float* e,
                  float& cost, float* slope, float* w = nullptr, float* V = nullptr) {
  float x[6], T2 = 0.f;
  x[0] = e[0];
  for (int j = 1; j < nd; j++) {
    x[j] = e[j] * ratio[j];
    T2 += x[j] * x[j];
  }
  const float Tn = sqrtf(T2);
  if (w)
    for (int k = 0; k < nd; k++) {
      w[k] = 0.f;
      for (int j = 0; j < nd; j++) V[k * nd + j] = 0.f;
    }
  if (!(x[0] < mu * Tn)) {
    cost = 0.f;
    for (int j = 0; j < nd; j++) slope[j] = 0.f;
    return 0;
  }
  if (mu * x[0] + Tn <= 0.f) {
    cost = 0.5f * D * (x[0] * x[0] + T2);
    for (int j = 0; j < nd; j++) slope[j] = D * x[j] * ratio[j];
    if (w)
      for (int k = 0; k < nd; k++) {
        w[k] = D * ratio[k] * ratio[k];
        V[k * nd + k] = 1.f;
      }
    return 2;
  }
  const float psi = mu * Tn - x[0], c = D / (1.f + mu * mu), inv = 1.f / Tn;
  cost = 0.5f * c * psi * psi;
  slope[0] = -c * psi;
  for (int j = 1; j < nd; j++) slope[j] = c * psi * mu * x[j] * inv * ratio[j];
  if (w) {
    w[0] = c;
    V[0] = -1.f;
    for (int j = 1; j < nd; j++) V[j] = mu * x[j] * inv * ratio[j];
    // the reflection I - beta u u^T (u = t + sign(t_1) e_1) takes t to -+e_1; its
    // other columns span the friction coordinates orthogonal to t
    const int mf = nd - 1;
    float u[5];
    for (int j = 0; j < mf; j++) u[j] = x[1 + j] * inv;
    u[0] += u[0] >= 0.f ? 1.f : -1.f;
    float uu = 0.f;
    for (int j = 0; j < mf; j++) uu += u[j] * u[j];
    const float beta = 2.f / uu, w2 = c * psi * mu * inv;
    for (int k = 1; k < mf; k++) {
      w[k] = w2;
      for (int j = 0; j < mf; j++)
        V[k * nd + 1 + j] = ((j == k ? 1.f : 0.f) - beta * u[j] * u[k]) * ratio[1 + j];
    }
  }
  return 1;
}

// contact c's rows (first, count), friction coefficient and per-row ratios r_j
DEV int cone_of(const DevModel& m, const float* con, int c, int& first, float& mu,
                float* ratio) {
  const float* r = con + kConRec * c;
  const int slot = __float_as_int(r[17]);
  first = m.con_nr ? m.con_nr * c : slot >> 8;
  const int nd = m.con_nr ? m.con_nr : (slot >> 4) & 15;
  mu = r[13];
  const int p = __float_as_int(r[16]);
  for (int j = 0; j < nd; j++)
    ratio[j] = j < 3 ? 1.f : (j == 3 ? m.pair_mu_t[p] : m.pair_mu_r[p]) / mu;
  return nd;
}

// The Newton solve of newton_impl for a model with elliptic cones.  Contact rows are
// handled per contact (a cone block, or one one-sided row for a frictionless contact),
// the others per row.  Each iteration evaluates every row's slope ds/de (sl) and the
// Hessian's rows (Jv: a cone's virtual rows, the other rows themselves, with their
// weights in the o_s words), assembles and factors H = M + sum_r w_r Jv_r^T Jv_r, takes
// the refined direction, and minimises phi(al) = F(a + al d) exactly: phi' is continuous
// and nondecreasing but not piecewise linear, so its root is bracketed by doubling from
// al = 1 and found by Newton steps on phi' kept inside the bracket (midpoint otherwise).
// On exit sl holds the final slopes (the rows' forces are -sl).
template <bool FR>
DEV void newton_cone(const DevModel& m, float* W, const Team& t, int& status, int iters,
                     float gtol) {
  const float* fl = W + m.o_fl;
  const int* scal = (const int*)(W + m.o_scal);
  const int nv = m.nv, nrow = scal[SC_NROW], nrc = scal[SC_NRC], ncon = scal[SC_NCON];
  const float* con = W + m.o_con;
  const float* M = W + m.o_M;
  const float* J = W + m.o_J;
  const float* aref = W + m.o_aref;
  const float* D = W + m.o_D;
  float* e = W + m.o_e;
  float* s = W + m.o_s;
  const float* a0 = W + m.o_a0;
  float* a = W + m.o_qacc;
  float* Mr = W + m.o_Mr;
  float* g = W + m.o_g;
  float* d = W + m.o_d;
  float* Md = W + m.o_Md;
  float* tmp = W + m.o_tmp;
  float* Jv = W + m.o_Jv;
  float* sl = W + m.o_sl;
  float* cv = W + m.o_cv;
  const int cw = m.conrows * m.conrows;
  if (nrow == 0) {
    for (int i = t.lane; i < nv; i += t.T) a[i] = a0[i];
    t.sync();
    return;
  }
  const int nru = pad_rows(m, W, t, nrow).nru;
  auto row_s = [&](int r, float ev) {  // a non-cone row's slope
    return FR ? row_slope(D[r], fl[r], ev) : fminf(D[r] * ev, 0.f);
  };
  auto row_q = [&](int r, float ev) {
    return FR ? row_quad(D[r], fl[r], ev) : ev < 0.f;
  };
  // cost of the rows at e + al s (per lane; sum over the team afterwards)
  auto rows_cost = [&](const float* ee, const float* ss, float al) {
    float cst = 0.f;
    for (int c = t.lane; c < ncon; c += t.T) {
      int first;
      float mu, ratio[6], ev[6], sv[6], cc;
      const int nd = cone_of(m, con, c, first, mu, ratio);
      for (int j = 0; j < nd; j++) ev[j] = ee[first + j] + (ss ? al * ss[first + j] : 0.f);
      if (nd == 1) {
        cst += ev[0] < 0.f ? 0.5f * D[first] * ev[0] * ev[0] : 0.f;
      } else {
        cone_eval(mu, D[first], ratio, nd, ev, cc, sv);
        cst += cc;
      }
    }
    for (int r = nrc + t.lane; r < nrow; r += t.T) {
      const float ev = ee[r] + (ss ? al * ss[r] : 0.f);
      cst += FR ? row_cost(D[r], fl[r], ev) : (ev < 0.f ? 0.5f * D[r] * ev * ev : 0.f);
    }
    return cst;
  };
  // ---- start point: cost of the warm start vs cost of a0
  for (int i = t.lane; i < nv; i += t.T) tmp[i] = a[i] - a0[i];
  t.sync();
  float qw = 0.f;
  for (int i = t.lane; i < nv; i += t.T) {
    float v = sym_row_dot(M, i, tmp, nv);
    Mr[i] = v;
    qw += 0.5f * tmp[i] * v;
  }
  for (int r = t.lane; r < nrow; r += t.T) {
    float jw = 0.f, j0 = 0.f;
    for (int i = 0; i < nv; i++) { jw += J[r * nv + i] * a[i]; j0 += J[r * nv + i] * a0[i]; }
    e[r] = jw - aref[r];
    s[r] = j0 - aref[r];  // stash
  }
  t.sync();
  const float cw0 = t.sum(rows_cost(e, nullptr, 0.f) + qw);
  const float c00 = t.sum(rows_cost(s, nullptr, 0.f));
  t.sync();
  if (!(cw0 <= c00)) {
    for (int i = t.lane; i < nv; i += t.T) { a[i] = a0[i]; Mr[i] = 0.f; }
    for (int r = t.lane; r < nrow; r += t.T) e[r] = s[r];
    t.sync();
  }
  float gstop = 0.f;
  if (gtol > 0.f) {
    const float* frc = W + m.o_frc;
    float fm = 1.f;
    for (int i = t.lane; i < nv; i += t.T) fm = fmaxf(fm, fabsf(frc[i]));
    gstop = gtol * t.max(fm);
  }
  bool kept = false;  // o_H holds the factor of the Hessian at the current zones
  for (int it = 0; it < iters; it++) {
    // ---- slopes, Hessian weights and the cones' virtual-row maps (cone_eval's, in
    // registers and the map's LDS words): sticking, the rows themselves with weights
    // D r_j^2; sliding, (-1, mu t) with D / (1 + mu^2) and the columns of the reflection
    // I - beta u u^T (u = t + sign(t_1) e_1) orthogonal to t with c psi mu / T;
    // separated, nothing
    for (int c = t.lane; c < ncon; c += t.T) {
      const float* rc = con + kConRec * c;
      const int slot = __float_as_int(rc[17]);
      const int first = m.con_nr ? m.con_nr * c : slot >> 8;
      const int nd = m.con_nr ? m.con_nr : (slot >> 4) & 15;
      const float Dn = D[first], x0 = e[first];
      if (nd == 1) {
        sl[first] = fminf(Dn * x0, 0.f);
        s[first] = x0 < 0.f ? Dn : 0.f;
        continue;
      }
      const float mu = rc[13];
      float rt = 1.f, rr = 1.f;
      if (nd > 3) {
        const int p = __float_as_int(rc[16]);
        rt = m.pair_mu_t[p] / mu;
        rr = m.pair_mu_r[p] / mu;
      }
      auto ratio = [&](int q) { return q < 3 ? 1.f : (q == 3 ? rt : rr); };
      float* V = cv + c * cw;
      for (int k = 0; k < nd * nd; k++) V[k] = 0.f;
      float xx = 0.f;
      for (int q = 1; q < nd; q++) {
        const float xq = e[first + q] * ratio(q);
        xx += xq * xq;
      }
      const float Tn = sqrtf(xx);
      for (int q = 0; q < nd; q++) { sl[first + q] = 0.f; s[first + q] = 0.f; }
      if (!(x0 < mu * Tn)) continue;  // separated
      if (mu * x0 + Tn <= 0.f) {       // sticking
        for (int q = 0; q < nd; q++) {
          const float rq = ratio(q);
          sl[first + q] = Dn * e[first + q] * rq * rq;
          s[first + q] = Dn * rq * rq;
          V[q * nd + q] = 1.f;
        }
        continue;
      }
      const float inv = 1.f / Tn, psi = mu * Tn - x0, cc = Dn / (1.f + mu * mu);
      sl[first] = -cc * psi;
      s[first] = cc;
      V[0] = -1.f;
      const float u0 = e[first + 1] * inv, sg = u0 >= 0.f ? 1.f : -1.f;
      float uu = 0.f;
      for (int q = 1; q < nd; q++) {
        const float rq = ratio(q), xq = e[first + q] * rq;
        sl[first + q] = cc * psi * mu * xq * inv * rq;
        V[q] = mu * xq * inv * rq;
        const float uq = xq * inv + (q == 1 ? sg : 0.f);
        uu += uq * uq;
      }
      const float beta = 2.f / uu, w2 = cc * psi * mu * inv;
      const int mf = nd - 1;
      for (int k = 1; k < mf; k++) {
        s[first + k] = w2;
        const float uk = e[first + 1 + k] * ratio(1 + k) * inv;
        for (int q = 0; q < mf; q++) {
          const float uq = e[first + 1 + q] * ratio(1 + q) * inv + (q == 0 ? sg : 0.f);
          V[k * nd + 1 + q] = ((q == k ? 1.f : 0.f) - beta * uq * uk) * ratio(1 + q);
        }
      }
    }
    for (int r = nrc + t.lane; r < nru; r += t.T) {
      sl[r] = row_s(r, e[r]);
      s[r] = row_q(r, e[r]) ? D[r] : 0.f;
    }
    t.sync();
    // Hessian rows: a cone's k-th virtual row sum_j V[k][j] J_j, the others copied
    for (int idx = t.lane; idx < nru * nv; idx += t.T) {
      const int r = idx / nv, i = idx - r * nv;
      float v = J[idx];
      if (r < nrc) {
        int c = m.con_nr ? r / m.con_nr : 0;
        if (!m.con_nr)
          while (c + 1 < ncon && (__float_as_int(con[kConRec * (c + 1) + 17]) >> 8) <= r) c++;
        const int slot = __float_as_int(con[kConRec * c + 17]);
        const int first = m.con_nr ? m.con_nr * c : slot >> 8;
        const int nd = m.con_nr ? m.con_nr : (slot >> 4) & 15;
        if (nd > 1) {
          const float* V = cv + c * cw + (r - first) * nd;
          v = 0.f;
          for (int j = 0; j < nd; j++) v += V[j] * J[(first + j) * nv + i];
        }
      }
      Jv[idx] = v;
    }
    // ---- gradient g = M (a - a0) + sum_r sl_r J_r
    float gmax = 0.f;
    t.sync();
    for (int i = t.lane; i < nv; i += t.T) {
      float v = Mr[i];
      for (int r = 0; r < nru; r++) v += sl[r] * J[r * nv + i];
      g[i] = v;
      gmax = fmaxf(gmax, fabsf(v));
    }
    if (gtol > 0.f && t.max(gmax) <= gstop) break;
    // ---- delta = -H^-1 g, then one step of iterative refinement (as in newton_impl).
    // With every zone unchanged by the last step and no cone sliding (whose curvature
    // moves with x), the Hessian is the last one and its factor is still in o_H.
    if (kept) {
      cholesky_solve(m, W, t, g, d, -1.f);
    } else {
      for (int i = t.lane; i < nv; i += t.T) d[i] = -g[i];
      if (!hessian_cholesky(m, W, t, nru, d, tmp, false, false, Jv, true)) { status |= 4; break; }
      cholesky_back(m, W, t, tmp, d);
    }
    for (int r = t.lane; r < nru; r += t.T) {
      float v = 0.f;
      for (int i = 0; i < nv; i++) v += Jv[r * nv + i] * d[i];
      s[r] *= v;  // weight times the virtual row's product
    }
    t.sync();
    for (int i = t.lane; i < nv; i += t.T) {
      float v = sym_row_dot(M, i, d, nv, g[i]);
      for (int r = 0; r < nru; r++) v += s[r] * Jv[r * nv + i];
      tmp[i] = v;
    }
    t.sync();
    cholesky_solve(m, W, t, tmp, tmp, 1.f);
    float cmax = 0.f;  // size of the correction: the unrefined direction's error
    for (int i = t.lane; i < nv; i += t.T) {
      d[i] -= tmp[i];
      cmax = fmaxf(cmax, fabsf(tmp[i]));
    }
    t.sync();
    // ---- line search quantities
    float gd = 0.f, dMd = 0.f, dMr = 0.f;
    for (int i = t.lane; i < nv; i += t.T) {
      float v = sym_row_dot(M, i, d, nv);
      Md[i] = v;
      gd += g[i] * d[i];
      dMd += d[i] * v;
      dMr += d[i] * Mr[i];
    }
    for (int r = t.lane; r < nru; r += t.T) {
      float v = 0.f;
      for (int i = 0; i < nv; i++) v += J[r * nv + i] * d[i];
      s[r] = v;
    }
    gd = t.sum(gd);
    dMd = t.sum(dMd);
    dMr = t.sum(dMr);
    t.sync();
    if (!(gd < 0.f)) break;
    // phi'(al) and phi''(al), summed over the team
    auto dphi = [&](float al, float& d2) {
      float v = 0.f, h2 = 0.f;
      // each contact's rows in registers, any condim (cone_eval's zones): with x_j = e_j
      // r_j and y_j = s_j r_j over the friction rows (r_j = mu_j / mu), sticking adds
      // D (x0 s0 + x.y) and D (s0^2 + |y|^2); sliding, with psi = mu T - x0 and
      // c = D / (1 + mu^2), adds c psi q0 and c q0^2 + (c psi mu / T)(|y|^2 - (x.y / T)^2),
      // q0 = mu x.y / T - s0: the curvature along (-1, mu t) and across t
      for (int c = t.lane; c < ncon; c += t.T) {
        const float* rc = con + kConRec * c;
        const int slot = __float_as_int(rc[17]);
        const int first = m.con_nr ? m.con_nr * c : slot >> 8;
        const int nd = m.con_nr ? m.con_nr : (slot >> 4) & 15;
        const float Dn = D[first], s0 = s[first], x0 = e[first] + al * s0;
        if (nd == 1) {
          if (x0 < 0.f) {
            v += s0 * Dn * x0;
            h2 += Dn * s0 * s0;
          }
          continue;
        }
        const float mu = rc[13];
        float rt = 1.f, rr = 1.f;
        if (nd > 3) {
          const int p = __float_as_int(rc[16]);
          rt = m.pair_mu_t[p] / mu;
          rr = m.pair_mu_r[p] / mu;
        }
        float xx = 0.f, xy = 0.f, yy = 0.f;
        for (int q = 1; q < nd; q++) {
          const float rq = q < 3 ? 1.f : (q == 3 ? rt : rr);
          const float yq = s[first + q] * rq, xq = (e[first + q] + al * s[first + q]) * rq;
          xx += xq * xq;
          xy += xq * yq;
          yy += yq * yq;
        }
        const float Tn = sqrtf(xx);
        if (!(x0 < mu * Tn)) continue;  // separated
        if (mu * x0 + Tn <= 0.f) {       // sticking
          v += Dn * (x0 * s0 + xy);
          h2 += Dn * (s0 * s0 + yy);
        } else {                         // sliding on the cone's surface
          const float inv = 1.f / Tn, psi = mu * Tn - x0, cc = Dn / (1.f + mu * mu);
          const float q0 = mu * xy * inv - s0, xt = xy * inv;
          v += cc * psi * q0;
          h2 += cc * q0 * q0 + cc * psi * mu * inv * fmaxf(yy - xt * xt, 0.f);
        }
      }
      for (int r = nrc + t.lane; r < nrow; r += t.T) {
        const float ep = e[r] + al * s[r];
        v += s[r] * row_s(r, ep);
        if (row_q(r, ep)) h2 += D[r] * s[r] * s[r];
      }
      d2 = t.sum(h2) + dMd;
      return t.sum(v) + dMr + al * dMd;
    };
    float d2, lo = 0.f, hi = 1.f;
    for (int k = 0; k < 30 && dphi(hi, d2) < 0.f; k++) { lo = hi; hi *= 2.f; }
    float al = lo < 1.f ? 1.f : hi;
    for (int k = 0; k < 24; k++) {
      const float v = dphi(al, d2);
      if (v == 0.f) break;
      if (v < 0.f) lo = al; else hi = al;
      float next = al - v / d2;
      if (!(next > lo && next < hi)) next = 0.5f * (lo + hi);
      const bool done = !(fabsf(next - al) > 1e-6f * al) || !(hi - lo > 1e-6f * hi);
      al = next;
      if (done) break;
    }
    // ---- update, and whether a row or cone changed zone along the step
    float amax = 1.f, dmax = 0.f;
    for (int i = t.lane; i < nv; i += t.T) {
      a[i] += al * d[i];
      Mr[i] += al * Md[i];
      amax = fmaxf(amax, fabsf(a[i]));
      dmax = fmaxf(dmax, fabsf(al * d[i]));
    }
    int moved = 0, sliding = 0;
    for (int c = t.lane; c < ncon; c += t.T) {
      const float* rc = con + kConRec * c;
      const int slot = __float_as_int(rc[17]);
      const int first = m.con_nr ? m.con_nr * c : slot >> 8;
      const int nd = m.con_nr ? m.con_nr : (slot >> 4) & 15;
      if (nd == 1) {
        moved |= (e[first] < 0.f) != (e[first] + al * s[first] < 0.f);
        continue;
      }
      const float mu = rc[13];
      float rt = 1.f, rr = 1.f;
      if (nd > 3) {
        const int p = __float_as_int(rc[16]);
        rt = m.pair_mu_t[p] / mu;
        rr = m.pair_mu_r[p] / mu;
      }
      // zone of x = e r at the old and new iterate: 0 separated, 2 sticking, 1 sliding
      float T0 = 0.f, T1 = 0.f, x0 = e[first], x1 = e[first] + al * s[first];
      for (int j2 = 1; j2 < nd; j2++) {
        const float rj = j2 < 3 ? 1.f : (j2 == 3 ? rt : rr);
        const float u0 = e[first + j2] * rj, u1 = (e[first + j2] + al * s[first + j2]) * rj;
        T0 += u0 * u0;
        T1 += u1 * u1;
      }
      T0 = sqrtf(T0);
      T1 = sqrtf(T1);
      const int z0 = !(x0 < mu * T0) ? 0 : (mu * x0 + T0 <= 0.f ? 2 : 1);
      const int z1 = !(x1 < mu * T1) ? 0 : (mu * x1 + T1 <= 0.f ? 2 : 1);
      moved |= z0 != z1;
      sliding |= z1 == 1;
    }
    for (int r = nrc + t.lane; r < nrow; r += t.T) {
      const float e1 = e[r] + al * s[r];
      moved |= FR ? (row_piece(D[r], fl[r], e[r]) != row_piece(D[r], fl[r], e1))
                  : ((e[r] < 0.f) != (e1 < 0.f));
    }
    t.sync();
    for (int r = t.lane; r < nrow; r += t.T) e[r] += al * s[r];
    // Exit as newton_impl does once the last step stayed on one piece of every row and
    // cone and its refinement correction was small: with no cone sliding the cost is
    // quadratic there and the iterate is its minimiser; a sliding cone's cost is smooth
    // but not quadratic, and there the step itself must also be below the tolerance
    // (Newton's quadratic convergence leaves the next one far smaller).
    moved = t.ior(moved);
    sliding = t.ior(sliding);
    const float cm = t.max(cmax), am = t.max(amax), dm = t.max(dmax);
    t.sync();
    if (!moved && cm <= kNewtonExitTol * am && (!sliding || dm <= kNewtonExitTol * am)) break;
    kept = !moved && !sliding;
  }
  // ---- the final slopes (the rows' forces are -sl)
  for (int c = t.lane; c < ncon; c += t.T) {
    int first;
    float mu, ratio[6], ev[6], sv[6], cc;
    const int nd = cone_of(m, con, c, first, mu, ratio);
    if (nd == 1) {
      sl[first] = fminf(D[first] * e[first], 0.f);
      continue;
    }
    for (int j = 0; j < nd; j++) ev[j] = e[first + j];
    cone_eval(mu, D[first], ratio, nd, ev, cc, sv);
    for (int j = 0; j < nd; j++) sl[first + j] = sv[j];
  }
  for (int r = nrc + t.lane; r < nrow; r += t.T) sl[r] = row_s(r, e[r]);
  t.sync();
}

// CONE: the instantiation that can solve elliptic-cone models (kept out of the others,
// whose registers it would crowd)
template <bool CONE = false>
DEV void newton(const DevModel& m, float* W, const Team& t, int& status, int iters,
                float gtol = 0.f) {
  if constexpr (CONE) {
    if (m.cone) {
      if (has_bounds(m)) newton_cone<true>(m, W, t, status, iters, gtol);
      else newton_cone<false>(m, W, t, status, iters, gtol);
      return;
    }
  }
  if (has_bounds(m)) newton_impl<true>(m, W, t, status, iters, gtol);
  else newton_impl<false>(m, W, t, status, iters, gtol);
}

// ------------------------------------------------- A10: forces, A11: integration
DEV void export_contacts(const DevModel& m, float* W, const Team& t, float* out, int* nout) {
  const int* scal = (const int*)(W + m.o_scal);
  const int ncon = scal[SC_NCON];
  const float* con = W + m.o_con;
  const float* D = W + m.o_D;
  const float* er = W + m.o_e;  // J qacc - aref, kept current by the Newton updates
  for (int idx = ncon * kConOut + t.lane; idx < m.nconmax * kConOut; idx += t.T) out[idx] = 0.f;
  for (int c = t.lane; c < ncon; c += t.T) {
    const float* r = con + kConRec * c;
    const int slot = __float_as_int(r[17]);
    const int first = m.con_nr ? m.con_nr * c : slot >> 8, nr = m.con_nr ? m.con_nr : (slot >> 4) & 15;
    float f[4] = {0.f, 0.f, 0.f, 0.f}, fn = 0.f;
    for (int e = 0; e < nr; e++) {
      const float fe = fmaxf(-D[first + e] * er[first + e], 0.f);
      fn += fe;
      if (e < 4) f[e] = fe;
    }
    float* o = out + kConOut * c;
    for (int k = 0; k < 13; k++) o[k] = r[k];
    for (int k = 0; k < 3; k++) o[1 + k] = r[1 + k] - W[m.o_xpos + k];  // world position
    if (m.cone) {  // elliptic: the frame rows' forces, minus their final slopes
      const float* sl = W + m.o_sl;
      o[13] = -sl[first];
      o[14] = nr > 1 ? -sl[first + 1] : 0.f;
      o[15] = nr > 1 ? -sl[first + 2] : 0.f;
    } else {  // the normal force sums every edge; torsion and rolling are not exported
      o[13] = fn;
      o[14] = r[13] * (f[0] - f[1]);
      o[15] = r[13] * (f[2] - f[3]);
    }
    o[16] = (float)__float_as_int(r[16]);
    o[17] = (float)(__float_as_int(r[17]) & 15);
  }
  if (t.lane == 0 && nout) *nout = ncon;
}

// Position update qout <- qin (+) h vel (qout may be qin): hinge and slide coordinates
// add h vel; a free joint's position adds h v and its orientation turns by the
// exponential map of the body-frame rotation h w (then renormalised).  `bad` flags a
// non-finite result.
DEV void integrate_pos(const DevModel& m, const Team& t, const float* qin, const float* vel,
                       float h, float* qout, bool& bad) {
  for (int j = t.lane; j < m.njnt; j += t.T) {
    const int qa = m.jnt_qposadr[j], da = m.jnt_dofadr[j];
    if (m.jnt_type[j] == JNT_FREE) {
      for (int k = 0; k < 3; k++) qout[qa + k] = qin[qa + k] + h * vel[da + k];
      float w[3] = {h * vel[da + 3], h * vel[da + 4], h * vel[da + 5]};
      float ang = sqrtf(dot3(w, w));
      float dq[4];
      if (ang > 1e-15f) {
        float sn, cs;
        sincosf(0.5f * ang, &sn, &cs);
        float sc = sn / ang;
        dq[0] = cs; dq[1] = w[0] * sc; dq[2] = w[1] * sc; dq[3] = w[2] * sc;
      } else {
        dq[0] = 1.f; dq[1] = 0.5f * w[0]; dq[2] = 0.5f * w[1]; dq[3] = 0.5f * w[2];
      }
      const float q0 = qin[qa + 3], q1 = qin[qa + 4], q2 = qin[qa + 5], q3 = qin[qa + 6];
      float r0 = q0 * dq[0] - q1 * dq[1] - q2 * dq[2] - q3 * dq[3];
      float r1 = q0 * dq[1] + q1 * dq[0] + q2 * dq[3] - q3 * dq[2];
      float r2 = q0 * dq[2] - q1 * dq[3] + q2 * dq[0] + q3 * dq[1];
      float r3 = q0 * dq[3] + q1 * dq[2] - q2 * dq[1] + q3 * dq[0];
      float inv = 1.f / sqrtf(r0 * r0 + r1 * r1 + r2 * r2 + r3 * r3);
      qout[qa + 3] = r0 * inv; qout[qa + 4] = r1 * inv;
      qout[qa + 5] = r2 * inv; qout[qa + 6] = r3 * inv;
      for (int k = 0; k < 7; k++) bad |= !isfinite(qout[qa + k]);
    } else {
      qout[qa] = qin[qa] + h * vel[da];
      bad |= !isfinite(qout[qa]);
    }
  }
}

// A11: semi-implicit Euler, velocity first, then the positions with the new velocity.
// With implicit damping or gains the velocity update takes the acceleration left in
// o_frc by implicit_damping; otherwise the solve's qacc.
DEV void integrate(const DevModel& m, float* W, const Team& t, int& status) {
  float* qpos = W + m.o_qpos;
  float* qvel = W + m.o_qvel;
  const float* a = W + (m.implicit ? m.o_frc : m.o_qacc);
  const float h = m.dt;
  for (int i = t.lane; i < m.nv; i += t.T) qvel[i] += h * a[i];
  t.sync();
  bool bad = false;
  for (int i = t.lane; i < m.nv; i += t.T) bad |= !isfinite(qvel[i]);
  integrate_pos(m, t, qpos, qvel, h, qpos, bad);
  if (bad) status |= 1;
  t.sync();
}

// ------------------------------------------------------------- one full step
// Phase timing for profiling builds only (-DMJH_PHASE_TIMING): every lane accumulates
// cycle counts per phase; release builds compile the marks away.
#ifdef MJH_PHASE_TIMING
#define MJH_MARK(k)                                           \
  do {                                                        \
    t.sync();                                                 \
    long long now_ = (long long)__builtin_readcyclecounter(); \
    if (ph) ph[k] += now_ - *last;                            \
    *last = now_;                                             \
  } while (0)
#else
#define MJH_MARK(k) \
  do {              \
  } while (0)
#endif

// Implicit damping (integrator 1): the forces linear in a dof's own velocity (joint
// damping, PD velocity gains) act at the end-of-step velocity, so the integrator's
// acceleration solves (M + h diag(b + kd)) a_int = qfrc_smooth + J^T f, with the row
// forces f of the solve that used M (f = -s'(e) per row piece).  Integrator 2 also
// takes the PD stiffness at the end-of-step position q + h qvel': the matrix gains
// h^2 diag(kp) (folded into dof_vgain) and the right-hand side -h diag(kp) qvel.
// a_int replaces the smooth force in o_frc; qacc keeps the solve's a* (reported, and
// the warm start).
DEV void implicit_damping(const DevModel& m, float* W, const Team& t) {
  const int* scal = (const int*)(W + m.o_scal);
  const int nv = m.nv, nrow = scal[SC_NROW];
  const float* D = W + m.o_D;
  const float* e = W + m.o_e;
  const float* fl = W + m.o_fl;
  const bool fr = has_bounds(m);
  float* rhs = W + m.o_frc;
  const float* qvel = W + m.o_qvel;
  const float* sl = W + m.o_sl;  // elliptic cones: the solve's final slopes
  if (m.implicit == 2)
    for (int i = t.lane; i < nv; i += t.T) rhs[i] -= m.dof_hkp[i] * qvel[i];
  const RowBounds rb = pad_rows(m, W, t, nrow);  // the solve's padding, rebuilt
  rows_t_times(m, W, t, rb, [&](int r) {
    if (r >= nrow) return 0.f;
    return -(m.cone ? sl[r] : (fr ? row_slope(D[r], fl[r], e[r]) : fminf(D[r] * e[r], 0.f)));
  }, rhs, rhs);
  if (nv <= t.T) {
    // the smooth phase's dense factor in leaves-first order, of M + h diag(dof_vgain),
    // solved in place in rhs in reversed order
    for (int i = t.lane; i < nv / 2; i += t.T) {
      const float u = rhs[i];
      rhs[i] = rhs[nv - 1 - i];
      rhs[nv - 1 - i] = u;
    }
    t.sync();
    hessian_cholesky(m, W, t, 0, rhs, rhs, true, true);
    cholesky_back(m, W, t, rhs, rhs);
    for (int i = t.lane; i < nv / 2; i += t.T) {
      const float u = rhs[i];
      rhs[i] = rhs[nv - 1 - i];
      rhs[nv - 1 - i] = u;
    }
    t.sync();
  } else {
    ltdl_factor(m, W, t, rhs, true);  // also solves L^T y = rhs in place
    ltdl_solve(m, W, t, nullptr, rhs, true);
  }
}

template <bool CONE = false>
DEV void world_step(const DevModel& m, float* W0, const Team& t0, const float* ctrl,
                    int& status, int iters, float gtol = 0.f, long long* ph = nullptr,
                    long long* last = nullptr, const float* dr = nullptr) {
#define MJH_PHASE_CTX                                   \
  float* W = W0 + opaque_zero();                        \
  const Team t{t0.lane + opaque_zero(), t0.T, t0.tp};
  {
    MJH_PHASE_CTX
    actuation(m, W, t, ctrl, dr);
    MJH_MARK(0);
  }
  {
    MJH_PHASE_CTX
    forward_sweep(m, W, t, nullptr, dr);
    MJH_MARK(1);
  }
  {
    MJH_PHASE_CTX
    backward_and_mass(m, W, t, dr);
    MJH_MARK(2);
  }
  {
    MJH_PHASE_CTX
    float* a0 = W + m.o_a0;
    const float* frc = W + m.o_frc;
    if (m.nv <= t.T) {
      // a0 = M^-1 frc by the blocked dense Cholesky of the Newton Hessian with no rows:
      // two barriers per four columns take fewer dependent steps than the tree LTDL's
      // one barrier per dof.  It factors M in reversed dof order (leaves first, the
      // LTDL's elimination order): a floating base eliminated first would subtract its
      // large coupling from the light links' inertias and lose FP32 digits there.
      // The solve runs in a0 in reversed order (P reverses the dofs).
      for (int i = t.lane; i < m.nv; i += t.T) a0[i] = frc[m.nv - 1 - i];
      t.sync();
      hessian_cholesky(m, W, t, 0, a0, a0, true);  // L y = P frc
      cholesky_back(m, W, t, a0, a0);              // L^T x = y, a0 = P x
      for (int i = t.lane; i < m.nv / 2; i += t.T) {
        const float u = a0[i];
        a0[i] = a0[m.nv - 1 - i];
        a0[m.nv - 1 - i] = u;
      }
      t.sync();
    } else {
      for (int i = t.lane; i < m.nv; i += t.T) a0[i] = frc[i];
      ltdl_factor(m, W, t, W + m.o_a0);  // also solves L^T y = frc in place
      ltdl_solve(m, W, t, nullptr, W + m.o_a0, true);
    }
    MJH_MARK(3);
  }
  {
    MJH_PHASE_CTX
    collide_candidates(m, W, t);
    select_contacts(m, W, t, status, dr);
    MJH_MARK(4);
  }
  {
    MJH_PHASE_CTX
    constraint_rows(m, W, t);
    MJH_MARK(5);
  }
  {
    MJH_PHASE_CTX
    newton<CONE>(m, W, t, status, iters, gtol);
    MJH_MARK(6);
  }
  if (m.implicit) {
    MJH_PHASE_CTX
    implicit_damping(m, W, t);
  }
#undef MJH_PHASE_CTX
}

// Fourth-order Runge-Kutta (integrator 3).  The step runs the whole forward pass at four
// stages, one `world_step` call site in a stage loop around these helpers: stage k = 2,
// 3, 4 starts at (q0 (+) c_k h v_{k-1}, v0 + c_k h a_{k-1}), c = (1/2, 1/2, 1), warm-
// started from a_{k-1}; afterwards q <- q0 (+) h/6 (v1 + 2 v2 + 2 v3 + v4) and
// qdot <- v0 + h/6 (a1 + 2 a2 + 2 a3 + a4), and qacc (reported, and the next warm
// start) is a1.  The block at o_rk holds q0, v0, a1 and the two weighted sums.

// set the state of stage k >= 1 from the previous stage's velocity and acceleration
DEV void rk4_begin(const DevModel& m, float* W, const Team& t, int k) {
  float* qvel = W + m.o_qvel;
  const float* q0 = W + m.o_rk;
  const float* v0 = q0 + m.nq;
  const float ch = (k == 3 ? 1.f : 0.5f) * m.dt;
  bool bad = false;  // a non-finite stage shows in the final state
  integrate_pos(m, t, q0, qvel, ch, W + m.o_qpos, bad);
  t.sync();
  const float* qacc = W + m.o_qacc;
  for (int i = t.lane; i < m.nv; i += t.T) qvel[i] = v0[i] + ch * qacc[i];
  t.sync();
}

// after stage k's forward pass: keep the step's start (k = 0) and add the stage's
// velocity and acceleration to the weighted sums (weights 1, 2, 2, 1)
DEV void rk4_accumulate(const DevModel& m, float* W, const Team& t, int k) {
  const int nq = m.nq, nv = m.nv;
  const float* qvel = W + m.o_qvel;
  const float* qacc = W + m.o_qacc;
  float* q0 = W + m.o_rk;
  float* v0 = q0 + nq;
  float* a1 = v0 + nv;
  float* vs = a1 + nv;
  float* as = vs + nv;
  if (k == 0) {
    const float* qpos = W + m.o_qpos;
    for (int i = t.lane; i < nq; i += t.T) q0[i] = qpos[i];
    for (int i = t.lane; i < nv; i += t.T) {
      v0[i] = qvel[i]; a1[i] = qacc[i];
      vs[i] = qvel[i]; as[i] = qacc[i];
    }
  } else {
    const float bk = k == 3 ? 1.f : 2.f;
    for (int i = t.lane; i < nv; i += t.T) {
      vs[i] += bk * qvel[i];
      as[i] += bk * qacc[i];
    }
  }
  t.sync();
}

DEV void rk4_combine(const DevModel& m, float* W, const Team& t, int& status) {
  const int nq = m.nq, nv = m.nv;
  const float h = m.dt;
  float* qvel = W + m.o_qvel;
  float* qacc = W + m.o_qacc;
  const float* q0 = W + m.o_rk;
  const float* v0 = q0 + nq;
  const float* a1 = v0 + nv;
  float* vs = const_cast<float*>(a1) + nv;
  const float* as = vs + nv;
  for (int i = t.lane; i < nv; i += t.T) vs[i] = vs[i] / 6.f;
  t.sync();
  bool bad = false;
  integrate_pos(m, t, q0, vs, h, W + m.o_qpos, bad);
  for (int i = t.lane; i < nv; i += t.T) {
    qvel[i] = v0[i] + h * (as[i] / 6.f);
    qacc[i] = a1[i];
    bad |= !isfinite(qvel[i]);
  }
  if (bad) status |= 1;
  t.sync();
}

// copy a model's triangular pair table to the head of the work-group's LDS (all
// threads of the work-group take part; call before any team leaves)
DEV void load_pair_table(const DevModel& m, unsigned* tab) {
  for (int k = threadIdx.x; k < (m.ntri + 3) / 4; k += blockDim.x) tab[k] = m.tri_pair[k];
  __syncthreads();
}

// initialise the world's constant LDS slots (world body, zero pattern of M)
DEV void world_init(const DevModel& m, float* W, const Team& t) {
  for (int k = t.lane; k < m.lds_words; k += t.T) W[k] = 0.f;
  t.sync();
  if (t.lane == 0) {
    float* xmat = W + m.o_xmat;
    xmat[0] = xmat[4] = xmat[8] = 1.f;
    float* cacc = W + m.o_cacc;
    cacc[3] = -m.grav[0]; cacc[4] = -m.grav[1]; cacc[5] = -m.grav[2];
  }
  t.sync();
}

}  // namespace mjh
