// Kernels of the batched physics step.
//
// mjh_step_kernel: one work-group per task (a run of worlds of one model); inside it a
// team of T lanes (16, 32 or 64, chosen per model) owns one world.  The world's state
// is loaded from HBM into LDS once, advanced `nstep` steps on chip (only the controls
// are read per step), and written back once.  The same kernel serves a batch of
// several models: each work-group reads its task and its group's model descriptor.
// No work-group barrier is used, so teams beyond a task's world count simply exit.
#include <hip/hip_runtime.h>

#include "mjh_device.h"
#include "mjh_kernels.h"

namespace mjh {

#ifdef MJH_PHASE_TIMING
// per-world phase cycle totals of the last launch (profiling builds only)
constexpr int kPhaseWorlds = 8192;
__device__ long long g_phase_cycles[kPhaseWorlds * 8];
#endif

// RK: the instantiation that can run fourth-order Runge-Kutta groups (four forward
// passes a step); the other compiles the one-pass step alone.  CONE: the one that can
// solve elliptic-cone models (with RK, for any batch that has one).
template <bool RK, bool CONE>
__device__ __forceinline__ void run_worlds(const DevGroup& G, float* W, int world, int nstep, int lane, int T,
                           const unsigned char* tab) {
  const DevModel& m = G.m;
  const Team t{lane, T, tab};
  world_init(m, W, t);
  const int nq = m.nq, nv = m.nv, nu = m.nu;
  const size_t w = (size_t)world;
  for (int i = lane; i < nq; i += T) W[m.o_qpos + i] = G.qpos[w * nq + i];
  for (int i = lane; i < nv; i += T) {
    W[m.o_qvel + i] = G.qvel[w * nv + i];
    W[m.o_qacc + i] = G.qacc[w * nv + i];
  }
  t.sync();
  int status = 0;
#ifdef MJH_PHASE_TIMING
  long long ph[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  long long last = (long long)__builtin_readcyclecounter();
#endif
  for (int s = 0; s < nstep; s++) {
    const float* u = G.ctrl ? G.ctrl + ((size_t)s * G.nworld + w) * nu : nullptr;
    const bool rk = RK && m.rk4;
    for (int k = 0; k < (rk ? 4 : 1); k++) {
      if (k > 0) rk4_begin(m, W, t, k);
#ifdef MJH_PHASE_TIMING
      world_step<CONE>(m, W, t, u, status, m.iterations, 0.f, ph, &last);
#else
      world_step<CONE>(m, W, t, u, status, m.iterations);
#endif
      if (k == 0 && s == nstep - 1 && G.con_out)
        export_contacts(m, W, t, G.con_out + w * m.nconmax * kConOut,
                        G.ncon_out ? G.ncon_out + w : nullptr);
      if (rk) rk4_accumulate(m, W, t, k);
    }
    if (rk) rk4_combine(m, W, t, status);
    else integrate(m, W, t, status);
#ifdef MJH_PHASE_TIMING
    t.sync();
    const long long now_ = (long long)__builtin_readcyclecounter();
    ph[7] += now_ - last;
    last = now_;
#endif
  }
#ifdef MJH_PHASE_TIMING
  if (lane == 0 && world < kPhaseWorlds)
    for (int k = 0; k < 8; k++) g_phase_cycles[world * 8 + k] = ph[k];
#endif
  for (int i = lane; i < nq; i += T) G.qpos[w * nq + i] = W[m.o_qpos + i];
  for (int i = lane; i < nv; i += T) {
    G.qvel[w * nv + i] = W[m.o_qvel + i];
    G.qacc[w * nv + i] = W[m.o_qacc + i];
  }
  status = t.ior(status);
  if (lane == 0 && G.status) G.status[w] = status;
}

template <bool RK, bool CONE>
__global__ void __launch_bounds__(kMaxBlock, 4)
mjh_step_kernel(const DevGroup* __restrict__ groups, const DevTask* __restrict__ tasks,
                int nstep, int tab_words) {
  extern __shared__ float lds[];
  const DevTask tk = tasks[blockIdx.x];
  const DevGroup& G = groups[tk.group];
  load_pair_table(G.m, (unsigned*)lds);
  const int T = G.team;
  const int team = threadIdx.x / T;
  if (team >= tk.nw) return;
  float* W = lds + tab_words + (size_t)team * G.m.lds_words;
  const int lane = threadIdx.x - team * T;
  const int world = tk.w0 + team;
  run_worlds<RK, CONE>(G, W, world, nstep, lane, T, (const unsigned char*)lds);
}

// ------------------------------------------------------------- environment step
// The joystick locomotion task around the physics step (the paper's locomotion
// appendix): per env step, `nsub` physics steps with the action held as the position
// actuators' targets, then from the new state
//   obs    = [g_b, v_b, w_b, q - q_default, qdot, a_{t-1}, cmd]  (b: root body frame;
//            g the gravity direction, v the root's world linear velocity rotated in)
//   reward = max(0, 1.0 exp(-|cmd_xy - v_xy|^2/0.25) + 0.5 exp(-(cmd_wz - w_z)^2/0.25)
//            - 2 v_z^2 - 0.05 |w_xy|^2 - 5 |g_xy|^2 - 2e-4 |tau|^2 - 0.1 |q - q_default|^2
//            - 0.01 |a_t - a_{t-1}|^2 - 1e-3 sum |qdot tau| + 0.5 exp(-|q - q_default|^2)
//            - done)                                  (tau: PD torques at the new state)
//   done   = the root's z axis points downwards (inverted), or the state is no longer
//            finite (then the reward is 0).
// A terminated world restarts from its reset state with a zero warm start and a zero
// previous action.  The root is a free joint; actuator k drives dof 6 + k.
// Domain randomisation (optional): each world's parameter record (layout at kDrFric)
// drives its physics, and the observation and reward see the calibrated joint reading
// q + offset and the world's gains; sensor noise, when given, is added to every entry
// of the observation.
constexpr float kEnvKv = 1.f, kEnvSv = 0.25f, kEnvKw = 0.5f, kEnvSw = 0.25f;
constexpr float kEnvLinZ = -2.f, kEnvAngXY = -0.05f, kEnvOri = -5.f, kEnvTau = -2e-4f;
constexpr float kEnvQ = -0.1f, kEnvRate = -0.01f, kEnvTerm = -1.f;
constexpr float kEnvEnergy = -1e-3f, kEnvPose = 0.5f;

template <bool RK>
__device__ __forceinline__ void env_worlds(const DevGroup& G, const EnvArgs& E, float* W, float* aprev, float* dr,
                           int world, int lane, int T, const unsigned char* tab) {
  const DevModel& m = G.m;
  const Team t{lane, T, tab};
  world_init(m, W, t);
  const int nq = m.nq, nv = m.nv, nu = m.nu;
  const size_t w = (size_t)world;
  float* qpos = W + m.o_qpos;
  float* qvel = W + m.o_qvel;
  float* qacc = W + m.o_qacc;
  for (int i = lane; i < nq; i += T) qpos[i] = G.qpos[w * nq + i];
  for (int i = lane; i < nv; i += T) {
    qvel[i] = G.qvel[w * nv + i];
    qacc[i] = G.qacc[w * nv + i];
  }
  t.sync();
  for (int k = lane; k < nu; k += T) aprev[k] = E.last_action[w * nu + k];
  if (dr)
    for (int k = lane; k < E.ndr; k += T) dr[k] = E.dr[w * E.ndr + k];
  t.sync();
  int status = 0;
  for (int e = 0; e < E.nenv; e++) {
    const float* u = E.action + ((size_t)e * G.nworld + w) * nu;
    for (int s = 0; s < E.nsub; s++) {
      const bool rk = RK && m.rk4;
      for (int k = 0; k < (rk ? 4 : 1); k++) {
        if (k > 0) rk4_begin(m, W, t, k);
        world_step(m, W, t, u, status, m.iterations, 0.f, nullptr, nullptr, dr);
        if (rk) rk4_accumulate(m, W, t, k);
      }
      if (rk) rk4_combine(m, W, t, status);
      else integrate(m, W, t, status);
    }
    // (read here, after the physics steps, rather than held across them)
    const float skp = dr ? dr[kDrKp] : 1.f, skd = dr ? dr[kDrKd] : 1.f;
    const float* cmd = E.command + w * 3;
    // root rotation from its quaternion (every lane)
    float qw = qpos[3], qx = qpos[4], qy = qpos[5], qz = qpos[6];
    const float qn = 1.f / sqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
    qw *= qn; qx *= qn; qy *= qn; qz *= qn;
    const float R[9] = {1.f - 2.f * (qy * qy + qz * qz), 2.f * (qx * qy - qw * qz),
                        2.f * (qx * qz + qw * qy), 2.f * (qx * qy + qw * qz),
                        1.f - 2.f * (qx * qx + qz * qz), 2.f * (qy * qz - qw * qx),
                        2.f * (qx * qz - qw * qy), 2.f * (qy * qz + qw * qx),
                        1.f - 2.f * (qx * qx + qy * qy)};
    float gb[3], vb[3];
    for (int k = 0; k < 3; k++) {
      gb[k] = -R[6 + k];
      vb[k] = R[k] * qvel[0] + R[3 + k] * qvel[1] + R[6 + k] * qvel[2];
    }
    // a state that is no longer finite also terminates the world (reward 0)
    int bad = 0;
    for (int i = lane; i < nq; i += T) bad |= !isfinite(qpos[i]);
    for (int i = lane; i < nv; i += T) bad |= !isfinite(qvel[i]);
    bad = t.ior(bad);
    const bool done = bad || R[8] < 0.f;
    // per-actuator terms, one lane each
    float jt = 0.f, pose = 0.f;
    for (int k = lane; k < nu; k += T) {
      const float lo = m.act_lo[k], hi = m.act_hi[k];
      const float uk = fminf(fmaxf(u[k], lo), hi);
      const float q = qpos[7 + k], qd = qvel[6 + k];
      const float q0 = dr ? m.act_qdef[k] - dr[kDrHead + k] : m.act_qdef[k];
      const float tau = skp * m.act_kp[k] * (q0 + m.act_gear[k] * uk - q) - skd * m.act_kd[k] * qd;
      const float dq = q - q0, da = u[k] - aprev[k];
      jt += kEnvTau * tau * tau + kEnvQ * dq * dq + kEnvRate * da * da +
            kEnvEnergy * fabsf(qd * tau);
      pose += dq * dq;
    }
    jt = t.sum(jt);
    pose = t.sum(pose);
    float* ob = E.obs + ((size_t)e * G.nworld + w) * E.nobs;
    for (int i = lane; i < E.nobs; i += T) {
      float v;
      if (i < 3) v = gb[i];
      else if (i < 6) v = vb[i - 3];
      else if (i < 9) v = qvel[i - 3];
      else if (i < 9 + nu) v = qpos[7 + (i - 9)] - (dr ? m.act_qdef[i - 9] - dr[kDrHead + i - 9]
                                                         : m.act_qdef[i - 9]);
      else if (i < 9 + 2 * nu) v = qvel[6 + (i - 9 - nu)];
      else if (i < 9 + 3 * nu) v = aprev[i - 9 - 2 * nu];
      else v = cmd[i - 9 - 3 * nu];
      if (E.noise) v += E.noise[((size_t)e * G.nworld + w) * E.nobs + i];
      ob[i] = v;
    }
    if (lane == 0) {
      const float ex = cmd[0] - vb[0], ey = cmd[1] - vb[1], ez = cmd[2] - qvel[5];
      float r = kEnvKv * expf(-(ex * ex + ey * ey) / kEnvSv) + kEnvKw * expf(-ez * ez / kEnvSw) +
                kEnvLinZ * vb[2] * vb[2] + kEnvAngXY * (qvel[3] * qvel[3] + qvel[4] * qvel[4]) +
                kEnvOri * (gb[0] * gb[0] + gb[1] * gb[1]) + jt + kEnvPose * expf(-pose) +
                (done ? kEnvTerm : 0.f);
      E.reward[(size_t)e * G.nworld + w] = bad ? 0.f : fmaxf(r, 0.f);
      E.done[(size_t)e * G.nworld + w] = done ? 1 : 0;
    }
    t.sync();  // every lane has read aprev and the state
    for (int k = lane; k < nu; k += T) aprev[k] = done ? 0.f : u[k];
    if (done) {
      for (int i = lane; i < nq; i += T) qpos[i] = E.reset_qpos[w * nq + i];
      for (int i = lane; i < nv; i += T) {
        qvel[i] = E.reset_qvel[w * nv + i];
        qacc[i] = 0.f;
      }
    }
    t.sync();
  }
  for (int i = lane; i < nq; i += T) G.qpos[w * nq + i] = qpos[i];
  for (int i = lane; i < nv; i += T) {
    G.qvel[w * nv + i] = qvel[i];
    G.qacc[w * nv + i] = qacc[i];
  }
  for (int k = lane; k < nu; k += T) E.last_action[w * nu + k] = aprev[k];
  status = t.ior(status);
  if (lane == 0 && G.status) G.status[w] = status;
}

// LDS: the pair table, then `ap_words` holding each team's previous action and, with
// randomisation, its parameter record (nu + ndr words a team), then the worlds' working
// sets at the usual stride.
template <bool RK, bool DR>
__global__ void __launch_bounds__(kMaxBlock, 4)
mjh_env_kernel(const DevGroup* __restrict__ groups, const DevTask* __restrict__ tasks,
               EnvArgs E, int tab_words, int ap_words) {
  extern __shared__ float lds[];
  const DevTask tk = tasks[blockIdx.x];
  const DevGroup& G = groups[tk.group];
  load_pair_table(G.m, (unsigned*)lds);
  const int T = G.team;
  const int team = threadIdx.x / T;
  if (team >= tk.nw) return;
  float* ap = lds + tab_words + team * (G.m.nu + E.ndr);
  float* W = lds + tab_words + ap_words + (size_t)team * G.m.lds_words;
  env_worlds<RK>(G, E, W, ap, DR ? ap + G.m.nu : nullptr, tk.w0 + team, threadIdx.x - team * T, T,
             (const unsigned char*)lds);
}

// Translational inverse weight of every body at qpos0:
//   w(b) = trace(J_com(b) M^-1 J_com(b)^T) / 3,
// and (M^-1)_kk of every dof k, one work-group of 64 lanes evaluating the model once.
__global__ void __launch_bounds__(64) mjh_invweight_kernel(DevModel m, int tab_words) {
  extern __shared__ float lds[];
  load_pair_table(m, (unsigned*)lds);
  float* W = lds + tab_words;
  const Team t{(int)threadIdx.x, 64, (const unsigned char*)lds};
  world_init(m, W, t);
  for (int i = t.lane; i < m.nq; i += t.T) W[m.o_qpos + i] = m.qpos0[i];
  t.sync();
  forward_sweep(m, W, t);
  backward_and_mass(m, W, t);
  ltdl_factor(m, W, t);
  // scratch: the smooth-force and unconstrained-acceleration vectors, unused here (the
  // Newton vectors share words with the poses read below, and the sweep scratch with
  // the factor in H)
  float* jr = W + m.o_frc;
  float* x = W + m.o_a0;
  const float* cdof = W + m.o_cdof;
  for (int b = 0; b < m.nbody; b++) {
    if (b == 0) {
      if (t.lane == 0) m.body_invweight[0] = 0.f;
      continue;
    }
    float c[3];
    mv3(W + m.o_xmat + 9 * b, m.body_ipos + 3 * b, c);
    for (int k = 0; k < 3; k++) c[k] += W[m.o_xpos + 3 * b + k];
    float tr = 0.f;
    for (int r = 0; r < 3; r++) {
      for (int i = t.lane; i < m.nv; i += t.T) {
        float v = 0.f;
        if (m.body_dofmask[b] >> i & 1ull) {
          float wx[3];
          cross3(cdof + 6 * i, c, wx);
          v = cdof[6 * i + 3 + r] + wx[r];
        }
        jr[i] = v;
      }
      t.sync();
      ltdl_solve(m, W, t, jr, x);
      float part = 0.f;
      for (int i = t.lane; i < m.nv; i += t.T) part += jr[i] * x[i];
      tr += t.sum(part);
      t.sync();
    }
    if (t.lane == 0) m.body_invweight[b] = tr / 3.f;
  }
  // joint-limit and friction-loss rows: (M^-1)_kk of every dof
  for (int k = 0; k < m.nv; k++) {
    for (int i = t.lane; i < m.nv; i += t.T) jr[i] = i == k ? 1.f : 0.f;
    t.sync();
    ltdl_solve(m, W, t, jr, x);
    if (t.lane == 0) m.dof_invweight[k] = x[k];
    t.sync();
  }
}

// ------------------------------------------------------------- host-side launchers
hipError_t launch_step(const DevGroup* groups, const DevTask* tasks, int ntask, int nstep,
                       int block, size_t lds_bytes, int tab_words, bool rk4, bool cone,
                       hipStream_t stream) {
  if (ntask <= 0) return hipSuccess;
  if (cone)
    hipLaunchKernelGGL((mjh_step_kernel<true, true>), dim3(ntask), dim3(block), lds_bytes,
                       stream, groups, tasks, nstep, tab_words);
  else if (rk4)
    hipLaunchKernelGGL((mjh_step_kernel<true, false>), dim3(ntask), dim3(block), lds_bytes,
                       stream, groups, tasks, nstep, tab_words);
  else
    hipLaunchKernelGGL((mjh_step_kernel<false, false>), dim3(ntask), dim3(block), lds_bytes,
                       stream, groups, tasks, nstep, tab_words);
  return hipGetLastError();
}

hipError_t set_step_lds_limit(size_t bytes) {
  hipError_t e = hipFuncSetAttribute((const void*)mjh_step_kernel<false, false>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)mjh_step_kernel<true, false>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)mjh_step_kernel<true, true>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_env(const DevGroup* groups, const DevTask* tasks, int ntask, const EnvArgs& E,
                      int block, size_t lds_bytes, int tab_words, int ap_words, bool rk4,
                      hipStream_t stream) {
  if (ntask <= 0) return hipSuccess;
  // one instantiation per case, so that the plain env step carries none of the
  // randomisation's live values; per-world records come with the Euler step only
  if (rk4)
    hipLaunchKernelGGL((mjh_env_kernel<true, false>), dim3(ntask), dim3(block), lds_bytes, stream,
                       groups, tasks, E, tab_words, ap_words);
  else if (E.dr)
    hipLaunchKernelGGL((mjh_env_kernel<false, true>), dim3(ntask), dim3(block), lds_bytes, stream,
                       groups, tasks, E, tab_words, ap_words);
  else
    hipLaunchKernelGGL((mjh_env_kernel<false, false>), dim3(ntask), dim3(block), lds_bytes, stream,
                       groups, tasks, E, tab_words, ap_words);
  return hipGetLastError();
}

hipError_t set_env_lds_limit(size_t bytes) {
  hipError_t e = hipFuncSetAttribute((const void*)mjh_env_kernel<false, false>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)mjh_env_kernel<false, true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)mjh_env_kernel<true, false>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_invweight(const DevModel& m, hipStream_t stream) {
  const int tab = table_words(m);
  const size_t lds = (size_t)(tab + m.lds_words) * sizeof(float);
  hipError_t e = hipFuncSetAttribute((const void*)mjh_invweight_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mjh_invweight_kernel, dim3(1), dim3(64), lds, stream, m, tab);
  return hipGetLastError();
}

#ifdef MJH_PHASE_TIMING
hipError_t read_phase_cycles(long long* host, int nworld) {
  const int n = nworld < kPhaseWorlds ? nworld : kPhaseWorlds;
  return hipMemcpyFromSymbol(host, HIP_SYMBOL(g_phase_cycles), sizeof(long long) * 8 * (size_t)n);
}
#endif

}  // namespace mjh
