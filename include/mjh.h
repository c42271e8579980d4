/*
 * mjh -- batched rigid-body physics step for AMD MI355X (gfx950), C ABI.
 *
 * The library advances many independent simulated worlds in lockstep on one GPU: the
 * physics step that MuJoCo Playground runs under its RL environments (the paper's
 * raw-throughput appendix times this "env step" alone with random actions; its
 * locomotion and manipulation PPO runs use 8192 parallel environments).  Each step
 * of each world runs, in order:
 *   actuation (motors, and the PD position mapping of eq. pd_mapping),
 *   forward kinematics, composite-rigid-body joint-space inertia with a tree-sparse
 *   L^T D L factorisation, recursive Newton-Euler bias forces, primitive collision
 *   (plane / sphere / capsule / box), a convex soft-constraint contact solve by Newton
 *   iterations with an exact line search over a pyramidal friction cone, and
 *   semi-implicit Euler integration.
 * The solver knobs are the MJCF options the paper edits per task (Table
 * tab:dm_control_envs): timestep, iterations, contact budget.
 *
 * Conventions
 *   - All device buffers are FP32 (state) or int32 (status), row-major [nworld][n],
 *     each world's row contiguous.  Quaternions are w-first.  A free joint's qpos is
 *     (x, y, z, qw, qx, qy, qz) and its qvel is (world linear velocity of the body
 *     origin, body-frame angular velocity).
 *   - Ownership: the library owns model arrays, scratch, checkpoint tapes and graphs
 *     (freed by mjh_world_free / mjh_destroy).  The caller owns state, controls,
 *     outputs and streams; a stream argument is a hipStream_t (NULL = default stream).
 *   - Execution: launches are asynchronous and stream-ordered.  mjh_model_upload,
 *     mjh_world_alloc, mjh_bind_* and mjh_autotune synchronise the device.
 *   - Errors: every call validates its arguments before launching anything.  A
 *     negative return is an error and mjh_last_error() describes it; nothing aborts
 *     the process.  Numerical trouble inside a world is not a call error: it is
 *     written to that world's status word and the other worlds continue.
 *   - Thread safety: one context must not be used from two host threads at once.
 */
#ifndef MJH_H_
#define MJH_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mjh_ctx mjh_ctx;
typedef struct mjh_batch mjh_batch;
typedef int32_t mjh_status;

enum {
  MJH_OK = 0,
  MJH_EINVAL = -1,       /* bad argument (NULL, size, range, unbound state)       */
  MJH_ENOMEM = -2,       /* device or host allocation failed                      */
  MJH_EHIP = -3,         /* a HIP runtime call failed (text in mjh_last_error)    */
  MJH_EMODEL = -4,       /* malformed model blob                                  */
  MJH_EUNSUPPORTED = -5, /* model feature outside what the kernels implement      */
  MJH_ESTATE = -6        /* call out of order (e.g. rollout_bwd before _fwd)      */
};

/* per-world status bits (OR-ed over the steps of one call) */
enum {
  MJH_WORLD_NONFINITE = 1, /* non-finite qpos/qvel after a step                    */
  MJH_WORLD_OVERFLOW = 2,  /* more penetrating candidates than nconmax; deepest kept*/
  MJH_WORLD_NODESCENT = 4  /* Newton Hessian factorisation failed; step truncated   */
};

/* contact record written by mjh_bind_io's contact_out: MJH_CON_SIZE floats each:
 * dist, pos[3], frame[9] (normal geom1->geom2, tangent1, tangent2),
 * f_normal, f_tangent1, f_tangent2, pair index, candidate index, 0, 0            */
#define MJH_CON_SIZE 20

typedef struct mjh_dims {
  int32_t nq, nv, nu, nbody, ngeom, npair;
  int32_t ncand;      /* candidate contact slots over all pairs                   */
  int32_t nconmax;    /* contact budget per world                                 */
  int32_t iterations; /* Newton iterations per step                              */
  int32_t lds_bytes;  /* on-chip working set of one world                        */
  float timestep;
  int32_t nlimit;     /* limited hinge/slide joints (at most one row each)        */
  int32_t nrowmax;    /* constraint rows per world: c nconmax + nlimit + nfric    */
                      /*   + (3 per connect, 6 per weld), c the widest contact's  */
                      /*   rows (1 frictionless, 4 / 6 / 10 for condim 3 / 4 / 6) */
  int32_t nfric;      /* dofs with friction loss (one row each, always present)   */
  int32_t neq;        /* equalities (connect or weld; rows always present)        */
} mjh_dims;

/* One context per device.  device: HIP device ordinal.  *out receives the handle. */
mjh_status mjh_create(int device, mjh_ctx** out);
void mjh_destroy(mjh_ctx* ctx);
/* Text of the last failing call on this context (never NULL; "" after success). */
const char* mjh_last_error(const mjh_ctx* ctx);

/* Parse a model blob (host memory, the layout written by the Python model module:
 * header, bodies, joints, geoms, pairs, actuators, qpos0), derive the tree tables,
 * upload FP32 constants and compute the bodies' translational inverse weights and the
 * limited dofs' inverse weights at qpos0 on the device.  *model_id receives a handle
 * valid until mjh_destroy.
 * Joint limits (a hinge or slide joint with range lo < hi) are one-sided soft
 * constraints of the same convex model as the contacts (Todorov 2014, which the paper's
 * MJX physics uses): a joint whose coordinate q lies outside its range adds one row
 * after the contact rows, in joint order, with distance r = q - lo and J = e_dof below
 * the range, r = hi - q and J = -e_dof above it, and the regulariser's A = (M^-1)_kk
 * at qpos0.  A hinge or slide joint with friction loss F > 0 (dry joint friction)
 * adds one row after those, in dof order, always present: J = e_dof, r = 0, the same
 * A, and a force confined to [-F, F] (a Huber term in the solver's cost).  A connect
 * equality (a point fixed in body1 held on a point fixed in body2, or in the world)
 * adds three two-sided rows last, one per world axis: J = J_p(b1, p1) - J_p(b2, p2),
 * r = p1 - p2, A = w(b1) + w(b2).  A weld equality also holds body1's orientation
 * relative to body2 at a stored reference Q: three more rows J = J_w(b1) - J_w(b2),
 * r = vee(E - E^T) / 2 with E = R1 Q R2^T, the same A.
 * A pair's contact dimension sets its rows per contact: condim 1 one normal row
 * (frictionless); 3 the sliding pyramid's four edges J_n +- mu J_t1, J_n +- mu J_t2;
 * 4 also J_n +- mu_t J_spin (torsion about the normal); 6 also J_n +- mu_r J_roll for
 * both tangents (rolling), all with R = (1-d)/d (1 + mu^2)(w1 + w2).
 * With the model option cone = 1 a contact's rows are instead its frame's (normal,
 * tangents, then spin and rolling for condim 4 / 6) under an elliptic cone: the rows
 * share the normal's impedance, friction rows have no distance term and R_j = R_n
 * (mu / mu_j)^2 with R_n = (1-d)/d (w1 + w2), and the contact's force is the projection
 * of -D x onto the round cone |g_t| <= mu g_n in the coordinates x_j = (J a - aref)_j
 * mu_j / mu (separated, sliding on the cone's surface, or sticking).
 * Integrator 1 takes joint damping and PD velocity gains implicitly, 2 also the PD
 * position gains, 3 is fourth-order Runge-Kutta (four forward passes a step).
 * mjh_rollout_fwd rejects the pairs its reverse pass does not differentiate and
 * elliptic cones (MJH_EUNSUPPORTED; the list is at mjh_rollout_fwd), and mjh_env_step
 * rejects elliptic cones.
 * MJH_EMODEL for a malformed blob, MJH_EUNSUPPORTED for nv > 64, box-box pairs,
 * a free joint below the root or two actuators on one dof. */
mjh_status mjh_model_upload(mjh_ctx* ctx, const void* blob, size_t nbytes,
                            int32_t* model_id);
mjh_status mjh_model_info(mjh_ctx* ctx, int32_t model_id, mjh_dims* out);
/* Copy the model's body translational inverse weights (nbody floats, host memory).
 * They scale the contact regulariser: R = (1-d)/d * (1+mu^2) * (w(body1) + w(body2)). */
mjh_status mjh_model_invweight(mjh_ctx* ctx, int32_t model_id, float* out);
/* Copy the limited joints' dof inverse weights (M^-1)_kk at qpos0 (nlimit floats, host
 * memory, joint order): the A of a joint-limit row, R = (1-d)/d * A. */
mjh_status mjh_model_limit_invweight(mjh_ctx* ctx, int32_t model_id, float* out);

/* A batch of worlds made of nmodel groups: counts[g] worlds of model model_ids[g].
 * Groups are stepped together in one launch.  counts[g] >= 0. */
mjh_status mjh_world_alloc(mjh_ctx* ctx, const int32_t* model_ids, const int32_t* counts,
                           int32_t nmodel, mjh_batch** out);
void mjh_world_free(mjh_batch* batch);

/* Bind caller-owned device state of group g: qpos [n][nq], qvel [n][nv],
 * qacc_ws [n][nv] (the Newton warm start; after a step it holds that step's
 * acceleration), status [n] (may be NULL).  The library reads and writes them in
 * every mjh_step.  Synchronous; must not overlap a step of this batch. */
mjh_status mjh_bind_state(mjh_batch* b, int32_t group, float* qpos, float* qvel,
                          float* qacc_ws, int32_t* status);
/* Bind per-call inputs/outputs of group g: ctrl [ctrl_nstep][n][nu] (device; NULL =
 * zero controls; step s of a call reads row s), contact_out [n][nconmax][MJH_CON_SIZE]
 * and ncon_out [n] (device, may be NULL) receive the last step's contacts. */
mjh_status mjh_bind_io(mjh_batch* b, int32_t group, const float* ctrl, int32_t ctrl_nstep,
                       float* contact_out, int32_t* ncon_out);

/* Advance every world of the batch by nstep steps (nstep <= bound ctrl_nstep unless
 * ctrl is NULL).  State stays on chip across the nstep steps of one launch. */
mjh_status mjh_step(mjh_batch* b, int32_t nstep, void* stream);

/* Joystick locomotion environment steps (the paper's locomotion appendix: observation
 * list, absolute joint-position actions through the PD mapping of eq. pd_mapping, a
 * subset of its reward table, termination when the robot inverts, and its domain
 * randomisation), fused around the physics step for a single-model batch whose body 1
 * is the free root and whose position actuator k drives dof 6 + k.  Each of `nenv` env
 * steps runs `nsub` physics steps with action[e] (device, [nenv][nworld][nu]) held as
 * the actuators' controls, then writes, from the new state, obs[e] ([nenv][nworld]
 * [12 + 3 nu]: gravity direction, root linear and angular velocity in the root frame,
 * joint readings minus their defaults, joint velocities, previous action, command[w]
 * ([nworld][3]: vx, vy, yaw rate)), reward[e] ([nenv][nworld]: max(0, 1.0 exp(-|cmd_xy -
 * v_xy|^2/0.25) + 0.5 exp(-(cmd_wz - w_z)^2/0.25) - 2 v_z^2 - 0.05 |w_xy|^2 - 5 |g_xy|^2
 * - 2e-4 |tau|^2 - 0.1 |q - q_default|^2 - 0.01 |a_t - a_{t-1}|^2 - 1e-3 sum |qdot tau|
 * + 0.5 exp(-|q - q_default|^2) - done)) and done[e]
 * ([nenv][nworld], 1 when the root's z axis points downwards or the state is no longer
 * finite, with reward 0 then).  A world that is done
 * restarts from reset_qpos / reset_qvel ([nworld][nq] / [nworld][nv]) with a zero warm
 * start and previous action.  last_action ([nworld][nu]) holds the previous action on
 * entry and on return.  The bound state advances in place.
 *
 * params (optional, [nworld][8 + 2 nu]): each world's randomised parameters --
 * [0] contact friction scale, [1] payload mass added to the root body at its centre of
 * mass, [2..4] shift of the root body's centre of mass (root frame), [5] kp scale,
 * [6] kd scale, [7] unused, [8 + k] calibration offset of joint 6 + k (the PD law, the
 * observation and the pose term see q + offset), [8 + nu + k] armature of dof 6 + k.
 * The rows' regularisers keep the model's nominal inverse weights.  NULL: the model as
 * uploaded.  obs_noise (optional, [nenv][nworld][12 + 3 nu]) is added to obs.
 * Stream-ordered; MJH_EUNSUPPORTED for other models, and for params with implicit
 * damping. */
mjh_status mjh_env_step(mjh_batch* b, int32_t nenv, int32_t nsub, const float* action,
                        const float* command, const float* reset_qpos, const float* reset_qvel,
                        const float* params, const float* obs_noise, float* last_action,
                        float* obs, float* reward, int32_t* done, void* stream);

/* Capture mjh_step(b, nstep) into a HIP graph (replayed by mjh_graph_launch).  The
 * graph's kernel reads the groups' bound pointers from a device table at replay time;
 * mjh_bind_state / mjh_bind_io rewrite that table in place, so a rebound batch replays
 * its graph with the new buffers, no recapture.  mjh_set_launch and mjh_autotune change
 * the launch shape and drop the graph: mjh_graph_launch then fails with MJH_ESTATE until
 * the next capture. */
mjh_status mjh_graph_capture(mjh_batch* b, int32_t nstep, void* stream);
mjh_status mjh_graph_launch(mjh_batch* b, void* stream);

/* Time candidate launch shapes (lanes per world, worlds per work-group) for every
 * group on the bound state with nstep_probe steps, keep the fastest, and restore the
 * state afterwards (also when a probe fails).  cache_path (may be NULL) names a text
 * file of choices kept across processes, one line per group shape: the model's
 * dimensions and the group's world count, " : ", team, block.  A group found there is
 * not probed; the file is rewritten with every choice after a successful call. */
mjh_status mjh_autotune(mjh_batch* b, int32_t nstep_probe, const char* cache_path);
/* Force a launch shape for group g: team in {16, 32, 64} lanes, block in {64..1024}. */
mjh_status mjh_set_launch(mjh_batch* b, int32_t group, int32_t team, int32_t block);
mjh_status mjh_get_launch(mjh_batch* b, int32_t group, int32_t* team, int32_t* block);

/* Differentiable rollout of group 0 (single-model batch).
 * Loss: sum_{t=1..horizon} (qpos_t[zidx] - ztarget)^2 + wctrl * sum_t |ctrl_t|^2.
 * For a model without actuators (nu = 0) ctrl and grad_ctrl may be NULL.
 * mjh_rollout_fwd runs horizon steps from the bound state with ctrl [horizon][n][nu],
 * keeps a checkpoint every ckpt_every steps, writes loss [n] and leaves the bound
 * state at the final step.  The checkpoint tapes belong to the batch and hold one
 * rollout: *generation (may be NULL) receives that rollout's number.
 * mjh_rollout_bwd(generation, dloss [n]) writes grad_qvel0 [n][nv] and
 * grad_ctrl [horizon][n][nu] by the adjoint of the step: implicit differentiation at
 * each Newton solution, reverse sweeps of RNE/kinematics and contact geometry,
 * segments recomputed from the checkpoints.  It fails with MJH_ESTATE when
 * `generation` is not the number of the batch's last rollout_fwd (its tapes were
 * overwritten), and reads the ctrl buffer that rollout_fwd was given, which must be
 * unchanged.  Inside rollouts Newton iterates until max|grad| <= 1e-5 * max(1,
 * max|smooth force|), at most 16 iterations.  The contacts differentiated are those of
 * planes, spheres and capsules against spheres and capsules, self-contacts included,
 * of planes against box corners,
 * and of spheres against a heightfield fixed in the world, as pyramids of any contact
 * dimension (MJH_EUNSUPPORTED for other pairs and for elliptic cones); connect and weld
 * equalities; semi-implicit Euler, fourth-order Runge-Kutta (each step's four stages
 * reversed from an on-chip image per stage, four times the tape of an Euler step), and
 * the implicit integrators when nv is at most the group's team size (MJH_EUNSUPPORTED
 * otherwise). */
mjh_status mjh_rollout_fwd(mjh_batch* b, int32_t horizon, int32_t ckpt_every,
                           const float* ctrl, int32_t zidx, float ztarget, float wctrl,
                           float* loss, int64_t* generation, void* stream);
mjh_status mjh_rollout_bwd(mjh_batch* b, int64_t generation, const float* dloss,
                           float* grad_qvel0, float* grad_ctrl, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * training loops, harnesses that forbid hipMalloc): mjh_rollout_fwd followed by
 * mjh_rollout_bwd in one call, with the same arguments, kernels and results (loss [n],
 * grad_qvel0 [n][nv], grad_ctrl [horizon][n][nu], all caller-owned device memory; dloss
 * [n] is an input), the bound state left at the final step.  The tapes live in a static
 * device array of the library (64 MiB on every device it runs on, held until the process
 * ends) instead of the batch's own tapes, so this call allocates nothing; the batch's
 * pending rollout_fwd, if any, stays valid.  A rollout whose tapes need more than the
 * array -- ceil(horizon / ckpt_every) + min(ckpt_every, horizon) + 1 states of
 * nq + 2 nv floats plus min(ckpt_every, horizon) on-chip images per world -- fails with
 * MJH_EINVAL before launching anything (about 1 000 quadruped worlds at horizon 64 and a
 * checkpoint every 8 steps fit).  Every call on one device shares the array: two calls
 * that overlap on one device (two streams, two threads, two contexts) race and give
 * undefined results.  Same model restrictions as mjh_rollout_fwd. */
mjh_status mjh_rollout_noalloc(mjh_batch* b, int32_t horizon, int32_t ckpt_every,
                               const float* ctrl, int32_t zidx, float ztarget, float wctrl,
                               const float* dloss, float* loss, float* grad_qvel0,
                               float* grad_ctrl, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* MJH_H_ */
