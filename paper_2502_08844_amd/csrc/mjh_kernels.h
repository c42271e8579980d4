// Kernel entry points shared between the kernel and host translation units.
#pragma once
#include <hip/hip_runtime.h>

#include "mjh_model.h"

namespace mjh {

constexpr int kMaxBlock = 256;  // threads per work-group of the step kernel

// LDS words of a work-group's triangular pair table (16-byte aligned)
__host__ __device__ inline int table_words(const DevModel& m) {
  return ((m.ntri + 3) / 4 + 3) & ~3;
}

// Launch the step kernel: one work-group of `block` threads per task; rk4 selects the
// instantiation that can run fourth-order Runge-Kutta groups, cone the one that can
// also solve elliptic-cone models.
hipError_t launch_step(const DevGroup* groups, const DevTask* tasks, int ntask, int nstep,
                       int block, size_t lds_bytes, int tab_words, bool rk4, bool cone,
                       hipStream_t stream);
// Allow the step kernel `bytes` of dynamic LDS per work-group.
hipError_t set_step_lds_limit(size_t bytes);
// Compute body_invweight of a freshly uploaded model (one work-group).
hipError_t launch_invweight(const DevModel& m, hipStream_t stream);

// Joystick environment steps of a single-group batch (the step kernel's tasks).
struct EnvArgs {
  int nenv, nsub, nobs;
  const float* action;      // [nenv][nworld][nu]
  const float* command;     // [nworld][3]
  const float* reset_qpos;  // [nworld][nq]
  const float* reset_qvel;  // [nworld][nv]
  float* last_action;       // [nworld][nu], read and updated
  float* obs;               // [nenv][nworld][nobs]
  float* reward;            // [nenv][nworld]
  int* done;                // [nenv][nworld]
  int ndr;                  // 8 + 2 nu with per-world parameters, else 0
  const float* dr;          // [nworld][ndr] or nullptr
  const float* noise;       // [nenv][nworld][nobs] or nullptr
};
// ap_words: LDS words after the pair table for the teams' previous actions
hipError_t launch_env(const DevGroup* groups, const DevTask* tasks, int ntask, const EnvArgs& E,
                      int block, size_t lds_bytes, int tab_words, int ap_words, bool rk4,
                      hipStream_t stream);
hipError_t set_env_lds_limit(size_t bytes);

}  // namespace mjh
