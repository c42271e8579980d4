// Differentiable rollout: checkpointed forward and reverse sweeps.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/mjh.h"
#include "mjh_model.h"

namespace mjh {

struct AdjointState;

// Run `horizon` steps of `nworld` worlds from the bound state, storing checkpoints
// every ckpt_every steps, accumulate the loss per world.  *generation (may be NULL)
// receives the rollout's number, which adjoint_backward must be given.
mjh_status adjoint_forward(AdjointState** st, const DevModel& m, int team, int nworld, float* qpos,
                           float* qvel, float* qacc, int horizon, int ckpt_every,
                           const float* ctrl, int zidx, float ztarget, float wctrl,
                           float* loss, int64_t* generation, hipStream_t stream,
                           std::string& err);
// Reverse sweep of the last forward rollout; MJH_ESTATE unless `generation` is its number.
mjh_status adjoint_backward(AdjointState* st, int64_t generation, const float* dloss,
                            float* grad_qvel0, float* grad_ctrl, hipStream_t stream,
                            std::string& err);
void adjoint_free(AdjointState* st);

}  // namespace mjh
