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

// Forward and reverse sweeps of one rollout in a single call, with the tapes in the
// library's static device scratch (no device allocation).  The scratch holds
// kNoAllocScratchBytes per device; MJH_EINVAL when the rollout's tapes need more.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
// Look up the scratch's device address on `device` (which must be current); once per
// device, later calls return at once.
hipError_t noalloc_scratch_init(int device);
// Bytes of tape a rollout of nworld worlds, horizon steps, a checkpoint every ckpt needs.
size_t noalloc_tape_bytes(const DevModel& m, int nworld, int horizon, int ckpt);
mjh_status adjoint_noalloc(int device, const DevModel& m, int team, int nworld, float* qpos,
                           float* qvel, float* qacc, int horizon, int ckpt_every,
                           const float* ctrl, int zidx, float ztarget, float wctrl,
                           const float* dloss, float* loss, float* grad_qvel0, float* grad_ctrl,
                           hipStream_t stream, std::string& err);

}  // namespace mjh
