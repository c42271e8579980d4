// Differentiable rollout (checkpointed forward, reverse sweep).
#include "mjh_adjoint.h"

namespace mjh {

struct AdjointState {
  int dummy = 0;
};

mjh_status adjoint_forward(AdjointState**, const DevModel&, int, float*, float*, float*, int,
                           int, const float*, int, float, float, float*, hipStream_t,
                           std::string& err) {
  err = "rollout_fwd: not available in this build";
  return MJH_EUNSUPPORTED;
}

mjh_status adjoint_backward(AdjointState*, const float*, float*, float*, hipStream_t,
                            std::string& err) {
  err = "rollout_bwd: not available in this build";
  return MJH_EUNSUPPORTED;
}

void adjoint_free(AdjointState* st) { delete st; }

}  // namespace mjh
