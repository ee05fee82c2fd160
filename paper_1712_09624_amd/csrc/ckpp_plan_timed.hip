// ckpp_plan_timed.hip -- the plan kernel with timed passes (plans with
// tables with timers, Sec. 4.2), compiled apart from the untimed one.

#include "ckpp_plan_dev.h"

namespace ckpp {

hipError_t launch_plan_timed(const PlanArgs &A, bool two_buffers, const ckpp_plan_launch_t &L,
                             int num_cus, hipStream_t s) {
  return launch_plan_block<true>(A, two_buffers, L, num_cus, s);
}

}  // namespace ckpp
