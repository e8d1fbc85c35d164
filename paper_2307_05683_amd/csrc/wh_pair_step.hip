// The pair layout's persistent step kernel (two planets per lane, wh_pair.h):
// wave w of the packing covers slots [128 w, 128 w + 128), lane l the slots
// 128 w + l and 128 w + 64 + l, each lane group one system of up to 2, 4 or
// 8 planets.  A translation unit of its own so that it can be compiled with
// the latency-first instruction schedule (build.py); everything it calls is
// in wh_step.h, shared with wh.hip, and the results do not depend on the
// schedule.
#include "wh_step.h"

namespace wh {

template <bool GR, int SCHEME, int KC>
__global__ __launch_bounds__(256) void k_step_pair(StepParams p) {
  const int lane = threadIdx.x & 63;
  int wave;
  if (!launch_wave(p, (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6), wave,
                   p.n_steps))
    return;
  const int sa = wave * 128 + lane;
  if (wave < p.w1) step_group_pair<1, GR, SCHEME, KC>(p, sa, lane);
  else if (wave < p.w2) step_group_pair<2, GR, SCHEME, KC>(p, sa, lane);
  else step_group_pair<4, GR, SCHEME, KC>(p, sa, lane);
}

template __global__ void k_step_pair<false, WH_DKD, 0>(StepParams);
template __global__ void k_step_pair<true, WH_DKD, 0>(StepParams);
template __global__ void k_step_pair<false, WH_KDK, 0>(StepParams);
template __global__ void k_step_pair<true, WH_KDK, 0>(StepParams);
template __global__ void k_step_pair<false, WH_DKD, 1>(StepParams);
template __global__ void k_step_pair<true, WH_DKD, 1>(StepParams);
template __global__ void k_step_pair<false, WH_KDK, 1>(StepParams);
template __global__ void k_step_pair<true, WH_KDK, 1>(StepParams);
template __global__ void k_step_pair<false, SCHEME_SABA, 0>(StepParams);

}  // namespace wh
