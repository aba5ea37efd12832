// 1-D stepper instantiations for 2 RK4 steps per kernel step (band P(Z)^2, radius 8).
#include "step1d_kernel.h"

namespace res {

int launch_step1d_m2(const Step1DArgs& a, hipStream_t st) { return launch_step1d_ms<2>(a, st); }
int step1d_coresident_m2(int fp64, int cfg, int device) { return step1d_coresident_ms<2>(fp64, cfg, device); }

}  // namespace res
