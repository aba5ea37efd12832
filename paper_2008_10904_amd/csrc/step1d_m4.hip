// 1-D stepper instantiations for 4 RK4 steps per kernel step (band P(Z)^4, radius 16).
#include "step1d_kernel.h"

namespace res {

int launch_step1d_m4(const Step1DArgs& a, hipStream_t st) { return launch_step1d_ms<4>(a, st); }
int step1d_coresident_m4(int fp64, int cfg, int device) { return step1d_coresident_ms<4>(fp64, cfg, device); }

}  // namespace res
