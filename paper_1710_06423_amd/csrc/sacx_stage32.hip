// sacx_stage32.hip -- FP32 instantiation of the fused RK stage kernel (FP32
// bulk arithmetic; dt, c_max and the conservation sums stay FP64).  Built
// with multiply-add contraction: this path is held to an error bound
// against the FP64 path, not to its bits.
#include "sacx_stage_kernel.h"

namespace sacx {

template hipError_t launch_stage<float>(int, bool, bool, const StageArgs<float> &, hipStream_t);
template hipError_t stage_blocks_per_cu<float>(int, bool, bool, bool, int *);

}  // namespace sacx
