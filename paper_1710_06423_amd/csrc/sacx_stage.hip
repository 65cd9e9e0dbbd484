// sacx_stage.hip -- FP64 instantiation of the fused RK stage kernel (built
// with -ffp-contract=off: every operation rounds once, in the order of the
// scheme's defining sequence).
#include "sacx_stage_kernel.h"

namespace sacx {

template hipError_t launch_stage<double>(int, bool, bool, const StageArgs<double> &, hipStream_t);
template hipError_t stage_blocks_per_cu<double>(int, bool, bool, bool, int *);

}  // namespace sacx
