// sacx_batch32.hip -- FP32 instantiation of the batched persistent launch
// (built with multiply-add contraction, like the FP32 stage kernel).
#include "sacx_batch_kernel.h"

namespace sacx {

template hipError_t launch_batch<float>(const BatchArgs<float> &, int, int, hipStream_t);
template hipError_t batch_blocks_per_cu<float>(int, int *);

}  // namespace sacx
