// sacx_batch.hip -- FP64 instantiation of the batched persistent launch (built
// without contraction, like the FP64 stage kernel).
#include "sacx_batch_kernel.h"

namespace sacx {

template hipError_t launch_batch<double>(const BatchArgs<double> &, int, int, hipStream_t);
template hipError_t batch_blocks_per_cu<double>(int, int *);

}  // namespace sacx
