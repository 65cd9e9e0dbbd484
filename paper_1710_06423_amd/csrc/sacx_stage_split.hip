// sacx_stage_split.hip -- the two-role FP64 stage kernel (k_stage_split), in
// a unit of its own: built, like sacx_stage.hip, without contraction (every
// operation rounds once, in the scheme's order), and with LLVM's iterative
// ILP-maximising scheduler, which measured 2-3 % faster for this kernel and
// 3 % slower for the one-thread tile.
#include "sacx_stage_kernel.h"

namespace sacx {

namespace {

template <int NC, int STAGE>
hipError_t launch_split_s(bool bg, bool sur, dim3 grid, const StageArgs<double> &a, hipStream_t s) {
    if (sur) hipLaunchKernelGGL((k_stage_split<double, NC, STAGE, false, true>), grid, dim3(2 * NC), 0, s, a);
    else if (bg) hipLaunchKernelGGL((k_stage_split<double, NC, STAGE, true>), grid, dim3(2 * NC), 0, s, a);
    else hipLaunchKernelGGL((k_stage_split<double, NC, STAGE, false>), grid, dim3(2 * NC), 0, s, a);
    return hipGetLastError();
}

template <int NC>
hipError_t launch_split_nc(int stage, bool bg, bool sur, dim3 grid, const StageArgs<double> &a, hipStream_t s) {
    switch (stage) {
        case 1: return launch_split_s<NC, 1>(bg, sur, grid, a, s);
        case 2: return launch_split_s<NC, 2>(bg, sur, grid, a, s);
        case 3: return launch_split_s<NC, 3>(bg, sur, grid, a, s);
        default: return launch_split_s<NC, 4>(bg, sur, grid, a, s);
    }
}

template <int NC>
hipError_t split_blocks_nc(bool bg, int *blocks) {
    return bg ? hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_stage_split<double, NC, 1, true>, 2 * NC, 0)
              : hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_stage_split<double, NC, 1, false>, 2 * NC, 0);
}

}  // namespace

hipError_t launch_split_fp64(int stage, int nc, bool bg, bool sur, dim3 grid, const StageArgs<double> &a,
                             hipStream_t s) {
    switch (nc) {
        case 64: return launch_split_nc<64>(stage, bg, sur, grid, a, s);
        case 128: return launch_split_nc<128>(stage, bg, sur, grid, a, s);
        default: return launch_split_nc<256>(stage, bg, sur, grid, a, s);
    }
}

hipError_t split_blocks_per_cu_fp64(int nc, bool bg, int *blocks) {
    switch (nc) {
        case 64: return split_blocks_nc<64>(bg, blocks);
        case 128: return split_blocks_nc<128>(bg, blocks);
        default: return split_blocks_nc<256>(bg, blocks);
    }
}

}  // namespace sacx
