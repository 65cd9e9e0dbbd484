// sacx_stage_kernel.h -- the fused RK stage kernel and its launchers, as
// templates; each precision is instantiated in its own translation unit
// (sacx_stage.hip: FP64, built without contraction for bit-exact results,
// with the two-role FP64 tile in sacx_stage_split.hip; sacx_stage32.hip:
// FP32 bulk arithmetic).
#pragma once

#include <type_traits>

#include "sacx_tile.h"
#include "sacx_tile_split.h"

namespace sacx {

// The chip hands consecutive blocks of a launch to its 8 XCDs in turn (the
// linear block index modulo 8), each XCD with its own L2.  The blocks are
// renumbered so that tiles that are neighbours in row-major order run on one
// XCD and fetch the apron columns they share into one L2: RUN > 0 gives each
// XCD runs of RUN neighbouring tiles while the launch keeps its row-major
// progress (blocks past the last whole group of 8 runs keep their index);
// RUN == 0 gives each XCD one contiguous run of n/8 tiles.  Either is a
// bijection of the block indices, so every tile is still computed once.
// Measured at 8000^2 against no renumbering (two or three runs each): FP32
// tiles are 2.7 % (Orszag-Tang) and 3.9 % (stratified) faster with one
// contiguous run, and no faster with runs of 4; FP64 tiles are faster with
// runs of 4 (split tile 0.8 %, the tile without hyper-diffusion 2.8 %) and
// slower with one contiguous run (6 % and 4 %).  FP64 kernels take 4 and FP32
// kernels 0.
constexpr int kXcds = 8;

template <int RUN>
__device__ __forceinline__ void xcd_tile(int &tx, int &ty) {
    const int gx = (int)gridDim.x;
    const int n = gx * (int)gridDim.y;
    const int b = (int)blockIdx.x + (int)blockIdx.y * gx;
    const int x = b % kXcds, i = b / kXcds;
    int l;
    if (RUN == 0) {
        const int q = n / kXcds, r = n % kXcds;
        l = x < r ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
    } else {
        l = b < n - n % (kXcds * RUN) ? ((i / RUN) * kXcds + x) * RUN + i % RUN : b;
    }
    tx = l % gx;
    ty = l / gx;
}

// FP32 builds are held to two waves per SIMD (all but the background
// stage-4 build fit without the bound; that one would otherwise take one
// register too many and run one wave per SIMD at half speed)
template <typename real, int NT, int STAGE, bool HD, bool BG, bool SUR = false>
__global__ __launch_bounds__(NT, sizeof(real) == 4 ? 2 : 1) void k_stage(StageArgs<real> a) {
    __shared__ TileLds<real, NT> lds;
    int tx, ty;
    xcd_tile<sizeof(real) == 4 ? 0 : 4>(tx, ty);
    stage_tile<real, NT, STAGE, HD, BG, SUR>(a, tx, ty, lds);
}

// two threads per column (x and y roles), two waves per SIMD
template <typename real, int NC, int STAGE, bool BG, bool SUR = false>
__global__ __launch_bounds__(2 * NC, 2) void k_stage_split(StageArgs<real> a) {
    __shared__ SplitLds<real, NC, BG> lds;
    int tx, ty;
    xcd_tile<4>(tx, ty);
    stage_tile_split<real, NC, STAGE, BG, SUR>(a, tx, ty, lds);
}

template <typename real, int NT, int STAGE, bool HD>
__global__ __launch_bounds__(NT) void k_stage_1d(StageArgs<real> a) {
    __shared__ TileLds<real, NT> lds;
    stage_tile_1d<real, NT, STAGE, HD>(a, blockIdx.x, lds);
}

// The two-role FP64 tile is compiled in a unit of its own
// (sacx_stage_split.hip), with a scheduling strategy that suits it but not
// the one-thread tile: these launch and size its kernels there.
hipError_t launch_split_fp64(int stage, int nc, bool bg, bool sur, dim3 grid, const StageArgs<double> &a,
                             hipStream_t s);
hipError_t split_blocks_per_cu_fp64(int nc, bool bg, int *blocks);

template <typename real, int NT, int STAGE>
static hipError_t launch_s(bool hd, bool bg, const StageArgs<real> &a, hipStream_t s) {
    constexpr int TX = NT - 2 * G;
    if (a.L.ny == 1 && a.L.nx >= 2 && !bg) {
        dim3 grid((a.L.nx + TX - 1) / TX, 1);
        if (hd) hipLaunchKernelGGL((k_stage_1d<real, NT, STAGE, true>), grid, dim3(NT), 0, s, a);
        else hipLaunchKernelGGL((k_stage_1d<real, NT, STAGE, false>), grid, dim3(NT), 0, s, a);
        return hipGetLastError();
    }
    dim3 grid((a.L.nx + TX - 1) / TX, (a.L.ny + a.ty - 1) / a.ty);
    if constexpr (std::is_same<real, double>::value) {
        if (a.split && hd && !(a.Rs && bg)) return launch_split_fp64(STAGE, NT, bg, a.Rs != nullptr, grid, a, s);
    }
    if (a.Rs && hd && !bg) {
        hipLaunchKernelGGL((k_stage<real, NT, STAGE, true, false, true>), grid, dim3(NT), 0, s, a);
        return hipGetLastError();
    }
    if (hd && bg) hipLaunchKernelGGL((k_stage<real, NT, STAGE, true, true>), grid, dim3(NT), 0, s, a);
    else if (hd) hipLaunchKernelGGL((k_stage<real, NT, STAGE, true, false>), grid, dim3(NT), 0, s, a);
    else if (bg) hipLaunchKernelGGL((k_stage<real, NT, STAGE, false, true>), grid, dim3(NT), 0, s, a);
    else hipLaunchKernelGGL((k_stage<real, NT, STAGE, false, false>), grid, dim3(NT), 0, s, a);
    return hipGetLastError();
}

template <typename real, int NT>
static hipError_t launch_nt(int stage, bool hd, bool bg, const StageArgs<real> &a, hipStream_t s) {
    switch (stage) {
        case 1: return launch_s<real, NT, 1>(hd, bg, a, s);
        case 2: return launch_s<real, NT, 2>(hd, bg, a, s);
        case 3: return launch_s<real, NT, 3>(hd, bg, a, s);
        default: return launch_s<real, NT, 4>(hd, bg, a, s);
    }
}

// resident blocks per compute unit of the 2-D stage kernel a launch with these
// settings uses (stage 1; the four stages differ little in resources)
template <typename real, int NT>
static hipError_t blocks_per_cu_nt(bool hd, bool bg, bool split, int *blocks) {
    if constexpr (std::is_same<real, double>::value) {
        if (split && hd) return split_blocks_per_cu_fp64(NT, bg, blocks);
    }
    if (hd && bg) return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_stage<real, NT, 1, true, true>, NT, 0);
    if (hd) return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_stage<real, NT, 1, true, false>, NT, 0);
    if (bg) return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_stage<real, NT, 1, false, true>, NT, 0);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_stage<real, NT, 1, false, false>, NT, 0);
}

template <typename real>
hipError_t stage_blocks_per_cu(int nt, bool hd, bool bg, bool split, int *blocks) {
    switch (nt) {
        case 64: return blocks_per_cu_nt<real, 64>(hd, bg, split, blocks);
        case 128: return blocks_per_cu_nt<real, 128>(hd, bg, split, blocks);
        default: return blocks_per_cu_nt<real, 256>(hd, bg, split, blocks);
    }
}

template <typename real>
hipError_t launch_stage(int stage, bool hd, bool bg, const StageArgs<real> &a, hipStream_t s) {
    switch (a.nt) {
        case 64: return launch_nt<real, 64>(stage, hd, bg, a, s);
        case 128: return launch_nt<real, 128>(stage, hd, bg, a, s);
        default: return launch_nt<real, 256>(stage, hd, bg, a, s);
    }
}

}  // namespace sacx
