// sacx_batch_kernel.h -- the batched persistent launch of many subdomains, as
// templates; each precision is instantiated in its own translation unit with
// the same floating-point contraction as that precision's stage kernel, so an
// instance evolves in a batch exactly as it does alone.
#pragma once

#include <hip/hip_cooperative_groups.h>

#include "sacx_tile.h"

namespace sacx {

// ---------------------------------------------------------------------------
// Batched persistent launch: every step of every instance in one cooperative
// launch (all blocks co-resident, which the runtime checks at launch).  Per
// step: each instance's dt from its own reduced wave speeds; then per stage a
// ghost fill of all instances' stage inputs, a grid barrier, all instances'
// tiles taken from a work queue (one atomic counter per step and stage,
// tiles ordered most expensive first), a grid barrier.  The tile arithmetic
// is the same device code as the per-subdomain kernels, so each instance
// evolves bit for bit as it does alone.
// ---------------------------------------------------------------------------
namespace cg = cooperative_groups;

__device__ __forceinline__ int bwrap(int i, int n, int periodic) {
    if (periodic) { int r = i % n; return r < 0 ? r + n : r; }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

template <typename real, int STAGE>
__device__ void batch_ghost_fill(const BatchArgs<real> &b, int n_blocks_threads, int gtid) {
    const long long total = b.gbeg[b.n];
    for (long long g = gtid; g < total; g += n_blocks_threads) {
        // instance by binary search over the prefix offsets
        int lo = 0, hi = b.n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (b.gbeg[mid] <= g) lo = mid; else hi = mid - 1;
        }
        const BatchInst<real> &I = b.inst[lo];
        const int nx = I.L.nx, ny = I.L.ny, W = nx + 2 * G;
        const long long gc = 2LL * G * W + 2LL * G * ny;   // ghost cells per field
        long long m = g - b.gbeg[lo];
        const int f = (int)(m / gc);
        m -= (long long)f * gc;
        int ci, rj;
        if (m < 2LL * G * W) {
            const int rr = (int)(m / W);
            ci = (int)(m % W) - G;
            rj = rr < G ? rr - G : ny + rr - G;
        } else {
            const long long m2 = m - 2LL * G * W;
            rj = (int)(m2 / (2 * G));
            const int cc = (int)(m2 % (2 * G));
            ci = cc < G ? cc - G : nx + cc - G;
        }
        real *S = const_cast<real *>(I.st[STAGE - 1].S[f]);
        const int si = bwrap(ci, nx, I.periodic_x), sj = bwrap(rj, ny, I.periodic_y);
        S[(int64_t)I.L.xoff + ci + (int64_t)(rj + G) * I.L.pitch] =
            S[(int64_t)I.L.xoff + si + (int64_t)(sj + G) * I.L.pitch];
    }
}

template <typename real, int NT, int STAGE>
__device__ void batch_stage(const BatchArgs<real> &b, int step, TileLds<real, NT> &lds, int &s_item,
                            cg::grid_group &grid) {
    batch_ghost_fill<real, STAGE>(b, (int)(gridDim.x * NT), (int)(blockIdx.x * NT + threadIdx.x));
    grid.sync();
    int *ctr = b.ctr + step * 4 + (STAGE - 1);
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = atomicAdd(ctr, 1);
        __syncthreads();
        const int it = s_item;
        if (it >= b.nitems) break;
        const BatchItem w = b.items[it];
        const BatchInst<real> &I = b.inst[w.inst];
        if (I.oned) stage_tile_1d<real, NT, STAGE, true>(I.st[STAGE - 1], w.tx, lds);
        else stage_tile<real, NT, STAGE, true, false>(I.st[STAGE - 1], w.tx, w.ty, lds);
    }
    grid.sync();
}

template <typename real, int NT>
__global__ __launch_bounds__(NT, sizeof(real) == 4 ? 2 : 1) void k_batch(BatchArgs<real> b) {
    __shared__ TileLds<real, NT> lds;
    __shared__ int s_item;
    cg::grid_group grid = cg::this_grid();
    for (int step = 0; step < b.nsteps; ++step) {
        if (blockIdx.x == 0)
            for (int i = threadIdx.x; i < b.n; i += NT) step_begin_dev(b.inst[i].sc, 0.0, b.inst[i].sk);
        grid.sync();
        batch_stage<real, NT, 1>(b, step, lds, s_item, grid);
        batch_stage<real, NT, 2>(b, step, lds, s_item, grid);
        batch_stage<real, NT, 3>(b, step, lds, s_item, grid);
        batch_stage<real, NT, 4>(b, step, lds, s_item, grid);
        if (blockIdx.x == 0)
            for (int i = threadIdx.x; i < b.n; i += NT) step_end_dev(b.inst[i].sc);
        grid.sync();
    }
}

template <typename real, int NT>
static hipError_t launch_batch_nt(const BatchArgs<real> &b, int blocks, hipStream_t s) {
    void *args[] = {(void *)&b};
    return hipLaunchCooperativeKernel((const void *)k_batch<real, NT>, dim3(blocks), dim3(NT), args, 0, s);
}

template <typename real>
hipError_t launch_batch(const BatchArgs<real> &b, int nt, int blocks, hipStream_t s) {
    switch (nt) {
        case 64: return launch_batch_nt<real, 64>(b, blocks, s);
        case 128: return launch_batch_nt<real, 128>(b, blocks, s);
        default: return launch_batch_nt<real, 256>(b, blocks, s);
    }
}

template <typename real>
hipError_t batch_blocks_per_cu(int nt, int *blocks) {
    switch (nt) {
        case 64: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_batch<real, 64>, 64, 0);
        case 128: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_batch<real, 128>, 128, 0);
        default: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_batch<real, 256>, 256, 0);
    }
}

}  // namespace sacx
