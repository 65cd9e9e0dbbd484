// sacx_batch_kernel.h -- the batched persistent launch of many subdomains, as
// templates; each precision is instantiated in its own translation unit with
// the same floating-point contraction as that precision's stage kernel, so an
// instance evolves in a batch exactly as it does alone.
#pragma once

#include <hip/hip_cooperative_groups.h>

#include "sacx_tile.h"

namespace sacx {

// ---------------------------------------------------------------------------
// Batched persistent launch: every step of every instance in one launch with
// all blocks resident (a cooperative launch, which the runtime checks).
//
// The instances are split into one group per XCD (balanced by cost on the
// host), and each group's work is one queue taken in order through its own
// counter by the blocks of that XCD (a block reads the XCD it runs on from
// the XCC_ID hardware register).  A queue's entries are, for each global
// stage g = 4 step + (stage - 1) of the launch, its per-stage list: instance
// by instance (most expensive first) the F_i pieces of the ghost fill of the
// instance's stage input (a fill by one block would hold up the instance's
// tiles for hundreds of microseconds), then its tiles (most expensive
// first); after the last stage, one entry per instance closes its last step.
// Each instance keeps two completion counters, and an entry waits only for
// its own instance:
//   fill piece (i, g): all tiles of (i, g - 1) done -> tiles[i] >= T_i g
//                 (piece 0 of a step's first stage also ends the previous
//                 step and computes this step's dt from the instance's own
//                 reduced wave speeds)
//   tile  (i, g): the fill of (i, g) done           -> fills[i] >= F_i (g + 1)
// so an instance's next stage starts as soon as its own tiles are done,
// while other instances are still in their previous stage: no grid barrier,
// and no partly filled round of tiles before one.  Every dependency points
// to an earlier entry of the same queue and every block is resident, so
// some block can always proceed.
//
// Everything an instance reads and writes during the launch stays in one
// XCD, whose L2 every block of the queue shares: a finished entry's waves
// wait for their stores to reach L2, then one thread increments the counter
// (an L2 atomic); a waiting thread polls the counter in L2, and after it
// every wave acquires at agent scope, which invalidates its compute unit's
// L1, before reading the instance's data.  (Kernel boundaries make the data
// visible to the other XCDs and the host.)  No L2 write-back is needed per
// entry.
//
// Every wait is bounded (spin_limit polls): one that exceeds it raises the
// abort flag, every block leaves its queue, and the host reports the error;
// so does a queue with work whose XCD has no block of the launch.  The tile
// arithmetic is the device code of the per-subdomain kernels, so each
// instance evolves bit for bit as it does alone.
// ---------------------------------------------------------------------------

__device__ __forceinline__ int bwrap(int i, int n, int periodic) {
    if (periodic) { int r = i % n; return r < 0 ? r + n : r; }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// one piece of the ghost fill of an instance's stage input, by one block:
// periodic images or zero-gradient copies of cells (every source is a cell,
// corners included); the pieces split the instance's ghost cells evenly.
// A tube (one row) fills only the ghost cells of its row: its tile reads
// nothing else.
template <typename real, int NT>
__device__ void batch_inst_fill(const BatchInst<real> &I, int stage, int piece) {
    const int nx = I.L.nx, ny = I.L.ny, W = nx + 2 * G;
    const int gy = I.oned ? 0 : 2 * G * W;   // ghost cells of the rows above and below, per field
    const int gc = gy + 2 * G * ny;          // ghost cells per field
    const int g0 = piece * kBatchFillPiece, g1 = min(NF * gc, g0 + kBatchFillPiece);
    for (int g = g0 + (int)threadIdx.x; g < g1; g += NT) {
        const int f = g / gc;
        const int m = g - f * gc;
        int ci, rj;
        if (m < gy) {
            const int rr = m / W;
            ci = m % W - G;
            rj = rr < G ? rr - G : ny + rr - G;
        } else {
            const int m2 = m - gy;
            rj = m2 / (2 * G);
            const int cc = m2 % (2 * G);
            ci = cc < G ? cc - G : nx + cc - G;
        }
        real *S = const_cast<real *>(I.st[stage - 1].S[f]);
        const int si = bwrap(ci, nx, I.periodic_x), sj = bwrap(rj, ny, I.periodic_y);
        S[(int64_t)I.L.xoff + ci + (int64_t)(rj + G) * I.L.pitch] =
            S[(int64_t)I.L.xoff + si + (int64_t)(sj + G) * I.L.pitch];
    }
}

// wait (one thread) until the L2 counter *p >= target; 0 if the wait was abandoned
__device__ __forceinline__ int batch_wait(int *p, int target, int *abort_flag, int spin_limit) {
    int spins = 0;
    while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return 0;
        if (++spins > spin_limit) {
            __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return 0;
        }
        __builtin_amdgcn_s_sleep(8);
    }
    return 1;
}

template <typename real, int NT>
__device__ __forceinline__ void batch_tile(const BatchInst<real> &I, const BatchItem &w, int stage,
                                           TileLds<real, NT> &lds) {
    if (I.oned) {
        switch (stage) {
            case 1: stage_tile_1d<real, NT, 1, true>(I.st[0], w.tx, lds); break;
            case 2: stage_tile_1d<real, NT, 2, true>(I.st[1], w.tx, lds); break;
            case 3: stage_tile_1d<real, NT, 3, true>(I.st[2], w.tx, lds); break;
            default: stage_tile_1d<real, NT, 4, true>(I.st[3], w.tx, lds); break;
        }
    } else {
        switch (stage) {
            case 1: stage_tile<real, NT, 1, true, false>(I.st[0], w.tx, w.ty, lds); break;
            case 2: stage_tile<real, NT, 2, true, false>(I.st[1], w.tx, w.ty, lds); break;
            case 3: stage_tile<real, NT, 3, true, false>(I.st[2], w.tx, w.ty, lds); break;
            default: stage_tile<real, NT, 4, true, false>(I.st[3], w.tx, w.ty, lds); break;
        }
    }
}

template <typename real, int NT>
__global__ __launch_bounds__(NT, sizeof(real) == 4 ? 2 : 1) void k_batch(BatchArgs<real> b) {
    __shared__ TileLds<real, NT> lds;
    __shared__ int s_item, s_ok;
    int *const abort_flag = b.sync + BATCH_ABORT;
    int *const fills = b.sync + BATCH_SYNC0;
    int *const tiles = b.sync + BATCH_SYNC0 + b.n;
    unsigned xcc;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID, 0, 4)" : "=s"(xcc));
    const int x = (int)xcc;
    // every queue with work needs a block on its XCD
    if (threadIdx.x == 0) {
        if (x < kBatchQueues) atomicAdd(b.sync + BATCH_BLOCKS0 + x, 1);
        else __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    cooperative_groups::this_grid().sync();
    if (threadIdx.x == 0) {
        int ok = __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
        for (int k = 0; k < kBatchQueues; ++k)
            if (b.qlen[k] > 0 && __hip_atomic_load(b.sync + BATCH_BLOCKS0 + k, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT) == 0)
                ok = 0;
        if (!ok) __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_ok = ok;
    }
    __syncthreads();
    if (!s_ok) return;
    int *const queue = b.sync + BATCH_QUEUE0 + x;
    const int qlen = b.qlen[x];
    const int body = b.nsteps * 4 * qlen;   // entries before the closing ones
    const int total = body + (b.ioff[x + 1] - b.ioff[x]);
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(queue, 1);
        __syncthreads();
        const int q = s_item;
        if (q >= total) break;
        int g, inst, kind;
        BatchItem w{0, 0, 0, 0};
        if (q < body) {
            g = q / qlen;
            w = b.items[b.qoff[x] + q - g * qlen];
            inst = w.inst;
            kind = w.kind;
        } else {
            g = 4 * b.nsteps;
            inst = b.qinst[b.ioff[x] + q - body];
            kind = -1;   // closes the instance's last step
        }
        const BatchInst<real> &I = b.inst[inst];
        if (threadIdx.x == 0)
            s_ok = kind == BATCH_TILE ? batch_wait(fills + inst, I.nfill * (g + 1), abort_flag, b.spin_limit)
                                      : batch_wait(tiles + inst, I.ntiles * g, abort_flag, b.spin_limit);
        __syncthreads();
        if (!s_ok) break;
        // this compute unit's L1 may hold lines of the instance from before
        // the entries just waited for: every wave acquires at agent scope,
        // which invalidates the L1 (a workgroup-scope invalidate does not:
        // all of a workgroup's waves share one L1)
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const int stage = (g & 3) + 1;
        if (kind == BATCH_TILE) {
            batch_tile<real, NT>(I, w, stage, lds);
        } else if (kind == BATCH_FILL) {
            if (stage == 1 && w.tx == 0 && threadIdx.x == 0) {
                if (g > 0) step_end_dev(I.sc);
                step_begin_dev(I.sc, 0.0, I.sk);
            }
            batch_inst_fill<real, NT>(I, stage, w.tx);
        } else if (threadIdx.x == 0) {
            step_end_dev(I.sc);
        }
        // every wave's stores of the entry have reached L2 (the block barrier
        // alone does not wait for them), then one thread publishes the entry
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
        if (threadIdx.x == 0 && kind >= 0)
            __hip_atomic_fetch_add(kind == BATCH_TILE ? tiles + inst : fills + inst, 1, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
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
