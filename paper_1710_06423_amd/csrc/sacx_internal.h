// sacx_internal.h -- device-side layout, scalar block and kernel launchers
// shared by the HIP translation units of libsacx (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sacx.h"

namespace sacx {

constexpr int G = SACX_GHOST;  // ghost cells per side
constexpr int NF = 6;          // evolved fields
constexpr int NBG = 4;         // background fields

// Field storage: one 2-D array per field, (ny + 2G) rows of `pitch` elements.
// Interior element (i, j), i in [-G, nx+G), j in [-G, ny+G), lives at
//   base[xoff + i + (j + G) * pitch]
// xoff is 256 bytes worth of elements so that interior column 0 of every row
// starts on a 256-byte boundary (coalesced, aligned row loads).
struct Layout {
    int nx, ny;
    int pitch;   // elements per row
    int xoff;    // element offset of column 0 within a row
    int rows;    // ny + 2G
    int64_t field_elems;  // elements per field array (rows * pitch, rounded)
};

// Device-resident step scalars.  c accumulators hold the IEEE bit patterns of
// non-negative doubles, so an unsigned 64-bit max is the floating max.
struct DevScalars {
    double t;            // current time
    double dt;           // time step of the step in progress / last taken
    double cmax;         // c_max used by the step in progress
    double t_end;        // end time of the current advance call (<= 0: none)
    // per-step constants derived from dt and c_max (computed once, read by
    // every stage kernel as uniform values)
    double hdt, dt6;     // dt/2, dt/6
    double kx2[4], ky2[4];  // c2 * h_d * c_max per constant class
    unsigned long long cacc[2][2];  // [slot][x, y] wave-speed maxima
    double last_cx, last_cy, last_cmax;
    long long steps;     // steps since init
    int cur;             // slot holding the maxima of the current state
    int active;          // 1 while the step in progress proceeds
    int nonphys;         // sticky: a non-physical state was reduced
    int pad;
};

// grid constants of the scheme, computed once on the host in FP64
// (reciprocals of grid spacings, closure constants, compression-term scales)
struct SchemeConsts {
    double gamma, gm1, igm1;
    double i12dx, i12dy, idx, idy, i2dx, i2dy;
    double kxs[4], kys[4];   // cshk * h_d * h_d
    double third;
};

template <typename real>
struct StageArgs {
    const real *S[NF];    // stage input (differenced; ghosts filled)
    const real *U[NF];    // step start state (pointwise)
    const real *A[NF];    // RK accumulator (pointwise, stage 4)
    real *out1[NF];       // stage output (w1, w2, w3 or the new state)
    real *out2[NF];       // accumulator output (stage 2)
    const real *BG[NBG];  // static background (optional)
    Layout L;
    int ty;               // output rows per block
    int nt;               // threads per block (one column each)
    SchemeConsts k;
    int hd_cross_on;
    DevScalars *sc;
};

// host-side launchers (defined in the .hip units)
template <typename real>
hipError_t launch_stage(int stage, bool hd, bool bg, const StageArgs<real> &a, hipStream_t s);

}  // namespace sacx
