// sacx_internal.h -- device-side layout, scalar block and kernel launchers
// shared by the HIP translation units of libsacx (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sacx.h"

namespace sacx {

// records the calling thread's last-error message and returns `code`
int set_error(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));

#define HIPCHK(expr)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return ::sacx::set_error(SACX_EDEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                                     __FILE__, __LINE__);                                  \
    } while (0)

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
    double gx, gy;           // gravity
    int grav;                // gravity non-zero: its sources are added
};

// constants of the time-step computation
struct StepConsts {
    double cfl, dx, dy;
    double c2[4];
    int ax, ay;  // direction has more than one cell
};

// dt for the step about to start: CFL time step from the reduced wave speeds
// with the end-time clamp, and the per-step constants derived from it
__device__ inline void step_begin_dev(DevScalars *sc, double t_end, const StepConsts &k) {
    sc->t_end = t_end;
    if (sc->nonphys) { sc->active = 0; return; }
    const double t = sc->t;
    if (t_end > 0.0 && t_end - t <= 1e-12 * t_end) { sc->active = 0; return; }
    const double cx = __longlong_as_double((long long)sc->cacc[sc->cur][0]);
    const double cy = __longlong_as_double((long long)sc->cacc[sc->cur][1]);
    const double dx = k.dx, dy = k.dy;
    double h;
    if (k.ax && k.ay) h = (dx / cx < dy / cy) ? dx / cx : dy / cy;
    else if (k.ax) h = dx / cx;
    else h = dy / cy;
    double dt = k.cfl * h;
    if (t_end > 0.0) dt = (dt < t_end - t) ? dt : t_end - t;
    sc->dt = dt;
    sc->cmax = (k.ax && k.ay) ? (cx > cy ? cx : cy) : (k.ax ? cx : cy);
    sc->last_cx = cx;
    sc->last_cy = cy;
    sc->last_cmax = sc->cmax;
    sc->hdt = 0.5 * dt;
    sc->dt6 = dt / 6.0;
    for (int m = 0; m < 4; ++m) {
        sc->kx2[m] = k.c2[m] * dx * sc->cmax;
        sc->ky2[m] = k.c2[m] * dy * sc->cmax;
    }
    sc->cacc[sc->cur ^ 1][0] = 0ull;
    sc->cacc[sc->cur ^ 1][1] = 0ull;
    sc->active = 1;
}

__device__ inline void step_end_dev(DevScalars *sc) {
    if (!sc->active) return;
    sc->t = sc->t + sc->dt;
    sc->steps = sc->steps + 1;
    sc->cur ^= 1;
}

template <typename real>
struct StageArgs {
    const real *S[NF];    // stage input (differenced; ghosts filled)
    const real *U[NF];    // step start state (pointwise)
    const real *A[NF];    // RK accumulator (pointwise, stage 4)
    real *out1[NF];       // stage output (w1, w2, w3 or the new state)
    real *out2[NF];       // accumulator output (stage 2)
    const real *BG[NBG];  // static background (optional)
    // elements from one field to the next in every buffer above (the stage
    // kernel addresses field f of a buffer as its field 0 + f * fstride;
    // the host checks that the buffers are laid out that way)
    int64_t fstride;
    Layout L;
    int ty;               // output rows per block
    int nt;               // columns per block (apron included)
    int split;            // FP64 2-D hyper-diffusion tiles without background:
                          // two threads per column (x and y roles)
    SchemeConsts k;
    int hd_cross_on;
    DevScalars *sc;
    // surrogate ratio planes (10: x-face sets then y-face sets, interior
    // cells, periodic): a value >= 0 replaces the plain coefficient ratio of
    // that face, a negative value keeps the plain ratio
    const float *Rs;
    int64_t rs_plane;     // elements per plane
    int rs_pitch;         // elements per row
    // per check tile (row-major, rs_ntx tiles of rs_tile x rs_tile cells per
    // row): 1 where the last check kept the prediction, 0 where it fell back;
    // the planes of a fallen-back tile are not read (its faces take the plain
    // ratio, as its planes' -1 would give)
    const unsigned char *Rk;
    int rs_tile, rs_ntx;
};

// arguments of the ratio-field kernels (plain ratios of a state whose halo is
// filled; no background)
template <typename real>
struct RatioArgs {
    const real *S[NF];
    Layout L;
    double gm1, igm1;
};

// device-side surrogate counters.  A check's blocks update one of kStatSlots
// copies of each counter (by block index), so that thousands of blocks do
// not contend for one word; the reader reduces the copies.
constexpr int kStatSlots = 64;
struct HdDevStats {
    unsigned long long tiles_fallback[kStatSlots];
    unsigned long long err_used[kStatSlots];   // IEEE bits of a non-negative double (max)
    unsigned long long err_all[kStatSlots];
    unsigned long long dmax[10];   // per plane max |first difference| of the current check
};

// round to the nearest BF16 value, ties to even (NaN stays a quiet NaN)
__device__ __forceinline__ unsigned short bf16_rne(float f) {
    unsigned u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

// ---------------------------------------------------------------- batches
// One instance of a batch: its per-stage kernel arguments, time-step
// constants and ghost-fill description.
template <typename real>
struct BatchInst {
    StageArgs<real> st[4];   // arguments of stages 1..4 (stage inputs, outputs)
    StepConsts sk;
    DevScalars *sc;
    Layout L;
    int periodic_x, periodic_y;
    int oned;                // ny == 1: one-dimensional tiles
    int ntiles;              // tiles of one stage
    int nfill;               // ghost-fill pieces of one stage
    int pad;
};

// ghost cells (all fields) per ghost-fill piece of a batched instance
constexpr int kBatchFillPiece = 2048;

// an entry of the per-stage work list: one piece (tx) of the ghost fill of an
// instance's stage input (kind BATCH_FILL; piece 0 of a step's first stage
// also takes the step's time step) or one tile of its stage (kind BATCH_TILE)
enum { BATCH_TILE = 0, BATCH_FILL = 1 };
struct BatchItem {
    int inst, tx, ty, kind;
};

// The batch's work is split into one queue per XCD (instances assigned to
// queues by cost); a block serves the queue of the XCD it runs on.
constexpr int kBatchQueues = 8;

// Batch synchronisation words: the abort flag of a dependency wait that
// exceeded its bound (sticky), per queue its work counter and the count of
// blocks serving it, then per instance the count of completed ghost fills and
// of completed tiles.  All but the abort flag are zeroed before every launch.
enum { BATCH_ABORT = 0, BATCH_QUEUE0 = 1, BATCH_BLOCKS0 = 1 + kBatchQueues, BATCH_SYNC0 = 1 + 2 * kBatchQueues };

template <typename real>
struct BatchArgs {
    const BatchInst<real> *inst;
    int n;
    const BatchItem *items;  // per queue one stage's work list (per instance its fill, then its tiles), queue after queue
    const int *qinst;        // the instances of each queue, queue after queue
    int qoff[kBatchQueues];  // first entry of each queue's list in items
    int qlen[kBatchQueues];  // entries of each queue's list
    int ioff[kBatchQueues + 1];  // prefix offsets of the queues' instances in qinst
    int *sync;               // BATCH_SYNC0 + 2 n words
    int nsteps;
    int spin_limit;          // bound of a dependency wait (polls)
};

// host-side launchers (defined in the .hip units)
template <typename real>
hipError_t launch_stage(int stage, bool hd, bool bg, const StageArgs<real> &a, hipStream_t s);
template <typename real>
hipError_t stage_blocks_per_cu(int nt, bool hd, bool bg, bool split, int *blocks);
template <typename real>
hipError_t launch_ratio_fields(const RatioArgs<real> &a, float *out, float *d1, int64_t pitch, hipStream_t s);
template <typename real>
hipError_t launch_hd_check(const RatioArgs<real> &a, float *rs, int64_t pitch, double bound, int tile, int metric,
                           HdDevStats *st, unsigned char *kept, hipStream_t s);
struct InputNorm {
    float v[12];   // shift[6], scale[6]
};
template <typename real>
hipError_t launch_cnn_inputs(const RatioArgs<real> &a, const InputNorm &norm, void *x, hipStream_t s);
hipError_t cnn_forward_dev(const void *packed, const void *x, int n, int h, int w, void *a1, void *a2, void *a3,
                           float *out, int64_t oimg, int64_t oplane, int64_t orow, hipStream_t s);
template <typename real>
hipError_t launch_batch(const BatchArgs<real> &b, int nt, int blocks, hipStream_t s);
template <typename real>
hipError_t batch_blocks_per_cu(int nt, int *blocks);

}  // namespace sacx
