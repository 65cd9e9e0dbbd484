/*
 * sacx.h -- C ABI of libsacx: the data-parallel hot path of the Sheffield
 * Advanced Code (SAC / SMAUG+) MHD scheme on one MI355X (gfx950) GPU.
 *
 * What the library computes (paper section 2): the ideal compressible MHD
 * equations in conservative form for background + perturbation split
 * variables, spatial derivatives by fourth-order central differences,
 * hyper-diffusion / hyper-viscosity / hyper-resistivity shock capturing whose
 * coefficient is the ratio of third- to first-order differences scaled by the
 * maximum wave speed (plus a compression term), classic fourth-order
 * Runge-Kutta in time with a CFL time step.  One context is one GPU's
 * subdomain; its halo ("ghost") layers are exchanged through device-side
 * pack/unpack buffers (paper section 3, the halo exchange of Fig. 1 and the
 * exchange_halo listing), with periodic self-exchange or open
 * (zero-gradient) boundaries applied locally.
 *
 * Conventions shared by every call
 *  - Grid: cell centred, x_i = x0 + (i + 1/2) dx, dx = (x1 - x0) / nx (same
 *    in y).  A 1-D problem has ny = 1 (or nx = 1); that direction must be
 *    periodic and all its differences vanish.
 *  - Evolved fields (the ABI unit, conserved variables), in this order:
 *      0 rho~  density perturbation        3 e~   total energy perturbation
 *      1 m_x   momentum x                  4 B~_x field perturbation x
 *      2 m_y   momentum y                  5 B~_y field perturbation y
 *    Optional static background, in this order: rho_b, e_b, B_bx, B_by.
 *  - Caller arrays are row-major (ny rows of nx values, x fastest) with a row
 *    pitch given in ELEMENTS (pitch >= nx); device pointers unless stated.
 *  - Boundary sides: 0 = x-, 1 = x+, 2 = y-, 3 = y+.
 *  - Every call returns an int status: SACX_OK (0) or a negative code.
 *    Nothing is thrown or aborted across the ABI.  Asynchronous device faults
 *    surface at the next synchronising call as SACX_EDEVICE.
 *  - A context is bound to the device current at sacx_create and to one
 *    stream; it is not thread-safe.  All device work of a context is enqueued
 *    on that stream in call order.
 *  - The library never allocates or frees device memory: all device storage
 *    is the caller-owned workspace given to sacx_create, which must stay
 *    valid and untouched until sacx_destroy.
 */
#ifndef SACX_H
#define SACX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SACX_ABI_VERSION 1

/* status codes */
#define SACX_OK 0
#define SACX_EINVAL (-1)   /* bad argument */
#define SACX_ENOSPC (-2)   /* workspace (or caller buffer) too small */
#define SACX_EDEVICE (-3)  /* HIP runtime error */
#define SACX_ENONPHYS (-4) /* a step start found rho <= 0, p <= 0 or a non-finite value */
#define SACX_EUNSUP (-5)   /* valid but unsupported request */
#define SACX_ESTATE (-6)   /* call out of order (e.g. advance before init_state) */

/* boundary kinds */
#define SACX_PERIODIC 0
#define SACX_OPEN 1

/* precisions */
#define SACX_FP64 0
#define SACX_FP32 1

/* number of ghost cells on every side (the hyper-diffusion stencil reaches 3 cells) */
#define SACX_GHOST 3

typedef struct sacx_grid {
    int32_t nx, ny;          /* interior cells of this subdomain */
    double x0, x1, y0, y1;   /* physical extent of this subdomain */
    int32_t precision;       /* SACX_FP64 or SACX_FP32: storage and bulk arithmetic;
                                time step and conservation sums are always FP64 */
    int32_t background_on;   /* 1: static background arrays are present */
} sacx_grid;

typedef struct sacx_params {
    double gamma;            /* adiabatic index (> 1) */
    double cfl;              /* dt = cfl * min_d h_d / max(|v_d| + c_f) */
    int32_t hd_on;           /* hyper-diffusion on/off (paper section 2; Table 1 "with/without HD") */
    int32_t hd_cross_on;     /* include off-diagonal stress / e.m.f. terms */
    double c2[4];            /* ratio-term constants: density, thermal energy, velocity, field */
    double cshk[4];          /* compression-term constants, same classes */
} sacx_params;

typedef struct sacx_diag {
    double t;                /* current time */
    double dt;               /* time step of the last step taken */
    double c_x, c_y, c_max;  /* max(|v_d| + c_f) of the current state */
    double sums[6];          /* sum over the interior of each evolved field times dx dy (FP64) */
    int64_t steps;           /* steps taken since sacx_init_state */
    int32_t nonphys;         /* 1 if the current state is non-physical */
} sacx_diag;

typedef struct sacx_ctx sacx_ctx;

/* ABI version (SACX_ABI_VERSION of the built library). */
int sacx_abi_version(void);

/* Static, library-owned description of a status code. */
const char *sacx_strerror(int code);

/* Library-owned description of the last error raised on the calling thread
 * (empty string if none). Valid until the next failing call on that thread. */
const char *sacx_last_error(void);

/* Bytes of device workspace a context with this grid/params needs.
 * Pure host arithmetic (no device call).  EINVAL on an invalid grid/params. */
int sacx_workspace_size(const sacx_grid *grid, const sacx_params *params, size_t *bytes);

/* Create a context on the current device.
 *  d_ws / ws_bytes : caller-owned device memory, >= sacx_workspace_size, 256-byte aligned;
 *                    it must outlive the context (ENOSPC if too small).
 *  hip_stream      : hipStream_t to enqueue on (NULL = the null stream).
 *  out             : receives a library-owned handle, released by sacx_destroy.
 * All four boundaries start PERIODIC. */
int sacx_create(const sacx_grid *grid, const sacx_params *params, void *d_ws, size_t ws_bytes,
                void *hip_stream, sacx_ctx **out);

/* Release a context (does not touch the workspace memory). NULL is a no-op. */
int sacx_destroy(sacx_ctx *ctx);

/* Set the boundary kind of each side (paper section 5: periodic for
 * Orszag-Tang; open for the shock tube).  Periodic sides must come in pairs
 * (x-, x+ and y-, y+), else EINVAL.  A direction with one cell must be
 * periodic.  Takes effect at the next halo fill. */
int sacx_set_boundaries(sacx_ctx *ctx, const int32_t bc[4]);

/* Load a state (paper section 3: the initial model configuration a process
 * receives).  d_fields: 6 device pointers (field order above), d_bg: 4 device
 * pointers or NULL (required iff background_on), pitch in elements,
 * in_precision SACX_FP64 or SACX_FP32 of the caller arrays.  The data are
 * copied (caller keeps ownership), halos are filled and the wave speeds are
 * reduced for the first time step.  Resets the step count, sets t = t0.
 * Enqueued on the stream; returns without synchronising. */
int sacx_init_state(sacx_ctx *ctx, const void *const *d_fields, const void *const *d_bg,
                    int64_t pitch, int32_t in_precision, double t0);

/* Enqueue up to nsteps RK4 steps (paper section 2; one step = 4 stages,
 * each preceded by a halo exchange).  t_end <= 0: no end time.  Otherwise
 * dt = min(dt, t_end - t) and stepping stops once t_end - t <= 1e-12 t_end.
 * A step whose start state is non-physical is not taken, and neither is any
 * later one; that state is kept.  If steps_done or t_now is non-NULL the call
 * synchronises the stream, fills them (steps taken by this call, current
 * time) and returns SACX_ENONPHYS if a non-physical state stopped it;
 * otherwise it returns after enqueuing. */
int sacx_advance(sacx_ctx *ctx, int32_t nsteps, double t_end, int32_t *steps_done, double *t_now);

/* Copy the interior of the evolved fields selected by field_mask (bit k =
 * field k) into caller device buffers d_out[k] (pitch in elements), converted
 * to out_precision.  Entries of d_out for unselected fields are ignored.
 * Enqueued on the stream (paper section 5: snapshots at fixed times). */
int sacx_read_fields(sacx_ctx *ctx, void *const *d_out, int64_t pitch, uint32_t field_mask,
                     int32_t out_precision);

/* Synchronise and report time, last dt, wave speeds, FP64 conservation sums,
 * step count and the non-physical flag. */
int sacx_diagnostics(sacx_ctx *ctx, sacx_diag *out);

/* Halo exchange building blocks (paper section 3, exchange_halo: gather the
 * halo into a device buffer / scatter a received buffer into the halo).
 *  side 0/1 (x-/x+): G = 3 columns x ny rows x 6 fields;
 *  side 2/3 (y-/y+): G rows x (nx + 2G) columns (x halos included, so corners
 *                    travel with the y exchange; do x before y) x 6 fields.
 * Buffer layout: [field][depth g = 0..G-1, increasing coordinate][along the side].
 * pack copies the G interior rows/columns next to `side` of the current
 * state; unpack writes the G ghost rows/columns of `side`.  For a periodic
 * neighbour, the buffer packed at x- is the one unpacked at x+.  Buffers are
 * caller-owned device memory in the context precision; sizes in bytes.
 * EUNSUP if that direction has fewer than G interior cells. */
int sacx_halo_buffer_size(const sacx_ctx *ctx, int32_t side, size_t *bytes);
int sacx_halo_pack(sacx_ctx *ctx, int32_t side, void *d_buf);
int sacx_halo_unpack(sacx_ctx *ctx, int32_t side, const void *d_buf);

/* Launch shape of the fused stage kernel: `threads` per block (64, 128 or
 * 256; a block owns threads - 6 columns) and `rows` output rows per block
 * strip (1..4096; each strip recomputes 6 rows of halo).  0 keeps the
 * current value.  Results do not depend on the shape (bit-identical); only
 * speed does.  Used by the tile autotuner.  Contexts with background_on
 * accept threads = 64 only (EUNSUP otherwise). */
int sacx_set_launch(sacx_ctx *ctx, int32_t threads, int32_t rows);
int sacx_get_launch(const sacx_ctx *ctx, int32_t *threads, int32_t *rows);

/* Per-phase timing on the context stream (HIP events around every launch
 * group), used to split a run into useful computation and halo exchange as in
 * the paper's cost model T = T_comp + T_comm + T_idle (section 6).
 *  ms_stage[s] / n_stage[s]: the fused stage-s kernel (s = 0..3 for stages 1..4);
 *  ms_halo / n_halo: halo pack + unpack (or boundary fill) before each stage;
 *  ms_scalar / n_scalar: the one-thread time-step kernels.
 * sacx_profile_enable(ctx, 1) resets the accumulators and starts recording;
 * (ctx, 0) stops.  sacx_profile_read synchronises and returns the totals. */
typedef struct sacx_profile {
    double ms_stage[4];
    double ms_halo;
    double ms_scalar;
    int64_t n_stage[4];
    int64_t n_halo;
    int64_t n_scalar;
} sacx_profile;

int sacx_profile_enable(sacx_ctx *ctx, int32_t on);
int sacx_profile_read(sacx_ctx *ctx, sacx_profile *out);

#ifdef __cplusplus
}
#endif

#endif /* SACX_H */
