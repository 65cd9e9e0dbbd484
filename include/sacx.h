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
 * (zero-gradient) boundaries applied locally, or, for a domain split into
 * subdomain contexts, filled from the neighbours before every stage.
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

#define SACX_ABI_VERSION 3

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
/* a side that borders another subdomain of a decomposed domain (paper
 * section 3, Fig. 1): the library never fills its ghost cells; the caller
 * unpacks the neighbour's strip there (sacx_halo_unpack) before every stage */
#define SACX_EXCHANGE 2

/* precisions */
#define SACX_FP64 0
#define SACX_FP32 1

/* number of ghost cells on every side (the hyper-diffusion stencil reaches 3 cells) */
#define SACX_GHOST 3

typedef struct sacx_grid {
    int32_t nx, ny;          /* interior cells of this subdomain */
    double x0, x1, y0, y1;   /* physical extent of this subdomain; the cell spacing is
                                (x1 - x0) / nx and (y1 - y0) / ny unless sacx_set_spacing
                                replaces it */
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
    double g[2];             /* gravity (x, y): the sources rho g and rho g.v of paper section 2.
                              * With the background taken to be in equilibrium under its own
                              * pressure and field they act on the perturbation density:
                              * rho~ g on the momentum, rho~ g.v on the energy (v of the total
                              * density).  {0, 0}: no gravity.  Must be finite (EINVAL). */
} sacx_params;

typedef struct sacx_diag {
    double t;                /* current time */
    double dt;               /* time step of the last step taken */
    double c_x, c_y, c_max;  /* max(|v_d| + c_f) over this context's cells of the current state */
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

/* Release a context: waits for the work queued on its stream (so the caller
 * may free the workspace once this returns), then frees the host object; the
 * workspace memory itself is not touched.  NULL is a no-op. */
int sacx_destroy(sacx_ctx *ctx);

/* Set the boundary kind of each side (paper section 5: periodic for
 * Orszag-Tang; open for the shock tube).  Periodic sides must come in pairs
 * (x-, x+ and y-, y+), else EINVAL.  A direction with one cell must be
 * periodic.  Takes effect at the next halo fill (the background's halos,
 * if any, are filled again at once).  While a learned coefficient is set
 * (sacx_hd_set_surrogate) only all-periodic boundaries are accepted (ESTATE
 * otherwise).  EXCHANGE sides: EUNSUP with a background or with fewer than
 * SACX_GHOST cells across; such a context steps with sacx_stage. */
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

/* The paper's verification problems (section 5), generated on the device
 * in place of sacx_init_state, evaluated at the cell centres of the
 * context's grid (x_i = x0 + (i + 1/2) dx), gamma from the parameters:
 *  SACX_PROBLEM_ORSZAG_TANG: rho = 25/(36 pi), p = 5/(12 pi),
 *    v = (-sin y, sin x), B = B0 (-sin y, sin 2x), B0 = prm[0]/sqrt(4 pi)
 *    (nprm 0 or 1, default prm[0] = 1); all boundaries PERIODIC.  The
 *    standard vortex is the grid [0, 2 pi]^2 with gamma = 5/3.
 *  SACX_PROBLEM_BRIO_WU: the shock tube, left of the middle of the domain
 *    rho = p = s_l, B = (0.75, 1), right rho = 0.125 s_r, p = 0.1 s_r,
 *    B = (0.75, -1), v = 0 (prm = {s_l, s_r}, nprm 0 to 2, default 1, each
 *    > 0).  Along y (field components swapped) when nx = 1 < ny, else along
 *    x; OPEN ends, PERIODIC across.  The standard tube is [0, 1], gamma = 2.
 * Sets those boundaries (as sacx_set_boundaries, with its errors), then
 * continues as sacx_init_state (time t0, step count reset).  EINVAL for an
 * unknown kind or bad parameters, EUNSUP with a background.  The sines come
 * from the device's sin: a cell may differ from a host evaluation in the
 * last bit.  Enqueued on the stream. */
#define SACX_PROBLEM_ORSZAG_TANG 0
#define SACX_PROBLEM_BRIO_WU 1
int sacx_init_problem(sacx_ctx *ctx, int32_t kind, const double *prm, int32_t nprm, double t0);

/* Enqueue up to nsteps RK4 steps (paper section 2; one step = 4 stages,
 * each preceded by a halo exchange).  ESTATE for a context with an EXCHANGE
 * side or while a step begun with sacx_stage is in progress.  t_end <= 0: no
 * end time.  Otherwise dt = min(dt, t_end - t) and stepping stops once
 * t_end - t <= 1e-12 t_end.
 * A step whose start state is non-physical is not taken, and neither is any
 * later one; that state is kept.  If steps_done or t_now is non-NULL the call
 * synchronises the stream, fills them (steps taken by this call, current
 * time) and returns SACX_ENONPHYS if a non-physical state stopped it;
 * otherwise it returns after enqueuing. */
int sacx_advance(sacx_ctx *ctx, int32_t nsteps, double t_end, int32_t *steps_done, double *t_now);

/* Copy the interior of the evolved fields selected by field_mask (bit k =
 * field k) into caller device buffers d_out[k] (pitch in elements), converted
 * to out_precision.  Entries of d_out for unselected fields are ignored.
 * During a step begun with sacx_stage these are the fields at the step's
 * start.  Enqueued on the stream (paper section 5: snapshots at fixed times). */
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
 * pack copies the G interior rows/columns next to `side` of the state the
 * next stage differences (the current state between steps; during a step
 * begun with sacx_stage, the intermediate state of the stage about to run);
 * unpack writes the G ghost rows/columns of `side` of that same state.  For
 * a periodic neighbour, the buffer packed at x- is the one unpacked at x+.
 * Buffers are caller-owned device memory in the context precision; sizes in
 * bytes.
 * EUNSUP if that direction has fewer than G interior cells. */
int sacx_halo_buffer_size(const sacx_ctx *ctx, int32_t side, size_t *bytes);
int sacx_halo_pack(sacx_ctx *ctx, int32_t side, void *d_buf);
int sacx_halo_unpack(sacx_ctx *ctx, int32_t side, const void *d_buf);

/* Decomposed stepping (paper section 3, Fig. 1: a domain split into
 * subdomains, one per process, whose halos are exchanged before every
 * stage; the time step is the one of the whole domain).  Every subdomain of
 * a domain is a context; a side that borders another subdomain is EXCHANGE.
 * Every subdomain takes the spacing of the whole domain (sacx_set_spacing).
 * One RK4 step of the whole domain, for stage = 1..4:
 *   1. sacx_fill_boundaries(ctx, 0) on every subdomain;
 *   2. for each x EXCHANGE side: the neighbour packs its facing side
 *      (sacx_halo_pack), this context unpacks that buffer (sacx_halo_unpack);
 *   3. sacx_fill_boundaries(ctx, 1);
 *   4. the same for the y EXCHANGE sides (their strips carry the x halos:
 *      the corners);
 *   5. sacx_stage(ctx, c, ...) on every subdomain, with c at stage 1 the
 *      maxima over all subdomains: on the host from sacx_wave_speeds, or
 *      on the device by sacx_wave_speeds_max into one zeroed array (the
 *      stand-in of an all-reduce(max); no synchronisation).
 * Each subdomain then evolves bit for bit as its part of the undivided
 * domain run with sacx_advance.  No end time; a non-physical step-start
 * state (sacx_diagnostics) stops that subdomain's steps, not the others'.
 *
 * sacx_fill_boundaries: fill the ghost cells of direction 0 (x, interior
 * rows) or 1 (y, whole padded width, so after x) of the state the next stage
 * differences, on the PERIODIC and OPEN sides (EXCHANGE sides untouched).
 *
 * sacx_stage: run the next stage of the step (1, 2, 3, 4, 1, ...) on the
 * state whose ghost cells the caller completed.  At stage 1 the step begins:
 * c_max = the x and y wave-speed maxima of the whole domain's current state
 * (each >= 0 and finite, > 0 along a direction with more than one cell;
 * NULL = this context's own); ignored at later stages.  c_max_on_device = 0:
 * c_max is host memory, read during the call, EINVAL for bad values; 1: it
 * is 2 device doubles (8-byte aligned), read on the stream when the step
 * begins, and a bad value stops this subdomain's stepping as a non-physical
 * state does (sacx_diagnostics reports it).
 * Stage 4 ends the step (t, step count, wave speeds of the new state).
 * stage_done (optional) receives the stage that was enqueued.  ESTATE with a
 * learned coefficient set.  Enqueued, not synchronised.
 *
 * sacx_wave_speeds: synchronise and return the x and y maxima of |v_d| + c_f
 * over this context's interior cells of the current state (the step-start
 * state while a step is in progress).
 *
 * sacx_wave_speeds_max: enqueue d_c_max[d] = max(d_c_max[d], this context's
 * maxima) on a device array of 2 doubles (8-byte aligned) that holds
 * non-negative values, e.g. zeros written before the first context of the
 * step.  ESTATE during a step.  Contexts on different streams must order
 * these updates before every stage 1 that reads the array. */
int sacx_fill_boundaries(sacx_ctx *ctx, int32_t direction);
/* sacx_set_spacing: set the cell spacing (dx, dy; finite, > 0) from which
 * the scheme's grid constants follow, in place of (x1 - x0) / nx and
 * (y1 - y0) / ny of the context's grid.  A subdomain takes the spacing of
 * the whole domain: its own extent over its own cell count can round
 * differently.  EINVAL for bad values, ESTATE during a step begun with
 * sacx_stage.  Host only; takes effect at the next step. */
int sacx_set_spacing(sacx_ctx *ctx, double dx, double dy);
int sacx_stage(sacx_ctx *ctx, const double *c_max, int32_t c_max_on_device, int32_t *stage_done);
int sacx_wave_speeds(sacx_ctx *ctx, double c_max[2]);
int sacx_wave_speeds_max(sacx_ctx *ctx, double *d_c_max);

/* A decomposed domain stepped natively: px x py subdomain contexts (row
 * major, subdomain (a, b) at subs[a + b px], x increasing with a, y with b)
 * whose halos the library exchanges itself, in the order described above,
 * with the maxima reduced on the device.  Requirements (EINVAL otherwise):
 * every context initialised (ESTATE otherwise), on one device and one
 * stream, with equal precision, scheme parameters and grid spacing; every
 * side that borders another subdomain is EXCHANGE, and so is the facing side
 * of the neighbour across every EXCHANGE side (across the domain's edge the
 * neighbour is the subdomain at the other end: a periodic domain); facing
 * strips have equal lengths; at most 4096 subdomains.  A context of a
 * domain is still the caller's (destroy the domain first); its own calls
 * keep working.
 *  sacx_domain_buffer_size: bytes of caller device memory the domain needs
 *    (one strip per EXCHANGE side and the maxima); host arithmetic.
 *  sacx_domain_create: d_buf (256-byte aligned, ENOSPC if smaller) must
 *    outlive the domain.
 *  sacx_domain_advance: enqueue nsteps steps of every subdomain on their
 *    stream (no synchronisation); ESTATE while a subdomain has a step begun
 *    with sacx_stage in progress or has other boundary kinds than when the
 *    domain was created.  A subdomain stopped by a non-physical state
 *    stays stopped (sacx_diagnostics); the others go on.
 *  sacx_domain_destroy: releases the host object (NULL is a no-op). */
typedef struct sacx_domain sacx_domain;
int sacx_domain_buffer_size(int32_t px, int32_t py, sacx_ctx *const *subs, size_t *bytes);
int sacx_domain_create(int32_t px, int32_t py, sacx_ctx *const *subs, void *d_buf, size_t buf_bytes,
                       sacx_domain **out);
int sacx_domain_advance(sacx_domain *d, int32_t nsteps);
int sacx_domain_destroy(sacx_domain *d);

/* Launch shape of the fused stage kernel: `threads` columns per block
 * including the 6-column apron (64, 128 or 256; the one-thread tile runs
 * that many threads per block, the FP64 split tile of sacx_set_column_split
 * twice as many) and `rows` output rows per
 * block strip (1..4096; each strip recomputes 6 rows of halo).  0 keeps the
 * current value.  Until rows is set, the strip height is chosen from the
 * device (compute units x resident blocks per unit): strips balanced to fit
 * one round of resident blocks when that needs at most 512 rows, else 256
 * rows (halved while there are fewer than 1024 blocks); it is chosen again
 * whenever threads or the tile kind change.  Results do not depend on the
 * shape (bit-identical); only speed does.  Used by the tile autotuner. */
int sacx_set_launch(sacx_ctx *ctx, int32_t threads, int32_t rows);
int sacx_get_launch(const sacx_ctx *ctx, int32_t *threads, int32_t *rows);

/* Tile kind of FP64 two-dimensional contexts with hyper-diffusion and the
 * plain coefficient (with or without a background): on = 1 (the default) gives every
 * column two threads, one for the x-direction terms and one for the
 * y-direction terms, in blocks of 2 * threads; on = 0 gives it one thread.
 * Results are bit-identical either way; the two-thread tile holds half the
 * per-thread state and runs two waves per SIMD.  Other contexts ignore the
 * setting.  EINVAL unless on is 0 or 1. */
int sacx_set_column_split(sacx_ctx *ctx, int32_t on);

/* Per-phase timing on the context stream (HIP events around every launch
 * group), used to split a run into useful computation and halo exchange as in
 * the paper's cost model T = T_comp + T_comm + T_idle (section 6).
 *  ms_stage[s] / n_stage[s]: the fused stage-s kernel (s = 0..3 for stages 1..4);
 *  ms_halo / n_halo: halo pack + unpack (or boundary fill) before each stage,
 *                    and each sacx_fill_boundaries, sacx_halo_pack and
 *                    sacx_halo_unpack call;
 *  ms_scalar / n_scalar: the one-thread time-step kernels;
 *  ms_surrogate / n_surrogate: surrogate refreshes (prediction and check).
 * sacx_profile_enable(ctx, 1) resets the accumulators and starts recording;
 * (ctx, 0) stops.  sacx_profile_read synchronises and returns the totals. */
typedef struct sacx_profile {
    double ms_stage[4];
    double ms_halo;
    double ms_scalar;
    int64_t n_stage[4];
    int64_t n_halo;
    int64_t n_scalar;
    double ms_surrogate;
    int64_t n_surrogate;
} sacx_profile;

int sacx_profile_enable(sacx_ctx *ctx, int32_t on);
int sacx_profile_read(sacx_ctx *ctx, sacx_profile *out);

/* ---------------------------------------------------------------------
 * Batches: many independent subdomains (shock tubes, vortex boxes of
 * different sizes, gamma, boundaries and time steps) advanced by one
 * persistent cooperative launch.  Each instance is an ordinary context
 * (sacx_batch_context) carved from the batch workspace: initialise, read and
 * inspect it with sacx_init_state / sacx_read_fields / sacx_diagnostics; it
 * may also be advanced alone with sacx_advance.  A batched step of an
 * instance gives the same bits as sacx_advance of that instance.
 * All instances share one precision; hd_on = 1, no background, nx >= 3.
 * --------------------------------------------------------------------- */
typedef struct sacx_batch sacx_batch;

/* Workspace bytes for n instances (grids[n], params[n]); host arithmetic. */
int sacx_batch_workspace_size(int32_t n, const sacx_grid *grids, const sacx_params *params, size_t *bytes);

/* Create a batch in caller-owned device memory (256-byte aligned).  bc: 4n
 * boundary kinds (x-, x+, y-, y+ per instance; PERIODIC or OPEN, EUNSUP for
 * EXCHANGE) or NULL for all periodic. */
int sacx_batch_create(int32_t n, const sacx_grid *grids, const sacx_params *params, const int32_t *bc,
                      void *d_ws, size_t ws_bytes, void *hip_stream, sacx_batch **out);
/* Release a batch and its instance contexts, after the work queued on its
 * stream has finished.  NULL is a no-op. */
int sacx_batch_destroy(sacx_batch *b);

/* The context of instance i (owned by the batch, valid until destroy). */
int sacx_batch_context(sacx_batch *b, int32_t i, sacx_ctx **out);

/* Tile shapes: threads per block for the whole launch (64/128/256; 0 keeps)
 * and output rows per tile strip for each instance (rows[n], 1..4096; NULL
 * keeps).  One-dimensional instances always use one-row tiles.  Results do
 * not depend on the shapes.  Used by the tile autotuner. */
int sacx_batch_set_tiles(sacx_batch *b, int32_t threads, const int32_t *rows);

/* Advance every instance by nsteps RK4 steps (each with its own dt) in one
 * persistent launch per 512 steps.  Every instance must have been
 * initialised (ESTATE otherwise).  With sync != 0 the call synchronises and
 * returns SACX_ENONPHYS if any instance stopped on a non-physical state.
 * The batch uses the plain hyper-diffusion coefficient: an instance whose
 * context has a learned coefficient set gives SACX_EUNSUP. */
int sacx_batch_advance(sacx_batch *b, int32_t nsteps, int32_t sync);


/* ---------------------------------------------------------------------
 * Learned hyper-diffusion coefficient.
 *
 * Paper section 2 sets each hyper-diffusion coefficient from the ratio R of
 * third- to first-order differences of the diffused quantity (R in [0, 4] in
 * this library's reading: the largest |third difference| over the 3 faces
 * around a face over the largest |first difference| over the 5 faces around
 * it).  Ten ratio fields are needed per state: on x faces (i+1/2, j) of
 * {rho~, eps~, v_x, v_y, B~_y} and on y faces (i, j+1/2) of
 * {rho~, eps~, v_x, v_y, B~_x}; as arrays they are 10 planes ("ratio
 * planes"), plane k row j element i holding the value of set k at the face
 * just above cell (i, j) in x (k < 5) or y (k >= 5).
 *
 * A small network predicts these ratio planes from the local state:
 * four 3x3 convolutions with periodic padding, 6 -> 32 -> 32 -> 32 -> 10
 * channels, ReLU between layers, output 4 sigmoid(z); BF16 weights and
 * activations with FP32 accumulation on the matrix cores.  Its input is
 * (rho, v_x, v_y, B_x, B_y, e) per cell, normalised as (f - shift) * scale.
 * With the surrogate on, a context predicts the ratio planes every K steps,
 * compares them tile by tile with the plain ratios of the same state and
 * keeps the prediction only in tiles where every face's error (ratio or
 * flux-weighted, SACX_HD_CHECK_*) is within a bound; the other tiles, and
 * any face given a negative value, use the plain ratio.
 * The coefficient itself keeps the exact maximum wave speed and compression
 * term.
 *
 * Network buffers (all device memory, caller-owned, 16-byte aligned):
 *   parameters : SACX_CNN_NPARAM floats, w0 b0 w1 b1 w2 b2 w3 b3, each w_l
 *                row-major over (out channel, in channel, ky, kx); w[o][c][ky][kx]
 *                multiplies input channel c at offset (ky-1, kx-1) in (y, x)
 *   packed     : SACX_CNN_PACKED_BYTES, BF16 weights in matrix-core operand
 *                order plus FP32 biases (sacx_cnn_pack)
 *   input      : BF16, n images of h x w pixels, 8 values per pixel (the six
 *                inputs, then 2 zeros), pixel (img, y, x) at ((img h + y) w + x) 8
 *   activations: BF16, three hidden layers of 32 values per pixel
 *   output     : FP32 ratio planes, [img][10][h][w]
 * Image width must be a multiple of 32.
 * --------------------------------------------------------------------- */
#define SACX_CNN_NPARAM 23146
#define SACX_CNN_PACKED_BYTES 99840

typedef struct sacx_cnn_sizes {
    size_t input_bytes;  /* input images */
    size_t act_bytes;    /* hidden activations kept by sacx_cnn_forward */
    size_t out_bytes;    /* output ratio planes */
    size_t work_bytes;   /* scratch of sacx_cnn_backward */
} sacx_cnn_sizes;

/* Buffer sizes for a batch of n images of h x w (host arithmetic). */
int sacx_cnn_buffer_sizes(int32_t n, int32_t h, int32_t w, sacx_cnn_sizes *out);

/* Convert FP32 parameters to the packed BF16 form (round to nearest even). */
int sacx_cnn_pack(const float *d_theta, void *d_packed, void *stream);

/* Forward pass: input -> activations (kept for the backward pass) and output. */
int sacx_cnn_forward(const void *d_packed, const void *d_x, int32_t n, int32_t h, int32_t w, void *d_act,
                     float *d_out, void *stream);

/* Mean over all outputs of w (out - target)^2 (w = 1 when d_weight is
 * NULL, else per-output weights in the output layout) into *d_loss (one
 * double, device) and its gradient with respect to every parameter into
 * d_grad (SACX_CNN_NPARAM floats, overwritten).  Sums over pixels are
 * reduced in a fixed order: results are deterministic. */
int sacx_cnn_backward(const void *d_packed, const void *d_x, const void *d_act, const float *d_out,
                      const float *d_target, const float *d_weight, int32_t n, int32_t h, int32_t w, void *d_work,
                      size_t work_bytes, float *d_grad, double *d_loss, void *stream);

/* The backward pass of sacx_cnn_backward (same arguments, same results bit
 * for bit) with no workspace argument, for callers that cannot allocate
 * device memory: code under HIP-graph capture, tight training loops,
 * harnesses that forbid allocation.  Its scratch is a static device array of
 * SACX_CNN_STATIC_WORK_BYTES (64 MiB), one per device, reserved from the
 * library's first use on that device until the process ends; the call
 * itself allocates and frees nothing.  ENOSPC when the batch needs more
 * scratch than that (sacx_cnn_buffer_sizes().work_bytes; e.g. 8 images of
 * 128 x 128 fit).  Every call on one device uses that device's one array:
 * calls that overlap on one device (other streams, other threads) race and
 * must be ordered by the caller.  Nothing in the scratch needs to start at
 * zero: each pass writes what it reads. */
#define SACX_CNN_STATIC_WORK_BYTES (64u << 20)
int sacx_cnn_backward_noalloc(const void *d_packed, const void *d_x, const void *d_act, const float *d_out,
                              const float *d_target, const float *d_weight, int32_t n, int32_t h, int32_t w,
                              float *d_grad, double *d_loss, void *stream);

/* One Adam update (bias-corrected, step counts from 1) of the FP32
 * parameters with moment buffers d_m, d_v (SACX_CNN_NPARAM floats each). */
int sacx_cnn_adam(float *d_theta, float *d_m, float *d_v, const float *d_grad, int32_t step, float lr,
                  float beta1, float beta2, float eps, void *stream);

/* The network input of the context's current state (one nx x ny image,
 * periodic), norm = shift[6] then scale[6]. */
int sacx_cnn_inputs(sacx_ctx *ctx, const float norm[12], void *d_x);

/* The plain ratio planes of the context's current state, as FP32, row pitch
 * `pitch` elements, plane stride pitch * ny (the training target); d_d1
 * (optional, same layout) receives each face's first difference of its set
 * (the hyper-diffusive flux of a face is proportional to R times it). */
int sacx_hd_ratio_fields(sacx_ctx *ctx, float *d_r, float *d_d1, int64_t pitch);

/* check metrics: the error of a predicted ratio r against the plain R at a face */
#define SACX_HD_CHECK_RATIO 0  /* |r - R| */
#define SACX_HD_CHECK_FLUX 1   /* |r - R| |d1| / D: d1 the face's first difference, D the largest
                                  |d1| of that plane over the domain (0 when D = 0); the
                                  error of the flux the value produces, relative */

typedef struct sacx_surrogate {
    const void *d_packed;   /* packed network (caller-owned, valid while in use);
                               NULL: the caller writes the ratio planes itself */
    float norm[12];         /* input shift[6], scale[6] */
    int32_t refresh_every;  /* K >= 1: predict and check every K steps */
    int32_t tile;           /* check tile side in cells (>= 1) */
    int32_t metric;         /* SACX_HD_CHECK_RATIO or SACX_HD_CHECK_FLUX */
    double bound;           /* largest error a kept tile may have */
} sacx_surrogate;

typedef struct sacx_hd_stats {
    int64_t refreshes;       /* checks done */
    int64_t tiles_checked;   /* tiles compared, summed over checks */
    int64_t tiles_fallback;  /* of which fell back to the plain ratio */
    double err_used;         /* max error (per the metric) over kept tiles */
    double err_all;          /* max over every finite comparison */
} sacx_hd_stats;

/* Device bytes the surrogate needs for this context (ratio planes, the
 * check's per-tile flags, network input and two activation buffers). */
int sacx_surrogate_workspace_size(const sacx_ctx *ctx, size_t *bytes);

/* Switch the surrogate on (caller-owned workspace, 256-byte aligned, valid
 * until sacx_hd_clear_surrogate or sacx_destroy).  Requires hd_on, no
 * background, all boundaries periodic, ny >= 2 and nx a multiple of 32
 * (SACX_EUNSUP otherwise).  The first step after this call refreshes.  With
 * d_packed == NULL the ratio planes (sacx_hd_ratio_buffer) are not
 * predicted but left as the caller wrote them; they are still checked. */
int sacx_hd_set_surrogate(sacx_ctx *ctx, const sacx_surrogate *cfg, void *d_ws, size_t ws_bytes);
int sacx_hd_clear_surrogate(sacx_ctx *ctx);

/* Device address and row pitch (elements) of the surrogate's ratio planes
 * (plane stride pitch * ny).  Checked tiles that fell back hold -1.  Until
 * the next check the stages read the planes of the tiles the last check kept
 * (values written there meanwhile are used) and no plane of a tile that fell
 * back (those take the plain ratio whatever the planes hold). */
int sacx_hd_ratio_buffer(sacx_ctx *ctx, float **d_r, int64_t *pitch);

/* Surrogate counters since sacx_hd_set_surrogate (synchronises). */
int sacx_hd_read_stats(sacx_ctx *ctx, sacx_hd_stats *out);

#ifdef __cplusplus
}
#endif

#endif /* SACX_H */
