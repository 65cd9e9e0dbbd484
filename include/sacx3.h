/*
 * sacx3.h -- C ABI of the three-dimensional form of the scheme in libsacx
 * (the paper states that the code is implemented in three dimensions,
 * sections 2 and 8; its 3-D results are announced as forthcoming).
 *
 * What a 3-D context computes (paper section 2, carried to three
 * dimensions): the ideal compressible MHD equations in conservative form for
 * eight evolved fields, fluxes along x, y and z differenced with the
 * fourth-order central difference, hyper-diffusion on every face with the
 * coefficient ratio of third- to first-order differences along the face
 * normal scaled by the maximum wave speed (plus the compression term), the
 * off-diagonal hyper-viscous stress and hyper-resistive e.m.f. terms, and
 * classic fourth-order Runge-Kutta with the CFL time step over the three
 * directions.  There is no background field and no gravity in 3-D; storage
 * and arithmetic are FP64.
 *
 * Conventions (as in sacx.h unless stated):
 *  - Grid: cell centred, x_i = x0 + (i + 1/2) dx, dx = (x1 - x0) / nx; the
 *    same in y and z.  A direction with one cell must be periodic; all its
 *    differences vanish.
 *  - Evolved fields (conserved variables), in this order:
 *      0 rho   density          4 e    total energy
 *      1 m_x   momentum x       5 B_x  field x
 *      2 m_y   momentum y       6 B_y  field y
 *      3 m_z   momentum z       7 B_z  field z
 *  - Caller arrays hold nz planes of ny rows of nx values (x fastest), with
 *    a row pitch and a plane pitch given in ELEMENTS (pitch >= nx,
 *    plane_pitch >= ny * pitch); device pointers.
 *  - Boundary sides: 0 = x-, 1 = x+, 2 = y-, 3 = y+, 4 = z-, 5 = z+; values
 *    SACX_PERIODIC or SACX_OPEN (zero-gradient), periodic in pairs.
 *  - Status codes, error strings (sacx_strerror, sacx_last_error), device
 *    and stream binding and the caller-owned workspace are those of sacx.h:
 *    the library never allocates or frees device memory.
 */
#ifndef SACX3_H
#define SACX3_H

#include <stddef.h>
#include <stdint.h>

#include "sacx.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sacx3_grid {
    int32_t nx, ny, nz;                   /* cells */
    double x0, x1, y0, y1, z0, z1;        /* physical extent */
} sacx3_grid;

typedef struct sacx3_params {
    double gamma;            /* adiabatic index (> 1) */
    double cfl;              /* dt = cfl * min over directions with more than one cell of h_d / c_d */
    int32_t hd_on;           /* hyper-diffusion on/off */
    int32_t hd_cross_on;     /* off-diagonal stress / e.m.f. terms */
    double c2[4];            /* ratio-term constants: density, thermal energy, velocity, field */
    double cshk[4];          /* compression-term constants, same classes */
} sacx3_params;

typedef struct sacx3_diag {
    double t;                /* current time */
    double dt;               /* time step of the last step taken */
    double c[3];             /* max(|v_d| + c_f) over the cells of the current state, d = x, y, z */
    double c_max;            /* maximum of c over the directions with more than one cell */
    double sums[8];          /* sum over the cells of each evolved field times dx dy dz (FP64) */
    int64_t steps;           /* steps taken since sacx3_init_state */
    int32_t nonphys;         /* 1 if the current state is non-physical */
} sacx3_diag;

typedef struct sacx3_ctx sacx3_ctx;

/* Bytes of device workspace a 3-D context needs (host arithmetic only).
 * EINVAL on an invalid grid or parameters. */
int sacx3_workspace_size(const sacx3_grid *grid, const sacx3_params *params, size_t *bytes);

/* Create a 3-D context on the current device.  d_ws: caller-owned device
 * memory of at least sacx3_workspace_size bytes, 256-byte aligned, that
 * outlives the context (ENOSPC if smaller).  hip_stream: hipStream_t (NULL =
 * null stream).  All six boundaries start PERIODIC. */
int sacx3_create(const sacx3_grid *grid, const sacx3_params *params, void *d_ws, size_t ws_bytes,
                 void *hip_stream, sacx3_ctx **out);

/* Wait for the context's queued work, then free the host object (the
 * workspace is not touched).  NULL is a no-op. */
int sacx3_destroy(sacx3_ctx *ctx);

/* Boundary kind of each of the six sides (paper section 5: periodic or open
 * boundaries).  Periodic sides come in pairs; a direction with one cell must
 * be periodic (EINVAL otherwise).  Takes effect at the next ghost fill. */
int sacx3_set_boundaries(sacx3_ctx *ctx, const int32_t bc[6]);

/* Load a state (paper section 3: the initial configuration): 8 device
 * pointers to FP64 arrays in the field order above, row and plane pitch in
 * elements.  Copies the cells in, fills the ghost layers and reduces the
 * wave speeds for the first step; t = t0, step count reset.  Enqueued. */
int sacx3_init_state(sacx3_ctx *ctx, const double *const *d_fields, int64_t pitch, int64_t plane_pitch,
                     double t0);

/* Enqueue up to nsteps RK4 steps (paper section 2; one step is 4 stages, the
 * ghost layers refilled before each).  t_end <= 0: no end time; otherwise
 * dt = min(dt, t_end - t) and stepping stops once t_end - t <= 1e-12 t_end.
 * A step whose start state is non-physical (rho <= 0, p <= 0 or not finite)
 * is not taken, nor any later one.  With steps_done or t_now non-NULL the
 * call synchronises, fills them and returns SACX_ENONPHYS if a non-physical
 * state stopped it; otherwise it returns after enqueuing. */
int sacx3_advance(sacx3_ctx *ctx, int32_t nsteps, double t_end, int32_t *steps_done, double *t_now);

/* Copy the cells of the fields selected by field_mask (bit k = field k) into
 * caller FP64 device buffers d_out[k] (pitches in elements).  Enqueued. */
int sacx3_read_fields(sacx3_ctx *ctx, double *const *d_out, int64_t pitch, int64_t plane_pitch,
                      uint32_t field_mask);

/* Synchronise; time, last dt, wave speeds, FP64 conservation sums. */
int sacx3_diagnostics(sacx3_ctx *ctx, sacx3_diag *out);

/* Launch shape of the stage kernels: planes per block along z (>= 1; 0
 * keeps the default).  Results never depend on it. */
int sacx3_set_launch(sacx3_ctx *ctx, int32_t planes);

#ifdef __cplusplus
}
#endif

#endif /* SACX3_H */
