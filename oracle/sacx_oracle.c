/*
 * sacx_oracle.c -- plain FP64 CPU oracle of the SAC/SMAUG+ MHD scheme.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The product path
 * (the HIP library) never calls it, links it or shares code with it.
 *
 * It is written for obviousness, not speed: every stage of the scheme is a
 * full-array pass with plain loops, in the order the scheme is defined.
 * Build with -O2 -ffp-contract=off (no fast-math) so every operation rounds
 * exactly as written.  OpenMP only distributes independent rows; reductions
 * are maxima (order free) or serial pairwise sums, so results do not depend
 * on the thread count.
 *
 * What is computed (paper section 2 and our reading of what it defers to the
 * SAC/SMAUG papers):
 *
 *  - ideal compressible MHD in conservative form (section 2, the governing
 *    equations), with the closure p_t = p_k + B^2/2,
 *    p_k = (gamma-1)(e - rho v^2/2 - B^2/2) (section 2, the two pressure
 *    definitions), written for static background + perturbation split
 *    variables (rho = rho_b + rho~, e = e_b + e~, B = B_b + B~, v_b = 0);
 *    the stray "+ grad p_t" of the printed energy equation is dropped;
 *  - spatial derivatives by fourth-order central differences (section 2);
 *  - hyper-diffusion / hyper-viscosity / hyper-resistivity whose coefficient
 *    is the ratio of third- to first-order differences of the variable and
 *    scales with the maximum wave speed, plus a term that grows with
 *    compression (section 2);
 *  - classic fourth-order Runge-Kutta in time (section 2);
 *  - gravity g through the sources rho g and rho g.v of section 2; with the
 *    background taken to be in equilibrium under its own pressure and field,
 *    what is left acts on the perturbation: rho~ g and rho~ g.v;
 *  - a CFL time step from the maximum fast speed;
 *  - halo (ghost) cells filled from periodic images or by zero-gradient
 *    copies (section 3, halo exchange; section 5 boundary conditions).
 *
 * Grid: cell centred, G = 3 ghost cells on every side, arrays row-major with
 * x fastest.  Field order: rho~, m_x, m_y, e~, B~_x, B~_y; background order:
 * rho_b, e_b, B_bx, B_by.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define G 3
#define NF 6
#define NB 4

enum { F_RHO = 0, F_MX = 1, F_MY = 2, F_E = 3, F_BX = 4, F_BY = 5 };
enum { B_RHO = 0, B_E = 1, B_BX = 2, B_BY = 3 };
/* hyper-diffusion constant classes */
enum { C_RHO = 0, C_EPS = 1, C_V = 2, C_B = 3 };

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENONPHYS = -4, ORC_ENOMEM = -7 };
enum { ORC_PERIODIC = 0, ORC_OPEN = 1 };

/* Two arithmetic forms of the same scheme.
 *
 * ORC_FORM_PAPER defines the oracle: classic RK4 combined as printed,
 * U+ = U + dt/6 (K1 + 2 K2 + 2 K3 + K4) from four kept right-hand sides, and
 * every division of the scheme (by 12h, 2h, h, rho, gamma - 1) done as a
 * division.
 *
 * ORC_FORM_LOWSTORE is an algebraically equal rearrangement that needs only
 * four state arrays (U, the stage input S, an accumulator A, and the current
 * K): the same stage inputs, the final combine as
 *   A = 2U + ((S1 - U) + dt K2),   U+ = S3 + (A - 2 S3)/3 + dt/6 K4,
 * and divisions by grid constants, by rho and by gamma - 1 done as
 * multiplications by a reciprocal formed once.  It is a second, fixed IEEE
 * operation sequence: the hyper-diffusion coefficient (a ratio of maxima)
 * amplifies rounding-order differences from one step to the next, so two
 * algebraically equal forms drift apart far above 1e-12 within 100 steps of a
 * shock-forming run.  A device implementation that follows this sequence
 * exactly can be compared with it bit for bit; the CPU tests tie it to the
 * paper form (many steps without hyper-diffusion, a few with it). */
enum { ORC_FORM_PAPER = 0, ORC_FORM_LOWSTORE = 1 };

typedef struct {
    int nx, ny;
    double x0, x1, y0, y1;
    double gamma, cfl;
    int hd_on, hd_cross_on;
    double c2[4];   /* rho, eps, v, B */
    double cshk[4]; /* rho, eps, v, B */
    int bc[4];      /* x-, x+, y-, y+ */
    int background_on;
    double g[2];    /* gravity (section 2 sources rho g, rho g.v), acting on rho~ */
    int form;       /* ORC_FORM_PAPER (the definition) or ORC_FORM_LOWSTORE */
} orc_cfg;

int orc_abi_version(void) { return 3; }

/* ------------------------------------------------------------------ */
/* small helpers                                                       */
/* ------------------------------------------------------------------ */

static double dmax(double a, double b) { return a > b ? a : b; }
static double dmin(double a, double b) { return a < b ? a : b; }

static int imod(int i, int n) { int r = i % n; return r < 0 ? r + n : r; }
static int iclamp(int i, int n) { return i < 0 ? 0 : (i >= n ? n - 1 : i); }

static double *alloc0(size_t n) { return (double *)calloc(n ? n : 1, sizeof(double)); }

typedef struct {
    int nxe, nye;          /* extended dims */
    double *f[NF];         /* evolved fields (ext layout) */
} block;

static int block_alloc(block *b, int nxe, int nye) {
    b->nxe = nxe; b->nye = nye;
    for (int k = 0; k < NF; ++k) b->f[k] = NULL;
    for (int k = 0; k < NF; ++k) {
        b->f[k] = alloc0((size_t)nxe * nye);
        if (!b->f[k]) return ORC_ENOMEM;
    }
    return ORC_OK;
}

static void block_free(block *b) {
    for (int k = 0; k < NF; ++k) { free(b->f[k]); b->f[k] = NULL; }
}

static int cfg_ok(const orc_cfg *c) {
    if (!c || c->nx < 1 || c->ny < 1) return 0;
    if (c->nx < 2 && c->ny < 2) return 0;
    if (!(c->x1 > c->x0) || !(c->y1 > c->y0)) return 0;
    if (!(c->gamma > 1.0) || !(c->cfl > 0.0)) return 0;
    for (int s = 0; s < 4; ++s)
        if (c->bc[s] != ORC_PERIODIC && c->bc[s] != ORC_OPEN) return 0;
    if (!isfinite(c->g[0]) || !isfinite(c->g[1])) return 0;
    if (c->form != ORC_FORM_PAPER && c->form != ORC_FORM_LOWSTORE) return 0;
    if ((c->bc[0] == ORC_PERIODIC) != (c->bc[1] == ORC_PERIODIC)) return 0;
    if ((c->bc[2] == ORC_PERIODIC) != (c->bc[3] == ORC_PERIODIC)) return 0;
    return 1;
}

/* ------------------------------------------------------------------ */
/* halo fill: periodic images or zero-gradient copies                  */
/* (the state is extended by G cells before every right-hand side;     */
/* x first over the interior rows, then y over the padded width, which */
/* also fills the corners)                                             */
/* ------------------------------------------------------------------ */

static void fill_ghosts_one(double *a, int nx, int ny, const int bc[4]) {
    const int nxe = nx + 2 * G;
#define A(i, j) a[(size_t)((i) + G) + (size_t)((j) + G) * nxe]
    for (int j = 0; j < ny; ++j) {
        for (int i = -G; i < 0; ++i) {
            int s = bc[0] == ORC_PERIODIC ? imod(i, nx) : iclamp(i, nx);
            A(i, j) = A(s, j);
        }
        for (int i = nx; i < nx + G; ++i) {
            int s = bc[1] == ORC_PERIODIC ? imod(i, nx) : iclamp(i, nx);
            A(i, j) = A(s, j);
        }
    }
    for (int i = -G; i < nx + G; ++i) {
        for (int j = -G; j < 0; ++j) {
            int s = bc[2] == ORC_PERIODIC ? imod(j, ny) : iclamp(j, ny);
            A(i, j) = A(i, s);
        }
        for (int j = ny; j < ny + G; ++j) {
            int s = bc[3] == ORC_PERIODIC ? imod(j, ny) : iclamp(j, ny);
            A(i, j) = A(i, s);
        }
    }
#undef A
}

/* ------------------------------------------------------------------ */
/* x / d: a division in the paper form; in the low-storage form a      */
/* multiplication by the reciprocal inv_d = 1/d formed once            */
/* ------------------------------------------------------------------ */

static double over(int paper, double x, double d, double inv_d) {
    return paper ? x / d : x * inv_d;
}

/* ------------------------------------------------------------------ */
/* the fourth-order central difference (section 2)                     */
/*   D f_i = [8 (f_{i+1} - f_{i-1}) - (f_{i+2} - f_{i-2})] / (12 h)     */
/* h12 = 12 h, inv12h = 1/(12 h)                                       */
/* ------------------------------------------------------------------ */

static double d4(int paper, const double *f, ptrdiff_t i, ptrdiff_t st, double h12, double inv12h) {
    return over(paper, 8.0 * (f[i + st] - f[i - st]) - (f[i + 2 * st] - f[i - 2 * st]), h12, inv12h);
}

/* ------------------------------------------------------------------ */
/* hyper-diffusion coefficient ratio at the face between q[0] and      */
/* q[st] (section 2: ratio of the third- to the first-order forward    */
/* difference of the variable).  Our reading: third differences on the */
/* three faces around the face, first differences on the five faces    */
/* around it, R = max|d3| / max|d1|, R = 0 when max|d1| = 0; R <= 4.   */
/* ------------------------------------------------------------------ */

static double d1_at(const double *q, ptrdiff_t i, ptrdiff_t st) {   /* face i+1/2 */
    return q[i + st] - q[i];
}

static double d3_at(const double *q, ptrdiff_t i, ptrdiff_t st) {   /* face i+1/2 */
    return (q[i + 2 * st] - q[i - st]) - 3.0 * (q[i + st] - q[i]);
}

static double hd_ratio(const double *q, ptrdiff_t i, ptrdiff_t st) {
    double n = 0.0, m = 0.0;
    for (int k = -1; k <= 1; ++k) n = dmax(n, fabs(d3_at(q, i + k * st, st)));
    for (int k = -2; k <= 2; ++k) m = dmax(m, fabs(d1_at(q, i + k * st, st)));
    return m > 0.0 ? n / m : 0.0;
}

/* ------------------------------------------------------------------ */
/* right-hand side L(S) on an extended block                            */
/* K is written on [G, nxe-G) x [G, nye-G); every other entry is zero.  */
/* ------------------------------------------------------------------ */

typedef struct {
    double dx, dy, gamma;
    int paper;      /* 1: ORC_FORM_PAPER arithmetic, 0: ORC_FORM_LOWSTORE */
    int hd_on, hd_cross_on, bg_on;
    double c2[4], cshk[4];
    double g[2];
    int grav_on;
    /* optional externally supplied coefficient ratios (the surrogate's
     * prediction): 10 planes of nx*ny face values, planes 0-4 the x-face
     * sets, 5-9 the y-face sets, face (i+1/2, j) / (i, j+1/2) stored at
     * interior cell (i, j).  A negative value selects the plain ratio.  Used
     * only with blocks that are the whole domain extended by G (periodic). */
    const float *rext;
    int rext_nx, rext_ny;
} rhs_par;

/* coefficient ratio of set `plane` at the face of block cell (i, j): the
 * supplied value when there is one and it is not negative, else the plain
 * ratio of the differences */
static double ratio_or_ext(const rhs_par *P, int plane, int i, int j, const double *q, ptrdiff_t c,
                           ptrdiff_t st) {
    if (P->rext) {
        const int nx = P->rext_nx, ny = P->rext_ny;
        const float v = P->rext[(size_t)plane * nx * ny + (size_t)imod(j - G, ny) * nx + imod(i - G, nx)];
        if (v >= 0.0f) return (double)v;
    }
    return hd_ratio(q, c, st);
}

static int rhs_block(int nxe, int nye, double *const S[NF], double *const BG[NB],
                     const rhs_par *P, double cmax, double *const K[NF]) {
    const size_t n = (size_t)nxe * nye;
    const int pf = P->paper;
    const double gm1 = P->gamma - 1.0;
    const double igm1 = 1.0 / gm1;
    const double dx = P->dx, dy = P->dy;
    const double h12x = 12.0 * dx, h12y = 12.0 * dy, h2x = 2.0 * dx, h2y = 2.0 * dy;
    const double i12dx = 1.0 / h12x, i12dy = 1.0 / h12y;
    const double i2dx = 1.0 / h2x, i2dy = 1.0 / h2y;
    const double idx = 1.0 / dx, idy = 1.0 / dy;
    int rc = ORC_OK;

    /* primitive / derived quantities on every cell of the block */
    double *rho = alloc0(n), *vx = alloc0(n), *vy = alloc0(n), *bxT = alloc0(n), *byT = alloc0(n);
    double *pkt = alloc0(n), *ptt = alloc0(n), *epst = alloc0(n), *ptb = alloc0(n);
    double *Fx[NF], *Fy[NF];
    for (int k = 0; k < NF; ++k) { Fx[k] = alloc0(n); Fy[k] = alloc0(n); }
    double *s = NULL, *Gx[5] = {0}, *Gy[5] = {0}, *Hx[NF] = {0}, *Hy[NF] = {0};
    int ok = rho && vx && vy && bxT && byT && pkt && ptt && epst && ptb;
    for (int k = 0; k < NF; ++k) ok = ok && Fx[k] && Fy[k];
    if (P->hd_on) {
        s = alloc0(n);
        ok = ok && s;
        for (int k = 0; k < 5; ++k) { Gx[k] = alloc0(n); Gy[k] = alloc0(n); ok = ok && Gx[k] && Gy[k]; }
        for (int k = 0; k < NF; ++k) { Hx[k] = alloc0(n); Hy[k] = alloc0(n); ok = ok && Hx[k] && Hy[k]; }
    }
    if (!ok) { rc = ORC_ENOMEM; goto done; }

    /* 1. totals and derived quantities (closure of section 2, split form) */
#pragma omp parallel for schedule(static)
    for (int j = 0; j < nye; ++j) {
        for (int i = 0; i < nxe; ++i) {
            size_t c = (size_t)i + (size_t)j * nxe;
            double rb = 0.0, eb = 0.0, bxb = 0.0, byb = 0.0;
            if (P->bg_on) { rb = BG[B_RHO][c]; eb = BG[B_E][c]; bxb = BG[B_BX][c]; byb = BG[B_BY][c]; }
            double rt = S[F_RHO][c], mx = S[F_MX][c], my = S[F_MY][c], et = S[F_E][c];
            double bxt = S[F_BX][c], byt = S[F_BY][c];
            double r = rb + rt;
            double ir = 1.0 / r;
            double ux = over(pf, mx, r, ir), uy = over(pf, my, r, ir);
            double kin = 0.5 * (mx * ux + my * uy);          /* rho v^2 / 2 */
            double bbdot = bxb * bxt + byb * byt;            /* B_b . B~ */
            double bt2 = bxt * bxt + byt * byt;              /* |B~|^2 */
            double pk = gm1 * (((et - kin) - bbdot) - 0.5 * bt2);   /* p~_k */
            rho[c] = r; vx[c] = ux; vy[c] = uy;
            bxT[c] = bxb + bxt; byT[c] = byb + byt;
            pkt[c] = pk;
            ptt[c] = (pk + 0.5 * bt2) + bbdot;                /* p~_t */
            epst[c] = over(pf, pk, gm1, igm1);                /* thermal energy perturbation */
            if (P->bg_on) {
                double b2b = bxb * bxb + byb * byb;
                double pkb = gm1 * (eb - 0.5 * b2b);
                ptb[c] = pkb + 0.5 * b2b;                     /* p_tb */
            }

            /* 2. ideal fluxes of the split system (section 2 equations) */
            double bv_t = bxt * ux + byt * uy;                /* B~ . v */
            double bv_b = bxb * ux + byb * uy;                /* B_b . v */
            double eflux = et + eb + ptt[c];
            Fx[F_RHO][c] = mx;
            Fx[F_MX][c] = (ux * mx - (bxt * bxt + 2.0 * bxt * bxb)) + ptt[c];
            Fx[F_MY][c] = ux * my - (bxt * byt + bxt * byb + bxb * byt);
            Fx[F_E][c] = ((ux * eflux - bxt * bv_t) - bxt * bv_b) - bxb * bv_t;
            Fx[F_BX][c] = 0.0;
            Fx[F_BY][c] = ux * byT[c] - bxT[c] * uy;
            Fy[F_RHO][c] = my;
            Fy[F_MX][c] = uy * mx - (byt * bxt + byt * bxb + byb * bxt);
            Fy[F_MY][c] = (uy * my - (byt * byt + 2.0 * byt * byb)) + ptt[c];
            Fy[F_E][c] = ((uy * eflux - byt * bv_t) - byt * bv_b) - byb * bv_t;
            Fy[F_BX][c] = uy * bxT[c] - byT[c] * ux;
            Fy[F_BY][c] = 0.0;
        }
    }

    /* 3. K_ideal = -(D_x F_x + D_y F_y) (+ background terms of e~) */
#pragma omp parallel for schedule(static)
    for (int j = 0; j < nye; ++j) {
        for (int i = 0; i < nxe; ++i) {
            size_t c = (size_t)i + (size_t)j * nxe;
            if (i < G || i >= nxe - G || j < G || j >= nye - G) {
                for (int k = 0; k < NF; ++k) K[k][c] = 0.0;
                continue;
            }
            for (int k = 0; k < NF; ++k) {
                double ddx = d4(pf, Fx[k], (ptrdiff_t)c, 1, h12x, i12dx);
                double ddy = d4(pf, Fy[k], (ptrdiff_t)c, nxe, h12y, i12dy);
                K[k][c] = -(ddx + ddy);
            }
            if (P->bg_on) {
                /* e~ gets -p_tb div v + sum_kl B_bk B_bl d_k v_l (non-conservative) */
                double dxvx = d4(pf, vx, (ptrdiff_t)c, 1, h12x, i12dx);
                double dyvy = d4(pf, vy, (ptrdiff_t)c, nxe, h12y, i12dy);
                double dxvy = d4(pf, vy, (ptrdiff_t)c, 1, h12x, i12dx);
                double dyvx = d4(pf, vx, (ptrdiff_t)c, nxe, h12y, i12dy);
                double bxb = BG[B_BX][c], byb = BG[B_BY][c];
                double bb = (bxb * bxb * dxvx + byb * byb * dyvy) + (bxb * byb * dxvy + byb * bxb * dyvx);
                K[F_E][c] = K[F_E][c] + (bb - ptb[c] * (dxvx + dyvy));
            }
            if (P->grav_on) {
                /* gravity: the sources rho g and rho g.v of section 2 less the
                 * background's share, which its own pressure and field carry
                 * (the equilibrium assumed for the split form), leave rho~ g
                 * and rho~ g.v, with v the velocity of the total density */
                double rt = S[F_RHO][c];
                K[F_MX][c] = K[F_MX][c] + rt * P->g[0];
                K[F_MY][c] = K[F_MY][c] + rt * P->g[1];
                K[F_E][c] = K[F_E][c] + rt * (P->g[0] * vx[c] + P->g[1] * vy[c]);
            }
        }
    }

    if (!P->hd_on) goto done;

    /* 4a. compression indicator s = max(0, -div v) (2nd-order centred) */
#pragma omp parallel for schedule(static)
    for (int j = 1; j < nye - 1; ++j) {
        for (int i = 1; i < nxe - 1; ++i) {
            size_t c = (size_t)i + (size_t)j * nxe;
            double dv = over(pf, vx[c + 1] - vx[c - 1], h2x, i2dx) + over(pf, vy[c + nxe] - vy[c - nxe], h2y, i2dy);
            s[c] = dmax(0.0, -dv);
        }
    }

    /* 4b. face diffusion fluxes G_d(q) = nu_f(q) d1_f(q) / h_d,
     *     nu_f(q) = c2(q) h c_max R_f(q) + cshk(q) h^2 s_f.
     * x-face sets {rho~, eps~, v_x, v_y, B~_y}; y-face sets {rho~, eps~, v_x, v_y, B~_x}.
     * Faces are indexed by their lower cell. */
    {
        double *qx[5] = {S[F_RHO], epst, vx, vy, S[F_BY]};
        double *qy[5] = {S[F_RHO], epst, vx, vy, S[F_BX]};
        const int cls[5] = {C_RHO, C_EPS, C_V, C_V, C_B};
#pragma omp parallel for schedule(static)
        for (int j = 1; j < nye - 1; ++j) {
            for (int i = 2; i <= nxe - 4; ++i) {
                size_t c = (size_t)i + (size_t)j * nxe;
                double sf = dmax(s[c], s[c + 1]);
                for (int k = 0; k < 5; ++k) {
                    double R = ratio_or_ext(P, k, i, j, qx[k], (ptrdiff_t)c, 1);
                    double nu = P->c2[cls[k]] * dx * cmax * R + P->cshk[cls[k]] * dx * dx * sf;
                    Gx[k][c] = over(pf, nu * d1_at(qx[k], (ptrdiff_t)c, 1), dx, idx);
                }
            }
        }
#pragma omp parallel for schedule(static)
        for (int j = 2; j <= nye - 4; ++j) {
            for (int i = 1; i < nxe - 1; ++i) {
                size_t c = (size_t)i + (size_t)j * nxe;
                double sf = dmax(s[c], s[c + nxe]);
                for (int k = 0; k < 5; ++k) {
                    double R = ratio_or_ext(P, 5 + k, i, j, qy[k], (ptrdiff_t)c, nxe);
                    double nu = P->c2[cls[k]] * dy * cmax * R + P->cshk[cls[k]] * dy * dy * sf;
                    Gy[k][c] = over(pf, nu * d1_at(qy[k], (ptrdiff_t)c, nxe), dy, idy);
                }
            }
        }
    }
    /* index of each quantity inside the G arrays */
    enum { Q_RHO = 0, Q_EPS = 1, Q_VX = 2, Q_VY = 3, Q_B = 4 };

    /* 4c. face fluxes: mass diffusion, hyper-viscous stress, hyper-resistive
     * e.m.f. and the matching energy fluxes (all in flux form).
     * A4_x[g] averages the four y-face values around an x-face and A4_y the
     * four x-face values around a y-face. */
#pragma omp parallel for schedule(static)
    for (int j = 3; j <= nye - 4; ++j) {
        for (int i = 2; i <= nxe - 4; ++i) {
            size_t c = (size_t)i + (size_t)j * nxe;          /* x-face (i+1/2, j) */
            double a4_vx = 0.0, a4_bx = 0.0;
            if (P->hd_cross_on) {
                a4_vx = ((Gy[Q_VX][c - nxe] + Gy[Q_VX][c]) + (Gy[Q_VX][c + 1 - nxe] + Gy[Q_VX][c + 1])) / 4.0;
                a4_bx = ((Gy[Q_B][c - nxe] + Gy[Q_B][c]) + (Gy[Q_B][c + 1 - nxe] + Gy[Q_B][c + 1])) / 4.0;
            }
            double rf = 0.5 * (rho[c] + rho[c + 1]);
            double vxf = 0.5 * (vx[c] + vx[c + 1]);
            double vyf = 0.5 * (vy[c] + vy[c + 1]);
            double byf = 0.5 * (byT[c] + byT[c + 1]);
            double txx = rf * Gx[Q_VX][c];
            double txy = 0.5 * rf * (Gx[Q_VY][c] + a4_vx);
            double ez = Gx[Q_B][c] - a4_bx;
            Hx[F_RHO][c] = Gx[Q_RHO][c];
            Hx[F_MX][c] = txx;
            Hx[F_MY][c] = txy;
            Hx[F_E][c] = (Gx[Q_EPS][c] + (vxf * txx + vyf * txy)) + byf * ez;
            Hx[F_BX][c] = 0.0;
            Hx[F_BY][c] = ez;
        }
    }
#pragma omp parallel for schedule(static)
    for (int j = 2; j <= nye - 4; ++j) {
        for (int i = 3; i <= nxe - 4; ++i) {
            size_t c = (size_t)i + (size_t)j * nxe;          /* y-face (i, j+1/2) */
            double a4_vy = 0.0, a4_by = 0.0;
            if (P->hd_cross_on) {
                a4_vy = ((Gx[Q_VY][c - 1] + Gx[Q_VY][c]) + (Gx[Q_VY][c - 1 + nxe] + Gx[Q_VY][c + nxe])) / 4.0;
                a4_by = ((Gx[Q_B][c - 1] + Gx[Q_B][c]) + (Gx[Q_B][c - 1 + nxe] + Gx[Q_B][c + nxe])) / 4.0;
            }
            double rf = 0.5 * (rho[c] + rho[c + nxe]);
            double vxf = 0.5 * (vx[c] + vx[c + nxe]);
            double vyf = 0.5 * (vy[c] + vy[c + nxe]);
            double bxf = 0.5 * (bxT[c] + bxT[c + nxe]);
            double tyy = rf * Gy[Q_VY][c];
            double tyx = 0.5 * rf * (Gy[Q_VX][c] + a4_vy);
            double ez = a4_by - Gy[Q_B][c];
            Hy[F_RHO][c] = Gy[Q_RHO][c];
            Hy[F_MX][c] = tyx;
            Hy[F_MY][c] = tyy;
            Hy[F_E][c] = (Gy[Q_EPS][c] + (vyf * tyy + vxf * tyx)) - bxf * ez;
            Hy[F_BX][c] = -ez;
            Hy[F_BY][c] = 0.0;
        }
    }

    /* 4d. K_HD = divergence of the face fluxes; L = K_ideal + K_HD */
#pragma omp parallel for schedule(static)
    for (int j = G; j < nye - G; ++j) {
        for (int i = G; i < nxe - G; ++i) {
            size_t c = (size_t)i + (size_t)j * nxe;
            for (int k = 0; k < NF; ++k) {
                double hd = over(pf, Hx[k][c] - Hx[k][c - 1], dx, idx) + over(pf, Hy[k][c] - Hy[k][c - nxe], dy, idy);
                K[k][c] = K[k][c] + hd;
            }
        }
    }

done:
    free(rho); free(vx); free(vy); free(bxT); free(byT); free(pkt); free(ptt); free(epst); free(ptb);
    for (int k = 0; k < NF; ++k) { free(Fx[k]); free(Fy[k]); free(Hx[k]); free(Hy[k]); }
    free(s);
    for (int k = 0; k < 5; ++k) { free(Gx[k]); free(Gy[k]); }
    return rc;
}

static void make_rhs_par(const orc_cfg *c, rhs_par *P) {
    P->dx = (c->x1 - c->x0) / c->nx;
    P->dy = (c->y1 - c->y0) / c->ny;
    P->gamma = c->gamma;
    P->paper = c->form == ORC_FORM_PAPER;
    P->hd_on = c->hd_on;
    P->hd_cross_on = c->hd_cross_on;
    P->bg_on = c->background_on;
    for (int k = 0; k < 4; ++k) { P->c2[k] = c->c2[k]; P->cshk[k] = c->cshk[k]; }
    P->g[0] = c->g[0];
    P->g[1] = c->g[1];
    P->grav_on = c->g[0] != 0.0 || c->g[1] != 0.0;
    P->rext = NULL;
    P->rext_nx = c->nx;
    P->rext_ny = c->ny;
}

/* ------------------------------------------------------------------ */
/* wave speeds, CFL time step, physicality check                        */
/*   c_f = sqrt((gamma p_k + |B|^2) / rho)  (upper bound of fast speed) */
/*   c_d = max_cells (|v_d| + c_f); c_max = max over active d            */
/*   dt  = CFL min_d (h_d / c_d) over active d                           */
/* ------------------------------------------------------------------ */

static int wavespeed_ext(const orc_cfg *cfg, double *const U[NF], double *const BG[NB],
                         int nxe, int i0, int i1, int j0, int j1, double out[3]) {
    const int pf = cfg->form == ORC_FORM_PAPER;
    const double gm1 = cfg->gamma - 1.0;
    double cx = 0.0, cy = 0.0;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(max : cx, cy) reduction(| : bad)
    for (int j = j0; j < j1; ++j) {
        for (int i = i0; i < i1; ++i) {
            size_t c = (size_t)i + (size_t)j * nxe;
            double rb = 0.0, eb = 0.0, bxb = 0.0, byb = 0.0;
            if (cfg->background_on) { rb = BG[B_RHO][c]; eb = BG[B_E][c]; bxb = BG[B_BX][c]; byb = BG[B_BY][c]; }
            double rt = U[F_RHO][c], mx = U[F_MX][c], my = U[F_MY][c], et = U[F_E][c];
            double bxt = U[F_BX][c], byt = U[F_BY][c];
            double r = rb + rt;
            double ir = 1.0 / r;
            double ux = over(pf, mx, r, ir), uy = over(pf, my, r, ir);
            double kin = 0.5 * (mx * ux + my * uy);
            double bbdot = bxb * bxt + byb * byt;
            double bt2 = bxt * bxt + byt * byt;
            double pkt = gm1 * (((et - kin) - bbdot) - 0.5 * bt2);
            double b2b = bxb * bxb + byb * byb;
            double pkb = gm1 * (eb - 0.5 * b2b);
            double pk = pkb + pkt;
            double bx = bxb + bxt, by = byb + byt;
            double cf = sqrt(over(pf, cfg->gamma * pk + (bx * bx + by * by), r, ir));
            int finite = isfinite(rt) && isfinite(mx) && isfinite(my) && isfinite(et) &&
                         isfinite(bxt) && isfinite(byt) && isfinite(cf);
            if (!(r > 0.0) || !(pk > 0.0) || !finite) { bad = 1; continue; }
            cx = dmax(cx, fabs(ux) + cf);
            cy = dmax(cy, fabs(uy) + cf);
        }
    }
    out[0] = cx; out[1] = cy;
    {
        int ax = cfg->nx > 1, ay = cfg->ny > 1;
        out[2] = (ax && ay) ? dmax(cx, cy) : (ax ? cx : cy);
    }
    return bad ? ORC_ENONPHYS : ORC_OK;
}

static double cfl_dt(const orc_cfg *cfg, const double c[3]) {
    double dx = (cfg->x1 - cfg->x0) / cfg->nx, dy = (cfg->y1 - cfg->y0) / cfg->ny;
    int ax = cfg->nx > 1, ay = cfg->ny > 1;
    double h;
    if (ax && ay) h = dmin(dx / c[0], dy / c[1]);
    else if (ax) h = dx / c[0];
    else h = dy / c[1];
    return cfg->cfl * h;
}

/* ------------------------------------------------------------------ */
/* full-domain state                                                    */
/* ------------------------------------------------------------------ */

typedef struct {
    orc_cfg cfg;
    rhs_par par;
    int nx, ny, nxe, nye;
    block U, S, A, K[4];   /* A: low-storage form only; K[1..3]: paper form only */
    double *BG[NB];
} dom;

static void dom_free(dom *d) {
    block_free(&d->U); block_free(&d->S); block_free(&d->A);
    for (int s = 0; s < 4; ++s) block_free(&d->K[s]);
    for (int k = 0; k < NB; ++k) { free(d->BG[k]); d->BG[k] = NULL; }
}

static int dom_init(dom *d, const orc_cfg *cfg, double *const f[NF], double *const bg[NB]) {
    memset(d, 0, sizeof(*d));
    d->cfg = *cfg;
    make_rhs_par(cfg, &d->par);
    d->nx = cfg->nx; d->ny = cfg->ny;
    d->nxe = cfg->nx + 2 * G; d->nye = cfg->ny + 2 * G;
    int rc = block_alloc(&d->U, d->nxe, d->nye);
    if (!rc) rc = block_alloc(&d->S, d->nxe, d->nye);
    if (!rc) rc = block_alloc(&d->K[0], d->nxe, d->nye);
    if (cfg->form == ORC_FORM_PAPER) {
        for (int s = 1; s < 4 && !rc; ++s) rc = block_alloc(&d->K[s], d->nxe, d->nye);
    } else if (!rc) {
        rc = block_alloc(&d->A, d->nxe, d->nye);
    }
    if (!rc && cfg->background_on) {
        for (int k = 0; k < NB; ++k) {
            d->BG[k] = alloc0((size_t)d->nxe * d->nye);
            if (!d->BG[k]) { rc = ORC_ENOMEM; break; }
        }
    }
    if (rc) { dom_free(d); return rc; }
    for (int k = 0; k < NF; ++k)
        for (int j = 0; j < d->ny; ++j)
            memcpy(d->U.f[k] + (size_t)G + (size_t)(j + G) * d->nxe, f[k] + (size_t)j * d->nx,
                   sizeof(double) * d->nx);
    if (cfg->background_on) {
        for (int k = 0; k < NB; ++k) {
            for (int j = 0; j < d->ny; ++j)
                memcpy(d->BG[k] + (size_t)G + (size_t)(j + G) * d->nxe, bg[k] + (size_t)j * d->nx,
                       sizeof(double) * d->nx);
            fill_ghosts_one(d->BG[k], d->nx, d->ny, cfg->bc);
        }
    }
    return ORC_OK;
}

static void dom_out(const dom *d, double *const f[NF]) {
    for (int k = 0; k < NF; ++k)
        for (int j = 0; j < d->ny; ++j)
            memcpy(f[k] + (size_t)j * d->nx, d->U.f[k] + (size_t)G + (size_t)(j + G) * d->nxe,
                   sizeof(double) * d->nx);
}

static void fill_block(dom *d, block *b) {
    for (int k = 0; k < NF; ++k) fill_ghosts_one(b->f[k], d->nx, d->ny, d->cfg.bc);
}

/* One classic RK4 step (section 2).  With K_s the right-hand side of the
 * s-th stage input (the halo refilled before every L):
 *   K1 = L(U),  K2 = L(U + dt/2 K1),  K3 = L(U + dt/2 K2),  K4 = L(U + dt K3)
 *   U+ = U + dt/6 (K1 + 2 K2 + 2 K3 + K4)
 * The paper form keeps the four K and combines them as written.  The
 * low-storage form builds the same stage inputs and folds the combine into
 *   A = 2U + ((S1 - U) + dt K2)       (stage 2, while S1 is still held)
 *   U+ = S3 + (A - 2 S3)/3 + dt/6 K4  (stage 4)
 * which is the same polynomial in dt (A - 2 S3 = dt (K1 + 2 K2 - 2 K3)/2, so
 * U+ = U + dt K3 + dt (K1 + 2 K2 - 2 K3)/6 + dt K4/6). */
static void rk_stage_input(dom *d, int stage, double dt, const block *K) {
    /* S_stage = U + c dt K_stage, c = 1/2, 1/2, 1 for stages 1-3 */
    const double c = stage == 3 ? dt : 0.5 * dt;
    for (int k = 0; k < NF; ++k) {
        const double *u = d->U.f[k], *kk = K->f[k];
        double *s = d->S.f[k], *acc = d->A.f[k];
#pragma omp parallel for schedule(static)
        for (int j = G; j < d->nye - G; ++j)
            for (int i = G; i < d->nxe - G; ++i) {
                size_t q = (size_t)i + (size_t)j * d->nxe;
                if (stage == 2 && acc) acc[q] = (u[q] + u[q]) + ((s[q] - u[q]) + dt * kk[q]);
                s[q] = u[q] + c * kk[q];
            }
    }
}

static void rk_final_paper(dom *d, double dt) {
    const double dt6 = dt / 6.0;
    for (int k = 0; k < NF; ++k) {
        double *u = d->U.f[k];
        const double *k1 = d->K[0].f[k], *k2 = d->K[1].f[k], *k3 = d->K[2].f[k], *k4 = d->K[3].f[k];
#pragma omp parallel for schedule(static)
        for (int j = G; j < d->nye - G; ++j)
            for (int i = G; i < d->nxe - G; ++i) {
                size_t q = (size_t)i + (size_t)j * d->nxe;
                u[q] = u[q] + dt6 * (((k1[q] + 2.0 * k2[q]) + 2.0 * k3[q]) + k4[q]);
            }
    }
}

static void rk_final_lowstore(dom *d, double dt) {
    const double dt6 = dt / 6.0, third = 1.0 / 3.0;
    for (int k = 0; k < NF; ++k) {
        double *u = d->U.f[k];
        const double *s = d->S.f[k], *acc = d->A.f[k], *kk = d->K[0].f[k];
#pragma omp parallel for schedule(static)
        for (int j = G; j < d->nye - G; ++j)
            for (int i = G; i < d->nxe - G; ++i) {
                size_t q = (size_t)i + (size_t)j * d->nxe;
                u[q] = (s[q] + (acc[q] - (s[q] + s[q])) * third) + dt6 * kk[q];
            }
    }
}

static int dom_step(dom *d, double dt, double cmax) {
    const int paper = d->cfg.form == ORC_FORM_PAPER;
    for (int stage = 1; stage <= 4; ++stage) {
        block *in = stage == 1 ? &d->U : &d->S;
        block *K = paper ? &d->K[stage - 1] : &d->K[0];
        fill_block(d, in);
        int rc = rhs_block(d->nxe, d->nye, in->f, d->BG, &d->par, cmax, K->f);
        if (rc) return rc;
        if (stage < 4) rk_stage_input(d, stage, dt, K);
    }
    if (paper) rk_final_paper(d, dt);
    else rk_final_lowstore(d, dt);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* exported entry points                                                */
/* ------------------------------------------------------------------ */

/* Advance up to nsteps RK4 steps.  t_end <= 0: no clamp.  Otherwise
 * dt = min(dt, t_end - t) and the run stops once t_end - t <= 1e-12 t_end.
 * The time step and c_max are taken from the state at the start of each
 * step.  A non-physical start state stops the run with ORC_ENONPHYS and
 * leaves that state in f.  info[0] = last dt, info[1] = last c_max,
 * info[2] = c_x, info[3] = c_y of the last step. */
static int advance_impl(const orc_cfg *cfg, double *const f[NF], double *const bg[NB], int nsteps,
                        double t_end, double *t, int *steps_done, double info[4], const float *rext) {
    if (!cfg_ok(cfg) || !f || !t || nsteps < 0) return ORC_EINVAL;
    if (cfg->background_on && !bg) return ORC_EINVAL;
    dom d;
    int rc = dom_init(&d, cfg, f, bg);
    if (rc) return rc;
    d.par.rext = rext;
    int done = 0;
    for (int step = 0; step < nsteps; ++step) {
        if (t_end > 0.0 && t_end - *t <= 1e-12 * t_end) break;
        double c[3];
        rc = wavespeed_ext(cfg, d.U.f, d.BG, d.nxe, G, G + d.nx, G, G + d.ny, c);
        if (rc) break;
        double dt = cfl_dt(cfg, c);
        if (t_end > 0.0) dt = dmin(dt, t_end - *t);
        if (info) { info[0] = dt; info[1] = c[2]; info[2] = c[0]; info[3] = c[1]; }
        rc = dom_step(&d, dt, c[2]);
        if (rc) break;
        *t = *t + dt;
        ++done;
    }
    dom_out(&d, f);
    dom_free(&d);
    if (steps_done) *steps_done = done;
    return rc;
}

int orc_advance(const orc_cfg *cfg, double *const f[NF], double *const bg[NB], int nsteps,
                double t_end, double *t, int *steps_done, double info[4]) {
    return advance_impl(cfg, f, bg, nsteps, t_end, t, steps_done, info, NULL);
}

/* As orc_advance, with the hyper-diffusion coefficient ratios taken from
 * rext (10 planes of nx*ny, see rhs_par) wherever a value is not negative,
 * held fixed for the whole run.  Doubly periodic domains without a
 * background only. */
int orc_advance_ext(const orc_cfg *cfg, double *const f[NF], int nsteps, double t_end, double *t,
                    int *steps_done, double info[4], const float *rext) {
    if (!cfg_ok(cfg) || !rext || cfg->background_on) return ORC_EINVAL;
    for (int s = 0; s < 4; ++s) if (cfg->bc[s] != ORC_PERIODIC) return ORC_EINVAL;
    return advance_impl(cfg, f, NULL, nsteps, t_end, t, steps_done, info, rext);
}

/* Wave speeds of a state: out = {c_x, c_y, c_max, dt}.  Returns
 * ORC_ENONPHYS if any cell has rho <= 0, p_k <= 0 or a non-finite value. */
int orc_wavespeed(const orc_cfg *cfg, double *const f[NF], double *const bg[NB], double out[4]) {
    if (!cfg_ok(cfg) || !f || !out) return ORC_EINVAL;
    if (cfg->background_on && !bg) return ORC_EINVAL;
    double c[3];
    int rc = wavespeed_ext(cfg, f, bg, cfg->nx, 0, cfg->nx, 0, cfg->ny, c);
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2];
    out[3] = cfl_dt(cfg, c);
    return rc;
}

/* Right-hand side L(U) on the interior (halo filled per cfg->bc) with a
 * given c_max for the hyper-diffusion coefficients. */
static int rhs_impl(const orc_cfg *cfg, double *const f[NF], double *const bg[NB], double cmax,
                    double *const K[NF], const float *rext) {
    if (!cfg_ok(cfg) || !f || !K) return ORC_EINVAL;
    if (cfg->background_on && !bg) return ORC_EINVAL;
    dom d;
    int rc = dom_init(&d, cfg, f, bg);
    if (rc) return rc;
    d.par.rext = rext;
    fill_block(&d, &d.U);
    rc = rhs_block(d.nxe, d.nye, d.U.f, d.BG, &d.par, cmax, d.K[0].f);
    if (!rc)
        for (int k = 0; k < NF; ++k)
            for (int j = 0; j < d.ny; ++j)
                memcpy(K[k] + (size_t)j * d.nx, d.K[0].f[k] + (size_t)G + (size_t)(j + G) * d.nxe,
                       sizeof(double) * d.nx);
    dom_free(&d);
    return rc;
}

int orc_rhs(const orc_cfg *cfg, double *const f[NF], double *const bg[NB], double cmax,
            double *const K[NF]) {
    return rhs_impl(cfg, f, bg, cmax, K, NULL);
}

/* As orc_rhs with externally supplied coefficient ratios (see orc_advance_ext). */
int orc_rhs_ext(const orc_cfg *cfg, double *const f[NF], double cmax, double *const K[NF],
                const float *rext) {
    if (!cfg_ok(cfg) || !rext || cfg->background_on) return ORC_EINVAL;
    for (int s = 0; s < 4; ++s) if (cfg->bc[s] != ORC_PERIODIC) return ORC_EINVAL;
    return rhs_impl(cfg, f, NULL, cmax, K, rext);
}

/* One RK4 step on a patch of a larger 2-D domain whose outer 12 cells are
 * supplied by the caller (no boundary condition is applied): each stage
 * consumes 3 cells of margin.  dt and c_max are those of the whole domain.
 * f: px*py fields (row-major), bg: px*py background (or NULL),
 * out: (px-24)*(py-24) fields. */
int orc_step_patch(const orc_cfg *cfg, int px, int py, double *const f[NF], double *const bg[NB],
                   double dt, double cmax, double *const out[NF]) {
    if (!cfg || px < 25 || py < 25 || !f || !out) return ORC_EINVAL;
    if (cfg->background_on && !bg) return ORC_EINVAL;
    rhs_par P;
    make_rhs_par(cfg, &P);
    int rc = ORC_OK;
    /* nested blocks: level L has size (px - 2 G L) x (py - 2 G L), offset G L */
    block U0, Sb[4], Kb[4];
    double *BGl[4][NB];
    memset(BGl, 0, sizeof(BGl));
    memset(Sb, 0, sizeof(Sb)); memset(Kb, 0, sizeof(Kb));
    rc = block_alloc(&U0, px, py);
    for (int l = 0; l < 4 && !rc; ++l) {
        rc = block_alloc(&Sb[l], px - 2 * G * l, py - 2 * G * l);
        if (!rc) rc = block_alloc(&Kb[l], px - 2 * G * l, py - 2 * G * l);
        if (!rc && cfg->background_on) {
            for (int k = 0; k < NB; ++k) {
                BGl[l][k] = alloc0((size_t)(px - 2 * G * l) * (py - 2 * G * l));
                if (!BGl[l][k]) { rc = ORC_ENOMEM; break; }
            }
        }
    }
    if (rc) goto out;
    for (int k = 0; k < NF; ++k) memcpy(U0.f[k], f[k], sizeof(double) * (size_t)px * py);
    for (int l = 0; l < 4 && cfg->background_on; ++l) {
        int w = px - 2 * G * l, h = py - 2 * G * l, o = G * l;
        for (int k = 0; k < NB; ++k)
            for (int j = 0; j < h; ++j)
                for (int i = 0; i < w; ++i)
                    BGl[l][k][(size_t)i + (size_t)j * w] = bg[k][(size_t)(i + o) + (size_t)(j + o) * px];
    }
    /* stage inputs: level 0 is U itself; the combine follows dom_step's
     * arithmetic exactly in either form (S1, S2 [and A] from U, then S3,
     * then U+ from the four K [or from S3, A and K4]) */
    for (int k = 0; k < NF; ++k) memcpy(Sb[0].f[k], f[k], sizeof(double) * (size_t)px * py);
    {
        const double hdt = 0.5 * dt, dt6 = dt / 6.0, third = 1.0 / 3.0;
        /* accumulator A lives on the level-2 region (where K2 is known) */
        block Ab;
        rc = block_alloc(&Ab, px - 4 * G, py - 4 * G);
        if (rc) goto out;
        for (int l = 0; l < 4; ++l) {
            int w = px - 2 * G * l, h = py - 2 * G * l;
            rc = rhs_block(w, h, Sb[l].f, cfg->background_on ? BGl[l] : NULL, &P, cmax, Kb[l].f);
            if (rc) { block_free(&Ab); goto out; }
            int wn = w - 2 * G, hn = h - 2 * G, on = G * (l + 1);
            for (int k = 0; k < NF; ++k)
                for (int j = 0; j < hn; ++j)
                    for (int i = 0; i < wn; ++i) {
                        size_t cu = (size_t)(i + on) + (size_t)(j + on) * px;       /* U at this cell */
                        size_t ck = (size_t)(i + G) + (size_t)(j + G) * w;          /* K and S of level l */
                        double u = U0.f[k][cu], kk = Kb[l].f[k][ck];
                        if (l == 0) {
                            Sb[1].f[k][(size_t)i + (size_t)j * wn] = u + hdt * kk;
                        } else if (l == 1) {
                            double s1 = Sb[1].f[k][ck];
                            Sb[2].f[k][(size_t)i + (size_t)j * wn] = u + hdt * kk;
                            Ab.f[k][(size_t)i + (size_t)j * wn] = (u + u) + ((s1 - u) + dt * kk);
                        } else if (l == 2) {
                            Sb[3].f[k][(size_t)i + (size_t)j * wn] = u + dt * kk;
                        } else {
                            /* level 3 block is the S3 block; A sits on level 2 (offset G more);
                             * K of level m at this cell is at offset (4 - m) G in its block */
                            double r;
                            if (cfg->form == ORC_FORM_PAPER) {
                                double k1 = Kb[0].f[k][(size_t)(i + 4 * G) + (size_t)(j + 4 * G) * px];
                                double k2 = Kb[1].f[k][(size_t)(i + 3 * G) + (size_t)(j + 3 * G) * (px - 2 * G)];
                                double k3 = Kb[2].f[k][(size_t)(i + 2 * G) + (size_t)(j + 2 * G) * (px - 4 * G)];
                                r = u + dt6 * (((k1 + 2.0 * k2) + 2.0 * k3) + kk);
                            } else {
                                double s3 = Sb[3].f[k][ck];
                                double acc = Ab.f[k][(size_t)(i + 2 * G) + (size_t)(j + 2 * G) * (px - 4 * G)];
                                r = (s3 + (acc - (s3 + s3)) * third) + dt6 * kk;
                            }
                            out[k][(size_t)i + (size_t)j * wn] = r;
                        }
                    }
        }
        block_free(&Ab);
    }
out:
    block_free(&U0);
    for (int l = 0; l < 4; ++l) {
        block_free(&Sb[l]); block_free(&Kb[l]);
        for (int k = 0; k < NB; ++k) free(BGl[l][k]);
    }
    return rc;
}

/* pairwise sum of a contiguous run */
static double psum(const double *a, size_t n) {
    if (n <= 8) {
        double s = 0.0;
        for (size_t i = 0; i < n; ++i) s += a[i];
        return s;
    }
    size_t h = n / 2;
    return psum(a, h) + psum(a + h, n - h);
}

/* Conservation sums: sum over the interior of each evolved field times
 * dx dy, by pairwise summation in row-major order. */
int orc_sums(const orc_cfg *cfg, double *const f[NF], double sums[NF]) {
    if (!cfg_ok(cfg) || !f || !sums) return ORC_EINVAL;
    double dx = (cfg->x1 - cfg->x0) / cfg->nx, dy = (cfg->y1 - cfg->y0) / cfg->ny;
    for (int k = 0; k < NF; ++k) sums[k] = psum(f[k], (size_t)cfg->nx * cfg->ny) * (dx * dy);
    return ORC_OK;
}

/* The fourth-order central difference of a periodic line, with spacing h
 * (the same routine the right-hand side uses). */
int orc_deriv_line(int n, const double *q, double h, double *out) {
    if (n < 1 || !q || !out) return ORC_EINVAL;
    double *e = alloc0((size_t)n + 2 * G);
    if (!e) return ORC_ENOMEM;
    for (int i = -G; i < n + G; ++i) e[i + G] = q[imod(i, n)];
    for (int i = 0; i < n; ++i) out[i] = d4(1, e, i + G, 1, 12.0 * h, 0.0);
    free(e);
    return ORC_OK;
}

/* Hyper-diffusion ratio R on the n faces i+1/2 (i = 0..n-1) of a periodic
 * line (the same routine the right-hand side uses). */
int orc_hd_ratio_line(int n, const double *q, double *R) {
    if (n < 1 || !q || !R) return ORC_EINVAL;
    double *e = alloc0((size_t)n + 2 * G + 2);
    if (!e) return ORC_ENOMEM;
    for (int i = -G; i < n + G + 1; ++i) e[i + G] = q[imod(i, n)];
    for (int i = 0; i < n; ++i) R[i] = hd_ratio(e, i + G, 1);
    free(e);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* coefficient-ratio fields of a state and the surrogate check          */
/* ------------------------------------------------------------------ */

/* Plain hyper-diffusion ratios of every face of a 2-D state (halo filled
 * per cfg->bc): R has 10 planes of nx*ny values, planes 0-4 the x-face sets
 * {rho~, eps~, v_x, v_y, B~_y} at faces (i+1/2, j), planes 5-9 the y-face
 * sets {rho~, eps~, v_x, v_y, B~_x} at faces (i, j+1/2).  The primitive
 * quantities are formed exactly as in the right-hand side.  D1 (optional,
 * same layout) receives the first difference of each set at each face. */
int orc_hd_face_fields(const orc_cfg *cfg, double *const f[NF], double *const bg[NB], double *R, double *D1) {
    if (!cfg_ok(cfg) || !f || !R || cfg->nx < 2 || cfg->ny < 2) return ORC_EINVAL;
    if (cfg->background_on && !bg) return ORC_EINVAL;
    dom d;
    int rc = dom_init(&d, cfg, f, bg);
    if (rc) return rc;
    fill_block(&d, &d.U);
    const size_t n = (size_t)d.nxe * d.nye;
    double *vx = alloc0(n), *vy = alloc0(n), *eps = alloc0(n);
    if (!vx || !vy || !eps) { rc = ORC_ENOMEM; goto out; }
    {
        const int pf = cfg->form == ORC_FORM_PAPER;
        const double gm1 = cfg->gamma - 1.0, igm1 = 1.0 / gm1;
        for (size_t c = 0; c < n; ++c) {
            double rb = 0.0, bxb = 0.0, byb = 0.0;
            if (cfg->background_on) { rb = d.BG[B_RHO][c]; bxb = d.BG[B_BX][c]; byb = d.BG[B_BY][c]; }
            double rt = d.U.f[F_RHO][c], mx = d.U.f[F_MX][c], my = d.U.f[F_MY][c], et = d.U.f[F_E][c];
            double bxt = d.U.f[F_BX][c], byt = d.U.f[F_BY][c];
            double r = rb + rt;
            double ir = 1.0 / r;
            double ux = over(pf, mx, r, ir), uy = over(pf, my, r, ir);
            double kin = 0.5 * (mx * ux + my * uy);
            double bbdot = bxb * bxt + byb * byt;
            double bt2 = bxt * bxt + byt * byt;
            double pk = gm1 * (((et - kin) - bbdot) - 0.5 * bt2);
            vx[c] = ux; vy[c] = uy; eps[c] = over(pf, pk, gm1, igm1);
        }
        double *qx[5] = {d.U.f[F_RHO], eps, vx, vy, d.U.f[F_BY]};
        double *qy[5] = {d.U.f[F_RHO], eps, vx, vy, d.U.f[F_BX]};
        const size_t pl = (size_t)d.nx * d.ny;
        for (int j = 0; j < d.ny; ++j)
            for (int i = 0; i < d.nx; ++i) {
                ptrdiff_t c = (ptrdiff_t)(i + G) + (ptrdiff_t)(j + G) * d.nxe;
                for (int k = 0; k < 5; ++k) {
                    R[(size_t)k * pl + (size_t)j * d.nx + i] = hd_ratio(qx[k], c, 1);
                    R[(size_t)(5 + k) * pl + (size_t)j * d.nx + i] = hd_ratio(qy[k], c, d.nxe);
                    if (D1) {
                        D1[(size_t)k * pl + (size_t)j * d.nx + i] = d1_at(qx[k], c, 1);
                        D1[(size_t)(5 + k) * pl + (size_t)j * d.nx + i] = d1_at(qy[k], c, d.nxe);
                    }
                }
            }
    }
out:
    free(vx); free(vy); free(eps);
    dom_free(&d);
    return rc;
}

int orc_hd_ratio_fields(const orc_cfg *cfg, double *const f[NF], double *const bg[NB], double *R) {
    return orc_hd_face_fields(cfg, f, bg, R, NULL);
}

/* The surrogate check: the interior is cut into tiles of tile x tile cells
 * (ragged at the high edges), tile (tx, ty) covering cells
 * [tx*tile, ...) x [ty*tile, ...), row-major tile index ty*ntx + tx.  Each
 * face value r of the 10 planes gets an error e:
 *   metric 0 (ratio): e = |r - R_plain|;
 *   metric 1 (flux):  e = |r - R_plain| |d1| / D, d1 the face's first
 *     difference of that set and D the largest |d1| of the plane over the
 *     whole domain (e = 0 when D = 0): the error of the hyper-diffusive flux
 *     the value produces (proportional to R d1), relative to the largest
 *     |d1| of that quantity.
 * A tile falls back when any of its values is not finite or has
 * NOT(e <= bound).  mask (ntx*nty ints): 1 = fallback.  err_used = max e over
 * the tiles that keep the prediction, err_all = max over every finite e.
 * Returns the number of fallback tiles in *nfall. */
int orc_hd_check(const orc_cfg *cfg, double *const f[NF], const float *rnn, double bound, int tile, int metric,
                 int *mask, int *nfall, double *err_used, double *err_all) {
    if (!cfg_ok(cfg) || !f || !rnn || !mask || tile < 1 || cfg->background_on) return ORC_EINVAL;
    if (metric != 0 && metric != 1) return ORC_EINVAL;
    const int nx = cfg->nx, ny = cfg->ny;
    const size_t pl = (size_t)nx * ny;
    double *R = alloc0(10 * pl), *D1 = alloc0(10 * pl);
    if (!R || !D1) { free(R); free(D1); return ORC_ENOMEM; }
    int rc = orc_hd_face_fields(cfg, f, NULL, R, D1);
    if (rc) { free(R); free(D1); return rc; }
    double Dk[10];
    for (int k = 0; k < 10; ++k) {
        Dk[k] = 0.0;
        for (size_t c = 0; c < pl; ++c) Dk[k] = dmax(Dk[k], fabs(D1[(size_t)k * pl + c]));
    }
    const int ntx = (nx + tile - 1) / tile, nty = (ny + tile - 1) / tile;
    double eu = 0.0, ea = 0.0;
    int nf = 0;
    for (int ty = 0; ty < nty; ++ty)
        for (int tx = 0; tx < ntx; ++tx) {
            int bad = 0;
            double et = 0.0;
            for (int k = 0; k < 10; ++k)
                for (int j = ty * tile; j < ny && j < (ty + 1) * tile; ++j)
                    for (int i = tx * tile; i < nx && i < (tx + 1) * tile; ++i) {
                        size_t c = (size_t)k * pl + (size_t)j * nx + i;
                        double r = (double)rnn[c];
                        double e = fabs(r - R[c]);
                        if (metric == 1) e = Dk[k] > 0.0 ? (e * fabs(D1[c])) / Dk[k] : 0.0;
                        if (!isfinite(r) || !(e <= bound)) bad = 1;
                        if (isfinite(e)) et = dmax(et, e);
                    }
            mask[ty * ntx + tx] = bad;
            nf += bad;
            ea = dmax(ea, et);
            if (!bad) eu = dmax(eu, et);
        }
    if (nfall) *nfall = nf;
    if (err_used) *err_used = eu;
    if (err_all) *err_all = ea;
    free(R);
    free(D1);
    return ORC_OK;
}
