/*
 * sacx_oracle3d.c -- plain FP64 CPU oracle of the SAC/SMAUG+ MHD scheme in
 * three dimensions.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite and the CPU-baseline leg of
 * the benchmark may load this library.  The product path (the HIP library)
 * never calls it, links it or shares code with it.
 *
 * The scheme is the two-dimensional one of sacx_oracle.c carried to three
 * dimensions (the paper states the code is implemented in 3-D; sections 2
 * and 8): eight evolved fields rho~, m_x, m_y, m_z, e~, B~_x, B~_y, B~_z, no
 * background (every configuration here has a zero background), ideal
 * fluxes differenced with the fourth-order central difference along each of
 * x, y, z, hyper-diffusion on every face with the coefficient ratio of third
 * to first differences along the face normal, and classic RK4 with the CFL
 * time step of the three directions.
 *
 * Written for obviousness: full-array passes with plain loops, in the order
 * the scheme is defined.  Where a sum runs over directions it runs x, y, z;
 * where a face sums over the other directions it takes its own direction
 * first, then the others in x, y, z order.  With that order a state that
 * does not vary along one direction (and has no velocity or field component
 * along it) gives, bit for bit, the two-dimensional oracle's result in the
 * other two: the CPU tests pin this oracle to the 2-D one that way, in all
 * three planes.
 *
 * Build with -O2 -ffp-contract=off (no fast-math).  OpenMP distributes
 * independent planes only.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define G 3
#define NF 8

enum { F_RHO = 0, F_MX = 1, F_MY = 2, F_MZ = 3, F_E = 4, F_BX = 5, F_BY = 6, F_BZ = 7 };
enum { C_RHO = 0, C_EPS = 1, C_V = 2, C_B = 3 };
enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENONPHYS = -4, ORC_ENOMEM = -7 };
enum { ORC_PERIODIC = 0, ORC_OPEN = 1 };
/* the two arithmetic forms of sacx_oracle.c: the paper's (classic RK4
 * combine, divisions as divisions; the definition) and the four-array
 * arrangement with reciprocals */
enum { ORC_FORM_PAPER = 0, ORC_FORM_LOWSTORE = 1 };

typedef struct {
    int nx, ny, nz;
    double x0, x1, y0, y1, z0, z1;
    double gamma, cfl;
    int hd_on, hd_cross_on;
    double c2[4];   /* rho, eps, v, B */
    double cshk[4]; /* rho, eps, v, B */
    int bc[6];      /* x-, x+, y-, y+, z-, z+ */
    int form;
} orc3_cfg;

static double dmax(double a, double b) { return a > b ? a : b; }
static double dmin(double a, double b) { return a < b ? a : b; }
static int imod(int i, int n) { int r = i % n; return r < 0 ? r + n : r; }
static int iclamp(int i, int n) { return i < 0 ? 0 : (i >= n ? n - 1 : i); }
static double *alloc0(size_t n) { return (double *)calloc(n ? n : 1, sizeof(double)); }
static double over(int paper, double x, double d, double inv_d) { return paper ? x / d : x * inv_d; }

static int cfg_ok(const orc3_cfg *c) {
    if (!c || c->nx < 1 || c->ny < 1 || c->nz < 1) return 0;
    if ((c->nx > 1) + (c->ny > 1) + (c->nz > 1) < 1) return 0;
    if (!(c->x1 > c->x0) || !(c->y1 > c->y0) || !(c->z1 > c->z0)) return 0;
    if (!(c->gamma > 1.0) || !(c->cfl > 0.0)) return 0;
    if (c->form != ORC_FORM_PAPER && c->form != ORC_FORM_LOWSTORE) return 0;
    for (int s = 0; s < 6; ++s)
        if (c->bc[s] != ORC_PERIODIC && c->bc[s] != ORC_OPEN) return 0;
    for (int d = 0; d < 3; ++d)
        if ((c->bc[2 * d] == ORC_PERIODIC) != (c->bc[2 * d + 1] == ORC_PERIODIC)) return 0;
    return 1;
}

/* extended (ghosted) box */
typedef struct {
    int nx, ny, nz;      /* interior */
    int ex, ey, ez;      /* extended = interior + 2 G */
    size_t n;
    ptrdiff_t sy, sz;    /* strides of y and z */
} box;

static box make_box(int nx, int ny, int nz) {
    box b;
    b.nx = nx; b.ny = ny; b.nz = nz;
    b.ex = nx + 2 * G; b.ey = ny + 2 * G; b.ez = nz + 2 * G;
    b.n = (size_t)b.ex * b.ey * b.ez;
    b.sy = b.ex;
    b.sz = (ptrdiff_t)b.ex * b.ey;
    return b;
}

static size_t at(const box *b, int i, int j, int k) {   /* extended indices */
    return (size_t)i + (size_t)j * b->sy + (size_t)k * b->sz;
}

/* ghosts: periodic images or zero-gradient copies; x over the interior
 * rows and planes, then y over the padded x width, then z over the padded
 * x and y extents (so edges and corners are filled) */
static void fill_ghosts(const box *b, double *a, const int bc[6]) {
    const int nx = b->nx, ny = b->ny, nz = b->nz;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j) {
            for (int i = -G; i < 0; ++i) {
                int s = bc[0] == ORC_PERIODIC ? imod(i, nx) : iclamp(i, nx);
                a[at(b, i + G, j + G, k + G)] = a[at(b, s + G, j + G, k + G)];
            }
            for (int i = nx; i < nx + G; ++i) {
                int s = bc[1] == ORC_PERIODIC ? imod(i, nx) : iclamp(i, nx);
                a[at(b, i + G, j + G, k + G)] = a[at(b, s + G, j + G, k + G)];
            }
        }
    for (int k = 0; k < nz; ++k)
        for (int i = -G; i < nx + G; ++i) {
            for (int j = -G; j < 0; ++j) {
                int s = bc[2] == ORC_PERIODIC ? imod(j, ny) : iclamp(j, ny);
                a[at(b, i + G, j + G, k + G)] = a[at(b, i + G, s + G, k + G)];
            }
            for (int j = ny; j < ny + G; ++j) {
                int s = bc[3] == ORC_PERIODIC ? imod(j, ny) : iclamp(j, ny);
                a[at(b, i + G, j + G, k + G)] = a[at(b, i + G, s + G, k + G)];
            }
        }
    for (int j = -G; j < ny + G; ++j)
        for (int i = -G; i < nx + G; ++i) {
            for (int k = -G; k < 0; ++k) {
                int s = bc[4] == ORC_PERIODIC ? imod(k, nz) : iclamp(k, nz);
                a[at(b, i + G, j + G, k + G)] = a[at(b, i + G, j + G, s + G)];
            }
            for (int k = nz; k < nz + G; ++k) {
                int s = bc[5] == ORC_PERIODIC ? imod(k, nz) : iclamp(k, nz);
                a[at(b, i + G, j + G, k + G)] = a[at(b, i + G, j + G, s + G)];
            }
        }
}

/* fourth-order central difference along stride st (section 2):
 *   D f = [8 (f_{+1} - f_{-1}) - (f_{+2} - f_{-2})] / (12 h) */
static double d4(int paper, const double *f, size_t c, ptrdiff_t st, double h12, double inv12h) {
    return over(paper, 8.0 * (f[c + st] - f[c - st]) - (f[c + 2 * st] - f[c - 2 * st]), h12, inv12h);
}

/* hyper-diffusion ratio at the face between c and c + st (section 2:
 * third- over first-order differences; the 3-face / 5-face maxima reading) */
static double d1_at(const double *q, size_t c, ptrdiff_t st) { return q[c + st] - q[c]; }
static double d3_at(const double *q, size_t c, ptrdiff_t st) {
    return (q[c + 2 * st] - q[c - st]) - 3.0 * (q[c + st] - q[c]);
}
static double hd_ratio(const double *q, size_t c, ptrdiff_t st) {
    double n = 0.0, m = 0.0;
    for (int k = -1; k <= 1; ++k) n = dmax(n, fabs(d3_at(q, c + k * st, st)));
    for (int k = -2; k <= 2; ++k) m = dmax(m, fabs(d1_at(q, c + k * st, st)));
    return m > 0.0 ? n / m : 0.0;
}

typedef struct {
    double h[3];
    double gamma;
    int paper, hd_on, hd_cross_on;
    double c2[4], cshk[4];
} rhs_par;

/* quantity sets of the face fluxes: index of each quantity in the per-
 * direction G arrays.  Along direction d the sets are rho~, eps~, v_x, v_y,
 * v_z and the two field components across d. */
enum { Q_RHO = 0, Q_EPS = 1, Q_V = 2 /* + component */, Q_B = 5 /* + slot of the component */, NQ = 7 };

/* slot of field component k (k != d) among the two field sets of direction
 * d, in x, y, z order */
static int bslot(int d, int k) { return Q_B + ((k < d) ? k : k - 1); }

/* L(S) on the box's interior; every other entry of K is zero. */
static int rhs_box(const box *B, double *const S[NF], const rhs_par *P, double cmax, double *const K[NF]) {
    const size_t n = B->n;
    const int pf = P->paper;
    const double gm1 = P->gamma - 1.0, igm1 = 1.0 / gm1;
    const ptrdiff_t st[3] = {1, B->sy, B->sz};
    double h12[3], i12[3], h2[3], i2[3], ih[3];
    for (int d = 0; d < 3; ++d) {
        h12[d] = 12.0 * P->h[d]; i12[d] = 1.0 / h12[d];
        h2[d] = 2.0 * P->h[d]; i2[d] = 1.0 / h2[d];
        ih[d] = 1.0 / P->h[d];
    }
    const int ex = B->ex, ey = B->ey, ez = B->ez;
    int rc = ORC_OK;

    double *rho = alloc0(n), *v[3], *bT[3], *ptt = alloc0(n), *epst = alloc0(n);
    double *F[3][NF];
    double *s = NULL, *Gf[3][NQ], *H[3][NF];
    memset(Gf, 0, sizeof(Gf));
    memset(H, 0, sizeof(H));
    int ok = rho && ptt && epst;
    for (int d = 0; d < 3; ++d) {
        v[d] = alloc0(n); bT[d] = alloc0(n);
        ok = ok && v[d] && bT[d];
        for (int f = 0; f < NF; ++f) { F[d][f] = alloc0(n); ok = ok && F[d][f]; }
    }
    if (P->hd_on) {
        s = alloc0(n);
        ok = ok && s;
        for (int d = 0; d < 3; ++d) {
            for (int q = 0; q < NQ; ++q) { Gf[d][q] = alloc0(n); ok = ok && Gf[d][q]; }
            for (int f = 0; f < NF; ++f) { H[d][f] = alloc0(n); ok = ok && H[d][f]; }
        }
    }
    if (!ok) { rc = ORC_ENOMEM; goto done; }

    /* 1. primitives, pressures and ideal fluxes (section 2) */
#pragma omp parallel for schedule(static)
    for (int kk = 0; kk < ez; ++kk)
        for (int j = 0; j < ey; ++j)
            for (int i = 0; i < ex; ++i) {
                size_t c = at(B, i, j, kk);
                double r = S[F_RHO][c], mx = S[F_MX][c], my = S[F_MY][c], mz = S[F_MZ][c], et = S[F_E][c];
                double bx = S[F_BX][c], by = S[F_BY][c], bz = S[F_BZ][c];
                double ir = 1.0 / r;
                double ux = over(pf, mx, r, ir), uy = over(pf, my, r, ir), uz = over(pf, mz, r, ir);
                double kin = 0.5 * ((mx * ux + my * uy) + mz * uz);
                double b2 = (bx * bx + by * by) + bz * bz;
                double pk = gm1 * ((et - kin) - 0.5 * b2);
                double pt = pk + 0.5 * b2;
                rho[c] = r;
                v[0][c] = ux; v[1][c] = uy; v[2][c] = uz;
                bT[0][c] = bx; bT[1][c] = by; bT[2][c] = bz;
                ptt[c] = pt;
                epst[c] = over(pf, pk, gm1, igm1);
                double bv = (bx * ux + by * uy) + bz * uz;
                double ef = et + pt;
                /* F_d(rho) = m_d; F_d(m_k) = v_d m_k - B_d B_k (+ p_t on k = d);
                 * F_d(e) = v_d (e + p_t) - B_d (B.v); F_d(B_k) = v_d B_k - B_d v_k */
                F[0][F_RHO][c] = mx;
                F[0][F_MX][c] = (ux * mx - bx * bx) + pt;
                F[0][F_MY][c] = ux * my - bx * by;
                F[0][F_MZ][c] = ux * mz - bx * bz;
                F[0][F_E][c] = ux * ef - bx * bv;
                F[0][F_BX][c] = 0.0;
                F[0][F_BY][c] = ux * by - bx * uy;
                F[0][F_BZ][c] = ux * bz - bx * uz;
                F[1][F_RHO][c] = my;
                F[1][F_MX][c] = uy * mx - by * bx;
                F[1][F_MY][c] = (uy * my - by * by) + pt;
                F[1][F_MZ][c] = uy * mz - by * bz;
                F[1][F_E][c] = uy * ef - by * bv;
                F[1][F_BX][c] = uy * bx - by * ux;
                F[1][F_BY][c] = 0.0;
                F[1][F_BZ][c] = uy * bz - by * uz;
                F[2][F_RHO][c] = mz;
                F[2][F_MX][c] = uz * mx - bz * bx;
                F[2][F_MY][c] = uz * my - bz * by;
                F[2][F_MZ][c] = (uz * mz - bz * bz) + pt;
                F[2][F_E][c] = uz * ef - bz * bv;
                F[2][F_BX][c] = uz * bx - bz * ux;
                F[2][F_BY][c] = uz * by - bz * uy;
                F[2][F_BZ][c] = 0.0;
            }

    /* 2. K_ideal = -((D_x F_x + D_y F_y) + D_z F_z) */
#pragma omp parallel for schedule(static)
    for (int kk = 0; kk < ez; ++kk)
        for (int j = 0; j < ey; ++j)
            for (int i = 0; i < ex; ++i) {
                size_t c = at(B, i, j, kk);
                int in = i >= G && i < ex - G && j >= G && j < ey - G && kk >= G && kk < ez - G;
                for (int f = 0; f < NF; ++f) {
                    if (!in) { K[f][c] = 0.0; continue; }
                    double a = d4(pf, F[0][f], c, st[0], h12[0], i12[0]);
                    double b = d4(pf, F[1][f], c, st[1], h12[1], i12[1]);
                    double e = d4(pf, F[2][f], c, st[2], h12[2], i12[2]);
                    K[f][c] = -((a + b) + e);
                }
            }

    if (!P->hd_on) goto done;

    /* 3a. compression s = max(0, -div v), second-order centred */
#pragma omp parallel for schedule(static)
    for (int kk = 1; kk < ez - 1; ++kk)
        for (int j = 1; j < ey - 1; ++j)
            for (int i = 1; i < ex - 1; ++i) {
                size_t c = at(B, i, j, kk);
                double dv = (over(pf, v[0][c + st[0]] - v[0][c - st[0]], h2[0], i2[0]) +
                             over(pf, v[1][c + st[1]] - v[1][c - st[1]], h2[1], i2[1])) +
                            over(pf, v[2][c + st[2]] - v[2][c - st[2]], h2[2], i2[2]);
                s[c] = dmax(0.0, -dv);
            }

    /* 3b. face diffusion fluxes G_d(q) = nu_f(q) d1_f(q) / h_d,
     *     nu_f(q) = c2(q) h_d c_max R_f(q) + cshk(q) h_d^2 s_f,
     * on the faces (c, c + e_d) indexed by c: along d the faces of cells
     * 2 .. e_d - 4, across it cells 1 .. e - 2 */
    for (int d = 0; d < 3; ++d) {
        const double h = P->h[d];
        double *qs[NQ];
        int cls[NQ];
        qs[Q_RHO] = S[F_RHO]; cls[Q_RHO] = C_RHO;
        qs[Q_EPS] = epst; cls[Q_EPS] = C_EPS;
        for (int k = 0; k < 3; ++k) { qs[Q_V + k] = v[k]; cls[Q_V + k] = C_V; }
        for (int k = 0; k < 3; ++k)
            if (k != d) { qs[bslot(d, k)] = S[F_BX + k]; cls[bslot(d, k)] = C_B; }
        const int lo[3] = {d == 0 ? 2 : 1, d == 1 ? 2 : 1, d == 2 ? 2 : 1};
        const int hi[3] = {d == 0 ? ex - 4 : ex - 2, d == 1 ? ey - 4 : ey - 2, d == 2 ? ez - 4 : ez - 2};
#pragma omp parallel for schedule(static)
        for (int kk = lo[2]; kk <= hi[2]; ++kk)
            for (int j = lo[1]; j <= hi[1]; ++j)
                for (int i = lo[0]; i <= hi[0]; ++i) {
                    size_t c = at(B, i, j, kk);
                    double sf = dmax(s[c], s[c + st[d]]);
                    for (int q = 0; q < NQ; ++q) {
                        double R = hd_ratio(qs[q], c, st[d]);
                        double nu = P->c2[cls[q]] * h * cmax * R + P->cshk[cls[q]] * h * h * sf;
                        Gf[d][q][c] = over(pf, nu * d1_at(qs[q], c, st[d]), h, ih[d]);
                    }
                }
    }

    /* 3c. face fluxes (flux form): mass diffusion, hyper-viscous stress,
     * hyper-resistive e.m.f. and the energy they carry.  On the d-face
     * (c, c + e_d), for each other direction k:
     *   A4_dk[g] = ((g_k(c - e_k) + g_k(c)) + (g_k(c + e_d - e_k) + g_k(c + e_d))) / 4,
     *   the mean of the four k-faces around it;
     *   tau_dd = rho_f G_d(v_d),  tau_dk = rho_f/2 (G_d(v_k) + A4_dk[G_k(v_d)]),
     *   H_d(B_k) = G_d(B_k) - A4_dk[G_k(B_d)],
     *   H_d(e) = (G_d(eps) + (v_f . tau_d, own component first)) + (B_f . H_d(B), x, y, z). */
    for (int d = 0; d < 3; ++d) {
        const int lo[3] = {d == 0 ? 2 : 3, d == 1 ? 2 : 3, d == 2 ? 2 : 3};
        const int hi[3] = {ex - 4, ey - 4, ez - 4};
        const ptrdiff_t sd = st[d];
#pragma omp parallel for schedule(static)
        for (int kk = lo[2]; kk <= hi[2]; ++kk)
            for (int j = lo[1]; j <= hi[1]; ++j)
                for (int i = lo[0]; i <= hi[0]; ++i) {
                    size_t c = at(B, i, j, kk);
                    double a4v[3] = {0.0, 0.0, 0.0}, a4b[3] = {0.0, 0.0, 0.0};
                    if (P->hd_cross_on)
                        for (int k = 0; k < 3; ++k) {
                            if (k == d) continue;
                            const ptrdiff_t sk = st[k];
                            const double *gv = Gf[k][Q_V + d], *gb = Gf[k][bslot(k, d)];
                            a4v[k] = ((gv[c - sk] + gv[c]) + (gv[c + sd - sk] + gv[c + sd])) / 4.0;
                            a4b[k] = ((gb[c - sk] + gb[c]) + (gb[c + sd - sk] + gb[c + sd])) / 4.0;
                        }
                    double rf = 0.5 * (rho[c] + rho[c + sd]);
                    double vf[3], bf[3], tau[3], hb[3];
                    for (int k = 0; k < 3; ++k) {
                        vf[k] = 0.5 * (v[k][c] + v[k][c + sd]);
                        bf[k] = 0.5 * (bT[k][c] + bT[k][c + sd]);
                    }
                    for (int k = 0; k < 3; ++k) {
                        if (k == d) {
                            tau[k] = rf * Gf[d][Q_V + d][c];
                            hb[k] = 0.0;
                        } else {
                            tau[k] = 0.5 * rf * (Gf[d][Q_V + k][c] + a4v[k]);
                            hb[k] = Gf[d][bslot(d, k)][c] - a4b[k];
                        }
                    }
                    /* the two directions other than d, in x, y, z order */
                    const int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
                    double work = (vf[d] * tau[d] + vf[o1] * tau[o1]) + vf[o2] * tau[o2];
                    double mag = bf[o1] * hb[o1] + bf[o2] * hb[o2];
                    H[d][F_RHO][c] = Gf[d][Q_RHO][c];
                    H[d][F_MX][c] = tau[0];
                    H[d][F_MY][c] = tau[1];
                    H[d][F_MZ][c] = tau[2];
                    H[d][F_E][c] = (Gf[d][Q_EPS][c] + work) + mag;
                    H[d][F_BX][c] = hb[0];
                    H[d][F_BY][c] = hb[1];
                    H[d][F_BZ][c] = hb[2];
                }
    }

    /* 3d. K += divergence of the face fluxes, summed x, y, z */
#pragma omp parallel for schedule(static)
    for (int kk = G; kk < ez - G; ++kk)
        for (int j = G; j < ey - G; ++j)
            for (int i = G; i < ex - G; ++i) {
                size_t c = at(B, i, j, kk);
                for (int f = 0; f < NF; ++f) {
                    double a = over(pf, H[0][f][c] - H[0][f][c - st[0]], P->h[0], ih[0]);
                    double b = over(pf, H[1][f][c] - H[1][f][c - st[1]], P->h[1], ih[1]);
                    double e = over(pf, H[2][f][c] - H[2][f][c - st[2]], P->h[2], ih[2]);
                    K[f][c] = K[f][c] + ((a + b) + e);
                }
            }

done:
    free(rho); free(ptt); free(epst); free(s);
    for (int d = 0; d < 3; ++d) {
        free(v[d]); free(bT[d]);
        for (int f = 0; f < NF; ++f) { free(F[d][f]); free(H[d][f]); }
        for (int q = 0; q < NQ; ++q) free(Gf[d][q]);
    }
    return rc;
}

static void make_par(const orc3_cfg *c, rhs_par *P) {
    P->h[0] = (c->x1 - c->x0) / c->nx;
    P->h[1] = (c->y1 - c->y0) / c->ny;
    P->h[2] = (c->z1 - c->z0) / c->nz;
    P->gamma = c->gamma;
    P->paper = c->form == ORC_FORM_PAPER;
    P->hd_on = c->hd_on;
    P->hd_cross_on = c->hd_cross_on;
    for (int k = 0; k < 4; ++k) { P->c2[k] = c->c2[k]; P->cshk[k] = c->cshk[k]; }
}

/* wave speeds c_d = max(|v_d| + c_f), c_f = sqrt((gamma p_k + |B|^2) / rho),
 * over the interior of an extended box (or a plain array: G0 = 0) */
static int wavespeed_box(const orc3_cfg *cfg, double *const U[NF], const box *B, int g0, double c[4]) {
    const int pf = cfg->form == ORC_FORM_PAPER;
    const double gm1 = cfg->gamma - 1.0;
    double cx = 0.0, cy = 0.0, cz = 0.0;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(max : cx, cy, cz) reduction(| : bad)
    for (int k = 0; k < cfg->nz; ++k)
        for (int j = 0; j < cfg->ny; ++j)
            for (int i = 0; i < cfg->nx; ++i) {
                size_t q = g0 ? at(B, i + G, j + G, k + G) : (size_t)i + (size_t)cfg->nx * ((size_t)j + (size_t)cfg->ny * k);
                double r = U[F_RHO][q], mx = U[F_MX][q], my = U[F_MY][q], mz = U[F_MZ][q], et = U[F_E][q];
                double bx = U[F_BX][q], by = U[F_BY][q], bz = U[F_BZ][q];
                double ir = 1.0 / r;
                double ux = over(pf, mx, r, ir), uy = over(pf, my, r, ir), uz = over(pf, mz, r, ir);
                double kin = 0.5 * ((mx * ux + my * uy) + mz * uz);
                double b2 = (bx * bx + by * by) + bz * bz;
                double pk = gm1 * ((et - kin) - 0.5 * b2);
                double cf = sqrt(over(pf, cfg->gamma * pk + b2, r, ir));
                int finite = isfinite(r) && isfinite(mx) && isfinite(my) && isfinite(mz) && isfinite(et) &&
                             isfinite(bx) && isfinite(by) && isfinite(bz) && isfinite(cf);
                if (!(r > 0.0) || !(pk > 0.0) || !finite) { bad = 1; continue; }
                cx = dmax(cx, fabs(ux) + cf);
                cy = dmax(cy, fabs(uy) + cf);
                cz = dmax(cz, fabs(uz) + cf);
            }
    c[0] = cx; c[1] = cy; c[2] = cz;
    /* c_max: the maximum over the directions with more than one cell, x, y, z */
    {
        const int act[3] = {cfg->nx > 1, cfg->ny > 1, cfg->nz > 1};
        double m = -1.0;
        for (int d = 0; d < 3; ++d)
            if (act[d]) m = m < 0.0 ? c[d] : dmax(m, c[d]);
        c[3] = m;
    }
    return bad ? ORC_ENONPHYS : ORC_OK;
}

/* dt = CFL min over active directions of h_d / c_d, taken x, y, z */
static double cfl_dt(const orc3_cfg *cfg, const double c[4]) {
    const double h[3] = {(cfg->x1 - cfg->x0) / cfg->nx, (cfg->y1 - cfg->y0) / cfg->ny, (cfg->z1 - cfg->z0) / cfg->nz};
    const int act[3] = {cfg->nx > 1, cfg->ny > 1, cfg->nz > 1};
    double m = -1.0;
    for (int d = 0; d < 3; ++d)
        if (act[d]) m = m < 0.0 ? h[d] / c[d] : dmin(m, h[d] / c[d]);
    return cfg->cfl * m;
}

typedef struct {
    orc3_cfg cfg;
    rhs_par par;
    box B;
    double *U[NF], *S[NF], *A[NF], *K[4][NF];
} dom;

static void dom_free(dom *d) {
    for (int f = 0; f < NF; ++f) {
        free(d->U[f]); free(d->S[f]); free(d->A[f]);
        for (int s = 0; s < 4; ++s) free(d->K[s][f]);
    }
}

static int dom_init(dom *d, const orc3_cfg *cfg, double *const f[NF]) {
    memset(d, 0, sizeof(*d));
    d->cfg = *cfg;
    make_par(cfg, &d->par);
    d->B = make_box(cfg->nx, cfg->ny, cfg->nz);
    const int paper = cfg->form == ORC_FORM_PAPER;
    int ok = 1;
    for (int q = 0; q < NF; ++q) {
        d->U[q] = alloc0(d->B.n); d->S[q] = alloc0(d->B.n); d->K[0][q] = alloc0(d->B.n);
        ok = ok && d->U[q] && d->S[q] && d->K[0][q];
        if (paper)
            for (int s = 1; s < 4; ++s) { d->K[s][q] = alloc0(d->B.n); ok = ok && d->K[s][q]; }
        else { d->A[q] = alloc0(d->B.n); ok = ok && d->A[q]; }
    }
    if (!ok) { dom_free(d); return ORC_ENOMEM; }
    for (int q = 0; q < NF; ++q)
        for (int k = 0; k < cfg->nz; ++k)
            for (int j = 0; j < cfg->ny; ++j)
                memcpy(d->U[q] + at(&d->B, G, j + G, k + G),
                       f[q] + (size_t)cfg->nx * ((size_t)j + (size_t)cfg->ny * k), sizeof(double) * cfg->nx);
    return ORC_OK;
}

static void dom_out(const dom *d, double *const f[NF]) {
    const orc3_cfg *cfg = &d->cfg;
    for (int q = 0; q < NF; ++q)
        for (int k = 0; k < cfg->nz; ++k)
            for (int j = 0; j < cfg->ny; ++j)
                memcpy(f[q] + (size_t)cfg->nx * ((size_t)j + (size_t)cfg->ny * k),
                       d->U[q] + at(&d->B, G, j + G, k + G), sizeof(double) * cfg->nx);
}

/* One classic RK4 step (section 2), the same two forms as the 2-D oracle:
 * paper: U+ = U + dt/6 (K1 + 2 K2 + 2 K3 + K4);
 * low-storage: A = 2U + ((S1 - U) + dt K2) at stage 2 and
 * U+ = S3 + (A - 2 S3)/3 + dt/6 K4 at stage 4. */
static int dom_step(dom *d, double dt, double cmax) {
    const int paper = d->cfg.form == ORC_FORM_PAPER;
    const box *B = &d->B;
    for (int stage = 1; stage <= 4; ++stage) {
        double **in = stage == 1 ? d->U : d->S;
        double **K = paper ? d->K[stage - 1] : d->K[0];
        for (int q = 0; q < NF; ++q) fill_ghosts(B, in[q], d->cfg.bc);
        int rc = rhs_box(B, in, &d->par, cmax, K);
        if (rc) return rc;
        if (stage == 4) break;
        /* S_stage = U + c dt K_stage, c = 1/2, 1/2, 1 */
        const double cc = stage == 3 ? dt : 0.5 * dt;
        for (int q = 0; q < NF; ++q) {
            const double *u = d->U[q], *kq = K[q];
            double *sq = d->S[q], *aq = d->A[q];
#pragma omp parallel for schedule(static)
            for (int kk = G; kk < B->ez - G; ++kk)
                for (int j = G; j < B->ey - G; ++j)
                    for (int i = G; i < B->ex - G; ++i) {
                        size_t c = at(B, i, j, kk);
                        if (stage == 2 && !paper) aq[c] = (u[c] + u[c]) + ((sq[c] - u[c]) + dt * kq[c]);
                        sq[c] = u[c] + cc * kq[c];
                    }
        }
    }
    const double dt6 = dt / 6.0, third = 1.0 / 3.0;
    for (int q = 0; q < NF; ++q) {
        double *u = d->U[q];
        const double *s3 = d->S[q], *aq = d->A[q];
        const double *k1 = d->K[0][q], *k2 = d->K[1][q], *k3 = d->K[2][q], *k4 = d->K[3][q];
#pragma omp parallel for schedule(static)
        for (int kk = G; kk < B->ez - G; ++kk)
            for (int j = G; j < B->ey - G; ++j)
                for (int i = G; i < B->ex - G; ++i) {
                    size_t c = at(B, i, j, kk);
                    if (paper) u[c] = u[c] + dt6 * (((k1[c] + 2.0 * k2[c]) + 2.0 * k3[c]) + k4[c]);
                    else u[c] = (s3[c] + (aq[c] - (s3[c] + s3[c])) * third) + dt6 * k1[c];
                }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* exported entry points                                                */
/* ------------------------------------------------------------------ */

int orc3_abi_version(void) { return 1; }

/* Advance up to nsteps RK4 steps (time step and c_max from each step's
 * start state; t_end <= 0: no end time, else dt = min(dt, t_end - t) and
 * the run stops once t_end - t <= 1e-12 t_end).  Fields are nx*ny*nz arrays,
 * x fastest then y then z.  info = {last dt, c_max, c_x, c_y, c_z}.  A
 * non-physical start state stops the run with ORC_ENONPHYS. */
int orc3_advance(const orc3_cfg *cfg, double *const f[NF], int nsteps, double t_end, double *t, int *steps_done,
                 double info[5]) {
    if (!cfg_ok(cfg) || !f || !t || nsteps < 0) return ORC_EINVAL;
    dom d;
    int rc = dom_init(&d, cfg, f);
    if (rc) return rc;
    int done = 0;
    for (int step = 0; step < nsteps; ++step) {
        if (t_end > 0.0 && t_end - *t <= 1e-12 * t_end) break;
        double c[4];
        rc = wavespeed_box(cfg, d.U, &d.B, 1, c);
        if (rc) break;
        double dt = cfl_dt(cfg, c);
        if (t_end > 0.0) dt = dmin(dt, t_end - *t);
        if (info) { info[0] = dt; info[1] = c[3]; info[2] = c[0]; info[3] = c[1]; info[4] = c[2]; }
        rc = dom_step(&d, dt, c[3]);
        if (rc) break;
        *t = *t + dt;
        ++done;
    }
    dom_out(&d, f);
    dom_free(&d);
    if (steps_done) *steps_done = done;
    return rc;
}

/* Right-hand side L(U) on the interior (halos filled per cfg->bc). */
int orc3_rhs(const orc3_cfg *cfg, double *const f[NF], double cmax, double *const K[NF]) {
    if (!cfg_ok(cfg) || !f || !K) return ORC_EINVAL;
    dom d;
    int rc = dom_init(&d, cfg, f);
    if (rc) return rc;
    for (int q = 0; q < NF; ++q) fill_ghosts(&d.B, d.U[q], cfg->bc);
    rc = rhs_box(&d.B, d.U, &d.par, cmax, d.K[0]);
    if (!rc)
        for (int q = 0; q < NF; ++q)
            for (int k = 0; k < cfg->nz; ++k)
                for (int j = 0; j < cfg->ny; ++j)
                    memcpy(K[q] + (size_t)cfg->nx * ((size_t)j + (size_t)cfg->ny * k),
                           d.K[0][q] + at(&d.B, G, j + G, k + G), sizeof(double) * cfg->nx);
    dom_free(&d);
    return rc;
}

/* out = {c_x, c_y, c_z, c_max, dt}; ORC_ENONPHYS for a non-physical state. */
int orc3_wavespeed(const orc3_cfg *cfg, double *const f[NF], double out[5]) {
    if (!cfg_ok(cfg) || !f || !out) return ORC_EINVAL;
    double c[4];
    int rc = wavespeed_box(cfg, f, NULL, 0, c);
    for (int k = 0; k < 4; ++k) out[k] = c[k];
    out[4] = cfl_dt(cfg, c);
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

/* Conservation sums: each field summed over the cells (pairwise, in
 * storage order) times the cell volume dx dy dz. */
int orc3_sums(const orc3_cfg *cfg, double *const f[NF], double sums[NF]) {
    if (!cfg_ok(cfg) || !f || !sums) return ORC_EINVAL;
    const double dx = (cfg->x1 - cfg->x0) / cfg->nx, dy = (cfg->y1 - cfg->y0) / cfg->ny,
                 dz = (cfg->z1 - cfg->z0) / cfg->nz;
    const size_t n = (size_t)cfg->nx * cfg->ny * cfg->nz;
    for (int q = 0; q < NF; ++q) sums[q] = psum(f[q], n) * ((dx * dy) * dz);
    return ORC_OK;
}
