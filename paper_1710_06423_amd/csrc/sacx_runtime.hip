// sacx_runtime.hip -- host runtime and C ABI of libsacx, plus the small
// auxiliary kernels (halo exchange, boundary fills, reductions, step scalars,
// field import/export).
//
// Time stepping (paper section 2, classic RK4) uses four state buffers U, B1,
// B2, A and the stage kernel's fused combine:
//   stage 1: B1 = U  + dt/2 L(U)
//   stage 2: B2 = U  + dt/2 L(B1),   A = 2U + ((B1 - U) + dt L(B1))
//   stage 3: B1 = U  + dt   L(B2)
//   stage 4: U  = B1 + (A - 2 B1)/3 + dt/6 L(B1)
// which is algebraically U + dt/6 (K1 + 2 K2 + 2 K3 + K4), leaves a state
// with L = 0 bit-for-bit unchanged, and moves 12 field values per cell and
// step (stencil reads 4, pointwise reads 3, writes 5).
//
// Before every stage the halo of the stage input is refilled (paper section 3,
// exchange_halo): periodic directions pack both boundary strips into device
// exchange buffers and unpack them into the opposite ghost layers (the
// self-exchange of a subdomain that is its own neighbour); open directions copy
// the edge cell outward.  x goes first, then y over the padded width, so the
// corners are filled.
//
// The time step is computed on the device: stage 4 reduces max(|v_d| + c_f)
// of the new state into the next slot of a double-buffered accumulator, a
// one-thread kernel turns it into dt (with the end-time clamp) before the
// next step, and another advances t after it.  Nothing synchronises with the
// host inside sacx_advance.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <array>
#include <vector>

#include "sacx_internal.h"

using namespace sacx;

// ------------------------------------------------------------------ errors

static thread_local std::string g_last_error;

int sacx::set_error(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}
#define fail sacx::set_error


// ------------------------------------------------------------------ context

struct sacx_ctx {
    sacx_grid grid;
    sacx_params params;
    int device;
    hipStream_t stream;
    Layout L;
    size_t elem;
    int bc[4];
    char *ws;
    size_t ws_bytes;
    DevScalars *sc;
    double *sums;      // 6 doubles
    double *partials;  // npart x 6
    int npart;
    void *U[NF], *B1[NF], *B2[NF], *A[NF], *BG[NBG];
    void *hx[2], *hy[2];
    bool initialized;
    int ty, nt;
    int split;         // FP64 hyper-diffusion tiles: two threads per column
    bool ty_auto;      // strip height chosen by auto_rows (until set explicitly)
    double dx, dy;
    SchemeConsts kc;
    // profiling: event pairs recorded around launch groups, resolved at read
    bool prof_on;
    std::vector<hipEvent_t> *ev_pool;
    std::vector<std::pair<int, std::pair<int, int>>> *ev_marks;  // (class, (start, stop) pool index)
    int ev_used;
    sacx_profile prof;
    // learned hyper-diffusion coefficient (off unless sacx_hd_set_surrogate)
    bool sur_on;
    sacx_surrogate sur;
    float *sur_r;          // ratio planes
    unsigned char *sur_k;  // per check tile: prediction kept (1) or fallen back (0)
    int64_t sur_pitch;
    void *sur_x, *sur_a1, *sur_a2;
    HdDevStats *sur_st;
    int64_t sur_since;     // steps enqueued since the last refresh
    int64_t sur_refreshes, sur_tiles_checked;
    // decomposed stepping (sacx_stage): the next RK4 stage, 0 between steps
    int stage_next;
    // bumped by every change a batch's instance table copies (boundaries,
    // spacing), so that the batch rebuilds its table
    unsigned long long gen;
};

namespace {

constexpr size_t kAlign = 256;
constexpr int kPartials = 512;

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Plan {
    Layout L;
    size_t elem;
    size_t field_bytes;
    size_t off_sc, off_sums, off_part, off_state, off_bg, off_hx, off_hy, total;
    size_t hx_bytes, hy_bytes;
};

int check_grid(const sacx_grid *g, const sacx_params *p) {
    if (!g || !p) return fail(SACX_EINVAL, "grid/params must not be NULL");
    if (g->nx < 1 || g->ny < 1) return fail(SACX_EINVAL, "nx, ny must be >= 1 (got %d, %d)", g->nx, g->ny);
    if (g->nx < 2 && g->ny < 2) return fail(SACX_EINVAL, "at least one direction needs 2 or more cells");
    if ((int64_t)g->nx * g->ny > ((int64_t)1 << 34)) return fail(SACX_EINVAL, "grid too large");
    if (g->nx > (1 << 24) || g->ny > (1 << 24)) return fail(SACX_EINVAL, "grid dimension too large");
    if (!(g->x1 > g->x0) || !(g->y1 > g->y0)) return fail(SACX_EINVAL, "empty physical extent");
    if (g->precision != SACX_FP64 && g->precision != SACX_FP32)
        return fail(SACX_EINVAL, "precision must be SACX_FP64 or SACX_FP32");
    if (g->background_on != 0 && g->background_on != 1) return fail(SACX_EINVAL, "background_on must be 0 or 1");
    if (!(p->gamma > 1.0) || !std::isfinite(p->gamma)) return fail(SACX_EINVAL, "gamma must be > 1");
    if (!(p->cfl > 0.0) || !std::isfinite(p->cfl)) return fail(SACX_EINVAL, "cfl must be > 0");
    for (int k = 0; k < 4; ++k)
        if (!(p->c2[k] >= 0.0) || !(p->cshk[k] >= 0.0) || !std::isfinite(p->c2[k]) || !std::isfinite(p->cshk[k]))
            return fail(SACX_EINVAL, "hyper-diffusion constants must be finite and >= 0");
    if (!std::isfinite(p->g[0]) || !std::isfinite(p->g[1])) return fail(SACX_EINVAL, "gravity must be finite");
    return SACX_OK;
}

Plan make_plan(const sacx_grid *g) {
    Plan P;
    P.elem = g->precision == SACX_FP64 ? 8 : 4;
    const int per = (int)(kAlign / P.elem);
    P.L.nx = g->nx;
    P.L.ny = g->ny;
    P.L.xoff = per;
    P.L.pitch = (int)round_up((size_t)per + g->nx + G, (size_t)per);
    P.L.rows = g->ny + 2 * G;
    P.L.field_elems = (int64_t)P.L.rows * P.L.pitch;
    P.field_bytes = round_up((size_t)P.L.field_elems * P.elem, kAlign);
    size_t off = 0;
    P.off_sc = off; off += round_up(sizeof(DevScalars), kAlign);
    P.off_sums = off; off += kAlign;
    P.off_part = off; off += round_up((size_t)kPartials * NF * sizeof(double), kAlign);
    P.off_state = off; off += 4 * NF * P.field_bytes;
    P.off_bg = off; off += g->background_on ? NBG * P.field_bytes : 0;
    P.hx_bytes = round_up((size_t)NF * G * g->ny * P.elem, kAlign);
    P.hy_bytes = round_up((size_t)NF * G * (g->nx + 2 * G) * P.elem, kAlign);
    P.off_hx = off; off += 2 * P.hx_bytes;
    P.off_hy = off; off += 2 * P.hy_bytes;
    P.total = off;
    return P;
}

// Output rows per strip.  When the whole grid fits in one round of resident
// blocks (slots) with strips of at most 512 rows, the strip count whose
// longest block (strip plus the 6-row warm-up) is shortest; otherwise strips
// of 256 rows, halved while the launch has fewer than 1024 blocks.  (Measured
// on MI355X: FP32 at 8000^2 and FP64 at 2048^2 fit one round and gain from
// balanced strips; FP64 at 8000^2 takes several rounds and, being partly
// bandwidth-bound, runs a part-filled last round faster than a full one, so
// rounding the block count gains nothing there; the FP64 kernel without
// hyper-diffusion loses 6 % with one round of 534-row strips.)
int rows_for_slots(const Layout &L, int nt, int64_t slots) {
    if (L.ny <= 8) return L.ny;
    const int64_t xt = (L.nx + nt - 2 * G - 1) / (nt - 2 * G);
    int one = 0;
    for (int64_t strips = (L.ny + 4095) / 4096; strips <= (L.ny + 7) / 8; ++strips) {
        const int64_t ty = (L.ny + strips - 1) / strips;
        if (ty < 8) break;
        if (xt * ((L.ny + ty - 1) / ty) <= slots) one = (int)ty;   // later strips are shorter
        else break;
    }
    if (one > 0 && one <= 512) return one;
    int ty = 256;
    while (ty > 8 && xt * ((L.ny + ty - 1) / ty) < 1024) ty /= 2;
    return ty;
}

// the strip height for the context's current launch settings: resident
// blocks from the device's compute units and the kernel's occupancy
void auto_rows(sacx_ctx *c) {
    int cus = 0, per = 0;
    const bool fp64 = c->grid.precision == SACX_FP64;
    const bool hd = c->params.hd_on != 0, bg = c->grid.background_on != 0;
    hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device);
    if (e == hipSuccess)
        e = fp64 ? stage_blocks_per_cu<double>(c->nt, hd, bg, c->split != 0, &per)
                 : stage_blocks_per_cu<float>(c->nt, hd, bg, c->split != 0, &per);
    if (e != hipSuccess || cus < 1 || per < 1) {
        (void)hipGetLastError();
        cus = 256;
        per = 2;
    }
    c->ty = rows_for_slots(c->L, c->nt, (int64_t)cus * per);
}

// ------------------------------------------------------------------ kernels

template <typename real>
struct FPtr {
    real *p[NF];
};

__device__ __forceinline__ int64_t eidx(const Layout &L, int i, int j) {
    return (int64_t)L.xoff + i + (int64_t)(j + G) * L.pitch;
}

__device__ __forceinline__ bool step_active(const DevScalars *sc) { return sc->active != 0; }

// x strips: buffer [f][g][j], j in [0, ny)
template <typename real>
__global__ void k_pack_x(FPtr<real> S, int nf, Layout L, real *b0, real *b1, int sides, const DevScalars *sc) {
    if (sc && !step_active(sc)) return;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int f = blockIdx.y;
    const int side = (sides == 2) ? (int)blockIdx.z : sides - 10;
    if (j >= L.ny || f >= nf) return;
    real *b = side == 0 ? b0 : b1;
    const int c0 = side == 0 ? 0 : L.nx - G;
#pragma unroll
    for (int g = 0; g < G; ++g) b[((int64_t)f * G + g) * L.ny + j] = S.p[f][eidx(L, c0 + g, j)];
}

template <typename real>
__global__ void k_unpack_x(FPtr<real> S, int nf, Layout L, const real *b0, const real *b1, int sides,
                           const DevScalars *sc) {
    if (sc && !step_active(sc)) return;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int f = blockIdx.y;
    const int side = (sides == 2) ? (int)blockIdx.z : sides - 10;
    if (j >= L.ny || f >= nf) return;
    const real *b = side == 0 ? b0 : b1;
    const int cg = side == 0 ? -G : L.nx;
#pragma unroll
    for (int g = 0; g < G; ++g) S.p[f][eidx(L, cg + g, j)] = b[((int64_t)f * G + g) * L.ny + j];
}

// y strips over the padded width: buffer [f][g][i + G], i in [-G, nx + G)
template <typename real>
__global__ void k_pack_y(FPtr<real> S, int nf, Layout L, real *b0, real *b1, int sides, const DevScalars *sc) {
    if (sc && !step_active(sc)) return;
    const int w = L.nx + 2 * G;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int f = blockIdx.y;
    const int side = (sides == 2) ? (int)blockIdx.z : sides - 10;
    if (i >= w || f >= nf) return;
    real *b = side == 0 ? b0 : b1;
    const int r0 = side == 0 ? 0 : L.ny - G;
#pragma unroll
    for (int g = 0; g < G; ++g) b[((int64_t)f * G + g) * w + i] = S.p[f][eidx(L, i - G, r0 + g)];
}

template <typename real>
__global__ void k_unpack_y(FPtr<real> S, int nf, Layout L, const real *b0, const real *b1, int sides,
                           const DevScalars *sc) {
    if (sc && !step_active(sc)) return;
    const int w = L.nx + 2 * G;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int f = blockIdx.y;
    const int side = (sides == 2) ? (int)blockIdx.z : sides - 10;
    if (i >= w || f >= nf) return;
    const real *b = side == 0 ? b0 : b1;
    const int rg = side == 0 ? -G : L.ny;
#pragma unroll
    for (int g = 0; g < G; ++g) S.p[f][eidx(L, i - G, rg + g)] = b[((int64_t)f * G + g) * w + i];
}

// open (zero-gradient) or small-periodic (index modulo n) fills; bit 0 / 1 of
// `skip` leaves the low / high side alone (a side filled by the caller)
template <typename real>
__global__ void k_fill_x(FPtr<real> S, int nf, Layout L, int periodic, int skip, const DevScalars *sc) {
    if (sc && !step_active(sc)) return;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int f = blockIdx.y;
    if (j >= L.ny || f >= nf) return;
    for (int g = 1; g <= G; ++g) {
        int il = -g, ir = L.nx - 1 + g;
        int sl, sr;
        if (periodic) {
            sl = ((il % L.nx) + L.nx) % L.nx;
            sr = ir % L.nx;
        } else {
            sl = 0;
            sr = L.nx - 1;
        }
        if (!(skip & 1)) S.p[f][eidx(L, il, j)] = S.p[f][eidx(L, sl, j)];
        if (!(skip & 2)) S.p[f][eidx(L, ir, j)] = S.p[f][eidx(L, sr, j)];
    }
}

template <typename real>
__global__ void k_fill_y(FPtr<real> S, int nf, Layout L, int periodic, int skip, const DevScalars *sc) {
    if (sc && !step_active(sc)) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x - G;
    const int f = blockIdx.y;
    if (i >= L.nx + G || f >= nf) return;
    for (int g = 1; g <= G; ++g) {
        int jl = -g, jr = L.ny - 1 + g;
        int sl, sr;
        if (periodic) {
            sl = ((jl % L.ny) + L.ny) % L.ny;
            sr = jr % L.ny;
        } else {
            sl = 0;
            sr = L.ny - 1;
        }
        if (!(skip & 1)) S.p[f][eidx(L, i, jl)] = S.p[f][eidx(L, i, sl)];
        if (!(skip & 2)) S.p[f][eidx(L, i, jr)] = S.p[f][eidx(L, i, sr)];
    }
}

// caller arrays <-> internal storage
template <typename T>
struct CPtr {
    const T *p[NF];
};
template <typename T>
struct MPtr {
    T *p[NF];
};

template <typename real, typename T>
__global__ void k_import(FPtr<real> D, CPtr<T> src, int nf, Layout L, int64_t pitch) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= L.nx) return;
    for (int f = 0; f < nf; ++f) D.p[f][eidx(L, i, j)] = (real)src.p[f][(int64_t)j * pitch + i];
}

// the verification problems evaluated at the cell centres x0 + (i + 1/2) hx,
// y0 + (j + 1/2) hy (the operations in the order the conserved variables are
// defined: e = p/(gamma-1) + rho |v|^2/2 + |B|^2/2)
template <typename real>
__global__ void k_init_problem(FPtr<real> D, Layout L, int kind, double x0, double hx, double y0, double hy,
                               double mid, int along_y, double gamma, double p0, double p1) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= L.nx) return;
    const double x = x0 + ((double)i + 0.5) * hx, y = y0 + ((double)j + 0.5) * hy;
    double rho, vx, vy, p, bx, by;
    if (kind == SACX_PROBLEM_ORSZAG_TANG) {
        const double pi = 3.141592653589793;   // the double nearest pi
        const double b0 = p0 / sqrt(4.0 * pi);
        rho = 25.0 / (36.0 * pi);
        p = 5.0 / (12.0 * pi);
        vx = -sin(y);
        vy = sin(x);
        bx = -b0 * sin(y);
        by = b0 * sin(2.0 * x);
    } else {
        const bool left = (along_y ? y : x) < mid;
        rho = left ? 1.0 * p0 : 0.125 * p1;
        p = left ? 1.0 * p0 : 0.1 * p1;
        vx = 0.0;
        vy = 0.0;
        const double bn = 0.75, bt = left ? 1.0 : -1.0;
        bx = along_y ? bt : bn;
        by = along_y ? bn : bt;
    }
    const double e = p / (gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy) + 0.5 * (bx * bx + by * by);
    const int64_t o = eidx(L, i, j);
    D.p[0][o] = (real)rho;
    D.p[1][o] = (real)(rho * vx);
    D.p[2][o] = (real)(rho * vy);
    D.p[3][o] = (real)e;
    D.p[4][o] = (real)bx;
    D.p[5][o] = (real)by;
}

template <typename real, typename T>
__global__ void k_export(FPtr<real> Sx, MPtr<T> dst, uint32_t mask, Layout L, int64_t pitch) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= L.nx) return;
    for (int f = 0; f < NF; ++f)
        if (mask & (1u << f)) dst.p[f][(int64_t)j * pitch + i] = (T)Sx.p[f][eidx(L, i, j)];
}

// wave speeds of a state into accumulator slot `slot`
template <typename real>
__global__ void k_wavespeed(FPtr<real> U, FPtr<real> B, int bg, Layout L, double gamma, DevScalars *sc, int slot) {
    double cx = 0.0, cy = 0.0;
    int bad = 0;
    const real gm1 = (real)(gamma - 1.0), half = (real)0.5, gam = (real)gamma;
    const int64_t n = (int64_t)L.nx * L.ny;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(k % L.nx), j = (int)(k / L.nx);
        const int64_t e = eidx(L, i, j);
        real rb = 0, eb = 0, bxb = 0, byb = 0;
        if (bg) { rb = B.p[0][e]; eb = B.p[1][e]; bxb = B.p[2][e]; byb = B.p[3][e]; }
        const real rt = U.p[0][e], mx = U.p[1][e], my = U.p[2][e], et = U.p[3][e], bxt = U.p[4][e], byt = U.p[5][e];
        const real r = rb + rt;
        const real ir = (real)1 / r;
        const real ux = mx * ir, uy = my * ir;
        const real kin = half * (mx * ux + my * uy);
        const real bbd = bxb * bxt + byb * byt;
        const real bt2 = bxt * bxt + byt * byt;
        const real pkt = gm1 * (((et - kin) - bbd) - half * bt2);
        const real b2b = bxb * bxb + byb * byb;
        const real pkb = gm1 * (eb - half * b2b);
        const real pk = pkb + pkt;
        const real bx = bxb + bxt, by = byb + byt;
        const real cf = sqrt((gam * pk + (bx * bx + by * by)) * ir);
        const bool fin = isfinite(rt) && isfinite(mx) && isfinite(my) && isfinite(et) && isfinite(bxt) &&
                         isfinite(byt) && isfinite(cf);
        if (!(r > (real)0) || !(pk > (real)0) || !fin) {
            bad = 1;
            continue;
        }
        cx = fmax(cx, (double)(fabs(ux) + cf));
        cy = fmax(cy, (double)(fabs(uy) + cf));
    }
    for (int off = 32; off > 0; off >>= 1) {
        cx = fmax(cx, __shfl_xor(cx, off));
        cy = fmax(cy, __shfl_xor(cy, off));
        bad |= __shfl_xor(bad, off);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(&sc->cacc[slot][0], (unsigned long long)__double_as_longlong(cx));
        atomicMax(&sc->cacc[slot][1], (unsigned long long)__double_as_longlong(cy));
        if (bad) atomicOr(&sc->nonphys, 1);
    }
}

__global__ void k_reset_scalars(DevScalars *sc, double t0) {
    sc->t = t0;
    sc->dt = 0.0;
    sc->cmax = 0.0;
    sc->t_end = 0.0;
    sc->cacc[0][0] = sc->cacc[0][1] = sc->cacc[1][0] = sc->cacc[1][1] = 0ull;
    sc->last_cx = sc->last_cy = sc->last_cmax = 0.0;
    sc->steps = 0;
    sc->cur = 0;
    sc->active = 1;
    sc->nonphys = 0;
    sc->pad = 0;
}

// dt for the step about to start (CFL time step with the end-time clamp)
__global__ void k_step_begin(DevScalars *sc, double t_end, StepConsts k) { step_begin_dev(sc, t_end, k); }

__global__ void k_step_end(DevScalars *sc) { step_end_dev(sc); }

// step start of decomposed stepping: the maxima over every subdomain replace
// this subdomain's own, so that all subdomains take one dt and one c_max.
// From a device array (dc != nullptr) the values are checked here: one that
// is not finite, negative, or zero along a direction with more than one cell
// stops stepping like a non-physical state.
__global__ void k_step_begin_global(DevScalars *sc, double cx, double cy, const double *dc, StepConsts k) {
    if (dc) {
        cx = dc[0];
        cy = dc[1];
        const bool ok = isfinite(cx) && isfinite(cy) && cx >= 0.0 && cy >= 0.0 && (!k.ax || cx > 0.0) &&
                        (!k.ay || cy > 0.0);
        if (!ok) sc->nonphys = 1;
    }
    sc->cacc[sc->cur][0] = (unsigned long long)__double_as_longlong(cx);
    sc->cacc[sc->cur][1] = (unsigned long long)__double_as_longlong(cy);
    step_begin_dev(sc, 0.0, k);
}

// the device stand-in of an all-reduce(max) over subdomains: this context's
// maxima of the current state into a caller array (non-negative doubles
// order as their bit patterns)
__global__ void k_speeds_max(const DevScalars *sc, unsigned long long *dc) {
    if (threadIdx.x < 2) atomicMax(&dc[threadIdx.x], sc->cacc[sc->cur][threadIdx.x]);
}

// conservation sums: per-block partial sums of rows, then a fixed-order final sum
template <typename real>
__global__ void k_sums_partial(FPtr<real> U, Layout L, double *partials, int npart) {
    __shared__ double red[NF][256];
    double acc[NF] = {0, 0, 0, 0, 0, 0};
    for (int j = blockIdx.x; j < L.ny; j += npart)
        for (int i = threadIdx.x; i < L.nx; i += blockDim.x)
            for (int f = 0; f < NF; ++f) acc[f] += (double)U.p[f][eidx(L, i, j)];
    for (int f = 0; f < NF; ++f) red[f][threadIdx.x] = acc[f];
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int f = 0; f < NF; ++f) red[f][threadIdx.x] += red[f][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int f = 0; f < NF; ++f) partials[(int64_t)blockIdx.x * NF + f] = red[f][0];
}

__global__ void k_sums_final(const double *partials, int npart, double *out, double cell) {
    if (threadIdx.x >= NF) return;
    double s = 0.0;
    for (int b = 0; b < npart; ++b) s += partials[(int64_t)b * NF + threadIdx.x];
    out[threadIdx.x] = s * cell;
}

// ------------------------------------------------------------------ host helpers

// event marks: class 0..3 = stage kernels, 4 = halo, 5 = scalar kernels
int prof_event(sacx_ctx *c) {
    if (c->ev_used == (int)c->ev_pool->size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return -1;
        c->ev_pool->push_back(e);
    }
    int k = c->ev_used++;
    if (hipEventRecord((*c->ev_pool)[k], c->stream) != hipSuccess) return -1;
    return k;
}

struct ProfScope {
    sacx_ctx *c;
    int cls, start;
    ProfScope(sacx_ctx *c_, int cls_) : c(c_), cls(cls_), start(-1) {
        if (c->prof_on) start = prof_event(c);
    }
    ~ProfScope() {
        if (c->prof_on && start >= 0) {
            int stop = prof_event(c);
            if (stop >= 0) c->ev_marks->push_back({cls, {start, stop}});
        }
    }
};


template <typename real>
FPtr<real> fptr(void *const *p, int nf) {
    FPtr<real> f;
    for (int k = 0; k < NF; ++k) f.p[k] = (real *)(k < nf ? p[k] : p[0]);
    return f;
}

// local boundary fill of one direction (0: x over the interior rows, 1: y over
// the padded width, corners included, so x goes first); exchange sides are
// left as the caller unpacked them
template <typename real>
void fill_dir_t(sacx_ctx *c, void *const *fields, int nf, bool gated, int dir) {
    const Layout &L = c->L;
    const DevScalars *sc = gated ? c->sc : nullptr;
    FPtr<real> S = fptr<real>(fields, nf);
    const int T = 256;
    const int lo = c->bc[2 * dir], hi = c->bc[2 * dir + 1];
    const int n = dir == 0 ? L.nx : L.ny;
    const int along = dir == 0 ? L.ny : L.nx + 2 * G;
    const int skip = (lo == SACX_EXCHANGE ? 1 : 0) | (hi == SACX_EXCHANGE ? 2 : 0);
    if (skip == 3) return;
    if (lo == SACX_PERIODIC && n >= G) {
        // self-exchange: what the low side packed becomes the high halo and vice versa
        void *const *h = dir == 0 ? c->hx : c->hy;
        dim3 g((along + T - 1) / T, nf, 2);
        if (dir == 0) {
            hipLaunchKernelGGL(k_pack_x<real>, g, dim3(T), 0, c->stream, S, nf, L, (real *)h[0], (real *)h[1], 2, sc);
            hipLaunchKernelGGL(k_unpack_x<real>, g, dim3(T), 0, c->stream, S, nf, L, (const real *)h[1],
                               (const real *)h[0], 2, sc);
        } else {
            hipLaunchKernelGGL(k_pack_y<real>, g, dim3(T), 0, c->stream, S, nf, L, (real *)h[0], (real *)h[1], 2, sc);
            hipLaunchKernelGGL(k_unpack_y<real>, g, dim3(T), 0, c->stream, S, nf, L, (const real *)h[1],
                               (const real *)h[0], 2, sc);
        }
    } else {
        dim3 g((along + T - 1) / T, nf);
        const int periodic = lo == SACX_PERIODIC ? 1 : 0;
        if (dir == 0)
            hipLaunchKernelGGL(k_fill_x<real>, g, dim3(T), 0, c->stream, S, nf, L, periodic, skip, sc);
        else
            hipLaunchKernelGGL(k_fill_y<real>, g, dim3(T), 0, c->stream, S, nf, L, periodic, skip, sc);
    }
}

template <typename real>
int fill_halo_t(sacx_ctx *c, void *const *fields, int nf, bool gated) {
    fill_dir_t<real>(c, fields, nf, gated, 0);
    fill_dir_t<real>(c, fields, nf, gated, 1);
    HIPCHK(hipGetLastError());
    return SACX_OK;
}

int fill_halo(sacx_ctx *c, void *const *fields, int nf, bool gated) {
    return c->grid.precision == SACX_FP64 ? fill_halo_t<double>(c, fields, nf, gated)
                                          : fill_halo_t<float>(c, fields, nf, gated);
}

// the state the next stage differences: U between steps, then w1, w2, w3
void *const *stage_input(sacx_ctx *c) {
    switch (c->stage_next) {
        case 1: return c->B1;
        case 2: return c->B2;
        case 3: return c->B1;
        default: return c->U;
    }
}

bool has_exchange(const sacx_ctx *c) {
    for (int s = 0; s < 4; ++s)
        if (c->bc[s] == SACX_EXCHANGE) return true;
    return false;
}

// grid spacing and the scheme constants derived from it, in the same FP64
// operations as the defining sequence
void set_spacing(sacx_ctx *c, double dx, double dy) {
    c->dx = dx;
    c->dy = dy;
    const sacx_params *params = &c->params;
    SchemeConsts &k = c->kc;
    k.gamma = params->gamma;
    k.gm1 = params->gamma - 1.0;
    k.igm1 = 1.0 / k.gm1;
    k.i12dx = 1.0 / (12.0 * c->dx);
    k.i12dy = 1.0 / (12.0 * c->dy);
    k.idx = 1.0 / c->dx;
    k.idy = 1.0 / c->dy;
    k.i2dx = 1.0 / (2.0 * c->dx);
    k.i2dy = 1.0 / (2.0 * c->dy);
    for (int m = 0; m < 4; ++m) {
        k.kxs[m] = params->cshk[m] * c->dx * c->dx;
        k.kys[m] = params->cshk[m] * c->dy * c->dy;
    }
    k.third = 1.0 / 3.0;
    k.gx = params->g[0];
    k.gy = params->g[1];
    k.grav = params->g[0] != 0.0 || params->g[1] != 0.0;
}

StepConsts step_consts(const sacx_ctx *c) {
    StepConsts sk;
    sk.cfl = c->params.cfl;
    sk.dx = c->dx;
    sk.dy = c->dy;
    for (int m = 0; m < 4; ++m) sk.c2[m] = c->params.c2[m];
    sk.ax = c->grid.nx > 1;
    sk.ay = c->grid.ny > 1;
    return sk;
}

template <typename real>
StageArgs<real> stage_args(sacx_ctx *c) {
    StageArgs<real> a;
    std::memset(&a, 0, sizeof(a));
    a.L = c->L;
    a.ty = c->ty;
    a.nt = c->nt;
    a.split = c->split;
    a.k = c->kc;
    a.hd_cross_on = c->params.hd_cross_on;
    a.sc = c->sc;
    a.fstride = (int64_t)(((const char *)c->U[1] - (const char *)c->U[0]) / (ptrdiff_t)sizeof(real));
    for (int k = 0; k < NBG; ++k) a.BG[k] = (const real *)(c->grid.background_on ? c->BG[k] : nullptr);
    if (c->sur_on) {
        a.Rs = c->sur_r;
        a.rs_pitch = (int)c->sur_pitch;
        a.rs_plane = c->sur_pitch * c->L.ny;
        a.Rk = c->sur_k;
        a.rs_tile = c->sur.tile;
        a.rs_ntx = (c->L.nx + c->sur.tile - 1) / c->sur.tile;
    }
    return a;
}

template <typename real>
RatioArgs<real> ratio_args(sacx_ctx *c) {
    RatioArgs<real> a;
    for (int f = 0; f < NF; ++f) a.S[f] = (const real *)c->U[f];
    a.L = c->L;
    a.gm1 = c->kc.gm1;
    a.igm1 = c->kc.igm1;
    return a;
}

// surrogate refresh at a step start: predict the ratio planes from U (unless
// the caller supplies them) and check them against the plain ratios of U
int sur_refresh(sacx_ctx *c) {
    int rc = fill_halo(c, c->U, NF, false);
    if (rc) return rc;
    const int nx = c->L.nx, ny = c->L.ny;
    InputNorm nm;
    for (int k = 0; k < 12; ++k) nm.v[k] = c->sur.norm[k];
    const bool fp64 = c->grid.precision == SACX_FP64;
    if (c->sur.d_packed) {
        HIPCHK(fp64 ? launch_cnn_inputs<double>(ratio_args<double>(c), nm, c->sur_x, c->stream)
                    : launch_cnn_inputs<float>(ratio_args<float>(c), nm, c->sur_x, c->stream));
        HIPCHK(cnn_forward_dev(c->sur.d_packed, c->sur_x, 1, ny, nx, c->sur_a1, c->sur_a2, c->sur_a1, c->sur_r, 0,
                               c->sur_pitch * ny, c->sur_pitch, c->stream));
    }
    HIPCHK(fp64 ? launch_hd_check<double>(ratio_args<double>(c), c->sur_r, c->sur_pitch, c->sur.bound, c->sur.tile,
                                          c->sur.metric, c->sur_st, c->sur_k, c->stream)
                : launch_hd_check<float>(ratio_args<float>(c), c->sur_r, c->sur_pitch, c->sur.bound, c->sur.tile,
                                         c->sur.metric, c->sur_st, c->sur_k, c->stream));
    const int64_t ntx = (nx + c->sur.tile - 1) / c->sur.tile, nty = (ny + c->sur.tile - 1) / c->sur.tile;
    c->sur_refreshes += 1;
    c->sur_tiles_checked += ntx * nty;
    return SACX_OK;
}

// the stage kernel addresses field f of a buffer as field 0 + f * fstride
template <typename real>
bool fields_uniform(const StageArgs<real> &a) {
    for (int f = 1; f < NF; ++f) {
        const int64_t o = f * a.fstride;
        if (a.S[f] != a.S[0] + o || a.U[f] != a.U[0] + o || a.A[f] != a.A[0] + o || a.out1[f] != a.out1[0] + o ||
            a.out2[f] != a.out2[0] + o)
            return false;
    }
    for (int k = 1; k < NBG; ++k)
        if (a.BG[0] && a.BG[k] != a.BG[0] + k * a.fstride) return false;
    return true;
}

template <typename real>
int run_stage(sacx_ctx *c, int stage, void *const *S, void *const *U, void *const *A, void *const *o1,
              void *const *o2) {
    StageArgs<real> a = stage_args<real>(c);
    for (int f = 0; f < NF; ++f) {
        a.S[f] = (const real *)S[f];
        a.U[f] = (const real *)(U ? U[f] : S[f]);
        a.A[f] = (const real *)(A ? A[f] : S[f]);
        a.out1[f] = (real *)o1[f];
        a.out2[f] = (real *)(o2 ? o2[f] : o1[f]);
    }
    if (!fields_uniform(a)) return fail(SACX_EINVAL, "internal: stage buffers are not laid out at a uniform field stride");
    HIPCHK(launch_stage<real>(stage, c->params.hd_on != 0, c->grid.background_on != 0, a, c->stream));
    return SACX_OK;
}

int stage(sacx_ctx *c, int s, void *const *S, void *const *U, void *const *A, void *const *o1, void *const *o2) {
    {
        ProfScope ps(c, 4);
        int rc = fill_halo(c, S, NF, true);
        if (rc) return rc;
    }
    ProfScope ps(c, s - 1);
    return c->grid.precision == SACX_FP64 ? run_stage<double>(c, s, S, U, A, o1, o2)
                                          : run_stage<float>(c, s, S, U, A, o1, o2);
}

int wavespeed_into(sacx_ctx *c, int slot) {
    const int64_t n = (int64_t)c->L.nx * c->L.ny;
    const int T = 256;
    int blocks = (int)std::min<int64_t>((n + T - 1) / T, 4096);
    if (c->grid.precision == SACX_FP64)
        hipLaunchKernelGGL(k_wavespeed<double>, dim3(blocks), dim3(T), 0, c->stream, fptr<double>(c->U, NF),
                           fptr<double>(c->grid.background_on ? c->BG : c->U, NBG), c->grid.background_on, c->L,
                           c->params.gamma, c->sc, slot);
    else
        hipLaunchKernelGGL(k_wavespeed<float>, dim3(blocks), dim3(T), 0, c->stream, fptr<float>(c->U, NF),
                           fptr<float>(c->grid.background_on ? c->BG : c->U, NBG), c->grid.background_on, c->L,
                           c->params.gamma, c->sc, slot);
    HIPCHK(hipGetLastError());
    return SACX_OK;
}

struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) { ok = false; return; }
        if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace

// ------------------------------------------------------------------ C ABI

extern "C" {

int sacx_abi_version(void) { return SACX_ABI_VERSION; }

const char *sacx_strerror(int code) {
    switch (code) {
        case SACX_OK: return "success";
        case SACX_EINVAL: return "invalid argument";
        case SACX_ENOSPC: return "workspace or buffer too small";
        case SACX_EDEVICE: return "HIP runtime error";
        case SACX_ENONPHYS: return "non-physical state (rho <= 0, p <= 0 or non-finite)";
        case SACX_EUNSUP: return "unsupported request";
        case SACX_ESTATE: return "call out of order";
        default: return "unknown status code";
    }
}

const char *sacx_last_error(void) { return g_last_error.c_str(); }

int sacx_workspace_size(const sacx_grid *grid, const sacx_params *params, size_t *bytes) {
    int rc = check_grid(grid, params);
    if (rc) return rc;
    if (!bytes) return fail(SACX_EINVAL, "bytes must not be NULL");
    *bytes = make_plan(grid).total;
    return SACX_OK;
}

int sacx_create(const sacx_grid *grid, const sacx_params *params, void *d_ws, size_t ws_bytes, void *hip_stream,
                sacx_ctx **out) {
    int rc = check_grid(grid, params);
    if (rc) return rc;
    if (!out) return fail(SACX_EINVAL, "out must not be NULL");
    *out = nullptr;
    if (!d_ws) return fail(SACX_EINVAL, "workspace pointer is NULL");
    if (((uintptr_t)d_ws) % kAlign) return fail(SACX_EINVAL, "workspace must be 256-byte aligned");
    Plan P = make_plan(grid);
    if (ws_bytes < P.total)
        return fail(SACX_ENOSPC, "workspace has %zu bytes, %zu needed", ws_bytes, P.total);
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    sacx_ctx *c = new (std::nothrow) sacx_ctx();
    if (!c) return fail(SACX_EINVAL, "out of host memory");
    std::memset((void *)c, 0, sizeof(*c));
    c->grid = *grid;
    c->params = *params;
    c->device = dev;
    c->stream = (hipStream_t)hip_stream;
    c->L = P.L;
    c->elem = P.elem;
    for (int s = 0; s < 4; ++s) c->bc[s] = SACX_PERIODIC;
    c->ws = (char *)d_ws;
    c->ws_bytes = ws_bytes;
    c->sc = (DevScalars *)(c->ws + P.off_sc);
    c->sums = (double *)(c->ws + P.off_sums);
    c->partials = (double *)(c->ws + P.off_part);
    c->npart = (int)std::min<int64_t>(kPartials, grid->ny);
    char *st = c->ws + P.off_state;
    for (int f = 0; f < NF; ++f) {
        c->U[f] = st + (0 * NF + f) * P.field_bytes;
        c->B1[f] = st + (1 * NF + f) * P.field_bytes;
        c->B2[f] = st + (2 * NF + f) * P.field_bytes;
        c->A[f] = st + (3 * NF + f) * P.field_bytes;
    }
    for (int k = 0; k < NBG; ++k) c->BG[k] = grid->background_on ? c->ws + P.off_bg + k * P.field_bytes : nullptr;
    c->hx[0] = c->ws + P.off_hx;
    c->hx[1] = c->ws + P.off_hx + P.hx_bytes;
    c->hy[0] = c->ws + P.off_hy;
    c->hy[1] = c->ws + P.off_hy + P.hy_bytes;
    // measured on MI355X: FP64 is best with 128-column blocks (OT 8000^2,
    // also with a background at 4000^2), FP32 with 256-column blocks
    c->nt = grid->precision == SACX_FP64 ? 128 : 256;
    c->split = 1;
    c->ty_auto = true;
    set_spacing(c, (grid->x1 - grid->x0) / grid->nx, (grid->y1 - grid->y0) / grid->ny);
    c->initialized = false;
    c->prof_on = false;
    c->sur_on = false;
    c->sur_r = nullptr;
    c->sur_k = nullptr;
    c->ev_pool = new (std::nothrow) std::vector<hipEvent_t>();
    c->ev_marks = new (std::nothrow) std::vector<std::pair<int, std::pair<int, int>>>();
    if (!c->ev_pool || !c->ev_marks) {
        delete c->ev_pool;
        delete c->ev_marks;
        delete c;
        return fail(SACX_EINVAL, "out of host memory");
    }
    c->ev_used = 0;
    auto_rows(c);
    *out = c;
    return SACX_OK;
}

int sacx_destroy(sacx_ctx *ctx) {
    if (!ctx) return SACX_OK;
    {
        // the caller frees the workspace after this call: the work queued
        // on it must be finished first
        DeviceGuard dg(ctx->device);
        (void)hipStreamSynchronize(ctx->stream);
    }
    if (ctx->ev_pool) {
        for (hipEvent_t e : *ctx->ev_pool) (void)hipEventDestroy(e);
        delete ctx->ev_pool;
    }
    delete ctx->ev_marks;
    delete ctx;
    return SACX_OK;
}

int sacx_set_launch(sacx_ctx *ctx, int32_t threads, int32_t rows) {
    if (!ctx) return fail(SACX_EINVAL, "ctx must not be NULL");
    if (threads != 0 && threads != 64 && threads != 128 && threads != 256)
        return fail(SACX_EINVAL, "threads must be 64, 128 or 256 (got %d)", threads);
    if (rows < 0 || rows > 4096) return fail(SACX_EINVAL, "rows must be in 1..4096 (got %d)", rows);
    if (threads) ctx->nt = threads;
    if (rows) {
        ctx->ty = rows;
        ctx->ty_auto = false;
    } else if (threads && ctx->ty_auto) {
        DeviceGuard dg(ctx->device);
        auto_rows(ctx);
    }
    return SACX_OK;
}

int sacx_set_column_split(sacx_ctx *ctx, int32_t on) {
    if (!ctx) return fail(SACX_EINVAL, "ctx must not be NULL");
    if (on != 0 && on != 1) return fail(SACX_EINVAL, "on must be 0 or 1 (got %d)", on);
    ctx->split = on;
    if (ctx->ty_auto) {
        DeviceGuard dg(ctx->device);
        auto_rows(ctx);
    }
    return SACX_OK;
}

int sacx_get_launch(const sacx_ctx *ctx, int32_t *threads, int32_t *rows) {
    if (!ctx || !threads || !rows) return fail(SACX_EINVAL, "ctx/threads/rows must not be NULL");
    *threads = ctx->nt;
    *rows = ctx->ty;
    return SACX_OK;
}

int sacx_profile_enable(sacx_ctx *ctx, int32_t on) {
    if (!ctx) return fail(SACX_EINVAL, "ctx must not be NULL");
    std::memset(&ctx->prof, 0, sizeof(ctx->prof));
    ctx->ev_marks->clear();
    ctx->ev_used = 0;
    ctx->prof_on = on != 0;
    return SACX_OK;
}

int sacx_profile_read(sacx_ctx *ctx, sacx_profile *out) {
    if (!ctx || !out) return fail(SACX_EINVAL, "ctx/out must not be NULL");
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(SACX_EDEVICE, "cannot select the context device");
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (const auto &m : *ctx->ev_marks) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, (*ctx->ev_pool)[m.second.first], (*ctx->ev_pool)[m.second.second]));
        if (m.first < 4) {
            ctx->prof.ms_stage[m.first] += ms;
            ctx->prof.n_stage[m.first] += 1;
        } else if (m.first == 4) {
            ctx->prof.ms_halo += ms;
            ctx->prof.n_halo += 1;
        } else if (m.first == 6) {
            ctx->prof.ms_surrogate += ms;
            ctx->prof.n_surrogate += 1;
        } else {
            ctx->prof.ms_scalar += ms;
            ctx->prof.n_scalar += 1;
        }
    }
    ctx->ev_marks->clear();
    ctx->ev_used = 0;
    *out = ctx->prof;
    return SACX_OK;
}

int sacx_set_boundaries(sacx_ctx *ctx, const int32_t bc[4]) {
    if (!ctx || !bc) return fail(SACX_EINVAL, "ctx/bc must not be NULL");
    bool exch = false;
    for (int s = 0; s < 4; ++s) {
        if (bc[s] != SACX_PERIODIC && bc[s] != SACX_OPEN && bc[s] != SACX_EXCHANGE)
            return fail(SACX_EINVAL, "bc[%d] = %d is not a boundary kind", s, bc[s]);
        exch = exch || bc[s] == SACX_EXCHANGE;
    }
    if ((bc[0] == SACX_PERIODIC) != (bc[1] == SACX_PERIODIC))
        return fail(SACX_EINVAL, "periodic x boundaries must be paired");
    if ((bc[2] == SACX_PERIODIC) != (bc[3] == SACX_PERIODIC))
        return fail(SACX_EINVAL, "periodic y boundaries must be paired");
    if (ctx->grid.nx == 1 && bc[0] != SACX_PERIODIC) return fail(SACX_EINVAL, "a one-cell direction must be periodic");
    if (ctx->grid.ny == 1 && bc[2] != SACX_PERIODIC) return fail(SACX_EINVAL, "a one-cell direction must be periodic");
    if (ctx->sur_on)
        for (int s = 0; s < 4; ++s)
            if (bc[s] != SACX_PERIODIC)
                return fail(SACX_ESTATE, "the surrogate's ratio planes are periodic: clear it before opening a boundary");
    if (exch && ctx->grid.background_on)
        return fail(SACX_EUNSUP, "exchange boundaries are not supported with a background");
    if ((bc[0] == SACX_EXCHANGE || bc[1] == SACX_EXCHANGE) && ctx->grid.nx < G)
        return fail(SACX_EUNSUP, "an exchange side needs at least %d cells across", G);
    if ((bc[2] == SACX_EXCHANGE || bc[3] == SACX_EXCHANGE) && ctx->grid.ny < G)
        return fail(SACX_EUNSUP, "an exchange side needs at least %d cells across", G);
    for (int s = 0; s < 4; ++s) ctx->bc[s] = bc[s];
    ctx->gen += 1;
    if (ctx->initialized && ctx->grid.background_on) {
        // the static background's halos follow the new boundaries
        DeviceGuard dg(ctx->device);
        if (!dg.ok) return fail(SACX_EDEVICE, "cannot select the context device");
        return fill_halo(ctx, ctx->BG, NBG, false);
    }
    return SACX_OK;
}

// after the evolved fields (and background) are in place: scalars, halos
// and the first wave-speed reduction
static int finish_init(sacx_ctx *ctx, double t0) {
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_reset_scalars, dim3(1), dim3(1), 0, ctx->stream, ctx->sc, t0);
    int rc = fill_halo(ctx, ctx->U, NF, false);
    if (rc) return rc;
    rc = wavespeed_into(ctx, 0);
    if (rc) return rc;
    HIPCHK(hipGetLastError());
    ctx->stage_next = 0;
    ctx->initialized = true;
    return SACX_OK;
}

int sacx_init_state(sacx_ctx *ctx, const void *const *d_fields, const void *const *d_bg, int64_t pitch,
                    int32_t in_precision, double t0) {
    if (!ctx || !d_fields) return fail(SACX_EINVAL, "ctx/fields must not be NULL");
    for (int f = 0; f < NF; ++f)
        if (!d_fields[f]) return fail(SACX_EINVAL, "field pointer %d is NULL", f);
    if (pitch < ctx->grid.nx) return fail(SACX_EINVAL, "pitch %lld < nx %d", (long long)pitch, ctx->grid.nx);
    if (in_precision != SACX_FP64 && in_precision != SACX_FP32) return fail(SACX_EINVAL, "bad input precision");
    if (ctx->grid.background_on && !d_bg) return fail(SACX_EINVAL, "background arrays required (background_on)");
    if (ctx->grid.background_on)
        for (int k = 0; k < NBG; ++k)
            if (!d_bg[k]) return fail(SACX_EINVAL, "background pointer %d is NULL", k);
    if (!std::isfinite(t0)) return fail(SACX_EINVAL, "t0 must be finite");
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(SACX_EDEVICE, "cannot select the context device");
    const Layout &L = ctx->L;
    dim3 g((L.nx + 255) / 256, L.ny);
    const bool f64 = ctx->grid.precision == SACX_FP64;
    auto import = [&](void *const *dst, const void *const *src, int nf) {
        if (f64) {
            if (in_precision == SACX_FP64) {
                CPtr<double> t;
                for (int k = 0; k < NF; ++k) t.p[k] = (const double *)src[k < nf ? k : 0];
                hipLaunchKernelGGL((k_import<double, double>), g, dim3(256), 0, ctx->stream, fptr<double>(dst, nf), t, nf, L, pitch);
            } else {
                CPtr<float> t;
                for (int k = 0; k < NF; ++k) t.p[k] = (const float *)src[k < nf ? k : 0];
                hipLaunchKernelGGL((k_import<double, float>), g, dim3(256), 0, ctx->stream, fptr<double>(dst, nf), t, nf, L, pitch);
            }
        } else {
            if (in_precision == SACX_FP64) {
                CPtr<double> t;
                for (int k = 0; k < NF; ++k) t.p[k] = (const double *)src[k < nf ? k : 0];
                hipLaunchKernelGGL((k_import<float, double>), g, dim3(256), 0, ctx->stream, fptr<float>(dst, nf), t, nf, L, pitch);
            } else {
                CPtr<float> t;
                for (int k = 0; k < NF; ++k) t.p[k] = (const float *)src[k < nf ? k : 0];
                hipLaunchKernelGGL((k_import<float, float>), g, dim3(256), 0, ctx->stream, fptr<float>(dst, nf), t, nf, L, pitch);
            }
        }
    };
    import(ctx->U, d_fields, NF);
    if (ctx->grid.background_on) {
        import(ctx->BG, d_bg, NBG);
        int rc = fill_halo(ctx, ctx->BG, NBG, false);
        if (rc) return rc;
    }
    return finish_init(ctx, t0);
}

int sacx_init_problem(sacx_ctx *ctx, int32_t kind, const double *prm, int32_t nprm, double t0) {
    if (!ctx) return fail(SACX_EINVAL, "ctx must not be NULL");
    if (kind != SACX_PROBLEM_ORSZAG_TANG && kind != SACX_PROBLEM_BRIO_WU) return fail(SACX_EINVAL, "unknown problem %d", kind);
    const int maxp = kind == SACX_PROBLEM_ORSZAG_TANG ? 1 : 2;
    if (nprm < 0 || nprm > maxp) return fail(SACX_EINVAL, "problem %d takes at most %d parameters", kind, maxp);
    if (nprm > 0 && !prm) return fail(SACX_EINVAL, "prm must not be NULL when nprm > 0");
    if (!std::isfinite(t0)) return fail(SACX_EINVAL, "t0 must be finite");
    if (ctx->grid.background_on) return fail(SACX_EUNSUP, "the problem generators set no background");
    const double p0 = nprm >= 1 ? prm[0] : 1.0, p1 = nprm >= 2 ? prm[1] : 1.0;
    if (!std::isfinite(p0) || !std::isfinite(p1)) return fail(SACX_EINVAL, "parameters must be finite");
    if (kind == SACX_PROBLEM_BRIO_WU && (!(p0 > 0.0) || !(p1 > 0.0)))
        return fail(SACX_EINVAL, "the shock tube's scale factors must be > 0");
    const sacx_grid &g = ctx->grid;
    const int along_y = kind == SACX_PROBLEM_BRIO_WU && g.nx == 1 && g.ny > 1;
    int32_t bc[4] = {SACX_PERIODIC, SACX_PERIODIC, SACX_PERIODIC, SACX_PERIODIC};
    if (kind == SACX_PROBLEM_BRIO_WU) {
        if (along_y) bc[2] = bc[3] = SACX_OPEN;
        else bc[0] = bc[1] = SACX_OPEN;
    }
    int rc = sacx_set_boundaries(ctx, bc);
    if (rc) return rc;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(SACX_EDEVICE, "cannot select the context device");
    const double hx = (g.x1 - g.x0) / g.nx, hy = (g.y1 - g.y0) / g.ny;
    const double mid = along_y ? (g.y0 + g.y1) * 0.5 : (g.x0 + g.x1) * 0.5;
    const Layout &L = ctx->L;
    dim3 grd((L.nx + 255) / 256, L.ny);
    if (g.precision == SACX_FP64)
        hipLaunchKernelGGL(k_init_problem<double>, grd, dim3(256), 0, ctx->stream, fptr<double>(ctx->U, NF), L, kind,
                           g.x0, hx, g.y0, hy, mid, along_y, ctx->params.gamma, p0, p1);
    else
        hipLaunchKernelGGL(k_init_problem<float>, grd, dim3(256), 0, ctx->stream, fptr<float>(ctx->U, NF), L, kind,
                           g.x0, hx, g.y0, hy, mid, along_y, ctx->params.gamma, p0, p1);
    return finish_init(ctx, t0);
}

int sacx_advance(sacx_ctx *ctx, int32_t nsteps, double t_end, int32_t *steps_done, double *t_now) {
    if (!ctx) return fail(SACX_EINVAL, "ctx must not be NULL");
    if (nsteps < 0) return fail(SACX_EINVAL, "nsteps must be >= 0");
    if (!std::isfinite(t_end)) return fail(SACX_EINVAL, "t_end must be finite");
    if (!ctx->initialized) return fail(SACX_ESTATE, "sacx_init_state has not been called");
    if (has_exchange(ctx)) return fail(SACX_ESTATE, "a context with exchange boundaries steps with sacx_stage");
    if (ctx->stage_next) return fail(SACX_ESTATE, "a step begun with sacx_stage is in progress");
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(SACX_EDEVICE, "cannot select the context device");
    long long steps0 = 0;
    const bool sync = steps_done || t_now;
    if (sync) {
        HIPCHK(hipMemcpyAsync(&steps0, &ctx->sc->steps, sizeof(steps0), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    const StepConsts sk = step_consts(ctx);
    // A synchronising call enqueues in chunks and stops early once the device
    // reports that stepping ended (end time reached or non-physical state).
    const int chunk = sync ? 128 : (nsteps > 0 ? nsteps : 1);
    for (int n0 = 0; n0 < nsteps; n0 += chunk) {
        const int n1 = std::min(nsteps, n0 + chunk);
        for (int n = n0; n < n1; ++n) {
            {
                ProfScope ps(ctx, 5);
                hipLaunchKernelGGL(k_step_begin, dim3(1), dim3(1), 0, ctx->stream, ctx->sc, t_end, sk);
            }
            int rc;
            if (ctx->sur_on) {
                if (ctx->sur_since % ctx->sur.refresh_every == 0) {
                    ProfScope ps(ctx, 6);
                    if ((rc = sur_refresh(ctx))) return rc;
                }
                ctx->sur_since += 1;
            }
            if ((rc = stage(ctx, 1, ctx->U, nullptr, nullptr, ctx->B1, nullptr))) return rc;
            if ((rc = stage(ctx, 2, ctx->B1, ctx->U, nullptr, ctx->B2, ctx->A))) return rc;
            if ((rc = stage(ctx, 3, ctx->B2, ctx->U, nullptr, ctx->B1, nullptr))) return rc;
            if ((rc = stage(ctx, 4, ctx->B1, nullptr, ctx->A, ctx->U, nullptr))) return rc;
            {
                ProfScope ps(ctx, 5);
                hipLaunchKernelGGL(k_step_end, dim3(1), dim3(1), 0, ctx->stream, ctx->sc);
            }
            HIPCHK(hipGetLastError());
        }
        if (sync && n1 < nsteps) {
            int act = 1;
            HIPCHK(hipMemcpyAsync(&act, &ctx->sc->active, sizeof(act), hipMemcpyDeviceToHost, ctx->stream));
            HIPCHK(hipStreamSynchronize(ctx->stream));
            if (!act) break;
        }
    }
    if (sync) {
        DevScalars h;
        HIPCHK(hipMemcpyAsync(&h, ctx->sc, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        if (steps_done) *steps_done = (int32_t)(h.steps - steps0);
        if (t_now) *t_now = h.t;
        if (h.nonphys) return fail(SACX_ENONPHYS, "non-physical state after %lld steps", h.steps);
    }
    return SACX_OK;
}

int sacx_read_fields(sacx_ctx *ctx, void *const *d_out, int64_t pitch, uint32_t field_mask, int32_t out_precision) {
    if (!ctx || !d_out) return fail(SACX_EINVAL, "ctx/out must not be NULL");
    if (!ctx->initialized) return fail(SACX_ESTATE, "sacx_init_state has not been called");
    if (pitch < ctx->grid.nx) return fail(SACX_EINVAL, "pitch < nx");
    if (out_precision != SACX_FP64 && out_precision != SACX_FP32) return fail(SACX_EINVAL, "bad output precision");
    if (field_mask & ~0x3Fu) return fail(SACX_EINVAL, "field_mask has bits beyond the 6 fields");
    for (int f = 0; f < NF; ++f)
        if ((field_mask & (1u << f)) && !d_out[f]) return fail(SACX_EINVAL, "output pointer %d is NULL", f);
    if (!field_mask) return SACX_OK;
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(SACX_EDEVICE, "cannot select the context device");
    const Layout &L = ctx->L;
    dim3 g((L.nx + 255) / 256, L.ny);
    MPtr<double> td;
    MPtr<float> tf;
    for (int f = 0; f < NF; ++f) {
        void *p = (field_mask & (1u << f)) ? d_out[f] : nullptr;
        td.p[f] = (double *)p;
        tf.p[f] = (float *)p;
    }
    if (ctx->grid.precision == SACX_FP64) {
        if (out_precision == SACX_FP64)
            hipLaunchKernelGGL((k_export<double, double>), g, dim3(256), 0, ctx->stream, fptr<double>(ctx->U, NF), td, field_mask, L, pitch);
        else
            hipLaunchKernelGGL((k_export<double, float>), g, dim3(256), 0, ctx->stream, fptr<double>(ctx->U, NF), tf, field_mask, L, pitch);
    } else {
        if (out_precision == SACX_FP64)
            hipLaunchKernelGGL((k_export<float, double>), g, dim3(256), 0, ctx->stream, fptr<float>(ctx->U, NF), td, field_mask, L, pitch);
        else
            hipLaunchKernelGGL((k_export<float, float>), g, dim3(256), 0, ctx->stream, fptr<float>(ctx->U, NF), tf, field_mask, L, pitch);
    }
    HIPCHK(hipGetLastError());
    return SACX_OK;
}

int sacx_diagnostics(sacx_ctx *ctx, sacx_diag *out) {
    if (!ctx || !out) return fail(SACX_EINVAL, "ctx/out must not be NULL");
    if (!ctx->initialized) return fail(SACX_ESTATE, "sacx_init_state has not been called");
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(SACX_EDEVICE, "cannot select the context device");
    if (ctx->grid.precision == SACX_FP64)
        hipLaunchKernelGGL(k_sums_partial<double>, dim3(ctx->npart), dim3(256), 0, ctx->stream,
                           fptr<double>(ctx->U, NF), ctx->L, ctx->partials, ctx->npart);
    else
        hipLaunchKernelGGL(k_sums_partial<float>, dim3(ctx->npart), dim3(256), 0, ctx->stream,
                           fptr<float>(ctx->U, NF), ctx->L, ctx->partials, ctx->npart);
    hipLaunchKernelGGL(k_sums_final, dim3(1), dim3(64), 0, ctx->stream, (const double *)ctx->partials, ctx->npart,
                       ctx->sums, ctx->dx * ctx->dy);
    HIPCHK(hipGetLastError());
    DevScalars h;
    double sums[NF];
    HIPCHK(hipMemcpyAsync(&h, ctx->sc, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipMemcpyAsync(sums, ctx->sums, sizeof(sums), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    const double cx = __builtin_bit_cast(double, h.cacc[h.cur][0]);
    const double cy = __builtin_bit_cast(double, h.cacc[h.cur][1]);
    out->t = h.t;
    out->dt = h.dt;
    out->c_x = cx;
    out->c_y = cy;
    const int ax = ctx->grid.nx > 1, ay = ctx->grid.ny > 1;
    out->c_max = (ax && ay) ? std::max(cx, cy) : (ax ? cx : cy);
    for (int f = 0; f < NF; ++f) out->sums[f] = sums[f];
    out->steps = h.steps;
    out->nonphys = h.nonphys;
    return SACX_OK;
}

int sacx_halo_buffer_size(const sacx_ctx *ctx, int32_t side, size_t *bytes) {
    if (!ctx || !bytes) return fail(SACX_EINVAL, "ctx/bytes must not be NULL");
    if (side < 0 || side > 3) return fail(SACX_EINVAL, "side must be 0..3");
    const size_t along = side < 2 ? (size_t)ctx->grid.ny : (size_t)ctx->grid.nx + 2 * G;
    *bytes = (size_t)NF * G * along * ctx->elem;
    return SACX_OK;
}

static int halo_io(sacx_ctx *ctx, int32_t side, void *buf, bool pack) {
    if (!ctx || !buf) return fail(SACX_EINVAL, "ctx/buffer must not be NULL");
    if (side < 0 || side > 3) return fail(SACX_EINVAL, "side must be 0..3");
    if (!ctx->initialized) return fail(SACX_ESTATE, "sacx_init_state has not been called");
    const Layout &L = ctx->L;
    if ((side < 2 && L.nx < G) || (side >= 2 && L.ny < G))
        return fail(SACX_EUNSUP, "halo exchange needs at least %d cells across", G);
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(SACX_EDEVICE, "cannot select the context device");
    ProfScope ps(ctx, 4);
    const int T = 256;
    const int s = side & 1;
    const bool f64 = ctx->grid.precision == SACX_FP64;
    void *const *S = stage_input(ctx);
    if (side < 2) {
        dim3 g((L.ny + T - 1) / T, NF, 1);
        if (f64) {
            if (pack) hipLaunchKernelGGL(k_pack_x<double>, g, dim3(T), 0, ctx->stream, fptr<double>(S, NF), NF, L, (double *)buf, (double *)buf, 10 + s, (const DevScalars *)nullptr);
            else hipLaunchKernelGGL(k_unpack_x<double>, g, dim3(T), 0, ctx->stream, fptr<double>(S, NF), NF, L, (const double *)buf, (const double *)buf, 10 + s, (const DevScalars *)nullptr);
        } else {
            if (pack) hipLaunchKernelGGL(k_pack_x<float>, g, dim3(T), 0, ctx->stream, fptr<float>(S, NF), NF, L, (float *)buf, (float *)buf, 10 + s, (const DevScalars *)nullptr);
            else hipLaunchKernelGGL(k_unpack_x<float>, g, dim3(T), 0, ctx->stream, fptr<float>(S, NF), NF, L, (const float *)buf, (const float *)buf, 10 + s, (const DevScalars *)nullptr);
        }
    } else {
        dim3 g((L.nx + 2 * G + T - 1) / T, NF, 1);
        if (f64) {
            if (pack) hipLaunchKernelGGL(k_pack_y<double>, g, dim3(T), 0, ctx->stream, fptr<double>(S, NF), NF, L, (double *)buf, (double *)buf, 10 + s, (const DevScalars *)nullptr);
            else hipLaunchKernelGGL(k_unpack_y<double>, g, dim3(T), 0, ctx->stream, fptr<double>(S, NF), NF, L, (const double *)buf, (const double *)buf, 10 + s, (const DevScalars *)nullptr);
        } else {
            if (pack) hipLaunchKernelGGL(k_pack_y<float>, g, dim3(T), 0, ctx->stream, fptr<float>(S, NF), NF, L, (float *)buf, (float *)buf, 10 + s, (const DevScalars *)nullptr);
            else hipLaunchKernelGGL(k_unpack_y<float>, g, dim3(T), 0, ctx->stream, fptr<float>(S, NF), NF, L, (const float *)buf, (const float *)buf, 10 + s, (const DevScalars *)nullptr);
        }
    }
    HIPCHK(hipGetLastError());
    return SACX_OK;
}

int sacx_halo_pack(sacx_ctx *ctx, int32_t side, void *d_buf) { return halo_io(ctx, side, d_buf, true); }

int sacx_halo_unpack(sacx_ctx *ctx, int32_t side, const void *d_buf) {
    return halo_io(ctx, side, const_cast<void *>(d_buf), false);
}

// ------------------------------------------------------------------ decomposed stepping

int sacx_fill_boundaries(sacx_ctx *ctx, int32_t direction) {
    if (!ctx) return fail(SACX_EINVAL, "ctx must not be NULL");
    if (direction != 0 && direction != 1) return fail(SACX_EINVAL, "direction must be 0 (x) or 1 (y)");
    if (!ctx->initialized) return fail(SACX_ESTATE, "sacx_init_state has not been called");
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(SACX_EDEVICE, "cannot select the context device");
    ProfScope ps(ctx, 4);
    if (ctx->grid.precision == SACX_FP64) fill_dir_t<double>(ctx, stage_input(ctx), NF, false, direction);
    else fill_dir_t<float>(ctx, stage_input(ctx), NF, false, direction);
    HIPCHK(hipGetLastError());
    return SACX_OK;
}

int sacx_stage(sacx_ctx *ctx, const double *c_max, int32_t c_max_on_device, int32_t *stage_done) {
    if (!ctx) return fail(SACX_EINVAL, "ctx must not be NULL");
    if (c_max_on_device != 0 && c_max_on_device != 1) return fail(SACX_EINVAL, "c_max_on_device must be 0 or 1");
    if (c_max_on_device && !c_max) return fail(SACX_EINVAL, "a device c_max must not be NULL");
    if (c_max_on_device && ((uintptr_t)c_max % alignof(double)))
        return fail(SACX_EINVAL, "a device c_max must be 8-byte aligned");
    if (!ctx->initialized) return fail(SACX_ESTATE, "sacx_init_state has not been called");
    if (ctx->sur_on) return fail(SACX_ESTATE, "a context with a learned coefficient steps with sacx_advance");
    if (ctx->stage_next == 0 && c_max && !c_max_on_device) {
        for (int d = 0; d < 2; ++d)
            if (!std::isfinite(c_max[d]) || c_max[d] < 0.0) return fail(SACX_EINVAL, "c_max[%d] must be finite and >= 0", d);
        if ((ctx->grid.nx > 1 && !(c_max[0] > 0.0)) || (ctx->grid.ny > 1 && !(c_max[1] > 0.0)))
            return fail(SACX_EINVAL, "c_max must be > 0 along every direction with more than one cell");
    }
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(SACX_EDEVICE, "cannot select the context device");
    const int s = ctx->stage_next + 1;
    if (s == 1) {
        ProfScope ps(ctx, 5);
        if (c_max_on_device)
            hipLaunchKernelGGL(k_step_begin_global, dim3(1), dim3(1), 0, ctx->stream, ctx->sc, 0.0, 0.0, c_max,
                               step_consts(ctx));
        else if (c_max)
            hipLaunchKernelGGL(k_step_begin_global, dim3(1), dim3(1), 0, ctx->stream, ctx->sc, c_max[0], c_max[1],
                               (const double *)nullptr, step_consts(ctx));
        else
            hipLaunchKernelGGL(k_step_begin, dim3(1), dim3(1), 0, ctx->stream, ctx->sc, 0.0, step_consts(ctx));
        HIPCHK(hipGetLastError());
    }
    int rc;
    {
        ProfScope ps(ctx, s - 1);
        const bool f64 = ctx->grid.precision == SACX_FP64;
        switch (s) {
            case 1: rc = f64 ? run_stage<double>(ctx, 1, ctx->U, nullptr, nullptr, ctx->B1, nullptr)
                             : run_stage<float>(ctx, 1, ctx->U, nullptr, nullptr, ctx->B1, nullptr); break;
            case 2: rc = f64 ? run_stage<double>(ctx, 2, ctx->B1, ctx->U, nullptr, ctx->B2, ctx->A)
                             : run_stage<float>(ctx, 2, ctx->B1, ctx->U, nullptr, ctx->B2, ctx->A); break;
            case 3: rc = f64 ? run_stage<double>(ctx, 3, ctx->B2, ctx->U, nullptr, ctx->B1, nullptr)
                             : run_stage<float>(ctx, 3, ctx->B2, ctx->U, nullptr, ctx->B1, nullptr); break;
            default: rc = f64 ? run_stage<double>(ctx, 4, ctx->B1, nullptr, ctx->A, ctx->U, nullptr)
                              : run_stage<float>(ctx, 4, ctx->B1, nullptr, ctx->A, ctx->U, nullptr); break;
        }
    }
    if (rc) return rc;
    if (s == 4) {
        ProfScope ps(ctx, 5);
        hipLaunchKernelGGL(k_step_end, dim3(1), dim3(1), 0, ctx->stream, ctx->sc);
        HIPCHK(hipGetLastError());
    }
    ctx->stage_next = s & 3;
    if (stage_done) *stage_done = s;
    return SACX_OK;
}

int sacx_set_spacing(sacx_ctx *ctx, double dx, double dy) {
    if (!ctx) return fail(SACX_EINVAL, "ctx must not be NULL");
    if (!std::isfinite(dx) || !std::isfinite(dy) || !(dx > 0.0) || !(dy > 0.0))
        return fail(SACX_EINVAL, "dx and dy must be finite and > 0");
    if (ctx->stage_next) return fail(SACX_ESTATE, "a step begun with sacx_stage is in progress");
    set_spacing(ctx, dx, dy);
    ctx->gen += 1;
    return SACX_OK;
}

int sacx_wave_speeds_max(sacx_ctx *ctx, double *d_c_max) {
    if (!ctx || !d_c_max) return fail(SACX_EINVAL, "ctx/d_c_max must not be NULL");
    if ((uintptr_t)d_c_max % alignof(double)) return fail(SACX_EINVAL, "d_c_max must be 8-byte aligned");
    if (!ctx->initialized) return fail(SACX_ESTATE, "sacx_init_state has not been called");
    if (ctx->stage_next) return fail(SACX_ESTATE, "a step begun with sacx_stage is in progress");
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(SACX_EDEVICE, "cannot select the context device");
    hipLaunchKernelGGL(k_speeds_max, dim3(1), dim3(64), 0, ctx->stream, (const DevScalars *)ctx->sc,
                       (unsigned long long *)d_c_max);
    HIPCHK(hipGetLastError());
    return SACX_OK;
}

int sacx_wave_speeds(sacx_ctx *ctx, double c_max[2]) {
    if (!ctx || !c_max) return fail(SACX_EINVAL, "ctx/c_max must not be NULL");
    if (!ctx->initialized) return fail(SACX_ESTATE, "sacx_init_state has not been called");
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(SACX_EDEVICE, "cannot select the context device");
    DevScalars h;
    HIPCHK(hipMemcpyAsync(&h, ctx->sc, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    c_max[0] = __builtin_bit_cast(double, h.cacc[h.cur][0]);
    c_max[1] = __builtin_bit_cast(double, h.cacc[h.cur][1]);
    return SACX_OK;
}

// ------------------------------------------------------------------ surrogate

}  // extern "C"

namespace {

__global__ void k_fill_f32(float *p, int64_t n, float v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_zero_stats(HdDevStats *st) {
    unsigned long long *p = (unsigned long long *)st;
    const int n = (int)(sizeof(HdDevStats) / sizeof(unsigned long long));
    for (int i = (int)threadIdx.x; i < n; i += (int)blockDim.x) p[i] = 0ull;
}

struct SurPlan {
    int64_t pitch;
    size_t off_r, off_st, off_k, off_x, off_a1, off_a2, total;
};

SurPlan sur_plan(const sacx_ctx *c) {
    SurPlan p;
    const int64_t nx = c->L.nx, ny = c->L.ny;
    p.pitch = (int64_t)round_up((size_t)nx, 64);
    size_t o = 0;
    p.off_r = o;  o = round_up(o + (size_t)10 * p.pitch * ny * sizeof(float), kAlign);
    p.off_st = o; o = round_up(o + sizeof(HdDevStats), kAlign);
    // one flag per check tile, sized for the smallest tile (one cell)
    p.off_k = o;  o = round_up(o + (size_t)nx * ny, kAlign);
    p.off_x = o;  o = round_up(o + (size_t)nx * ny * 8 * 2, kAlign);
    p.off_a1 = o; o = round_up(o + (size_t)nx * ny * 32 * 2, kAlign);
    p.off_a2 = o; o = round_up(o + (size_t)nx * ny * 32 * 2, kAlign);
    p.total = o;
    return p;
}

int sur_supported(const sacx_ctx *c) {
    if (!c->params.hd_on) return fail(SACX_EUNSUP, "the surrogate replaces hyper-diffusion ratios: hd_on must be 1");
    if (c->grid.background_on) return fail(SACX_EUNSUP, "the surrogate needs a context without background");
    for (int s = 0; s < 4; ++s)
        if (c->bc[s] != SACX_PERIODIC) return fail(SACX_EUNSUP, "the surrogate needs periodic boundaries on every side");
    if (c->L.ny < 2) return fail(SACX_EUNSUP, "the surrogate needs ny >= 2");
    if (c->L.nx % 32 != 0) return fail(SACX_EUNSUP, "the surrogate needs nx to be a multiple of 32 (got %d)", c->L.nx);
    return SACX_OK;
}

}  // namespace

extern "C" {

int sacx_surrogate_workspace_size(const sacx_ctx *ctx, size_t *bytes) {
    if (!ctx || !bytes) return fail(SACX_EINVAL, "ctx/bytes must not be NULL");
    *bytes = sur_plan(ctx).total;
    return SACX_OK;
}

int sacx_hd_set_surrogate(sacx_ctx *ctx, const sacx_surrogate *cfg, void *d_ws, size_t ws_bytes) {
    if (!ctx || !cfg || !d_ws) return fail(SACX_EINVAL, "ctx/cfg/workspace must not be NULL");
    int rc = sur_supported(ctx);
    if (rc) return rc;
    if (cfg->refresh_every < 1) return fail(SACX_EINVAL, "refresh_every must be >= 1");
    if (cfg->tile < 1) return fail(SACX_EINVAL, "tile must be >= 1");
    if (cfg->metric != SACX_HD_CHECK_RATIO && cfg->metric != SACX_HD_CHECK_FLUX)
        return fail(SACX_EINVAL, "metric must be SACX_HD_CHECK_RATIO or SACX_HD_CHECK_FLUX");
    if (!(cfg->bound >= 0.0)) return fail(SACX_EINVAL, "bound must be >= 0");
    for (int k = 0; k < 12; ++k)
        if (!std::isfinite(cfg->norm[k])) return fail(SACX_EINVAL, "input normalisation must be finite");
    if ((uintptr_t)d_ws % kAlign) return fail(SACX_EINVAL, "surrogate workspace must be 256-byte aligned");
    if (cfg->d_packed && (uintptr_t)cfg->d_packed % 16) return fail(SACX_EINVAL, "packed weights must be 16-byte aligned");
    const SurPlan p = sur_plan(ctx);
    if (ws_bytes < p.total)
        return fail(SACX_ENOSPC, "surrogate workspace too small (%zu < %zu bytes)", ws_bytes, p.total);
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(SACX_EDEVICE, "cannot select the context device");
    char *w = (char *)d_ws;
    ctx->sur = *cfg;
    ctx->sur_pitch = p.pitch;
    ctx->sur_r = (float *)(w + p.off_r);
    ctx->sur_st = (HdDevStats *)(w + p.off_st);
    ctx->sur_k = (unsigned char *)(w + p.off_k);
    ctx->sur_x = w + p.off_x;
    ctx->sur_a1 = w + p.off_a1;
    ctx->sur_a2 = w + p.off_a2;
    ctx->sur_since = 0;
    ctx->sur_refreshes = 0;
    ctx->sur_tiles_checked = 0;
    const int64_t nr = (int64_t)10 * p.pitch * ctx->L.ny;
    hipLaunchKernelGGL(k_fill_f32, dim3(1024), dim3(256), 0, ctx->stream, ctx->sur_r, nr, -1.0f);
    // every tile flag 0 (fallen back) until the first check (its bytes as
    // float zeros: the flag region is a whole number of 256-byte blocks)
    const int64_t nk = (int64_t)(p.off_x - p.off_k) / 4;
    hipLaunchKernelGGL(k_fill_f32, dim3(256), dim3(256), 0, ctx->stream, (float *)ctx->sur_k, nk, 0.0f);
    hipLaunchKernelGGL(k_zero_stats, dim3(1), dim3(64), 0, ctx->stream, ctx->sur_st);
    HIPCHK(hipGetLastError());
    ctx->sur_on = true;
    return SACX_OK;
}

int sacx_hd_clear_surrogate(sacx_ctx *ctx) {
    if (!ctx) return fail(SACX_EINVAL, "ctx must not be NULL");
    ctx->sur_on = false;
    ctx->sur_r = nullptr;
    ctx->sur_k = nullptr;
    return SACX_OK;
}

int sacx_hd_ratio_buffer(sacx_ctx *ctx, float **d_r, int64_t *pitch) {
    if (!ctx || !d_r || !pitch) return fail(SACX_EINVAL, "ctx/d_r/pitch must not be NULL");
    if (!ctx->sur_on) return fail(SACX_ESTATE, "the surrogate is not set");
    *d_r = ctx->sur_r;
    *pitch = ctx->sur_pitch;
    return SACX_OK;
}

int sacx_hd_read_stats(sacx_ctx *ctx, sacx_hd_stats *out) {
    if (!ctx || !out) return fail(SACX_EINVAL, "ctx/out must not be NULL");
    if (!ctx->sur_on) return fail(SACX_ESTATE, "the surrogate is not set");
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(SACX_EDEVICE, "cannot select the context device");
    HdDevStats h;
    HIPCHK(hipMemcpyAsync(&h, ctx->sur_st, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    out->refreshes = ctx->sur_refreshes;
    out->tiles_checked = ctx->sur_tiles_checked;
    // reduce the counters' copies (maxima of non-negative doubles are the
    // maxima of their bit patterns)
    unsigned long long nf = 0, bu = 0, ba = 0;
    for (int k = 0; k < kStatSlots; ++k) {
        nf += h.tiles_fallback[k];
        bu = std::max(bu, h.err_used[k]);
        ba = std::max(ba, h.err_all[k]);
    }
    out->tiles_fallback = (int64_t)nf;
    double eu, ea;
    std::memcpy(&eu, &bu, sizeof(eu));
    std::memcpy(&ea, &ba, sizeof(ea));
    out->err_used = eu;
    out->err_all = ea;
    return SACX_OK;
}

int sacx_cnn_inputs(sacx_ctx *ctx, const float norm[12], void *d_x) {
    if (!ctx || !norm || !d_x) return fail(SACX_EINVAL, "ctx/norm/x must not be NULL");
    if (!ctx->initialized) return fail(SACX_ESTATE, "sacx_init_state has not been called");
    if (ctx->grid.background_on) return fail(SACX_EUNSUP, "network inputs need a context without background");
    if ((uintptr_t)d_x % 16) return fail(SACX_EINVAL, "input buffer must be 16-byte aligned");
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(SACX_EDEVICE, "cannot select the context device");
    InputNorm nm;
    for (int k = 0; k < 12; ++k) nm.v[k] = norm[k];
    HIPCHK(ctx->grid.precision == SACX_FP64 ? launch_cnn_inputs<double>(ratio_args<double>(ctx), nm, d_x, ctx->stream)
                                            : launch_cnn_inputs<float>(ratio_args<float>(ctx), nm, d_x, ctx->stream));
    return SACX_OK;
}

int sacx_hd_ratio_fields(sacx_ctx *ctx, float *d_r, float *d_d1, int64_t pitch) {
    if (!ctx || !d_r) return fail(SACX_EINVAL, "ctx/d_r must not be NULL");
    if (!ctx->initialized) return fail(SACX_ESTATE, "sacx_init_state has not been called");
    if (ctx->grid.background_on) return fail(SACX_EUNSUP, "ratio fields need a context without background");
    if (pitch < ctx->L.nx) return fail(SACX_EINVAL, "pitch must be >= nx");
    DeviceGuard dg(ctx->device);
    if (!dg.ok) return fail(SACX_EDEVICE, "cannot select the context device");
    int rc = fill_halo(ctx, ctx->U, NF, false);
    if (rc) return rc;
    HIPCHK(ctx->grid.precision == SACX_FP64
               ? launch_ratio_fields<double>(ratio_args<double>(ctx), d_r, d_d1, pitch, ctx->stream)
               : launch_ratio_fields<float>(ratio_args<float>(ctx), d_r, d_d1, pitch, ctx->stream));
    return SACX_OK;
}


}  // extern "C"

// ------------------------------------------------------------------ batches

struct sacx_batch {
    int n;
    int precision;
    int device;
    hipStream_t stream;
    std::vector<sacx_ctx *> *ctx;
    char *tab;          // BatchInst array
    int *sync;          // abort flag, queue counters, per-instance completion counters
    BatchItem *items;
    int *qinst;         // instances of each XCD queue
    int qoff[kBatchQueues], qlen[kBatchQueues], ioff[kBatchQueues + 1];
    int items_cap;
    int nitems;
    int nt;
    std::vector<int> *rows;
    bool dirty;
    unsigned long long gen_built;  // sum of the instance generations the table was built from
    int blocks;
};

namespace {

// polls of a batch dependency wait before it gives up (about a second);
// SACX_BATCH_SPIN_LIMIT replaces it (a debugging knob: 0 makes every wait
// that is not already satisfied abort the launch)
constexpr int kBatchSpinLimit = 1 << 20;
constexpr size_t kInstBytes = sizeof(BatchInst<double>) > sizeof(BatchInst<float>) ? sizeof(BatchInst<double>)
                                                                                    : sizeof(BatchInst<float>);

// ghost-fill pieces of one stage of a batched instance (a tube, one row
// with one-row tiles, fills only the ghost cells of its row)
int batch_fill_pieces(const sacx_grid &g) {
    const bool oned = g.ny == 1 && g.nx >= 2;
    const int64_t cells = (int64_t)NF * ((oned ? 0 : 2LL * G * (g.nx + 2 * G)) + 2LL * G * g.ny);
    return (int)((cells + kBatchFillPiece - 1) / kBatchFillPiece);
}

// entries of one stage's work lists (tiles of at most 58 columns, the
// narrowest tile, and one row; fill pieces)
int64_t batch_items_bound(int n, const sacx_grid *g) {
    int64_t t = 0;
    for (int i = 0; i < n; ++i) {
        const int64_t xt = (g[i].nx + 57) / 58;
        t += (g[i].ny == 1 ? xt : xt * g[i].ny) + batch_fill_pieces(g[i]);
    }
    return t;
}

struct BatchPlan {
    size_t off_tab, off_sync, off_items, off_qinst, off_inst, total;
    std::vector<size_t> inst_off, inst_bytes;
};

int batch_plan(int n, const sacx_grid *grids, const sacx_params *params, BatchPlan *P) {
    if (n < 1 || n > 65536) return fail(SACX_EINVAL, "batch size must be 1..65536");
    if (!grids || !params) return fail(SACX_EINVAL, "grids/params must not be NULL");
    P->inst_off.resize(n);
    P->inst_bytes.resize(n);
    for (int i = 0; i < n; ++i) {
        int rc = check_grid(&grids[i], &params[i]);
        if (rc) return rc;
        if (grids[i].precision != grids[0].precision) return fail(SACX_EINVAL, "all batch instances need one precision");
        if (grids[i].background_on) return fail(SACX_EUNSUP, "batched instances have no background");
        if (grids[i].nx < G) return fail(SACX_EUNSUP, "batched instances need nx >= %d", G);
        if (!params[i].hd_on) return fail(SACX_EUNSUP, "batched instances run with hyper-diffusion on");
        P->inst_bytes[i] = make_plan(&grids[i]).total;
    }
    size_t off = 0;
    P->off_tab = off; off += round_up((size_t)n * kInstBytes, kAlign);
    P->off_sync = off; off += round_up((size_t)(BATCH_SYNC0 + 2 * n) * sizeof(int), kAlign);
    P->off_items = off; off += round_up((size_t)batch_items_bound(n, grids) * sizeof(BatchItem), kAlign);
    P->off_qinst = off; off += round_up((size_t)n * sizeof(int), kAlign);
    P->off_inst = off;
    for (int i = 0; i < n; ++i) { P->inst_off[i] = off; off += round_up(P->inst_bytes[i], kAlign); }
    P->total = off;
    return SACX_OK;
}

__global__ void k_zero_ints(int *p, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

template <typename real>
int batch_build(sacx_batch *b) {
    const int n = b->n;
    const int TX = b->nt - 2 * G;
    std::vector<BatchInst<real>> tab(n);
    struct Costed { int64_t cost; BatchItem it; };
    std::vector<std::vector<Costed>> tiles(n);
    std::vector<int64_t> icost(n, 0);
    for (int i = 0; i < n; ++i) {
        sacx_ctx *c = (*b->ctx)[i];
        if (c->sur_on)
            return fail(SACX_EUNSUP, "instance %d has a learned coefficient set: the batch kernel uses the plain one", i);
        BatchInst<real> &I = tab[i];
        std::memset((void *)&I, 0, sizeof(I));
        void *const *S[4] = {c->U, c->B1, c->B2, c->B1};
        void *const *U[4] = {c->U, c->U, c->U, c->U};
        void *const *A[4] = {c->A, c->A, c->A, c->A};
        void *const *O1[4] = {c->B1, c->B2, c->B1, c->U};
        void *const *O2[4] = {c->B1, c->A, c->B1, c->U};
        for (int st = 0; st < 4; ++st) {
            StageArgs<real> a = stage_args<real>(c);
            a.nt = b->nt;
            a.ty = (*b->rows)[i];
            for (int f = 0; f < NF; ++f) {
                a.S[f] = (const real *)S[st][f];
                a.U[f] = (const real *)U[st][f];
                a.A[f] = (const real *)A[st][f];
                a.out1[f] = (real *)O1[st][f];
                a.out2[f] = (real *)O2[st][f];
            }
            if (!fields_uniform(a))
                return fail(SACX_EINVAL, "internal: instance %d buffers are not laid out at a uniform field stride", i);
            I.st[st] = a;
        }
        I.sk.cfl = c->params.cfl;
        I.sk.dx = c->dx;
        I.sk.dy = c->dy;
        for (int m = 0; m < 4; ++m) I.sk.c2[m] = c->params.c2[m];
        I.sk.ax = c->grid.nx > 1;
        I.sk.ay = c->grid.ny > 1;
        I.sc = c->sc;
        I.L = c->L;
        I.periodic_x = c->bc[0] == SACX_PERIODIC;
        I.periodic_y = c->bc[2] == SACX_PERIODIC;
        I.oned = (c->grid.ny == 1 && c->grid.nx >= 2) ? 1 : 0;
        const int xt = (c->L.nx + TX - 1) / TX;
        if (I.oned) {
            for (int x = 0; x < xt; ++x) tiles[i].push_back({1, {i, x, 0, BATCH_TILE}});
        } else {
            const int ty = (*b->rows)[i];
            const int yt = (c->L.ny + ty - 1) / ty;
            for (int y = 0; y < yt; ++y) {
                const int rows = std::min(ty, c->L.ny - y * ty);
                for (int x = 0; x < xt; ++x) tiles[i].push_back({(int64_t)rows + 2 * G, {i, x, y, BATCH_TILE}});
            }
        }
        std::stable_sort(tiles[i].begin(), tiles[i].end(), [](const Costed &p, const Costed &q) { return p.cost > q.cost; });
        I.ntiles = (int)tiles[i].size();
        I.nfill = batch_fill_pieces(c->grid);
        for (const Costed &t : tiles[i]) icost[i] += t.cost;
    }
    // instances to the XCD queues, most expensive first to the least loaded
    // queue; each queue's list: its instances most expensive first, each its
    // fill pieces then its tiles
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int p, int q) { return icost[p] > icost[q]; });
    std::vector<std::vector<int>> group(kBatchQueues);
    std::vector<int64_t> load(kBatchQueues, 0);
    for (int i : order) {
        const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        group[k].push_back(i);
        load[k] += icost[i];
    }
    std::vector<BatchItem> flat;
    std::vector<int> qinst;
    for (int k = 0; k < kBatchQueues; ++k) {
        b->qoff[k] = (int)flat.size();
        b->ioff[k] = (int)qinst.size();
        for (int i : group[k]) {
            qinst.push_back(i);
            for (int k2 = 0; k2 < tab[i].nfill; ++k2) flat.push_back({i, k2, 0, BATCH_FILL});
            for (const Costed &t : tiles[i]) flat.push_back(t.it);
        }
        b->qlen[k] = (int)flat.size() - b->qoff[k];
    }
    b->ioff[kBatchQueues] = (int)qinst.size();
    if ((int64_t)flat.size() > b->items_cap) return fail(SACX_ENOSPC, "batch work list exceeds its bound");
    b->nitems = (int)flat.size();
    HIPCHK(hipMemcpyAsync(b->qinst, qinst.data(), sizeof(int) * n, hipMemcpyHostToDevice, b->stream));
    HIPCHK(hipMemcpyAsync(b->tab, tab.data(), sizeof(BatchInst<real>) * n, hipMemcpyHostToDevice, b->stream));
    HIPCHK(hipMemcpyAsync(b->items, flat.data(), sizeof(BatchItem) * flat.size(), hipMemcpyHostToDevice, b->stream));
    // host vectors go out of scope: finish the copies first
    HIPCHK(hipStreamSynchronize(b->stream));
    int per_cu = 0, cus = 0;
    HIPCHK(batch_blocks_per_cu<real>(b->nt, &per_cu));
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device));
    if (per_cu < 1) return fail(SACX_EUNSUP, "batched kernel does not fit on a compute unit with %d threads", b->nt);
    b->blocks = per_cu * cus;
    b->dirty = false;
    return SACX_OK;
}

template <typename real>
void batch_args(const sacx_batch *b, int nsteps, int spin, BatchArgs<real> *a) {
    a->inst = (const BatchInst<real> *)b->tab;
    a->n = b->n;
    a->items = b->items;
    a->qinst = b->qinst;
    for (int k = 0; k < kBatchQueues; ++k) { a->qoff[k] = b->qoff[k]; a->qlen[k] = b->qlen[k]; a->ioff[k] = b->ioff[k]; }
    a->ioff[kBatchQueues] = b->ioff[kBatchQueues];
    a->sync = b->sync;
    a->nsteps = nsteps;
    a->spin_limit = spin;
}

}  // namespace

extern "C" {

int sacx_batch_workspace_size(int32_t n, const sacx_grid *grids, const sacx_params *params, size_t *bytes) {
    if (!bytes) return fail(SACX_EINVAL, "bytes must not be NULL");
    BatchPlan P;
    int rc = batch_plan(n, grids, params, &P);
    if (rc) return rc;
    *bytes = P.total;
    return SACX_OK;
}

int sacx_batch_destroy(sacx_batch *b) {
    if (!b) return SACX_OK;
    {
        DeviceGuard dg(b->device);
        (void)hipStreamSynchronize(b->stream);
    }
    if (b->ctx)
        for (sacx_ctx *c : *b->ctx) sacx_destroy(c);
    delete b->ctx;
    delete b->rows;
    delete b;
    return SACX_OK;
}

int sacx_batch_create(int32_t n, const sacx_grid *grids, const sacx_params *params, const int32_t *bc, void *d_ws,
                      size_t ws_bytes, void *hip_stream, sacx_batch **out) {
    if (!out) return fail(SACX_EINVAL, "out must not be NULL");
    *out = nullptr;
    BatchPlan P;
    int rc = batch_plan(n, grids, params, &P);
    if (rc) return rc;
    if (!d_ws || ((uintptr_t)d_ws) % kAlign) return fail(SACX_EINVAL, "workspace must be non-NULL and 256-byte aligned");
    if (ws_bytes < P.total) return fail(SACX_ENOSPC, "workspace has %zu bytes, %zu needed", ws_bytes, P.total);
    sacx_batch *b = new (std::nothrow) sacx_batch;
    if (!b) return fail(SACX_EINVAL, "out of host memory");
    std::memset((void *)b, 0, sizeof(*b));
    b->ctx = new (std::nothrow) std::vector<sacx_ctx *>();
    b->rows = new (std::nothrow) std::vector<int>();
    if (!b->ctx || !b->rows) { sacx_batch_destroy(b); return fail(SACX_EINVAL, "out of host memory"); }
    b->n = n;
    b->precision = grids[0].precision;
    b->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&b->device) != hipSuccess) { sacx_batch_destroy(b); return fail(SACX_EDEVICE, "no current device"); }
    char *ws = (char *)d_ws;
    b->tab = ws + P.off_tab;
    b->sync = (int *)(ws + P.off_sync);
    b->items = (BatchItem *)(ws + P.off_items);
    b->qinst = (int *)(ws + P.off_qinst);
    b->items_cap = (int)batch_items_bound(n, grids);
    b->nt = b->precision == SACX_FP64 ? 128 : 256;
    hipLaunchKernelGGL(k_zero_ints, dim3(8), dim3(256), 0, b->stream, b->sync, BATCH_SYNC0 + 2 * n);
    if (hipGetLastError() != hipSuccess) {
        sacx_batch_destroy(b);
        return fail(SACX_EDEVICE, "clearing the batch's synchronisation words failed");
    }
    for (int i = 0; i < n; ++i) {
        sacx_ctx *c = nullptr;
        rc = sacx_create(&grids[i], &params[i], ws + P.inst_off[i], P.inst_bytes[i], hip_stream, &c);
        if (rc) { sacx_batch_destroy(b); return rc; }
        b->ctx->push_back(c);
        if (bc) {
            for (int k = 0; k < 4; ++k)
                if (bc[4 * i + k] == SACX_EXCHANGE) {
                    sacx_batch_destroy(b);
                    return fail(SACX_EUNSUP, "instance %d: a batched instance cannot have exchange boundaries", i);
                }
            rc = sacx_set_boundaries(c, bc + 4 * i);
            if (rc) { sacx_batch_destroy(b); return rc; }
        }
        b->rows->push_back(grids[i].ny == 1 ? 1 : std::min(64, grids[i].ny));
    }
    b->dirty = true;
    *out = b;
    return SACX_OK;
}

int sacx_batch_context(sacx_batch *b, int32_t i, sacx_ctx **out) {
    if (!b || !out) return fail(SACX_EINVAL, "batch/out must not be NULL");
    if (i < 0 || i >= b->n) return fail(SACX_EINVAL, "instance %d out of range", i);
    *out = (*b->ctx)[i];
    return SACX_OK;
}

int sacx_batch_set_tiles(sacx_batch *b, int32_t threads, const int32_t *rows) {
    if (!b) return fail(SACX_EINVAL, "batch must not be NULL");
    if (threads != 0 && threads != 64 && threads != 128 && threads != 256)
        return fail(SACX_EINVAL, "threads must be 64, 128 or 256");
    if (rows)
        for (int i = 0; i < b->n; ++i)
            if (rows[i] < 1 || rows[i] > 4096) return fail(SACX_EINVAL, "rows[%d] = %d out of 1..4096", i, rows[i]);
    if (threads) b->nt = threads;
    if (rows)
        for (int i = 0; i < b->n; ++i) (*b->rows)[i] = (*b->ctx)[i]->grid.ny == 1 ? 1 : rows[i];
    b->dirty = true;
    return SACX_OK;
}

int sacx_batch_advance(sacx_batch *b, int32_t nsteps, int32_t sync) {
    if (!b) return fail(SACX_EINVAL, "batch must not be NULL");
    if (nsteps < 0) return fail(SACX_EINVAL, "nsteps must be >= 0");
    unsigned long long gsum = 0;
    for (sacx_ctx *c : *b->ctx) {
        if (!c->initialized) return fail(SACX_ESTATE, "every batch instance needs sacx_init_state first");
        if (has_exchange(c)) return fail(SACX_ESTATE, "a batched instance cannot have exchange boundaries");
        if (c->stage_next) return fail(SACX_ESTATE, "a batched instance has a step begun with sacx_stage in progress");
        gsum += c->gen;
    }
    DeviceGuard dg(b->device);
    if (!dg.ok) return fail(SACX_EDEVICE, "cannot select the batch device");
    if (b->dirty || gsum != b->gen_built) {
        int rc = b->precision == SACX_FP64 ? batch_build<double>(b) : batch_build<float>(b);
        if (rc) return rc;
        b->gen_built = gsum;
    }
    int spin = kBatchSpinLimit;
    if (const char *env = getenv("SACX_BATCH_SPIN_LIMIT")) spin = std::max(0, atoi(env));
    // steps per launch: every queue index stays within an int
    int qmax = 1;
    for (int k = 0; k < kBatchQueues; ++k) qmax = std::max(qmax, b->qlen[k]);
    const int per_launch = (int)std::max<int64_t>(1, std::min<int64_t>(4096, (INT32_MAX - 2LL * b->n) / (4LL * qmax)));
    for (int done = 0; done < nsteps; done += per_launch) {
        const int k = std::min(per_launch, nsteps - done);
        // the queue counters, block counts and completion counters start at
        // zero; the abort flag is sticky (a launch after an abandoned one
        // does nothing)
        hipLaunchKernelGGL(k_zero_ints, dim3(8), dim3(256), 0, b->stream, b->sync + BATCH_QUEUE0,
                           BATCH_SYNC0 - BATCH_QUEUE0 + 2 * b->n);
        if (b->precision == SACX_FP64) {
            BatchArgs<double> a;
            batch_args(b, k, spin, &a);
            HIPCHK(launch_batch<double>(a, b->nt, b->blocks, b->stream));
        } else {
            BatchArgs<float> a;
            batch_args(b, k, spin, &a);
            HIPCHK(launch_batch<float>(a, b->nt, b->blocks, b->stream));
        }
    }
    if (sync) {
        // a wait that exceeded its bound left the batch part-way through a
        // launch: report it (the instance states are then undefined, and the
        // flag stays set, so later launches of this batch do nothing)
        int ab = 0;
        HIPCHK(hipMemcpyAsync(&ab, b->sync + BATCH_ABORT, sizeof(int), hipMemcpyDeviceToHost, b->stream));
        HIPCHK(hipStreamSynchronize(b->stream));
        if (ab) return fail(SACX_EDEVICE, "a batch dependency wait exceeded its bound; the instance states are undefined");
    }
    if (sync) {
        HIPCHK(hipStreamSynchronize(b->stream));
        for (sacx_ctx *c : *b->ctx) {
            int np = 0;
            HIPCHK(hipMemcpy(&np, &c->sc->nonphys, sizeof(int), hipMemcpyDeviceToHost));
            if (np) return fail(SACX_ENONPHYS, "a batch instance reached a non-physical state");
        }
    }
    return SACX_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ decomposed domain

namespace {

__global__ void k_zero_doubles(double *p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0.0;
}

constexpr size_t kDomainAlign = 256;

// the neighbour across `side` of subdomain (a, b) in a px x py layout,
// wrapping around the domain (a periodic image is a neighbour too)
int domain_neighbour(int px, int py, int a, int b, int side) {
    switch (side) {
        case 0: return ((a - 1 + px) % px) + b * px;
        case 1: return ((a + 1) % px) + b * px;
        case 2: return a + ((b - 1 + py) % py) * px;
        default: return a + ((b + 1) % py) * px;
    }
}

bool domain_edge(int px, int py, int a, int b, int side) {
    switch (side) {
        case 0: return a == 0;
        case 1: return a == px - 1;
        case 2: return b == 0;
        default: return b == py - 1;
    }
}

}  // namespace

struct sacx_domain {
    int px, py;
    std::vector<sacx_ctx *> *subs;            // row-major, px x py
    std::vector<std::array<void *, 4>> *buf;  // per subdomain and side: the strip it packs (exchange sides)
    std::vector<std::array<int, 4>> *nbr;     // per subdomain and side: the neighbour (exchange sides)
    std::vector<std::array<int, 4>> *bc;      // per subdomain: the boundary kinds the layout was checked with
    double *cmax;                             // the whole domain's wave-speed maxima (device)
};

extern "C" {

// checks shared by the size query and creation; on success *bytes is the
// caller memory the domain needs
static int domain_check(int32_t px, int32_t py, sacx_ctx *const *subs, size_t *bytes) {
    if (px < 1 || py < 1 || (int64_t)px * py > 4096) return fail(SACX_EINVAL, "px, py must be >= 1 (at most 4096 subdomains)");
    if (!subs || !bytes) return fail(SACX_EINVAL, "subs/bytes must not be NULL");
    const int n = px * py;
    for (int i = 0; i < n; ++i) {
        if (!subs[i]) return fail(SACX_EINVAL, "subdomain %d is NULL", i);
        for (int j = 0; j < i; ++j)
            if (subs[j] == subs[i]) return fail(SACX_EINVAL, "subdomain %d appears twice", i);
    }
    const sacx_ctx *c0 = subs[0];
    size_t total = kDomainAlign;  // the maxima
    for (int b = 0; b < py; ++b)
        for (int a = 0; a < px; ++a) {
            const int i = a + b * px;
            const sacx_ctx *c = subs[i];
            if (!c->initialized) return fail(SACX_ESTATE, "subdomain %d has no state (sacx_init_state)", i);
            if (c->device != c0->device || c->stream != c0->stream)
                return fail(SACX_EINVAL, "subdomain %d is not on the device and stream of subdomain 0", i);
            if (c->grid.precision != c0->grid.precision) return fail(SACX_EINVAL, "subdomain %d has another precision", i);
            if (std::memcmp(&c->params, &c0->params, sizeof(sacx_params)) != 0)
                return fail(SACX_EINVAL, "subdomain %d has other scheme parameters", i);
            if (c->dx != c0->dx || c->dy != c0->dy)
                return fail(SACX_EINVAL, "subdomain %d has another grid spacing (sacx_set_spacing)", i);
            if (c->sur_on) return fail(SACX_ESTATE, "subdomain %d has a learned coefficient", i);
            for (int side = 0; side < 4; ++side) {
                const bool edge = domain_edge(px, py, a, b, side);
                if (c->bc[side] != SACX_EXCHANGE) {
                    if (!edge) return fail(SACX_EINVAL, "subdomain %d side %d borders a subdomain but is not EXCHANGE", i, side);
                    continue;
                }
                const sacx_ctx *nb = subs[domain_neighbour(px, py, a, b, side)];
                if (nb->bc[side ^ 1] != SACX_EXCHANGE)
                    return fail(SACX_EINVAL, "subdomain %d side %d: the neighbour's facing side is not EXCHANGE", i, side);
                if ((side < 2 && nb->grid.ny != c->grid.ny) || (side >= 2 && nb->grid.nx != c->grid.nx))
                    return fail(SACX_EINVAL, "subdomain %d side %d: the neighbour's strip has another length", i, side);
                size_t sb = 0;
                int rc = sacx_halo_buffer_size(c, side, &sb);
                if (rc) return rc;
                total += round_up(sb, kDomainAlign);
            }
        }
    *bytes = total;
    return SACX_OK;
}

int sacx_domain_buffer_size(int32_t px, int32_t py, sacx_ctx *const *subs, size_t *bytes) {
    return domain_check(px, py, subs, bytes);
}

int sacx_domain_create(int32_t px, int32_t py, sacx_ctx *const *subs, void *d_buf, size_t buf_bytes, sacx_domain **out) {
    if (!out) return fail(SACX_EINVAL, "out must not be NULL");
    *out = nullptr;
    size_t need = 0;
    int rc = domain_check(px, py, subs, &need);
    if (rc) return rc;
    if (!d_buf) return fail(SACX_EINVAL, "buffer pointer is NULL");
    if (((uintptr_t)d_buf) % kDomainAlign) return fail(SACX_EINVAL, "buffer must be 256-byte aligned");
    if (buf_bytes < need) return fail(SACX_ENOSPC, "buffer has %zu bytes, %zu needed", buf_bytes, need);
    sacx_domain *d = new (std::nothrow) sacx_domain();
    if (!d) return fail(SACX_EINVAL, "out of host memory");
    d->px = px;
    d->py = py;
    d->subs = new (std::nothrow) std::vector<sacx_ctx *>(subs, subs + (size_t)px * py);
    d->buf = new (std::nothrow) std::vector<std::array<void *, 4>>((size_t)px * py);
    d->nbr = new (std::nothrow) std::vector<std::array<int, 4>>((size_t)px * py);
    d->bc = new (std::nothrow) std::vector<std::array<int, 4>>((size_t)px * py);
    if (!d->subs || !d->buf || !d->nbr || !d->bc) {
        sacx_domain_destroy(d);
        return fail(SACX_EINVAL, "out of host memory");
    }
    char *p = (char *)d_buf;
    d->cmax = (double *)p;
    p += kDomainAlign;
    for (int b = 0; b < py; ++b)
        for (int a = 0; a < px; ++a) {
            const int i = a + b * px;
            for (int side = 0; side < 4; ++side) {
                (*d->buf)[i][side] = nullptr;
                (*d->nbr)[i][side] = -1;
                (*d->bc)[i][side] = subs[i]->bc[side];
                if (subs[i]->bc[side] != SACX_EXCHANGE) continue;
                size_t sb = 0;
                sacx_halo_buffer_size(subs[i], side, &sb);
                (*d->buf)[i][side] = p;
                (*d->nbr)[i][side] = domain_neighbour(px, py, a, b, side);
                p += round_up(sb, kDomainAlign);
            }
        }
    *out = d;
    return SACX_OK;
}

int sacx_domain_destroy(sacx_domain *d) {
    if (!d) return SACX_OK;
    delete d->subs;
    delete d->buf;
    delete d->nbr;
    delete d->bc;
    delete d;
    return SACX_OK;
}

// both strips of one direction of a context's stage input in one launch
// (the two-sided form of the pack / unpack kernels): b0 for the low side,
// b1 for the high side
static int halo_io_both(sacx_ctx *ctx, int dir, void *b0, void *b1, bool pack) {
    ProfScope ps(ctx, 4);
    const Layout &L = ctx->L;
    const int T = 256;
    void *const *S = stage_input(ctx);
    const bool f64 = ctx->grid.precision == SACX_FP64;
    const int along = dir == 0 ? L.ny : L.nx + 2 * G;
    dim3 g((along + T - 1) / T, NF, 2);
    const DevScalars *none = nullptr;
    if (dir == 0) {
        if (f64) {
            if (pack) hipLaunchKernelGGL(k_pack_x<double>, g, dim3(T), 0, ctx->stream, fptr<double>(S, NF), NF, L, (double *)b0, (double *)b1, 2, none);
            else hipLaunchKernelGGL(k_unpack_x<double>, g, dim3(T), 0, ctx->stream, fptr<double>(S, NF), NF, L, (const double *)b0, (const double *)b1, 2, none);
        } else {
            if (pack) hipLaunchKernelGGL(k_pack_x<float>, g, dim3(T), 0, ctx->stream, fptr<float>(S, NF), NF, L, (float *)b0, (float *)b1, 2, none);
            else hipLaunchKernelGGL(k_unpack_x<float>, g, dim3(T), 0, ctx->stream, fptr<float>(S, NF), NF, L, (const float *)b0, (const float *)b1, 2, none);
        }
    } else {
        if (f64) {
            if (pack) hipLaunchKernelGGL(k_pack_y<double>, g, dim3(T), 0, ctx->stream, fptr<double>(S, NF), NF, L, (double *)b0, (double *)b1, 2, none);
            else hipLaunchKernelGGL(k_unpack_y<double>, g, dim3(T), 0, ctx->stream, fptr<double>(S, NF), NF, L, (const double *)b0, (const double *)b1, 2, none);
        } else {
            if (pack) hipLaunchKernelGGL(k_pack_y<float>, g, dim3(T), 0, ctx->stream, fptr<float>(S, NF), NF, L, (float *)b0, (float *)b1, 2, none);
            else hipLaunchKernelGGL(k_unpack_y<float>, g, dim3(T), 0, ctx->stream, fptr<float>(S, NF), NF, L, (const float *)b0, (const float *)b1, 2, none);
        }
    }
    HIPCHK(hipGetLastError());
    return SACX_OK;
}

// one direction's exchange: every subdomain packs its exchange strips, then
// unpacks the strips its neighbours packed facing it (both sides of the
// direction in one launch where both are exchange sides)
static int domain_exchange(sacx_domain *d, int dir) {
    const int n = d->px * d->py;
    const int lo = 2 * dir, hi = 2 * dir + 1;
    for (int i = 0; i < n; ++i) {
        sacx_ctx *c = (*d->subs)[i];
        void *const *b = (*d->buf)[i].data();
        int rc = SACX_OK;
        if (b[lo] && b[hi]) rc = halo_io_both(c, dir, b[lo], b[hi], true);
        else if (b[lo]) rc = sacx_halo_pack(c, lo, b[lo]);
        else if (b[hi]) rc = sacx_halo_pack(c, hi, b[hi]);
        if (rc) return rc;
    }
    for (int i = 0; i < n; ++i) {
        sacx_ctx *c = (*d->subs)[i];
        void *const *b = (*d->buf)[i].data();
        // the strip a side receives is the one its neighbour packed facing it
        void *from_lo = b[lo] ? (*d->buf)[(*d->nbr)[i][lo]][hi] : nullptr;
        void *from_hi = b[hi] ? (*d->buf)[(*d->nbr)[i][hi]][lo] : nullptr;
        int rc = SACX_OK;
        if (from_lo && from_hi) rc = halo_io_both(c, dir, from_lo, from_hi, false);
        else if (from_lo) rc = sacx_halo_unpack(c, lo, from_lo);
        else if (from_hi) rc = sacx_halo_unpack(c, hi, from_hi);
        if (rc) return rc;
    }
    return SACX_OK;
}

int sacx_domain_advance(sacx_domain *d, int32_t nsteps) {
    if (!d) return fail(SACX_EINVAL, "domain must not be NULL");
    if (nsteps < 0) return fail(SACX_EINVAL, "nsteps must be >= 0");
    const int n = d->px * d->py;
    for (int i = 0; i < n; ++i) {
        const sacx_ctx *c = (*d->subs)[i];
        if (c->stage_next) return fail(SACX_ESTATE, "subdomain %d has a step in progress", i);
        for (int side = 0; side < 4; ++side)
            if (c->bc[side] != (*d->bc)[i][side])
                return fail(SACX_ESTATE, "subdomain %d changed its boundaries after the domain was created", i);
        if (c->sur_on) return fail(SACX_ESTATE, "subdomain %d has a learned coefficient", i);
    }
    sacx_ctx *c0 = (*d->subs)[0];
    DeviceGuard dg(c0->device);
    if (!dg.ok) return fail(SACX_EDEVICE, "cannot select the domain's device");
    for (int step = 0; step < nsteps; ++step) {
        hipLaunchKernelGGL(k_zero_doubles, dim3(1), dim3(64), 0, c0->stream, d->cmax, 2);
        HIPCHK(hipGetLastError());
        int rc;
        for (int i = 0; i < n; ++i)
            if ((rc = sacx_wave_speeds_max((*d->subs)[i], d->cmax))) return rc;
        for (int s = 0; s < 4; ++s) {
            for (int i = 0; i < n; ++i)
                if ((rc = sacx_fill_boundaries((*d->subs)[i], 0))) return rc;
            if ((rc = domain_exchange(d, 0))) return rc;
            for (int i = 0; i < n; ++i)
                if ((rc = sacx_fill_boundaries((*d->subs)[i], 1))) return rc;
            if ((rc = domain_exchange(d, 1))) return rc;
            for (int i = 0; i < n; ++i)
                if ((rc = sacx_stage((*d->subs)[i], d->cmax, 1, nullptr))) return rc;
        }
    }
    return SACX_OK;
}

}  // extern "C"
