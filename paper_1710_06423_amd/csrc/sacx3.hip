// sacx3.hip -- the three-dimensional form of the scheme (paper sections 2
// and 8: the code is implemented in 3-D): kernels, host runtime and the
// sacx3_* C ABI.
//
// A stage of RK4 is two launches over the ghosted state (G = 3 cells on
// every side):
//
//   k3_faces   the hyper-diffusion face quantities G_d(q) = nu_f(q) d1_f(q) / h_d
//              for the three face directions and the seven quantities of each
//              face set (rho~, eps~, v_x, v_y, v_z and the two field
//              components across the face), on the faces the fluxes need:
//              along d from cell -1 to n_d - 1, across d from -1 to n.  It
//              marches up z over a tile of (x, y) columns: each plane's
//              primitives go to LDS (the x- and y-face coefficient ratios and
//              the compression s take their neighbours there); the z-face
//              ratio takes its six planes from a per-thread register window.
//   k3_stage   L(S) and the RK4 stage combine: ideal fluxes differenced with
//              the fourth-order central difference (x and y fluxes through
//              LDS, the z flux from a register window), the hyper-diffusive
//              face fluxes H_d (hyper-viscous stress, hyper-resistive e.m.f.,
//              the energy they carry) from the stored G and their divergence,
//              then the storage-saving RK4 combine; stage 4 also reduces the
//              wave speeds of the new state.  The G that the x- and y-face
//              fluxes of a plane read are staged in LDS tiles by loads that
//              write LDS directly, issued before the plane's state loads.
//
// Splitting the stage in two moves the 21 face quantities through HBM (a
// fused 3-D kernel would need the z windows of both launches in one thread):
// as laid out, about 592 B per cell and stage against the 192 B of the
// stage's own state accesses.
//
// Arithmetic: every value is the IEEE operation sequence of the scheme's
// definition in its storage-saving arrangement (divisions by grid constants
// as multiplications by FP64 reciprocals, no contraction: this unit is built
// with -ffp-contract=off), so results are bit-identical to the test oracle's
// low-storage form.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "sacx3.h"
#include "sacx_internal.h"
#include "sacx_tile.h"

namespace sacx3i {

using sacx::G;

constexpr int NF3 = 8;    // evolved fields
constexpr int NQF = 7;    // quantities of one face set
constexpr int kAlign = 256;
constexpr int kPartials = 1024;
constexpr int TXF = 32, TYF = 8;   // column tile of both launches
constexpr int NT = TXF * TYF;

// field slots of the state
enum { FR = 0, FMX = 1, FMY = 2, FMZ = 3, FE = 4, FBX = 5, FBY = 6, FBZ = 7 };
// primitive slots of the face launch's LDS planes
enum { PR = 0, PE = 1, PVX = 2, PVY = 3, PVZ = 4, PBX = 5, PBY = 6, PBZ = 7, NP = 8 };
// G slots of a face set: rho~, eps~, v_x, v_y, v_z, first and second field
// component across the face (x faces: B_y, B_z; y faces: B_x, B_z; z faces:
// B_x, B_y)
enum { GR = 0, GE = 1, GVX = 2, GVY = 3, GVZ = 4, GB1 = 5, GB2 = 6 };

__host__ __device__ constexpr int gclass(int q) { return q == GR ? 0 : (q == GE ? 1 : (q >= GB1 ? 3 : 2)); }

// Storage of one field: nz + 2G planes of ny + 2G rows of `pitch` elements;
// cell (i, j, k), each index from -G, at xoff + i + (j + G) pitch + (k + G) plane.
// xoff puts cell column 0 of every row on a 256-byte boundary.
struct Layout3 {
    int nx, ny, nz;
    int pitch, xoff;
    int64_t plane, field_elems;
    __host__ __device__ int64_t at(int i, int j, int k) const {
        return (int64_t)xoff + i + (int64_t)(j + G) * pitch + (int64_t)(k + G) * plane;
    }
    // byte offset of cell (i, j, k) (every field array is below 4 GiB)
    __device__ uint32_t off(int i, int j, int k) const {
        return (uint32_t)(xoff + i + (j + G) * pitch) * 8u + (uint32_t)(k + G) * (uint32_t)(plane * 8);
    }
};

// step scalars on the device; the wave-speed accumulators hold IEEE bit
// patterns of non-negative doubles (unsigned max is the floating max)
struct Dev3 {
    double t, dt, cmax, t_end, hdt, dt6;
    double kd2[3][4];                 // c2 * h_d * c_max per constant class
    unsigned long long cacc[2][3];    // [slot][x, y, z]
    double last_c[3], last_cmax;
    long long steps;
    int cur, active, nonphys, pad;
};

// grid constants, computed once on the host in FP64
struct Consts3 {
    double gamma, gm1, igm1, third;
    double h[3], ih[3], i12[3], i2[3];
    double kds[3][4];                 // cshk * h_d * h_d per constant class
    double cfl, c2[4];
    int act[3];                       // direction has more than one cell
    int pad;
};

struct Face3Args {
    const double *S;   // stage input: field f at S + f * fs
    double *Gf;        // face quantities: (direction d, slot q) at Gf + (7 d + q) * fs
    int64_t fs;
    Layout3 L;
    Consts3 k;
    const Dev3 *sc;
    int tz, ntx, nty;
};

struct Stage3Args {
    const double *S;   // stage input (differenced; ghosts filled)
    const double *U;   // step start state (pointwise)
    const double *A;   // RK accumulator (stage 4)
    double *out1;      // stage output
    double *out2;      // accumulator output (stage 2)
    const double *Gf;
    int64_t fs;
    Layout3 L;
    Consts3 k;
    Dev3 *sc;
    int tz, ntx, nty;
    int cross;
};

// The chip hands consecutive blocks to its 8 XCDs in turn; blocks are
// renumbered so that runs of 4 neighbouring tiles share one XCD (and its L2)
// for the apron they both read.  A bijection of the block indices.
__device__ __forceinline__ int xcd_block() {
    const int n = (int)gridDim.x, b = (int)blockIdx.x;
    const int x = b % 8, i = b / 8;
    return b < n - n % 32 ? ((i / 4) * 8 + x) * 4 + i % 4 : b;
}

// Global accesses take a wave-uniform array base plus a 32-bit per-lane byte
// offset (every field array is below 4 GiB), which the compiler turns into
// scalar-base addressing instead of per-lane 64-bit address arithmetic.
__device__ __forceinline__ double ldo(const double *base, uint32_t off) {
    return *(const double *)((const char *)base + off);
}
__device__ __forceinline__ void sto(double *base, uint32_t off, double v) { *(double *)((char *)base + off) = v; }

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }
__device__ __forceinline__ int ring3(int r) { return (r + 3 * 4096) % 3; }

// ---------------------------------------------------------------- face launch

template <int TX, int TY>
struct FaceLds {
    double q[2][NP][TY + 5][TX + 5];   // primitives of planes r, r-1 (by parity) over the tile + apron
    double vz[3][TY + 1][TX + 1];      // v_z over the compression region, ring of 3 planes
    double s[TY + 1][TX + 1];          // compression s of plane r-1
};

template <int TX, int TY>
__global__ __launch_bounds__(TX *TY, 2) void k3_faces(Face3Args a) {
    __shared__ FaceLds<TX, TY> lds;
    constexpr int BX = TX + 5, BY = TY + 5, BOX = BX * BY;
    constexpr int SX = TX + 1, SY = TY + 1, SREG = SX * SY;
    const Dev3 *sc = a.sc;
    if (!sc->active) return;
    const Layout3 L = a.L;
    const Consts3 &kc = a.k;
    const int64_t fs = a.fs;
    const int blk = xcd_block();
    const int X0 = -1 + (blk % a.ntx) * TX;
    const int Y0 = -1 + ((blk / a.ntx) % a.nty) * TY;
    const int zb = -1 + (blk / (a.ntx * a.nty)) * a.tz;
    const int ze = min(zb + a.tz, L.nz + 1);
    const int tid = threadIdx.x, tx = tid % TX, ty = tid / TX;
    const int x = X0 + tx, y = Y0 + ty;
    const bool colv = x <= L.nx && y <= L.ny;
    const bool xf = colv && x <= L.nx - 1;   // owns an x face
    const bool yf = colv && y <= L.ny - 1;   // owns a y face
    const double gm1 = kc.gm1, igm1 = kc.igm1;
    const double half = 0.5, zero = 0.0;
    // the step's coefficients, read once: read where they are used, each
    // would be read again behind the previous face store (which may alias it)
    double kd2[3][4];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int c = 0; c < 4; ++c) kd2[d][c] = sc->kd2[d][c];

    double w[NQF][6];   // z-face set rho~, eps~, v_x, v_y, v_z, B_x, B_y of planes r-5..r
#pragma unroll
    for (int q = 0; q < NQF; ++q)
#pragma unroll
        for (int k = 0; k < 6; ++k) w[q][k] = 0.0;
    double sA = 0.0, sB = 0.0;   // own column's s of planes r-3, r-2

    const int rend = max(min(ze, L.nz) + 2, ze + 1);
    for (int r = zb - 2; r <= rend; ++r) {
        const int slot = r & 1, pslot = slot ^ 1;
        // ---- P1: plane r over the tile and its apron -> primitives in LDS
        for (int p = tid; p < BOX; p += TX * TY) {
            const int bx = p % BX, by = p / BX;
            const int gx = clampi(X0 - 2 + bx, -G, L.nx + G - 1), gy = clampi(Y0 - 2 + by, -G, L.ny + G - 1);
            const uint32_t o = L.off(gx, gy, r);
            const double rt = ldo(a.S, o), mx = ldo(a.S + FMX * fs, o), my = ldo(a.S + FMY * fs, o),
                         mz = ldo(a.S + FMZ * fs, o);
            const double et = ldo(a.S + FE * fs, o), bx_ = ldo(a.S + FBX * fs, o), by_ = ldo(a.S + FBY * fs, o),
                         bz_ = ldo(a.S + FBZ * fs, o);
            const double ir = 1.0 / rt;
            const double ux = mx * ir, uy = my * ir, uz = mz * ir;
            const double kin = half * ((mx * ux + my * uy) + mz * uz);
            const double b2 = (bx_ * bx_ + by_ * by_) + bz_ * bz_;
            const double pk = gm1 * ((et - kin) - half * b2);
            lds.q[slot][PR][by][bx] = rt;
            lds.q[slot][PE][by][bx] = pk * igm1;
            lds.q[slot][PVX][by][bx] = ux;
            lds.q[slot][PVY][by][bx] = uy;
            lds.q[slot][PVZ][by][bx] = uz;
            lds.q[slot][PBX][by][bx] = bx_;
            lds.q[slot][PBY][by][bx] = by_;
            lds.q[slot][PBZ][by][bx] = bz_;
            if (bx >= 2 && bx < 2 + SX && by >= 2 && by < 2 + SY) lds.vz[ring3(r)][by - 2][bx - 2] = uz;
        }
        __syncthreads();
        // ---- P2: own column's z window; compression s of plane r-1
        {
            const int bx = tx + 2, by = ty + 2;
            const int src[NQF] = {PR, PE, PVX, PVY, PVZ, PBX, PBY};
#pragma unroll
            for (int q = 0; q < NQF; ++q) {
#pragma unroll
                for (int k = 0; k < 5; ++k) w[q][k] = w[q][k + 1];
                w[q][5] = lds.q[slot][src[q]][by][bx];
            }
        }
        const bool splane = r - 1 >= zb && r - 1 <= ze;
        if (splane) {
            const int z0 = ring3(r), z2 = ring3(r - 2);
            for (int p = tid; p < SREG; p += TX * TY) {
                const int sx = p % SX, sy = p / SX;
                const int bx = sx + 2, by = sy + 2;
                const double dv = ((lds.q[pslot][PVX][by][bx + 1] - lds.q[pslot][PVX][by][bx - 1]) * kc.i2[0] +
                                   (lds.q[pslot][PVY][by + 1][bx] - lds.q[pslot][PVY][by - 1][bx]) * kc.i2[1]) +
                                  (lds.vz[z0][sy][sx] - lds.vz[z2][sy][sx]) * kc.i2[2];
                lds.s[sy][sx] = fmax(zero, -dv);
            }
        }
        __syncthreads();
        // ---- P3: x and y faces of plane r-1, z face (r-3)+1/2
        const int wpl = r - 1;
        if (wpl >= zb && wpl < ze) {
            if (xf) {
                const int by = ty + 2;
                const double sf = fmax(lds.s[ty][tx], lds.s[ty][tx + 1]);
                const int src[NQF] = {PR, PE, PVX, PVY, PVZ, PBY, PBZ};
                const uint32_t o = L.off(x, y, wpl);
#pragma unroll
                for (int q = 0; q < NQF; ++q) {
                    const double *row = &lds.q[pslot][src[q]][by][0];
                    const double q0 = row[tx], q1 = row[tx + 1], q2 = row[tx + 2], q3 = row[tx + 3],
                                 q4 = row[tx + 4], q5 = row[tx + 5];
                    const double R = sacx::hd_ratio(q0, q1, q2, q3, q4, q5);
                    const int cl = gclass(q);
                    const double nu = kd2[0][cl] * R + kc.kds[0][cl] * sf;
                    sto(a.Gf + (0 * NQF + q) * fs, o, (nu * (q3 - q2)) * kc.ih[0]);
                }
            }
            if (yf) {
                const int bx = tx + 2;
                const double sf = fmax(lds.s[ty][tx], lds.s[ty + 1][tx]);
                const int src[NQF] = {PR, PE, PVX, PVY, PVZ, PBX, PBZ};
                const uint32_t o = L.off(x, y, wpl);
#pragma unroll
                for (int q = 0; q < NQF; ++q) {
                    const double q0 = lds.q[pslot][src[q]][ty][bx], q1 = lds.q[pslot][src[q]][ty + 1][bx],
                                 q2 = lds.q[pslot][src[q]][ty + 2][bx], q3 = lds.q[pslot][src[q]][ty + 3][bx],
                                 q4 = lds.q[pslot][src[q]][ty + 4][bx], q5 = lds.q[pslot][src[q]][ty + 5][bx];
                    const double R = sacx::hd_ratio(q0, q1, q2, q3, q4, q5);
                    const int cl = gclass(q);
                    const double nu = kd2[1][cl] * R + kc.kds[1][cl] * sf;
                    sto(a.Gf + (1 * NQF + q) * fs, o, (nu * (q3 - q2)) * kc.ih[1]);
                }
            }
        }
        const int f = r - 3;
        if (colv && f >= zb && f < ze && f <= L.nz - 1) {
            const double sf = fmax(sA, sB);
            const uint32_t o = L.off(x, y, f);
#pragma unroll
            for (int q = 0; q < NQF; ++q) {
                const double R = sacx::hd_ratio(w[q][0], w[q][1], w[q][2], w[q][3], w[q][4], w[q][5]);
                const int cl = gclass(q);
                const double nu = kd2[2][cl] * R + kc.kds[2][cl] * sf;
                sto(a.Gf + (2 * NQF + q) * fs, o, (nu * (w[q][3] - w[q][2])) * kc.ih[2]);
            }
        }
        if (splane) {
            sA = sB;
            sB = lds.s[ty][tx];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- stage launch

template <int TX, int TY, bool HD>
struct StageLds3 {
    double pr[7][TY + 4][TX + 4];   // rho, v_x, v_y, v_z, B_x, B_y, B_z of plane r
    double fx[7][TY + 4][TX + 4];   // x fluxes of rho, m_x, m_y, m_z, e, B_y, B_z
    double fy[7][TY + 4][TX + 4];   // y fluxes of rho, m_x, m_y, m_z, e, B_x, B_z
    // with hyper-diffusion, the face quantities the x- and y-face fluxes of
    // plane r read, staged from the face arrays once per plane: element
    // [.][j][i] is the face stored at (X0 - 2 + i, Y0 - 1 + j).  Rows are
    // GW = TX + 4 doubles, filled as 16-byte pairs from an even x, 128
    // doubles per wave instruction; each tile is padded to whole instructions.
    static constexpr int HX = HD ? TX : 0, HY = HD ? TY : 0, GW = HD ? TX + 4 : 2;
    static constexpr int fill128(int rows) { return (rows * GW + 127) / 128 * 128; }
    struct GzTile {
        alignas(16) double v[4][HY + 2][GW];   // G_z of v_x, B_x, v_y, B_y
        double pad[fill128(4 * (HY + 2)) - 4 * (HY + 2) * GW + 2];
    };
    alignas(16) double gx[NQF][HY + 2][GW];    // G_x, all seven, plane r
    double gx_pad[fill128(NQF * (HY + 2)) - NQF * (HY + 2) * GW + 2];
    alignas(16) double gy[NQF][HY + 1][GW];    // G_y, all seven, plane r
    double gy_pad[fill128(NQF * (HY + 1)) - NQF * (HY + 1) * GW + 2];
    GzTile gz[2];                              // planes r-1 and r (by parity)
    double red[4][TX * TY / 64];
};

typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) void glb_void;

// Fill an LDS tile of face quantities with loads that write LDS directly: no
// registers are held, and the loads overlap whatever the block does until its
// next barrier (which waits for them).  The tile holds NQ quantities x H rows
// x GW columns; row j of quantity q is slot q of direction d (for the G_z
// tile, its q-th of v_x, B_x, v_y, B_y) at y = Y0 - 1 + j, x = X0 - 2 ..
// X0 - 3 + GW, plane k.  Lane l of a wave instruction moves the pair p =
// 64 c + l of the tile (two doubles, 16-byte aligned in both memories: x is
// even and column 0 of every row is on a 256-byte boundary); lanes past the
// tile repeat its last pair into the padding.  Positions past the ghost
// layers read whatever follows in the array (a later row or plane: staged
// planes end at n_z - 1 and three ghost planes follow); no output reads them.
template <int NQ, int H, int GW, bool ZSEL, int NWAVE>
__device__ __forceinline__ void dma_tile(double *dst, const double *Gf, int64_t fs, const Layout3 &L, int d, int X0,
                                         int Y0, int k, int wv, int lane) {
    constexpr int PR = GW / 2, NP = NQ * H * PR, NCH = (NP + 63) / 64;
    static_assert(GW % 2 == 0, "rows are filled in pairs");
#pragma unroll 1
    for (int c = wv; c < NCH; c += NWAVE) {
        const int p = min(c * 64 + lane, NP - 1);
        const int row = p / PR, pr = p - row * PR;
        const int q = row / H, j = row - q * H;
        const int qs = ZSEL ? (q == 0 ? GVX : (q == 1 ? GB1 : (q == 2 ? GVY : GB2))) : q;
        const char *src = (const char *)(Gf + (int64_t)(NQF * d + qs) * fs) + L.off(X0 - 2 + 2 * pr, Y0 - 1 + j, k);
        __builtin_amdgcn_global_load_lds((glb_void *)src, (lds_void *)(dst + c * 128), 16, 0, 0);
    }
}

// the eight face fluxes of one face from its seven G values, the cross-term
// means A4 of the two other directions (first, second in x, y, z order) and
// the face means of rho, v and B; d is the face direction
struct FaceFlux {
    double h[NF3];
};

template <int D>
__device__ __forceinline__ FaceFlux face_flux(const double (&g)[NQF], double a4v1, double a4b1, double a4v2,
                                              double a4b2, double rf, const double (&vf)[3], const double (&bf)[3]) {
    // the two directions other than D, in x, y, z order
    constexpr int O1 = D == 0 ? 1 : 0, O2 = D == 2 ? 1 : 2;
    const double half = 0.5;
    double tau[3], hb[3];
    tau[D] = rf * g[GVX + D];
    hb[D] = 0.0;
    tau[O1] = half * rf * (g[GVX + O1] + a4v1);
    tau[O2] = half * rf * (g[GVX + O2] + a4v2);
    hb[O1] = g[GB1] - a4b1;
    hb[O2] = g[GB2] - a4b2;
    const double work = (vf[D] * tau[D] + vf[O1] * tau[O1]) + vf[O2] * tau[O2];
    const double mag = bf[O1] * hb[O1] + bf[O2] * hb[O2];
    FaceFlux H;
    H.h[FR] = g[GR];
    H.h[FMX] = tau[0];
    H.h[FMY] = tau[1];
    H.h[FMZ] = tau[2];
    H.h[FE] = (g[GE] + work) + mag;
    H.h[FBX] = hb[0];
    H.h[FBY] = hb[1];
    H.h[FBZ] = hb[2];
    return H;
}

template <int STAGE, bool HD, int TX, int TY>
__global__ __launch_bounds__(TX *TY, 1) void k3_stage(Stage3Args a) {
    __shared__ StageLds3<TX, TY, HD> lds;
    constexpr int BX = TX + 4, BY = TY + 4;
    constexpr int NFRAME = BX * BY - TX * TY;
    Dev3 *sc = a.sc;
    if (!sc->active) return;
    const Layout3 L = a.L;
    const Consts3 &kc = a.k;
    const int64_t fs = a.fs;
    const int blk = xcd_block();
    const int X0 = (blk % a.ntx) * TX;
    const int Y0 = ((blk / a.ntx) % a.nty) * TY;
    const int zb = (blk / (a.ntx * a.nty)) * a.tz;
    const int ze = min(zb + a.tz, L.nz);
    const int tid = threadIdx.x, tx = tid % TX, ty = tid / TX;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int x = X0 + tx, y = Y0 + ty;
    const bool colv = x < L.nx && y < L.ny;
    const int xc = min(x, L.nx - 1), yc = min(y, L.ny - 1);   // column clamped into the cells
    const double gm1 = kc.gm1;
    const double half = 0.5, eight = 8.0;
    const double dt = sc->dt, hdt = sc->hdt, dt6 = sc->dt6;
    const bool cross = a.cross != 0;
    const double *Gf = a.Gf;
    auto garr = [&](int d, int q) { return Gf + (int64_t)(NQF * d + q) * fs; };

    // The own column's z fluxes and rho, v, B are streamed two planes ahead
    // of the plane being finished: at iteration r its z fluxes cover planes
    // r-2..r+2 and its rho, v, B planes r..r+2, so the z difference and the
    // z face above plane r are complete when plane r's x and y terms are.
    // (The state of plane r+2 is read again when plane r+2 is finished;
    // keeping it in registers for two planes would spill.)
    double fzw[4][7];   // z fluxes (rho, m_x, m_y, m_z, e, B_x, B_y) of planes r-2..r+1
    double pq[2][7];    // rho, v, B of planes r, r+1
    double hzp[NF3];    // H_z of face (r-1)+1/2
#pragma unroll
    for (int f = 0; f < NF3; ++f) hzp[f] = 0.0;
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        pq[0][k] = pq[1][k] = 0.0;
#pragma unroll
        for (int m = 0; m < 4; ++m) fzw[m][k] = 0.0;
    }
    double cx_t = 0.0, cy_t = 0.0, cz_t = 0.0;
    int bad_t = 0;
    // the streamed column: the thread's own (x, y), clamped into the ghost
    // layers like every box point, so that columns past the last cell hold
    // the ghost values their neighbours difference
    const int cx = min(x, L.nx + G - 1), cy = min(y, L.ny + G - 1);
    const uint32_t sy = (uint32_t)L.pitch * 8u, sz = (uint32_t)(L.plane * 8);   // byte strides

    // The own column's loads that a plane consumes after its tile work (its
    // state two planes ahead, the G of H_z and, at stages 2-4, the combine's
    // stored operand) are issued one plane early, as soon as the previous
    // plane has consumed its own, into registers consumed in place: they
    // land during that plane's x and y terms, and no barrier waits for them
    // before the next plane's tile barrier.  Past the block's last plane
    // they read ghost planes, unused.
    const double *usrc = STAGE == 4 ? a.A : a.U;
    double psn[NF3];                 // state of the own column, plane r+2
    double puo[NF3];                 // the combine's stored operand of the own cell, plane r
    double pgz[NQF];                 // G_z of the own column's face r+1/2
    double pgc[4][4];                // G_x(v_z), G_x(B_z), G_y(v_z), G_y(B_z) around that face
    auto prefetch = [&](int rr) __attribute__((always_inline)) {
        const uint32_t o = L.off(cx, cy, rr + 2);
#pragma unroll
        for (int f = 0; f < NF3; ++f) psn[f] = ldo(a.S + f * fs, o);
        if (STAGE > 1 && HD) {
            // columns past the last cell and planes before the first output
            // plane read a cell of the block and discard it
            const uint32_t ou = L.off(xc, yc, max(rr, zb));
#pragma unroll
            for (int f = 0; f < NF3; ++f) puo[f] = ldo(usrc + f * fs, ou);
        }
        if (HD) {
            const uint32_t c = L.off(xc, yc, max(rr, zb - 1));
#pragma unroll
            for (int q = 0; q < NQF; ++q) pgz[q] = ldo(garr(2, q), c);
            if (cross) {
                // x faces around the z face, then y faces: (-1, r), (0, r),
                // (-1, r+1), (0, r+1) relative to the own column
                const uint32_t c00 = c - 8u, c01 = c, c10 = c - 8u + sz, c11 = c + sz;
                const uint32_t d00 = c - sy, d01 = c, d10 = c - sy + sz, d11 = c + sz;
                pgc[0][0] = ldo(garr(0, GVZ), c00); pgc[0][1] = ldo(garr(0, GVZ), c01);
                pgc[0][2] = ldo(garr(0, GVZ), c10); pgc[0][3] = ldo(garr(0, GVZ), c11);
                pgc[1][0] = ldo(garr(0, GB2), c00); pgc[1][1] = ldo(garr(0, GB2), c01);
                pgc[1][2] = ldo(garr(0, GB2), c10); pgc[1][3] = ldo(garr(0, GB2), c11);
                pgc[2][0] = ldo(garr(1, GVZ), d00); pgc[2][1] = ldo(garr(1, GVZ), d01);
                pgc[2][2] = ldo(garr(1, GVZ), d10); pgc[2][3] = ldo(garr(1, GVZ), d11);
                pgc[3][0] = ldo(garr(1, GB2), d00); pgc[3][1] = ldo(garr(1, GB2), d01);
                pgc[3][2] = ldo(garr(1, GB2), d10); pgc[3][3] = ldo(garr(1, GB2), d11);
            }
        }
    };
    prefetch(zb - 4);

    for (int r = zb - 4; r < ze; ++r) {
        const bool body = r >= zb;   // plane r is an output plane of this block
        if (HD) {
            // ---- the face quantities of plane r that the x- and y-face
            // fluxes read, into LDS while the state of the plane is loaded
            // (G_z also for the plane before the first output plane); the
            // previous plane's closing barrier has freed the tiles
            constexpr int NW = TX * TY / 64, GW = StageLds3<TX, TY, HD>::GW;
            if (body) {
                dma_tile<NQF, TY + 2, GW, false, NW>(&lds.gx[0][0][0], Gf, fs, L, 0, X0, Y0, r, wv, lane);
                dma_tile<NQF, TY + 1, GW, false, NW>(&lds.gy[0][0][0], Gf, fs, L, 1, X0, Y0, r, wv, lane);
            }
            if (r >= zb - 1)
                dma_tile<4, TY + 2, GW, true, NW>(&lds.gz[r & 1].v[0][0][0], Gf, fs, L, 2, X0, Y0, r, wv, lane);
        }
        // ---- P1: plane r over the tile and its apron -> primitives, x and y fluxes in LDS
        double so[NF3];   // own cell's stage input (the combine's pointwise operand)
        if (body) {
            // the own point first, then the apron frame
            for (int p = tid; p < TX * TY + NFRAME; p += TX * TY) {
                int bx, by;
                if (p < TX * TY) {
                    bx = tx + 2;
                    by = ty + 2;
                } else {
                    const int i = p - TX * TY;
                    if (i < 2 * BX) { by = i / BX; bx = i % BX; }
                    else if (i < 4 * BX) { by = TY + 2 + (i - 2 * BX) / BX; bx = (i - 2 * BX) % BX; }
                    else { const int j = i - 4 * BX, c4 = j % 4; by = 2 + j / 4; bx = c4 < 2 ? c4 : TX + c4; }
                }
                const int gx = clampi(X0 - 2 + bx, -G, L.nx + G - 1), gy = clampi(Y0 - 2 + by, -G, L.ny + G - 1);
                const uint32_t o = L.off(gx, gy, r);
                double s[NF3];
#pragma unroll
                for (int f = 0; f < NF3; ++f) s[f] = ldo(a.S + f * fs, o);
                if (p < TX * TY) {
#pragma unroll
                    for (int f = 0; f < NF3; ++f) so[f] = s[f];
                }
                const double rt = s[FR], mx = s[FMX], my = s[FMY], mz = s[FMZ], et = s[FE];
                const double bx_ = s[FBX], by_ = s[FBY], bz_ = s[FBZ];
                const double ir = 1.0 / rt;
                const double ux = mx * ir, uy = my * ir, uz = mz * ir;
                const double kin = half * ((mx * ux + my * uy) + mz * uz);
                const double b2 = (bx_ * bx_ + by_ * by_) + bz_ * bz_;
                const double pk = gm1 * ((et - kin) - half * b2);
                const double pt = pk + half * b2;
                const double bv = (bx_ * ux + by_ * uy) + bz_ * uz;
                const double ef = et + pt;
                lds.pr[0][by][bx] = rt;
                lds.pr[1][by][bx] = ux;
                lds.pr[2][by][bx] = uy;
                lds.pr[3][by][bx] = uz;
                lds.pr[4][by][bx] = bx_;
                lds.pr[5][by][bx] = by_;
                lds.pr[6][by][bx] = bz_;
                lds.fx[0][by][bx] = mx;
                lds.fx[1][by][bx] = (ux * mx - bx_ * bx_) + pt;
                lds.fx[2][by][bx] = ux * my - bx_ * by_;
                lds.fx[3][by][bx] = ux * mz - bx_ * bz_;
                lds.fx[4][by][bx] = ux * ef - bx_ * bv;
                lds.fx[5][by][bx] = ux * by_ - bx_ * uy;
                lds.fx[6][by][bx] = ux * bz_ - bx_ * uz;
                lds.fy[0][by][bx] = my;
                lds.fy[1][by][bx] = uy * mx - by_ * bx_;
                lds.fy[2][by][bx] = (uy * my - by_ * by_) + pt;
                lds.fy[3][by][bx] = uy * mz - by_ * bz_;
                lds.fy[4][by][bx] = uy * ef - by_ * bv;
                lds.fy[5][by][bx] = uy * bx_ - by_ * ux;
                lds.fy[6][by][bx] = uy * bz_ - by_ * uz;
            }
        }
        __syncthreads();

        // ---- own column, plane r+2: state, primitives, z fluxes
        double pn[7], fzn[7];
        {
            const double *sn = psn;
            const double rt = sn[FR], mx = sn[FMX], my = sn[FMY], mz = sn[FMZ], et = sn[FE];
            const double bx_ = sn[FBX], by_ = sn[FBY], bz_ = sn[FBZ];
            const double ir = 1.0 / rt;
            const double ux = mx * ir, uy = my * ir, uz = mz * ir;
            const double kin = half * ((mx * ux + my * uy) + mz * uz);
            const double b2 = (bx_ * bx_ + by_ * by_) + bz_ * bz_;
            const double pk = gm1 * ((et - kin) - half * b2);
            const double pt = pk + half * b2;
            const double bv = (bx_ * ux + by_ * uy) + bz_ * uz;
            const double ef = et + pt;
            pn[0] = rt; pn[1] = ux; pn[2] = uy; pn[3] = uz; pn[4] = bx_; pn[5] = by_; pn[6] = bz_;
            fzn[0] = mz;
            fzn[1] = uz * mx - bz_ * bx_;
            fzn[2] = uz * my - bz_ * by_;
            fzn[3] = (uz * mz - bz_ * bz_) + pt;
            fzn[4] = uz * ef - bz_ * bv;
            fzn[5] = uz * bx_ - bz_ * ux;
            fzn[6] = uz * by_ - bz_ * uy;
        }

        // ---- P2: H_z on the face r+1/2 (planes r, r+1 of the own column)
        FaceFlux hz;
#pragma unroll
        for (int f = 0; f < NF3; ++f) hz.h[f] = 0.0;
        if (HD && r >= zb - 1) {
            double v1 = 0.0, b1 = 0.0, v2 = 0.0, b2 = 0.0;
            if (cross) {
                // means of the four x faces (G of v_z, B_z), then y faces
                v1 = ((pgc[0][0] + pgc[0][1]) + (pgc[0][2] + pgc[0][3])) * 0.25;
                b1 = ((pgc[1][0] + pgc[1][1]) + (pgc[1][2] + pgc[1][3])) * 0.25;
                v2 = ((pgc[2][0] + pgc[2][1]) + (pgc[2][2] + pgc[2][3])) * 0.25;
                b2 = ((pgc[3][0] + pgc[3][1]) + (pgc[3][2] + pgc[3][3])) * 0.25;
            }
            const double rf = half * (pq[0][0] + pq[1][0]);
            double vf[3], bf[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                vf[k] = half * (pq[0][1 + k] + pq[1][1 + k]);
                bf[k] = half * (pq[0][4 + k] + pq[1][4 + k]);
            }
            hz = face_flux<2>(pgz, v1, b1, v2, b2, rf, vf, bf);
        }
        // the combine operand leaves the prefetch registers (with
        // hyper-diffusion its loads are complete: the barrier above waited
        // for the tile fill issued after them), which then take the next
        // plane's loads for the whole of this plane's x and y terms
        double uo[NF3];
        if (STAGE > 1 && HD) {
#pragma unroll
            for (int f = 0; f < NF3; ++f) uo[f] = puo[f];
        }
        prefetch(r + 1);
        __builtin_amdgcn_sched_barrier(0);

        // ---- P3: x and y terms of plane r and its output
        if (body && colv) {
            const int bx = tx + 2, by = ty + 2;
            double K[NF3];
            {
                double ax[7], ay[7];
#pragma unroll
                for (int k = 0; k < 7; ++k) {
                    ax[k] = (eight * (lds.fx[k][by][bx + 1] - lds.fx[k][by][bx - 1]) -
                             (lds.fx[k][by][bx + 2] - lds.fx[k][by][bx - 2])) * kc.i12[0];
                    ay[k] = (eight * (lds.fy[k][by + 1][bx] - lds.fy[k][by - 1][bx]) -
                             (lds.fy[k][by + 2][bx] - lds.fy[k][by - 2][bx])) * kc.i12[1];
                }
                double ab[NF3], ez[NF3];
                const double zero = 0.0;
                ab[FR] = ax[0] + ay[0];
                ab[FMX] = ax[1] + ay[1];
                ab[FMY] = ax[2] + ay[2];
                ab[FMZ] = ax[3] + ay[3];
                ab[FE] = ax[4] + ay[4];
                ab[FBX] = zero + ay[5];
                ab[FBY] = ax[5] + zero;
                ab[FBZ] = ax[6] + ay[6];
#pragma unroll
                for (int f = 0; f < 7; ++f) ez[f] = (eight * (fzw[3][f] - fzw[1][f]) - (fzn[f] - fzw[0][f])) * kc.i12[2];
                ez[FBZ] = zero;
#pragma unroll
                for (int f = 0; f < NF3; ++f) K[f] = -(ab[f] + ez[f]);
            }
            if (HD) {
                // H_x on the faces x-1/2 and x+1/2, then H_y on y-1/2 and
                // y+1/2, one face at a time (a scheduling barrier after each
                // keeps the G loads of later faces from being hoisted into
                // the registers of earlier ones)
                double ah[NF3], bh[NF3];
                const int zc = r & 1, zp = zc ^ 1;   // G_z slots of planes r and r-1
#pragma unroll 1
                for (int side = 0; side < 2; ++side) {
                    const int lb = bx - 1 + side;         // box column of the face's left cell xx = x - 1 + side
                    const int i = tx + side + 1;          // staged column of xx
                    double g[NQF];
#pragma unroll
                    for (int q = 0; q < NQF; ++q) g[q] = lds.gx[q][ty + 1][i];
                    double v1 = 0.0, b1 = 0.0, v2 = 0.0, b2 = 0.0;
                    if (cross) {
                        // y faces around the x face (G of v_x, B_x): (xx, y-1), (xx, y),
                        // (xx+1, y-1), (xx+1, y); then z faces: (xx, r-1), (xx, r),
                        // (xx+1, r-1), (xx+1, r)
                        v1 = ((lds.gy[GVX][ty][i] + lds.gy[GVX][ty + 1][i]) +
                              (lds.gy[GVX][ty][i + 1] + lds.gy[GVX][ty + 1][i + 1])) * 0.25;
                        b1 = ((lds.gy[GB1][ty][i] + lds.gy[GB1][ty + 1][i]) +
                              (lds.gy[GB1][ty][i + 1] + lds.gy[GB1][ty + 1][i + 1])) * 0.25;
                        v2 = ((lds.gz[zp].v[0][ty + 1][i] + lds.gz[zc].v[0][ty + 1][i]) +
                              (lds.gz[zp].v[0][ty + 1][i + 1] + lds.gz[zc].v[0][ty + 1][i + 1])) * 0.25;
                        b2 = ((lds.gz[zp].v[1][ty + 1][i] + lds.gz[zc].v[1][ty + 1][i]) +
                              (lds.gz[zp].v[1][ty + 1][i + 1] + lds.gz[zc].v[1][ty + 1][i + 1])) * 0.25;
                    }
                    const double rf = half * (lds.pr[0][by][lb] + lds.pr[0][by][lb + 1]);
                    double vf[3], bf[3];
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        vf[k] = half * (lds.pr[1 + k][by][lb] + lds.pr[1 + k][by][lb + 1]);
                        bf[k] = half * (lds.pr[4 + k][by][lb] + lds.pr[4 + k][by][lb + 1]);
                    }
                    const FaceFlux h = face_flux<0>(g, v1, b1, v2, b2, rf, vf, bf);
#pragma unroll
                    for (int f = 0; f < NF3; ++f) ah[f] = side == 0 ? h.h[f] : (h.h[f] - ah[f]) * kc.ih[0];
                    __builtin_amdgcn_sched_barrier(0);
                }
#pragma unroll 1
                for (int side = 0; side < 2; ++side) {
                    const int lb = by - 1 + side;         // box row of the face's lower cell yy = y - 1 + side
                    const int j = ty + side;              // staged row of yy
                    double g[NQF];
#pragma unroll
                    for (int q = 0; q < NQF; ++q) g[q] = lds.gy[q][j][tx + 2];
                    double v1 = 0.0, b1 = 0.0, v2 = 0.0, b2 = 0.0;
                    if (cross) {
                        // x faces around the y face (G of v_y, B_y): (x-1, yy), (x, yy),
                        // (x-1, yy+1), (x, yy+1); then z faces: (yy, r-1), (yy, r),
                        // (yy+1, r-1), (yy+1, r)
                        v1 = ((lds.gx[GVY][j][tx + 1] + lds.gx[GVY][j][tx + 2]) +
                              (lds.gx[GVY][j + 1][tx + 1] + lds.gx[GVY][j + 1][tx + 2])) * 0.25;
                        b1 = ((lds.gx[GB1][j][tx + 1] + lds.gx[GB1][j][tx + 2]) +
                              (lds.gx[GB1][j + 1][tx + 1] + lds.gx[GB1][j + 1][tx + 2])) * 0.25;
                        v2 = ((lds.gz[zp].v[2][j][tx + 2] + lds.gz[zc].v[2][j][tx + 2]) +
                              (lds.gz[zp].v[2][j + 1][tx + 2] + lds.gz[zc].v[2][j + 1][tx + 2])) * 0.25;
                        b2 = ((lds.gz[zp].v[3][j][tx + 2] + lds.gz[zc].v[3][j][tx + 2]) +
                              (lds.gz[zp].v[3][j + 1][tx + 2] + lds.gz[zc].v[3][j + 1][tx + 2])) * 0.25;
                    }
                    const double rf = half * (lds.pr[0][lb][bx] + lds.pr[0][lb + 1][bx]);
                    double vf[3], bf[3];
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        vf[k] = half * (lds.pr[1 + k][lb][bx] + lds.pr[1 + k][lb + 1][bx]);
                        bf[k] = half * (lds.pr[4 + k][lb][bx] + lds.pr[4 + k][lb + 1][bx]);
                    }
                    const FaceFlux h = face_flux<1>(g, v1, b1, v2, b2, rf, vf, bf);
#pragma unroll
                    for (int f = 0; f < NF3; ++f) bh[f] = side == 0 ? h.h[f] : (h.h[f] - bh[f]) * kc.ih[1];
                    __builtin_amdgcn_sched_barrier(0);
                }
#pragma unroll
                for (int f = 0; f < NF3; ++f) K[f] = K[f] + ((ah[f] + bh[f]) + (hz.h[f] - hzp[f]) * kc.ih[2]);
            }
            const uint32_t oo = L.off(x, y, r);
            auto uop = [&](int f) __attribute__((always_inline)) { return HD ? uo[f] : ldo(usrc + f * fs, oo); };
            if (STAGE == 1) {
#pragma unroll
                for (int f = 0; f < NF3; ++f) sto(a.out1 + f * fs, oo, so[f] + hdt * K[f]);
            } else if (STAGE == 2) {
#pragma unroll
                for (int f = 0; f < NF3; ++f) {
                    const double u = uop(f), sv = so[f];
                    sto(a.out1 + f * fs, oo, u + hdt * K[f]);
                    sto(a.out2 + f * fs, oo, (u + u) + ((sv - u) + dt * K[f]));
                }
            } else if (STAGE == 3) {
#pragma unroll
                for (int f = 0; f < NF3; ++f) sto(a.out1 + f * fs, oo, uop(f) + dt * K[f]);
            } else {
                double un[NF3];
#pragma unroll
                for (int f = 0; f < NF3; ++f) {
                    const double av = uop(f), sv = so[f];
                    un[f] = (sv + (av - (sv + sv)) * kc.third) + dt6 * K[f];
                    sto(a.out1 + f * fs, oo, un[f]);
                }
                // wave speeds of the new state (the next step's dt and c_max)
                const double ir = 1.0 / un[FR];
                const double ux = un[FMX] * ir, uy = un[FMY] * ir, uz = un[FMZ] * ir;
                const double kin = half * ((un[FMX] * ux + un[FMY] * uy) + un[FMZ] * uz);
                const double b2 = (un[FBX] * un[FBX] + un[FBY] * un[FBY]) + un[FBZ] * un[FBZ];
                const double pk = gm1 * ((un[FE] - kin) - half * b2);
                const double cf = sqrt((kc.gamma * pk + b2) * ir);
                bool fin = isfinite(cf);
#pragma unroll
                for (int f = 0; f < NF3; ++f) fin = fin && isfinite(un[f]);
                if (!(un[FR] > 0.0) || !(pk > 0.0) || !fin) {
                    bad_t = 1;
                } else {
                    cx_t = fmax(cx_t, fabs(ux) + cf);
                    cy_t = fmax(cy_t, fabs(uy) + cf);
                    cz_t = fmax(cz_t, fabs(uz) + cf);
                }
            }
        }
        // ---- shift the windows
#pragma unroll
        for (int f = 0; f < NF3; ++f) hzp[f] = hz.h[f];
#pragma unroll
        for (int k = 0; k < 7; ++k) {
            pq[0][k] = pq[1][k]; pq[1][k] = pn[k];
            fzw[0][k] = fzw[1][k]; fzw[1][k] = fzw[2][k]; fzw[2][k] = fzw[3][k]; fzw[3][k] = fzn[k];
        }
        __syncthreads();
    }

    if (STAGE == 4) {
        for (int off = 32; off > 0; off >>= 1) {
            cx_t = fmax(cx_t, __shfl_xor(cx_t, off));
            cy_t = fmax(cy_t, __shfl_xor(cy_t, off));
            cz_t = fmax(cz_t, __shfl_xor(cz_t, off));
            bad_t |= __shfl_xor(bad_t, off);
        }
        const int wv = tid >> 6;
        if ((tid & 63) == 0) {
            lds.red[0][wv] = cx_t; lds.red[1][wv] = cy_t; lds.red[2][wv] = cz_t; lds.red[3][wv] = (double)bad_t;
        }
        __syncthreads();
        if (tid == 0) {
            double m0 = 0.0, m1 = 0.0, m2 = 0.0, bb = 0.0;
            for (int k = 0; k < TX * TY / 64; ++k) {
                m0 = fmax(m0, lds.red[0][k]); m1 = fmax(m1, lds.red[1][k]);
                m2 = fmax(m2, lds.red[2][k]); bb = fmax(bb, lds.red[3][k]);
            }
            const int ns = sc->cur ^ 1;
            atomicMax(&sc->cacc[ns][0], (unsigned long long)__double_as_longlong(m0));
            atomicMax(&sc->cacc[ns][1], (unsigned long long)__double_as_longlong(m1));
            atomicMax(&sc->cacc[ns][2], (unsigned long long)__double_as_longlong(m2));
            if (bb > 0.0) atomicOr(&sc->nonphys, 1);
        }
    }
}

// ---------------------------------------------------------------- small kernels

// ghost fills: x over the cell rows and planes, then y over the padded x
// width, then z over the padded x and y extents (edges and corners filled);
// periodic images or zero-gradient copies
__global__ void k3_fill_x(double *S, int64_t fs, Layout3 L, int pm, int pp, const Dev3 *sc) {
    if (!sc->active) return;
    const int64_t n = (int64_t)2 * G * L.ny * L.nz;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const int g = (int)(t % (2 * G));
        const int64_t jk = t / (2 * G);
        const int j = (int)(jk % L.ny), k = (int)(jk / L.ny);
        const int i = g < G ? g - G : L.nx + (g - G);
        const int per = g < G ? pm : pp;
        const int s = per ? ((i % L.nx) + L.nx) % L.nx : (i < 0 ? 0 : L.nx - 1);
        const int64_t d = L.at(i, j, k), o = L.at(s, j, k);
#pragma unroll
        for (int f = 0; f < NF3; ++f) S[d + f * fs] = S[o + f * fs];
    }
}

__global__ void k3_fill_y(double *S, int64_t fs, Layout3 L, int pm, int pp, const Dev3 *sc) {
    if (!sc->active) return;
    const int wx = L.nx + 2 * G;
    const int64_t n = (int64_t)2 * G * wx * L.nz;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(t % wx) - G;
        const int64_t gk = t / wx;
        const int g = (int)(gk % (2 * G)), k = (int)(gk / (2 * G));
        const int j = g < G ? g - G : L.ny + (g - G);
        const int per = g < G ? pm : pp;
        const int s = per ? ((j % L.ny) + L.ny) % L.ny : (j < 0 ? 0 : L.ny - 1);
        const int64_t d = L.at(i, j, k), o = L.at(i, s, k);
#pragma unroll
        for (int f = 0; f < NF3; ++f) S[d + f * fs] = S[o + f * fs];
    }
}

__global__ void k3_fill_z(double *S, int64_t fs, Layout3 L, int pm, int pp, const Dev3 *sc) {
    if (!sc->active) return;
    const int wx = L.nx + 2 * G, wy = L.ny + 2 * G;
    const int64_t n = (int64_t)2 * G * wx * wy;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(t % wx) - G;
        const int64_t r = t / wx;
        const int j = (int)(r % wy) - G;
        const int g = (int)(r / wy);
        const int k = g < G ? g - G : L.nz + (g - G);
        const int per = g < G ? pm : pp;
        const int s = per ? ((k % L.nz) + L.nz) % L.nz : (k < 0 ? 0 : L.nz - 1);
        const int64_t d = L.at(i, j, k), o = L.at(i, j, s);
#pragma unroll
        for (int f = 0; f < NF3; ++f) S[d + f * fs] = S[o + f * fs];
    }
}

struct Ptr8 {
    const double *p[NF3];
};
struct MPtr8 {
    double *p[NF3];
};

__global__ void k3_import(double *U, int64_t fs, Layout3 L, Ptr8 src, int64_t pitch, int64_t ppitch) {
    const int64_t n = (int64_t)L.nx * L.ny * L.nz;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(t % L.nx);
        const int64_t jk = t / L.nx;
        const int j = (int)(jk % L.ny), k = (int)(jk / L.ny);
        const int64_t d = L.at(i, j, k), s = i + j * pitch + k * ppitch;
#pragma unroll
        for (int f = 0; f < NF3; ++f) U[d + f * fs] = src.p[f][s];
    }
}

__global__ void k3_export(const double *U, int64_t fs, Layout3 L, MPtr8 dst, uint32_t mask, int64_t pitch,
                          int64_t ppitch) {
    const int64_t n = (int64_t)L.nx * L.ny * L.nz;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(t % L.nx);
        const int64_t jk = t / L.nx;
        const int j = (int)(jk % L.ny), k = (int)(jk / L.ny);
        const int64_t s = L.at(i, j, k), d = i + j * pitch + k * ppitch;
#pragma unroll
        for (int f = 0; f < NF3; ++f)
            if (mask & (1u << f)) dst.p[f][d] = U[s + f * fs];
    }
}

// wave speeds of a state into accumulator slot `slot` (non-physical flag set)
__global__ void k3_wavespeed(const double *U, int64_t fs, Layout3 L, double gamma, Dev3 *sc, int slot) {
    __shared__ double red[4][4];
    const double gm1 = gamma - 1.0, half = 0.5;
    double c0 = 0.0, c1 = 0.0, c2 = 0.0;
    int bad = 0;
    const int64_t n = (int64_t)L.nx * L.ny * L.nz;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(t % L.nx);
        const int64_t jk = t / L.nx;
        const int j = (int)(jk % L.ny), k = (int)(jk / L.ny);
        const int64_t o = L.at(i, j, k);
        double u[NF3];
#pragma unroll
        for (int f = 0; f < NF3; ++f) u[f] = U[o + f * fs];
        const double ir = 1.0 / u[FR];
        const double ux = u[FMX] * ir, uy = u[FMY] * ir, uz = u[FMZ] * ir;
        const double kin = half * ((u[FMX] * ux + u[FMY] * uy) + u[FMZ] * uz);
        const double b2 = (u[FBX] * u[FBX] + u[FBY] * u[FBY]) + u[FBZ] * u[FBZ];
        const double pk = gm1 * ((u[FE] - kin) - half * b2);
        const double cf = sqrt((gamma * pk + b2) * ir);
        bool fin = isfinite(cf);
#pragma unroll
        for (int f = 0; f < NF3; ++f) fin = fin && isfinite(u[f]);
        if (!(u[FR] > 0.0) || !(pk > 0.0) || !fin) {
            bad = 1;
        } else {
            c0 = fmax(c0, fabs(ux) + cf);
            c1 = fmax(c1, fabs(uy) + cf);
            c2 = fmax(c2, fabs(uz) + cf);
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        c0 = fmax(c0, __shfl_xor(c0, off));
        c1 = fmax(c1, __shfl_xor(c1, off));
        c2 = fmax(c2, __shfl_xor(c2, off));
        bad |= __shfl_xor(bad, off);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { red[0][w] = c0; red[1][w] = c1; red[2][w] = c2; red[3][w] = bad; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double m0 = 0.0, m1 = 0.0, m2 = 0.0, bb = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
            m0 = fmax(m0, red[0][k]); m1 = fmax(m1, red[1][k]); m2 = fmax(m2, red[2][k]); bb = fmax(bb, red[3][k]);
        }
        atomicMax(&sc->cacc[slot][0], (unsigned long long)__double_as_longlong(m0));
        atomicMax(&sc->cacc[slot][1], (unsigned long long)__double_as_longlong(m1));
        atomicMax(&sc->cacc[slot][2], (unsigned long long)__double_as_longlong(m2));
        if (bb > 0.0) atomicOr(&sc->nonphys, 1);
    }
}

__global__ void k3_reset(Dev3 *sc, double t0) {
    memset(sc, 0, sizeof(Dev3));
    sc->t = t0;
    sc->active = 1;
}

// dt of the step about to start from the reduced wave speeds (minimum of
// h_d / c_d over the directions with more than one cell, taken x, y, z, then
// the end-time clamp) and the per-step constants
__global__ void k3_step_begin(Dev3 *sc, double t_end, Consts3 k) {
    sc->t_end = t_end;
    if (sc->nonphys) { sc->active = 0; return; }
    const double t = sc->t;
    if (t_end > 0.0 && t_end - t <= 1e-12 * t_end) { sc->active = 0; return; }
    double c[3];
    for (int d = 0; d < 3; ++d) c[d] = __longlong_as_double((long long)sc->cacc[sc->cur][d]);
    double m = -1.0, cm = -1.0;
    for (int d = 0; d < 3; ++d) {
        if (!k.act[d]) continue;
        const double q = k.h[d] / c[d];
        m = m < 0.0 ? q : (m < q ? m : q);
        cm = cm < 0.0 ? c[d] : (cm > c[d] ? cm : c[d]);
    }
    double dt = k.cfl * m;
    if (t_end > 0.0) dt = (dt < t_end - t) ? dt : t_end - t;
    sc->dt = dt;
    sc->cmax = cm;
    for (int d = 0; d < 3; ++d) sc->last_c[d] = c[d];
    sc->last_cmax = cm;
    sc->hdt = 0.5 * dt;
    sc->dt6 = dt / 6.0;
    for (int d = 0; d < 3; ++d)
        for (int q = 0; q < 4; ++q) sc->kd2[d][q] = k.c2[q] * k.h[d] * cm;
    for (int d = 0; d < 3; ++d) sc->cacc[sc->cur ^ 1][d] = 0ull;
    sc->active = 1;
}

__global__ void k3_step_end(Dev3 *sc) {
    if (!sc->active) return;
    sc->t = sc->t + sc->dt;
    sc->steps = sc->steps + 1;
    sc->cur ^= 1;
}

// conservation sums: each block sums a contiguous run of cells (storage
// order) per field; the partials are added in block order
__global__ void k3_sums_partial(const double *U, int64_t fs, Layout3 L, double *part, int npart) {
    __shared__ double red[NF3][4];
    const int64_t n = (int64_t)L.nx * L.ny * L.nz;
    const int64_t per = (n + npart - 1) / npart;
    const int64_t b0 = blockIdx.x * per, b1 = min(n, b0 + per);
    double acc[NF3];
#pragma unroll
    for (int f = 0; f < NF3; ++f) acc[f] = 0.0;
    for (int64_t t = b0 + threadIdx.x; t < b1; t += blockDim.x) {
        const int i = (int)(t % L.nx);
        const int64_t jk = t / L.nx;
        const int j = (int)(jk % L.ny), k = (int)(jk / L.ny);
        const int64_t o = L.at(i, j, k);
#pragma unroll
        for (int f = 0; f < NF3; ++f) acc[f] += U[o + f * fs];
    }
#pragma unroll
    for (int f = 0; f < NF3; ++f)
        for (int off = 32; off > 0; off >>= 1) acc[f] += __shfl_down(acc[f], off);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int f = 0; f < NF3; ++f) red[f][w] = acc[f];
    __syncthreads();
    if (threadIdx.x < NF3) {
        double s = 0.0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[threadIdx.x][k];
        part[blockIdx.x * NF3 + threadIdx.x] = s;
    }
}

__global__ void k3_sums_final(const double *part, int npart, double *out, double cell) {
    const int f = threadIdx.x;
    if (f >= NF3) return;
    double s = 0.0;
    for (int b = 0; b < npart; ++b) s += part[b * NF3 + f];
    out[f] = s * cell;
}

struct Plan3 {
    Layout3 L;
    size_t field_bytes;
    size_t off_sc, off_part, off_sums, off_state, off_g, total;
};

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int check3(const sacx3_grid *g, const sacx3_params *p) {
    using sacx::set_error;
    if (!g || !p) return set_error(SACX_EINVAL, "grid and params must not be NULL");
    if (g->nx < 1 || g->ny < 1 || g->nz < 1) return set_error(SACX_EINVAL, "nx, ny, nz must be >= 1");
    if ((int64_t)g->nx * g->ny * g->nz < 2) return set_error(SACX_EINVAL, "a grid needs more than one cell");
    if (g->nx > (1 << 20) || g->ny > (1 << 20) || g->nz > (1 << 20))
        return set_error(SACX_EINVAL, "a side exceeds 2^20 cells");
    if (!(g->x1 > g->x0) || !(g->y1 > g->y0) || !(g->z1 > g->z0) || !std::isfinite(g->x0) ||
        !std::isfinite(g->x1) || !std::isfinite(g->y0) || !std::isfinite(g->y1) || !std::isfinite(g->z0) ||
        !std::isfinite(g->z1))
        return set_error(SACX_EINVAL, "the extent must be finite with x1 > x0, y1 > y0, z1 > z0");
    if (!(p->gamma > 1.0) || !std::isfinite(p->gamma)) return set_error(SACX_EINVAL, "gamma must be > 1");
    if (!(p->cfl > 0.0) || !std::isfinite(p->cfl)) return set_error(SACX_EINVAL, "cfl must be > 0");
    for (int k = 0; k < 4; ++k)
        if (!(p->c2[k] >= 0.0) || !(p->cshk[k] >= 0.0) || !std::isfinite(p->c2[k]) || !std::isfinite(p->cshk[k]))
            return set_error(SACX_EINVAL, "hyper-diffusion constants must be finite and >= 0");
    // the kernels address a field array with 32-bit byte offsets
    const int64_t pitch = (int64_t)round_up((size_t)kAlign / sizeof(double) + g->nx + G, kAlign / sizeof(double));
    const double bytes = 8.0 * (double)pitch * (double)(g->ny + 2 * G) * (double)(g->nz + 2 * G);
    if (bytes > 4294967040.0)
        return set_error(SACX_EUNSUP, "one field array would take %.3g bytes; at most 4 GiB (about 800^3 cells)", bytes);
    return SACX_OK;
}

Plan3 plan3(const sacx3_grid *g, const sacx3_params *p) {
    Plan3 P;
    Layout3 &L = P.L;
    L.nx = g->nx; L.ny = g->ny; L.nz = g->nz;
    L.xoff = kAlign / (int)sizeof(double);
    L.pitch = (int)round_up((size_t)L.xoff + L.nx + G, kAlign / sizeof(double));
    L.plane = (int64_t)L.pitch * (L.ny + 2 * G);
    L.field_elems = (int64_t)round_up((size_t)(L.plane * (L.nz + 2 * G)), kAlign / sizeof(double));
    P.field_bytes = (size_t)L.field_elems * sizeof(double);
    size_t o = 0;
    P.off_sc = o; o = round_up(o + sizeof(Dev3), kAlign);
    P.off_part = o; o = round_up(o + sizeof(double) * NF3 * kPartials, kAlign);
    P.off_sums = o; o = round_up(o + sizeof(double) * NF3, kAlign);
    P.off_state = o; o += 4 * NF3 * P.field_bytes;
    P.off_g = o; o += p->hd_on ? 3 * NQF * P.field_bytes : 0;
    P.total = o;
    return P;
}

struct DevGuard {
    int prev = -1;
    bool ok = false;
    explicit DevGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) return;
        ok = prev == dev || hipSetDevice(dev) == hipSuccess;
    }
    ~DevGuard() {
        if (ok && prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace sacx3i

using namespace sacx3i;

struct sacx3_ctx {
    sacx3_grid grid;
    sacx3_params params;
    int device;
    hipStream_t stream;
    Plan3 P;
    char *ws;
    Dev3 *sc;
    double *part, *sums;
    double *U, *B1, *B2, *A, *Gf;
    int64_t fs;
    Consts3 kc;
    int bc[6];
    int tz;
    bool initialized;
};

namespace sacx3i {

#define HIPCHK3(expr)                                                                                      \
    do {                                                                                                   \
        hipError_t e_ = (expr);                                                                            \
        if (e_ != hipSuccess)                                                                              \
            return sacx::set_error(SACX_EDEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                                   __LINE__);                                                              \
    } while (0)

int blocks_for(int64_t n, int nt) {
    int64_t b = (n + nt - 1) / nt;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, 65536));
}

int fill3(sacx3_ctx *c, double *S) {
    const Layout3 &L = c->P.L;
    const int nt = 256;
    hipLaunchKernelGGL(k3_fill_x, dim3(blocks_for((int64_t)2 * G * L.ny * L.nz, nt)), dim3(nt), 0, c->stream, S,
                       c->fs, L, c->bc[0] == SACX_PERIODIC, c->bc[1] == SACX_PERIODIC, c->sc);
    hipLaunchKernelGGL(k3_fill_y, dim3(blocks_for((int64_t)2 * G * (L.nx + 2 * G) * L.nz, nt)), dim3(nt), 0,
                       c->stream, S, c->fs, L, c->bc[2] == SACX_PERIODIC, c->bc[3] == SACX_PERIODIC, c->sc);
    hipLaunchKernelGGL(k3_fill_z, dim3(blocks_for((int64_t)2 * G * (L.nx + 2 * G) * (L.ny + 2 * G), nt)), dim3(nt),
                       0, c->stream, S, c->fs, L, c->bc[4] == SACX_PERIODIC, c->bc[5] == SACX_PERIODIC, c->sc);
    HIPCHK3(hipGetLastError());
    return SACX_OK;
}

template <int STAGE>
int launch_stage3(sacx3_ctx *c, const Stage3Args &a, int nblocks) {
    if (c->params.hd_on)
        hipLaunchKernelGGL((k3_stage<STAGE, true, TXF, TYF>), dim3(nblocks), dim3(NT), 0, c->stream, a);
    else
        hipLaunchKernelGGL((k3_stage<STAGE, false, TXF, TYF>), dim3(nblocks), dim3(NT), 0, c->stream, a);
    HIPCHK3(hipGetLastError());
    return SACX_OK;
}

int stage3(sacx3_ctx *c, int s, double *S, double *U, double *A, double *o1, double *o2) {
    int rc = fill3(c, S);
    if (rc) return rc;
    const Layout3 &L = c->P.L;
    if (c->params.hd_on) {
        Face3Args f;
        f.S = S; f.Gf = c->Gf; f.fs = c->fs; f.L = L; f.k = c->kc; f.sc = c->sc; f.tz = c->tz;
        f.ntx = (L.nx + 2 + TXF - 1) / TXF;
        f.nty = (L.ny + 2 + TYF - 1) / TYF;
        const int nzs = (L.nz + 2 + c->tz - 1) / c->tz;
        hipLaunchKernelGGL((k3_faces<TXF, TYF>), dim3(f.ntx * f.nty * nzs), dim3(NT), 0, c->stream, f);
        HIPCHK3(hipGetLastError());
    }
    Stage3Args a;
    a.S = S; a.U = U; a.A = A; a.out1 = o1; a.out2 = o2; a.Gf = c->Gf; a.fs = c->fs; a.L = L; a.k = c->kc;
    a.sc = c->sc; a.tz = c->tz; a.cross = c->params.hd_cross_on;
    a.ntx = (L.nx + TXF - 1) / TXF;
    a.nty = (L.ny + TYF - 1) / TYF;
    const int nb = a.ntx * a.nty * ((L.nz + c->tz - 1) / c->tz);
    switch (s) {
        case 1: return launch_stage3<1>(c, a, nb);
        case 2: return launch_stage3<2>(c, a, nb);
        case 3: return launch_stage3<3>(c, a, nb);
        default: return launch_stage3<4>(c, a, nb);
    }
}

}  // namespace sacx3i

#define fail sacx::set_error

extern "C" {

int sacx3_workspace_size(const sacx3_grid *grid, const sacx3_params *params, size_t *bytes) {
    if (!bytes) return fail(SACX_EINVAL, "bytes must not be NULL");
    int rc = check3(grid, params);
    if (rc) return rc;
    *bytes = plan3(grid, params).total;
    return SACX_OK;
}

int sacx3_create(const sacx3_grid *grid, const sacx3_params *params, void *d_ws, size_t ws_bytes, void *hip_stream,
                 sacx3_ctx **out) {
    if (!out) return fail(SACX_EINVAL, "out must not be NULL");
    *out = nullptr;
    int rc = check3(grid, params);
    if (rc) return rc;
    if (!d_ws) return fail(SACX_EINVAL, "d_ws must not be NULL");
    if ((uintptr_t)d_ws % kAlign) return fail(SACX_EINVAL, "d_ws must be 256-byte aligned");
    const Plan3 P = plan3(grid, params);
    if (ws_bytes < P.total) return fail(SACX_ENOSPC, "workspace of %zu bytes, %zu needed", ws_bytes, P.total);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(SACX_EDEVICE, "no current device");
    sacx3_ctx *c = new (std::nothrow) sacx3_ctx();
    if (!c) return fail(SACX_EINVAL, "out of host memory");
    c->grid = *grid;
    c->params = *params;
    c->device = dev;
    c->stream = (hipStream_t)hip_stream;
    c->P = P;
    c->ws = (char *)d_ws;
    c->sc = (Dev3 *)(c->ws + P.off_sc);
    c->part = (double *)(c->ws + P.off_part);
    c->sums = (double *)(c->ws + P.off_sums);
    c->fs = P.L.field_elems;
    const size_t blk = (size_t)NF3 * P.field_bytes;
    c->U = (double *)(c->ws + P.off_state);
    c->B1 = (double *)(c->ws + P.off_state + blk);
    c->B2 = (double *)(c->ws + P.off_state + 2 * blk);
    c->A = (double *)(c->ws + P.off_state + 3 * blk);
    c->Gf = params->hd_on ? (double *)(c->ws + P.off_g) : nullptr;
    for (int s = 0; s < 6; ++s) c->bc[s] = SACX_PERIODIC;
    c->tz = 64;
    // constants of the scheme (FP64, once)
    Consts3 &k = c->kc;
    memset(&k, 0, sizeof(k));
    const double ext[3][2] = {{grid->x0, grid->x1}, {grid->y0, grid->y1}, {grid->z0, grid->z1}};
    const int n[3] = {grid->nx, grid->ny, grid->nz};
    k.gamma = params->gamma;
    k.gm1 = params->gamma - 1.0;
    k.igm1 = 1.0 / k.gm1;
    k.third = 1.0 / 3.0;
    k.cfl = params->cfl;
    for (int q = 0; q < 4; ++q) k.c2[q] = params->c2[q];
    for (int d = 0; d < 3; ++d) {
        const double h = (ext[d][1] - ext[d][0]) / n[d];
        k.h[d] = h;
        k.ih[d] = 1.0 / h;
        k.i12[d] = 1.0 / (12.0 * h);
        k.i2[d] = 1.0 / (2.0 * h);
        for (int q = 0; q < 4; ++q) k.kds[d][q] = params->cshk[q] * h * h;
        k.act[d] = n[d] > 1;
    }
    c->initialized = false;
    *out = c;
    return SACX_OK;
}

int sacx3_destroy(sacx3_ctx *ctx) {
    if (!ctx) return SACX_OK;
    int rc = SACX_OK;
    {
        DevGuard dg(ctx->device);
        if (dg.ok && hipStreamSynchronize(ctx->stream) != hipSuccess)
            rc = fail(SACX_EDEVICE, "waiting for the context's stream failed");
    }
    delete ctx;
    return rc;
}

int sacx3_set_boundaries(sacx3_ctx *ctx, const int32_t bc[6]) {
    if (!ctx || !bc) return fail(SACX_EINVAL, "ctx and bc must not be NULL");
    const int n[3] = {ctx->grid.nx, ctx->grid.ny, ctx->grid.nz};
    for (int s = 0; s < 6; ++s)
        if (bc[s] != SACX_PERIODIC && bc[s] != SACX_OPEN) return fail(SACX_EINVAL, "side %d: unknown boundary %d", s, bc[s]);
    for (int d = 0; d < 3; ++d) {
        if ((bc[2 * d] == SACX_PERIODIC) != (bc[2 * d + 1] == SACX_PERIODIC))
            return fail(SACX_EINVAL, "direction %d: periodic sides must come in pairs", d);
        if (n[d] == 1 && bc[2 * d] != SACX_PERIODIC)
            return fail(SACX_EINVAL, "direction %d has one cell and must be periodic", d);
    }
    for (int s = 0; s < 6; ++s) ctx->bc[s] = bc[s];
    return SACX_OK;
}

int sacx3_set_launch(sacx3_ctx *ctx, int32_t planes) {
    if (!ctx) return fail(SACX_EINVAL, "ctx must not be NULL");
    if (planes < 0 || planes > 4096) return fail(SACX_EINVAL, "planes must be in [0, 4096]");
    ctx->tz = planes == 0 ? 64 : planes;
    return SACX_OK;
}

int sacx3_init_state(sacx3_ctx *ctx, const double *const *d_fields, int64_t pitch, int64_t plane_pitch, double t0) {
    if (!ctx || !d_fields) return fail(SACX_EINVAL, "ctx and d_fields must not be NULL");
    for (int f = 0; f < NF3; ++f)
        if (!d_fields[f]) return fail(SACX_EINVAL, "field %d pointer is NULL", f);
    if (pitch < ctx->grid.nx || plane_pitch < pitch * ctx->grid.ny)
        return fail(SACX_EINVAL, "pitch must be >= nx and plane_pitch >= ny * pitch");
    if (!std::isfinite(t0)) return fail(SACX_EINVAL, "t0 must be finite");
    DevGuard dg(ctx->device);
    if (!dg.ok) return fail(SACX_EDEVICE, "cannot select the context device");
    const Layout3 &L = ctx->P.L;
    Ptr8 src;
    for (int f = 0; f < NF3; ++f) src.p[f] = d_fields[f];
    const int64_t ncell = (int64_t)L.nx * L.ny * L.nz;
    hipLaunchKernelGGL(k3_reset, dim3(1), dim3(1), 0, ctx->stream, ctx->sc, t0);
    hipLaunchKernelGGL(k3_import, dim3(blocks_for(ncell, 256)), dim3(256), 0, ctx->stream, ctx->U, ctx->fs, L, src,
                       pitch, plane_pitch);
    hipLaunchKernelGGL(k3_wavespeed, dim3(std::min(blocks_for(ncell, 256), 2048)), dim3(256), 0, ctx->stream,
                       ctx->U, ctx->fs, L, ctx->kc.gamma, ctx->sc, 0);
    HIPCHK3(hipGetLastError());
    ctx->initialized = true;
    return SACX_OK;
}

int sacx3_advance(sacx3_ctx *ctx, int32_t nsteps, double t_end, int32_t *steps_done, double *t_now) {
    if (!ctx) return fail(SACX_EINVAL, "ctx must not be NULL");
    if (nsteps < 0) return fail(SACX_EINVAL, "nsteps must be >= 0");
    if (!std::isfinite(t_end)) return fail(SACX_EINVAL, "t_end must be finite");
    if (!ctx->initialized) return fail(SACX_ESTATE, "sacx3_init_state has not been called");
    DevGuard dg(ctx->device);
    if (!dg.ok) return fail(SACX_EDEVICE, "cannot select the context device");
    const bool sync = steps_done || t_now;
    long long steps0 = 0;
    if (sync) {
        HIPCHK3(hipMemcpyAsync(&steps0, &ctx->sc->steps, sizeof(steps0), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK3(hipStreamSynchronize(ctx->stream));
    }
    const int chunk = sync ? 64 : (nsteps > 0 ? nsteps : 1);
    for (int n0 = 0; n0 < nsteps; n0 += chunk) {
        const int n1 = std::min(nsteps, n0 + chunk);
        for (int n = n0; n < n1; ++n) {
            hipLaunchKernelGGL(k3_step_begin, dim3(1), dim3(1), 0, ctx->stream, ctx->sc, t_end, ctx->kc);
            int rc;
            if ((rc = stage3(ctx, 1, ctx->U, nullptr, nullptr, ctx->B1, nullptr))) return rc;
            if ((rc = stage3(ctx, 2, ctx->B1, ctx->U, nullptr, ctx->B2, ctx->A))) return rc;
            if ((rc = stage3(ctx, 3, ctx->B2, ctx->U, nullptr, ctx->B1, nullptr))) return rc;
            if ((rc = stage3(ctx, 4, ctx->B1, nullptr, ctx->A, ctx->U, nullptr))) return rc;
            hipLaunchKernelGGL(k3_step_end, dim3(1), dim3(1), 0, ctx->stream, ctx->sc);
            HIPCHK3(hipGetLastError());
        }
        if (sync && n1 < nsteps) {
            int act = 1;
            HIPCHK3(hipMemcpyAsync(&act, &ctx->sc->active, sizeof(act), hipMemcpyDeviceToHost, ctx->stream));
            HIPCHK3(hipStreamSynchronize(ctx->stream));
            if (!act) break;
        }
    }
    if (sync) {
        Dev3 h;
        HIPCHK3(hipMemcpyAsync(&h, ctx->sc, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK3(hipStreamSynchronize(ctx->stream));
        if (steps_done) *steps_done = (int32_t)(h.steps - steps0);
        if (t_now) *t_now = h.t;
        if (h.nonphys) return fail(SACX_ENONPHYS, "non-physical state after %lld steps", h.steps);
    }
    return SACX_OK;
}

int sacx3_read_fields(sacx3_ctx *ctx, double *const *d_out, int64_t pitch, int64_t plane_pitch, uint32_t field_mask) {
    if (!ctx || !d_out) return fail(SACX_EINVAL, "ctx and d_out must not be NULL");
    if (!ctx->initialized) return fail(SACX_ESTATE, "sacx3_init_state has not been called");
    if (pitch < ctx->grid.nx || plane_pitch < pitch * ctx->grid.ny)
        return fail(SACX_EINVAL, "pitch must be >= nx and plane_pitch >= ny * pitch");
    if (field_mask & ~0xFFu) return fail(SACX_EINVAL, "field_mask has bits beyond the 8 fields");
    MPtr8 dst;
    for (int f = 0; f < NF3; ++f) {
        dst.p[f] = (field_mask & (1u << f)) ? d_out[f] : nullptr;
        if ((field_mask & (1u << f)) && !d_out[f]) return fail(SACX_EINVAL, "output %d pointer is NULL", f);
    }
    DevGuard dg(ctx->device);
    if (!dg.ok) return fail(SACX_EDEVICE, "cannot select the context device");
    const Layout3 &L = ctx->P.L;
    hipLaunchKernelGGL(k3_export, dim3(blocks_for((int64_t)L.nx * L.ny * L.nz, 256)), dim3(256), 0, ctx->stream,
                       ctx->U, ctx->fs, L, dst, field_mask, pitch, plane_pitch);
    HIPCHK3(hipGetLastError());
    return SACX_OK;
}

int sacx3_diagnostics(sacx3_ctx *ctx, sacx3_diag *out) {
    if (!ctx || !out) return fail(SACX_EINVAL, "ctx and out must not be NULL");
    if (!ctx->initialized) return fail(SACX_ESTATE, "sacx3_init_state has not been called");
    DevGuard dg(ctx->device);
    if (!dg.ok) return fail(SACX_EDEVICE, "cannot select the context device");
    const Layout3 &L = ctx->P.L;
    const int64_t n = (int64_t)L.nx * L.ny * L.nz;
    const int npart = (int)std::max<int64_t>(1, std::min<int64_t>(kPartials, (n + 255) / 256));
    hipLaunchKernelGGL(k3_sums_partial, dim3(npart), dim3(256), 0, ctx->stream, ctx->U, ctx->fs, L, ctx->part, npart);
    const double cell = (ctx->kc.h[0] * ctx->kc.h[1]) * ctx->kc.h[2];
    hipLaunchKernelGGL(k3_sums_final, dim3(1), dim3(64), 0, ctx->stream, ctx->part, npart, ctx->sums, cell);
    HIPCHK3(hipGetLastError());
    Dev3 h;
    double sums[NF3];
    HIPCHK3(hipMemcpyAsync(&h, ctx->sc, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK3(hipMemcpyAsync(sums, ctx->sums, sizeof(sums), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK3(hipStreamSynchronize(ctx->stream));
    out->t = h.t;
    out->dt = h.dt;
    double c[3], cm = -1.0;
    for (int d = 0; d < 3; ++d) {
        const unsigned long long bits = h.cacc[h.cur][d];
        memcpy(&c[d], &bits, sizeof(double));
        out->c[d] = c[d];
        if (ctx->kc.act[d]) cm = cm < 0.0 ? c[d] : std::max(cm, c[d]);
    }
    out->c_max = cm;
    for (int f = 0; f < NF3; ++f) out->sums[f] = sums[f];
    out->steps = h.steps;
    out->nonphys = h.nonphys;
    return SACX_OK;
}

}  // extern "C"
