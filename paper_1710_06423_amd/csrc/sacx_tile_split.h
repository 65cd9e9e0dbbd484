// sacx_tile_split.h -- the fused RK stage with the work of each column split
// between two waves: one for the x-direction terms, one for the y-direction
// terms (hyper-diffusion on, plain coefficient, with or without a background).
//
// Why: the one-thread-per-column tile holds about a hundred FP64 values of
// sliding windows per thread, more than the 256 registers that allow two
// waves per SIMD, so it runs one wave per SIMD and moves part of its state
// through the accumulation registers.  Splitting the column's work by
// direction halves the state each thread carries (x role: D_x F_x, x-face G
// and face means; y role: the y-flux and y-face windows, the ideal L, the
// y-face fluxes) so that each role fits in 256 registers and two waves share
// every SIMD; what one role needs from the other goes through LDS.
//
// With the learned coefficient (SUR), a face whose check tile was kept and
// whose supplied ratio is >= 0 takes that value in place of the plain ratio,
// exactly as in the one-thread tile.
//
// Block: 2*NC threads over NC columns (column t = tid mod NC, the first NC
// threads are the x role).  Per iteration r (row r is the newest state row):
//   phase 1  X: primitives and x fluxes of row r, published with the state
//               row (ring of 5 rows) and D_x F_x of row r-2
//            Y: L(S) and the stage combine of row r-4 (stage 4: its wave
//               speeds); pointwise operands of row r-3 (HBM)
//   phase 2  X: compression s of row r-1, coefficient ratios of its x faces
//            Y: y-face G of face (r-3)+1/2
//   phase 3  X: D_x F_x of row r, x-face G of row r-1, H_x at row r-3
//            Y: y fluxes of row r, D_y F_y and ideal L of row r-2, H_y at
//               face (r-3)+1/2
// with a barrier after each phase; the y role's last output row follows the
// loop.  Each role keeps its state in registers across iterations; LDS holds
// only what the other role or a neighbouring column needs.  Every value is
// the same IEEE operation on the same operands as in the one-thread tile, so
// both tiles give the same bits.
#pragma once

#include "sacx_tile.h"

namespace sacx {

enum { SQR = 0, SQE = 1, SQVX = 2, SQVY = 3, SQB = 4, SQRHO = 5, SQBYT = 6, SQPT = 7, SNQ = 8 };

template <typename real, int NC, bool BG = false>
struct SplitLds {
    real fx[5][NC];          // x fluxes of row r
    real q[2][SNQ][NC];      // primitives of rows r, r-1 (by row parity)
    real ps[5][NF][NC];      // state rows r-4..r (ring mod 5)
    real s[3][NC];           // compression s (ring over rows mod 3)
    real dx[BG ? 7 : 5][NC]; // D_x F_x of row r-2 (with a background also D_x v_x, D_x v_y)
    real gx[2][3][NC];       // x-face G(v_y), G(B~_y), ring over rows (mod 3)
    real gy[2][2][NC];       // y-face G(v_x), G(B~_x), ring over faces (mod 2)
    real hx[5][NC];          // x-face fluxes H_x of row r-3
    double red[3][2 * NC / 64];
};

// what both roles of a tile share: scalars of the step, constants of the
// scheme and the tile's geometry
template <typename real, int NC>
struct SplitCommon {
    real dt, hdt, dt6, kx2[4], ky2[4];
    real gamma, gm1, igm1, i12dx, i12dy, idx, idy, i2dx, i2dy, third, gx, gy;
    int t, c, y0, rbeg, rend, tm1, tm2, tp1, tp2, tp3;
    bool outcol, cross, grav;
    int64_t colofs;

    __device__ __forceinline__ SplitCommon(const StageArgs<real> &a, int tx_, int ty_, int t_) {
        constexpr int TX = NC - 2 * G;
        const DevScalars *sc = a.sc;
        dt = (real)sc->dt;
        hdt = (real)sc->hdt;
        dt6 = (real)sc->dt6;
#pragma unroll
        for (int k = 0; k < 4; ++k) { kx2[k] = (real)sc->kx2[k]; ky2[k] = (real)sc->ky2[k]; }
        const SchemeConsts &kc = a.k;
        gamma = (real)kc.gamma; gm1 = (real)kc.gm1; igm1 = (real)kc.igm1;
        i12dx = (real)kc.i12dx; i12dy = (real)kc.i12dy; idx = (real)kc.idx; idy = (real)kc.idy;
        i2dx = (real)kc.i2dx; i2dy = (real)kc.i2dy; third = (real)kc.third;
        gx = (real)kc.gx; gy = (real)kc.gy; grav = kc.grav != 0;
        const Layout &L = a.L;
        t = t_;
        c = tx_ * TX - G + t;
        y0 = ty_ * a.ty;
        const int y1 = min(y0 + a.ty, L.ny);
        rbeg = y0 - G;
        rend = y1 - 1 + G;
        outcol = t >= G && t < NC - G && c < L.nx;
        cross = a.hd_cross_on != 0;
        tm1 = t >= 1 ? t - 1 : 0;
        tm2 = t >= 2 ? t - 2 : 0;
        tp1 = t + 1 < NC ? t + 1 : NC - 1;
        tp2 = t + 2 < NC ? t + 2 : NC - 1;
        tp3 = t + 3 < NC ? t + 3 : NC - 1;
        const bool colv = c < L.nx + G;
        colofs = (int64_t)L.xoff + (colv ? c : L.nx + G - 1);
    }
};

// ring slots (rows >= -6)
__device__ __forceinline__ int ring5(int r) { return (r + 5 * 4096) % 5; }
__device__ __forceinline__ int ring3(int r) { return (r + 3 * 4096) % 3; }

// Wave speeds of one cell of the new state (stage 4): the running maxima of
// |v_d| + c_f, and the non-physical flag.  Without a background the x role
// evaluates it (the y role leaves the new state in the state ring's slot of
// that row, which no one reads again before the x role refills it five rows
// later): the y role's first phase is the longest of the row otherwise.
template <typename real, int NC>
__device__ __forceinline__ void new_state_speeds(const SplitCommon<real, NC> &m, const real (&un)[6], real rb0,
                                                 real eb0, real bxb0, real byb0, double &cx_t, double &cy_t,
                                                 int &bad_t) {
    const real half = (real)0.5;
    const real r0 = rb0 + un[0];
    const real ir0 = (real)1 / r0;
    const real ux = un[1] * ir0, uy = un[2] * ir0;
    const real kn = half * (un[1] * ux + un[2] * uy);
    const real bbd = bxb0 * un[4] + byb0 * un[5];
    const real b2t = un[4] * un[4] + un[5] * un[5];
    const real pkt = m.gm1 * (((un[3] - kn) - bbd) - half * b2t);
    const real b2b = bxb0 * bxb0 + byb0 * byb0;
    const real pkb = m.gm1 * (eb0 - half * b2b);
    const real pkk = pkb + pkt;
    const real bxx = bxb0 + un[4], byy = byb0 + un[5];
    const real cf = sqrt((m.gamma * pkk + (bxx * bxx + byy * byy)) * ir0);
    const bool fin = isfinite(un[0]) && isfinite(un[1]) && isfinite(un[2]) && isfinite(un[3]) &&
                     isfinite(un[4]) && isfinite(un[5]) && isfinite(cf);
    if (!(r0 > (real)0) || !(pkk > (real)0) || !fin) {
        bad_t = 1;
    } else {
        cx_t = fmax(cx_t, (double)(fabs(ux) + cf));
        cy_t = fmax(cy_t, (double)(fabs(uy) + cf));
    }
}

// x role: primitives and x fluxes of the newest row, D_x F_x, compression,
// x-face G and x-face fluxes
template <typename real, int NC, int STAGE, bool BG, bool SUR>
__device__ __forceinline__ void split_x(const StageArgs<real> &a, const SplitCommon<real, NC> &m,
                                        SplitLds<real, NC, BG> &lds, double &cx_t, double &cy_t, int &bad_t) {
    const real half = (real)0.5, two = (real)2, eight = (real)8, zero = (real)0;
    const Layout L = a.L;
    const int64_t fs = a.fstride;
    const SchemeConsts &kc = a.k;
    const int t = m.t, tm1 = m.tm1, tm2 = m.tm2, tp1 = m.tp1, tp2 = m.tp2, tp3 = m.tp3;

    real dxd[2][5];      // D_x F_x of rows r-2, r-1
    real gxw[2][5];      // own x-face G of rows r-3, r-2
    real fmx[2][4];      // x-face means (rho, v_x, v_y, B_y) of rows r-3, r-2
    real vyw[2];         // v_y of rows r-2, r-1
    real bgx[2][2];      // background on: D_x v_x, D_x v_y of rows r-2, r-1
#pragma unroll
    for (int k = 0; k < 5; ++k) dxd[0][k] = dxd[1][k] = gxw[0][k] = gxw[1][k] = 0;
    bgx[0][0] = bgx[0][1] = bgx[1][0] = bgx[1][1] = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) fmx[0][k] = fmx[1][k] = 0;
    vyw[0] = vyw[1] = 0;
    // rings read before the rows that fill them (warm-up faces only)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        lds.s[k][t] = 0;
        lds.gx[0][k][t] = lds.gx[1][k][t] = 0;
    }
    lds.gy[0][0][t] = lds.gy[0][1][t] = lds.gy[1][0][t] = lds.gy[1][1][t] = 0;

    // state rows r+1 and r+2 in flight (with their background)
    Row6<real> n1, n2;
    real g1[NBG], g2[NBG];
    {
        const int64_t ro = m.colofs + (int64_t)(m.rbeg + G) * L.pitch;
#pragma unroll
        for (int f = 0; f < NF; ++f) n1.v[f] = a.S[0][ro + f * fs];
        if (BG) {
#pragma unroll
            for (int f = 0; f < NBG; ++f) g1[f] = a.BG[0][ro + f * fs];
        }
        if (m.rbeg < m.rend) {
#pragma unroll
            for (int f = 0; f < NF; ++f) n2.v[f] = a.S[0][ro + L.pitch + f * fs];
            if (BG) {
#pragma unroll
                for (int f = 0; f < NBG; ++f) g2[f] = a.BG[0][ro + L.pitch + f * fs];
            }
        }
    }

    // surrogate: this column's periodic image in the ratio planes, its
    // column of check tiles and the tile flag of the x faces of row r-1
    // (loaded one iteration ahead, when the row enters a new row of check
    // tiles)
    const int cw = SUR ? ((m.c % L.nx) + L.nx) % L.nx : 0;
    const int ckx = SUR ? cw / a.rs_tile : 0;
    SurRow wx{};
    int fk = 0;
    if (SUR) {
        wx.set(a, m.rbeg - 1);
        fk = sur_kept(a, wx, ckx);
    }

    for (int r = m.rbeg; r <= m.rend; ++r) {
        const int slot = r & 1, pslot = slot ^ 1;
        const int s1 = ring3(r - 1);              // ring slot of row r-1
        const int sy = (r - 3 + 2 * 4096) & 1;    // ring slot of face (r-3)+1/2
        const int syp = sy ^ 1;
        // surrogate ratios of the x faces of row r-1 (used in phase 2); a
        // wave none of whose lanes is in a kept tile takes the plain path
        float rsx[5];
        bool wk = false;
        if (SUR) {
            wk = __ballot(fk) != 0;
            if (wk) sur_planes(a, wx, fk, cw, 0, rsx);
            wx.next(a);
            if (wx.in == 0) fk = sur_kept(a, wx, ckx);   // a new row of check tiles
        }
        // ---------- phase 1: row r ----------
        const Row6<real> cur = n1;
        n1 = n2;
        // the background terms of the one-thread tile; without a background
        // the same code with these zero (the operations on them are kept:
        // they decide signed zeros)
        real rb = 0, eb = 0, bxb = 0, byb = 0;
        if (BG) {
            rb = g1[0]; eb = g1[1]; bxb = g1[2]; byb = g1[3];
#pragma unroll
            for (int f = 0; f < NBG; ++f) g1[f] = g2[f];
        }
        // (with the surrogate the load is unconditional: past the last row
        // it re-reads that row, unused)
        if (SUR || r + 2 <= m.rend) {
            const int rn_row = SUR ? min(r + 2, m.rend) : r + 2;
            const int64_t rn = m.colofs + (int64_t)(rn_row + G) * L.pitch;
#pragma unroll
            for (int f = 0; f < NF; ++f) n2.v[f] = a.S[0][rn + f * fs];
            if (BG) {
#pragma unroll
                for (int f = 0; f < NBG; ++f) g2[f] = a.BG[0][rn + f * fs];
            }
        }
        const int pr = ring5(r);
        if (STAGE == 4 && !BG && r - 5 >= m.y0 && m.outcol) {
            // the slot of row r holds the new state of output row r-5
            real un[6];
#pragma unroll
            for (int f = 0; f < NF; ++f) un[f] = lds.ps[pr][f][t];
            new_state_speeds<real, NC>(m, un, zero, zero, zero, zero, cx_t, cy_t, bad_t);
        }
#pragma unroll
        for (int f = 0; f < NF; ++f) lds.ps[pr][f][t] = cur.v[f];
        const real rt = cur.v[0], mx = cur.v[1], my = cur.v[2], et = cur.v[3], bxt = cur.v[4], byt = cur.v[5];
        const real rho = rb + rt;
        const real irho = (real)1 / rho;
        const real vx = mx * irho, vy = my * irho;
        const real kin = half * (mx * vx + my * vy);
        const real bbdot = bxb * bxt + byb * byt;
        const real bt2 = bxt * bxt + byt * byt;
        const real pk = m.gm1 * (((et - kin) - bbdot) - half * bt2);
        const real pt = (pk + half * bt2) + bbdot;
        const real eps = pk * m.igm1;
        const real bxT = bxb + bxt, byT = byb + byt;
        const real bvt = bxt * vx + byt * vy;
        const real bvb = bxb * vx + byb * vy;
        const real ef = et + eb + pt;
        lds.fx[CR][t] = mx;
        lds.fx[CMX][t] = (vx * mx - (bxt * bxt + two * bxt * bxb)) + pt;
        lds.fx[CMY][t] = vx * my - (bxt * byt + bxt * byb + bxb * byt);
        lds.fx[CE][t] = ((vx * ef - bxt * bvt) - bxt * bvb) - bxb * bvt;
        lds.fx[CB][t] = vx * byT - bxT * vy;
        lds.q[slot][SQR][t] = rt;
        lds.q[slot][SQE][t] = eps;
        lds.q[slot][SQVX][t] = vx;
        lds.q[slot][SQVY][t] = vy;
        lds.q[slot][SQB][t] = byt;
        lds.q[slot][SQRHO][t] = rho;
        lds.q[slot][SQBYT][t] = byT;
        lds.q[slot][SQPT][t] = pt;
#pragma unroll
        for (int k = 0; k < 5; ++k) lds.dx[k][t] = dxd[0][k];
        if (BG) {
            lds.dx[5][t] = bgx[0][0];
            lds.dx[6][t] = bgx[0][1];
        }
        __syncthreads();  // P1

        // ---------- phase 2: s of row r-1, coefficient ratios of its x faces ----------
        // d_x v_x from the previous row buffer, d_y v_y from v_y of rows r and r-2
        const real dv = (lds.q[pslot][SQVX][tp1] - lds.q[pslot][SQVX][tm1]) * m.i2dx + (vy - vyw[0]) * m.i2dy;
        const real s_new = fmax(zero, -dv);
        lds.s[s1][t] = s_new;
        vyw[0] = vyw[1];
        vyw[1] = vy;
        real Rx[5];
        if (SUR && wk) {
            // a face takes its supplied value where it is >= 0; the plain
            // ratios are computed only by waves with a lane that needs one
            bool plain = false;
#pragma unroll
            for (int k = 0; k < 5; ++k) { Rx[k] = zero; plain = plain || !(rsx[k] >= 0.0f); }
            if (plain) {
#pragma unroll
                for (int k = 0; k < 5; ++k)
                    Rx[k] = hd_ratio(lds.q[pslot][k][tm2], lds.q[pslot][k][tm1], lds.q[pslot][k][t],
                                     lds.q[pslot][k][tp1], lds.q[pslot][k][tp2], lds.q[pslot][k][tp3]);
            }
#pragma unroll
            for (int k = 0; k < 5; ++k)
                if (rsx[k] >= 0.0f) Rx[k] = (real)rsx[k];
        } else {
#pragma unroll
            for (int k = 0; k < 5; ++k)
                Rx[k] = hd_ratio(lds.q[pslot][k][tm2], lds.q[pslot][k][tm1], lds.q[pslot][k][t],
                                 lds.q[pslot][k][tp1], lds.q[pslot][k][tp2], lds.q[pslot][k][tp3]);
        }
        __syncthreads();  // P2

        // ---------- phase 3: D_x F_x of row r, x-face G of row r-1, H_x at row r-3 ----------
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            dxd[0][k] = dxd[1][k];
            dxd[1][k] = (eight * (lds.fx[k][tp1] - lds.fx[k][tm1]) - (lds.fx[k][tp2] - lds.fx[k][tm2])) * m.i12dx;
        }
        if (BG) {
            // D_x v_x, D_x v_y of row r for the background's energy terms
            bgx[0][0] = bgx[1][0];
            bgx[0][1] = bgx[1][1];
            bgx[1][0] = (eight * (lds.q[slot][SQVX][tp1] - lds.q[slot][SQVX][tm1]) -
                         (lds.q[slot][SQVX][tp2] - lds.q[slot][SQVX][tm2])) * m.i12dx;
            bgx[1][1] = (eight * (lds.q[slot][SQVY][tp1] - lds.q[slot][SQVY][tm1]) -
                         (lds.q[slot][SQVY][tp2] - lds.q[slot][SQVY][tm2])) * m.i12dx;
        }
        const real sfx = fmax(s_new, lds.s[s1][tp1]);
        real gxn[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            const int cl = qclass(k);
            const real q2 = lds.q[pslot][k][t], q3 = lds.q[pslot][k][tp1];
            const real nu = m.kx2[cl] * Rx[k] + (real)kc.kxs[cl] * sfx;
            gxn[k] = nu * (q3 - q2) * m.idx;
        }
        real fmn[4];
        fmn[0] = half * (lds.q[pslot][SQRHO][t] + lds.q[pslot][SQRHO][tp1]);
        fmn[1] = half * (lds.q[pslot][SQVX][t] + lds.q[pslot][SQVX][tp1]);
        fmn[2] = half * (lds.q[pslot][SQVY][t] + lds.q[pslot][SQVY][tp1]);
        fmn[3] = half * (lds.q[pslot][SQBYT][t] + lds.q[pslot][SQBYT][tp1]);
        lds.gx[0][s1][t] = gxn[QVY];
        lds.gx[1][s1][t] = gxn[QB];
        real a4vx = 0, a4bx = 0;
        if (m.cross) {
            // the four y-face G around the x face (c+1/2, r-3)
            const real q = (real)0.25;
            a4vx = ((lds.gy[0][syp][t] + lds.gy[0][sy][t]) + (lds.gy[0][syp][tp1] + lds.gy[0][sy][tp1])) * q;
            a4bx = ((lds.gy[1][syp][t] + lds.gy[1][sy][t]) + (lds.gy[1][syp][tp1] + lds.gy[1][sy][tp1])) * q;
        }
        {
            const real rf = fmx[0][0], vxf = fmx[0][1], vyf = fmx[0][2], byf = fmx[0][3];
            const real txx = rf * gxw[0][QVX];
            const real txy = half * rf * (gxw[0][QVY] + a4vx);
            const real ez = gxw[0][QB] - a4bx;
            lds.hx[CR][t] = gxw[0][QR];
            lds.hx[CMX][t] = txx;
            lds.hx[CMY][t] = txy;
            lds.hx[CE][t] = (gxw[0][QE] + (vxf * txx + vyf * txy)) + byf * ez;
            lds.hx[CB][t] = ez;
        }
#pragma unroll
        for (int k = 0; k < 5; ++k) { gxw[0][k] = gxw[1][k]; gxw[1][k] = gxn[k]; }
#pragma unroll
        for (int k = 0; k < 4; ++k) { fmx[0][k] = fmx[1][k]; fmx[1][k] = fmn[k]; }
        __syncthreads();  // P3
    }
}

// L(S) of output row j from the ideal part, the x-face fluxes in LDS and the
// own y-face fluxes above (hn) and below (hp) the cell, and the stage combine
template <typename real, int NC, int STAGE, bool BG>
__device__ __forceinline__ void split_output(const StageArgs<real> &a, const SplitCommon<real, NC> &m,
                                             SplitLds<real, NC, BG> &lds, int j, const real (&kid)[6],
                                             const real (&hn)[5], const real (&hp)[5], const Row6<real> &pU,
                                             double &cx_t, double &cy_t, int &bad_t) {
    const real half = (real)0.5, zero = (real)0;
    const int64_t fs = a.fstride;
    const int t = m.t, tm1 = m.tm1;
    const int64_t oo = (int64_t)a.L.xoff + m.c + (int64_t)(j + G) * a.L.pitch;
    real K[6];
#pragma unroll
    for (int f = 0; f < 6; ++f) K[f] = kid[f];
    K[0] = K[0] + ((lds.hx[CR][t] - lds.hx[CR][tm1]) * m.idx + (hn[CR] - hp[CR]) * m.idy);
    K[1] = K[1] + ((lds.hx[CMX][t] - lds.hx[CMX][tm1]) * m.idx + (hn[CMX] - hp[CMX]) * m.idy);
    K[2] = K[2] + ((lds.hx[CMY][t] - lds.hx[CMY][tm1]) * m.idx + (hn[CMY] - hp[CMY]) * m.idy);
    K[3] = K[3] + ((lds.hx[CE][t] - lds.hx[CE][tm1]) * m.idx + (hn[CE] - hp[CE]) * m.idy);
    K[4] = K[4] + (zero + (hn[CB] - hp[CB]) * m.idy);
    K[5] = K[5] + ((lds.hx[CB][t] - lds.hx[CB][tm1]) * m.idx + zero);
    const int pj = ring5(j);   // ring slot of state row j
    if (STAGE == 1) {
#pragma unroll
        for (int f = 0; f < NF; ++f) a.out1[0][oo + f * fs] = lds.ps[pj][f][t] + m.hdt * K[f];
    } else if (STAGE == 2) {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const real u = pU.v[f], s = lds.ps[pj][f][t];
            a.out1[0][oo + f * fs] = u + m.hdt * K[f];
            a.out2[0][oo + f * fs] = (u + u) + ((s - u) + m.dt * K[f]);
        }
    } else if (STAGE == 3) {
#pragma unroll
        for (int f = 0; f < NF; ++f) a.out1[0][oo + f * fs] = pU.v[f] + m.dt * K[f];
    } else {
        real un[6];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            const real av = pU.v[f], s = lds.ps[pj][f][t];
            un[f] = (s + (av - (s + s)) * m.third) + m.dt6 * K[f];
            a.out1[0][oo + f * fs] = un[f];
        }
        // wave speeds of the new state (next step's dt and c_max): here with
        // a background, else by the x role from the state ring
        if (BG) {
            const real rb0 = a.BG[0][oo], eb0 = a.BG[0][oo + 1 * fs], bxb0 = a.BG[0][oo + 2 * fs],
                       byb0 = a.BG[0][oo + 3 * fs];
            new_state_speeds<real, NC>(m, un, rb0, eb0, bxb0, byb0, cx_t, cy_t, bad_t);
        } else {
#pragma unroll
            for (int f = 0; f < NF; ++f) lds.ps[pj][f][t] = un[f];
        }
    }
}

// y role: y-face G, y fluxes, D_y F_y, the ideal L, y-face fluxes, and one
// iteration later L(S) of the output row and the stage combine
template <typename real, int NC, int STAGE, bool BG, bool SUR>
__device__ __forceinline__ void split_y(const StageArgs<real> &a, const SplitCommon<real, NC> &m,
                                        SplitLds<real, NC, BG> &lds, double &cx_t, double &cy_t, int &bad_t) {
    const real half = (real)0.5, two = (real)2, eight = (real)8, zero = (real)0;
    const Layout L = a.L;
    const int64_t fs = a.fstride;
    const SchemeConsts &kc = a.k;
    const int t = m.t, tm1 = m.tm1;

    real qw[5][6];       // y-face set {rho~, eps~, v_x, v_y, B~_x}, rows r-5..r
    real fyw[5][4];      // y fluxes of rows r-4..r-1
    real kia[6], kib[6]; // ideal L of rows r-4, r-3
    real ha[5], hb[5];   // own y-face H at faces (r-5)+1/2, (r-4)+1/2
    Row6<real> pUa;      // pointwise operand of row r-4
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        ha[k] = hb[k] = 0;
#pragma unroll
        for (int q = 0; q < 6; ++q) qw[k][q] = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) fyw[k][q] = 0;
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) kia[k] = kib[k] = 0;
#pragma unroll
    for (int f = 0; f < NF; ++f) pUa.v[f] = 0;

    // surrogate: the tile flag of the y faces (r-3)+1/2 (loaded one
    // iteration ahead, when the face row enters a new row of check tiles)
    const int cw = SUR ? ((m.c % L.nx) + L.nx) % L.nx : 0;
    const int ckx = SUR ? cw / a.rs_tile : 0;
    SurRow wy{};
    int fy = 0;
    if (SUR) {
        wy.set(a, m.rbeg - 3);
        fy = sur_kept(a, wy, ckx);
    }

    for (int r = m.rbeg; r <= m.rend; ++r) {
        const int slot = r & 1;
        const int s2 = ring3(r - 2), s3 = ring3(r - 3);
        const int sy = (r - 3 + 2 * 4096) & 1;
        // surrogate ratios of the y faces (r-3)+1/2 (used in phase 2); a
        // wave none of whose lanes is in a kept tile takes the plain path
        float rsy[5];
        bool wk = false;
        if (SUR) {
            wk = __ballot(fy) != 0;
            if (wk) sur_planes(a, wy, fy, cw, 5, rsy);
            wy.next(a);
            if (wy.in == 0) fy = sur_kept(a, wy, ckx);   // a new row of check tiles
        }
        // ---------- phase 1: output row r-4, operands of row r-3 ----------
        if (r - 4 >= m.y0 && m.outcol)
            split_output<real, NC, STAGE, BG>(a, m, lds, r - 4, kia, hb, ha, pUa, cx_t, cy_t, bad_t);
        const int j = r - G;
        const bool outrow = j >= m.y0 && m.outcol;
        Row6<real> pUb;
        if (SUR || outrow) {
            // (with the surrogate the load is unconditional: a thread without
            // an output row reads a cell of its own column instead, unused)
            const int64_t oo = SUR && !outrow ? m.colofs + (int64_t)(max(j, m.y0) + G) * L.pitch
                                              : (int64_t)L.xoff + m.c + (int64_t)(j + G) * L.pitch;
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                if (STAGE == 2 || STAGE == 3) pUb.v[f] = a.U[0][oo + f * fs];
                if (STAGE == 4) pUb.v[f] = a.A[0][oo + f * fs];
            }
        }
        __syncthreads();  // P1

        // ---------- phase 2: y-face G of face (r-3)+1/2 ----------
        // background of rows r (y fluxes), r-2 (energy terms, y-face means)
        // and r-3 (y-face means), rows below -G clamped as in the one-thread
        // tile (those rows only feed warm-up faces); without a background the
        // zeros of the one-thread tile
        real eb = 0, bxb = 0, byb = 0, rb2 = 0, eb2 = 0, bxb2 = 0, byb2 = 0, rb3 = 0, bxb3 = 0;
        if (BG) {
            const int64_t rr = m.colofs + (int64_t)(r + G) * L.pitch;
            const int64_t r2 = m.colofs + (int64_t)((r - 2 < -G ? -G : r - 2) + G) * L.pitch;
            const int64_t r3 = m.colofs + (int64_t)((r - 3 < -G ? -G : r - 3) + G) * L.pitch;
            eb = a.BG[0][rr + 1 * fs]; bxb = a.BG[0][rr + 2 * fs]; byb = a.BG[0][rr + 3 * fs];
            rb2 = a.BG[0][r2]; eb2 = a.BG[0][r2 + 1 * fs]; bxb2 = a.BG[0][r2 + 2 * fs]; byb2 = a.BG[0][r2 + 3 * fs];
            rb3 = a.BG[0][r3]; bxb3 = a.BG[0][r3 + 2 * fs];
        }
        const int pr = ring5(r);
        const real rt = lds.ps[pr][0][t], bxt = lds.ps[pr][4][t];
        const real eps = lds.q[slot][SQE][t], vx = lds.q[slot][SQVX][t], vy = lds.q[slot][SQVY][t];
#pragma unroll
        for (int k = 0; k < 5; ++k)
#pragma unroll
            for (int q = 0; q < 5; ++q) qw[k][q] = qw[k][q + 1];
        qw[QR][5] = rt; qw[QE][5] = eps; qw[QVX][5] = vx; qw[QVY][5] = vy; qw[QB][5] = bxt;
        // s of rows r-3 and r-2
        const real sfy = fmax(lds.s[s3][t], lds.s[s2][t]);
        real gyn[5];
        if (SUR && wk) {
            // a face takes its supplied value where it is >= 0; the plain
            // ratios are computed only by waves with a lane that needs one
            real Ry[5];
            bool plain = false;
#pragma unroll
            for (int k = 0; k < 5; ++k) { Ry[k] = zero; plain = plain || !(rsy[k] >= 0.0f); }
            if (plain) {
#pragma unroll
                for (int k = 0; k < 5; ++k)
                    Ry[k] = hd_ratio(qw[k][0], qw[k][1], qw[k][2], qw[k][3], qw[k][4], qw[k][5]);
            }
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                if (rsy[k] >= 0.0f) Ry[k] = (real)rsy[k];
                const int cl = qclass(k);
                const real nu = m.ky2[cl] * Ry[k] + (real)kc.kys[cl] * sfy;
                gyn[k] = nu * (qw[k][3] - qw[k][2]) * m.idy;
            }
        } else {
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                const int cl = qclass(k);
                const real R = hd_ratio(qw[k][0], qw[k][1], qw[k][2], qw[k][3], qw[k][4], qw[k][5]);
                const real nu = m.ky2[cl] * R + (real)kc.kys[cl] * sfy;
                gyn[k] = nu * (qw[k][3] - qw[k][2]) * m.idy;
            }
        }
        lds.gy[0][sy][t] = gyn[QVX];
        lds.gy[1][sy][t] = gyn[QB];
        __syncthreads();  // P2

        // ---------- phase 3: y fluxes of row r, ideal L of row r-2, H_y at face (r-3)+1/2 ----------
        {
            const real mx = lds.ps[pr][1][t], my = lds.ps[pr][2][t], et = lds.ps[pr][3][t];
            const real byt = lds.ps[pr][5][t];
            const real pt = lds.q[slot][SQPT][t];
            const real bxT = bxb + bxt, byT = byb + byt;
            const real bvt = bxt * vx + byt * vy;
            const real bvb = bxb * vx + byb * vy;
            const real ef = et + eb + pt;
            real fy[5];
            fy[CR] = my;
            fy[CMX] = vy * mx - (byt * bxt + byt * bxb + byb * bxt);
            fy[CMY] = (vy * my - (byt * byt + two * byt * byb)) + pt;
            fy[CE] = ((vy * ef - byt * bvt) - byt * bvb) - byb * bvt;
            fy[CB] = vy * bxT - byT * vx;
            real dyn[5];
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                dyn[k] = (eight * (fyw[k][3] - fyw[k][1]) - (fy[k] - fyw[k][0])) * m.i12dy;
                fyw[k][0] = fyw[k][1]; fyw[k][1] = fyw[k][2]; fyw[k][2] = fyw[k][3]; fyw[k][3] = fy[k];
            }
#pragma unroll
            for (int k = 0; k < 6; ++k) kia[k] = kib[k];
            kib[0] = -(lds.dx[CR][t] + dyn[CR]);
            kib[1] = -(lds.dx[CMX][t] + dyn[CMX]);
            kib[2] = -(lds.dx[CMY][t] + dyn[CMY]);
            kib[3] = -(lds.dx[CE][t] + dyn[CE]);
            kib[4] = -(zero + dyn[CB]);   // B~_x has no x flux
            kib[5] = -(lds.dx[CB][t] + zero);  // B~_y has no y flux
            if (BG) {
                // e~ of row r-2 gets -p_tb div v + sum_kl B_bk B_bl d_k v_l
                const real dxvx = lds.dx[5][t], dxvy = lds.dx[6][t];
                const real dyvx = (eight * (qw[QVX][4] - qw[QVX][2]) - (qw[QVX][5] - qw[QVX][1])) * m.i12dy;
                const real dyvy = (eight * (qw[QVY][4] - qw[QVY][2]) - (qw[QVY][5] - qw[QVY][1])) * m.i12dy;
                const real b2b = bxb2 * bxb2 + byb2 * byb2;
                const real pkb = m.gm1 * (eb2 - half * b2b);
                const real ptb = pkb + half * b2b;
                const real bb = (bxb2 * bxb2 * dxvx + byb2 * byb2 * dyvy) + (bxb2 * byb2 * dxvy + byb2 * bxb2 * dyvx);
                kib[3] = kib[3] + (bb - ptb * (dxvx + dyvy));
            }
            if (m.grav) {
                // gravity on the perturbation density of row r-2 (window index 3)
                const real rg = qw[QR][3];
                kib[1] = kib[1] + rg * m.gx;
                kib[2] = kib[2] + rg * m.gy;
                kib[3] = kib[3] + rg * (m.gx * qw[QVX][3] + m.gy * qw[QVY][3]);
            }
        }
        real a4vy = 0, a4by = 0;
        if (m.cross) {
            // the four x-face G around the y face (c, (r-3)+1/2)
            const real q = (real)0.25;
            a4vy = ((lds.gx[0][s3][tm1] + lds.gx[0][s3][t]) + (lds.gx[0][s2][tm1] + lds.gx[0][s2][t])) * q;
            a4by = ((lds.gx[1][s3][tm1] + lds.gx[1][s3][t]) + (lds.gx[1][s2][tm1] + lds.gx[1][s2][t])) * q;
        }
#pragma unroll
        for (int k = 0; k < 5; ++k) ha[k] = hb[k];
        {
            const real rj = BG ? rb3 + qw[QR][2] : qw[QR][2];
            const real rj1 = BG ? rb2 + qw[QR][3] : qw[QR][3];
            const real bj = BG ? bxb3 + qw[QB][2] : qw[QB][2];
            const real bj1 = BG ? bxb2 + qw[QB][3] : qw[QB][3];
            const real rf = half * (rj + rj1);
            const real vxf = half * (qw[QVX][2] + qw[QVX][3]);
            const real vyf = half * (qw[QVY][2] + qw[QVY][3]);
            const real bxf = half * (bj + bj1);
            const real tyy = rf * gyn[QVY];
            const real tyx = half * rf * (gyn[QVX] + a4vy);
            const real ez = a4by - gyn[QB];
            hb[CR] = gyn[QR];
            hb[CMX] = tyx;
            hb[CMY] = tyy;
            hb[CE] = (gyn[QE] + (vyf * tyy + vxf * tyx)) - bxf * ez;
            hb[CB] = -ez;
        }
        pUa = pUb;
        __syncthreads();  // P3
    }
    // the last output row (its x-face fluxes were published before P3)
    if (m.rend - G >= m.y0 && m.outcol)
        split_output<real, NC, STAGE, BG>(a, m, lds, m.rend - G, kia, hb, ha, pUa, cx_t, cy_t, bad_t);
}

template <typename real, int NC, int STAGE, bool BG, bool SUR = false>
__device__ __forceinline__ void stage_tile_split(const StageArgs<real> &a, int tile_x, int tile_y,
                                                 SplitLds<real, NC, BG> &lds) {
    if (!a.sc->active) return;
    // the role is a property of the wave (NC is a multiple of 64): taking it
    // from a wave-uniform value keeps the two role loops apart in the
    // compiled code, so their windows share registers
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const bool xrole = wave < NC / 64;
    const SplitCommon<real, NC> m(a, tile_x, tile_y, xrole ? (int)threadIdx.x : (int)threadIdx.x - NC);
    double cx_t = 0.0, cy_t = 0.0;
    int bad_t = 0;
    if (xrole)
        split_x<real, NC, STAGE, BG, SUR>(a, m, lds, cx_t, cy_t, bad_t);
    else
        split_y<real, NC, STAGE, BG, SUR>(a, m, lds, cx_t, cy_t, bad_t);

    if (STAGE == 4 && !BG) {
        // the new state of the last two output rows (rend-4, rend-3), left
        // in the ring by the y role's last iteration and its final row
        __syncthreads();
        if (xrole) {
#pragma unroll
            for (int k = 4; k >= 3; --k) {
                const int jj = m.rend - k;
                if (jj >= m.y0 && m.outcol) {
                    const int pj = ring5(jj);
                    real un[6];
#pragma unroll
                    for (int f = 0; f < NF; ++f) un[f] = lds.ps[pj][f][m.t];
                    new_state_speeds<real, NC>(m, un, (real)0, (real)0, (real)0, (real)0, cx_t, cy_t, bad_t);
                }
            }
        }
    }
    if (STAGE == 4) {
        // block reduction of the wave speeds, one atomic per block
        auto &red = lds.red;
        for (int off = 32; off > 0; off >>= 1) {
            cx_t = fmax(cx_t, __shfl_xor(cx_t, off));
            cy_t = fmax(cy_t, __shfl_xor(cy_t, off));
            bad_t |= __shfl_xor(bad_t, off);
        }
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) { red[0][w] = cx_t; red[1][w] = cy_t; red[2][w] = (double)bad_t; }
        __syncthreads();
        if (threadIdx.x == 0) {
            double mx_ = 0.0, my_ = 0.0, bb = 0.0;
            for (int k = 0; k < 2 * NC / 64; ++k) { mx_ = fmax(mx_, red[0][k]); my_ = fmax(my_, red[1][k]); bb = fmax(bb, red[2][k]); }
            DevScalars *scw = a.sc;
            const int nslot = scw->cur ^ 1;
            atomicMax(&scw->cacc[nslot][0], (unsigned long long)__double_as_longlong(mx_));
            atomicMax(&scw->cacc[nslot][1], (unsigned long long)__double_as_longlong(my_));
            if (bb > 0.0) atomicOr(&scw->nonphys, 1);
        }
    }
}

}  // namespace sacx
