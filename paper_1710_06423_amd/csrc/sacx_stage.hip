// sacx_stage.hip -- the fused RK stage kernel of the SAC MHD hot path on gfx950.
//
// One launch evaluates L(S) (ideal split-variable MHD fluxes differenced with
// fourth-order central differences, plus the hyper-diffusive fluxes) for every
// interior cell of one subdomain and applies the stage's Runge-Kutta combine
// (paper section 2).  Stage 4 also reduces the wave speeds of the new state
// for the next CFL time step.
//
// Work decomposition (MI355X: wave64, 160 KB LDS per CU, HBM-bound stencil):
//  * a block of NT = 256 threads owns TX = 250 output columns; thread t holds
//    column c = x0 - 3 + t, so the 3-cell apron on each side is computed by
//    the 6 edge threads (2.4 % redundant work in x);
//  * the block marches up a strip of `ty` output rows, loading each state row
//    once (coalesced 2 KB row segments); quantities that only couple cells of
//    one column (y differences, y-face hyper-diffusion windows) live in
//    per-thread register windows, so the 3-cell y apron costs 6 warm-up rows
//    per strip instead of an LDS tile halo;
//  * cross-column coupling (x differences, x-face windows, the four-face
//    averages of the cross terms) goes through small LDS row buffers, four
//    barriers per row;
//  * the stage combine, and in stage 4 the wave-speed reduction, are fused in
//    the epilogue: each evolved field is read once as a stencil input and
//    once pointwise, then written once, so the whole RK4 step moves 12 field
//    values per cell (the 12-access form described in sacx_runtime.hip).
//
// Pipeline of iteration r (row r is the newest row loaded):
//   A  : load S(r); primitives, ideal fluxes; publish x-neighbour data
//   A' : D_x F_x(r); x-face ratio R and first difference at row r; x-face
//        means; compression s at row r-1 (needs v_y of rows r-2 and r)
//   C  : x-face G = nu d1 / h at row r-1; y-face G at face (r-3)+1/2
//   D  : face fluxes H_x at (c+1/2, r-3) and H_y at (c, (r-3)+1/2)
//   E  : L(S) at row j = r-3 and the stage combine
//
// Arithmetic: every operation is the same IEEE double (or float) operation,
// in the same order, as in the scheme's defining sequence (the test oracle):
// divisions by grid constants are multiplications by reciprocals computed in
// FP64, no multiply-add is fused (the library is built with
// -ffp-contract=off), and the stage combine is the storage-saving RK4
// arrangement.  The hyper-diffusion coefficient, a ratio of maxima of
// differences, amplifies any rounding difference by many orders of magnitude
// over a run, so FP64 results are reproduced bit for bit instead.
#include "sacx_internal.h"

namespace sacx {

constexpr int NT = 256;
constexpr int TX = NT - 2 * G;

// slots of the hyper-diffusion quantity sets: x faces {rho~, eps~, v_x, v_y, B~_y},
// y faces {rho~, eps~, v_x, v_y, B~_x}
enum { QR = 0, QE = 1, QVX = 2, QVY = 3, QB = 4 };
// flux component slots: x {rho, m_x, m_y, e, B_y}, y {rho, m_x, m_y, e, B_x}
enum { CR = 0, CMX = 1, CMY = 2, CE = 3, CB = 4 };
// constant class of each quantity slot: density, thermal energy, velocity, field
__device__ __forceinline__ int qclass(int k) { return k == QR ? 0 : (k == QE ? 1 : (k == QB ? 3 : 2)); }

template <typename real>
__device__ __forceinline__ real rmax(real a, real b) { return a > b ? a : b; }

// Hyper-diffusion coefficient ratio at the face between q2 and q3, from the
// six values q[i-2..i+3]: max |third difference| over the 3 faces around the
// face divided by max |first difference| over the 5 faces around it (0 when
// the latter vanishes).
template <typename real>
__device__ __forceinline__ real hd_ratio(real q0, real q1, real q2, real q3, real q4, real q5) {
    const real three = (real)3;
    real d3a = (q3 - q0) - three * (q2 - q1);
    real d3b = (q4 - q1) - three * (q3 - q2);
    real d3c = (q5 - q2) - three * (q4 - q3);
    real n = 0;
    n = rmax(n, fabs(d3a));
    n = rmax(n, fabs(d3b));
    n = rmax(n, fabs(d3c));
    real m = 0;
    m = rmax(m, fabs(q1 - q0));
    m = rmax(m, fabs(q2 - q1));
    m = rmax(m, fabs(q3 - q2));
    m = rmax(m, fabs(q4 - q3));
    m = rmax(m, fabs(q5 - q4));
    return m > (real)0 ? n / m : (real)0;
}

template <typename real, int STAGE, bool HD, bool BG>
__global__ __launch_bounds__(NT) void k_stage(StageArgs<real> a) {
    DevScalars *sc = a.sc;
    if (!sc->active) return;
    const double dtd = sc->dt;
    const real cmax = (real)sc->cmax;
    const real dt = (real)dtd, hdt = (real)(0.5 * dtd), dt6 = (real)(dtd / 6.0);
    const real third = (real)(1.0 / 3.0);

    const Layout L = a.L;
    const int tid = threadIdx.x;
    const int x0 = blockIdx.x * TX;
    const int c = x0 - G + tid;
    const bool colv = c < L.nx + G;
    const int y0 = blockIdx.y * a.ty;
    const int y1 = min(y0 + a.ty, L.ny);
    const bool outcol = tid >= G && tid < NT - G && c < L.nx;

    const real gamma = (real)a.gamma;
    const real gm1 = (real)(a.gamma - 1.0);
    const real igm1 = (real)(1.0 / (a.gamma - 1.0));
    const real half = (real)0.5, two = (real)2, eight = (real)8;
    const real i12dx = (real)(1.0 / (12.0 * a.dx)), i12dy = (real)(1.0 / (12.0 * a.dy));
    const real idx = (real)(1.0 / a.dx), idy = (real)(1.0 / a.dy);
    const real i2dx = (real)(1.0 / (2.0 * a.dx)), i2dy = (real)(1.0 / (2.0 * a.dy));
    real kx2[4], kxs[4], ky2[4], kys[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        kx2[k] = (real)(a.c2[k] * a.dx * (double)sc->cmax);
        ky2[k] = (real)(a.c2[k] * a.dy * (double)sc->cmax);
        kxs[k] = (real)(a.cshk[k] * a.dx * a.dx);
        kys[k] = (real)(a.cshk[k] * a.dy * a.dy);
    }
    (void)cmax;
    const bool cross = a.hd_cross_on != 0;

    // clamped LDS neighbour indices (edge threads compute unused values)
    const int tm1 = tid >= 1 ? tid - 1 : 0;
    const int tm2 = tid >= 2 ? tid - 2 : 0;
    const int tp1 = tid + 1 < NT ? tid + 1 : NT - 1;
    const int tp2 = tid + 2 < NT ? tid + 2 : NT - 1;
    const int tp3 = tid + 3 < NT ? tid + 3 : NT - 1;

    __shared__ real sh_fx[5][NT];   // x fluxes of the newest row
    __shared__ real sh_qx[5][NT];   // x-face quantity set of the newest row
    __shared__ real sh_rho[NT];     // total density, newest row
    __shared__ real sh_byT[NT];     // total B_y, newest row
    __shared__ real sh_s[NT];       // compression s, row r-1
    __shared__ real sh_gx[2][3][NT];  // x-face G(v_y), G(B~_y), ring over rows (mod 3)
    __shared__ real sh_gy[2][2][NT];  // y-face G(v_x), G(B~_x), ring over faces (mod 2)
    __shared__ real sh_hx[5][NT];     // x-face fluxes H_x at row r-3

    const int64_t colofs = (int64_t)L.xoff + (colv ? c : L.nx + G - 1);

    // ---------------- per-thread windows (column-local data) ----------------
    real qw[5][6];      // y-face set, rows r-5..r
    real rhow[4], bxTw[4];  // totals rows r-3..r (background on)
    real fyw[5][5];     // y fluxes rows r-4..r
    real dyd[5];        // D_y F_y of row r-3
    real dxd[3][5];     // D_x F_x of rows r-3..r-1
    real bgv[4][4];     // D_x v_x, D_x v_y of rows r-3..r-1 (background on): [row][0..1]
    real rxd[5], d1xd[5];   // x-face R and d1 of row r-1
    real fmx[3][4];     // x-face means (rho, v_x, v_y, B_y) of rows r-3..r-1
    real dvxp;          // d_x v_x of row r-1
    real sw[2];         // s of rows r-3, r-2
    real gxw[2][5];     // own x-face G of rows r-3, r-2
    real gyp[2];        // own y-face G(v_x), G(B~_x) at face (r-4)+1/2
    real hyp[5];        // own y-face H at face (r-4)+1/2
#pragma unroll
    for (int k = 0; k < 5; ++k) {
#pragma unroll
        for (int m = 0; m < 6; ++m) qw[k][m] = 0;
#pragma unroll
        for (int m = 0; m < 5; ++m) fyw[k][m] = 0;
        dyd[k] = 0; rxd[k] = 0; d1xd[k] = 0; hyp[k] = 0;
        gxw[0][k] = 0; gxw[1][k] = 0;
#pragma unroll
        for (int m = 0; m < 3; ++m) dxd[m][k] = 0;
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        rhow[m] = 0; bxTw[m] = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) bgv[m][k] = 0;
    }
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int k = 0; k < 4; ++k) fmx[m][k] = 0;
    dvxp = 0; sw[0] = sw[1] = 0; gyp[0] = gyp[1] = 0;

    double cx_t = 0.0, cy_t = 0.0;
    int bad_t = 0;

    for (int r = y0 - G; r <= y1 - 1 + G; ++r) {
        const int64_t ro = colofs + (int64_t)(r + G) * L.pitch;
        // ================= A: load row r, primitives, fluxes =================
        const real rt = a.S[0][ro], mx = a.S[1][ro], my = a.S[2][ro];
        const real et = a.S[3][ro], bxt = a.S[4][ro], byt = a.S[5][ro];
        real rb = 0, eb = 0, bxb = 0, byb = 0;
        if (BG) { rb = a.BG[0][ro]; eb = a.BG[1][ro]; bxb = a.BG[2][ro]; byb = a.BG[3][ro]; }
        const real rho = rb + rt;
        const real irho = (real)1 / rho;
        const real vx = mx * irho, vy = my * irho;
        const real kin = half * (mx * vx + my * vy);
        const real bbdot = bxb * bxt + byb * byt;
        const real bt2 = bxt * bxt + byt * byt;
        const real pk = gm1 * (((et - kin) - bbdot) - half * bt2);
        const real pt = (pk + half * bt2) + bbdot;
        const real eps = pk * igm1;
        const real bxT = bxb + bxt, byT = byb + byt;
        const real bvt = bxt * vx + byt * vy;
        const real bvb = bxb * vx + byb * vy;
        const real ef = et + eb + pt;
        real fx[5], fy[5];
        fx[CR] = mx;
        fx[CMX] = (vx * mx - (bxt * bxt + two * bxt * bxb)) + pt;
        fx[CMY] = vx * my - (bxt * byt + bxt * byb + bxb * byt);
        fx[CE] = ((vx * ef - bxt * bvt) - bxt * bvb) - bxb * bvt;
        fx[CB] = vx * byT - bxT * vy;
        fy[CR] = my;
        fy[CMX] = vy * mx - (byt * bxt + byt * bxb + byb * bxt);
        fy[CMY] = (vy * my - (byt * byt + two * byt * byb)) + pt;
        fy[CE] = ((vy * ef - byt * bvt) - byt * bvb) - byb * bvt;
        fy[CB] = vy * bxT - byT * vx;

#pragma unroll
        for (int k = 0; k < 5; ++k) sh_fx[k][tid] = fx[k];
        if (HD || BG) {
            sh_qx[QR][tid] = rt;
            sh_qx[QE][tid] = eps;
            sh_qx[QVX][tid] = vx;
            sh_qx[QVY][tid] = vy;
            sh_qx[QB][tid] = byt;
            sh_rho[tid] = rho;
            sh_byT[tid] = byT;
        }
        // shift column windows and insert row r
#pragma unroll
        for (int k = 0; k < 5; ++k) {
#pragma unroll
            for (int m = 0; m < 5; ++m) qw[k][m] = qw[k][m + 1];
#pragma unroll
            for (int m = 0; m < 4; ++m) fyw[k][m] = fyw[k][m + 1];
            fyw[k][4] = fy[k];
        }
        qw[QR][5] = rt; qw[QE][5] = eps; qw[QVX][5] = vx; qw[QVY][5] = vy; qw[QB][5] = bxt;
#pragma unroll
        for (int m = 0; m < 3; ++m) { rhow[m] = rhow[m + 1]; bxTw[m] = bxTw[m + 1]; }
        rhow[3] = rho; bxTw[3] = bxT;
        __syncthreads();  // B1

        // ================= A': x work on row r =================
        real dxn[5];
#pragma unroll
        for (int k = 0; k < 5; ++k)
            dxn[k] = (eight * (sh_fx[k][tp1] - sh_fx[k][tm1]) - (sh_fx[k][tp2] - sh_fx[k][tm2])) * i12dx;
        real bgn0 = 0, bgn1 = 0;
        if (BG) {
            bgn0 = (eight * (sh_qx[QVX][tp1] - sh_qx[QVX][tm1]) - (sh_qx[QVX][tp2] - sh_qx[QVX][tm2])) * i12dx;
            bgn1 = (eight * (sh_qx[QVY][tp1] - sh_qx[QVY][tm1]) - (sh_qx[QVY][tp2] - sh_qx[QVY][tm2])) * i12dx;
        }
        real rxn[5], d1xn[5], fmn[4], gxn[5], gyn[5], hyn[5];
        real s_new = 0, dvxn = 0;
        if (HD) {
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                const real q0 = sh_qx[k][tm2], q1 = sh_qx[k][tm1], q2 = sh_qx[k][tid];
                const real q3 = sh_qx[k][tp1], q4 = sh_qx[k][tp2], q5 = sh_qx[k][tp3];
                rxn[k] = hd_ratio(q0, q1, q2, q3, q4, q5);
                d1xn[k] = q3 - q2;
            }
            fmn[0] = half * (rho + sh_rho[tp1]);
            fmn[1] = half * (vx + sh_qx[QVX][tp1]);
            fmn[2] = half * (vy + sh_qx[QVY][tp1]);
            fmn[3] = half * (byT + sh_byT[tp1]);
            dvxn = (sh_qx[QVX][tp1] - sh_qx[QVX][tm1]) * i2dx;
            // s at row r-1: v_y of rows r (qw idx 5) and r-2 (idx 3)
            const real dv = dvxp + (qw[QVY][5] - qw[QVY][3]) * i2dy;
            s_new = rmax((real)0, -dv);
            sh_s[tid] = s_new;
            __syncthreads();  // B2

            // ================= C: x-face G at row r-1, y-face G at face (r-3)+1/2 ===
            const real sfx = rmax(s_new, sh_s[tp1]);
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                const int cl = qclass(k);
                const real nu = kx2[cl] * rxd[k] + kxs[cl] * sfx;
                gxn[k] = nu * d1xd[k] * idx;
            }
            const real sfy = rmax(sw[0], sw[1]);
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                const int cl = qclass(k);
                const real R = hd_ratio(qw[k][0], qw[k][1], qw[k][2], qw[k][3], qw[k][4], qw[k][5]);
                const real nu = ky2[cl] * R + kys[cl] * sfy;
                gyn[k] = nu * (qw[k][3] - qw[k][2]) * idy;
            }
            const int sx = (r - 1 + 3 * 4096) % 3;   // ring slot of row r-1 (rows >= -3)
            const int sy = (r - 3 + 2 * 4096) & 1;   // ring slot of face (r-3)+1/2
            sh_gx[0][sx][tid] = gxn[QVY];
            sh_gx[1][sx][tid] = gxn[QB];
            sh_gy[0][sy][tid] = gyn[QVX];
            sh_gy[1][sy][tid] = gyn[QB];
            __syncthreads();  // B3

            // ================= D: face fluxes of row j = r-3 =================
            const int sxj = (r - 3 + 3 * 4096) % 3, sxj1 = (r - 2 + 3 * 4096) % 3;
            const int syp = sy ^ 1;
            // H_x at (c+1/2, j)
            real a4vx = 0, a4bx = 0, a4vy = 0, a4by = 0;
            if (cross) {
                a4vx = ((gyp[0] + gyn[QVX]) + (sh_gy[0][syp][tp1] + sh_gy[0][sy][tp1])) * (real)0.25;
                a4bx = ((gyp[1] + gyn[QB]) + (sh_gy[1][syp][tp1] + sh_gy[1][sy][tp1])) * (real)0.25;
                a4vy = ((sh_gx[0][sxj][tm1] + gxw[0][QVY]) + (sh_gx[0][sxj1][tm1] + gxw[1][QVY])) * (real)0.25;
                a4by = ((sh_gx[1][sxj][tm1] + gxw[0][QB]) + (sh_gx[1][sxj1][tm1] + gxw[1][QB])) * (real)0.25;
            }
            {
                const real rf = fmx[0][0], vxf = fmx[0][1], vyf = fmx[0][2], byf = fmx[0][3];
                const real txx = rf * gxw[0][QVX];
                const real txy = half * rf * (gxw[0][QVY] + a4vx);
                const real ez = gxw[0][QB] - a4bx;
                sh_hx[CR][tid] = gxw[0][QR];
                sh_hx[CMX][tid] = txx;
                sh_hx[CMY][tid] = txy;
                sh_hx[CE][tid] = (gxw[0][QE] + (vxf * txx + vyf * txy)) + byf * ez;
                sh_hx[CB][tid] = ez;
            }
            {
                // H_y at (c, j+1/2): rows j (idx 2 of qw / 0 of rhow) and j+1
                const real rf = half * (rhow[0] + rhow[1]);
                const real vxf = half * (qw[QVX][2] + qw[QVX][3]);
                const real vyf = half * (qw[QVY][2] + qw[QVY][3]);
                const real bxf = half * (bxTw[0] + bxTw[1]);
                const real tyy = rf * gyn[QVY];
                const real tyx = half * rf * (gyn[QVX] + a4vy);
                const real ez = a4by - gyn[QB];
                hyn[CR] = gyn[QR];
                hyn[CMX] = tyx;
                hyn[CMY] = tyy;
                hyn[CE] = (gyn[QE] + (vyf * tyy + vxf * tyx)) - bxf * ez;
                hyn[CB] = -ez;
            }
        }
        __syncthreads();  // B4 (also orders the next row's LDS writes after all reads)

        // ================= E: output row j = r-3 =================
        const int j = r - G;
        if (j >= y0 && outcol) {
            const int64_t oo = (int64_t)L.xoff + c + (int64_t)(j + G) * L.pitch;
            // ideal part: -(D_x F_x + D_y F_y) per evolved field
            real K[6];
            K[0] = -(dxd[0][CR] + dyd[CR]);
            K[1] = -(dxd[0][CMX] + dyd[CMX]);
            K[2] = -(dxd[0][CMY] + dyd[CMY]);
            K[3] = -(dxd[0][CE] + dyd[CE]);
            // B~_x has no x flux and B~_y no y flux: their (zero) differences
            // still enter the sums, as in the defining sequence
            K[4] = -((real)0 + dyd[CB]);
            K[5] = -(dxd[0][CB] + (real)0);
            if (BG) {
                // e~ gets -p_tb div v + sum_kl B_bk B_bl d_k v_l
                const real bxb0 = a.BG[2][oo], byb0 = a.BG[3][oo], eb0 = a.BG[1][oo];
                const real dxvx = bgv[0][0], dxvy = bgv[0][1];
                const real dyvx = (eight * (qw[QVX][3] - qw[QVX][1]) - (qw[QVX][4] - qw[QVX][0])) * i12dy;
                const real dyvy = (eight * (qw[QVY][3] - qw[QVY][1]) - (qw[QVY][4] - qw[QVY][0])) * i12dy;
                const real b2b = bxb0 * bxb0 + byb0 * byb0;
                const real pkb = gm1 * (eb0 - half * b2b);
                const real ptb = pkb + half * b2b;
                const real bb = (bxb0 * bxb0 * dxvx + byb0 * byb0 * dyvy) + (bxb0 * byb0 * dxvy + byb0 * bxb0 * dyvx);
                K[3] = K[3] + (bb - ptb * (dxvx + dyvy));
            }
            if (HD) {
                K[0] = K[0] + ((sh_hx[CR][tid] - sh_hx[CR][tm1]) * idx + (hyn[CR] - hyp[CR]) * idy);
                K[1] = K[1] + ((sh_hx[CMX][tid] - sh_hx[CMX][tm1]) * idx + (hyn[CMX] - hyp[CMX]) * idy);
                K[2] = K[2] + ((sh_hx[CMY][tid] - sh_hx[CMY][tm1]) * idx + (hyn[CMY] - hyp[CMY]) * idy);
                K[3] = K[3] + ((sh_hx[CE][tid] - sh_hx[CE][tm1]) * idx + (hyn[CE] - hyp[CE]) * idy);
                K[4] = K[4] + ((real)0 + (hyn[CB] - hyp[CB]) * idy);
                K[5] = K[5] + ((sh_hx[CB][tid] - sh_hx[CB][tm1]) * idx + (real)0);
            }
            if (STAGE == 1) {
#pragma unroll
                for (int f = 0; f < NF; ++f) a.out1[f][oo] = a.S[f][oo] + hdt * K[f];
            } else if (STAGE == 2) {
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    const real u = a.U[f][oo], s = a.S[f][oo];
                    a.out1[f][oo] = u + hdt * K[f];
                    a.out2[f][oo] = (u + u) + ((s - u) + dt * K[f]);
                }
            } else if (STAGE == 3) {
#pragma unroll
                for (int f = 0; f < NF; ++f) a.out1[f][oo] = a.U[f][oo] + dt * K[f];
            } else {
                real un[6];
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    const real av = a.A[f][oo], s = a.S[f][oo];
                    un[f] = (s + (av - (s + s)) * third) + dt6 * K[f];
                    a.out1[f][oo] = un[f];
                }
                // wave speeds of the new state (for the next step's dt and c_max)
                real rb0 = 0, eb0 = 0, bxb0 = 0, byb0 = 0;
                if (BG) { rb0 = a.BG[0][oo]; eb0 = a.BG[1][oo]; bxb0 = a.BG[2][oo]; byb0 = a.BG[3][oo]; }
                const real r0 = rb0 + un[0];
                const real ir0 = (real)1 / r0;
                const real ux = un[1] * ir0, uy = un[2] * ir0;
                const real kn = half * (un[1] * ux + un[2] * uy);
                const real bbd = bxb0 * un[4] + byb0 * un[5];
                const real b2t = un[4] * un[4] + un[5] * un[5];
                const real pkt = gm1 * (((un[3] - kn) - bbd) - half * b2t);
                const real b2b = bxb0 * bxb0 + byb0 * byb0;
                const real pkb = gm1 * (eb0 - half * b2b);
                const real pkk = pkb + pkt;
                const real bxx = bxb0 + un[4], byy = byb0 + un[5];
                const real cf = sqrt((gamma * pkk + (bxx * bxx + byy * byy)) * ir0);
                const bool fin = isfinite(un[0]) && isfinite(un[1]) && isfinite(un[2]) && isfinite(un[3]) &&
                                 isfinite(un[4]) && isfinite(un[5]) && isfinite(cf);
                if (!(r0 > (real)0) || !(pkk > (real)0) || !fin) {
                    bad_t = 1;
                } else {
                    cx_t = fmax(cx_t, (double)(fabs(ux) + cf));
                    cy_t = fmax(cy_t, (double)(fabs(uy) + cf));
                }
            }
        }

        // ================= end of row: advance the windows =================
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            dxd[0][k] = dxd[1][k]; dxd[1][k] = dxd[2][k]; dxd[2][k] = dxn[k];
            dyd[k] = (eight * (fyw[k][3] - fyw[k][1]) - (fyw[k][4] - fyw[k][0])) * i12dy;
        }
        if (BG) {
            bgv[0][0] = bgv[1][0]; bgv[1][0] = bgv[2][0]; bgv[2][0] = bgn0;
            bgv[0][1] = bgv[1][1]; bgv[1][1] = bgv[2][1]; bgv[2][1] = bgn1;
        }
        if (HD) {
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                rxd[k] = rxn[k]; d1xd[k] = d1xn[k];
                gxw[0][k] = gxw[1][k]; gxw[1][k] = gxn[k];
                hyp[k] = hyn[k];
            }
#pragma unroll
            for (int m = 0; m < 4; ++m) { fmx[0][m] = fmx[1][m]; fmx[1][m] = fmx[2][m]; fmx[2][m] = fmn[m]; }
            dvxp = dvxn;
            sw[0] = sw[1]; sw[1] = s_new;
            gyp[0] = gyn[QVX]; gyp[1] = gyn[QB];
        }
    }

    if (STAGE == 4) {
        // block reduction of the wave speeds, one atomic per block
        __shared__ double red[3][NT / 64];
        for (int off = 32; off > 0; off >>= 1) {
            cx_t = fmax(cx_t, __shfl_xor(cx_t, off));
            cy_t = fmax(cy_t, __shfl_xor(cy_t, off));
            bad_t |= __shfl_xor(bad_t, off);
        }
        const int w = tid >> 6;
        if ((tid & 63) == 0) { red[0][w] = cx_t; red[1][w] = cy_t; red[2][w] = (double)bad_t; }
        __syncthreads();
        if (tid == 0) {
            double mx_ = 0.0, my_ = 0.0, bb = 0.0;
            for (int k = 0; k < NT / 64; ++k) { mx_ = fmax(mx_, red[0][k]); my_ = fmax(my_, red[1][k]); bb = fmax(bb, red[2][k]); }
            const int nslot = sc->cur ^ 1;
            atomicMax(&sc->cacc[nslot][0], (unsigned long long)__double_as_longlong(mx_));
            atomicMax(&sc->cacc[nslot][1], (unsigned long long)__double_as_longlong(my_));
            if (bb > 0.0) atomicOr(&sc->nonphys, 1);
        }
    }
}

template <typename real, int STAGE>
static hipError_t launch_s(bool hd, bool bg, const StageArgs<real> &a, dim3 grid, hipStream_t s) {
    if (hd && bg) hipLaunchKernelGGL((k_stage<real, STAGE, true, true>), grid, dim3(NT), 0, s, a);
    else if (hd) hipLaunchKernelGGL((k_stage<real, STAGE, true, false>), grid, dim3(NT), 0, s, a);
    else if (bg) hipLaunchKernelGGL((k_stage<real, STAGE, false, true>), grid, dim3(NT), 0, s, a);
    else hipLaunchKernelGGL((k_stage<real, STAGE, false, false>), grid, dim3(NT), 0, s, a);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_stage(int stage, bool hd, bool bg, const StageArgs<real> &a, hipStream_t s) {
    dim3 grid((a.L.nx + TX - 1) / TX, (a.L.ny + a.ty - 1) / a.ty);
    switch (stage) {
        case 1: return launch_s<real, 1>(hd, bg, a, grid, s);
        case 2: return launch_s<real, 2>(hd, bg, a, grid, s);
        case 3: return launch_s<real, 3>(hd, bg, a, grid, s);
        default: return launch_s<real, 4>(hd, bg, a, grid, s);
    }
}

template hipError_t launch_stage<double>(int, bool, bool, const StageArgs<double> &, hipStream_t);
template hipError_t launch_stage<float>(int, bool, bool, const StageArgs<float> &, hipStream_t);

}  // namespace sacx
