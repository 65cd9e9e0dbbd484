// sacx_ratio.hip -- plain coefficient-ratio fields, the surrogate check and the
// network inputs of a state (learned hyper-diffusion coefficient).
#include <algorithm>

#include "sacx_tile.h"

namespace sacx {

// ---------------------------------------------------------------------------
// Plain coefficient-ratio fields (the surrogate's training target and judge).
// The quantities are formed from the state exactly as in the stage kernel
// (same operations, same order, no background), so a ratio computed here is
// the one the plain stage would use at that face.
// ---------------------------------------------------------------------------

// quantity sets at cell (i, j): q = {rho~, eps~, v_x, v_y, B~_y, B~_x}
template <typename real>
__device__ __forceinline__ void cell_quantities(const RatioArgs<real> &a, int i, int j, real q[6]) {
    const int64_t o = (int64_t)a.L.xoff + i + (int64_t)(j + G) * a.L.pitch;
    const real gm1 = (real)a.gm1, igm1 = (real)a.igm1, half = (real)0.5;
    const real rb = 0, bxb = 0, byb = 0;
    const real rt = a.S[0][o], mx = a.S[1][o], my = a.S[2][o], et = a.S[3][o], bxt = a.S[4][o], byt = a.S[5][o];
    const real rho = rb + rt;
    const real irho = (real)1 / rho;
    const real vx = mx * irho, vy = my * irho;
    const real kin = half * (mx * vx + my * vy);
    const real bbdot = bxb * bxt + byb * byt;
    const real bt2 = bxt * bxt + byt * byt;
    const real pk = gm1 * (((et - kin) - bbdot) - half * bt2);
    q[0] = rt; q[1] = pk * igm1; q[2] = vx; q[3] = vy; q[4] = byt; q[5] = bxt;
}

// the ten plain ratios of the faces above cell (i, j): R[k] x-face set k,
// R[5 + k] y-face set k; D1 (optional) the first differences at those faces
template <typename real>
__device__ __forceinline__ void cell_ratios(const RatioArgs<real> &a, int i, int j, real R[10], real *D1 = nullptr) {
    real qx[6][6], qy[6][6];   // [offset -2..3][quantity]
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        cell_quantities(a, i - 2 + m, j, qx[m]);
        if (m == 2) {
#pragma unroll
            for (int k = 0; k < 6; ++k) qy[m][k] = qx[m][k];
        } else {
            cell_quantities(a, i, j - 2 + m, qy[m]);
        }
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const int kx = k == 4 ? 4 : k, ky = k == 4 ? 5 : k;   // B~_y on x faces, B~_x on y faces
        R[k] = hd_ratio(qx[0][kx], qx[1][kx], qx[2][kx], qx[3][kx], qx[4][kx], qx[5][kx]);
        R[5 + k] = hd_ratio(qy[0][ky], qy[1][ky], qy[2][ky], qy[3][ky], qy[4][ky], qy[5][ky]);
        if (D1) {
            D1[k] = qx[3][kx] - qx[2][kx];
            D1[5 + k] = qy[3][ky] - qy[2][ky];
        }
    }
}

// first differences of the ten sets at the faces above cell (i, j)
template <typename real>
__device__ __forceinline__ void cell_d1(const RatioArgs<real> &a, int i, int j, real D1[10]) {
    real q0[6], qx[6], qy[6];
    cell_quantities(a, i, j, q0);
    cell_quantities(a, i + 1, j, qx);
    cell_quantities(a, i, j + 1, qy);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const int kx = k == 4 ? 4 : k, ky = k == 4 ? 5 : k;
        D1[k] = qx[kx] - q0[kx];
        D1[5 + k] = qy[ky] - q0[ky];
    }
}

template <typename real>
__global__ __launch_bounds__(256) void k_ratio_fields(RatioArgs<real> a, float *out, float *d1, int64_t pitch) {
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= a.L.nx || j >= a.L.ny) return;
    real R[10], D[10];
    cell_ratios(a, i, j, R, D);
    const int64_t plane = pitch * a.L.ny;
#pragma unroll
    for (int k = 0; k < 10; ++k) out[k * plane + (int64_t)j * pitch + i] = (float)R[k];
    if (d1) {
#pragma unroll
        for (int k = 0; k < 10; ++k) d1[k * plane + (int64_t)j * pitch + i] = (float)D[k];
    }
}

template <typename real>
hipError_t launch_ratio_fields(const RatioArgs<real> &a, float *out, float *d1, int64_t pitch, hipStream_t s) {
    dim3 grid((a.L.nx + 63) / 64, (a.L.ny + 3) / 4);
    hipLaunchKernelGGL(k_ratio_fields<real>, grid, dim3(256), 0, s, a, out, d1, pitch);
    return hipGetLastError();
}

// per-plane largest |first difference| over the domain (flux metric scale)
__global__ void k_check_reset(HdDevStats *st) {
    if (threadIdx.x < 10) st->dmax[threadIdx.x] = 0ull;
}

template <typename real>
__global__ __launch_bounds__(256) void k_d1_max(RatioArgs<real> a, HdDevStats *st) {
    __shared__ double red[4][10];
    double m[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) m[k] = 0.0;
    const int64_t n = (int64_t)a.L.nx * a.L.ny;
    for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < n; c += (int64_t)gridDim.x * 256) {
        const int j = (int)(c / a.L.nx), i = (int)(c - (int64_t)j * a.L.nx);
        real D[10];
        cell_d1(a, i, j, D);
#pragma unroll
        for (int k = 0; k < 10; ++k) m[k] = fmax(m[k], (double)fabs(D[k]));
    }
#pragma unroll
    for (int k = 0; k < 10; ++k)
        for (int off = 32; off > 0; off >>= 1) m[k] = fmax(m[k], __shfl_xor(m[k], off));
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < 10; ++k) red[threadIdx.x >> 6][k] = m[k];
    }
    __syncthreads();
    if (threadIdx.x < 10) {
        const int k = threadIdx.x;
        const double v = fmax(fmax(red[0][k], red[1][k]), fmax(red[2][k], red[3][k]));
        const unsigned long long vb = (unsigned long long)__double_as_longlong(v);
        if (vb > __hip_atomic_load(&st->dmax[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax(&st->dmax[k], vb);
    }
}

// The surrogate check: one block per tile x tile cells.  Each ratio-plane
// value r gets an error e = |r - R_plain| (METRIC 0) or the flux-weighted
// e = |r - R_plain| |d1| / D (METRIC 1; d1 the face's first difference, D the
// plane's largest |d1| over the domain, e = 0 when D = 0).  A tile falls
// back when any value is not finite or has NOT(e <= bound); then the whole
// tile of every plane is set to -1 (plain ratio).  kept[tile] records the
// outcome (1 kept, 0 fell back) for the stage kernels, which read no plane
// of a fallen-back tile.  Arithmetic in the working precision.
//
// The tile is worked in sub-tiles of at most 256 cells (kCheckW x kCheckH
// for the tile's side): the quantity sets of the sub-tile's cells and of
// the apron its faces reach (two cells before, three after, in each
// direction) are formed once into LDS, then each thread takes one cell's
// ten faces from there.  The values are those of cell_ratios.
__host__ __device__ constexpr int check_sub_w(int tile) { return tile < 64 ? tile : 64; }
__host__ __device__ constexpr int check_sub_h(int tile) {
    return (256 / check_sub_w(tile)) < tile ? (256 / check_sub_w(tile)) : tile;
}
// largest (w + 5) (h + 5) over every tile side (reached from side 64 on)
constexpr int kCheckLds = 69 * 9;

template <typename real, int METRIC>
__global__ __launch_bounds__(256) void k_hd_check(RatioArgs<real> a, float *rs, int64_t pitch, double bound,
                                                  int tile, HdDevStats *st, unsigned char *kept) {
    __shared__ real sq[6][kCheckLds];
    __shared__ double s_err[4];
    __shared__ int s_bad[4];
    const int ntx = (a.L.nx + tile - 1) / tile;
    const int tx = blockIdx.x % ntx, ty = blockIdx.x / ntx;
    const int i0 = tx * tile, j0 = ty * tile;
    const int wx = min(tile, a.L.nx - i0), wy = min(tile, a.L.ny - j0);
    const int SW = check_sub_w(tile), SH = check_sub_h(tile);
    const int LW = SW + 5;
    const int64_t plane = pitch * a.L.ny;
    const real b = (real)bound;
    real dm[10];
    if (METRIC == 1) {
#pragma unroll
        for (int k = 0; k < 10; ++k) dm[k] = (real)__longlong_as_double((long long)st->dmax[k]);
    }
    double emax = 0.0;
    int bad = 0;
    for (int sj = 0; sj < wy; sj += SH) {
        for (int si = 0; si < wx; si += SW) {
            const int bi = i0 + si, bj = j0 + sj;               // sub-tile origin
            const int cw = min(SW, wx - si), ch = min(SH, wy - sj);
            const bool own = (int)threadIdx.x < cw * ch;
            const int li = own ? threadIdx.x % cw : 0, lj = own ? threadIdx.x / cw : 0;
            const int i = bi + li, j = bj + lj;
            // this thread's plane values, issued before the quantity loads so
            // that the two groups of loads are in flight together
            float rv[10];
#pragma unroll
            for (int k = 0; k < 10; ++k) rv[k] = own ? rs[k * plane + (int64_t)j * pitch + i] : 0.0f;
            __syncthreads();   // the previous sub-tile's reads are done
            // quantity sets of the cells the faces use: the sub-tile's rows
            // with the x apron, its columns with the y apron (LDS cell (ci, cj)
            // is cell (bi - 2 + ci, bj - 2 + cj)); at most three per thread,
            // their loads issued together
            const int nc = LW * (ch + 5);
#pragma unroll
            for (int u = 0; u < (kCheckLds + 255) / 256; ++u) {
                const int c = (int)threadIdx.x + 256 * u;
                const int ci = c % LW, cj = c / LW;
                const bool need = c < nc && ((cj >= 2 && cj < 2 + ch && ci < cw + 5) || (ci >= 2 && ci < 2 + cw));
                if (need) {
                    real q[6];
                    cell_quantities(a, bi - 2 + ci, bj - 2 + cj, q);
#pragma unroll
                    for (int k = 0; k < 6; ++k) sq[k][c] = q[k];
                }
            }
            __syncthreads();
            if (own) {
                const int cx = (lj + 2) * LW + li;   // x faces: row lj + 2, columns li .. li + 5
                const int cy = lj * LW + li + 2;     // y faces: column li + 2, rows lj .. lj + 5
#pragma unroll
                for (int k = 0; k < 10; ++k) {
                    // B~_y on x faces, B~_x on y faces
                    const int kq = k < 5 ? k : (k == 9 ? 5 : k - 5);
                    const real *p = sq[kq] + (k < 5 ? cx : cy);
                    const int st_ = k < 5 ? 1 : LW;
                    const real R = hd_ratio(p[0], p[st_], p[2 * st_], p[3 * st_], p[4 * st_], p[5 * st_]);
                    real e = fabs((real)rv[k] - R);
                    if (METRIC == 1) {
                        const real D = p[3 * st_] - p[2 * st_];
                        e = dm[k] > (real)0 ? (e * fabs(D)) / dm[k] : (real)0;
                    }
                    if (!isfinite(rv[k]) || !(e <= b)) bad = 1;
                    if (isfinite(e)) emax = fmax(emax, (double)e);
                }
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        emax = fmax(emax, __shfl_xor(emax, off));
        bad |= __shfl_xor(bad, off);
    }
    if ((threadIdx.x & 63) == 0) { s_err[threadIdx.x >> 6] = emax; s_bad[threadIdx.x >> 6] = bad; }
    __syncthreads();
    const double et = fmax(fmax(s_err[0], s_err[1]), fmax(s_err[2], s_err[3]));
    const int bt = s_bad[0] | s_bad[1] | s_bad[2] | s_bad[3];
    if (threadIdx.x == 0) {
        kept[blockIdx.x] = bt ? 0 : 1;
        // this block's copy of the counters; a maximum is only sent when it
        // may raise the copy (the atomic decides)
        const int sl = blockIdx.x & (kStatSlots - 1);
        const unsigned long long eb = (unsigned long long)__double_as_longlong(et);
        if (eb > __hip_atomic_load(&st->err_all[sl], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax(&st->err_all[sl], eb);
        if (bt) atomicAdd(&st->tiles_fallback[sl], 1ull);
        else if (eb > __hip_atomic_load(&st->err_used[sl], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax(&st->err_used[sl], eb);
    }
    if (bt) {
        for (int c = threadIdx.x; c < wx * wy; c += 256) {
            const int i = i0 + c % wx, j = j0 + c / wx;
#pragma unroll
            for (int k = 0; k < 10; ++k) rs[k * plane + (int64_t)j * pitch + i] = -1.0f;
        }
    }
}

template <typename real>
hipError_t launch_hd_check(const RatioArgs<real> &a, float *rs, int64_t pitch, double bound, int tile, int metric,
                           HdDevStats *st, unsigned char *kept, hipStream_t s) {
    const int ntx = (a.L.nx + tile - 1) / tile, nty = (a.L.ny + tile - 1) / tile;
    if (metric == 1) {
        hipLaunchKernelGGL(k_check_reset, dim3(1), dim3(64), 0, s, st);
        const int64_t n = (int64_t)a.L.nx * a.L.ny;
        const int blocks = (int)std::min<int64_t>((n + 255) / 256, 2048);
        hipLaunchKernelGGL(k_d1_max<real>, dim3(blocks), dim3(256), 0, s, a, st);
        hipLaunchKernelGGL((k_hd_check<real, 1>), dim3(ntx * nty), dim3(256), 0, s, a, rs, pitch, bound, tile, st, kept);
    } else {
        hipLaunchKernelGGL((k_hd_check<real, 0>), dim3(ntx * nty), dim3(256), 0, s, a, rs, pitch, bound, tile, st, kept);
    }
    return hipGetLastError();
}

// Network input of a state: (rho, v_x, v_y, B_x, B_y, e) per cell, then
// (f - shift) * scale in FP32, rounded to BF16; 8 values per pixel (two zero).
template <typename real>
__global__ __launch_bounds__(256) void k_cnn_inputs(RatioArgs<real> a, InputNorm nm, unsigned short *x) {
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int j = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= a.L.nx || j >= a.L.ny) return;
    const int64_t o = (int64_t)a.L.xoff + i + (int64_t)(j + G) * a.L.pitch;
    const real rt = a.S[0][o];
    const real irho = (real)1 / rt;
    const float f[6] = {(float)rt, (float)(a.S[1][o] * irho), (float)(a.S[2][o] * irho), (float)a.S[4][o],
                        (float)a.S[5][o], (float)a.S[3][o]};
    unsigned short h[8];
#pragma unroll
    for (int k = 0; k < 6; ++k) h[k] = bf16_rne((f[k] - nm.v[k]) * nm.v[6 + k]);
    h[6] = h[7] = 0;
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    *(u32x4 *)(x + ((int64_t)j * a.L.nx + i) * 8) =
        u32x4{h[0] | ((unsigned)h[1] << 16), h[2] | ((unsigned)h[3] << 16), h[4] | ((unsigned)h[5] << 16), 0u};
}

template <typename real>
hipError_t launch_cnn_inputs(const RatioArgs<real> &a, const InputNorm &norm, void *x, hipStream_t s) {
    dim3 grid((a.L.nx + 63) / 64, (a.L.ny + 3) / 4);
    hipLaunchKernelGGL(k_cnn_inputs<real>, grid, dim3(256), 0, s, a, norm, (unsigned short *)x);
    return hipGetLastError();
}

template hipError_t launch_ratio_fields<double>(const RatioArgs<double> &, float *, float *, int64_t, hipStream_t);
template hipError_t launch_ratio_fields<float>(const RatioArgs<float> &, float *, float *, int64_t, hipStream_t);
template hipError_t launch_hd_check<double>(const RatioArgs<double> &, float *, int64_t, double, int, int,
                                            HdDevStats *, unsigned char *, hipStream_t);
template hipError_t launch_hd_check<float>(const RatioArgs<float> &, float *, int64_t, double, int, int,
                                           HdDevStats *, unsigned char *, hipStream_t);
template hipError_t launch_cnn_inputs<double>(const RatioArgs<double> &, const InputNorm &, void *, hipStream_t);
template hipError_t launch_cnn_inputs<float>(const RatioArgs<float> &, const InputNorm &, void *, hipStream_t);


}  // namespace sacx
