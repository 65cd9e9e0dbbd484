// sacx_cnn.hip -- the hyper-diffusion surrogate network on gfx950 matrix cores.
//
// Network: four 3x3 convolutions with periodic padding, 6 -> 32 -> 32 -> 32 -> 10
// channels, ReLU between them, output 4 sigmoid(z) (the plain coefficient
// ratio of paper section 2 lies in [0, 4]).  Weights and activations are BF16,
// every product is accumulated in FP32 by v_mfma_f32_16x16x32_bf16.
//
// Convolution as an implicit GEMM on the matrix cores: for 16 output pixels
// of one image row and one 16-channel block of the result,
//   D[o][p] = sum_k A[o][k] B[k][p],  k = (tap, input channel),
// A = the weights (pre-packed into the exact per-lane operand order, held in
// registers for the whole kernel), B = the input pixels at the tap offsets
// (one 16-byte load per lane: 8 consecutive channels of one pixel, NHWC).
// The backward data pass is the same kernel with the transposed weights and
// negated tap offsets; the weight gradient reduces over pixels, with both
// operands transposed through LDS so that K runs over 32 pixels.  Reductions
// over pixels (weight and bias gradients, the loss) go through per-block
// partial sums and a fixed-order second pass, so results are deterministic.
//
// Memory layouts (all caller-owned device buffers):
//   input image  : BF16 NHWC, 8 channels per pixel (6 used, 2 zero)
//   activations  : BF16 NHWC, 32 channels (the outputs of layers 0, 1, 2)
//   output       : FP32 planes, [image][10][h][w]
//   error signals: BF16 NHWC, 16 channels (output layer, 10 used) or 32
//   parameters   : FP32 vector, w0 b0 w1 b1 w2 b2 w3 b3, each weight array
//                  row-major over (out channel, in channel, ky, kx)
#include <algorithm>
#include <cmath>
#include <mutex>

#include "sacx_internal.h"

namespace sacx {
namespace cnn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

constexpr int NL = 4;
__host__ __device__ constexpr int cin_of(int l) { return l == 0 ? 6 : 32; }
__host__ __device__ constexpr int cout_of(int l) { return l == 3 ? 10 : 32; }
// offsets of w_l and b_l in the parameter vector
__host__ __device__ constexpr int woff(int l) {
    return l == 0 ? 0 : woff(l - 1) + cout_of(l - 1) * cin_of(l - 1) * 9 + cout_of(l - 1);
}
__host__ __device__ constexpr int boff(int l) { return woff(l) + cout_of(l) * cin_of(l) * 9; }
constexpr int NPARAM = woff(NL);
static_assert(NPARAM == SACX_CNN_NPARAM, "parameter count");

constexpr int X0C = 8;    // input channels in memory
constexpr int AC = 32;    // hidden activation channels
constexpr int G3C = 16;   // output-layer error channels in memory

// packed operand blocks, in 16-byte vectors: [chunk][m-block][lane]
//   F0..F3: forward A = W[o][(tap, c)], B0..B2 below: backward-data
//   A = W[o][c][tap] transposed to [c][(tap, o)] (layers 3, 2, 1)
// forward chunks: ceil(9 * cin_pad / 32) = 3, 9, 9, 9 with 2, 2, 2, 1 m-blocks;
// backward-data chunks: ceil(9 * cout_pad / 32) = 9, 9, 5 (layers 1, 2, 3)
constexpr int VF0 = 0;
constexpr int VF1 = VF0 + 3 * 2 * 64;
constexpr int VF2 = VF1 + 9 * 2 * 64;
constexpr int VF3 = VF2 + 9 * 2 * 64;
constexpr int VB3 = VF3 + 9 * 1 * 64;
constexpr int VB2 = VB3 + 5 * 2 * 64;
constexpr int VB1 = VB2 + 9 * 2 * 64;
constexpr int VEND = VB1 + 9 * 2 * 64;
constexpr size_t BIAS_OFF = (size_t)VEND * 16;                // 4 x 32 FP32 biases
constexpr size_t PACKED_BYTES = BIAS_OFF + 4 * 32 * sizeof(float);
static_assert(PACKED_BYTES == SACX_CNN_PACKED_BYTES, "packed size");

// ------------------------------------------------------------- BF16 helpers
// round to nearest even (NaN stays a quiet NaN)
__device__ __forceinline__ unsigned short f2bf(float f) {
    unsigned u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }
__device__ __forceinline__ unsigned pack2(float a, float b) {
    return (unsigned)f2bf(a) | ((unsigned)f2bf(b) << 16);
}
__device__ __forceinline__ bf16x8 as_bf(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }
__device__ __forceinline__ int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// ------------------------------------------------------------- packing
__global__ void k_pack(const float *__restrict__ th, unsigned short *__restrict__ pk, float *__restrict__ bias) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;   // one BF16 element
    if (idx < 4 * 32) {
        const int l = idx / 32, o = idx % 32;
        bias[idx] = o < cout_of(l) ? th[boff(l) + o] : 0.0f;
    }
    if (idx >= VEND * 8) return;
    const int v = idx >> 3, e = idx & 7;
    int base, mbn, fwd, l;
    if (v < VF1) { base = VF0; mbn = 2; fwd = 1; l = 0; }
    else if (v < VF2) { base = VF1; mbn = 2; fwd = 1; l = 1; }
    else if (v < VF3) { base = VF2; mbn = 2; fwd = 1; l = 2; }
    else if (v < VB3) { base = VF3; mbn = 1; fwd = 1; l = 3; }
    else if (v < VB2) { base = VB3; mbn = 2; fwd = 0; l = 3; }
    else if (v < VB1) { base = VB2; mbn = 2; fwd = 0; l = 2; }
    else { base = VB1; mbn = 2; fwd = 0; l = 1; }
    const int r = v - base;
    const int lane = r & 63, mb = (r >> 6) % mbn, q = (r >> 6) / mbn;
    const int row = mb * 16 + (lane & 15);
    const int k = 32 * q + 8 * (lane >> 4) + e;
    const int ci = cin_of(l), co = cout_of(l);
    float val = 0.0f;
    if (fwd) {
        const int cp = l == 0 ? X0C : AC;
        const int t = k / cp, c = k % cp, o = row;
        if (t < 9 && c < ci && o < co) val = th[woff(l) + (o * ci + c) * 9 + t];
    } else {
        const int op = l == 3 ? G3C : AC;
        const int t = k / op, o = k % op, c = row;
        if (t < 9 && o < co && c < ci) val = th[woff(l) + (o * ci + c) * 9 + t];
    }
    pk[idx] = f2bf(val);
}

// ------------------------------------------------------------- convolution
enum { MODE_HIDDEN = 0, MODE_FINAL = 1, MODE_BWD = 2 };

struct ConvArgs {
    const u32x4 *wa;             // packed A operands [chunk][m-block][64]
    const float *bias;           // 32 biases (forward modes)
    const unsigned short *x;     // input, NHWC with CIN channels
    const unsigned short *mask;  // backward: the layer's input activation (NHWC32)
    unsigned short *y;           // hidden / backward output, NHWC32
    float *out;                  // final output planes
    int64_t out_img, out_plane, out_row;
    int n, h, w;
    int rows;                    // output rows per block
};

// Row-streamed implicit GEMM: a block of 4 waves owns a strip of kStrip
// output pixels (16 per wave) of one image over a.rows output rows.  The
// input rows its taps reach -- the strip's pixels and one more on each side,
// periodic -- pass through an LDS ring of 4 rows: each is loaded from memory
// once per strip, while the row before it is being multiplied, and every
// tap's B operand is a 16-byte LDS read.  One barrier per output row.
constexpr int kStrip = 64;

template <int CIN, int NCHUNK, int MB, int MODE>
__global__ __launch_bounds__(256) void k_conv(ConvArgs a) {
    constexpr int LW = kStrip + 2;          // pixels of an LDS row
    constexpr int VPP = CIN / 8;            // 16-byte vectors per pixel
    constexpr int NV = LW * VPP;            // vectors per LDS row
    constexpr int NLD = (NV + 255) / 256;   // row loads per thread
    constexpr int SIGN = MODE == MODE_BWD ? -1 : 1;
    // (rows padded to whole loads per thread, so that every thread stores
    // its loads unconditionally)
    __shared__ u32x4 ring[4][NLD * 256];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int kg = lane >> 4, px = lane & 15;
    const int strips = (a.w + kStrip - 1) / kStrip;
    const int groups = (a.h + a.rows - 1) / a.rows;
    int b = blockIdx.x;
    const int img = b / (strips * groups);
    b -= img * strips * groups;
    const int gy = b / strips, sx = b - gy * strips;
    const int x0 = sx * kStrip, y0 = gy * a.rows, y1 = min(y0 + a.rows, a.h);
    const int x = x0 + 16 * wv + px;         // this lane's output pixel
    const bool act = x0 + 16 * wv < a.w;     // the wave has output pixels (w is a multiple of 16)
    const int64_t ibase = (int64_t)img * a.h;

    bf16x8 A[NCHUNK][MB];
#pragma unroll
    for (int q = 0; q < NCHUNK; ++q)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) A[q][mb] = as_bf(a.wa[(q * MB + mb) * 64 + lane]);

    // this thread's share of an LDS row: vector i = threadIdx.x + 256 u is
    // part i % VPP of LDS pixel i / VPP, image column x0 - 1 + i / VPP
    // (periodic); threads past the row re-load its last vector, unused
    int64_t coff[NLD];
#pragma unroll
    for (int u = 0; u < NLD; ++u) {
        const int i = min((int)threadIdx.x + 256 * u, NV - 1);
        const int p = i / VPP;
        const int xx = ((x0 - 1 + p) % a.w + a.w) % a.w;
        coff[u] = (int64_t)xx * CIN + (i - p * VPP) * 8;
    }
    auto load_row = [&](int yy, u32x4 (&v)[NLD]) __attribute__((always_inline)) {
        const int64_t rb = (ibase + wrapi(yy, a.h)) * a.w * CIN;
#pragma unroll
        for (int u = 0; u < NLD; ++u) v[u] = *(const u32x4 *)(a.x + rb + coff[u]);
    };
    auto store_row = [&](int slot, const u32x4 (&v)[NLD]) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < NLD; ++u) ring[slot][threadIdx.x + 256 * u] = v[u];
    };
    // this lane's biases (forward modes), read once: a global read in the
    // row loop would make the wave wait for the rows in flight
    float bias[MB][4];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int o = mb * 16 + 4 * kg + e;
            bias[mb][e] = MODE == MODE_BWD || (MODE == MODE_FINAL && o >= 10) ? 0.0f : a.bias[o];
        }
    // backward: the layer-input activation of the row's pixels (the ReLU
    // mask), issued before the row loads that follow it
    auto load_mask = [&](int y, u32x2 (&m)[MB]) __attribute__((always_inline)) {
        const int64_t pix = (ibase + y) * a.w + (act ? x : 0);
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) m[mb] = *(const u32x2 *)(a.mask + pix * AC + mb * 16 + 4 * kg);
    };
    auto mul_store = [&](int y, const u32x2 (&mk)[MB]) __attribute__((always_inline)) {
        if (!act) return;
        f32x4 acc[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) acc[mb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < NCHUNK; ++q) {
            const int k0 = 32 * q + 8 * kg;
            const int t = k0 / CIN, c0 = k0 % CIN;
            u32x4 bv = u32x4{0u, 0u, 0u, 0u};
            if (t < 9) {
                const int ry = y + SIGN * (t / 3 - 1);
                const int lx = 16 * wv + px + 1 + SIGN * (t % 3 - 1);
                bv = ring[(ry - y0 + 1) & 3][lx * VPP + c0 / 8];
            }
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
                acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[q][mb], as_bf(bv), acc[mb], 0, 0, 0);
        }
        // this lane holds pixel x, channels mb*16 + 4 kg + e
        const int64_t pix = (ibase + y) * a.w + x;
        if (MODE == MODE_HIDDEN) {
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                const int o0 = mb * 16 + 4 * kg;
                float v[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] = fmaxf(acc[mb][e] + bias[mb][e], 0.0f);
                *(u32x2 *)(a.y + pix * AC + o0) = u32x2{pack2(v[0], v[1]), pack2(v[2], v[3])};
            }
        } else if (MODE == MODE_FINAL) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int o = 4 * kg + e;
                if (o < 10) {
                    const float z = acc[0][e] + bias[0][e];
                    a.out[img * a.out_img + o * a.out_plane + y * a.out_row + x] = 4.0f / (1.0f + expf(-z));
                }
            }
        } else {
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                const int c0 = mb * 16 + 4 * kg;
                const u32x2 m = mk[mb];
                const unsigned short mh[4] = {(unsigned short)(m[0] & 0xffff), (unsigned short)(m[0] >> 16),
                                              (unsigned short)(m[1] & 0xffff), (unsigned short)(m[1] >> 16)};
                float v[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] = ((short)mh[e] > 0) ? acc[mb][e] : 0.0f;
                *(u32x2 *)(a.y + pix * AC + c0) = u32x2{pack2(v[0], v[1]), pack2(v[2], v[3])};
            }
        }
    };

    // input row r lives in slot (r - y0 + 1) & 3; rows y0-1, y0, y0+1 first.
    // An output row y multiplies from the ring and stores its outputs, then
    // issues the loads of row y+3 and stores row y+2, in flight since the
    // previous output row: each row has a row of work to arrive.  The loop
    // is unrolled over the two register sets so that neither is copied while
    // its loads are in flight, and a row's loads come after the output
    // stores, so that the wait for the row before it leaves them in flight.
    // Past the strip's last row the loads re-read that row, unused.
    u32x4 ra[NLD], rb[NLD];
    {
        u32x4 v0[NLD], v1[NLD], v2[NLD];
        load_row(y0 - 1, v0);
        load_row(y0, v1);
        load_row(y0 + 1, v2);
        load_row(min(y0 + 2, y1), ra);
        store_row(0, v0);
        store_row(1, v1);
        store_row(2, v2);
    }
    __syncthreads();
    u32x2 mk[MB];
    for (int y = y0; y < y1; y += 2) {
        if (MODE == MODE_BWD) load_mask(y, mk);
        mul_store(y, mk);
        load_row(min(y + 3, y1), rb);
        // slot of row y+2 held row y-2, read by no one since the last barrier
        store_row((y + 3 - y0) & 3, ra);
        __syncthreads();
        if (y + 1 >= y1) break;
        if (MODE == MODE_BWD) load_mask(y + 1, mk);
        mul_store(y + 1, mk);
        load_row(min(y + 4, y1), ra);
        store_row((y + 4 - y0) & 3, rb);
        __syncthreads();
    }
}

// ------------------------------------------------------------- loss
// error signal of the output layer, d(mean squared error)/dz, and per-block
// partial sums of the squared error
__global__ __launch_bounds__(256) void k_loss(const float *__restrict__ out, const float *__restrict__ tgt,
                                              const float *__restrict__ wgt, int n, int h, int w, float scale,
                                              unsigned short *__restrict__ g3, double *__restrict__ part) {
    __shared__ double red[4];
    const int64_t hw = (int64_t)h * w;
    const int64_t np = (int64_t)n * hw;
    double s = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t img = p / hw, q = p - img * hw;
        float g[16];
#pragma unroll
        for (int o = 0; o < 10; ++o) {
            const int64_t i = (img * 10 + o) * hw + q;
            const float r = out[i];
            const float d = r - tgt[i];
            const float wt = wgt ? wgt[i] : 1.0f;
            s += (double)wt * ((double)d * (double)d);
            g[o] = ((scale * (wt * d)) * r) * (1.0f - r * 0.25f);
        }
#pragma unroll
        for (int o = 10; o < 16; ++o) g[o] = 0.0f;
        u32x4 *dst = (u32x4 *)(g3 + p * G3C);
        dst[0] = u32x4{pack2(g[0], g[1]), pack2(g[2], g[3]), pack2(g[4], g[5]), pack2(g[6], g[7])};
        dst[1] = u32x4{pack2(g[8], g[9]), pack2(g[10], g[11]), pack2(g[12], g[13]), pack2(g[14], g[15])};
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// fixed-order sum of the per-block loss partials: thread t sums partials
// t, t + 256, ... in order, then a fixed tree over the 256 threads (one block)
__global__ __launch_bounds__(256) void k_loss_final(const double *__restrict__ part, int nb, double inv_count,
                                                    double *__restrict__ loss) {
    __shared__ double red[256];
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) s += part[b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = red[0] * inv_count;
}

// ------------------------------------------------------------- weight gradient
struct WgradArgs {
    const unsigned short *g;   // error signal of the layer's output, NHWC (COUTP)
    const unsigned short *x;   // the layer's input, NHWC (CINP)
    float *part;               // per-block partial gradients [block][cout*cin*9 + cout]
    int n, h, w, rows;
    int cin, cout;
};

// A block owns a 32-pixel row segment of one image over `rows` rows.  Per row
// the error signal (32 px x COUTP) and the three input rows around it
// (34 px x CINP, stored as three x-shifted copies so every operand read is
// an aligned 16-byte LDS load) are transposed into LDS; the 9 taps x
// 16x16 (out, in) tiles are spread over the 4 waves.
template <int CINP, int COUTP>
__global__ __launch_bounds__(256) void k_wgrad(WgradArgs a) {
    constexpr int CN = CINP < 16 ? 16 : CINP;
    constexpr int MB = COUTP / 16, NB = CN / 16;
    constexpr int NTILE = 9 * MB * NB;
    constexpr int TPW = (NTILE + 3) / 4;
    __shared__ __align__(16) unsigned short sG[COUTP][32];
    __shared__ __align__(16) unsigned short sX[3][3][CN][32];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int nxs = a.w / 32;
    const int nyb = (a.h + a.rows - 1) / a.rows;
    const int b = blockIdx.x;
    const int img = b / (nxs * nyb);
    const int r1 = b - img * nxs * nyb;
    const int yb = r1 / nxs, xs = r1 - yb * nxs;
    const int x0 = xs * 32;
    const int y0 = yb * a.rows, y1 = min(y0 + a.rows, a.h);
    const int64_t ibase = (int64_t)img * a.h;

    if (CN > CINP) {
        for (int i = tid; i < 3 * 3 * (CN - CINP) * 32; i += 256) {
            const int p = i % 32, c = CINP + (i / 32) % (CN - CINP), s = i / (32 * (CN - CINP));
            sX[s / 3][s % 3][c][p] = 0;
        }
    }
    f32x4 acc[TPW];
#pragma unroll
    for (int i = 0; i < TPW; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    float db = 0.0f;

    for (int y = y0; y < y1; ++y) {
        __syncthreads();
        for (int v = tid; v < 32 * (COUTP / 8); v += 256) {
            const int p = v / (COUTP / 8), cg = v % (COUTP / 8);
            const u32x4 d = *(const u32x4 *)(a.g + (((ibase + y) * a.w + x0 + p) * COUTP + cg * 8));
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                sG[cg * 8 + 2 * e][p] = (unsigned short)(d[e] & 0xffff);
                sG[cg * 8 + 2 * e + 1][p] = (unsigned short)(d[e] >> 16);
            }
        }
        for (int v = tid; v < 3 * 34 * (CINP / 8); v += 256) {
            const int dyi = v / (34 * (CINP / 8));
            const int rr = v - dyi * 34 * (CINP / 8);
            const int r = rr / (CINP / 8) - 1, cg = rr % (CINP / 8);
            const int yy = wrapi(y + dyi - 1, a.h), xx = wrapi(x0 + r, a.w);
            const u32x4 d = *(const u32x4 *)(a.x + (((ibase + yy) * a.w + xx) * CINP + cg * 8));
#pragma unroll
            for (int dxi = 0; dxi < 3; ++dxi) {
                const int p = r - (dxi - 1);
                if (p >= 0 && p < 32) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        sX[dyi][dxi][cg * 8 + 2 * e][p] = (unsigned short)(d[e] & 0xffff);
                        sX[dyi][dxi][cg * 8 + 2 * e + 1][p] = (unsigned short)(d[e] >> 16);
                    }
                }
            }
        }
        __syncthreads();
        if (tid < COUTP) {
            float s = 0.0f;
            for (int p = 0; p < 32; ++p) s += bf2f(sG[tid][p]);
            db += s;
        }
#pragma unroll
        for (int i = 0; i < TPW; ++i) {
            const int tile = wv + 4 * i;
            if (tile < NTILE) {
                const int t = tile / (MB * NB), r2 = tile % (MB * NB);
                const int mb = r2 / NB, nb = r2 % NB;
                const u32x4 av = *(const u32x4 *)&sG[mb * 16 + (lane & 15)][8 * (lane >> 4)];
                const u32x4 bv = *(const u32x4 *)&sX[t / 3][t % 3][nb * 16 + (lane & 15)][8 * (lane >> 4)];
                acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(av), as_bf(bv), acc[i], 0, 0, 0);
            }
        }
    }
    const int nw = a.cout * a.cin * 9;
    float *pp = a.part + (int64_t)b * (nw + a.cout);
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
        const int tile = wv + 4 * i;
        if (tile < NTILE) {
            const int t = tile / (MB * NB), r2 = tile % (MB * NB);
            const int mb = r2 / NB, nb = r2 % NB;
            const int c = nb * 16 + (lane & 15);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int o = mb * 16 + 4 * (lane >> 4) + e;
                if (o < a.cout && c < a.cin) pp[(o * a.cin + c) * 9 + t] = acc[i][e];
            }
        }
    }
    if (tid < a.cout) pp[nw + tid] = db;
}

// fixed-order sum of the per-block partials, in two levels: group g of
// blockIdx.y sums blocks [g*chunk, min((g+1)*chunk, nblocks)) in order and
// leaves its sum in the first row of its chunk; k_reduce2 then sums the group
// sums in order.  Each column is read and written by one thread only.
__global__ void k_reduce(float *__restrict__ part, int nblocks, int np, int chunk) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int b0 = blockIdx.y * chunk;
    if (i >= np || b0 >= nblocks) return;
    const int b1 = min(b0 + chunk, nblocks);
    float s = 0.0f;
    for (int b = b0; b < b1; ++b) s += part[(int64_t)b * np + i];
    part[(int64_t)b0 * np + i] = s;
}

__global__ void k_reduce2(const float *__restrict__ part, int nblocks, int np, int chunk, float *__restrict__ dst) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    float s = 0.0f;
    for (int b0 = 0; b0 < nblocks; b0 += chunk) s += part[(int64_t)b0 * np + i];
    dst[i] = s;
}

// ------------------------------------------------------------- Adam
__global__ void k_adam(float *__restrict__ th, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * (gi * gi);
    m[i] = mi;
    v[i] = vi;
    th[i] = th[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// ------------------------------------------------------------- host side
// output rows per block: about 2048 blocks (a few per compute unit), at
// least 4 rows (each strip re-reads two apron rows)
static int conv_rows(int n, int h, int w) {
    const int64_t strips = (int64_t)n * ((w + kStrip - 1) / kStrip);
    const int64_t r = (strips * h + 2047) / 2048;
    return (int)std::min<int64_t>(h, std::max<int64_t>(4, r));
}

static hipError_t launch_conv(int layer, int mode, const unsigned char *pk, const void *x, const void *mask,
                              void *y, float *out, int64_t oimg, int64_t oplane, int64_t orow, int n, int h, int w,
                              hipStream_t s) {
    ConvArgs a;
    a.bias = (const float *)(pk + BIAS_OFF) + 32 * layer;
    a.x = (const unsigned short *)x;
    a.mask = (const unsigned short *)mask;
    a.y = (unsigned short *)y;
    a.out = out;
    a.out_img = oimg; a.out_plane = oplane; a.out_row = orow;
    a.n = n; a.h = h; a.w = w;
    a.rows = conv_rows(n, h, w);
    const int blocks = n * ((w + kStrip - 1) / kStrip) * ((h + a.rows - 1) / a.rows);
    const u32x4 *v = (const u32x4 *)pk;
    if (mode == MODE_BWD) {
        if (layer == 3) { a.wa = v + VB3; k_conv<G3C, 5, 2, MODE_BWD><<<blocks, 256, 0, s>>>(a); }
        else if (layer == 2) { a.wa = v + VB2; k_conv<AC, 9, 2, MODE_BWD><<<blocks, 256, 0, s>>>(a); }
        else { a.wa = v + VB1; k_conv<AC, 9, 2, MODE_BWD><<<blocks, 256, 0, s>>>(a); }
    } else if (layer == 0) { a.wa = v + VF0; k_conv<X0C, 3, 2, MODE_HIDDEN><<<blocks, 256, 0, s>>>(a); }
    else if (layer == 1) { a.wa = v + VF1; k_conv<AC, 9, 2, MODE_HIDDEN><<<blocks, 256, 0, s>>>(a); }
    else if (layer == 2) { a.wa = v + VF2; k_conv<AC, 9, 2, MODE_HIDDEN><<<blocks, 256, 0, s>>>(a); }
    else { a.wa = v + VF3; k_conv<AC, 9, 1, MODE_FINAL><<<blocks, 256, 0, s>>>(a); }
    return hipGetLastError();
}

static int wgrad_rows(int n, int h, int w) {
    const int64_t segs = (int64_t)n * (w / 32) * h;
    int rows = (int)std::max<int64_t>(1, (segs + 1023) / 1024);
    return std::min(rows, h);
}
static int wgrad_blocks(int n, int h, int w) {
    const int rows = wgrad_rows(n, h, w);
    return n * (w / 32) * ((h + rows - 1) / rows);
}

}  // namespace cnn

// forward pass of an n-image batch into three activation buffers (a1, a2,
// a3 may alias a1 when the activations are not kept: a1 and a2 ping-pong)
hipError_t cnn_forward_dev(const void *packed, const void *x, int n, int h, int w, void *a1, void *a2, void *a3,
                           float *out, int64_t oimg, int64_t oplane, int64_t orow, hipStream_t s) {
    using namespace cnn;
    const unsigned char *pk = (const unsigned char *)packed;
    hipError_t e;
    if ((e = launch_conv(0, MODE_HIDDEN, pk, x, nullptr, a1, nullptr, 0, 0, 0, n, h, w, s)) != hipSuccess) return e;
    if ((e = launch_conv(1, MODE_HIDDEN, pk, a1, nullptr, a2, nullptr, 0, 0, 0, n, h, w, s)) != hipSuccess) return e;
    if ((e = launch_conv(2, MODE_HIDDEN, pk, a2, nullptr, a3, nullptr, 0, 0, 0, n, h, w, s)) != hipSuccess) return e;
    return launch_conv(3, MODE_FINAL, pk, a3, nullptr, nullptr, out, oimg, oplane, orow, n, h, w, s);
}

}  // namespace sacx

using namespace sacx;
using namespace sacx::cnn;

static int cnn_shape_ok(int n, int h, int w) {
    if (n < 1 || h < 1 || w < 32 || w % 32 != 0)
        return set_error(SACX_EINVAL, "network images need n >= 1, h >= 1 and w a positive multiple of 32 "
                                      "(got n=%d h=%d w=%d)", n, h, w);
    if ((int64_t)n * h * w > ((int64_t)1 << 31) / AC)
        return set_error(SACX_EINVAL, "network batch too large (%lld pixels)", (long long)n * h * w);
    return SACX_OK;
}

extern "C" {

int sacx_cnn_pack(const float *d_theta, void *d_packed, void *stream) {
    if (!d_theta || !d_packed) return set_error(SACX_EINVAL, "NULL buffer");
    if ((uintptr_t)d_packed % 16) return set_error(SACX_EINVAL, "packed weights must be 16-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    const int n = VEND * 8;
    k_pack<<<(n + 255) / 256, 256, 0, s>>>(d_theta, (unsigned short *)d_packed,
                                           (float *)((unsigned char *)d_packed + BIAS_OFF));
    HIPCHK(hipGetLastError());
    return SACX_OK;
}

int sacx_cnn_buffer_sizes(int n, int h, int w, sacx_cnn_sizes *out) {
    if (!out) return set_error(SACX_EINVAL, "NULL output");
    int rc = cnn_shape_ok(n, h, w);
    if (rc) return rc;
    const size_t px = (size_t)n * h * w;
    out->input_bytes = px * X0C * 2;
    out->act_bytes = 3 * px * AC * 2;
    out->out_bytes = px * 10 * sizeof(float);
    const int nb = wgrad_blocks(n, h, w);
    const size_t part = (size_t)nb * (32 * 32 * 9 + 32) * sizeof(float);
    out->work_bytes = px * G3C * 2 + 2 * px * AC * 2 + part + 2048 * sizeof(double) + 256;
    return SACX_OK;
}

int sacx_cnn_forward(const void *d_packed, const void *d_x, int n, int h, int w, void *d_act, float *d_out,
                     void *stream) {
    if (!d_packed || !d_x || !d_act || !d_out) return set_error(SACX_EINVAL, "NULL buffer");
    int rc = cnn_shape_ok(n, h, w);
    if (rc) return rc;
    if (((uintptr_t)d_packed | (uintptr_t)d_x | (uintptr_t)d_act) % 16)
        return set_error(SACX_EINVAL, "network buffers must be 16-byte aligned");
    const size_t px = (size_t)n * h * w;
    unsigned char *act = (unsigned char *)d_act;
    HIPCHK(cnn_forward_dev(d_packed, d_x, n, h, w, act, act + px * AC * 2, act + 2 * px * AC * 2, d_out,
                           (int64_t)10 * h * w, (int64_t)h * w, w, (hipStream_t)stream));
    return SACX_OK;
}

}  // extern "C"

// The backward pass proper, on a scratch buffer `d_work` of at least
// sacx_cnn_buffer_sizes().work_bytes whose size the caller has checked.
// Every scratch byte it reads was written earlier in the same pass (no
// kernel accumulates into the scratch), so its previous contents never
// matter.
static int cnn_backward_on(const void *d_packed, const void *d_x, const void *d_act, const float *d_out,
                           const float *d_target, const float *d_weight, int n, int h, int w, void *d_work,
                           float *d_grad, double *d_loss, hipStream_t s) {
    const unsigned char *pk = (const unsigned char *)d_packed;
    const size_t px = (size_t)n * h * w;
    const unsigned char *act = (const unsigned char *)d_act;
    const void *A[4] = {d_x, act, act + px * AC * 2, act + 2 * px * AC * 2};
    unsigned char *wk = (unsigned char *)d_work;
    unsigned short *g3 = (unsigned short *)wk;
    unsigned short *ga = (unsigned short *)(wk + px * G3C * 2);
    unsigned short *gb = (unsigned short *)(wk + px * G3C * 2 + px * AC * 2);
    float *part = (float *)(wk + px * G3C * 2 + 2 * px * AC * 2);
    const int nbw = wgrad_blocks(n, h, w);
    double *lpart = (double *)((unsigned char *)part + (size_t)nbw * (32 * 32 * 9 + 32) * sizeof(float));

    // output layer error signal and the loss
    const double count = (double)px * 10.0;
    const int lb = (int)std::min<size_t>(2048, (px + 255) / 256);
    k_loss<<<lb, 256, 0, s>>>(d_out, d_target, d_weight, n, h, w, (float)(2.0 / count), g3, lpart);
    HIPCHK(hipGetLastError());
    k_loss_final<<<1, 256, 0, s>>>(lpart, lb, 1.0 / count, d_loss);
    HIPCHK(hipGetLastError());

    const int rows = wgrad_rows(n, h, w);
    // layers 3..0: weight gradient from (G_l, A_l), then G_{l-1} = conv^T(G_l) * [A_l > 0]
    const unsigned short *gl = g3;
    for (int l = 3; l >= 0; --l) {
        WgradArgs wa;
        wa.g = gl;
        wa.x = (const unsigned short *)A[l];
        wa.part = part;
        wa.n = n; wa.h = h; wa.w = w; wa.rows = rows;
        wa.cin = cin_of(l); wa.cout = cout_of(l);
        if (l == 3) k_wgrad<AC, G3C><<<nbw, 256, 0, s>>>(wa);
        else if (l == 0) k_wgrad<X0C, AC><<<nbw, 256, 0, s>>>(wa);
        else k_wgrad<AC, AC><<<nbw, 256, 0, s>>>(wa);
        HIPCHK(hipGetLastError());
        const int np = cout_of(l) * cin_of(l) * 9 + cout_of(l);
        {
            const int chunk = std::max(1, (nbw + 63) / 64);   // at most 64 groups
            const int groups = (nbw + chunk - 1) / chunk;
            k_reduce<<<dim3((np + 255) / 256, groups), 256, 0, s>>>(part, nbw, np, chunk);
            HIPCHK(hipGetLastError());
            k_reduce2<<<(np + 255) / 256, 256, 0, s>>>(part, nbw, np, chunk, d_grad + woff(l));
            HIPCHK(hipGetLastError());
        }
        if (l > 0) {
            unsigned short *gn = (l % 2 == 1) ? ga : gb;
            HIPCHK(launch_conv(l, MODE_BWD, pk, gl, A[l], gn, nullptr, 0, 0, 0, n, h, w, s));
            gl = gn;
        }
    }
    return SACX_OK;
}

static int cnn_backward_args(const void *d_packed, const void *d_x, const void *d_act, const float *d_out,
                             const float *d_target, const float *d_grad, const double *d_loss, int n, int h,
                             int w, sacx_cnn_sizes *sz) {
    if (!d_packed || !d_x || !d_act || !d_out || !d_target || !d_grad || !d_loss)
        return set_error(SACX_EINVAL, "NULL buffer");
    int rc = sacx_cnn_buffer_sizes(n, h, w, sz);
    if (rc) return rc;
    if (((uintptr_t)d_packed | (uintptr_t)d_x | (uintptr_t)d_act) % 16)
        return set_error(SACX_EINVAL, "network buffers must be 16-byte aligned");
    return SACX_OK;
}

// Scratch of the allocation-free backward pass: one array per device,
// reserved when the library's code object is loaded on that device and held
// until the process ends.  Host code never names it directly (in host code
// the name is only a stand-in, not a device address): the device address is
// looked up once per device with hipGetSymbolAddress and kept below.
static __device__ __align__(256) unsigned char scratch[SACX_CNN_STATIC_WORK_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

static int scratch_for_current_device(void **out) {
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return set_error(SACX_EUNSUP, "device %d beyond the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return set_error(SACX_EDEVICE, "hipGetSymbolAddress of the static network scratch failed: %s",
                             hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SACX_OK;
}

extern "C" {

int sacx_cnn_backward(const void *d_packed, const void *d_x, const void *d_act, const float *d_out,
                      const float *d_target, const float *d_weight, int n, int h, int w, void *d_work,
                      size_t work_bytes, float *d_grad, double *d_loss, void *stream) {
    sacx_cnn_sizes sz;
    int rc = cnn_backward_args(d_packed, d_x, d_act, d_out, d_target, d_grad, d_loss, n, h, w, &sz);
    if (rc) return rc;
    if (!d_work) return set_error(SACX_EINVAL, "NULL buffer");
    if (work_bytes < sz.work_bytes)
        return set_error(SACX_ENOSPC, "network work buffer too small (%zu < %zu bytes)", work_bytes, sz.work_bytes);
    if ((uintptr_t)d_work % 16) return set_error(SACX_EINVAL, "network buffers must be 16-byte aligned");
    return cnn_backward_on(d_packed, d_x, d_act, d_out, d_target, d_weight, n, h, w, d_work, d_grad, d_loss,
                           (hipStream_t)stream);
}

int sacx_cnn_backward_noalloc(const void *d_packed, const void *d_x, const void *d_act, const float *d_out,
                              const float *d_target, const float *d_weight, int n, int h, int w, float *d_grad,
                              double *d_loss, void *stream) {
    sacx_cnn_sizes sz;
    int rc = cnn_backward_args(d_packed, d_x, d_act, d_out, d_target, d_grad, d_loss, n, h, w, &sz);
    if (rc) return rc;
    if (sz.work_bytes > (size_t)SACX_CNN_STATIC_WORK_BYTES)
        return set_error(SACX_ENOSPC, "batch of %d images of %d x %d needs %zu scratch bytes, more than the %zu of "
                                      "the static scratch (use sacx_cnn_backward with a workspace)",
                         n, h, w, sz.work_bytes, (size_t)SACX_CNN_STATIC_WORK_BYTES);
    void *wk = nullptr;
    rc = scratch_for_current_device(&wk);
    if (rc) return rc;
    return cnn_backward_on(d_packed, d_x, d_act, d_out, d_target, d_weight, n, h, w, wk, d_grad, d_loss,
                           (hipStream_t)stream);
}

int sacx_cnn_adam(float *d_theta, float *d_m, float *d_v, const float *d_grad, int step, float lr, float beta1,
                  float beta2, float eps, void *stream) {
    if (!d_theta || !d_m || !d_v || !d_grad) return set_error(SACX_EINVAL, "NULL buffer");
    if (step < 1) return set_error(SACX_EINVAL, "Adam step count starts at 1 (got %d)", step);
    if (!(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(lr >= 0.f) || !(eps >= 0.f))
        return set_error(SACX_EINVAL, "invalid Adam hyper-parameters");
    const double c1 = 1.0 / (1.0 - std::pow((double)beta1, step));
    const double c2 = 1.0 / (1.0 - std::pow((double)beta2, step));
    k_adam<<<(NPARAM + 255) / 256, 256, 0, (hipStream_t)stream>>>(d_theta, d_m, d_v, d_grad, NPARAM, lr, beta1,
                                                                   beta2, eps, (float)c1, (float)c2);
    HIPCHK(hipGetLastError());
    return SACX_OK;
}

}  // extern "C"
