// bf_lfilter.hip -- learned current filter on the gfx950 matrix cores.
//
// The filter is three 5x5 convolutions with channels 1 -> 16 -> 16 -> 1, identity activations
// and no bias, shared by J_x, J_y and J_z.  It is linear and shift-invariant, so like the
// bilinear filter of Sec. 4.1 it commutes with the discrete divergence and keeps Gauss's law;
// its 13x13 footprint contains the 11x11 separable kernel of 4 bilinear passes + compensation,
// which it represents exactly (factors (1,4,6,4,1)/16, (1,4,6,4,1)/16 and (-1,3,-1) per axis).
//
// Precision: weights are BF16; every layer input x is split into hi = bf16(x) and
// lo = bf16(x - hi), both multiplied by the BF16 weights, accumulated in FP32, so the products
// keep ~16 significant bits of the input (BF16 rounding of the input alone would not be
// linear).  Each layer is an implicit GEMM on v_mfma_f32_16x16x32_bf16:
//   M = 16 consecutive output pixels of a row, N = 16 output channels (1-channel outputs pad N),
//   K = 25 taps x C_in x {hi, lo}, ordered k = t (2 C_in) + part C_in + ci.
// Operand layouts of the 16x16x32 BF16 MFMA (64 lanes, l = 16 g + i):
//   A (16x32): lane holds row i, k = 8g .. 8g+7;  B (32x16): lane holds column i, k = 8g .. 8g+7;
//   D (16x16 FP32): lane holds column i, rows 4g .. 4g+3.
//
// Training: backward-data is the same convolution with the adjoint weights
// W'(t, a, b) = W(24 - t, b, a); the weight gradient dW(t, ci, co) = sum_p in(p + o_t, ci)
// g(p, co) is an MFMA GEMM over pixels (hi/lo products hi*hi + hi*lo + lo*hi); Adam (Kingma &
// Ba 2015) updates the FP32 master weights.
#include "bf_lfilter.h"
#include <algorithm>

namespace bf {
namespace lf {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));

constexpr int LTX = 64, LTY = 4;   // output tile: 4 rows of 64 pixels, one row per wave
constexpr int LHX = LTX + 4, LHY = LTY + 4;   // staged input tile with the 2-pixel halo

__device__ __forceinline__ unsigned short bf16_rne(float x)
{
    unsigned u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest even (finite inputs)
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_val(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

__device__ __forceinline__ f32x4 mfma(us8 a, us8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

__device__ __forceinline__ long vaddr(const View& v, int img, int y, int x)
{
    int r = y + v.zoff;
    if (r >= v.rows) r -= v.rows;
    return (long)img * v.istride + (long)r * v.rstride + (long)x * v.ch;
}

// domain coordinate after the boundary rule: wrap on periodic axes, -1 outside otherwise
__device__ __forceinline__ int dwrap(int i, int n, int per)
{
    if (per) { i %= n; return i < 0 ? i + n : i; }
    return (i < 0 || i >= n) ? -1 : i;
}

// stage the input tile (halo 2) as [pixel][hi c0..c(C-1)][lo c0..c(C-1)]
template <int CIN>
__device__ __forceinline__ void stage_input(const View& in, const Domain& d, int img, int x0, int y0,
                                            unsigned short* tile)
{
    for (int q = threadIdx.x; q < LHY * LHX * CIN; q += blockDim.x) {
        const int ci = q % CIN, pix = q / CIN;
        const int x = dwrap(x0 - 2 + pix % LHX, d.nx, d.perx);
        const int y = dwrap(y0 - 2 + pix / LHX, d.ny, d.pery);
        const float v = (x >= 0 && y >= 0) ? in.p[vaddr(in, img, y, x) + ci] : 0.f;
        const unsigned short hi = bf16_rne(v);
        tile[pix * 2 * CIN + ci] = hi;
        tile[pix * 2 * CIN + CIN + ci] = bf16_rne(v - bf16_val(hi));
    }
}

// one convolution layer: out(p, co) = sum_{t, ci} W(t, ci, co) in(p + o_t, ci) on the
// domain, zero padding (or wrap) outside.  wpk holds the packed B fragments (nq x 64 lanes).
template <int CIN, int COUT>
__global__ void __launch_bounds__(256) k_lf_conv(View in, View out, Domain d, const us8* __restrict__ wpk)
{
    constexpr int NQ = (TAPS * CIN * 2 + 31) / 32;
    __shared__ __attribute__((aligned(16))) unsigned short tile[LHY * LHX * 2 * CIN];
    const int img = blockIdx.z, x0 = blockIdx.x * LTX, y0 = blockIdx.y * LTY;
    stage_input<CIN>(in, d, img, x0, y0, tile);
    __syncthreads();
    const int ty = threadIdx.x >> 6, lane = threadIdx.x & 63, i = lane & 15, g = lane >> 4;
    f32x4 acc[LTX / 16];
#pragma unroll
    for (int m = 0; m < LTX / 16; m++) acc[m] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int q = 0; q < NQ; q++) {
        const us8 b = wpk[q * 64 + lane];
#pragma unroll
        for (int m = 0; m < LTX / 16; m++) {
            const int px = m * 16 + i;
            us8 a;
            if constexpr (CIN == 16) {
                const int pix = (ty + q / 5) * LHX + px + q % 5;   // tap q: offset (q/5-2, q%5-2)
                a = *reinterpret_cast<const us8*>(&tile[pix * 32 + g * 8]);
            } else {
#pragma unroll
                for (int j = 0; j < 8; j += 2) {
                    const int t = 16 * q + 4 * g + j / 2;
                    unsigned short h = 0, l = 0;
                    if (t < TAPS) {
                        const int pix = (ty + t / 5) * LHX + px + t % 5;
                        h = tile[pix * 2];
                        l = tile[pix * 2 + 1];
                    }
                    a[j] = h;
                    a[j + 1] = l;
                }
            }
            acc[m] = mfma(a, b, acc[m]);
        }
    }
    const int y = y0 + ty;
    if (y < d.ny && i < COUT) {
#pragma unroll
        for (int m = 0; m < LTX / 16; m++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int x = x0 + m * 16 + 4 * g + r;
                if (x < d.nx) out.p[vaddr(out, img, y, x) + i] = acc[m][r];
            }
    }
}

// packed B fragments of a layer (or of its adjoint), one block per K chunk, 64 threads
__global__ void k_lf_pack(const float* __restrict__ w, int cin, int cout, int adjoint, us8* wpk)
{
    const int q = blockIdx.x, lane = threadIdx.x, n = lane & 15, g = lane >> 4;
    const int ci_n = adjoint ? cout : cin, co_n = adjoint ? cin : cout;
    us8 v;
#pragma unroll
    for (int j = 0; j < 8; j++) {
        const int k = 32 * q + 8 * g + j;
        const int t = k / (2 * ci_n), c = (k % (2 * ci_n)) % ci_n;
        float x = 0.f;
        if (t < TAPS && n < co_n)
            x = adjoint ? w[((TAPS - 1 - t) * cin + n) * cout + c] : w[(t * cin + c) * cout + n];
        v[j] = bf16_rne(x);
    }
    wpk[q * 64 + lane] = v;
}

// weight gradient of one layer: dw(t, ci, co) += sum over the tile's pixels of
// in(p + o_t, ci) g(p, co); rows (t, ci) in M tiles of 16, pixels in K chunks of 32
template <int CIN, int COUT>
__global__ void __launch_bounds__(256) k_lf_wgrad(View in, View gout, Domain d, float* dw)
{
    constexpr int MR = TAPS * CIN, NMT = (MR + 15) / 16;
    __shared__ __attribute__((aligned(16))) unsigned short tin[LHY * LHX * 2 * CIN];
    __shared__ __attribute__((aligned(16))) unsigned short tg[LTY * LTX * 32];   // [p][hi 16][lo 16]
    const int img = blockIdx.z, x0 = blockIdx.x * LTX, y0 = blockIdx.y * LTY;
    stage_input<CIN>(in, d, img, x0, y0, tin);
    for (int q = threadIdx.x; q < LTY * LTX * 16; q += blockDim.x) {
        const int c = q % 16, p = q / 16;
        const int x = x0 + p % LTX, y = y0 + p / LTX;
        float v = 0.f;
        if (c < COUT && x < d.nx && y < d.ny) v = gout.p[vaddr(gout, img, y, x) + c];
        const unsigned short hi = bf16_rne(v);
        tg[p * 32 + c] = hi;
        tg[p * 32 + 16 + c] = bf16_rne(v - bf16_val(hi));
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, i = lane & 15, g = lane >> 4;
    for (int mt = wave; mt < NMT; mt += 4) {
        const int r = mt * 16 + i;
        const bool rowok = r < MR;
        const int t = rowok ? r / CIN : 0, ci = rowok ? r % CIN : 0;
        f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int kc = 0; kc < LTY * LTX / 32; kc++) {
            us8 ahi, alo, bhi, blo;
#pragma unroll
            for (int j = 0; j < 8; j++) {
                const int p = kc * 32 + 8 * g + j;
                const int pix = (p / LTX + t / 5) * LHX + p % LTX + t % 5;
                ahi[j] = rowok ? tin[pix * 2 * CIN + ci] : (unsigned short)0;
                alo[j] = rowok ? tin[pix * 2 * CIN + CIN + ci] : (unsigned short)0;
                bhi[j] = tg[p * 32 + i];
                blo[j] = tg[p * 32 + 16 + i];
            }
            acc = mfma(ahi, bhi, acc);
            acc = mfma(ahi, blo, acc);
            acc = mfma(alo, bhi, acc);
        }
        if (i < COUT) {
#pragma unroll
            for (int rr = 0; rr < 4; rr++) {
                const int row = mt * 16 + 4 * g + rr;
                if (row < MR) atomicAdd(&dw[row * COUT + i], acc[rr]);
            }
        }
    }
}

// mean squared error over the pixels at least `margin` from the image edges:
// loss += sum (out - target)^2 / count, g = 2 (out - target) / count there, 0 elsewhere
__global__ void __launch_bounds__(256) k_lf_loss(const float* __restrict__ out,
                                                 const float* __restrict__ target, float* g, Domain d,
                                                 int margin, double inv_count, double* loss)
{
    __shared__ double red[4];
    const long n = (long)d.nimg * d.ny * d.nx;
    double s = 0.0;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) {
        const int x = (int)(q % d.nx), y = (int)((q / d.nx) % d.ny);
        const bool in = x >= margin && x < d.nx - margin && y >= margin && y < d.ny - margin;
        const double e = in ? (double)out[q] - (double)target[q] : 0.0;
        s += e * e;
        g[q] = (float)(2.0 * e * inv_count);
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(loss, (red[0] + red[1] + red[2] + red[3]) * inv_count);
}

// Adam on the FP32 master weights; c1 = 1/(1 - beta1^t), c2 = 1/(1 - beta2^t)
__global__ void k_lf_adam(float* w, float* m, float* v, const float* g, int n, float lr, float b1,
                          float b2, float eps, float c1, float c2)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const float gq = g[q];
    const float mq = b1 * m[q] + (1.f - b1) * gq;
    const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    w[q] -= lr * (mq * c1) / (sqrtf(vq * c2) + eps);
}

__global__ void k_lf_zero(float* p, int n)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) p[q] = 0.f;
}

// ---- streamed forward pass (inference) ---------------------------------------------------
// A workgroup walks down a strip of SOW output columns, one row per step, with all three
// layers in flight: at step s layer 1 produces h1 row s+1, layer 2 consumes h1 row s and
// completes h2 row s-2, layer 3 consumes h2 row s-3 and completes output row s-5.  Each layer
// reads its source one row at a time from small LDS rings (the input 8 rows, h1 and h2 two):
//  * layer 2 (16 -> 16) keeps five accumulator tiles for the h2 rows s-2 .. s+2, so one A
//    fragment of h1 row s (16 pixels x 16 channels, tap dx) feeds five MFMAs (taps dy = 0..4);
//    its 25 B fragments stay in registers;
//  * layer 3 (16 -> 1) puts the tap row dy in the MFMA's N dimension: column dy of the
//    accumulator holds the partial sum of output row r + 2 - dy after h2 row r; shifting the
//    columns by one lane (DPP row_shr) before each row moves every partial to its next dy, and
//    column 4 leaves complete;
//  * layer 1 (1 -> 16) gathers its 25 taps x {hi, lo} from the input ring (two MFMAs).
// Layers 1 and 2 take the weights as the MFMA's A operand and the pixels as B, so that a lane
// ends with four consecutive channels of one pixel: their hi and lo BF16 parts are converted in
// hardware and stored as two 8-byte words.  The input ring keeps every row twice (rows r and
// r + SIR of a 2 SIR-row buffer), so the five rows a layer-1 tap set reads are contiguous.
// Out-of-domain h1 and h2 pixels on non-periodic axes are written as zeros, as the separate
// layers read them.  Four waves: wave w computes h1 strip w, h2 strip w and output strip w,
// strips of 16 columns; the last four columns of h1 and h2 are zero padding that only feeds
// columns beyond the workgroup's outputs.
constexpr int SOW = 56;              // output columns per workgroup: [x0, x0 + 56)
constexpr int SH1W = 68;             // h1 columns [x0 - 4, x0 + 64): 64 computed, 4 of padding
constexpr int SH2W = 68;             // h2 columns [x0 - 2, x0 + 66): 64 computed, 4 of padding
constexpr int SIW = 68;              // input columns: [x0 - 6, x0 + 62)
constexpr int SIR = 8;               // input ring rows

// one image plane per blockIdx.z % n (up to 3: the current components), images blockIdx.z / n
struct Planes {
    View in[3], out[3];
    Domain d[3];
    int n, oh;                      // planes, output rows per workgroup
};

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// hi and lo BF16 parts (round to nearest even, in hardware) of four consecutive channels of one
// pixel, stored as two 8-byte words: hi at channel offset 4g, lo at 16 + 4g
__device__ __forceinline__ unsigned pk_bf16(float a, float b)
{
    const bf16x2 p = {(__bf16)a, (__bf16)b};
    return __builtin_bit_cast(unsigned, p);
}

// A row of h1 or h2 in LDS is four planes of W pixels x 8 BF16 words: the 32 words of a pixel
// (hi parts of channels 0-7, 8-15, then lo parts of 0-7, 8-15) split into 16-byte chunks by k, so
// the 16 lanes that read one k chunk of a fragment (consecutive pixels) touch 256 consecutive
// bytes.  Channels 4g .. 4g + 3 of pixel c go to chunk g / 2 (hi) and 2 + g / 2 (lo), half g % 2.
__device__ __forceinline__ void store_ch4(unsigned short* row, int W, int c, int g, f32x4 v)
{
    const unsigned h01 = pk_bf16(v[0], v[1]), h23 = pk_bf16(v[2], v[3]);
    const unsigned l01 = pk_bf16(v[0] - __uint_as_float(h01 << 16), v[1] - __uint_as_float(h01 & 0xffff0000u));
    const unsigned l23 = pk_bf16(v[2] - __uint_as_float(h23 << 16), v[3] - __uint_as_float(h23 & 0xffff0000u));
    unsigned short* p = row + ((g >> 1) * W + c) * 8 + 4 * (g & 1);
    *reinterpret_cast<uint2*>(p) = make_uint2(h01, h23);
    *reinterpret_cast<uint2*>(p + 2 * W * 8) = make_uint2(l01, l23);
}

// hi | lo << 16 of one value
__device__ __forceinline__ unsigned hilo(float v)
{
    const unsigned h = pk_bf16(v, 0.f) & 0xffffu;
    return h | (pk_bf16(v - __uint_as_float(h << 16), 0.f) << 16);
}

__device__ __forceinline__ f32x4 shift_columns(f32x4 t)
{
    // lane i of each 16-lane row takes lane i - 1; lane 0 takes 0 (row_shr:1, bound_ctrl)
    f32x4 r;
#pragma unroll
    for (int k = 0; k < 4; k++)
        r[k] = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(t[k]), 0x111, 0xf, 0xf, true));
    return r;
}

__global__ void __launch_bounds__(256) k_lf_stream(Planes P, const us8* __restrict__ w1, const us8* __restrict__ w2,
                                                   const us8* __restrict__ w3)
{
    __shared__ unsigned sin[2 * SIR * SIW];                               // hi | lo << 16
    __shared__ __attribute__((aligned(16))) unsigned short sh1[2 * SH1W * 32];   // [row][k chunk][col][8]
    __shared__ __attribute__((aligned(16))) unsigned short sh2[2 * SH2W * 32];
    const int pl = blockIdx.z % P.n, img = blockIdx.z / P.n;
    const View in = P.in[pl], out = P.out[pl];
    const Domain d = P.d[pl];
    const int x0 = blockIdx.x * SOW, y0 = blockIdx.y * P.oh;
    if (x0 >= d.nx || y0 >= d.ny || img >= d.nimg) return;
    const int yend = min(y0 + P.oh, d.ny);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, i = lane & 15, g = lane >> 4;

    for (int q = threadIdx.x; q < SH1W * 32; q += 256) reinterpret_cast<unsigned*>(sh1)[q] = 0u;
    for (int q = threadIdx.x; q < SH2W * 32; q += 256) reinterpret_cast<unsigned*>(sh2)[q] = 0u;
    us8 b1[2], b2[TAPS], b3[5];
#pragma unroll
    for (int q = 0; q < 2; q++) b1[q] = w1[q * 64 + lane];
#pragma unroll
    for (int t = 0; t < TAPS; t++) b2[t] = w2[t * 64 + lane];
#pragma unroll
    for (int dx = 0; dx < 5; dx++) b3[dx] = i < 5 ? w3[(5 * i + dx) * 64 + 16 * g] : us8{0, 0, 0, 0, 0, 0, 0, 0};

    // this thread's column of input row r (wrapped or zero outside the domain)
    const int xin = threadIdx.x < SIW ? dwrap(x0 - 6 + (int)threadIdx.x, d.nx, d.perx) : -1;
    auto load_in = [&](int r) -> float {
        const int y = dwrap(r, d.ny, d.pery);
        return (xin >= 0 && y >= 0) ? in.p[vaddr(in, img, y, xin)] : 0.f;
    };
    auto put_in = [&](int r, float v) {
        if (threadIdx.x < SIW) {
            const unsigned h = hilo(v);
            sin[(r & (SIR - 1)) * SIW + threadIdx.x] = h;
            sin[((r & (SIR - 1)) + SIR) * SIW + threadIdx.x] = h;
        }
    };
    // layer 1's taps t = 16 q + 4 g + jj of this lane: offset from the first of its five input
    // rows, and whether the tap exists (t < 25; the weights of the padding are zero)
    int toff[2][4];
    bool tok[2][4];
#pragma unroll
    for (int q = 0; q < 2; q++)
#pragma unroll
        for (int jj = 0; jj < 4; jj++) {
            const int t = 16 * q + 4 * g + jj;
            tok[q][jj] = t < TAPS;
            toff[q][jj] = t < TAPS ? (t / 5) * SIW + t % 5 + i : 0;
        }
    // this lane's h1 and h2 columns lie in the domain (or x is periodic)
    const int xh1 = x0 - 4 + 16 * wave + i, xh2 = x0 - 2 + 16 * wave + i;
    const bool ok1 = d.perx || (xh1 >= 0 && xh1 < d.nx), ok2 = d.perx || (xh2 >= 0 && xh2 < d.nx);
    const int s0 = y0 - 5;
    for (int r = s0 - 1; r <= s0 + 3; r++) put_in(r, load_in(r));
    // input rows in flight ten rows ahead: at row s = s5 + u, q0[u] holds row s + 4 (staged at
    // the end of the row) and q1[u] row s + 9
    float q0[5], q1[5];
#pragma unroll
    for (int u = 0; u < 5; u++) {
        q0[u] = load_in(s0 + 4 + u);
        q1[u] = load_in(s0 + 9 + u);
    }
    __syncthreads();

    f32x4 acc[5], T = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < 5; k++) acc[k] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int nsteps = (yend - y0 + 10 + 4) / 5 * 5;
    for (int s5 = s0; s5 < s0 + nsteps; s5 += 5) {
#pragma unroll
        for (int u = 0; u < 5; u++) {
            const int s = s5 + u;
            // every LDS read of the row first: all of it was written before the last barrier,
            // and the row's writes go to ring slots the row does not read (h1 row s + 1, h2 row
            // s - 2, input row s + 4)
            const unsigned* rows = sin + ((s - 1) & (SIR - 1)) * SIW + 16 * wave;
            unsigned A1[2][4];
#pragma unroll
            for (int q = 0; q < 2; q++)
#pragma unroll
                for (int jj = 0; jj < 4; jj++) A1[q][jj] = rows[toff[q][jj]];
            const unsigned short* src2 = sh1 + (s & 1) * SH1W * 32 + (g * SH1W + 16 * wave + i) * 8;
            const unsigned short* src3 = sh2 + ((s - 3) & 1) * SH2W * 32 + (g * SH2W + 16 * wave + i) * 8;
            us8 A2[5], A3[5];
#pragma unroll
            for (int dx = 0; dx < 5; dx++) {
                A2[dx] = *reinterpret_cast<const us8*>(src2 + dx * 8);
                A3[dx] = *reinterpret_cast<const us8*>(src3 + dx * 8);
            }
            // layer 1: h1 row s + 1 from input rows s - 1 .. s + 3
            f32x4 a = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int q = 0; q < 2; q++) {
#pragma unroll
                for (int jj = 0; jj < 4; jj++) A1[q][jj] = q == 0 || tok[q][jj] ? A1[q][jj] : 0u;   // taps 0 .. 15 exist
                a = mfma(b1[q], __builtin_bit_cast(us8, A1[q]), a);
            }
            // layer 2: h1 row s into the h2 rows s - 2 .. s + 2; row s - 2 (tap row dy = 4)
            // first, so that its conversion and store overlap the other 20 MFMAs
#pragma unroll
            for (int dx = 0; dx < 5; dx++) acc[(u + 3) % 5] = mfma(b2[20 + dx], A2[dx], acc[(u + 3) % 5]);
            {
                unsigned short* h1 = sh1 + ((s + 1) & 1) * SH1W * 32;
                const int yr = s + 1;
                const bool ok = (d.pery || (yr >= 0 && yr < d.ny)) && ok1;
#pragma unroll
                for (int r = 0; r < 4; r++) a[r] = ok ? a[r] : 0.f;
                store_ch4(h1, SH1W, 16 * wave + i, g, a);
            }
#pragma unroll
            for (int dx = 0; dx < 5; dx++)
#pragma unroll
                for (int dy = 0; dy < 4; dy++) {
                    const int k = (u + 7 - dy) % 5;
                    acc[k] = mfma(b2[5 * dy + dx], A2[dx], acc[k]);
                }
            // layer 3: h2 row s - 3; output row s - 5 completes in column 4
            T = shift_columns(T);
#pragma unroll
            for (int dx = 0; dx < 5; dx++) T = mfma(A3[dx], b3[dx], T);
            {
                f32x4& c2 = acc[(u + 3) % 5];
                unsigned short* h2 = sh2 + ((s - 2) & 1) * SH2W * 32;
                const int yr = s - 2;
                const bool ok = (d.pery || (yr >= 0 && yr < d.ny)) && ok2;
#pragma unroll
                for (int r = 0; r < 4; r++) c2[r] = ok ? c2[r] : 0.f;
                store_ch4(h2, SH2W, 16 * wave + i, g, c2);
                c2 = f32x4{0.f, 0.f, 0.f, 0.f};
            }
            {
                const int y = s - 5;
                if (i == 4 && y >= y0 && y < yend) {
#pragma unroll
                    for (int r = 0; r < 4; r++) {
                        const int c = 16 * wave + 4 * g + r, x = x0 + c;
                        if (c < SOW && x < d.nx) out.p[vaddr(out, img, y, x)] = T[r];
                    }
                }
            }
            put_in(s + 4, q0[u]);
            q0[u] = q1[u];
            q1[u] = load_in(s + 14);
            __syncthreads();
        }
    }
}

// ---- host launchers ---------------------------------------------------------------------

int chunks(int cin) { return (TAPS * cin * 2 + 31) / 32; }

void launch_pack(const float* w, int cin, int cout, bool adjoint, void* wpk, hipStream_t s)
{
    const int nq = chunks(adjoint ? cout : cin);
    hipLaunchKernelGGL(k_lf_pack, dim3(nq), dim3(64), 0, s, w, cin, cout, adjoint ? 1 : 0,
                       reinterpret_cast<us8*>(wpk));
}

template <int CIN, int COUT>
void launch_conv(const View& in, const View& out, const Domain& d, const void* wpk, hipStream_t s)
{
    const dim3 grid((d.nx + LTX - 1) / LTX, (d.ny + LTY - 1) / LTY, d.nimg);
    hipLaunchKernelGGL((k_lf_conv<CIN, COUT>), grid, dim3(256), 0, s, in, out, d,
                       reinterpret_cast<const us8*>(wpk));
}

template <int CIN, int COUT>
void launch_wgrad(const View& in, const View& gout, const Domain& d, float* dw, hipStream_t s)
{
    const dim3 grid((d.nx + LTX - 1) / LTX, (d.ny + LTY - 1) / LTY, d.nimg);
    hipLaunchKernelGGL((k_lf_wgrad<CIN, COUT>), grid, dim3(256), 0, s, in, gout, d, dw);
}

template void launch_conv<1, 16>(const View&, const View&, const Domain&, const void*, hipStream_t);
template void launch_conv<16, 16>(const View&, const View&, const Domain&, const void*, hipStream_t);
template void launch_conv<16, 1>(const View&, const View&, const Domain&, const void*, hipStream_t);

void launch_loss(const float* out, const float* target, float* g, const Domain& d, int margin,
                 double inv_count, double* loss, hipStream_t s)
{
    hipLaunchKernelGGL(k_lf_loss, dim3(256), dim3(256), 0, s, out, target, g, d, margin, inv_count, loss);
}

void launch_adam(float* w, float* m, float* v, const float* g, int n, float lr, float b1, float b2,
                 float eps, float c1, float c2, hipStream_t s)
{
    hipLaunchKernelGGL(k_lf_adam, dim3((n + 255) / 256), dim3(256), 0, s, w, m, v, g, n, lr, b1, b2,
                       eps, c1, c2);
}

void launch_zero(float* p, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_lf_zero, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
}

// the three-layer forward pass: in (1 channel) -> h1 (16) -> h2 (16) -> out (1 channel), kept
// in separate layers when the intermediates are needed (training)
void forward(const View& in, const View& h1, const View& h2, const View& out, const Domain& d,
             const Packed& pk, hipStream_t s)
{
    launch_conv<1, 16>(in, h1, d, pk.fwd[0], s);
    launch_conv<16, 16>(h1, h2, d, pk.fwd[1], s);
    launch_conv<16, 1>(h2, out, d, pk.fwd[2], s);
}

// the forward pass streamed in one kernel (inference), on up to three image planes at once
void forward_fused(const View* in, const View* out, const Domain* d, int nplanes, const Packed& pk, hipStream_t s)
{
    Planes P{};
    P.n = nplanes;
    int nx = 0, ny = 0, nimg = 0;
    for (int k = 0; k < nplanes; k++) {
        P.in[k] = in[k];
        P.out[k] = out[k];
        P.d[k] = d[k];
        nx = std::max(nx, d[k].nx);
        ny = std::max(ny, d[k].ny);
        nimg = std::max(nimg, d[k].nimg);
    }
    // rows per workgroup: each workgroup also walks 10 rows of reach (rounded up to 5), so take
    // the height for which (rounds of resident workgroups) x (rows walked) is least
    static int slots = 0;
    if (!slots) {
        int dev = 0, cus = 0, occ = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            cus = 256;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)k_lf_stream, 256, 0) != hipSuccess ||
            occ < 1)
            occ = 1;
        slots = occ * cus;
    }
    const long cols = (long)((nx + SOW - 1) / SOW) * nimg * nplanes;
    int oh = 16;
    double best = 1e300;
    for (int c = 16; c <= 512; c += 8) {
        const long wg = cols * ((ny + c - 1) / c);
        const double t = (double)((wg + slots - 1) / slots) * ((c + 14) / 5 * 5);
        if (t < best * (1.0 - 1e-9)) {
            best = t;
            oh = c;
        }
        if (c >= ny) break;
    }
    P.oh = oh;
    const dim3 grid((nx + SOW - 1) / SOW, (ny + oh - 1) / oh, nimg * nplanes);
    hipLaunchKernelGGL(k_lf_stream, grid, dim3(256), 0, s, P, reinterpret_cast<const us8*>(pk.fwd[0]),
                       reinterpret_cast<const us8*>(pk.fwd[1]), reinterpret_cast<const us8*>(pk.fwd[2]));
}

void pack_forward(const float* params, const Packed& pk, hipStream_t s)
{
    launch_pack(params + OFF_W1, 1, C, false, pk.fwd[0], s);
    launch_pack(params + OFF_W2, C, C, false, pk.fwd[1], s);
    launch_pack(params + OFF_W3, C, 1, false, pk.fwd[2], s);
}

void pack_adjoint(const float* params, const Packed& pk, hipStream_t s)
{
    launch_pack(params + OFF_W2, C, C, true, pk.adj[1], s);
    launch_pack(params + OFF_W3, C, 1, true, pk.adj[2], s);
}

// one training pass: forward, loss, backward (data and weights); adds the gradient to dw
void backward(const View& in, const View& h1, const View& h2, const View& out, const View& gout,
              const View& gh1, const View& gh2, const Domain& d, const Packed& pk, float* dw,
              hipStream_t s)
{
    launch_wgrad<16, 1>(h2, gout, d, dw + OFF_W3, s);
    launch_conv<1, 16>(gout, gh2, d, pk.adj[2], s);
    launch_wgrad<16, 16>(h1, gh2, d, dw + OFF_W2, s);
    launch_conv<16, 16>(gh2, gh1, d, pk.adj[1], s);
    launch_wgrad<1, 16>(in, gh1, d, dw + OFF_W1, s);
}

}  // namespace lf
}  // namespace bf

// ======================================================================================
// C ABI: standalone learned filter (batched inference and training on device images)
// ======================================================================================

#include <algorithm>
#include <cmath>
#include <vector>
#include "../../include/bfpic.h"

namespace {

using namespace bf::lf;

size_t up256(size_t v) { return (v + 255) / 256 * 256; }

// sub-allocation of the caller's work buffer for nimg images of ny x nx
struct LfWork {
    size_t packed[5], h1, h2, gh1, gh2, out, gout, dw, loss, bytes;
};

LfWork lf_work(int nimg, int ny, int nx)
{
    LfWork w;
    size_t o = 0;
    auto take = [&](size_t b) { size_t r = o; o = up256(o + b); return r; };
    const int nq[5] = {chunks(1), chunks(C), chunks(C), chunks(C), chunks(1)};
    for (int k = 0; k < 5; k++) w.packed[k] = take((size_t)nq[k] * CHUNK_BYTES);
    const size_t px = (size_t)nimg * ny * nx;
    w.h1 = take(px * C * 4);
    w.h2 = take(px * C * 4);
    w.gh1 = take(px * C * 4);
    w.gh2 = take(px * C * 4);
    w.out = take(px * 4);
    w.gout = take(px * 4);
    w.dw = take((size_t)NPARAM * 4);
    w.loss = take(2 * sizeof(double));
    w.bytes = o;
    return w;
}

Packed packed_of(unsigned char* base, const LfWork& w)
{
    Packed p;
    p.fwd[0] = base + w.packed[0];
    p.fwd[1] = base + w.packed[1];
    p.fwd[2] = base + w.packed[2];
    p.adj[0] = nullptr;
    p.adj[1] = base + w.packed[3];
    p.adj[2] = base + w.packed[4];
    return p;
}

View image_view(const float* p, int ny, int nx, int ch)
{
    View v;
    v.p = const_cast<float*>(p);
    v.rstride = (long)nx * ch;
    v.istride = (long)ny * nx * ch;
    v.ch = ch;
    v.zoff = 0;
    v.rows = ny;
    return v;
}

bool dims_ok(int nimg, int ny, int nx)
{
    return nimg > 0 && ny > 0 && nx > 0 && nimg <= 65535 && (long)nimg * ny * nx <= (1L << 31) / C;
}

// exact learned-filter form of the n-pass bilinear filter + compensation (Sec. 4.1): per axis
// the composed 1D stencil ((1 + z) / 2)^(2n) (times the compensation pass) is cut into three
// factors of at most five taps; each layer carries the outer product of its factor with itself
// in channel 0
bool bilinear_params(int npass, int comp, float* out)
{
    const int room[3] = {4, 4, comp ? 2 : 4};
    int left = 2 * npass;
    std::vector<double> st[3];
    for (int l = 0; l < 3; l++) {
        const int k = std::min(room[l], left);
        left -= k;
        std::vector<double> f{1.0};
        for (int r = 0; r < k; r++) {                   // convolve with (1/2, 1/2)
            std::vector<double> g(f.size() + 1, 0.0);
            for (size_t i = 0; i < f.size(); i++) {
                g[i] += 0.5 * f[i];
                g[i + 1] += 0.5 * f[i];
            }
            f.swap(g);
        }
        st[l] = f;
    }
    if (left > 0) return false;
    if (comp) {                                         // (1 - a)/2, a, (1 - a)/2 with a = n/2 + 1
        const double a = 0.5 * npass + 1.0;
        const double c3[3] = {0.5 * (1.0 - a), a, 0.5 * (1.0 - a)};
        std::vector<double> g(st[2].size() + 2, 0.0);
        for (size_t i = 0; i < st[2].size(); i++)
            for (int j = 0; j < 3; j++) g[i + j] += st[2][i] * c3[j];
        st[2].swap(g);
    }
    for (int i = 0; i < NPARAM; i++) out[i] = 0.f;
    const int off[3] = {OFF_W1, OFF_W2, OFF_W3}, cc[3] = {C, C * C, C};   // (t, ci, co) strides
    for (int l = 0; l < 3; l++) {
        double s5[5] = {0, 0, 0, 0, 0};
        const int n = (int)st[l].size(), o = (5 - n) / 2;
        for (int i = 0; i < n; i++) s5[o + i] = st[l][i];
        for (int a = 0; a < 5; a++)
            for (int b = 0; b < 5; b++) out[off[l] + (5 * a + b) * cc[l]] = (float)(s5[a] * s5[b]);
    }
    return true;
}

}  // namespace

extern "C" {

bf_status bf_lf_bilinear_params(int npass, int compensate, float* host_params, int64_t n)
{
    if (!host_params || n != NPARAM || npass < 0) return BF_EINVAL;
    return bilinear_params(npass, compensate ? 1 : 0, host_params) ? BF_OK : BF_EINVAL;
}

int64_t bf_lf_work_bytes(int nimg, int ny, int nx)
{
    if (!dims_ok(nimg, ny, nx)) return -1;
    return (int64_t)lf_work(nimg, ny, nx).bytes;
}

bf_status bf_lf_apply(void* work, int64_t work_bytes, const float* params, const float* in, float* out,
                      int nimg, int ny, int nx, int periodic_x, int periodic_y, void* hip_stream)
{
    if (!work || !params || !in || !out || !dims_ok(nimg, ny, nx)) return BF_EINVAL;
    const LfWork w = lf_work(nimg, ny, nx);
    if (work_bytes < (int64_t)w.bytes) return BF_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    unsigned char* b = static_cast<unsigned char*>(work);
    const Packed pk = packed_of(b, w);
    const Domain d{nimg, ny, nx, periodic_x ? 1 : 0, periodic_y ? 1 : 0};
    (void)hipGetLastError();
    pack_forward(params, pk, s);
    const View vin = image_view(in, ny, nx, 1), vout = image_view(out, ny, nx, 1);
    forward_fused(&vin, &vout, &d, 1, pk, s);
    return hipGetLastError() == hipSuccess ? BF_OK : BF_EDEVICE;
}

bf_status bf_lf_train_step(void* work, int64_t work_bytes, float* params, float* adam_m, float* adam_v,
                           const float* in, const float* target, int nimg, int ny, int nx, int margin,
                           int periodic_x, int periodic_y, float lr, float beta1, float beta2, float eps,
                           int64_t step, float* grad_out, double* loss_out, void* hip_stream)
{
    if (!work || !params || !in || !target || !dims_ok(nimg, ny, nx)) return BF_EINVAL;
    if (margin < 0 || 2 * margin >= ny || 2 * margin >= nx) return BF_EINVAL;
    if (lr != 0.f && (!adam_m || !adam_v || step < 1)) return BF_EINVAL;
    const LfWork w = lf_work(nimg, ny, nx);
    if (work_bytes < (int64_t)w.bytes) return BF_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    unsigned char* b = static_cast<unsigned char*>(work);
    const Packed pk = packed_of(b, w);
    const Domain d{nimg, ny, nx, periodic_x ? 1 : 0, periodic_y ? 1 : 0};
    float* dw = reinterpret_cast<float*>(b + w.dw);
    double* loss = reinterpret_cast<double*>(b + w.loss);
    const View vin = image_view(in, ny, nx, 1);
    const View h1 = image_view(reinterpret_cast<float*>(b + w.h1), ny, nx, C);
    const View h2 = image_view(reinterpret_cast<float*>(b + w.h2), ny, nx, C);
    const View gh1 = image_view(reinterpret_cast<float*>(b + w.gh1), ny, nx, C);
    const View gh2 = image_view(reinterpret_cast<float*>(b + w.gh2), ny, nx, C);
    const View vout = image_view(reinterpret_cast<float*>(b + w.out), ny, nx, 1);
    const View gout = image_view(reinterpret_cast<float*>(b + w.gout), ny, nx, 1);
    (void)hipGetLastError();
    pack_forward(params, pk, s);
    pack_adjoint(params, pk, s);
    forward(vin, h1, h2, vout, d, pk, s);
    launch_zero(reinterpret_cast<float*>(loss), 4, s);
    const double count = (double)nimg * (ny - 2 * margin) * (nx - 2 * margin);
    launch_loss(vout.p, target, gout.p, d, margin, 1.0 / count, loss, s);
    launch_zero(dw, NPARAM, s);
    backward(vin, h1, h2, vout, gout, gh1, gh2, d, pk, dw, s);
    if (grad_out && hipMemcpyAsync(grad_out, dw, (size_t)NPARAM * 4, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return BF_EDEVICE;
    if (loss_out && hipMemcpyAsync(loss_out, loss, sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
        return BF_EDEVICE;
    if (lr != 0.f) {
        const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, (double)step)));
        const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, (double)step)));
        launch_adam(params, adam_m, adam_v, dw, NPARAM, lr, beta1, beta2, eps, c1, c2, s);
    }
    return hipGetLastError() == hipSuccess ? BF_OK : BF_EDEVICE;
}

}  // extern "C"
