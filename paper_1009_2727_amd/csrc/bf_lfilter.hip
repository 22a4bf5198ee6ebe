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

// the three-layer forward pass: in (1 channel) -> h1 (16) -> h2 (16) -> out (1 channel)
void forward(const View& in, const View& h1, const View& h2, const View& out, const Domain& d,
             const Packed& pk, hipStream_t s)
{
    launch_conv<1, 16>(in, h1, d, pk.fwd[0], s);
    launch_conv<16, 16>(h1, h2, d, pk.fwd[1], s);
    launch_conv<16, 1>(h2, out, d, pk.fwd[2], s);
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

#include <cmath>
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

}  // namespace

extern "C" {

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
    forward(image_view(in, ny, nx, 1), image_view(reinterpret_cast<float*>(b + w.h1), ny, nx, C),
            image_view(reinterpret_cast<float*>(b + w.h2), ny, nx, C), image_view(out, ny, nx, 1), d, pk, s);
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
