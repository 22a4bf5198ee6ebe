// bf_lfilter.h -- learned current filter: shared types of the MFMA kernels and the host code.
#pragma once
#include <hip/hip_runtime.h>

namespace bf {
namespace lf {

constexpr int C = 16;      // hidden channels
constexpr int TAPS = 25;   // 5 x 5 taps, t = 5 (dy + 2) + (dx + 2), dy along rows (z), dx along x
// FP32 master parameters: W1(t, co) [25 x 16], W2(t, ci, co) [25 x 16 x 16], W3(t, ci) [25 x 16]
constexpr int OFF_W1 = 0;
constexpr int OFF_W2 = TAPS * C;
constexpr int OFF_W3 = OFF_W2 + TAPS * C * C;
constexpr int NPARAM = OFF_W3 + TAPS * C;   // 7200
constexpr int CHUNK_BYTES = 64 * 16;        // one packed B fragment chunk (64 lanes x 8 BF16)

// a batch of images of `ch` channels: element (img, y, x, c) at
// p[img * istride + ((y + zoff) mod rows) * rstride + x * ch + c]  (zoff: ring-buffered rows)
struct View {
    float* p;
    long istride, rstride;
    int ch, zoff, rows;
};

// the domain the convolution runs on: nimg images of ny x nx pixels; outside it the input is
// zero (non-periodic axis) or wrapped (periodic axis)
struct Domain {
    int nimg, ny, nx, perx, pery;
};

// packed BF16 B fragments: forward layers 1..3 and the adjoints of layers 2 and 3
struct Packed {
    void* fwd[3];
    void* adj[3];
};

int chunks(int cin);
void launch_pack(const float* w, int cin, int cout, bool adjoint, void* wpk, hipStream_t s);
template <int CIN, int COUT>
void launch_conv(const View& in, const View& out, const Domain& d, const void* wpk, hipStream_t s);
void launch_loss(const float* out, const float* target, float* g, const Domain& d, int margin,
                 double inv_count, double* loss, hipStream_t s);
void launch_adam(float* w, float* m, float* v, const float* g, int n, float lr, float b1, float b2,
                 float eps, float c1, float c2, hipStream_t s);
void launch_zero(float* p, int n, hipStream_t s);
void pack_forward(const float* params, const Packed& pk, hipStream_t s);
void pack_adjoint(const float* params, const Packed& pk, hipStream_t s);
void forward(const View& in, const View& h1, const View& h2, const View& out, const Domain& d,
             const Packed& pk, hipStream_t s);
void forward_fused(const View* in, const View* out, const Domain* d, int nplanes, const Packed& pk, hipStream_t s);
void backward(const View& in, const View& h1, const View& h2, const View& out, const View& gout,
              const View& gh1, const View& gh2, const Domain& d, const Packed& pk, float* dw,
              hipStream_t s);

}  // namespace lf
}  // namespace bf
