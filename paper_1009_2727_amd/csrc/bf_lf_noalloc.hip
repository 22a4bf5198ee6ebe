// bf_lf_noalloc.hip -- the learned current filter's inference on device images without any
// device allocation: the variant of bf_lf_apply for callers that cannot allocate (code under
// HIP graph capture, tight serving loops).  The packed BF16 forward weights, the only device
// scratch the fused inference kernel reads besides its input and output, live in a file-scope
// device array instead of a caller's work buffer.  Each device holds its own copy of the array
// (it stays allocated until the process ends); its address is looked up with
// hipGetSymbolAddress once per device, on the entry point's first call with that device
// current, and only that address is ever passed to kernels.  Every call on one device shares
// the array, so calls that overlap on one device (different streams, or host threads) race.
#include <mutex>
#include "bf_lfilter.h"
#include "../../include/bfpic.h"

namespace {

using namespace bf::lf;

constexpr size_t SCRATCH_BYTES = 65536;            // the packed forward weights take 53,248 bytes
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void* scratch_ptr[MAX_DEVICES] = {};

size_t up256(size_t v) { return (v + 255) / 256 * 256; }

// offsets of the three packed forward layers inside the scratch; returns the bytes used
size_t layout(size_t off[3])
{
    size_t o = 0;
    const int nq[3] = {chunks(1), chunks(C), chunks(C)};
    for (int k = 0; k < 3; k++) {
        off[k] = o;
        o = up256(o + (size_t)nq[k] * CHUNK_BYTES);
    }
    return o;
}

// device address of `scratch` on the current device
hipError_t scratch_address(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        scratch_ptr[dev] = p;
    }
    *out = scratch_ptr[dev];
    return hipSuccess;
}

View image(const float* p, int ny, int nx)
{
    View v;
    v.p = const_cast<float*>(p);
    v.rstride = nx;
    v.istride = (long)ny * nx;
    v.ch = 1;
    v.zoff = 0;
    v.rows = ny;
    return v;
}

}  // namespace

extern "C" bf_status bf_lf_apply_noalloc(const float* params, const float* in, float* out, int nimg, int ny,
                                         int nx, int periodic_x, int periodic_y, void* hip_stream)
{
    // same image limits as bf_lf_apply (the fused kernel keeps its intermediates in LDS, so the
    // scratch need does not grow with the images)
    if (!params || !in || !out || nimg < 1 || ny < 1 || nx < 1 || nimg > 65535 ||
        (long)nimg * ny * nx > (1L << 31) / C)
        return BF_EINVAL;
    size_t off[3];
    if (layout(off) > SCRATCH_BYTES) return BF_EINVAL;
    void* base = nullptr;
    if (scratch_address(&base) != hipSuccess) return BF_EDEVICE;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    unsigned char* b = static_cast<unsigned char*>(base);
    Packed pk;
    pk.fwd[0] = b + off[0];
    pk.fwd[1] = b + off[1];
    pk.fwd[2] = b + off[2];
    pk.adj[0] = pk.adj[1] = pk.adj[2] = nullptr;
    const Domain d{nimg, ny, nx, periodic_x ? 1 : 0, periodic_y ? 1 : 0};
    (void)hipGetLastError();
    pack_forward(params, pk, s);            // rewrites every scratch byte the kernel reads
    const View vin = image(in, ny, nx), vout = image(out, ny, nx);
    forward_fused(&vin, &vout, &d, 1, pk, s);
    return hipGetLastError() == hipSuccess ? BF_OK : BF_EDEVICE;
}
