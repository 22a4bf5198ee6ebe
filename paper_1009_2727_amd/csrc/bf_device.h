// bf_device.h -- device-side types and helpers shared by the gfx950 kernels.
//
// Grid layout: every field component is one array of stored_z rows x pitch elements,
// x fastest.  Logical row k (0 = outer edge of the back PML, or the first row of a periodic
// axis) lives in physical row (k + zoff) mod stored_z: the moving window advances by
// changing zoff and clearing one row instead of copying the arrays.
//
// Stagger: a component is either on nodes (index j at position j) or on half-nodes (index
// j at position j + 1/2) along each axis, as in the Yee mesh of Sec. 4.2:
//   Ex (half, node)  Ey (node, node)  Ez (node, half)
//   Bx (node, half)  By (half, half)  Bz (half, node)     J like E, rho like Ey.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bf {

// sticky status bits
enum : int { ST_CAPACITY = 1, ST_NONFINITE = 2, ST_SEGMENTS = 4 };

struct Geo {
    int Nx, Nz;       // interior cells
    int Px, Pz;       // PML cells (0 on periodic axes)
    int Sx, Sz;       // stored extents
    int pitch;        // row pitch in elements
    int perx, perz;   // periodic flags
    int zoff;         // ring offset, 0 <= zoff < Sz
};

__device__ __forceinline__ int prow(const Geo& g, int k)
{
    int r = k + g.zoff;
    return r >= g.Sz ? r - g.Sz : r;
}
__device__ __forceinline__ long gofs(const Geo& g, int i, int k)
{
    return (long)prow(g, k) * g.pitch + i;
}

// wrap/clip a stored index: periodic axes wrap, others return -1 outside [0, S)
__device__ __forceinline__ int swrap(int i, int S, int per)
{
    if (per) { i %= S; return i < 0 ? i + S : i; }
    return (i < 0 || i >= S) ? -1 : i;
}

// last valid stored index of a component with stagger h on an axis (non-periodic axes keep
// the half-node beyond the wall unused)
__device__ __forceinline__ int smax(int S, int per, int h) { return per ? S - 1 : S - 1 - h; }

// cubic B-spline weights of the 4 nodes j-1..j+2 around x = j + f, 0 <= f < 1
template <typename R>
__device__ __forceinline__ void bspline3(R f, R w[4])
{
    const R one = R(1), sixth = R(1) / R(6);
    R g = one - f;
    R f2 = f * f, f3 = f2 * f;
    w[0] = g * g * g * sixth;
    w[1] = (R(3) * f3 - R(6) * f2 + R(4)) * sixth;
    w[2] = (R(-3) * f3 + R(3) * f2 + R(3) * f + one) * sixth;
    w[3] = f3 * sixth;
}

// wave-aggregated atomic add of 1 to counter[key] for the active lanes; returns the
// per-lane slot (old value + rank among the lanes with the same key)
__device__ __forceinline__ int wave_slot(int* counter, int key, bool active)
{
    int res = 0;
    bool pending = active;
    const int lane = __lane_id();
    for (;;) {
        unsigned long long m = __ballot(pending);
        if (m == 0ull) break;
        int leader = __ffsll((long long)m) - 1;
        int lkey = __shfl(key, leader);
        bool mine = pending && (key == lkey);
        unsigned long long mm = __ballot(mine);
        int old = 0;
        if (lane == leader) old = atomicAdd(&counter[lkey], __popcll(mm));
        old = __shfl(old, leader);
        if (mine) {
            res = old + __popcll(mm & ((1ull << lane) - 1ull));
            pending = false;
        }
    }
    return res;
}

// block-wide min/max reduction of 4 ints (x0, x1, z0, z1) for a 256-thread block
__device__ __forceinline__ void block_bbox(int& x0, int& x1, int& z0, int& z1, int4* red)
{
    for (int o = 32; o > 0; o >>= 1) {
        x0 = min(x0, __shfl_xor(x0, o));
        x1 = max(x1, __shfl_xor(x1, o));
        z0 = min(z0, __shfl_xor(z0, o));
        z1 = max(z1, __shfl_xor(z1, o));
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) red[w] = make_int4(x0, x1, z0, z1);
    __syncthreads();
    if (threadIdx.x == 0) {
        int4 r = red[0];
        const int nw = blockDim.x >> 6;
        for (int q = 1; q < nw; q++) {
            r.x = min(r.x, red[q].x); r.y = max(r.y, red[q].y);
            r.z = min(r.z, red[q].z); r.w = max(r.w, red[q].w);
        }
        red[0] = r;
    }
    __syncthreads();
    int4 r = red[0];
    x0 = r.x; x1 = r.y; z0 = r.z; z1 = r.w;
}

// A device work queue over the items of several runs: run r owns items [off[r], off[r+1]);
// workgroups take items in increasing order, from an atomic counter (zero before the launch) or
// in a static grid-stride share.
struct QueueRef {
    const int* off;
    int nrun, total;
    int* counter;
};

// the workgroup's next item, or -1 once the queue is drained (every thread gets the same value)
__device__ __forceinline__ int next_item(const QueueRef& q, int* slot)
{
    __syncthreads();   // the previous item is done with the LDS and with *slot
    if (threadIdx.x == 0) *slot = atomicAdd(q.counter, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(*slot);
    return it < q.total ? it : -1;
}

// the workgroup's k-th item of a static grid-stride share of the queue (blockIdx.x + k gridDim.x),
// or -1 past the end; for phases whose items cost about the same, it spares the counter's atomic
// round trip per item
__device__ __forceinline__ int stride_item(const QueueRef& q, int k)
{
    __syncthreads();   // the previous item is done with the LDS
    const int it = (int)blockIdx.x + k * (int)gridDim.x;
    return it < q.total ? it : -1;
}

// run owning item `it`; items arrive in increasing order, so the search resumes from `r`
__device__ __forceinline__ int run_of(const QueueRef& q, int it, int r)
{
    while (r + 1 < q.nrun && q.off[r + 1] <= it) r++;
    return __builtin_amdgcn_readfirstlane(r);
}

}  // namespace bf
