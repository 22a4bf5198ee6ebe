// bf_particles.hip -- particle kernels of the boosted-frame PIC step for gfx950.
//
//  * k_gpd: one workgroup per particle segment (a tile after the last sort, or a row chunk
//    injected since).  The segment's bounding box plus a halo is staged in LDS: E^n and
//    B^n = (B^{n-1/2} + B^{n+1/2})/2 (6 components) for the cubic "energy-conserving" gather
//    straight from the staggered Yee locations (Sec. 5.1), and a zeroed J tile (3
//    components).  Each thread then pushes particles (Boris), deposits the Esirkepov current
//    (charge-conserving, Sec. 4.2.2) into the LDS tile with LDS atomics, writes the particle
//    back (positions FP64, rebased by the window shift), and the tile is flushed to HBM with
//    global atomics.  A segment whose box does not fit the LDS budget (or a particle outside
//    its box) takes the same code with global memory accessors.
//  * k_ions: rigid ions (at rest in the lab) deposit their J_z from z0 - beta c t.
//  * k_antenna: the laser antenna's +/- sheet particles (Sec. 3.1.2), in FP64 per pair.
//  * k_inject: creates plasma lattice rows at the front plane (Sec. 3.1.1).
//  * k_sort_*: counting sort by tile (histogram, scan, scatter) that also drops absorbed
//    particles and folds periodic coordinates back into the box.
#include <climits>
#include "bf_kernels.h"

namespace bf {

constexpr int NTHR = 256;

// sum of v over the workgroup, returned to every thread (red: NTHR/64 doubles of LDS)
__device__ __forceinline__ double block_sum(double v, double* red)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NTHR / 64; w++) t += red[w];
    return t;
}

// ---- accessors ---------------------------------------------------------------------------
// The staged tile has a fixed row pitch, so every stencil offset is a compile-time immediate of
// the LDS instruction.  The 8-byte current adds are served 16 lanes at a time, two lanes
// conflicting when their word indices agree mod 16; a pitch of 0 (mod 16) keeps a lane whose
// stencil starts one row lower (a z face crossed in the step) on the slot of its column.
constexpr int TPX = 32;                 // row pitch of the staged tile (cells)
// rows of the staged tile: 6 field planes + 3 FP64 current planes stay under 64 KB
template <typename R> constexpr int trows() { return sizeof(R) == 4 ? 31 : 21; }
template <typename R> constexpr int tcells() { return TPX * trows<R>(); }

// Current accumulator of the staged tile.  FP32 runs accumulate in 64-bit integer fixed
// point: the integer LDS add is faster than the FP64 one on gfx950 (the FP32 LDS add is far
// slower than either), and integer sums do not depend on the order of the adds.  The quantum q
// of a segment is max|fj| * sum|w| / 2^46, so no cell's sum reaches 2^46 quanta.  A
// contribution v is rounded by one FMA, t = v/q + 1.5 * 2^52, whose bit pattern is the
// constant 0x4338000000000000 plus round(v/q) as a 64-bit two's-complement integer.  The raw
// bit patterns are summed: the constant only touches bits 48..63, so the low 48 bits of the
// sum, sign-extended, are the exact sum of the rounded contributions.  FP64 runs accumulate
// in FP64.
template <typename R> struct JAcc { using T = double; static constexpr bool fixed = false; };
template <> struct JAcc<float> { using T = unsigned long long; static constexpr bool fixed = true; };
constexpr double FIX_MAGIC = 6755399441055744.0;   // 1.5 * 2^52
constexpr double FIX_RANGE = 70368744177664.0;     // 2^46

// value of a fixed-point tile sum: sign-extended low 48 bits
__device__ __forceinline__ double fix_value(unsigned long long t)
{
    return (double)((long long)(t << 16) >> 16);
}

// field component ids inside the staged tile: 0..2 E, 3..5 B (time-centred).
// A handle is the offset of a stencil's lower corner; stencil nodes are (handle, a, b).
template <typename R>
struct LdsAcc {
    static constexpr int TCELLS = tcells<R>();
    static constexpr bool FIX = JAcc<R>::fixed;
    using JT = typename JAcc<R>::T;
    R* f;       // 6 planes of TCELLS
    JT* j;      // 3 planes of TCELLS
    int xb, zb, lx, lz;
    __device__ __forceinline__ bool inside(int jx0, int jx1, int jz0, int jz1) const
    {
        return jx0 >= xb && jx1 < xb + lx && jz0 >= zb && jz1 < zb + lz;
    }
    __device__ __forceinline__ int handle(int jx, int jz) const { return (jz - zb) * TPX + (jx - xb); }
    __device__ __forceinline__ R fld(int h, int c, int a, int b) const
    {
        return f[c * TCELLS + h + b * TPX + a];
    }
    // contributions a*b and a*b + c*d, already in quanta for the fixed-point tile
    __device__ __forceinline__ double prod(double a, double b) const
    {
        if constexpr (FIX) return fma(a, b, FIX_MAGIC);
        else return a * b;
    }
    __device__ __forceinline__ double prod2(double a, double b, double c, double d) const
    {
        if constexpr (FIX) return fma(a, b, fma(c, d, FIX_MAGIC));
        else return a * b + c * d;
    }
    __device__ __forceinline__ void dep(int h, int c, int a, int b, double v) const
    {
        if constexpr (FIX)
            atomicAdd(&j[c * TCELLS + h + b * TPX + a], (unsigned long long)__double_as_longlong(v));
        else
            atomicAdd(&j[c * TCELLS + h + b * TPX + a], v);
    }
};

template <typename R>
struct GlobAcc {
    Geo g;
    const R* E[3];
    const R* B[3];
    const R* Bn[3];
    const R* G[6];     // node values (momentum-conserving gather), or null
    R* J[3];
    __device__ __forceinline__ bool inside(int, int, int, int) const { return true; }
    __device__ __forceinline__ int2 handle(int jx, int jz) const { return make_int2(jx, jz); }
    __device__ __forceinline__ R fld(int2 h, int c, int a, int b) const
    {
        int i = swrap(h.x + a + g.Px, g.Sx, g.perx), k = swrap(h.y + b + g.Pz, g.Sz, g.perz);
        if (i < 0 || k < 0) return R(0);
        long o = gofs(g, i, k);
        if (G[0]) return G[c][o];
        if (c < 3) return E[c][o];
        return R(0.5) * (B[c - 3][o] + Bn[c - 3][o]);
    }
    __device__ __forceinline__ double prod(double a, double b) const { return a * b; }
    __device__ __forceinline__ double prod2(double a, double b, double c, double d) const
    {
        return a * b + c * d;
    }
    __device__ __forceinline__ void dep(int2 h, int c, int a, int b, double v) const
    {
        int i = swrap(h.x + a + g.Px, g.Sx, g.perx), k = swrap(h.y + b + g.Pz, g.Sz, g.perz);
        if (i < 0 || k < 0) return;
        atomicAdd(&J[c][gofs(g, i, k)], (R)v);
    }
};

template <bool MC, typename R>
__device__ __forceinline__ GlobAcc<R> make_glob(const Geo& g, const FieldSet<R>& f)
{
    GlobAcc<R> a;
    a.g = g;
    for (int c = 0; c < 3; c++) {
        a.E[c] = f.E[c];
        a.B[c] = f.B[c];
        a.Bn[c] = f.Bn[c];
        a.J[c] = f.J[c];
    }
    for (int c = 0; c < 6; c++) a.G[c] = MC ? f.G[c] : nullptr;
    return a;
}

// reciprocal and reciprocal square root: the hardware instructions (1 ulp) in FP32, exact
// division in FP64
__device__ __forceinline__ float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_(double x) { return 1.0 / x; }
__device__ __forceinline__ float rsqrt_(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_(double x) { return 1.0 / sqrt(x); }

// cubic B-spline weights (FP64) of a particle at fraction f of its cell, on the 5-node window
// starting one node below the particle's (hi = false) or two below (hi = true)
__device__ __forceinline__ void window5(double f, bool hi, double s[5])
{
    const double g = 1.0 - f, f2 = f * f, f3 = f2 * f, sixth = 1.0 / 6.0;
    const double w0 = g * g * g * sixth;
    const double w1 = (3.0 * f3 - 6.0 * f2 + 4.0) * sixth;
    const double w2 = (-3.0 * f3 + 3.0 * f2 + 3.0 * f + 1.0) * sixth;
    const double w3 = f3 * sixth;
    s[0] = hi ? 0.0 : w0;
    s[1] = hi ? w0 : w1;
    s[2] = hi ? w1 : w2;
    s[3] = hi ? w2 : w3;
    s[4] = hi ? w3 : 0.0;
}

// Esirkepov (2001) current of one particle moving (ix+fx, iz+fz) -> (ix1+fx1, iz1+fz1),
// |displacement| < 1 cell per axis, on the 5x5 window whose lower corner is
// (min(ix,ix1)-1, min(iz,iz1)-1).  With S0, S1 the old and new shape factors and
// DS = S1 - S0, the 2-1/2D weights are
//   W_x = DS_x (S0_z + DS_z/2),  W_z = DS_z (S0_x + DS_x/2),
//   W_y = S0_x S0_z + DS_x S0_z/2 + S0_x DS_z/2 + DS_x DS_z/3,
// J_x(i+1/2) - J_x(i-1/2) = cx W_x(i) (likewise z), J_y = cy W_y.  Evaluated in factored
// form: J_x(m,b) = cx (S0_z+S1_z)(b)/2 * sum_{k<=m} DS_x(k),  J_z likewise, and
// W_y = S0_x (S0_z/3 + S1_z/6) + S1_x (S0_z/6 + S1_z/3).
template <typename A>
__device__ __forceinline__ void esirkepov(const A& acc, int ix, double fx, int iz, double fz, int ix1,
                                          double fx1, int iz1, double fz1, double cx, double cz,
                                          double cy)
{
    const int bx = min(ix, ix1) - 1, bz = min(iz, iz1) - 1;
    double S0x[5], S1x[5], S0z[5], S1z[5];
    window5(fx, ix > bx + 1, S0x);
    window5(fx1, ix1 > bx + 1, S1x);
    window5(fz, iz > bz + 1, S0z);
    window5(fz1, iz1 > bz + 1, S1z);
    const auto h = acc.handle(bx, bz);
    if (cx != 0.0) {
        double czf[5];
#pragma unroll
        for (int b = 0; b < 5; b++) czf[b] = 0.5 * cx * (S0z[b] + S1z[b]);
        double pd = 0.0;
#pragma unroll
        for (int m = 0; m < 4; m++) {
            pd += S1x[m] - S0x[m];
#pragma unroll
            for (int b = 0; b < 5; b++) acc.dep(h, 0, m, b, acc.prod(pd, czf[b]));
        }
    }
    {
        double cxf[5];
#pragma unroll
        for (int m = 0; m < 5; m++) cxf[m] = 0.5 * cz * (S0x[m] + S1x[m]);
        double pd = 0.0;
#pragma unroll
        for (int b = 0; b < 4; b++) {
            pd += S1z[b] - S0z[b];
#pragma unroll
            for (int m = 0; m < 5; m++) acc.dep(h, 2, m, b, acc.prod(pd, cxf[m]));
        }
    }
    if (cy != 0.0) {
        const double c3 = cy * (1.0 / 3.0), c6 = cy * (1.0 / 6.0);
        double P[5], Q[5];
#pragma unroll
        for (int b = 0; b < 5; b++) {
            P[b] = c3 * S0z[b] + c6 * S1z[b];
            Q[b] = c6 * S0z[b] + c3 * S1z[b];
        }
#pragma unroll
        for (int b = 0; b < 5; b++)
#pragma unroll
            for (int m = 0; m < 5; m++) acc.dep(h, 1, m, b, acc.prod2(S0x[m], P[b], S1x[m], Q[b]));
    }
}

// gather E^n, B^n at (x, z) (cells) with cubic weights at each component's stagger (energy
// conserving), or from the node values with nodal weights for every component (MC: momentum
// conserving, the accessor then serves the node arrays)
template <bool MC, typename R, typename A>
__device__ __forceinline__ void gather(const A& acc, double x, double z, R E[3], R B[3])
{
    const int ix = (int)floor(x), iz = (int)floor(z);
    const double xh = MC ? x : x - 0.5, zh = MC ? z : z - 0.5;
    const int ixh = (int)floor(xh), izh = (int)floor(zh);
    R wxn[4], wxh[4], wzn[4], wzh[4];
    bspline3((R)(x - ix), wxn);
    bspline3((R)(xh - ixh), wxh);
    bspline3((R)(z - iz), wzn);
    bspline3((R)(zh - izh), wzh);
    const auto hnn = acc.handle(ix - 1, iz - 1), hhn = acc.handle(ixh - 1, iz - 1);
    const auto hnh = acc.handle(ix - 1, izh - 1), hhh = acc.handle(ixh - 1, izh - 1);
    R e0 = 0, e1 = 0, e2 = 0, b0 = 0, b1 = 0, b2 = 0;
#pragma unroll
    for (int b = 0; b < 4; b++) {
        R ex = 0, ey = 0, ez = 0, bx = 0, by = 0, bz = 0;
#pragma unroll
        for (int a = 0; a < 4; a++) {
            ex += wxh[a] * acc.fld(hhn, 0, a, b);
            ey += wxn[a] * acc.fld(hnn, 1, a, b);
            bz += wxh[a] * acc.fld(hhn, 5, a, b);
            ez += wxn[a] * acc.fld(hnh, 2, a, b);
            bx += wxn[a] * acc.fld(hnh, 3, a, b);
            by += wxh[a] * acc.fld(hhh, 4, a, b);
        }
        e0 += wzn[b] * ex; e1 += wzn[b] * ey; b2 += wzn[b] * bz;
        e2 += wzh[b] * ez; b0 += wzh[b] * bx; b1 += wzh[b] * by;
    }
    E[0] = e0; E[1] = e1; E[2] = e2;
    B[0] = b0; B[1] = b1; B[2] = b2;
}

// Boris rotation (q/m folded into h = q dt / 2m)
template <typename R>
__device__ __forceinline__ void boris(R h, const R E[3], const R B[3], R& ux, R& uy, R& uz)
{
    R umx = ux + h * E[0], umy = uy + h * E[1], umz = uz + h * E[2];
    R ig = rsqrt_(R(1) + umx * umx + umy * umy + umz * umz);
    R tx = h * B[0] * ig, ty = h * B[1] * ig, tz = h * B[2] * ig;
    R t2 = tx * tx + ty * ty + tz * tz;
    R sf = R(2) * rcp_(R(1) + t2);
    R sx = sf * tx, sy = sf * ty, sz = sf * tz;
    R upx = umx + (umy * tz - umz * ty);
    R upy = umy + (umz * tx - umx * tz);
    R upz = umz + (umx * ty - umy * tx);
    R uqx = umx + (upy * sz - upz * sy);
    R uqy = umy + (upz * sx - upx * sz);
    R uqz = umz + (upx * sy - upy * sx);
    ux = uqx + h * E[0];
    uy = uqy + h * E[1];
    uz = uqz + h * E[2];
}

// Vay's pusher (Phys. Plasmas 15, 056701, 2008): u' = u + (q dt/m)(E + v x B/2), tau = (q dt/2m) B,
// u* = u'.tau, sigma = gamma'^2 - tau^2, gamma^2 = (sigma + sqrt(sigma^2 + 4(tau^2 + u*^2)))/2,
// t = tau/gamma, u = (u' + (u'.t) t + u' x t) / (1 + t^2); h = q dt / 2m
template <typename R>
__device__ __forceinline__ void vay(R h, const R E[3], const R B[3], R& ux, R& uy, R& uz)
{
    const R ig = rsqrt_(R(1) + ux * ux + uy * uy + uz * uz);
    const R vx = ux * ig, vy = uy * ig, vz = uz * ig;
    const R tx0 = h * B[0], ty0 = h * B[1], tz0 = h * B[2];
    const R upx = ux + R(2) * h * E[0] + (vy * tz0 - vz * ty0);
    const R upy = uy + R(2) * h * E[1] + (vz * tx0 - vx * tz0);
    const R upz = uz + R(2) * h * E[2] + (vx * ty0 - vy * tx0);
    const R us = upx * tx0 + upy * ty0 + upz * tz0;
    const R tau2 = tx0 * tx0 + ty0 * ty0 + tz0 * tz0;
    const R sigma = R(1) + upx * upx + upy * upy + upz * upz - tau2;
    const R gn2 = R(0.5) * (sigma + sqrt(sigma * sigma + R(4) * (tau2 + us * us)));
    const R ign = rsqrt_(gn2);
    const R tx = tx0 * ign, ty = ty0 * ign, tz = tz0 * ign;
    const R sf = rcp_(R(1) + tx * tx + ty * ty + tz * tz);
    const R ut = upx * tx + upy * ty + upz * tz;
    ux = sf * (upx + ut * tx + (upy * tz - upz * ty));
    uy = sf * (upy + ut * ty + (upz * tx - upx * tz));
    uz = sf * (upz + ut * tz + (upx * ty - upy * tx));
}

// the state of one electron as read from HBM
template <typename R>
struct EState {
    double x, z;
    R ux, uy, uz, w;
};

template <typename R>
__device__ __forceinline__ EState<R> load_electron(const ElectronArrays<R>& e, int p)
{
    return EState<R>{e.x[p], e.z[p], e.ux[p], e.uy[p], e.uz[p], e.w[p]};
}

// writes back an advanced state (the weight only when the particle was absorbed)
template <typename R>
__device__ __forceinline__ void store_electron(const ElectronArrays<R>& e, int p, const EState<R>& st)
{
    e.x[p] = st.x;
    e.z[p] = st.z;
    e.ux[p] = st.ux;
    e.uy[p] = st.uy;
    e.uz[p] = st.uz;
    if (st.w == R(0)) e.w[p] = R(0);
}

// one electron with accessor A: gather, push, deposit, absorb (w = 0), rebase; st is advanced
// in place (the caller writes it back) and the box is updated.  The caller guarantees the
// gather window [ix-2, ix+2] and the deposit window [ix-2, ix+3] (one-cell move) are
// addressable through A.  js scales the current into A's units.
template <bool MC, typename R, typename A>
__device__ __forceinline__ void advance_electron(const A& acc, const Geo& g, const PushParams<R>& pp,
                                                 EState<R>& st, double js, int* status, int& x0,
                                                 int& x1, int& z0, int& z1)
{
    const double x = st.x, z = st.z;
    const R w = st.w;
    R ux = st.ux, uy = st.uy, uz = st.uz;
    const int ix = (int)floor(x), iz = (int)floor(z);
    R E[3], B[3];
    gather<MC>(acc, x, z, E, B);
    if (pp.vay) vay(pp.qdt2, E, B, ux, uy, uz);
    else boris(pp.qdt2, E, B, ux, uy, uz);
    const R ig = rsqrt_(R(1) + ux * ux + uy * uy + uz * uz);
    const R vx = ux * ig, vy = uy * ig, vz = uz * ig;
    const double xn = x + (double)(pp.dtdx * vx), zn = z + (double)(pp.dtdz * vz);
    const int ix1 = (int)floor(xn), iz1 = (int)floor(zn);
    if (abs(ix1 - ix) <= 1 && abs(iz1 - iz) <= 1) {
        const double jw = js * (double)w;
        esirkepov(acc, ix, x - ix, iz, z - iz, ix1, xn - ix1, iz1, zn - iz1, jw * (double)pp.fjx,
                  jw * (double)pp.fjz, jw * (double)(pp.fjy * vy));
    } else {
        atomicOr(status, ST_NONFINITE);   // faster than light: only a non-finite state gets here
    }
    if (!isfinite(ux + uy + uz)) atomicOr(status, ST_NONFINITE);
    bool alive = true;
    if (!g.perx && (xn < 0.0 || xn >= (double)g.Nx)) alive = false;
    if (!g.perz && (zn < 0.0 || zn >= (double)g.Nz)) alive = false;
    const double zr = zn - (double)pp.shift;   // rebase into the next window frame
    st.x = xn;
    st.z = zr;
    st.ux = ux;
    st.uy = uy;
    st.uz = uz;
    if (!alive) {
        st.w = R(0);
    } else {
        const int cx = (int)floor(xn), cz = (int)floor(zr);
        x0 = min(x0, cx); x1 = max(x1, cx);
        z0 = min(z0, cz); z1 = max(z1, cz);
    }
}

constexpr int MISFIT_CAP = 256;

// gather, push and deposit of particle segment s by one workgroup
template <typename R, bool MC = false>
__device__ __forceinline__ void gpd_segment(const Geo& g, const FieldSet<R>& f, const ElectronArrays<R>& e,
                                            const Segment* __restrict__ seg, const int4* __restrict__ bbin,
                                            int4* __restrict__ bbout, const PushParams<R>& pp, int* status,
                                            int s)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];   // 16-byte aligned: FP64 DS ops
    __shared__ int4 red[NTHR / 64];
    __shared__ double redd[NTHR / 64];
    __shared__ int misfit[MISFIT_CAP];
    __shared__ int nmisfit;
    const Segment sg = seg[s];
    const int4 bb = bbin[s];
    if (sg.count <= 0 || bb.x > bb.y || bb.z > bb.w) {
        if (threadIdx.x == 0) bbout[s] = make_int4(INT_MAX, INT_MIN, INT_MAX, INT_MIN);
        return;
    }
    LdsAcc<R> lds;
    lds.xb = bb.x - 2;
    lds.zb = bb.z - 2;
    lds.lx = bb.y - bb.x + 6;
    lds.lz = bb.w - bb.z + 6;
    lds.f = reinterpret_cast<R*>(smem_raw);
    constexpr int TCELLS = tcells<R>();
    using JT = typename LdsAcc<R>::JT;
    lds.j = reinterpret_cast<JT*>(lds.f + 6 * TCELLS);   // 6 TCELLS elements: 8-byte aligned
    // A box larger than the staged tile (particles spread since the last sort, as in a heated
    // plasma) still stages the largest window, centred on the box, while each thread can
    // remember which of its particles fall outside (at most 64 per thread); those are pushed with
    // the global accessors after the tile is flushed.  Larger segments take the global accessors
    // throughout.
    const bool fits = lds.lx <= TPX && lds.lz <= trows<R>();
    const bool use_lds = fits || sg.count <= 64 * NTHR;
    if (!fits && use_lds) {
        // a particle in cell ix fits while xb + 2 <= ix <= xb + lx - 4
        if (lds.lx > TPX) {
            lds.xb = ((bb.x + bb.y) >> 1) - 2 - (TPX - 6) / 2;
            lds.lx = TPX;
        }
        if (lds.lz > trows<R>()) {
            lds.zb = ((bb.z + bb.w) >> 1) - 2 - (trows<R>() - 6) / 2;
            lds.lz = trows<R>();
        }
    }
    int x0 = INT_MAX, x1 = INT_MIN, z0 = INT_MAX, z1 = INT_MIN;
    const int end = sg.start + sg.count;
    const int L = lds.lx * lds.lz;
    if (use_lds) {
        double js = 1.0, jq = 1.0;   // current into tile units and back
        if constexpr (LdsAcc<R>::FIX) {
            double sw = 0.0;
            for (int p = sg.start + threadIdx.x; p < end; p += NTHR) sw += fabs((double)e.w[p]);
            sw = block_sum(sw, redd);
            const double fj = fmax(fabs((double)pp.fjx), fmax(fabs((double)pp.fjz), fabs((double)pp.fjy)));
            const double bound = fj * sw;   // |v_y| < 1 and every weight factor is <= 1
            if (bound > 0.0) { js = FIX_RANGE / bound; jq = bound / FIX_RANGE; }
        }
        if (threadIdx.x == 0) nmisfit = 0;
        for (int q = threadIdx.x; q < L; q += NTHR) {
            const int a = q % lds.lx, b = q / lds.lx;
            const int i = swrap(lds.xb + a + g.Px, g.Sx, g.perx);
            const int k = swrap(lds.zb + b + g.Pz, g.Sz, g.perz);
            R v[6] = {0, 0, 0, 0, 0, 0};
            if (i >= 0 && k >= 0) {
                const long o = gofs(g, i, k);
                if constexpr (MC) {
#pragma unroll
                    for (int c = 0; c < 6; c++) v[c] = f.G[c][o];
                } else {
#pragma unroll
                    for (int c = 0; c < 3; c++) {
                        v[c] = f.E[c][o];
                        v[3 + c] = R(0.5) * (f.B[c][o] + f.Bn[c][o]);
                    }
                }
            }
            const int t = b * TPX + a;
#pragma unroll
            for (int c = 0; c < 6; c++) lds.f[c * TCELLS + t] = v[c];
#pragma unroll
            for (int c = 0; c < 3; c++) lds.j[c * TCELLS + t] = JT(0);
        }
        __syncthreads();
        // the next particle's state is read while the current one is pushed (the loop is
        // otherwise bound by the HBM latency of its loads); its result is written back at the
        // top of the next iteration, ahead of the following prefetch, so that waiting for the
        // prefetch never waits for fresh stores
        int p = sg.start + threadIdx.x;
        EState<R> nxt{}, done{};
        int pdone = -1;
        uint64_t late = 0;   // bit k: this thread's k-th particle lies outside the staged window
        if (p < end) nxt = load_electron(e, p);
        for (int k = 0; p < end; p += NTHR, k++) {
            EState<R> cur = nxt;
            // the prefetched registers are taken here, before this iteration's stores and
            // loads are issued, so the wait for them covers only memory operations issued one
            // iteration ago (an empty asm that reads them; it emits no instruction)
            asm volatile("" ::"v"(cur.x), "v"(cur.z), "v"(cur.ux), "v"(cur.uy), "v"(cur.uz), "v"(cur.w)
                         : "memory");
            if (pdone >= 0) store_electron(e, pdone, done);
            pdone = -1;
            if (p + NTHR < end) nxt = load_electron(e, p + NTHR);
            if (cur.w == R(0)) continue;
            const int ix = (int)floor(cur.x), iz = (int)floor(cur.z);
            if (!lds.inside(ix - 2, ix + 3, iz - 2, iz + 3)) {
                if (k < 64) {
                    late |= 1ull << k;
                } else {
                    const int slot = atomicAdd(&nmisfit, 1);
                    if (slot < MISFIT_CAP) misfit[slot] = p;
                    else atomicOr(status, ST_SEGMENTS);
                }
                continue;
            }
            advance_electron<MC>(lds, g, pp, cur, js, status, x0, x1, z0, z1);
            done = cur;
            pdone = p;
        }
        if (pdone >= 0) store_electron(e, pdone, done);
        __syncthreads();
        for (int q = threadIdx.x; q < L; q += NTHR) {
            const int a = q % lds.lx, b = q / lds.lx;
            const int i = swrap(lds.xb + a + g.Px, g.Sx, g.perx);
            const int k = swrap(lds.zb + b + g.Pz, g.Sz, g.perz);
            if (i < 0 || k < 0) continue;
            const long o = gofs(g, i, k);
            const int t = b * TPX + a;
#pragma unroll
            for (int c = 0; c < 3; c++) {
                R v;
                if constexpr (LdsAcc<R>::FIX) v = (R)(fix_value(lds.j[c * TCELLS + t]) * jq);
                else v = (R)lds.j[c * TCELLS + t];
                if (v != R(0)) atomicAdd(&f.J[c][o], v);
            }
        }
        // particles outside the staged window: global accessors
        const int nm = min(nmisfit, MISFIT_CAP);
        if (nm > 0 || late) {
            const GlobAcc<R> glb = make_glob<MC>(g, f);
            while (late) {
                const int b = __builtin_ctzll(late);
                late &= late - 1;
                const int q = sg.start + threadIdx.x + b * NTHR;
                EState<R> st = load_electron(e, q);
                advance_electron<MC>(glb, g, pp, st, 1.0, status, x0, x1, z0, z1);
                store_electron(e, q, st);
            }
            for (int q = threadIdx.x; q < nm; q += NTHR) {
                const int p = misfit[q];
                EState<R> st = load_electron(e, p);
                advance_electron<MC>(glb, g, pp, st, 1.0, status, x0, x1, z0, z1);
                store_electron(e, p, st);
            }
        }
    } else {
        const GlobAcc<R> glb = make_glob<MC>(g, f);
        for (int p = sg.start + threadIdx.x; p < end; p += NTHR) {
            EState<R> st = load_electron(e, p);
            if (st.w == R(0)) continue;
            advance_electron<MC>(glb, g, pp, st, 1.0, status, x0, x1, z0, z1);
            store_electron(e, p, st);
        }
    }
    block_bbox(x0, x1, z0, z1, red);
    if (threadIdx.x == 0) bbout[s] = make_int4(x0, x1, z0, z1);
}

template <typename R, bool MC>
__global__ void __launch_bounds__(NTHR, sizeof(R) == 4 ? 3 : 1) k_gpd(Geo g, FieldSet<R> f, ElectronArrays<R> e,
                                              const Segment* __restrict__ seg,
                                              const int4* __restrict__ bbin, int4* __restrict__ bbout,
                                              PushParams<R> pp, int* status)
{
    gpd_segment<R, MC>(g, f, e, seg, bbin, bbout, pp, status, blockIdx.x);
}

template <typename R>
__global__ void __launch_bounds__(NTHR, sizeof(R) == 4 ? 3 : 1) k_gpd_batch(const GpdDesc<R>* __restrict__ d,
                                                                            QueueRef q)
{
    __shared__ int slot;
    int r = 0;
    for (;;) {
        const int it = next_item(q, &slot);
        if (it < 0) return;
        r = run_of(q, it, r);
        const GpdDesc<R>& D = d[r];
        gpd_segment<R>(D.g, D.f, D.e, D.seg, D.bbin, D.bbout, D.pp, D.status, it - q.off[r]);
    }
}

// ---- rigid ions --------------------------------------------------------------------------
// J_z of a particle at fixed x moving (iz+fz) -> (iz1+fz1): the Esirkepov form with DS_x = 0,
// J_z(m,b) = cz S_x(m) sum_{k<=b} DS_z(k) on the 4 x 5 window with lower corner
// (ix-1, min(iz,iz1)-1).
template <typename A>
__device__ __forceinline__ void ion_current(const A& acc, int ix, double fx, int iz, double fz, int iz1,
                                            double fz1, double cz)
{
    const int bz = min(iz, iz1) - 1;
    double Sx[5], S0z[5], S1z[5];
    window5(fx, false, Sx);
    window5(fz, iz > bz + 1, S0z);
    window5(fz1, iz1 > bz + 1, S1z);
    double cxs[4];
#pragma unroll
    for (int m = 0; m < 4; m++) cxs[m] = cz * Sx[m];
    const auto h = acc.handle(ix - 1, bz);
    double pd = 0.0;
#pragma unroll
    for (int b = 0; b < 4; b++) {
        pd += S1z[b] - S0z[b];
#pragma unroll
        for (int m = 0; m < 4; m++) acc.dep(h, 2, m, b, acc.prod(pd, cxs[m]));
    }
}

template <typename R>
__device__ __forceinline__ void ion_segment(const Geo& g, const FieldSet<R>& f, const IonArrays<R>& ion,
                                            const Segment* __restrict__ seg, const int4* __restrict__ bbin,
                                            int4* __restrict__ bbout, double zsh_a, double zsh_b, int shift,
                                            R fjz, int s)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];   // 16-byte aligned: FP64 DS ops
    __shared__ int4 red[NTHR / 64];
    __shared__ double redd[NTHR / 64];
    const Segment sg = seg[s];
    const int4 bb = bbin[s];
    if (sg.count <= 0 || bb.x > bb.y || bb.z > bb.w) {
        if (threadIdx.x == 0) bbout[s] = make_int4(INT_MAX, INT_MIN, INT_MAX, INT_MIN);
        return;
    }
    using JT = typename LdsAcc<R>::JT;
    GlobAcc<R> glb = make_glob<false>(g, f);
    LdsAcc<R> lds;
    lds.xb = bb.x - 2;
    lds.zb = bb.z - 2;
    lds.lx = bb.y - bb.x + 6;
    lds.lz = bb.w - bb.z + 6;
    constexpr int TCELLS = tcells<R>();
    const bool use_lds = lds.lx <= TPX && lds.lz <= trows<R>();
    // only J_z (component 2) is staged: point j so that component 2 starts at smem
    lds.f = nullptr;
    lds.j = reinterpret_cast<JT*>(smem_raw) - 2 * TCELLS;
    if (!use_lds) { lds.lx = 0; lds.lz = 0; }
    const int L = lds.lx * lds.lz;
    JT* jz = reinterpret_cast<JT*>(smem_raw);
    const int end = sg.start + sg.count;
    double js = 1.0, jq = 1.0;   // current into tile units and back (fixed-point tile)
    if (use_lds) {
        if constexpr (LdsAcc<R>::FIX) {
            double sw = 0.0;
            for (int p = sg.start + threadIdx.x; p < end; p += NTHR) sw += fabs((double)ion.w[p]);
            sw = block_sum(sw, redd);
            const double bound = fabs((double)fjz) * sw;
            if (bound > 0.0) { js = FIX_RANGE / bound; jq = bound / FIX_RANGE; }
        }
        for (int q = threadIdx.x; q < L; q += NTHR) jz[(q / lds.lx) * TPX + q % lds.lx] = JT(0);
        __syncthreads();
    }
    int x0 = INT_MAX, x1 = INT_MIN, z0 = INT_MAX, z1 = INT_MIN;
    // the next ion is read while the current one deposits
    int p = sg.start + threadIdx.x;
    double nx_ = 0.0, nz_ = 0.0;
    R nw = R(0);
    if (p < end) { nx_ = ion.x[p]; nz_ = ion.z0[p]; nw = ion.w[p]; }
    for (; p < end; p += NTHR) {
        const R w = nw;
        const double x = nx_, zc0 = nz_;
        if (p + NTHR < end) { nx_ = ion.x[p + NTHR]; nz_ = ion.z0[p + NTHR]; nw = ion.w[p + NTHR]; }
        if (w == R(0)) continue;
        const double za = zc0 - zsh_a, zb = zc0 - zsh_b;
        const int ix = (int)floor(x), iz = (int)floor(za), iz1 = (int)floor(zb);
        const double fx = x - ix, fz = za - iz, fz1 = zb - iz1;
        const int bz = min(iz, iz1) - 1;
        if (lds.inside(ix - 1, ix + 2, bz, bz + 4) && abs(iz1 - iz) <= 1)
            ion_current(lds, ix, fx, iz, fz, iz1, fz1, js * (double)(fjz * w));
        else
            ion_current(glb, ix, fx, iz, fz, iz1, fz1, (double)(fjz * w));
        bool alive = !(!g.perz && (zb < 0.0 || zb >= (double)g.Nz));
        if (!alive) {
            ion.w[p] = R(0);
        } else {
            const int cz = (int)floor(zb - (double)shift);
            x0 = min(x0, ix); x1 = max(x1, ix);
            z0 = min(z0, cz); z1 = max(z1, cz);
        }
    }
    if (use_lds) {
        __syncthreads();
        for (int q = threadIdx.x; q < L; q += NTHR) {
            const int a = q % lds.lx, b = q / lds.lx;
            R v;
            if constexpr (LdsAcc<R>::FIX) v = (R)(fix_value(jz[b * TPX + a]) * jq);
            else v = (R)jz[b * TPX + a];
            if (v == R(0)) continue;
            const int i = swrap(lds.xb + a + g.Px, g.Sx, g.perx);
            const int k = swrap(lds.zb + b + g.Pz, g.Sz, g.perz);
            if (i < 0 || k < 0) continue;
            atomicAdd(&f.J[2][gofs(g, i, k)], v);
        }
    }
    block_bbox(x0, x1, z0, z1, red);
    if (threadIdx.x == 0) bbout[s] = make_int4(x0, x1, z0, z1);
}

template <typename R>
__global__ void __launch_bounds__(NTHR) k_ions(Geo g, FieldSet<R> f, IonArrays<R> ion,
                                               const Segment* __restrict__ seg,
                                               const int4* __restrict__ bbin, int4* __restrict__ bbout,
                                               double zsh_a, double zsh_b, int shift, R fjz)
{
    ion_segment<R>(g, f, ion, seg, bbin, bbout, zsh_a, zsh_b, shift, fjz, blockIdx.x);
}


// ---- antenna (FP64) ------------------------------------------------------------------------

// Esirkepov current of one particle moving (x0, z0) -> (x1, z1) (cells, |move| < 1 cell) with
// out-of-plane velocity vy, charge factor qw, at cell (cx, cz) of the grid: J_x on (cx + 1/2, cz),
// J_z on (cx, cz + 1/2), J_y on the node (cx, cz) (2-1/2D weights as in esirkepov()).  FP64
// throughout.
__device__ __forceinline__ void esirkepov_cell(double x0, double z0, double x1, double z1, double qw,
                                               double vy, double dx, double dz, double dt, int cx, int cz,
                                               double& jx, double& jy, double& jz)
{
    const int ix = (int)floor(x0), iz = (int)floor(z0), ix1 = (int)floor(x1), iz1 = (int)floor(z1);
    if (abs(ix1 - ix) > 1 || abs(iz1 - iz) > 1) return;   // one step moves less than a cell
    const int bx = min(ix, ix1) - 1, bz = min(iz, iz1) - 1;
    const int m = cx - bx, b = cz - bz;                    // node of the 5 x 5 window
    if (m < 0 || m > 4 || b < 0 || b > 4) return;
    double S0x[5], S1x[5], S0z[5], S1z[5];
    window5(x0 - ix, ix > bx + 1, S0x);
    window5(x1 - ix1, ix1 > bx + 1, S1x);
    window5(z0 - iz, iz > bz + 1, S0z);
    window5(z1 - iz1, iz1 > bz + 1, S1z);
    if (m < 4) {
        double pd = 0.0;
        for (int k = 0; k <= m; k++) pd += S1x[k] - S0x[k];
        jx += -qw / (dz * dt) * pd * 0.5 * (S0z[b] + S1z[b]);
    }
    if (b < 4) {
        double pd = 0.0;
        for (int k = 0; k <= b; k++) pd += S1z[k] - S0z[k];
        jz += -qw / (dx * dt) * pd * 0.5 * (S0x[m] + S1x[m]);
    }
    if (vy != 0.0) {
        // W_y: time average of S_x S_z along the straight move
        const double dsx = S1x[m] - S0x[m], dsz = S1z[b] - S0z[b];
        const double wy = S0x[m] * S0z[b] + 0.5 * dsx * S0z[b] + 0.5 * S0x[m] * dsz + dsx * dsz / 3.0;
        jy += qw * vy * wy / (dx * dz);
    }
}

// One wave per sheet pair, one lane per cell of the pair's 6 x 6 patch: the + particle stays at
// its home x and moves with the plane, the - particle also moves along the polarisation so that
// the pair carries the sheet current K = -2 E_perp (Sec. 3.1.2): along x it moves in the plane
// (J_x), along y it keeps its home x and its velocity enters J_y.  Both deposit by Esirkepov in
// FP64.
template <typename R>
__global__ void __launch_bounds__(64) k_antenna(Geo g, FieldSet<R> f, double* xm, AntennaParams ap)
{
    const int i = blockIdx.x;
    const int lane = threadIdx.x;
    if (i >= ap.n) return;
    const double xh = i + 0.5;                   // home position (cells)
    const double xum = xh * ap.dx_um;
    // field to emit: (E0/gamma) f sin(omega t'/gamma - phase) with the lab time elapsed at the
    // lab-fixed plane t'/gamma; the sheet current is K = -2 E_perp (eps0 = c = 1)
    const double tau = ap.tmid / ap.gamma - ap.t0;
    const double env = exp(-(xum - ap.xc_um) * (xum - ap.xc_um) / (ap.w0 * ap.w0)) *
                       exp(-tau * tau / (2.0 * ap.sig_t * ap.sig_t));
    const double Ep = (ap.e0 / ap.gamma) * env * sin(ap.omega * tau);
    const double K = -2.0 * Ep;
    const double v = K * ap.dx / (-ap.weight);    // moving sheet has charge -w
    const double xa = xm[i];
    const double xb = ap.pol == 0 ? xa + v * ap.dt / ap.dx : xa;
    const double vy = ap.pol == 0 ? 0.0 : v;
    const int px = (int)floor(xh) - 2;
    const int pz = (int)floor(fmin(ap.za, ap.zb)) - 1;
    if (lane < 36) {
        const int cx = px + lane % 6, cz = pz + lane / 6;
        double jx = 0.0, jy = 0.0, jz = 0.0;
        esirkepov_cell(xa, ap.za, xb, ap.zb, -ap.weight, vy, ap.dx, ap.dz, ap.dt, cx, cz, jx, jy, jz);
        esirkepov_cell(xh, ap.za, xh, ap.zb, ap.weight, 0.0, ap.dx, ap.dz, ap.dt, cx, cz, jx, jy, jz);
        const int si = swrap(cx + g.Px, g.Sx, g.perx), sk = swrap(cz + g.Pz, g.Sz, g.perz);
        if (si >= 0 && sk >= 0) {
            const long o = gofs(g, si, sk);
            if (jx != 0.0) atomicAdd(&f.J[0][o], (R)jx);
            if (jy != 0.0) atomicAdd(&f.J[1][o], (R)jy);
            if (jz != 0.0) atomicAdd(&f.J[2][o], (R)jz);
        }
    }
    if (lane == 0) xm[i] = xb;
}

// ---- particle beam through a lab-fixed plane (Sec. 3.1.1) ---------------------------------

__device__ __forceinline__ bool beam_inside(const Geo& g, double x, double z)
{
    if (!g.perx && (x < 0.0 || x >= (double)g.Nx)) return false;
    if (!g.perz && (z < 0.0 || z >= (double)g.Nz)) return false;
    return true;
}

__device__ __forceinline__ double beam_wrap(double v, int N, int per)
{
    if (!per) return v;
    return v < 0.0 ? v + N : (v >= (double)N ? v - N : v);
}

// One thread per beam particle.  A frozen particle (transverse position and momentum fixed)
// moves along z at the boosted mean velocity until a step starts at t_n >= t'*; it then
// becomes an ordinary electron (energy-conserving or momentum-conserving gather, Boris or
// Vay in FP64, Esirkepov deposit through global atomics).  Particles activated outside the
// interior, or leaving it, are lost.  Each block adds its active particles' lab-frame sums
// (gamma_lab = gamma (gamma' + beta u'_z), z_lab = gamma (z' + beta t'), ...) to the record.
template <typename R, bool MC>
__global__ void __launch_bounds__(NTHR) k_beam(Geo g, FieldSet<R> f, BeamArrays b, BeamParams bp,
                                               PushParams<double> pp, int* status)
{
    __shared__ double red[NTHR / 64];
    const int p = blockIdx.x * NTHR + threadIdx.x;
    double a[7] = {0, 0, 0, 0, 0, 0, 0};
    if (p < bp.n && b.state[p] != 2) {
        const GlobAcc<R> acc = make_glob<MC>(g, f);
        int st = b.state[p];
        const double x = b.x[p], z = b.z[p], w = b.w[p];
        if (st == 0 && b.tact[p] <= bp.t0) st = beam_inside(g, x, z) ? 1 : 2;
        const int ix = (int)floor(x), iz = (int)floor(z);
        if (st == 0) {
            const double zn = z + bp.vbar_cells;
            if (bp.deposit && beam_inside(g, x, z)) {
                const int iz1 = (int)floor(zn);
                esirkepov(acc, ix, x - ix, iz, z - iz, ix, x - ix, iz1, zn - iz1, w * pp.fjx, w * pp.fjz, 0.0);
            }
            b.z[p] = beam_wrap(zn, g.Nz, g.perz) - (double)pp.shift;
        } else if (st == 1) {
            R Er[3], Br[3];
            gather<MC>(acc, x, z, Er, Br);
            const double E[3] = {(double)Er[0], (double)Er[1], (double)Er[2]};
            const double B[3] = {(double)Br[0], (double)Br[1], (double)Br[2]};
            double ux = b.ux[p], uy = b.uy[p], uz = b.uz[p];
            if (pp.vay) vay(pp.qdt2, E, B, ux, uy, uz);
            else boris(pp.qdt2, E, B, ux, uy, uz);
            const double gp = sqrt(1.0 + ux * ux + uy * uy + uz * uz);
            const double xn = x + pp.dtdx * ux / gp, zn = z + pp.dtdz * uz / gp;
            const int ix1 = (int)floor(xn), iz1 = (int)floor(zn);
            if (abs(ix1 - ix) <= 1 && abs(iz1 - iz) <= 1) {
                if (bp.deposit)
                    esirkepov(acc, ix, x - ix, iz, z - iz, ix1, xn - ix1, iz1, zn - iz1, w * pp.fjx, w * pp.fjz,
                              w * pp.fjy * (uy / gp));
            } else {
                atomicOr(status, ST_NONFINITE);   // faster than light: only a non-finite state gets here
            }
            if (!isfinite(ux + uy + uz)) atomicOr(status, ST_NONFINITE);
            b.ux[p] = ux; b.uy[p] = uy; b.uz[p] = uz;
            if (!beam_inside(g, xn, zn)) {
                st = 2;
                b.x[p] = xn; b.z[p] = zn;
            } else {
                const double za = (zn + bp.shift) * bp.dz_um;   // window-independent boosted z'
                const double zl = bp.gamma * (za + bp.beta * bp.t1), tl = bp.gamma * (bp.t1 + bp.beta * za);
                const double gl = bp.gamma * (gp + bp.beta * uz), ul = bp.gamma * (uz + bp.beta * gp);
                a[0] = 1.0; a[1] = w; a[2] = w * zl; a[3] = w * tl; a[4] = w * gl; a[5] = w * ul; a[6] = w * ul * ul;
                b.x[p] = beam_wrap(xn, g.Nx, g.perx);
                b.z[p] = beam_wrap(zn, g.Nz, g.perz) - (double)pp.shift;
            }
        }
        b.state[p] = st;
    }
    if (bp.rec < 0) return;   // uniform over the launch
    double* r = b.hist + 8 * (long)bp.rec;
    for (int k = 0; k < 7; k++) {
        const double v = block_sum(a[k], red);
        __syncthreads();   // red is reused by the next sum
        if (threadIdx.x == 0 && v != 0.0) atomicAdd(&r[1 + k], v);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) r[0] = bp.t1;
}

// ---- plasma injection --------------------------------------------------------------------------
__device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t k)
{
    // SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): output number k of the generator
    // started at `seed` (state advances by the golden gamma, output = mix(state))
    uint64_t z = seed + k * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double u01(uint64_t seed, uint64_t k)
{
    return (double)(splitmix64(seed, k) >> 11) * (1.0 / 9007199254740992.0);
}

template <typename R>
__global__ void __launch_bounds__(NTHR) k_inject(Geo g, ElectronArrays<R> e, IonArrays<R> ion,
                                                 Segment* seg_e, int4* bbox_e, Segment* seg_i,
                                                 int4* bbox_i, int* nused_e, int* nused_i,
                                                 InjectParams ip, int* status)
{
    __shared__ int sh_start[2];
    __shared__ int4 red[NTHR / 64];
    const int chunk = blockIdx.x, r = blockIdx.y;
    const int64_t row = ip.row0 + r;
    const int cx0 = chunk * ip.tile_x;
    const int ncell = min(ip.tile_x, g.Nx - cx0);
    const int count = ncell * ip.ppc;
    const int slot = ip.seg_base + r * ip.nchunks + chunk;
    if (threadIdx.x == 0) {
        int se = atomicAdd(nused_e, count);
        int si = ip.ion_mode ? atomicAdd(nused_i, count) : 0;
        if ((int64_t)se + count > ip.cap || (int64_t)si + count > ip.cap) {
            atomicOr(status, ST_CAPACITY);
            se = -1;
        }
        sh_start[0] = se;
        sh_start[1] = si;
    }
    __syncthreads();
    const int se = sh_start[0], si = sh_start[1];
    if (se < 0) {
        if (threadIdx.x == 0) {
            seg_e[slot] = Segment{0, 0};
            bbox_e[slot] = make_int4(INT_MAX, INT_MIN, INT_MAX, INT_MIN);
            if (ip.ion_mode) {
                seg_i[slot] = Segment{0, 0};
                bbox_i[slot] = make_int4(INT_MAX, INT_MIN, INT_MAX, INT_MIN);
            }
        }
        return;
    }
    int x0 = INT_MAX, x1 = INT_MIN, z0 = INT_MAX, z1 = INT_MIN;
    for (int q = threadIdx.x; q < count; q += NTHR) {
        const int cell = q % ncell, k = q / ncell;   // consecutive lanes in consecutive cells
        const int ix = cx0 + cell;
        const uint64_t id = ((uint64_t)row * (uint64_t)g.Nx + (uint64_t)ix) * (uint64_t)ip.ppc + (uint64_t)k;
        const double rx = u01(ip.seed, 2 * id + 1), rz = u01(ip.seed, 2 * id + 2);
        const double zbc = (double)row + rz;                 // boosted position at t = 0, cells
        const double zl = ip.gamma * (zbc * ip.dz_um);       // lab position of the element
        double n = 0.0;
        if (zl >= ip.ramp_start) {
            n = ip.n0;
            if (ip.ramp_len > 0.0 && zl < ip.ramp_start + ip.ramp_len)
                n = ip.n0 * (zl - ip.ramp_start) / ip.ramp_len;
        }
        const double wgt = ip.wfac * n;
        const double x = (double)ix + rx;
        const double z = zbc - ip.beta * ip.t / ip.dz_um - ip.shift;
        const int p = se + q;
        e.x[p] = x;
        e.z[p] = z;
        e.ux[p] = R(0);
        e.uy[p] = R(0);
        e.uz[p] = (R)ip.uz0;
        e.w[p] = (R)wgt;
        e.id[p] = (uint32_t)id;
        if (ip.ion_mode) {
            const int pi = si + q;
            ion.x[pi] = x;
            ion.z0[pi] = zbc;
            ion.w[pi] = (R)wgt;
            ion.id[pi] = (uint32_t)id;
        }
        if (wgt != 0.0) {
            const int ci = (int)floor(x), ck = (int)floor(z);
            x0 = min(x0, ci); x1 = max(x1, ci);
            z0 = min(z0, ck); z1 = max(z1, ck);
        }
    }
    block_bbox(x0, x1, z0, z1, red);
    if (threadIdx.x == 0) {
        seg_e[slot] = Segment{se, count};
        bbox_e[slot] = make_int4(x0, x1, z0, z1);
        if (ip.ion_mode) {
            seg_i[slot] = Segment{si, count};
            bbox_i[slot] = make_int4(x0, x1, z0, z1);
        }
    }
}

// modular inverse of a mod n (gcd(a, n) == 1), extended Euclid
__device__ __forceinline__ int64_t inv_mod(int64_t a, int64_t n)
{
    int64_t t = 0, nt = 1, r = n, nr = a % n;
    while (nr != 0) {
        const int64_t q = r / nr, tt = t - q * nt, rr = r - q * nr;
        t = nt; nt = tt; r = nr; nr = rr;
    }
    return t < 0 ? t + n : t;
}

__device__ __forceinline__ int64_t gcd64(int64_t a, int64_t b)
{
    while (b) { const int64_t t = a % b; a = b; b = t; }
    return a;
}

// Exclusive scan of the tile counts; writes the new segment table (one per tile), each
// tile's box (the tile rectangle), the scatter rank counters (zero) and the new slot count.
// counts[] is overwritten with each tile's slot multiplier, 1: the first pass of the sort
// writes each tile's particles to consecutive slots in arrival order (a source wave's
// particles mostly share a destination tile, so its writes stay coalesced); the second pass
// (k_sort_disperse_*) orders them within the tile.
__global__ void __launch_bounds__(1024) k_sort_scan(int* counts, int ntiles, int ntx, int tx, int tz,
                                                    int Nx, int Nz, Segment* seg, int4* bbox, int* cursor,
                                                    int* nused)
{
    __shared__ int part[1024];
    const int t = threadIdx.x;
    const int per = (ntiles + 1023) / 1024;
    const int lo = min(t * per, ntiles), hi = min(lo + per, ntiles);
    int sum = 0;
    for (int i = lo; i < hi; i++) sum += counts[i];
    part[t] = sum;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        int v = t >= o ? part[t - o] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = part[t] - sum;   // exclusive prefix of this thread's chunk
    for (int i = lo; i < hi; i++) {
        const int c = counts[i];
        seg[i] = Segment{run, c};
        cursor[i] = 0;
        counts[i] = 1;
        const int cxi = i % ntx, czi = i / ntx;
        const int xa = cxi * tx, za = czi * tz;
        bbox[i] = c > 0 ? make_int4(xa, min(xa + tx, Nx) - 1, za, min(za + tz, Nz) - 1)
                        : make_int4(INT_MAX, INT_MIN, INT_MAX, INT_MIN);
        run += c;
    }
    if (t == 1023) *nused = part[1023];
}

__device__ __forceinline__ int tile_slot(const Segment* seg, const int* mult, int key, int rank)
{
    const Segment sg = seg[key];
    return sg.start + (int)(((int64_t)rank * (int64_t)mult[key]) % (int64_t)sg.count);
}

// ---- counting sort by tile ----------------------------------------------------------------------
__device__ __forceinline__ double fold(double v, int N, int per)
{
    if (!per) return v;
    double r = v - floor(v / (double)N) * (double)N;
    return r >= (double)N ? r - (double)N : r;
}

__device__ __forceinline__ int tile_key(double x, double z, const Geo& g, int tx, int tz, int ntx,
                                        int ntz)
{
    int cx = min(max((int)floor(x), 0), g.Nx - 1) / tx;
    int cz = min(max((int)floor(z), 0), g.Nz - 1) / tz;
    (void)ntz;
    return cz * ntx + cx;
}

template <typename R>
__global__ void __launch_bounds__(NTHR) k_sort_count_e(Geo g, ElectronArrays<R> e,
                                                       const Segment* seg, int tx, int tz, int ntx,
                                                       int ntz, int* counts)
{
    const Segment sg = seg[blockIdx.x];
    for (int base = 0; base < sg.count; base += NTHR) {
        const int q = base + threadIdx.x;
        bool act = false;
        int key = 0;
        if (q < sg.count) {
            const int p = sg.start + q;
            if (e.w[p] != R(0)) {
                act = true;
                key = tile_key(fold(e.x[p], g.Nx, g.perx), fold(e.z[p], g.Nz, g.perz), g, tx, tz, ntx, ntz);
            }
        }
        wave_slot(counts, key, act);
    }
}

template <typename R>
__global__ void __launch_bounds__(NTHR) k_sort_scatter_e(Geo g, ElectronArrays<R> src,
                                                         ElectronArrays<R> dst, const Segment* seg,
                                                         int tx, int tz, int ntx, int ntz, int* cursor,
                                                         const Segment* seg_new, const int* mult)
{
    const Segment sg = seg[blockIdx.x];
    for (int base = 0; base < sg.count; base += NTHR) {
        const int q = base + threadIdx.x;
        bool act = false;
        int key = 0, p = 0;
        double x = 0, z = 0;
        if (q < sg.count) {
            p = sg.start + q;
            if (src.w[p] != R(0)) {
                act = true;
                x = fold(src.x[p], g.Nx, g.perx);
                z = fold(src.z[p], g.Nz, g.perz);
                key = tile_key(x, z, g, tx, tz, ntx, ntz);
            }
        }
        const int r = wave_slot(cursor, key, act);
        const int d = act ? tile_slot(seg_new, mult, key, r) : 0;
        if (act) {
            dst.x[d] = x;
            dst.z[d] = z;
            dst.ux[d] = src.ux[p];
            dst.uy[d] = src.uy[p];
            dst.uz[d] = src.uz[p];
            dst.w[d] = src.w[p];
            dst.id[d] = src.id[p];
        }
    }
}

template <typename R>
__global__ void __launch_bounds__(NTHR) k_sort_count_i(Geo g, IonArrays<R> ion, const Segment* seg,
                                                       double zsh, int tx, int tz, int ntx, int ntz,
                                                       int* counts)
{
    const Segment sg = seg[blockIdx.x];
    for (int base = 0; base < sg.count; base += NTHR) {
        const int q = base + threadIdx.x;
        bool act = false;
        int key = 0;
        if (q < sg.count) {
            const int p = sg.start + q;
            if (ion.w[p] != R(0)) {
                act = true;
                key = tile_key(fold(ion.x[p], g.Nx, g.perx), ion.z0[p] - zsh, g, tx, tz, ntx, ntz);
            }
        }
        wave_slot(counts, key, act);
    }
}

template <typename R>
__global__ void __launch_bounds__(NTHR) k_sort_scatter_i(Geo g, IonArrays<R> src, IonArrays<R> dst,
                                                         const Segment* seg, double zsh, int tx,
                                                         int tz, int ntx, int ntz, int* cursor,
                                                         const Segment* seg_new, const int* mult)
{
    const Segment sg = seg[blockIdx.x];
    for (int base = 0; base < sg.count; base += NTHR) {
        const int q = base + threadIdx.x;
        bool act = false;
        int key = 0, p = 0;
        double x = 0;
        if (q < sg.count) {
            p = sg.start + q;
            if (src.w[p] != R(0)) {
                act = true;
                x = fold(src.x[p], g.Nx, g.perx);
                key = tile_key(x, src.z0[p] - zsh, g, tx, tz, ntx, ntz);
            }
        }
        const int r = wave_slot(cursor, key, act);
        const int d = act ? tile_slot(seg_new, mult, key, r) : 0;
        if (act) {
            dst.x[d] = x;
            dst.z0[d] = src.z0[p];
            dst.w[d] = src.w[p];
            dst.id[d] = src.id[p];
        }
    }
}

// ---- second pass of the sort: order within each tile --------------------------------------------
// One block per tile reads the tile's particles (consecutive after the first pass) and ranks
// them by cell in row-major order (LDS histogram, scan, per-cell counters).  The particle of
// rank r goes to slot (r m) mod N of the tile, m the inverse of a spacing d coprime to N that
// is at least the largest cell count of the tile: consecutive slots hold ranks d apart, so a
// run of slots holds at most one particle per cell (while 64 d fits in N) and the 64 lanes of
// a wave of the particle kernel deposit into 64 distinct cells of a compact block -- its LDS
// current atomics neither collide nor pile up in a bank.  The copy runs in slot order (slot s
// takes rank s d mod N through an LDS rank -> particle table), so the writes are coalesced and
// the scattered reads stay within the tile's particles.  A tile with more particles than the
// table holds writes each particle to its slot directly.  Particle order changes no result
// (the FP32 tile sums are exact integer sums).
constexpr int SORT_MAX_CELLS = 64 * 64;   // the largest tile the configuration accepts
constexpr int SORT_TABLE = 8192;          // particles per tile ordered through the LDS table
constexpr int SORT_THREADS = 512;

struct TileCells {
    int xa, za, w, h;
    __device__ __forceinline__ int of(double x, double z, const Geo& g) const
    {
        const int cx = min(max((int)floor(x), 0), g.Nx - 1) - xa;
        const int cz = min(max((int)floor(z), 0), g.Nz - 1) - za;
        return min(max(cz, 0), h - 1) * w + min(max(cx, 0), w - 1);
    }
};

__device__ __forceinline__ TileCells tile_cells(const Geo& g, int tx, int tz, int ntx)
{
    TileCells t;
    t.xa = (blockIdx.x % ntx) * tx;
    t.za = (blockIdx.x / ntx) * tz;
    t.w = min(tx, g.Nx - t.xa);
    t.h = min(tz, g.Nz - t.za);
    return t;
}

// LDS state of the tile ordering
struct TileSort {
    int cnt[SORT_MAX_CELLS], base[SORT_MAX_CELLS], idx[SORT_TABLE];
    int part[SORT_THREADS], pmax[SORT_THREADS];
    int mult, spacing;
};

// cnt[] holds the tile's cell counts: replaces them by zeros, fills base[] with the exclusive
// scan and sets the slot multiplier m and the spacing d
__device__ void tile_ranks(TileSort& ts, int C, int N)
{
    const int t = threadIdx.x;
    const int per = (C + SORT_THREADS - 1) / SORT_THREADS, lo = min(t * per, C), hi = min(lo + per, C);
    int sum = 0, mx = 0;
    for (int i = lo; i < hi; i++) {
        sum += ts.cnt[i];
        mx = max(mx, ts.cnt[i]);
    }
    ts.part[t] = sum;
    ts.pmax[t] = mx;
    __syncthreads();
    for (int o = 1; o < SORT_THREADS; o <<= 1) {
        const int v = t >= o ? ts.part[t - o] : 0, m = t >= o ? ts.pmax[t - o] : 0;
        __syncthreads();
        ts.part[t] += v;
        ts.pmax[t] = max(ts.pmax[t], m);
        __syncthreads();
    }
    int run = ts.part[t] - sum;
    for (int i = lo; i < hi; i++) {
        ts.base[i] = run;
        run += ts.cnt[i];
        ts.cnt[i] = 0;
    }
    if (t == 0) {
        int64_t d = 1, m = 1;
        if (N > 2) {
            d = max(ts.pmax[SORT_THREADS - 1], 1);
            while (d < N && gcd64(d, N) != 1) d++;
            if (d < N) m = inv_mod(d, N);
            else d = m = 1;
        }
        ts.mult = (int)m;
        ts.spacing = (int)d;
    }
    __syncthreads();
}

// pos(q) -> (x, z) of the tile's q-th particle; copy(q, slot) moves it
template <typename Pos, typename Copy>
__device__ void order_tile(TileSort& ts, const Segment& sg, const TileCells& tc, const Geo& g, Pos pos, Copy copy)
{
    const int C = tc.w * tc.h, N = sg.count;
    for (int i = threadIdx.x; i < C; i += SORT_THREADS) ts.cnt[i] = 0;
    __syncthreads();
    for (int q = threadIdx.x; q < N; q += SORT_THREADS) {
        const double2 xz = pos(q);
        atomicAdd(&ts.cnt[tc.of(xz.x, xz.y, g)], 1);
    }
    __syncthreads();
    tile_ranks(ts, C, N);
    const int m = ts.mult, d = ts.spacing;
    const bool table = N <= SORT_TABLE;
    for (int q = threadIdx.x; q < N; q += SORT_THREADS) {
        const double2 xz = pos(q);
        const int c = tc.of(xz.x, xz.y, g);
        const int r = ts.base[c] + atomicAdd(&ts.cnt[c], 1);
        if (table) ts.idx[r] = q;
        else copy(q, (int)(((int64_t)r * m) % N));
    }
    if (!table) return;
    __syncthreads();
    for (int sl = threadIdx.x; sl < N; sl += SORT_THREADS) copy(ts.idx[(int)(((int64_t)sl * d) % N)], sl);
}

template <typename R>
__global__ void __launch_bounds__(SORT_THREADS) k_sort_disperse_e(Geo g, ElectronArrays<R> src,
                                                                  ElectronArrays<R> dst, const Segment* seg,
                                                                  int tx, int tz, int ntx)
{
    __shared__ TileSort ts;
    const Segment sg = seg[blockIdx.x];
    if (sg.count == 0) return;
    const TileCells tc = tile_cells(g, tx, tz, ntx);
    const int o = sg.start;
    order_tile(
        ts, sg, tc, g, [&](int q) { return make_double2(src.x[o + q], src.z[o + q]); },
        [&](int q, int sl) {
            const int p = o + q, d = o + sl;
            dst.x[d] = src.x[p];
            dst.z[d] = src.z[p];
            dst.ux[d] = src.ux[p];
            dst.uy[d] = src.uy[p];
            dst.uz[d] = src.uz[p];
            dst.w[d] = src.w[p];
            dst.id[d] = src.id[p];
        });
}

template <typename R>
__global__ void __launch_bounds__(SORT_THREADS) k_sort_disperse_i(Geo g, IonArrays<R> src, IonArrays<R> dst,
                                                                  const Segment* seg, double zsh, int tx, int tz,
                                                                  int ntx)
{
    __shared__ TileSort ts;
    const Segment sg = seg[blockIdx.x];
    if (sg.count == 0) return;
    const TileCells tc = tile_cells(g, tx, tz, ntx);
    const int o = sg.start;
    order_tile(
        ts, sg, tc, g, [&](int q) { return make_double2(src.x[o + q], src.z0[o + q] - zsh); },
        [&](int q, int sl) {
            const int p = o + q, d = o + sl;
            dst.x[d] = src.x[p];
            dst.z0[d] = src.z0[p];
            dst.w[d] = src.w[p];
            dst.id[d] = src.id[p];
        });
}

// ---- launchers ---------------------------------------------------------------------------------
template <typename R>
void launch_gpd(const Geo& g, const FieldSet<R>& f, const ElectronArrays<R>& e, const Segment* seg,
                const int4* bbox_in, int4* bbox_out, int nseg, const PushParams<R>& pp, int* status,
                bool mc, hipStream_t s)
{
    if (nseg <= 0) return;
    const size_t lds = (size_t)tcells<R>() * (6 * sizeof(R) + 3 * sizeof(typename LdsAcc<R>::JT));
    if (mc)
        hipLaunchKernelGGL((k_gpd<R, true>), dim3(nseg), dim3(NTHR), lds, s, g, f, e, seg, bbox_in, bbox_out,
                           pp, status);
    else
        hipLaunchKernelGGL((k_gpd<R, false>), dim3(nseg), dim3(NTHR), lds, s, g, f, e, seg, bbox_in, bbox_out,
                           pp, status);
}

template <typename R>
void launch_ions(const Geo& g, const FieldSet<R>& f, const IonArrays<R>& ion, const Segment* seg,
                 const int4* bbox_in, int4* bbox_out, int nseg, double zsh_a, double zsh_b, int shift,
                 R fjz, hipStream_t s)
{
    if (nseg <= 0) return;
    const size_t lds = (size_t)tcells<R>() * sizeof(typename LdsAcc<R>::JT);
    hipLaunchKernelGGL((k_ions<R>), dim3(nseg), dim3(NTHR), lds, s, g, f, ion, seg, bbox_in, bbox_out,
                       zsh_a, zsh_b, shift, fjz);
}

template <typename R>
void launch_gpd_batch(const GpdDesc<R>* d, const QueueRef& q, int nblocks, hipStream_t s)
{
    const size_t lds = (size_t)tcells<R>() * (6 * sizeof(R) + 3 * sizeof(typename LdsAcc<R>::JT));
    if (q.total > 0)
        hipLaunchKernelGGL((k_gpd_batch<R>), dim3(nblocks), dim3(NTHR), lds, s, d, q);
}


template <typename R>
void launch_antenna(const Geo& g, const FieldSet<R>& f, double* xminus, const AntennaParams& ap,
                    hipStream_t s)
{
    if (!ap.active || ap.n <= 0) return;
    hipLaunchKernelGGL((k_antenna<R>), dim3(ap.n), dim3(64), 0, s, g, f, xminus, ap);
}

template <typename R>
void launch_beam(const Geo& g, const FieldSet<R>& f, const BeamArrays& b, const BeamParams& bp,
                 const PushParams<double>& pp, int* status, bool mc, hipStream_t s)
{
    if (bp.n <= 0) return;
    const dim3 grid((bp.n + NTHR - 1) / NTHR);
    if (mc) hipLaunchKernelGGL((k_beam<R, true>), grid, dim3(NTHR), 0, s, g, f, b, bp, pp, status);
    else hipLaunchKernelGGL((k_beam<R, false>), grid, dim3(NTHR), 0, s, g, f, b, bp, pp, status);
}

template <typename R>
void launch_inject(const Geo& g, const ElectronArrays<R>& e, const IonArrays<R>& ion, Segment* seg_e,
                   int4* bbox_e, Segment* seg_i, int4* bbox_i, int* nused_e, int* nused_i,
                   const InjectParams& ip, int* status, hipStream_t s)
{
    if (ip.nrows <= 0) return;
    hipLaunchKernelGGL((k_inject<R>), dim3(ip.nchunks, ip.nrows), dim3(NTHR), 0, s, g, e, ion, seg_e,
                       bbox_e, seg_i, bbox_i, nused_e, nused_i, ip, status);
}

// two-pass sort: a -> b by tile (consecutive slots per tile), then b -> a ordered within each
// tile; the particles end in a under the new segment table
template <typename R>
void launch_sort_electrons(const Geo& g, int tile_x, int tile_z, int ntx, int ntiles,
                           const ElectronArrays<R>& a, const ElectronArrays<R>& b,
                           const Segment* seg_old, int nseg_old, Segment* seg_new, int4* bbox_new,
                           int* counts, int* cursor, int* nused, hipStream_t s)
{
    const int ntz = ntiles / ntx;
    launch_fill_int(counts, ntiles, 0, s);
    if (nseg_old > 0)
        hipLaunchKernelGGL((k_sort_count_e<R>), dim3(nseg_old), dim3(NTHR), 0, s, g, a, seg_old,
                           tile_x, tile_z, ntx, ntz, counts);
    hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(1024), 0, s, counts, ntiles, ntx, tile_x, tile_z, g.Nx,
                       g.Nz, seg_new, bbox_new, cursor, nused);
    if (nseg_old > 0)
        hipLaunchKernelGGL((k_sort_scatter_e<R>), dim3(nseg_old), dim3(NTHR), 0, s, g, a, b,
                           seg_old, tile_x, tile_z, ntx, ntz, cursor, (const Segment*)seg_new,
                           (const int*)counts);
    hipLaunchKernelGGL((k_sort_disperse_e<R>), dim3(ntiles), dim3(SORT_THREADS), 0, s, g, b, a, (const Segment*)seg_new,
                       tile_x, tile_z, ntx);
}

template <typename R>
void launch_sort_ions(const Geo& g, int tile_x, int tile_z, int ntx, int ntiles, const IonArrays<R>& a,
                      const IonArrays<R>& b, const Segment* seg_old, int nseg_old, Segment* seg_new,
                      int4* bbox_new, double zsh, int* counts, int* cursor, int* nused, hipStream_t s)
{
    const int ntz = ntiles / ntx;
    launch_fill_int(counts, ntiles, 0, s);
    if (nseg_old > 0)
        hipLaunchKernelGGL((k_sort_count_i<R>), dim3(nseg_old), dim3(NTHR), 0, s, g, a, seg_old, zsh,
                           tile_x, tile_z, ntx, ntz, counts);
    hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(1024), 0, s, counts, ntiles, ntx, tile_x, tile_z, g.Nx,
                       g.Nz, seg_new, bbox_new, cursor, nused);
    if (nseg_old > 0)
        hipLaunchKernelGGL((k_sort_scatter_i<R>), dim3(nseg_old), dim3(NTHR), 0, s, g, a, b, seg_old,
                           zsh, tile_x, tile_z, ntx, ntz, cursor, (const Segment*)seg_new,
                           (const int*)counts);
    hipLaunchKernelGGL((k_sort_disperse_i<R>), dim3(ntiles), dim3(SORT_THREADS), 0, s, g, b, a, (const Segment*)seg_new,
                       zsh, tile_x, tile_z, ntx);
}

#define BF_INST(R)                                                                                    \
    template void launch_gpd<R>(const Geo&, const FieldSet<R>&, const ElectronArrays<R>&,             \
                                const Segment*, const int4*, int4*, int, const PushParams<R>&, int*,  \
                                bool, hipStream_t);                                                   \
    template void launch_ions<R>(const Geo&, const FieldSet<R>&, const IonArrays<R>&,                 \
                                 const Segment*, const int4*, int4*, int, double, double, int, R,     \
                                 hipStream_t);                                                        \
    template void launch_gpd_batch<R>(const GpdDesc<R>*, const QueueRef&, int, hipStream_t);          \
    template void launch_antenna<R>(const Geo&, const FieldSet<R>&, double*, const AntennaParams&,    \
                                    hipStream_t);                                                     \
    template void launch_beam<R>(const Geo&, const FieldSet<R>&, const BeamArrays&, const BeamParams&, \
                                 const PushParams<double>&, int*, bool, hipStream_t);                 \
    template void launch_inject<R>(const Geo&, const ElectronArrays<R>&, const IonArrays<R>&,         \
                                   Segment*, int4*, Segment*, int4*, int*, int*,                      \
                                   const InjectParams&, int*, hipStream_t);                           \
    template void launch_sort_electrons<R>(const Geo&, int, int, int, int, const ElectronArrays<R>&,  \
                                           const ElectronArrays<R>&, const Segment*, int, Segment*,   \
                                           int4*, int*, int*, int*, hipStream_t);                     \
    template void launch_sort_ions<R>(const Geo&, int, int, int, int, const IonArrays<R>&,            \
                                      const IonArrays<R>&, const Segment*, int, Segment*, int4*,      \
                                      double, int*, int*, int*, hipStream_t);
BF_INST(float)
BF_INST(double)

}  // namespace bf
