// bf_sim3.hip -- kernels of the 3D boosted-frame step (x, y transverse, z the boost axis).
//
// The method is the 2-1/2D one in three dimensions:
//   * Faraday with the tunable (Cole-Karkkainen) operator Delta* = (alpha + beta S^1 + gamma
//     S^2) Delta, S^1 the four one-cell shifts along the two transverse axes and S^2 the four
//     diagonal shifts, and Friedman damping (Sec. 4.2, Sec. 4.3); Ampere with Yee differences;
//   * split-field PML on every component (Appendix II): each component's two curl terms are
//     damped by the conductivity of their derivative's axis; the stored split part is the one
//     along the axis cyclically next to the component, and it carries the current source;
//   * cubic B-spline gather from the staggered locations (Sec. 5.1), Boris push, Esirkepov's
//     charge-conserving deposit in 3D (Sec. 4.2.2) on 5-node windows;
//   * n-pass bilinear filter plus compensation along x, y and z (Sec. 4.1);
//   * laser sheets on a lab-fixed plane with one +/- pair per transverse cell (Sec. 3.1.2);
//   * moving window as a ring offset of the z planes, plane-wise plasma injection.
// Faraday and Ampere march up z over (x, y) tiles with the planes they difference in LDS; the
// other field stages run one thread per cell on the arrays in HBM.  Particles are binned by tile
// (periodic counting sort) and pushed one segment per workgroup on an LDS-staged box; the
// deposited current is summed in FP64 in HBM (fixed point or FP64 in LDS).
#include "bf_kernels3.h"
#include "bf_device.h"
#include <algorithm>
#include <climits>
#include <cmath>
#include <type_traits>

namespace bf3 {

constexpr int NT = 256;

__device__ __forceinline__ int nb(int i, int o, int S, int per)
{
    int j = i + o;
    if (per) {
        j %= S;
        return j < 0 ? j + S : j;
    }
    return (j < 0 || j >= S) ? -1 : j;
}

__device__ __forceinline__ long o3(const G3& g, int i, int j, int k)
{
    int kk = k + g.zoff;
    if (kk >= g.S[2]) kk -= g.S[2];
    return (long)kk * g.plane + (long)j * g.pitch + i;
}

// stored index of interior-relative node (or half node) j along axis a; -1 outside
__device__ __forceinline__ int sidx(const G3& g, int a, int j)
{
    if (g.per[a]) {
        j %= g.N[a];
        return j < 0 ? j + g.N[a] : j;
    }
    j += g.P[a];
    return (j < 0 || j >= g.S[a]) ? -1 : j;
}

// cell of a thread in the per-cell launches: 32 x 8 threads per workgroup over (x, y), one
// workgroup row per z plane
constexpr int CBX = 32, CBY = 8;

__device__ __forceinline__ bool cell_of(const G3& g, int q[3])
{
    q[0] = (int)(blockIdx.x * CBX + threadIdx.x);
    q[1] = (int)(blockIdx.y * CBY + threadIdx.y);
    q[2] = (int)blockIdx.z;
    return q[0] < g.S[0] && q[1] < g.S[1];
}

inline dim3 cells_grid(const G3& g)
{
    return dim3((unsigned)((g.S[0] + CBX - 1) / CBX), (unsigned)((g.S[1] + CBY - 1) / CBY), (unsigned)g.S[2]);
}

inline dim3 cells_block() { return dim3(CBX, CBY); }
static_assert(CBX * CBY == NT, "per-cell launches use NT threads");

// ---- field solver ---------------------------------------------------------------------------

// split update of one component from its curl terms t1 (axis A1, the stored part) and t2
template <int A1, int A2, typename R>
__device__ __forceinline__ R split_update(R old, R* sp, long o, R t1, R t2, const Pml3& pml, const int q[3],
                                          const int h[3], R dt)
{
    const double s1 = pml.sig[A1][h[A1]][q[A1]], s2 = pml.sig[A2][h[A2]][q[A2]];
    if (s1 == 0.0 && s2 == 0.0) return old + dt * (t1 + t2);
    const R x1 = (R)pml.xi[A1][h[A1]][q[A1]], c1 = (R)pml.c[A1][h[A1]][q[A1]];
    const R x2 = (R)pml.xi[A2][h[A2]][q[A2]], c2 = (R)pml.c[A2][h[A2]][q[A2]];
    R p1 = sp[o];
    R p2 = old - p1;
    p1 = x1 * p1 + c1 * t1;
    p2 = x2 * p2 + c2 * t2;
    sp[o] = p1;
    return p1 + p2;
}

// Faraday with Friedman's E-tilde made on the fly.  A workgroup owns a 32 x 8 tile of (x, y)
// and FMZ planes along z; it marches up z keeping three planes (k - 1, k, k + 1) of E-tilde with
// a one-cell (x, y) halo in LDS, so each E value is read from HBM once per tile instead of once
// per stencil point.  Delta* (Sec. 4.2) reaches one cell along every axis.  With Friedman
// damping (Sec. 4.3), E-tilde = (1 + theta/4) E^n - E^{n-1}/2 + (1/2 - theta/4) Ebar^n with the
// recursion Ebar^n = (1 - theta/2) E^{n-1} + (theta/2) Ebar^{n-1}; the new Ebar goes to the
// second Ebar buffer (f.T), written by the tile that owns the cell, so no workgroup reads a
// value another one has already replaced.  Cells beyond a non-periodic edge read 0.
constexpr int FMX = CBX, FMY = CBY, FMZ = 16;
constexpr int FPX = FMX + 2, FPP = (FMX + 2) * (FMY + 2);

// Delta*_AX of one E-tilde component from the three LDS planes pl[0..2] = k - 1, k, k + 1 at
// padded tile position (cx, cy): alpha D + beta (the four S^1 shifts) + gamma (the four S^2
// shifts), times 1/d
template <int AX, typename R>
__device__ __forceinline__ R dstar_lds(const R* const pl[3], int cx, int cy, int ht, R a, R b, R c, R id)
{
    constexpr int T1 = (AX + 1) % 3, T2 = (AX + 2) % 3;
    auto D = [&](int t1, int t2) {
        int s[3];
        s[T1] = t1;
        s[T2] = t2;
        s[AX] = ht;
        const R hi = pl[s[2] + 1][(cy + s[1]) * FPX + cx + s[0]];
        s[AX] = ht - 1;
        const R lo = pl[s[2] + 1][(cy + s[1]) * FPX + cx + s[0]];
        return hi - lo;
    };
    R v = a * D(0, 0);
    if (b != R(0) || c != R(0)) {
        v += b * (D(1, 0) + D(-1, 0) + D(0, 1) + D(0, -1));
        if (c != R(0)) v += c * (D(1, 1) + D(1, -1) + D(-1, 1) + D(-1, -1));
    }
    return v * id;
}

// dB_C/dt = -(Delta*_A1 E_A2 - Delta*_A2 E_A1), (C, A1, A2) cyclic; B_C sits on a node along C
// and on half nodes along A1, A2
template <int C, typename R>
__device__ __forceinline__ void faraday_cell(const G3& g, const F3<R>& f, const Pml3& pml, const R (*sT)[3][FPP],
                                             const int sl[3], const int q[3], long o, int cx, int cy, R a, R b,
                                             R cg, R dt)
{
    constexpr int A1 = (C + 1) % 3, A2 = (C + 2) % 3;
    const int h[3] = {C == 0 ? 0 : 1, C == 1 ? 0 : 1, C == 2 ? 0 : 1};
    const R old = f.B[C][o];
    f.Bo[C][o] = old;
#pragma unroll
    for (int d = 0; d < 3; d++)
        if (!g.per[d] && q[d] > g.S[d] - 1 - h[d]) return;
    const R* p2[3] = {sT[sl[0]][A2], sT[sl[1]][A2], sT[sl[2]][A2]};
    const R* p1[3] = {sT[sl[0]][A1], sT[sl[1]][A1], sT[sl[2]][A1]};
    const R t1 = -dstar_lds<A1>(p2, cx, cy, h[A1], a, b, cg, (R)(1.0 / g.d[A1]));
    const R t2 = dstar_lds<A2>(p1, cx, cy, h[A2], a, b, cg, (R)(1.0 / g.d[A2]));
    f.B[C][o] = split_update<A1, A2>(old, f.SB[C], o, t1, t2, pml, q, h, dt);
}

// the E-tilde inputs of the padded-plane cells a thread loads (two at most: FPP <= 2 NT)
template <typename R>
struct PlaneRegs {
    R e[2][3], eo[2][3], eb[2][3];
    long o[2];
    bool ok[2], own[2];
};

template <typename R, bool FRIED>
__global__ void __launch_bounds__(NT) k3_faraday(G3 g, F3<R> f, Pml3 pml, R a, R b, R cg, R dt, R th)
{
    static_assert(FPP <= 2 * NT, "a thread loads at most two cells of a padded plane");
    __shared__ R sT[3][3][FPP];   // [ring slot][component][padded plane cell]
    const int tid = (int)(threadIdx.y * FMX + threadIdx.x);
    const int x0 = (int)blockIdx.x * FMX, y0 = (int)blockIdx.y * FMY;
    const int k0 = (int)blockIdx.z * FMZ, k1 = min(k0 + FMZ, g.S[2]);
    // issue the loads of plane kk (stored z index, k0 - 1 .. k1); they complete while the
    // previous plane is computed
    auto fetch = [&](int kk, PlaneRegs<R>& r) {
        const int kz = nb(kk, 0, g.S[2], g.per[2]);
#pragma unroll
        for (int m = 0; m < 2; m++) {
            const int i = tid + m * NT;
            const int lx = i % FPX, ly = i / FPX;
            const int xr = x0 - 1 + lx, yr = y0 - 1 + ly;
            const int x = nb(xr, 0, g.S[0], g.per[0]), y = nb(yr, 0, g.S[1], g.per[1]);
            r.ok[m] = i < FPP && x >= 0 && y >= 0 && kz >= 0;
            r.own[m] = lx >= 1 && lx <= FMX && ly >= 1 && ly <= FMY && xr < g.S[0] && yr < g.S[1] && kk >= k0 &&
                       kk < k1;
            r.o[m] = r.ok[m] ? o3(g, x, y, kz) : 0;
#pragma unroll
            for (int c = 0; c < 3; c++) {
                r.e[m][c] = r.ok[m] ? f.E[c][r.o[m]] : R(0);
                if constexpr (FRIED) {
                    r.eo[m][c] = r.ok[m] ? f.Eo[c][r.o[m]] : R(0);
                    r.eb[m][c] = r.ok[m] ? f.Eb[c][r.o[m]] : R(0);
                }
            }
        }
    };
    // E-tilde of the fetched plane into its ring slot (kk - k0 + 1) mod 3; the owner of each
    // cell stores the new Ebar
    auto store = [&](int kk, const PlaneRegs<R>& r) {
        const int sl = (kk - k0 + 1) % 3;
#pragma unroll
        for (int m = 0; m < 2; m++) {
            const int i = tid + m * NT;
            if (i >= FPP) continue;
#pragma unroll
            for (int c = 0; c < 3; c++) {
                R v = r.e[m][c];
                if constexpr (FRIED) {
                    const R eo = r.eo[m][c];
                    const R eb = (R(1) - R(0.5) * th) * eo + R(0.5) * th * r.eb[m][c];
                    v = (R(1) + R(0.25) * th) * r.e[m][c] - R(0.5) * eo + (R(0.5) - R(0.25) * th) * eb;
                    if (r.ok[m] && r.own[m]) f.T[c][r.o[m]] = eb;
                }
                sT[sl][c][i] = r.ok[m] ? v : R(0);
            }
        }
    };
    PlaneRegs<R> pr;
    fetch(k0 - 1, pr);
    store(k0 - 1, pr);
    fetch(k0, pr);
    store(k0, pr);
    fetch(k0 + 1, pr);
    const int q0 = x0 + (int)threadIdx.x, q1 = y0 + (int)threadIdx.y;
    const int cx = (int)threadIdx.x + 1, cy = (int)threadIdx.y + 1;
    for (int k = k0; k < k1; k++) {
        store(k + 1, pr);
        __syncthreads();
        if (k + 2 <= k1) fetch(k + 2, pr);
        if (q0 < g.S[0] && q1 < g.S[1]) {
            const int q[3] = {q0, q1, k};
            const long o = o3(g, q0, q1, k);
            const int sl[3] = {(k - k0) % 3, (k - k0 + 1) % 3, (k - k0 + 2) % 3};
            faraday_cell<0>(g, f, pml, sT, sl, q, o, cx, cy, a, b, cg, dt);
            faraday_cell<1>(g, f, pml, sT, sl, q, o, cx, cy, a, b, cg, dt);
            faraday_cell<2>(g, f, pml, sT, sl, q, o, cx, cy, a, b, cg, dt);
        }
        __syncthreads();
    }
}

// dE_C/dt = Delta_A1 B_A2 - Delta_A2 B_A1 - J_C; E_C sits on a half node along C, nodes along
// A1, A2, so each difference takes B at the cell and one cell below; conducting walls keep the
// tangential components at 0 (nodes 0 and S-1 of a non-periodic axis stay untouched).  A
// workgroup owns a 32 x 8 (x, y) tile and FMZ planes and marches up z with planes k - 1 and k of
// B (and the cells one below in x and y) in LDS, loading plane k + 1 while computing plane k.
constexpr int APX = FMX + 1, APP = (FMX + 1) * (FMY + 1);

template <int C, typename R>
__device__ __forceinline__ void ampere_cell(const G3& g, const F3<R>& f, const R* const* J, const Pml3& pml,
                                            const R (*sB)[3][APP], int s0, int s1, const int q[3], long o, int cx,
                                            int cy, R dt)
{
    constexpr int A1 = (C + 1) % 3, A2 = (C + 2) % 3;
    const int h[3] = {C == 0 ? 1 : 0, C == 1 ? 1 : 0, C == 2 ? 1 : 0};
    const R old = f.E[C][o];
    f.Eo[C][o] = old;
#pragma unroll
    for (int d = 0; d < 3; d++) {
        if (g.per[d]) continue;
        if (q[d] < (h[d] ? 0 : 1) || q[d] > g.S[d] - 2) return;
    }
    // B at the cell and one cell below along axis ax
    auto diff = [&](int comp, int ax) {
        const R hi = sB[s1][comp][cy * APX + cx];
        const R lo = ax == 0 ? sB[s1][comp][cy * APX + cx - 1]
                             : (ax == 1 ? sB[s1][comp][(cy - 1) * APX + cx] : sB[s0][comp][cy * APX + cx]);
        return (hi - lo) / (R)g.d[ax];
    };
    const R t1 = diff(A2, A1) - J[C][o];
    const R t2 = -diff(A1, A2);
    f.E[C][o] = split_update<A1, A2>(old, f.SE[C], o, t1, t2, pml, q, h, dt);
}

template <typename R>
__global__ void __launch_bounds__(NT) k3_ampere(G3 g, F3<R> f, const R* J0, const R* J1, const R* J2, Pml3 pml, R dt)
{
    static_assert(APP <= 2 * NT, "a thread loads at most two cells of a padded plane");
    __shared__ R sB[2][3][APP];
    const R* J[3] = {J0, J1, J2};
    const int tid = (int)(threadIdx.y * FMX + threadIdx.x);
    const int x0 = (int)blockIdx.x * FMX, y0 = (int)blockIdx.y * FMY;
    const int k0 = (int)blockIdx.z * FMZ, k1 = min(k0 + FMZ, g.S[2]);
    R rv[2][3];
    auto fetch = [&](int kk) {
        const int kz = nb(kk, 0, g.S[2], g.per[2]);
#pragma unroll
        for (int m = 0; m < 2; m++) {
            const int i = tid + m * NT;
            const int lx = i % APX, ly = i / APX;
            const int x = nb(x0 - 1 + lx, 0, g.S[0], g.per[0]), y = nb(y0 - 1 + ly, 0, g.S[1], g.per[1]);
            const bool ok = i < APP && x >= 0 && y >= 0 && kz >= 0;
            const long o = ok ? o3(g, x, y, kz) : 0;
#pragma unroll
            for (int c = 0; c < 3; c++) rv[m][c] = ok ? f.B[c][o] : R(0);
        }
    };
    auto store = [&](int kk) {
        const int sl = (kk - k0 + 1) & 1;
#pragma unroll
        for (int m = 0; m < 2; m++) {
            const int i = tid + m * NT;
            if (i >= APP) continue;
#pragma unroll
            for (int c = 0; c < 3; c++) sB[sl][c][i] = rv[m][c];
        }
    };
    fetch(k0 - 1);
    store(k0 - 1);
    fetch(k0);
    const int q0 = x0 + (int)threadIdx.x, q1 = y0 + (int)threadIdx.y;
    const int cx = (int)threadIdx.x + 1, cy = (int)threadIdx.y + 1;
    for (int k = k0; k < k1; k++) {
        store(k);
        __syncthreads();
        if (k + 1 < k1) fetch(k + 1);
        if (q0 < g.S[0] && q1 < g.S[1]) {
            const int q[3] = {q0, q1, k};
            const long o = o3(g, q0, q1, k);
            const int s0 = (k - k0) & 1, s1 = (k - k0 + 1) & 1;
            ampere_cell<0>(g, f, J, pml, sB, s0, s1, q, o, cx, cy, dt);
            ampere_cell<1>(g, f, J, pml, sB, s0, s1, q, o, cx, cy, dt);
            ampere_cell<2>(g, f, J, pml, sB, s0, s1, q, o, cx, cy, dt);
        }
        __syncthreads();
    }
}

// ---- current filter: all passes along one axis in LDS ------------------------------------------
// A workgroup holds a segment of tseg cells along AX plus the reach on both sides, for BC lines
// (AX = x: BC whole x lines; AX = y, z: BC consecutive x columns, so every load and store is a
// contiguous run of x).  It runs the pass sequence in LDS, ping-ponging between two buffers:
// each pass is phi_j <- alpha phi_j + (1 - alpha)(phi_{j-s} + phi_{j+s}) / 2, positions beyond
// the component's stored range held at 0 after every pass (zero padding; periodic axes wrap).
// Positions beyond the segment's halo read 0; the error that causes moves inwards by at most
// one stride per pass, so the tseg central cells are exact.  Cells beyond the component's range
// (its last half node on a non-periodic axis) are copied.
template <typename TI, typename TO>
struct Lines3 {
    const TI* in[3];
    TO* out[3];
    int h[3];                          // stagger of each component along the launch's axis
};

template <int AX> constexpr int fline_bc() { return AX == 0 ? 8 : 32; }

template <int AX, typename TI, typename TO, typename T>
__global__ void __launch_bounds__(NT) k3_fline(G3 g, Lines3<TI, TO> L, FiltSeq fs, int tseg, int nseg, int ncolb)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    constexpr int BC = fline_bc<AX>();
    constexpr int TPC = NT / BC;                  // threads per line (x) or per column (y, z)
    const int R = fs.reach;
    const int A = tseg + 2 * R;
    const int ld = AX == 0 ? A + 1 : BC + 1;
    T* src = reinterpret_cast<T*>(smem_raw);
    T* dst = src + (AX == 0 ? BC * ld : A * ld);
    // block -> (component, segment, column block, plane or row across)
    int bid = (int)blockIdx.x;
    const int nother = AX == 0 ? 1 : g.S[AX == 1 ? 2 : 1];
    const int per_comp = nseg * ncolb * nother;
    const int c = bid / per_comp;
    bid -= c * per_comp;
    const int seg = bid % nseg;
    bid /= nseg;
    const int cb = bid % ncolb;
    const int other = bid / ncolb;
    const TI* __restrict__ in = L.in[c];
    TO* __restrict__ out = L.out[c];
    const int S = g.S[AX], per = g.per[AX];
    const int hi = per ? S - 1 : S - 1 - L.h[c];
    const int seg0 = seg * tseg;
    // this thread's line / column and first row; the HBM offset of position jj along AX is
    // base + jj * step, with the z ring applied to whichever index runs along z
    const int col = AX == 0 ? (int)threadIdx.x / TPC : (int)threadIdx.x % BC;
    const int a0 = AX == 0 ? (int)threadIdx.x % TPC : (int)threadIdx.x / BC;
    bool ok;
    long base = 0;
    if (AX == 0) {
        const int l = cb * BC + col;
        ok = l < g.S[1] * g.S[2];
        const int jy = ok ? l % g.S[1] : 0, k = ok ? l / g.S[1] : 0;
        base = o3(g, 0, jy, k);
    } else {
        const int x = cb * BC + col;
        ok = x < g.S[0];
        base = AX == 1 ? o3(g, ok ? x : 0, 0, other) : (long)other * g.pitch + (ok ? x : 0);
    }
    auto at = [&](int jj) -> long {           // 0 <= jj < S
        if (AX == 0) return base + jj;
        if (AX == 1) return base + (long)jj * g.pitch;
        int kk = jj + g.zoff;
        if (kk >= g.S[2]) kk -= g.S[2];
        return base + (long)kk * g.plane;
    };
    auto wrap = [&](int j) {
        if (j >= 0 && j < S) return j;
        int jj = j % S;
        return jj < 0 ? jj + S : jj;
    };
    auto idx = [&](int a) { return AX == 0 ? col * ld + a : a * ld + col; };
    for (int a = a0; a < A; a += TPC) {
        const int j = seg0 - R + a;
        T v = T(0);
        if (ok && (per || (j >= 0 && j <= hi))) v = (T)in[at(per ? wrap(j) : j)];
        src[idx(a)] = v;
    }
    __syncthreads();
    for (int p = 0; p < fs.n; p++) {
        const T al = (T)fs.alpha[p], be = (T(1) - al) * T(0.5);
        const int st = fs.stride[p];
        for (int a = a0; a < A; a += TPC) {
            const int j = seg0 - R + a;
            const T l = a >= st ? src[idx(a - st)] : T(0);
            const T r = a + st < A ? src[idx(a + st)] : T(0);
            const T v = al * src[idx(a)] + be * (l + r);
            dst[idx(a)] = (per || (j >= 0 && j <= hi)) ? v : T(0);
        }
        __syncthreads();
        T* t = src;
        src = dst;
        dst = t;
    }
    if (!ok) return;
    for (int a = a0; a < tseg; a += TPC) {
        const int j = seg0 + a;
        if (j >= S) break;
        const long o = at(j);
        out[o] = (per || j <= hi) ? (TO)src[idx(a + R)] : (TO)in[o];
    }
}

// ---- current filter: the three axes in one launch ---------------------------------------------
// For a sequence of unit-stride passes the whole sequence along one axis is one symmetric stencil
// of 2 reach + 1 taps (the product of the passes), c[m] weighting the values m cells to either
// side.  Holding the positions just outside a component's range at zero after every pass is the
// same as applying that stencil to the line continued oddly about those two positions (-1 and
// hi + 1): a symmetric pass keeps an odd continuation odd, so the two pivots stay at zero and
// nothing else outside is ever read.  The edges therefore need no coefficients of their own.
// The filter is separable, so the three axes commute and are applied x, y, z as the line passes
// do.  A workgroup owns an FT_TX x FT_TY tile of (x, y) columns of one component and a run of
// z planes.  For each plane it stages the tile with its x and y reach in LDS (the odd
// continuation is built by the loads), filters along x, then along y, and keeps its columns'
// last 2 reach + 1 filtered planes in registers for the z stencil; the continuation along z is
// made from the planes already in that ring.  A component's cells beyond its range (the last
// half node of its own axis when that axis is not periodic) are copied along that axis: the x
// copy column and the y copy row are staged beside the tile, the z copy plane is written as it
// is filtered.  Consecutive work items (neighbouring y tiles at the same z run) go to the same
// XCD so that the reach they share is read once from its L2.
constexpr int FT_TX = 32, FT_TY = 32, FT_QY = 4, FT_NT = 256, FT_RMAX = 6;
static_assert(FT_TX * FT_TY == FT_NT * FT_QY, "one thread per x column and FT_QY rows");

struct FiltStencil {
    double c[FT_RMAX + 1];
};

template <typename T> struct Vec16;
template <> struct Vec16<float> {
    typedef float type __attribute__((ext_vector_type(4)));
    static constexpr int n = 4;
};
template <> struct Vec16<double> {
    typedef double type __attribute__((ext_vector_type(2)));
    static constexpr int n = 2;
};

// stored index of position p on an axis of S stored cells whose component range is [0, hi],
// under the odd continuation about -1 and hi + 1 (periodic axes wrap); sg = 0 at the pivots and
// where the continuation would leave the range (no output within the reach reads those)
__device__ __forceinline__ int odd_pos(int p, int S, int hi, int per, int& sg)
{
    if (per) {
        sg = 1;
        int j = p % S;
        return j < 0 ? j + S : j;
    }
    if (p >= 0 && p <= hi) {
        sg = 1;
        return p;
    }
    const int q = p < 0 ? -2 - p : 2 * (hi + 1) - p;
    sg = (p == -1 || p == hi + 1 || q < 0 || q > hi) ? 0 : -1;
    return sg ? q : 0;
}

// calls f(std::integral_constant<int, K>) for the K == k among 0 <= K < N (k uniform: the
// choice is a scalar branch and every K is a compile-time constant in its body)
template <int K, int N, typename F>
__device__ __forceinline__ void static_switch(int k, F&& f)
{
    if constexpr (K < N) {
        if (k == K) f(std::integral_constant<int, K>{});
        else static_switch<K + 1, N>(k, f);
    }
}

template <int RC, typename T>
struct FtGeom {
    static constexpr int VW = Vec16<T>::n;
    static constexpr int RW = FT_TY + 2 * RC;                     // staged rows (+1 copy row)
    static constexpr int NRD = (2 * RC + 4 + VW - 1) / VW;        // vector reads per x item
    static constexpr int W0 = FT_TX + 2 * RC > FT_TX - 4 + NRD * VW ? FT_TX + 2 * RC : FT_TX - 4 + NRD * VW;
    static constexpr int LA = (W0 + VW - 1) / VW * VW;            // staged columns = row pitch
    static constexpr int NMAIN = (RW + 1) * LA;                   // tile + copy row
    static constexpr int CXB = NMAIN;                             // copy column after them
    static constexpr int NLOAD = NMAIN + RW;
    static constexpr int NSLOT = (NLOAD + FT_NT - 1) / FT_NT;
    static constexpr int DUMMY = NLOAD;                           // sink of unused slots
    static constexpr int NA = DUMMY + 1;
    static constexpr int NB = (RW + 1) * FT_TX;
};

template <int RC, typename T, typename TO>
__global__ void __launch_bounds__(FT_NT) k3_filt3(G3 g, Lines3<double, TO> L, FiltStencil st, int seg, int nzs,
                                                  int nwork, int nxt, int nyt)
{
    using Gm = FtGeom<RC, T>;
    using V = typename Vec16<T>::type;
    __shared__ __attribute__((aligned(16))) T sA[Gm::NA];
    __shared__ __attribute__((aligned(16))) T sB[Gm::NB];
    // work item w: y tile fastest, then x tile, z run, component; the grid is a multiple of 8
    // and blocks are dealt to the XCDs in turn, so block b works on item (b % 8) n8 + b / 8
    const int n8 = (int)gridDim.x / 8;
    int w = ((int)blockIdx.x % 8) * n8 + (int)blockIdx.x / 8;
    if (w >= nwork) return;
    const int yt = w % nyt;
    w /= nyt;
    const int xt = w % nxt;
    w /= nxt;
    const int zs = w % nzs;
    const int comp = w / nzs;
    const double* __restrict__ in = L.in[comp];
    TO* __restrict__ out = L.out[comp];
    const int S0 = g.S[0], S1 = g.S[1], S2 = g.S[2];
    const int hx = g.per[0] ? S0 - 1 : S0 - 1 - (comp == 0);
    const int hy = g.per[1] ? S1 - 1 : S1 - 1 - (comp == 1);
    const int hz = g.per[2] ? S2 - 1 : S2 - 1 - (comp == 2);
    const int x0 = xt * FT_TX, y0 = yt * FT_TY;
    const bool xcopy = comp == 0 && !g.per[0] && hx + 1 >= x0 && hx + 1 < x0 + FT_TX;
    const bool ycopy = comp == 1 && !g.per[1] && hy + 1 >= y0 && hy + 1 < y0 + FT_TY;
    const int k0 = zs * seg, k1 = min(S2, k0 + seg);
    T c[RC + 1];
#pragma unroll
    for (int m = 0; m <= RC; m++) c[m] = (T)st.c[m];

    // load slots: in-plane offset and sign of the continuation, fixed for the run; slot i lands
    // at LDS index i (rows of LA staged columns, the copy row, the copy column), unused ones in
    // the sink
    unsigned soff[Gm::NSLOT];
    T ssg[Gm::NSLOT];
#pragma unroll
    for (int m = 0; m < Gm::NSLOT; m++) {
        const int i = (int)threadIdx.x + m * FT_NT;
        int sx = 0, sy = 0, ix = 0, iy = 0;
        if (i < Gm::NMAIN) {
            const int r = i / Gm::LA, cc = i % Gm::LA;
            ix = odd_pos(x0 - RC + cc, S0, hx, g.per[0], sx);
            if (r < Gm::RW) iy = odd_pos(y0 - RC + r, S1, hy, g.per[1], sy);
            else if (ycopy) {
                iy = hy + 1;
                sy = 1;
            }
        } else if (i < Gm::NLOAD) {
            const int r = i - Gm::NMAIN;
            if (xcopy) {
                ix = hx + 1;
                sx = 1;
                iy = odd_pos(y0 - RC + r, S1, hy, g.per[1], sy);
            }
        }
        soff[m] = (unsigned)(iy * (int)g.pitch + ix);
        ssg[m] = (T)(sx * sy);
    }
    double pre[Gm::NSLOT];
    auto fetch = [&](int p) {           // logical plane p, 0 <= p < S2 unless z is periodic
        int kk = p % S2;
        if (kk < 0) kk += S2;
        kk += g.zoff;
        if (kk >= S2) kk -= S2;
        const double* src = in + (long)kk * g.plane;
#pragma unroll
        for (int m = 0; m < Gm::NSLOT; m++)
            if (ssg[m] != T(0)) pre[m] = src[soff[m]];
    };
    auto stage = [&]() {
#pragma unroll
        for (int m = 0; m < Gm::NSLOT; m++) {
            const int i = (int)threadIdx.x + m * FT_NT;
            sA[(m + 1) * FT_NT <= Gm::NLOAD || i < Gm::NLOAD ? i : Gm::DUMMY] =
                ssg[m] != T(0) ? ssg[m] * (T)pre[m] : T(0);
        }
    };
    // x stencil on every staged row (the copy row only when it is staged) into sB
    auto xfilter = [&]() {
        constexpr int NQ = FT_TX / 4;
        const int nrow = ycopy ? Gm::RW + 1 : Gm::RW;
        for (int it = (int)threadIdx.x; it < nrow * NQ; it += FT_NT) {
            const int r = it / NQ, xq = it % NQ;
            T a[Gm::NRD * Gm::VW];
            const T* row = sA + r * Gm::LA + 4 * xq;
#pragma unroll
            for (int v = 0; v < Gm::NRD; v++) {
                const V t = *reinterpret_cast<const V*>(row + v * Gm::VW);
#pragma unroll
                for (int e = 0; e < Gm::VW; e++) a[v * Gm::VW + e] = t[e];
            }
            T o[4];
#pragma unroll
            for (int q = 0; q < 4; q++) {
                T s = c[0] * a[q + RC];
#pragma unroll
                for (int m = 1; m <= RC; m++) s += c[m] * (a[q + RC - m] + a[q + RC + m]);
                o[q] = s;
            }
            if (xcopy) {
#pragma unroll
                for (int q = 0; q < 4; q++)
                    if (x0 + 4 * xq + q == hx + 1) o[q] = r < Gm::RW ? sA[Gm::CXB + r] : T(0);
            }
            T* dst = sB + r * FT_TX + 4 * xq;
#pragma unroll
            for (int v = 0; v < 4 / Gm::VW; v++) {
                V t;
#pragma unroll
                for (int e = 0; e < Gm::VW; e++) t[e] = o[v * Gm::VW + e];
                *reinterpret_cast<V*>(dst + v * Gm::VW) = t;
            }
        }
    };
    // y stencil for this thread's column x0 + tx, rows y0 + FT_QY ty + q
    const int tx = (int)threadIdx.x % FT_TX, ty = (int)threadIdx.x / FT_TX;
    auto yfilter = [&](T v[FT_QY]) {
        T b[FT_QY + 2 * RC];
#pragma unroll
        for (int i = 0; i < FT_QY + 2 * RC; i++) b[i] = sB[(FT_QY * ty + i) * FT_TX + tx];
#pragma unroll
        for (int q = 0; q < FT_QY; q++) {
            T s = c[0] * b[q + RC];
#pragma unroll
            for (int m = 1; m <= RC; m++) s += c[m] * (b[q + RC - m] + b[q + RC + m]);
            v[q] = s;
        }
        if (ycopy) {
#pragma unroll
            for (int q = 0; q < FT_QY; q++)
                if (y0 + FT_QY * ty + q == hy + 1) v[q] = sB[Gm::RW * FT_TX + tx];
        }
    };
    // one plane through x and y; prefetches plane pn when pn is not -1 << 30
    constexpr int NOPLANE = -(1 << 30);
    auto plane = [&](T v[FT_QY], int pn) {
        stage();
        __syncthreads();
        if (pn != NOPLANE) fetch(pn);
        xfilter();
        __syncthreads();
        yfilter(v);
    };
    // the z ring: plane p sits in slot (p - p0) mod NR, p0 the run's first plane, so that a plane
    // is written once and never moved; the slot is uniform and selected by a scalar branch
    constexpr int NR = 2 * RC + 1;
    T rg[FT_QY][NR];
#pragma unroll
    for (int q = 0; q < FT_QY; q++)
#pragma unroll
        for (int i = 0; i < NR; i++) rg[q][i] = T(0);
    const int xg = x0 + tx;
    unsigned coff[FT_QY];               // in-plane offsets of this thread's columns
#pragma unroll
    for (int q = 0; q < FT_QY; q++) coff[q] = (unsigned)((y0 + FT_QY * ty + q) * (int)g.pitch + xg);
    auto store_out = [&](int j, int q, T v) {
        const int yg = y0 + FT_QY * ty + q;
        if (xg >= S0 || yg >= S1) return;
        int kk = j + g.zoff;
        if (kk >= S2) kk -= S2;
        (out + (long)kk * g.plane)[coff[q]] = (TO)v;
    };
    // plane j from the ring, its centre in slot C
    auto emit_at = [&](auto cc, int j) {
        constexpr int C = decltype(cc)::value;
        if (j < k0 || j >= k1 || j > hz) return;
#pragma unroll
        for (int q = 0; q < FT_QY; q++) {
            T s = c[0] * rg[q][C];
#pragma unroll
            for (int m = 1; m <= RC; m++) s += c[m] * (rg[q][(C + NR - m) % NR] + rg[q][(C + m) % NR]);
            store_out(j, q, s);
        }
    };
    const bool per = g.per[2] != 0;
    const bool first = !per && k0 == 0;
    const int p0 = first ? 0 : k0 - RC;
    const int plast = per ? k1 - 1 + RC : min(k1 - 1 + RC, hz);
    T v[FT_QY];
    int p = p0, slot = 0;
    fetch(p);
    for (; p <= plast; p++) {
        plane(v, p < plast ? p + 1 : NOPLANE);
        static_switch<0, NR>(slot, [&](auto kc) {
            constexpr int K = decltype(kc)::value;
#pragma unroll
            for (int q = 0; q < FT_QY; q++) rg[q][K] = v[q];
            if (K == RC && first && p == RC) {
                // planes -1 .. -RC (slots NR - 1 .. NR - RC, not yet used): the pivot and the odd
                // continuation of planes 0 .. RC - 2 (slots 0 .. RC - 2)
#pragma unroll
                for (int q = 0; q < FT_QY; q++) {
                    rg[q][NR - 1] = T(0);
#pragma unroll
                    for (int i = 1; i < RC; i++) rg[q][(NR - 1 - i) % NR] = -rg[q][(i - 1 + NR) % NR];
                }
            }
            emit_at(std::integral_constant<int, (K + NR - RC) % NR>{}, p - RC);
        });
        slot = slot + 1 == NR ? 0 : slot + 1;
    }
    if (!per && k1 - 1 + RC > hz) {
        // the far end: put the ring in shift-register order (rg[q][NR - 1] the newest plane,
        // hz), then push the pivot plane hz + 1 and the continuation hz + 1 + m = -(hz + 1 - m)
        static_switch<0, NR>(slot, [&](auto kc) {
            constexpr int K = decltype(kc)::value;      // the oldest plane's slot
            T t[FT_QY][NR];
#pragma unroll
            for (int q = 0; q < FT_QY; q++)
#pragma unroll
                for (int i = 0; i < NR; i++) t[q][i] = rg[q][(K + i) % NR];
#pragma unroll
            for (int q = 0; q < FT_QY; q++)
#pragma unroll
                for (int i = 0; i < NR; i++) rg[q][i] = t[q][i];
        });
        auto push = [&](const T w[FT_QY]) {
#pragma unroll
            for (int q = 0; q < FT_QY; q++) {
#pragma unroll
                for (int i = 0; i < NR - 1; i++) rg[q][i] = rg[q][i + 1];
                rg[q][NR - 1] = w[q];
            }
        };
        if (comp == 2) {                // the copy plane of the z component
            fetch(hz + 1);
            plane(v, NOPLANE);
            if (hz + 1 >= k0 && hz + 1 < k1) {
#pragma unroll
                for (int q = 0; q < FT_QY; q++) store_out(hz + 1, q, v[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < FT_QY; q++) v[q] = T(0);
        push(v);
        emit_at(std::integral_constant<int, RC>{}, hz + 1 - RC);
#pragma unroll
        for (int m = 1; m < RC; m++) {
#pragma unroll
            for (int q = 0; q < FT_QY; q++) v[q] = -rg[q][NR - 2 * m];
            push(v);
            emit_at(std::integral_constant<int, RC>{}, hz + 1 + m - RC);
        }
    }
}

__global__ void __launch_bounds__(NT) k3_zero3(G3 g, double* a, double* b, double* c)
{
    int q[3];
    if (!cell_of(g, q)) return;
    const long o = o3(g, q[0], q[1], q[2]);
    a[o] = 0.0;
    b[o] = 0.0;
    c[o] = 0.0;
}

// ---- particles --------------------------------------------------------------------------------

// cubic B-spline weights of nodes j0-1 .. j0+2 for a particle at fraction f of cell j0
template <typename R>
__device__ __forceinline__ void bspline4(R f, R w[4])
{
    const R g = R(1) - f, f2 = f * f, f3 = f2 * f, sixth = R(1) / R(6);
    w[0] = g * g * g * sixth;
    w[1] = (R(3) * f3 - R(6) * f2 + R(4)) * sixth;
    w[2] = (-R(3) * f3 + R(3) * f2 + R(3) * f + R(1)) * sixth;
    w[3] = f3 * sixth;
}

// the same weights on the 5-node window starting one node below the particle's (hi = false)
// or two below (hi = true), FP64 (Esirkepov)
__device__ __forceinline__ void window5(double f, bool hi, double s[5])
{
    const double g = 1.0 - f, f2 = f * f, f3 = f2 * f, sixth = 1.0 / 6.0;
    const double w0 = g * g * g * sixth, w1 = (3.0 * f3 - 6.0 * f2 + 4.0) * sixth;
    const double w2 = (-3.0 * f3 + 3.0 * f2 + 3.0 * f + 1.0) * sixth, w3 = f3 * sixth;
    s[0] = hi ? 0.0 : w0;
    s[1] = hi ? w0 : w1;
    s[2] = hi ? w1 : w2;
    s[3] = hi ? w2 : w3;
    s[4] = hi ? w3 : 0.0;
}

// gather of E^n and B^n = (B^{n-1/2} + B^{n+1/2}) / 2 at r (cells), cubic weights at each
// component's stagger
template <bool MC, typename R>
__device__ void gather3(const G3& g, const F3<R>& f, const double r[3], R E[3], R B[3])
{
    R w[3][2][4];
    int id[3][2][4];
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const double xs = r[a] - 0.5 * h;
            const int j0 = (int)floor(xs);
            bspline4((R)(xs - j0), w[a][h]);
#pragma unroll
            for (int m = 0; m < 4; m++) id[a][h][m] = sidx(g, a, j0 - 1 + m);
        }
#pragma unroll
    for (int c = 0; c < 6; c++) {
        int hx = c < 3 ? (c == 0) : (c != 3), hy = c < 3 ? (c == 1) : (c != 4), hz = c < 3 ? (c == 2) : (c != 5);
        if (MC) hx = hy = hz = 0;
        R acc = R(0), acc2 = R(0);
        const R* F = MC ? f.G[c] : (c < 3 ? f.E[c] : f.B[c - 3]);
        const R* Fo = c < 3 ? f.E[c] : f.Bo[c - 3];
        for (int k = 0; k < 4; k++) {
            const int sk = id[2][hz][k];
            if (sk < 0) continue;
            for (int j = 0; j < 4; j++) {
                const int sj = id[1][hy][j];
                if (sj < 0) continue;
                const R wjk = w[1][hy][j] * w[2][hz][k];
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    const int si = id[0][hx][i];
                    if (si < 0) continue;
                    const long o = o3(g, si, sj, sk);
                    acc += w[0][hx][i] * wjk * F[o];
                    if (!MC && c >= 3) acc2 += w[0][hx][i] * wjk * Fo[o];
                }
            }
        }
        if (c < 3) E[c] = acc;
        else B[c - 3] = MC ? acc : R(0.5) * (acc + acc2);
    }
}

// Esirkepov's 3D deposit of one particle moving r0 -> r1 (cells, |move| < 1 cell per axis):
//   W_C = DS_C (S0_A1 S0_A2 + DS_A1 S0_A2 / 2 + S0_A1 DS_A2 / 2 + DS_A1 DS_A2 / 3),
//   J_C(node + 1/2) - J_C(node - 1/2) = k_C W_C   (k_C = -q w / (d_A1 d_A2 dt))
__device__ void esirkepov3(const G3& g, double* const* J, const double r0[3], const double r1[3], const double k[3])
{
    double S0[3][5], DS[3][5];
    int base[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const int i0 = (int)floor(r0[a]), i1 = (int)floor(r1[a]);
        const int b = min(i0, i1) - 1;
        base[a] = b;
        double s1[5];
        window5(r0[a] - i0, i0 > b + 1, S0[a]);
        window5(r1[a] - i1, i1 > b + 1, s1);
#pragma unroll
        for (int m = 0; m < 5; m++) DS[a][m] = s1[m] - S0[a][m];
    }
#pragma unroll
    for (int c = 0; c < 3; c++) {
        if (k[c] == 0.0) continue;
        const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
        int sc[4];
#pragma unroll
        for (int m = 0; m < 4; m++) sc[m] = sidx(g, c, base[c] + m);
        for (int m1 = 0; m1 < 5; m1++) {
            const int s1 = sidx(g, a1, base[a1] + m1);
            if (s1 < 0) continue;
            for (int m2 = 0; m2 < 5; m2++) {
                const int s2 = sidx(g, a2, base[a2] + m2);
                if (s2 < 0) continue;
                const double T = S0[a1][m1] * S0[a2][m2] + 0.5 * DS[a1][m1] * S0[a2][m2] +
                                 0.5 * S0[a1][m1] * DS[a2][m2] + DS[a1][m1] * DS[a2][m2] * (1.0 / 3.0);
                if (T == 0.0) continue;
                double acc = 0.0;
#pragma unroll
                for (int mc = 0; mc < 4; mc++) {
                    acc += k[c] * DS[c][mc] * T;
                    if (acc == 0.0 || sc[mc] < 0) continue;
                    int q[3];
                    q[c] = sc[mc];
                    q[a1] = s1;
                    q[a2] = s2;
                    atomicAdd(&J[c][o3(g, q[0], q[1], q[2])], acc);
                }
            }
        }
    }
}

template <typename R>
__device__ __forceinline__ R rsq(R x)
{
    if constexpr (sizeof(R) == 4) return __builtin_amdgcn_rsqf(x);
    else return 1.0 / sqrt(x);
}

// ---- particles: segments staged in LDS --------------------------------------------------------
//
// One workgroup per particle segment: a tile of the last sort, or a transverse chunk of a
// plane injected since.  The segment's cell box, widened by the stencil reach (2 cells below,
// 3 above), is staged in LDS: E^n and B^n = (B^{n-1/2} + B^{n+1/2}) / 2 in the run's type and a
// zeroed current accumulator.  Each thread gathers, pushes and deposits its particles into
// the accumulator, then the box is added to the FP64 current in HBM with one atomic per cell
// and component.  FP32 runs accumulate in 64-bit integer fixed point, exact and independent
// of the order of the adds: a contribution v becomes round(v / q), q = max|k| sum|w| / 2^46
// over the segment, through one FMA with 1.5 * 2^52 whose bit pattern is 0x4338000000000000 +
// round(v / q); the low 48 bits of the raw sum, sign-extended, are the exact sum.  FP64 runs
// add in FP64.  A particle whose cell lies outside its segment's box, and every particle of a
// segment whose box exceeds the LDS pitches, takes the same steps on the fields and current
// in HBM.

constexpr int GT = 768;        // threads of an electron segment workgroup
constexpr int GTI = 256;       // threads of an ion segment workgroup
constexpr int HBM_GRID = 1024; // workgroups of the pass over the particles left to HBM
constexpr int BPX = BOX_PX, BPY = BOX_PY, BPL = BOX_PL;

template <typename R> struct Acc3 { using T = double; static constexpr bool fixed = false; };
template <> struct Acc3<float> { using T = unsigned long long; static constexpr bool fixed = true; };
constexpr double FX_MAGIC = 6755399441055744.0;   // 1.5 * 2^52
constexpr double FX_RANGE = 70368744177664.0;     // 2^46

__device__ __forceinline__ double fx_value(unsigned long long t)
{
    return (double)((long long)(t << 16) >> 16);
}

// stride of axis a in the LDS box (cells)
__host__ __device__ constexpr int bstride(int a) { return a == 0 ? 1 : (a == 1 ? BPX : BPL); }

template <typename R>
struct BoxL {
    using JT = typename Acc3<R>::T;
    JT* j;         // current planes of n cells (3 for electrons, J_z only for ions)
    R* f;          // 6 field planes of n cells: E x, y, z and B x, y, z (time-centred)
    int n;         // cells per plane: BPL * planes
    int lo[3];     // interior cell index of box cell (0, 0, 0)
    int ext[3];    // box extent (cells)
};

template <typename R>
__device__ __forceinline__ void jadd(typename Acc3<R>::T* p, double a, double b)
{
    if constexpr (Acc3<R>::fixed) atomicAdd(p, (unsigned long long)__double_as_longlong(fma(a, b, FX_MAGIC)));
    else atomicAdd(p, a * b);
}

template <typename R>
__device__ __forceinline__ double jvalue(typename Acc3<R>::T t, double jq)
{
    if constexpr (Acc3<R>::fixed) return fx_value(t) * jq;
    else return t;
}

// the cell of r and its stencils lie inside the box
template <typename R>
__device__ __forceinline__ bool in_box(const BoxL<R>& bx, const double r[3])
{
    bool in = true;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const int c = (int)floor(r[a]);
        in = in && c - 2 >= bx.lo[a] && c + 3 < bx.lo[a] + bx.ext[a];
    }
    return in;
}

// gather of E^n, B^n at r from the staged box, cubic weights at each component's stagger
template <bool MC, typename R>
__device__ __forceinline__ void gather_box(const BoxL<R>& bx, const double r[3], R E[3], R B[3])
{
    R w[3][2][4];
    int ob[3][2];
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const double xs = r[a] - 0.5 * h;
            const int j0 = (int)floor(xs);
            bspline4((R)(xs - j0), w[a][h]);
            ob[a][h] = (j0 - 1 - bx.lo[a]) * bstride(a);
        }
#pragma unroll
    for (int c = 0; c < 6; c++) {
        const int hx = MC ? 0 : (c < 3 ? (c == 0) : (c != 3)), hy = MC ? 0 : (c < 3 ? (c == 1) : (c != 4)),
                  hz = MC ? 0 : (c < 3 ? (c == 2) : (c != 5));
        const R* F = bx.f + c * bx.n + ob[0][hx] + ob[1][hy] + ob[2][hz];
        R acc = R(0);
#pragma unroll
        for (int k = 0; k < 4; k++) {
            R tk = R(0);
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const R* row = F + j * BPX + k * BPL;
                const R rr = w[0][hx][0] * row[0] + w[0][hx][1] * row[1] + w[0][hx][2] * row[2] + w[0][hx][3] * row[3];
                tk += w[1][hy][j] * rr;
            }
            acc += w[2][hz][k] * tk;
        }
        if (c < 3) E[c] = acc;
        else B[c - 3] = acc;
    }
}

// Esirkepov's 3D deposit into the box: with (C, A1, A2) cyclic and T = S0_A1 (S0_A2 + DS_A2 / 2)
// + DS_A1 (S0_A2 / 2 + DS_A2 / 3) (the four-term weight regrouped), J_C at node base + m along
// C gains k_C (DS_C[0] + ... + DS_C[m]) T(m1, m2).  Along an axis that no particle of the wave
// crosses a cell face on, the fifth window node has zero weight and the prefix sum is complete
// at the fourth node: those adds are skipped for the whole wave.
template <typename R>
__device__ __forceinline__ void deposit_box(const BoxL<R>& bx, const double r0[3], const double r1[3],
                                            const double k[3])
{
    double S0[3][5], DS[3][5];
    bool any[3];
    int base = 0;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const int i0 = (int)floor(r0[a]), i1 = (int)floor(r1[a]);
        const int b = min(i0, i1) - 1;
        double s1[5];
        window5(r0[a] - i0, i0 > b + 1, S0[a]);
        window5(r1[a] - i1, i1 > b + 1, s1);
#pragma unroll
        for (int m = 0; m < 5; m++) DS[a][m] = s1[m] - S0[a][m];
        base += (b - bx.lo[a]) * bstride(a);
        any[a] = __ballot(i1 != i0) != 0ull;
    }
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
        double P[5], Q[5], kp[4];
#pragma unroll
        for (int m = 0; m < 5; m++) {
            P[m] = S0[a2][m] + 0.5 * DS[a2][m];
            Q[m] = 0.5 * S0[a2][m] + (1.0 / 3.0) * DS[a2][m];
        }
        double pd = 0.0;
#pragma unroll
        for (int m = 0; m < 4; m++) {
            pd += DS[c][m];
            kp[m] = k[c] * pd;
        }
        typename Acc3<R>::T* J = bx.j + c * bx.n + base;
#pragma unroll
        for (int m1 = 0; m1 < 5; m1++) {
            if (m1 == 4 && !any[a1]) continue;
#pragma unroll
            for (int m2 = 0; m2 < 5; m2++) {
                if (m2 == 4 && !any[a2]) continue;
                const double T = S0[a1][m1] * P[m2] + DS[a1][m1] * Q[m2];
#pragma unroll
                for (int mc = 0; mc < 4; mc++) {
                    if (mc == 3 && !any[c]) continue;
                    jadd<R>(J + mc * bstride(c) + m1 * bstride(a1) + m2 * bstride(a2), kp[mc], T);
                }
            }
        }
    }
}

// the same for a rigid ion moving along z only (x, y fixed): T = Sx Sy on 4 x 4 nodes
template <typename R>
__device__ __forceinline__ void deposit_box_z(const BoxL<R>& bx, double x, double y, double z0, double z1, double kz)
{
    const int ix = (int)floor(x), iy = (int)floor(y), i0 = (int)floor(z0), i1 = (int)floor(z1);
    const int b = min(i0, i1) - 1;
    double Sx[5], Sy[5], S0[5], S1[5], kp[4];
    window5(x - ix, false, Sx);
    window5(y - iy, false, Sy);
    window5(z0 - i0, i0 > b + 1, S0);
    window5(z1 - i1, i1 > b + 1, S1);
    double pd = 0.0;
#pragma unroll
    for (int m = 0; m < 4; m++) {
        pd += S1[m] - S0[m];
        kp[m] = kz * pd;
    }
    typename Acc3<R>::T* J = bx.j + (ix - 1 - bx.lo[0]) + (iy - 1 - bx.lo[1]) * BPX + (b - bx.lo[2]) * BPL;
#pragma unroll
    for (int m1 = 0; m1 < 4; m1++)
#pragma unroll
        for (int m2 = 0; m2 < 4; m2++) {
            const double T = Sx[m1] * Sy[m2];
#pragma unroll
            for (int mc = 0; mc < 4; mc++) jadd<R>(J + mc * BPL + m2 * BPX + m1, kp[mc], T);
        }
}

// box cell (a, b, c) of linear index q = a + ext0 (b + ext1 c), by float reciprocals: q stays below
// 2^16 and the quotients below 64, so (q + 1/2) / d is at least 1/(2 d) from an integer and the
// float product lands on the right side of it
template <typename R>
__device__ __forceinline__ void box_cell(const BoxL<R>& bx, int q, int& a, int& b, int& c)
{
    const int e0 = bx.ext[0], e01 = bx.ext[0] * bx.ext[1];
    c = (int)(((float)q + 0.5f) * (1.0f / (float)e01));
    const int r = q - c * e01;
    b = (int)(((float)r + 0.5f) * (1.0f / (float)e0));
    a = r - b * e0;
}

// stage the box: fields (electrons) and zeroed accumulators (nj planes)
template <int NTH, typename R, bool FIELDS, bool MC = false>
__device__ void stage_box(const G3& g, const F3<R>& f, const BoxL<R>& bx, int nj)
{
    const int L = bx.ext[0] * bx.ext[1] * bx.ext[2];
    for (int q = threadIdx.x; q < L; q += NTH) {
        int a, b, c;
        box_cell(bx, q, a, b, c);
        const int t = a + BPX * b + BPL * c;
        if constexpr (FIELDS) {
            const int si = sidx(g, 0, bx.lo[0] + a), sj = sidx(g, 1, bx.lo[1] + b), sk = sidx(g, 2, bx.lo[2] + c);
            R v[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
            if (si >= 0 && sj >= 0 && sk >= 0) {
                const long o = o3(g, si, sj, sk);
                if constexpr (MC) {
#pragma unroll
                    for (int cc = 0; cc < 6; cc++) v[cc] = f.G[cc][o];
                } else {
#pragma unroll
                    for (int cc = 0; cc < 3; cc++) {
                        v[cc] = f.E[cc][o];
                        v[3 + cc] = R(0.5) * (f.B[cc][o] + f.Bo[cc][o]);
                    }
                }
            }
#pragma unroll
            for (int cc = 0; cc < 6; cc++) bx.f[cc * bx.n + t] = v[cc];
        }
        for (int cc = 0; cc < nj; cc++) bx.j[cc * bx.n + t] = typename Acc3<R>::T(0);
    }
}

// add the box's accumulators to the FP64 current (planes c0 .. c0 + nj - 1 of J)
template <int NTH, typename R>
__device__ void flush_box(const G3& g, const F3<R>& f, const BoxL<R>& bx, int c0, int nj, double jq)
{
    const int L = bx.ext[0] * bx.ext[1] * bx.ext[2];
    for (int q = threadIdx.x; q < L; q += NTH) {
        int a, b, c;
        box_cell(bx, q, a, b, c);
        const int si = sidx(g, 0, bx.lo[0] + a), sj = sidx(g, 1, bx.lo[1] + b), sk = sidx(g, 2, bx.lo[2] + c);
        if (si < 0 || sj < 0 || sk < 0) continue;
        const long o = o3(g, si, sj, sk);
        const int t = a + BPX * b + BPL * c;
        for (int cc = 0; cc < nj; cc++) {
            const double v = jvalue<R>(bx.j[cc * bx.n + t], jq);
            if (v != 0.0) atomicAdd(&f.J[c0 + cc][o], v);
        }
    }
}

template <int NTH>
__device__ __forceinline__ double block_sum3(double v, double* red)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < NTH / 64; w++) t += red[w];
    return t;
}

// min/max of the 6 box bounds over the workgroup, written by thread 0
template <int NTH>
__device__ __forceinline__ void block_box(int nb[6], int (*red)[NTH / 64], Box3* out)
{
#pragma unroll
    for (int q = 0; q < 6; q++)
        for (int o = 32; o > 0; o >>= 1) {
            const int v = __shfl_xor(nb[q], o);
            nb[q] = (q & 1) ? max(nb[q], v) : min(nb[q], v);
        }
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int q = 0; q < 6; q++) red[q][threadIdx.x >> 6] = nb[q];
    __syncthreads();
    if (threadIdx.x == 0) {
        Box3 b;
        for (int a = 0; a < 3; a++) {
            int lo = INT_MAX, hi = INT_MIN;
            for (int w = 0; w < NTH / 64; w++) {
                lo = min(lo, red[2 * a][w]);
                hi = max(hi, red[2 * a + 1][w]);
            }
            b.lo[a] = lo;
            b.hi[a] = hi;
        }
        *out = b;
    }
}

__device__ __forceinline__ void grow(int nb[6], int a, int c)
{
    nb[2 * a] = min(nb[2 * a], c);
    nb[2 * a + 1] = max(nb[2 * a + 1], c);
}

// one electron: gather, Boris push (q/m = -1), deposit, absorption, window rebase; on the
// staged box (LDS) or on the fields and current in HBM.  The staged form returns false,
// leaving the particle untouched, when its cell lies outside the box.
template <bool LDS, bool MC, typename R>
__device__ __forceinline__ bool electron3(const G3& g, const F3<R>& f, const BoxL<R>& bx, const E3<R>& e, int p,
                                          const Push3& pp, double js, int* status, int nb[6])
{
    const R w = e.w[p];
    if (w == R(0)) return true;
    const double r0[3] = {e.x[p], e.y[p], e.z[p]};
    if (LDS && !in_box(bx, r0)) return false;
    R E[3], B[3];
    if constexpr (LDS) gather_box<MC>(bx, r0, E, B);
    else gather3<MC>(g, f, r0, E, B);
    const R h = (R)(-0.5 * pp.dt);
    R ux = e.ux[p], uy = e.uy[p], uz = e.uz[p];
    if (pp.vay) {
        // Vay (Phys. Plasmas 15, 056701): u' = u + (q dt/m)(E + v x B/2), tau = (q dt/2m) B,
        // gamma^2 = (sigma + sqrt(sigma^2 + 4 (tau^2 + (u'.tau)^2)))/2 with sigma = gamma'^2 - tau^2,
        // t = tau/gamma, u = (u' + (u'.t) t + u' x t)/(1 + t^2)
        const R ig0 = rsq(R(1) + ux * ux + uy * uy + uz * uz);
        const R vx = ux * ig0, vy = uy * ig0, vz = uz * ig0;
        const R t0x = h * B[0], t0y = h * B[1], t0z = h * B[2];
        const R upx = ux + R(2) * h * E[0] + (vy * t0z - vz * t0y);
        const R upy = uy + R(2) * h * E[1] + (vz * t0x - vx * t0z);
        const R upz = uz + R(2) * h * E[2] + (vx * t0y - vy * t0x);
        const R us = upx * t0x + upy * t0y + upz * t0z;
        const R tau2 = t0x * t0x + t0y * t0y + t0z * t0z;
        const R sig = R(1) + upx * upx + upy * upy + upz * upz - tau2;
        const R ign = rsq(R(0.5) * (sig + sqrt(sig * sig + R(4) * (tau2 + us * us))));
        const R tx = t0x * ign, ty = t0y * ign, tz = t0z * ign;
        const R sf = R(1) / (R(1) + tx * tx + ty * ty + tz * tz);
        const R ut = upx * tx + upy * ty + upz * tz;
        ux = sf * (upx + ut * tx + (upy * tz - upz * ty));
        uy = sf * (upy + ut * ty + (upz * tx - upx * tz));
        uz = sf * (upz + ut * tz + (upx * ty - upy * tx));
    } else {
        const R umx = ux + h * E[0], umy = uy + h * E[1], umz = uz + h * E[2];
        const R ig = rsq(R(1) + umx * umx + umy * umy + umz * umz);
        const R tx = h * B[0] * ig, ty = h * B[1] * ig, tz = h * B[2] * ig;
        const R sf = R(2) / (R(1) + tx * tx + ty * ty + tz * tz);
        const R sx = sf * tx, sy = sf * ty, sz = sf * tz;
        const R upx = umx + (umy * tz - umz * ty), upy = umy + (umz * tx - umx * tz), upz = umz + (umx * ty - umy * tx);
        ux = umx + (upy * sz - upz * sy) + h * E[0];
        uy = umy + (upz * sx - upx * sz) + h * E[1];
        uz = umz + (upx * sy - upy * sx) + h * E[2];
    }
    const R gi = rsq(R(1) + ux * ux + uy * uy + uz * uz);
    double r1[3] = {r0[0] + pp.dtd[0] * (double)(ux * gi), r0[1] + pp.dtd[1] * (double)(uy * gi),
                    r0[2] + pp.dtd[2] * (double)(uz * gi)};
    bool ok = true;
#pragma unroll
    for (int a = 0; a < 3; a++) ok = ok && fabs(r1[a] - r0[a]) < 1.0;
    if (ok) {
        const double k[3] = {pp.jk[0] * (double)w, pp.jk[1] * (double)w, pp.jk[2] * (double)w};   // q = -1
        if constexpr (LDS) {
            const double ks[3] = {k[0] * js, k[1] * js, k[2] * js};
            deposit_box(bx, r0, r1, ks);
        } else {
            esirkepov3(g, f.J, r0, r1, k);
        }
    } else {
        atomicOr(status, ST3_NONFINITE);
    }
    if (!isfinite((double)(ux + uy + uz))) atomicOr(status, ST3_NONFINITE);
    bool alive = true;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const double L = (double)g.N[a];
        if (g.per[a]) {
            if (r1[a] < 0.0) r1[a] += L;
            else if (r1[a] >= L) r1[a] -= L;
        } else if (r1[a] < 0.0 || r1[a] >= L) {
            alive = false;
        }
    }
    if (!alive) {
        e.w[p] = R(0);
        return true;
    }
    const double zr = r1[2] - pp.shift;
    e.x[p] = r1[0];
    e.y[p] = r1[1];
    e.z[p] = zr;
    e.ux[p] = ux;
    e.uy[p] = uy;
    e.uz[p] = uz;
    grow(nb, 0, (int)floor(r1[0]));
    grow(nb, 1, (int)floor(r1[1]));
    grow(nb, 2, (int)floor(zr));
    return true;
}

template <typename R>
__device__ __forceinline__ void box_of(const Box3& bb, int pz, BoxL<R>& bx, bool& lds)
{
#pragma unroll
    for (int a = 0; a < 3; a++) {
        bx.lo[a] = bb.lo[a] - 2;
        bx.ext[a] = bb.hi[a] - bb.lo[a] + 6;
    }
    bx.n = BPL * pz;
    lds = bx.ext[0] <= BPX && bx.ext[1] <= BPY && bx.ext[2] <= pz;
}

// Staged segments.  A segment whose box exceeds the LDS pitches goes to the list big, a particle
// outside its segment's box to the list mis (segment, particle); k3_gpd_hbm pushes both.
template <typename R, bool MC>
__global__ void __launch_bounds__(GT) k3_gpd(G3 g, F3<R> f, E3<R> e, const Seg3* __restrict__ seg,
                                             const Box3* __restrict__ bin, Box3* __restrict__ bout, Push3 pp, int pz,
                                             int* status, int* big, int* nbig, int2* mis, int* nmis)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem3[];
    __shared__ int red[6][GT / 64];
    __shared__ double redd[GT / 64];
    const Seg3 sg = seg[blockIdx.x];
    const Box3 bb = bin[blockIdx.x];
    int nb[6] = {INT_MAX, INT_MIN, INT_MAX, INT_MIN, INT_MAX, INT_MIN};
    if (sg.count > 0 && bb.lo[0] <= bb.hi[0] && bb.lo[1] <= bb.hi[1] && bb.lo[2] <= bb.hi[2]) {
        BoxL<R> bx;
        bool lds;
        box_of(bb, pz, bx, lds);
        bx.j = reinterpret_cast<typename Acc3<R>::T*>(smem3);
        bx.f = reinterpret_cast<R*>(bx.j + 3 * bx.n);
        const int end = sg.start + sg.count;
        double js = 1.0, jq = 1.0;
        if (lds) {
            if constexpr (Acc3<R>::fixed) {
                double sw = 0.0;
                for (int p = sg.start + threadIdx.x; p < end; p += GT) sw += fabs((double)e.w[p]);
                sw = block_sum3<GT>(sw, redd);
                const double bound = fmax(fabs(pp.jk[0]), fmax(fabs(pp.jk[1]), fabs(pp.jk[2]))) * sw;
                if (bound > 0.0) { js = FX_RANGE / bound; jq = bound / FX_RANGE; }
            }
            stage_box<GT, R, true, MC>(g, f, bx, 3);
            __syncthreads();
            for (int p = sg.start + threadIdx.x; p < end; p += GT)
                if (!electron3<true, MC>(g, f, bx, e, p, pp, js, status, nb)) mis[atomicAdd(nmis, 1)] = make_int2(blockIdx.x, p);
            __syncthreads();
            flush_box<GT>(g, f, bx, 0, 3, jq);
        } else if (threadIdx.x == 0) {
            big[atomicAdd(nbig, 1)] = blockIdx.x;
        }
    }
    block_box<GT>(nb, red, &bout[blockIdx.x]);
}

// box bounds of a wave's particles into a segment's box (one lane per wave)
__device__ __forceinline__ void wave_grow(int nb[6], Box3* out)
{
#pragma unroll
    for (int q = 0; q < 6; q++)
        for (int o = 32; o > 0; o >>= 1) {
            const int v = __shfl_xor(nb[q], o);
            nb[q] = (q & 1) ? max(nb[q], v) : min(nb[q], v);
        }
    if (__lane_id() == 0 && nb[0] <= nb[1]) {
#pragma unroll
        for (int a = 0; a < 3; a++) {
            atomicMin(&out->lo[a], nb[2 * a]);
            atomicMax(&out->hi[a], nb[2 * a + 1]);
        }
    }
}

// the particles k3_gpd left: whole segments of list big (one workgroup each, in turn) and
// single particles of list mis, on the fields and current in HBM; their cells widen the
// segments' next boxes
template <typename R, bool MC>
__global__ void __launch_bounds__(NT) k3_gpd_hbm(G3 g, F3<R> f, E3<R> e, const Seg3* __restrict__ seg,
                                                 Box3* __restrict__ bout, Push3 pp, int* status, const int* big,
                                                 const int* nbig, const int2* mis, const int* nmis)
{
    const BoxL<R> none{};
    const int nb_ = *nbig;
    for (int b = blockIdx.x; b < nb_; b += gridDim.x) {
        const int q = big[b];
        const Seg3 sg = seg[q];
        const int end = sg.start + sg.count;
        for (int base = sg.start; base < end; base += NT) {
            int nb[6] = {INT_MAX, INT_MIN, INT_MAX, INT_MIN, INT_MAX, INT_MIN};
            const int p = base + threadIdx.x;
            if (p < end) electron3<false, MC>(g, f, none, e, p, pp, 1.0, status, nb);
            wave_grow(nb, &bout[q]);
        }
    }
    const int nm = *nmis;
    for (int base = blockIdx.x * NT; base < nm; base += gridDim.x * NT) {
        int nb[6] = {INT_MAX, INT_MIN, INT_MAX, INT_MIN, INT_MAX, INT_MIN};
        const int i = base + threadIdx.x;
        int q = 0;
        if (i < nm) {
            const int2 m = mis[i];
            q = m.x;
            electron3<false, MC>(g, f, none, e, m.y, pp, 1.0, status, nb);
        }
        // lanes may belong to different segments: one atomic set per lane
        if (i < nm && nb[0] <= nb[1]) {
            for (int a = 0; a < 3; a++) {
                atomicMin(&bout[q].lo[a], nb[2 * a]);
                atomicMax(&bout[q].hi[a], nb[2 * a + 1]);
            }
        }
    }
}

// rigid ions (q = +1): z(t) = z0 - (beta t / dz + shift), J_z only.  Bounded to four waves per
// SIMD (four 256-thread workgroups per CU, at most 128 VGPRs): the extra workgroup hides more of
// the HBM latency of the ion loads than the few spilled registers cost.
template <typename R>
__global__ void __launch_bounds__(GTI, 4) k3_gpi(G3 g, F3<R> f, I3<R> ion, const Seg3* __restrict__ seg,
                                             const Box3* __restrict__ bin, Box3* __restrict__ bout, double zsa,
                                             double zsb, double zsn, Push3 pp, int pz)
{
    extern __shared__ __attribute__((aligned(16))) unsigned char smem3[];
    __shared__ int red[6][GTI / 64];
    __shared__ double redd[GTI / 64];
    const Seg3 sg = seg[blockIdx.x];
    const Box3 bb = bin[blockIdx.x];
    int nb[6] = {INT_MAX, INT_MIN, INT_MAX, INT_MIN, INT_MAX, INT_MIN};
    if (sg.count > 0 && bb.lo[0] <= bb.hi[0] && bb.lo[1] <= bb.hi[1] && bb.lo[2] <= bb.hi[2]) {
        BoxL<R> bx;
        bool lds;
        box_of(bb, pz, bx, lds);
        bx.j = reinterpret_cast<typename Acc3<R>::T*>(smem3);
        bx.f = nullptr;
        const int end = sg.start + sg.count;
        double js = 1.0, jq = 1.0;
        if (lds) {
            if constexpr (Acc3<R>::fixed) {
                double sw = 0.0;
                for (int p = sg.start + threadIdx.x; p < end; p += GTI) sw += fabs((double)ion.w[p]);
                sw = block_sum3<GTI>(sw, redd);
                const double bound = fabs(pp.jk[2]) * sw;
                if (bound > 0.0) { js = FX_RANGE / bound; jq = bound / FX_RANGE; }
            }
            stage_box<GTI, R, false>(g, f, bx, 1);
            __syncthreads();
        }
        // the next ion's state is loaded while the current one deposits, so each iteration
        // waits only for loads issued an iteration earlier
        int p = sg.start + threadIdx.x;
        R wq = R(0);
        double xq = 0.0, yq = 0.0, zq = 0.0;
        if (p < end) {
            wq = ion.w[p];
            xq = ion.x[p];
            yq = ion.y[p];
            zq = ion.z0[p];
        }
        for (; p < end; p += GTI) {
            const R w = wq;
            const double x = xq, y = yq, z0 = zq;
            if (p + GTI < end) {
                wq = ion.w[p + GTI];
                xq = ion.x[p + GTI];
                yq = ion.y[p + GTI];
                zq = ion.z0[p + GTI];
            }
            if (w == R(0)) continue;
            const double r0[3] = {x, y, z0 - zsa}, r1[3] = {x, y, z0 - zsb};
            const double kz = -pp.jk[2] * (double)w;
            if (lds && in_box(bx, r0)) {
                deposit_box_z(bx, x, y, r0[2], r1[2], kz * js);
            } else {
                const double k[3] = {0.0, 0.0, kz};
                esirkepov3(g, f.J, r0, r1, k);
            }
            if (!g.per[2] && (r1[2] < 0.0 || r1[2] >= (double)g.N[2])) {
                ion.w[p] = R(0);
                continue;
            }
            grow(nb, 0, (int)floor(x));
            grow(nb, 1, (int)floor(y));
            grow(nb, 2, (int)floor(z0 - zsn));
        }
        if (lds) {
            __syncthreads();
            flush_box<GTI>(g, f, bx, 2, 1, jq);
        }
    }
    block_box<GTI>(nb, red, &bout[blockIdx.x]);
}

// laser antenna: per transverse cell a + particle fixed at the cell centre and a - particle
// moving along the polarisation (x or y) with the sheet current K = -2 E_perp (FP64
// throughout); xm holds the moving particle's coordinate along the polarisation
template <typename R>
__global__ void __launch_bounds__(64) k3_antenna(G3 g, F3<R> f, double* xm, const double* xh, const double* yh,
                                                 Antenna3 a, Push3 pp)
{
    const int q = blockIdx.x * 64 + threadIdx.x;
    if (q >= a.n) return;
    const double xu = xh[q] * g.d[0], yu = yh[q] * g.d[1];
    const double tau = a.tm / a.gamma - a.t0;
    const double r2 = (xu - a.xc) * (xu - a.xc) + (yu - a.yc) * (yu - a.yc);
    const double E = a.e0g * exp(-r2 / (a.w0 * a.w0)) * exp(-tau * tau / (2.0 * a.sig_t * a.sig_t)) * sin(a.omega * tau);
    const double K = -2.0 * E;
    const double v = K * g.d[0] * g.d[1] / (-1.0 * a.aw);    // um per unit time, along pol
    const double x0 = xm[q], x1 = x0 + v * pp.dt / g.d[a.pol];
    double m0[3] = {xh[q], yh[q], a.za}, m1[3] = {xh[q], yh[q], a.zb};
    m0[a.pol] = x0;
    m1[a.pol] = x1;
    const double km[3] = {pp.jk[0] * a.aw, pp.jk[1] * a.aw, pp.jk[2] * a.aw};   // q = -1
    esirkepov3(g, f.J, m0, m1, km);
    const double h0[3] = {xh[q], yh[q], a.za}, h1[3] = {xh[q], yh[q], a.zb};
    const double kp[3] = {-km[0], -km[1], -km[2]};                           // q = +1
    esirkepov3(g, f.J, h0, h1, kp);
    xm[q] = x1;
}

// ---- charge density (Gauss diagnostic) ---------------------------------------------------------
// rho on the nodes with the cubic shape of the gather and deposit, FP64 atomics
__device__ __forceinline__ void rho3_add(const G3& g, double* rho, double qw, double x, double y, double z)
{
    const double r[3] = {x, y, z};
    int j0[3];
    double S[3][4];
    for (int a = 0; a < 3; a++) {
        j0[a] = (int)floor(r[a]);
        bspline4<double>(r[a] - j0[a], S[a]);
    }
    for (int c = 0; c < 4; c++) {
        const int k = sidx(g, 2, j0[2] - 1 + c);
        if (k < 0) continue;
        for (int b = 0; b < 4; b++) {
            const int j = sidx(g, 1, j0[1] - 1 + b);
            if (j < 0) continue;
            for (int a = 0; a < 4; a++) {
                const int i = sidx(g, 0, j0[0] - 1 + a);
                if (i < 0) continue;
                atomicAdd(&rho[o3(g, i, j, k)], qw * S[0][a] * S[1][b] * S[2][c]);
            }
        }
    }
}

template <typename R>
__global__ void __launch_bounds__(NT) k3_rho(G3 g, E3<R> e, int ne, I3<R> ion, int ni, double zsh, const double* ant,
                                             int na, int pol, double za, double aw, double vol_inv, double* rho)
{
    const long p = (long)blockIdx.x * NT + threadIdx.x;
    if (p < ne) {
        const double w = (double)e.w[p];
        if (w != 0.0) rho3_add(g, rho, -w * vol_inv, e.x[p], e.y[p], e.z[p]);
    } else if (p < (long)ne + ni) {
        const long q = p - ne;
        const double w = (double)ion.w[q];
        if (w != 0.0) rho3_add(g, rho, w * vol_inv, ion.x[q], ion.y[q], ion.z0[q] - zsh);
    } else if (p < (long)ne + ni + na) {
        const long q = p - ne - ni;
        const double xh = ant[na + q], yh = ant[2 * (long)na + q], m = ant[q];
        rho3_add(g, rho, aw * vol_inv, xh, yh, za);
        rho3_add(g, rho, -aw * vol_inv, pol == 0 ? m : xh, pol == 0 ? yh : m, za);
    }
}

__global__ void __launch_bounds__(NT) k3_zero1(G3 g, double* a)
{
    int q[3];
    if (!cell_of(g, q)) return;
    a[o3(g, q[0], q[1], q[2])] = 0.0;
}

// SplitMix64 (Steele, Lea, Flood 2014): output number k of the generator started at seed
__device__ __forceinline__ double u01(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + k * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

// lattice planes row0 .. row0+nrows-1 of the lab-fixed plasma into slots base.. (base = the
// particles in use), one thread per particle.  A plane is laid out in transverse tile chunks
// (rows of chunks along y, chunks along x, then ppc, then the chunk's cells x-fastest); each
// chunk becomes a segment whose box spans its cells and the plane's z cells.  The particle id
// (and so its random offsets) depends only on the plane, the cell and k.
template <typename R>
__global__ void __launch_bounds__(NT) k3_inject(G3 g, Tiles3 tl, E3<R> e, I3<R> ion, const int* nused_e,
                                                const int* nused_i, Seg3* seg_e, Box3* box_e, Seg3* seg_i,
                                                Box3* box_i, int seg_base, Inject3 ip, int* status)
{
    const int N0 = g.N[0], N1 = g.N[1], tx = tl.t[0], ty = tl.t[1];
    const int64_t per_plane = (int64_t)N0 * N1 * ip.ppc;
    const int64_t total = per_plane * ip.nrows;
    const int64_t gq = (int64_t)blockIdx.x * NT + threadIdx.x;
    if (gq >= total) return;
    const int be = *nused_e, bi = ip.ion_mode ? *nused_i : 0;
    const bool room = (int64_t)be + total <= ip.cap && (int64_t)bi + total <= ip.cap;
    if (!room) {
        if (gq == 0) atomicOr(status, ST3_CAPACITY);
    }
    const int64_t r = gq / per_plane, rem = gq - r * per_plane;
    const int64_t rowp = (int64_t)ty * N0 * ip.ppc;           // particles of a full row of chunks
    const int cyi = (int)(rem / rowp);
    const int64_t rem1 = rem - (int64_t)cyi * rowp;
    const int hy = min(ty, N1 - cyi * ty);
    const int64_t chp = (int64_t)tx * hy * ip.ppc;            // particles of a full chunk of this row
    const int cxi = (int)(rem1 / chp);
    const int64_t rem2 = rem1 - (int64_t)cxi * chp;
    const int hx = min(tx, N0 - cxi * tx);
    const int ncc = hx * hy;
    const int k = (int)(rem2 / ncc), lc = (int)(rem2 - (int64_t)k * ncc);
    const int i = cxi * tx + lc % hx, j = cyi * ty + lc / hx;
    const int64_t l = ip.row0 + r;
    const double c = ip.beta * ip.t / ip.dz + ip.shift;
    if (rem2 == 0) {
        // this chunk's segment (count 0 when the particle arrays are full)
        const int q = seg_base + (int)r * tl.nt[0] * tl.nt[1] + cyi * tl.nt[0] + cxi;
        const int64_t off = r * per_plane + (int64_t)cyi * rowp + (int64_t)cxi * chp;
        Box3 b;
        b.lo[0] = cxi * tx; b.hi[0] = cxi * tx + hx - 1;
        b.lo[1] = cyi * ty; b.hi[1] = cyi * ty + hy - 1;
        b.lo[2] = (int)floor((double)l - c) - 1;
        b.hi[2] = (int)floor((double)l + 1.0 - c) + 1;
        const int cnt = room ? (int)(hx * hy * ip.ppc) : 0;
        seg_e[q] = Seg3{be + (int)off, cnt};
        box_e[q] = b;
        if (ip.ion_mode) {
            seg_i[q] = Seg3{bi + (int)off, cnt};
            box_i[q] = b;
        }
    }
    if (!room) return;
    const uint64_t id = (((uint64_t)l * (uint64_t)N1 + (uint64_t)j) * (uint64_t)N0 + (uint64_t)i) *
                            (uint64_t)ip.ppc + (uint64_t)k;
    const double rx = u01(ip.seed, 3 * id + 1), ry = u01(ip.seed, 3 * id + 2), rz = u01(ip.seed, 3 * id + 3);
    const double zbc = (double)l + rz;
    const double zl = ip.gamma * (zbc * ip.dz);
    double n = 0.0;
    if (zl >= ip.ramp_start) {
        n = ip.n0;
        if (ip.ramp_len > 0.0 && zl < ip.ramp_start + ip.ramp_len) n = ip.n0 * (zl - ip.ramp_start) / ip.ramp_len;
    }
    const double wgt = ip.gamma * n * ip.dx * ip.dy * ip.dz / (double)ip.ppc;
    const int p = be + (int)gq;
    e.x[p] = (double)i + rx;
    e.y[p] = (double)j + ry;
    e.z[p] = zbc - ip.beta * ip.t / ip.dz - ip.shift;
    e.ux[p] = R(0);
    e.uy[p] = R(0);
    e.uz[p] = (R)ip.uz0;
    e.w[p] = (R)wgt;
    e.id[p] = (uint32_t)id;
    if (ip.ion_mode) {
        const int pi = bi + (int)gq;
        ion.x[pi] = (double)i + rx;
        ion.y[pi] = (double)j + ry;
        ion.z0[pi] = zbc;
        ion.w[pi] = (R)wgt;
        ion.id[pi] = (uint32_t)id;
    }
}

// the injected particles enter the counters once the injection kernel has read them
__global__ void k3_bump(int* nused_e, int* nused_i, int64_t total, int64_t cap, int ion_mode)
{
    const int be = *nused_e, bi = ion_mode ? *nused_i : 0;
    if ((int64_t)be + total > cap || (int64_t)bi + total > cap) return;
    *nused_e = be + (int)total;
    if (ion_mode) *nused_i = bi + (int)total;
}


// window moved by d planes (zoff already advanced)
template <typename R>
__global__ void __launch_bounds__(NT) k3_window(G3 g, F3<R> f, int d)
{
    int q[3];
    if (!cell_of(g, q)) return;
    const int Sz = g.S[2], k = q[2];
    const long o = o3(g, q[0], q[1], k);
    if ((d > 0 && k >= Sz - d) || (d < 0 && k < -d)) {
        R* all[30] = {f.E[0], f.E[1], f.E[2], f.Eo[0], f.Eo[1], f.Eo[2], f.Eb[0], f.Eb[1], f.Eb[2],
                      f.B[0], f.B[1], f.B[2], f.Bo[0], f.Bo[1], f.Bo[2], f.Jg[0], f.Jg[1], f.Jg[2],
                      f.Jf[0], f.Jf[1], f.Jf[2], f.SE[0], f.SE[1], f.SE[2], f.SB[0], f.SB[1], f.SB[2],
                      f.T[0], f.T[1], f.T[2]};
#pragma unroll
        for (int m = 0; m < 30; m++) all[m][o] = R(0);
#pragma unroll
        for (int c = 0; c < 3; c++) f.J[c][o] = 0.0;
    } else {
        // a split part is meaningful only where one of its two axes has a conductivity: drop
        // it in planes whose content just came out of the z PML
        auto inside = [&](int a, int idx, int h) {
            if (g.per[a]) return true;
            const double pos = (double)(idx - g.P[a]) + 0.5 * h;
            return pos >= 0.0 && pos <= (double)g.N[a];
        };
#pragma unroll
        for (int c = 0; c < 2; c++) {   // x and y components: the only ones with a z derivative
            const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
            // E_c: half along c, nodes elsewhere; B_c: node along c, half elsewhere
            const int hE[3] = {c == 0 ? 1 : 0, c == 1 ? 1 : 0, 0};
            const int hB[3] = {c == 0 ? 0 : 1, c == 1 ? 0 : 1, 1};
            if (inside(2, k, hE[2]) && !inside(2, k + d, hE[2]) && inside(a1, q[a1], hE[a1]) &&
                inside(a2, q[a2], hE[a2]))
                f.SE[c][o] = R(0);
            if (inside(2, k, hB[2]) && !inside(2, k + d, hB[2]) && inside(a1, q[a1], hB[a1]) &&
                inside(a2, q[a2], hB[a2]))
                f.SB[c][o] = R(0);
        }
    }
    // tangential E stays zero on the conducting end walls
    if (!g.per[2] && (k == 0 || k == Sz - 1)) {
        f.E[0][o] = R(0); f.E[1][o] = R(0);
        f.Eo[0][o] = R(0); f.Eo[1][o] = R(0);
        f.Eb[0][o] = R(0); f.Eb[1][o] = R(0);
    }
}

// ---- tile sort ----------------------------------------------------------------------------------

// tile of a position (cells, clamped into the interior)
__device__ __forceinline__ int tile_key3(const G3& g, const Tiles3& tl, double x, double y, double z)
{
    const double r[3] = {x, y, z};
    int key = 0;
#pragma unroll
    for (int a = 2; a >= 0; a--) {
        const int c = min(max((int)floor(r[a]), 0), g.N[a] - 1);
        key = key * tl.nt[a] + c / tl.t[a];
    }
    return key;
}

constexpr int SORT_GRID = 4096;   // workgroups of the grid-stride sort passes

template <typename R>
__global__ void __launch_bounds__(NT) k3_sort_count_e(G3 g, Tiles3 tl, E3<R> e, const int* nused, int* counts)
{
    const int n = *nused;
    for (int base = blockIdx.x * NT; base < n; base += gridDim.x * NT) {
        const int p = base + threadIdx.x;
        const bool act = p < n && e.w[p] != R(0);
        const int key = act ? tile_key3(g, tl, e.x[p], e.y[p], e.z[p]) : 0;
        bf::wave_slot(counts, key, act);
    }
}

template <typename R>
__global__ void __launch_bounds__(NT) k3_sort_count_i(G3 g, Tiles3 tl, I3<R> ion, double zsh, const int* nused,
                                                      int* counts)
{
    const int n = *nused;
    for (int base = blockIdx.x * NT; base < n; base += gridDim.x * NT) {
        const int p = base + threadIdx.x;
        const bool act = p < n && ion.w[p] != R(0);
        const int key = act ? tile_key3(g, tl, ion.x[p], ion.y[p], ion.z0[p] - zsh) : 0;
        bf::wave_slot(counts, key, act);
    }
}

// exclusive scan of the tile counts (one workgroup): segment t = tile t with the tile's cells
// as its box, cursor t = its first slot, *tot = the live count
__global__ void __launch_bounds__(1024) k3_sort_scan(G3 g, Tiles3 tl, const int* counts, int* cursor, Seg3* seg,
                                                     Box3* box, int* tot)
{
    __shared__ int part[1024];
    const int per = (tl.ntiles + 1023) / 1024;
    const int b0 = min(tl.ntiles, (int)threadIdx.x * per), b1 = min(tl.ntiles, b0 + per);
    int s = 0;
    for (int i = b0; i < b1; i++) s += counts[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int v = (int)threadIdx.x >= o ? part[threadIdx.x - o] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int off = threadIdx.x ? part[threadIdx.x - 1] : 0;
    for (int i = b0; i < b1; i++) {
        const int c = counts[i];
        seg[i] = Seg3{off, c};
        cursor[i] = off;
        const int ti[3] = {i % tl.nt[0], (i / tl.nt[0]) % tl.nt[1], i / (tl.nt[0] * tl.nt[1])};
        Box3 b;
        for (int a = 0; a < 3; a++) {
            b.lo[a] = ti[a] * tl.t[a];
            b.hi[a] = min(g.N[a], (ti[a] + 1) * tl.t[a]) - 1;
        }
        box[i] = b;
        off += c;
    }
    if (threadIdx.x == 1023) *tot = part[1023];
}

template <typename R>
__global__ void __launch_bounds__(NT) k3_sort_scatter_e(G3 g, Tiles3 tl, E3<R> src, E3<R> dst, const int* nused,
                                                        int* cursor)
{
    const int n = *nused;
    for (int base = blockIdx.x * NT; base < n; base += gridDim.x * NT) {
        const int p = base + threadIdx.x;
        const bool act = p < n && src.w[p] != R(0);
        double x = 0, y = 0, z = 0;
        int key = 0;
        if (act) {
            x = src.x[p]; y = src.y[p]; z = src.z[p];
            key = tile_key3(g, tl, x, y, z);
        }
        const int d = bf::wave_slot(cursor, key, act);
        if (act) {
            dst.x[d] = x; dst.y[d] = y; dst.z[d] = z;
            dst.ux[d] = src.ux[p]; dst.uy[d] = src.uy[p]; dst.uz[d] = src.uz[p];
            dst.w[d] = src.w[p]; dst.id[d] = src.id[p];
        }
    }
}

template <typename R>
__global__ void __launch_bounds__(NT) k3_sort_scatter_i(G3 g, Tiles3 tl, I3<R> src, I3<R> dst, double zsh,
                                                        const int* nused, int* cursor)
{
    const int n = *nused;
    for (int base = blockIdx.x * NT; base < n; base += gridDim.x * NT) {
        const int p = base + threadIdx.x;
        const bool act = p < n && src.w[p] != R(0);
        double x = 0, y = 0, z0 = 0;
        int key = 0;
        if (act) {
            x = src.x[p]; y = src.y[p]; z0 = src.z0[p];
            key = tile_key3(g, tl, x, y, z0 - zsh);
        }
        const int d = bf::wave_slot(cursor, key, act);
        if (act) {
            dst.x[d] = x; dst.y[d] = y; dst.z0[d] = z0; dst.w[d] = src.w[p]; dst.id[d] = src.id[p];
        }
    }
}

__global__ void k3_set_count(int* nused, const int* tot) { *nused = *tot; }

// Order within each tile after the scatter, by the particle's place in the plasma lattice: its
// id encodes the lattice plane l, the cell (i, j) and the index k < ppc within the cell, and
// the tile is laid out by (l, k, j, i), i fastest, over the tile's i, j range.  A wave of 64
// lanes then holds the k-th particles of one lattice plane over an 8 x 8 block of cells: the
// lanes sit in distinct (x, y) cells and differ in z by at most one plane (the plasma drifts
// rigidly), which the LDS box layout keeps in distinct bank pairs.  Ids outside the pattern
// (particles loaded from outside) only fall in clamped places: any order is valid.  Equal
// keys are spread level by level (the k-th particle with a key in level k).
constexpr int ORD_THREADS = 512;
constexpr int ORD_MAX_CELLS = 8192;   // keys of a tile ordered in LDS
constexpr int ORD_TABLE = 8192;       // particles of a tile ordered in LDS (more keep the scatter order)

constexpr int ORD_GROUPS = 1024;     // (plane, k) groups of a tile regrouped complete-first

struct TileOrder {
    int cnt[ORD_MAX_CELLS], pos[ORD_MAX_CELLS];
    int tab[ORD_TABLE];               // per particle: key | level << 16
    int part[ORD_THREADS];
    int gcnt[ORD_GROUPS], grank[ORD_GROUPS];
    int kmax, lmin, grouped;
};

// lattice key of a particle id within a tile (origin o, width w), planes from lmin, lr planes
struct LatticeKey {
    int n0, n1, ppc, o0, o1, w0, w1, lmin, lr;
    __device__ __forceinline__ int row(uint32_t id) const { return (int)(id / (uint32_t)ppc / (uint32_t)(n0 * n1)); }
    __device__ __forceinline__ int of(uint32_t id) const
    {
        const int k = (int)(id % (uint32_t)ppc);
        const uint32_t rest = id / (uint32_t)ppc;
        const int i = (int)(rest % (uint32_t)n0), j = (int)((rest / (uint32_t)n0) % (uint32_t)n1);
        const int l = (int)(rest / (uint32_t)(n0 * n1));
        const int li = min(max(i - o0, 0), w0 - 1), lj = min(max(j - o1, 0), w1 - 1);
        const int ll = min(max(l - lmin, 0), lr - 1);
        return ((ll * ppc + k) * w1 + lj) * w0 + li;
    }
};

// A tile's z faces cut the first and last lattice planes at random in-cell offsets, so some
// (plane, k) groups are incomplete; the complete groups go first (each then fills whole waves
// from a wave boundary) and the incomplete ones last.  Returns the regrouped key of a particle.
__device__ void regroup(TileOrder& ts, const LatticeKey& lk, const uint32_t* ids, int N)
{
    const int W = lk.w0 * lk.w1, G = lk.lr * lk.ppc;
    if (G > ORD_GROUPS) {   // too many groups for the table: plain lattice order
        if (threadIdx.x == 0) ts.grouped = 0;
        __syncthreads();
        return;
    }
    for (int q = threadIdx.x; q < G; q += ORD_THREADS) ts.gcnt[q] = 0;
    __syncthreads();
    for (int q = threadIdx.x; q < N; q += ORD_THREADS) atomicAdd(&ts.gcnt[lk.of(ids[q]) / W], 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        int r = 0;
        for (int q = 0; q < G; q++)
            if (ts.gcnt[q] == W) ts.grank[q] = r++;
        for (int q = 0; q < G; q++)
            if (ts.gcnt[q] != W) ts.grank[q] = r++;
        ts.grouped = 1;
    }
    __syncthreads();
}

__device__ __forceinline__ int regrouped(const TileOrder& ts, const LatticeKey& lk, uint32_t id)
{
    const int W = lk.w0 * lk.w1, key = lk.of(id);
    return ts.grouped ? ts.grank[key / W] * W + key % W : key;
}

// the lattice key of the tile's particles (ids ids[0..N)) for block t
__device__ LatticeKey lattice_key(TileOrder& ts, const G3& g, const Tiles3& tl, int t, int ppc, const uint32_t* ids,
                                  int N)
{
    LatticeKey lk;
    const int ti[2] = {t % tl.nt[0], (t / tl.nt[0]) % tl.nt[1]};
    lk.n0 = g.N[0];
    lk.n1 = g.N[1];
    lk.ppc = max(ppc, 1);
    lk.o0 = ti[0] * tl.t[0];
    lk.o1 = ti[1] * tl.t[1];
    lk.w0 = min(tl.t[0], g.N[0] - lk.o0);
    lk.w1 = min(tl.t[1], g.N[1] - lk.o1);
    lk.lr = max(1, ORD_MAX_CELLS / (lk.ppc * lk.w0 * lk.w1));
    if (threadIdx.x == 0) ts.lmin = INT_MAX;
    __syncthreads();
    int lm = INT_MAX;
    for (int q = threadIdx.x; q < N; q += ORD_THREADS) lm = min(lm, lk.row(ids[q]));
    for (int o = 32; o > 0; o >>= 1) lm = min(lm, __shfl_xor(lm, o));
    if ((threadIdx.x & 63) == 0) atomicMin(&ts.lmin, lm);
    __syncthreads();
    lk.lmin = ts.lmin;
    return lk;
}

// cell of a tile (clamped as the tile key clamps)
struct TileBox3 {
    int o[3], w[3];
    __device__ __forceinline__ int of(const G3& g, double x, double y, double z) const
    {
        const double r[3] = {x, y, z};
        int c = 0;
#pragma unroll
        for (int a = 2; a >= 0; a--) {
            const int v = min(max((int)floor(r[a]), 0), g.N[a] - 1) - o[a];
            c = c * w[a] + min(max(v, 0), w[a] - 1);
        }
        return c;
    }
};

__device__ __forceinline__ TileBox3 tile_box3(const G3& g, const Tiles3& tl, int t)
{
    const int ti[3] = {t % tl.nt[0], (t / tl.nt[0]) % tl.nt[1], t / (tl.nt[0] * tl.nt[1])};
    TileBox3 b;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        b.o[a] = ti[a] * tl.t[a];
        b.w[a] = min(tl.t[a], g.N[a] - b.o[a]);
    }
    return b;
}

// exclusive scan of flag over the tile's C cells into pos; returns the total
__device__ int scan_cells(TileOrder& ts, int C, int k)
{
    const int t = threadIdx.x;
    const int per = (C + ORD_THREADS - 1) / ORD_THREADS, lo = min(t * per, C), hi = min(lo + per, C);
    int s = 0;
    for (int i = lo; i < hi; i++) s += ts.cnt[i] > k;
    ts.part[t] = s;
    __syncthreads();
    for (int o = 1; o < ORD_THREADS; o <<= 1) {
        const int v = t >= o ? ts.part[t - o] : 0;
        __syncthreads();
        ts.part[t] += v;
        __syncthreads();
    }
    int run = ts.part[t] - s;
    for (int i = lo; i < hi; i++) {
        ts.pos[i] = run;
        run += ts.cnt[i] > k;
    }
    const int total = ts.part[ORD_THREADS - 1];
    __syncthreads();
    return total;
}

// pos3(q) -> cell of the tile's q-th particle, copy(q, slot) moves it
template <typename Cell, typename Copy>
__device__ void order_tile3(TileOrder& ts, int C, int N, Cell cell_of_q, Copy copy)
{
    if (C > ORD_MAX_CELLS || N > ORD_TABLE) {
        for (int q = threadIdx.x; q < N; q += ORD_THREADS) copy(q, q);
        return;
    }
    for (int i = threadIdx.x; i < C; i += ORD_THREADS) ts.cnt[i] = 0;
    if (threadIdx.x == 0) ts.kmax = 0;
    __syncthreads();
    int km = 0;
    for (int q = threadIdx.x; q < N; q += ORD_THREADS) {
        const int c = cell_of_q(q);
        const int k = atomicAdd(&ts.cnt[c], 1);
        ts.tab[q] = c | (k << 16);
        km = max(km, k + 1);
    }
    for (int o = 32; o > 0; o >>= 1) km = max(km, __shfl_xor(km, o));
    if ((threadIdx.x & 63) == 0) atomicMax(&ts.kmax, km);
    __syncthreads();
    const int K = ts.kmax;
    int base = 0;
    for (int k = 0; k < K; k++) {
        const int L = scan_cells(ts, C, k);
        for (int q = threadIdx.x; q < N; q += ORD_THREADS) {
            const int v = ts.tab[q];
            if ((v >> 16) == k) copy(q, base + ts.pos[v & 0xffff]);
        }
        base += L;
        __syncthreads();
    }
}

template <typename R>
__global__ void __launch_bounds__(ORD_THREADS) k3_sort_order_e(G3 g, Tiles3 tl, E3<R> src, E3<R> dst,
                                                               const Seg3* seg, int ppc)
{
    __shared__ TileOrder ts;
    const Seg3 sg = seg[blockIdx.x];
    if (sg.count <= 0) return;
    const int o = sg.start;
    const LatticeKey lk = lattice_key(ts, g, tl, blockIdx.x, ppc, src.id + o, min(sg.count, ORD_TABLE));
    regroup(ts, lk, src.id + o, min(sg.count, ORD_TABLE));
    order_tile3(
        ts, lk.lr * lk.ppc * lk.w0 * lk.w1, sg.count, [&](int q) { return regrouped(ts, lk, src.id[o + q]); },
        [&](int q, int sl) {
            const int p = o + q, d = o + sl;
            dst.x[d] = src.x[p]; dst.y[d] = src.y[p]; dst.z[d] = src.z[p];
            dst.ux[d] = src.ux[p]; dst.uy[d] = src.uy[p]; dst.uz[d] = src.uz[p];
            dst.w[d] = src.w[p]; dst.id[d] = src.id[p];
        });
}

template <typename R>
__global__ void __launch_bounds__(ORD_THREADS) k3_sort_order_i(G3 g, Tiles3 tl, I3<R> src, I3<R> dst,
                                                               const Seg3* seg, int ppc)
{
    __shared__ TileOrder ts;
    const Seg3 sg = seg[blockIdx.x];
    if (sg.count <= 0) return;
    const int o = sg.start;
    const LatticeKey lk = lattice_key(ts, g, tl, blockIdx.x, ppc, src.id + o, min(sg.count, ORD_TABLE));
    regroup(ts, lk, src.id + o, min(sg.count, ORD_TABLE));
    order_tile3(
        ts, lk.lr * lk.ppc * lk.w0 * lk.w1, sg.count, [&](int q) { return regrouped(ts, lk, src.id[o + q]); },
        [&](int q, int sl) {
            const int p = o + q, d = o + sl;
            dst.x[d] = src.x[p]; dst.y[d] = src.y[p]; dst.z0[d] = src.z0[p];
            dst.w[d] = src.w[p]; dst.id[d] = src.id[p];
        });
}



// number of live particles (w != 0) among n slots, one atomic per workgroup
template <typename R>
__global__ void __launch_bounds__(NT) k3_count_live(const R* w, int n, int* cnt)
{
    __shared__ int part[NT / 64];
    int c = 0;
    for (int p = blockIdx.x * NT + threadIdx.x; p - (int)threadIdx.x < n; p += gridDim.x * NT)
        c += __popcll(__ballot(p < n && w[p] != R(0)));
    if (__lane_id() == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int q = 0; q < NT / 64; q++) t += part[q];
        if (t) atomicAdd(cnt, t);
    }
}

// trilinear sample of a component with staggers h at r (cells)
template <typename R>
__device__ double trilin(const G3& g, const R* F, const int h[3], const double r[3])
{
    int j[3];
    double fr[3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const double xs = r[a] - 0.5 * h[a];
        j[a] = (int)floor(xs);
        fr[a] = xs - j[a];
    }
    double v = 0.0;
    for (int c = 0; c < 2; c++)
        for (int b = 0; b < 2; b++)
            for (int a = 0; a < 2; a++) {
                const int i0 = sidx(g, 0, j[0] + a), i1 = sidx(g, 1, j[1] + b), i2 = sidx(g, 2, j[2] + c);
                if (i0 < 0 || i1 < 0 || i2 < 0) continue;
                v += (a ? fr[0] : 1.0 - fr[0]) * (b ? fr[1] : 1.0 - fr[1]) * (c ? fr[2] : 1.0 - fr[2]) *
                     (double)F[o3(g, i0, i1, i2)];
            }
    return v;
}

template <typename R>
__global__ void k3_stations(G3 g, F3<R> f, const double* zlab, int nst, double gamma, double beta, double t,
                            double shift_cells, double* rec, int* cnt, int cap)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nst) return;
    const double zb = zlab[q] / gamma - beta * t;
    const double zc = zb / g.d[2] - shift_cells;
    if (zc < 0.0 || zc >= (double)g.N[2] || cnt[q] >= cap) return;
    const double r[3] = {0.5 * g.N[0], 0.5 * g.N[1], zc};
    double E[3], B[3];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const int hE[3] = {c == 0, c == 1, c == 2}, hB[3] = {c != 0, c != 1, c != 2};
        E[c] = trilin(g, f.E[c], hE, r);
        B[c] = 0.5 * (trilin(g, f.Bo[c], hB, r) + trilin(g, f.B[c], hB, r));
    }
    double* o = rec + ((size_t)q * cap + cnt[q]) * 7;
    o[0] = gamma * (t + beta * zb);
    o[1] = gamma * (E[0] + beta * B[1]);
    o[2] = gamma * (E[1] - beta * B[0]);
    o[3] = E[2];
    o[4] = gamma * (B[0] - beta * E[1]);
    o[5] = gamma * (B[1] + beta * E[0]);
    o[6] = B[2];
    cnt[q] += 1;
}

// ---- launchers ----------------------------------------------------------------------------------

template <typename R>
void launch3_faraday(const G3& g, const F3<R>& f, const Pml3& pml, const double ck[3], double theta, double dt,
                     hipStream_t s)
{
    const dim3 grid((unsigned)((g.S[0] + FMX - 1) / FMX), (unsigned)((g.S[1] + FMY - 1) / FMY),
                    (unsigned)((g.S[2] + FMZ - 1) / FMZ));
    if (theta > 0.0)
        hipLaunchKernelGGL((k3_faraday<R, true>), grid, cells_block(), 0, s, g, f, pml, (R)ck[0], (R)ck[1], (R)ck[2],
                           (R)dt, (R)theta);
    else
        hipLaunchKernelGGL((k3_faraday<R, false>), grid, cells_block(), 0, s, g, f, pml, (R)ck[0], (R)ck[1],
                           (R)ck[2], (R)dt, (R)theta);
}

template <typename R>
void launch3_ampere(const G3& g, const F3<R>& f, const R* const J[3], const Pml3& pml, double dt, hipStream_t s)
{
    const dim3 grid((unsigned)((g.S[0] + FMX - 1) / FMX), (unsigned)((g.S[1] + FMY - 1) / FMY),
                    (unsigned)((g.S[2] + FMZ - 1) / FMZ));
    hipLaunchKernelGGL((k3_ampere<R>), grid, cells_block(), 0, s, g, f, J[0], J[1], J[2], pml, (R)dt);
}

bool filter_seq(int npass, int comp, int stride_mask, FiltSeq* fs)
{
    fs->n = 0;
    fs->reach = 0;
    if (npass <= 0) return true;
    const int mask = stride_mask ? stride_mask : 1;
    for (int st = 1; st <= 16; st++) {
        if (!(mask & (1 << (st - 1)))) continue;
        const int k = npass + (comp ? 1 : 0);
        if (fs->n + k > FSEQ_MAX || fs->reach + k * st > FREACH_MAX) return false;
        for (int p = 0; p < k; p++) {
            fs->alpha[fs->n] = p < npass ? 0.5 : 0.5 * npass + 1.0;
            fs->stride[fs->n] = st;
            fs->n++;
            fs->reach += st;
        }
    }
    return true;
}

// one launch of k3_fline along AX for ncomp components
template <int AX, typename TI, typename TO, typename T>
void fline(const G3& g, const Lines3<TI, TO>& L, int ncomp, const FiltSeq& fs, hipStream_t s)
{
    constexpr int BC = fline_bc<AX>();
    constexpr size_t LDS_MAX = 144 * 1024;
    const int S = g.S[AX];
    auto lds_of = [&](int t) {
        const int A = t + 2 * fs.reach;
        return 2 * (size_t)(AX == 0 ? BC * (A + 1) : A * (BC + 1)) * sizeof(T);
    };
    // segments along AX: the whole line when its halo-padded copy fits a third of the LDS (three
    // workgroups per CU), else equal segments of at most 128 (FP32) or 64 (FP64) cells, so that
    // no segment is mostly halo
    int tseg;
    if (AX == 0) tseg = S + 2 * fs.reach <= 1024 ? S : 512;
    else if (lds_of(S) <= 48 * 1024) tseg = S;
    else {
        const int cap = sizeof(T) == 4 ? 128 : 64;
        const int n = (S + cap - 1) / cap;
        tseg = (S + n - 1) / n;
    }
    while (tseg > 16 && lds_of(tseg) > LDS_MAX) tseg /= 2;       // long reaches: shorter segments
    const size_t lds = lds_of(tseg);
    const int nseg = (S + tseg - 1) / tseg;
    const int ncolb = AX == 0 ? (g.S[1] * g.S[2] + BC - 1) / BC : (g.S[0] + BC - 1) / BC;
    const int nother = AX == 0 ? 1 : g.S[AX == 1 ? 2 : 1];
    const long blocks = (long)ncomp * nseg * ncolb * nother;
    (void)hipFuncSetAttribute((const void*)k3_fline<AX, TI, TO, T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
    hipLaunchKernelGGL((k3_fline<AX, TI, TO, T>), dim3((unsigned)blocks), dim3(NT), lds, s, g, L, fs, tseg, nseg,
                       ncolb);
}

// the stencil of a sequence of unit-stride passes (the product of its 3-point stencils); false
// for strided passes and for reaches beyond FT_RMAX
static bool unit_stencil(const FiltSeq& fs, FiltStencil& st)
{
    const int R = fs.reach;
    if (fs.n < 1 || R < 1 || R > FT_RMAX) return false;
    for (int p = 0; p < fs.n; p++)
        if (fs.stride[p] != 1) return false;
    double a[2 * FT_RMAX + 1] = {}, b[2 * FT_RMAX + 1];
    const int L = 2 * R + 1;
    a[R] = 1.0;
    for (int p = 0; p < fs.n; p++) {
        const double al = fs.alpha[p], be = 0.5 * (1.0 - al);
        for (int j = 0; j < L; j++) b[j] = al * a[j] + be * ((j > 0 ? a[j - 1] : 0.0) + (j + 1 < L ? a[j + 1] : 0.0));
        for (int j = 0; j < L; j++) a[j] = b[j];
    }
    for (int m = 0; m <= FT_RMAX; m++) st.c[m] = m <= R ? a[R + m] : 0.0;
    return true;
}

// the three-axis filter of J into Jf in one launch; false where it does not apply (an axis
// shorter than the stencil's continuation needs), leaving the line passes to do it
template <int RC, typename R>
bool filt3(const G3& g, const F3<R>& f, const FiltStencil& st, hipStream_t s)
{
    for (int a = 0; a < 3; a++)
        if (!g.per[a] && g.S[a] < 2 * RC + 3) return false;
    static int slots = 0;          // workgroups resident on the device at once
    if (!slots) {
        int dev = 0, cus = 0, occ = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            cus = 256;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void*)k3_filt3<RC, R, R>, FT_NT, 0) !=
                hipSuccess || occ < 1)
            occ = 1;
        slots = occ * cus;
    }
    const int nxt = (g.S[0] + FT_TX - 1) / FT_TX, nyt = (g.S[1] + FT_TY - 1) / FT_TY;
    const long base = 3L * nxt * nyt;
    // z runs: the count for which (rounds of resident workgroups) x (run length + its reach) is
    // least; a run of a non-periodic axis after the first starts at least 2 reach + 2 planes in
    const int S2 = g.S[2];
    int seg = S2;
    double best = 1e300;
    for (int n = 1; n <= 512; n++) {
        const int sg = (S2 + n - 1) / n;
        if (n > 1 && sg < 2 * RC + 2) break;
        const int nz = (S2 + sg - 1) / sg;
        const double t = (double)((base * nz + slots - 1) / slots) * (sg + 2 * RC);
        if (t < best * (1.0 - 1e-9)) {
            best = t;
            seg = sg;
        }
    }
    const int nzs = (S2 + seg - 1) / seg;
    const long nwork = base * nzs;
    const long blocks = (nwork + 7) / 8 * 8;
    Lines3<double, R> L{};
    for (int c = 0; c < 3; c++) {
        L.in[c] = f.J[c];
        L.out[c] = f.Jf[c];
    }
    hipLaunchKernelGGL((k3_filt3<RC, R, R>), dim3((unsigned)blocks), dim3(FT_NT), 0, s, g, L, st, seg, nzs,
                       (int)nwork, nxt, nyt);
    return true;
}

template <typename R>
void launch3_filter(const G3& g, const F3<R>& f, const FiltSeq& fs, const R* out[3], hipStream_t s)
{
    Lines3<double, R> lx;
    Lines3<R, R> ly, lz;
    for (int c = 0; c < 3; c++) {
        lx.in[c] = f.J[c];
        lx.out[c] = f.Jf[c];
        ly.in[c] = f.Jf[c];
        ly.out[c] = f.Jg[c];
        lz.in[c] = f.Jg[c];
        lz.out[c] = f.Jf[c];
        lx.h[c] = c == 0;
        ly.h[c] = c == 1;
        lz.h[c] = c == 2;
        out[c] = f.Jf[c];
    }
    if (fs.n) {
        FiltStencil st;
        if (unit_stencil(fs, st)) {
            bool done = false;
            switch (fs.reach) {
            case 1: done = filt3<1>(g, f, st, s); break;
            case 2: done = filt3<2>(g, f, st, s); break;
            case 3: done = filt3<3>(g, f, st, s); break;
            case 4: done = filt3<4>(g, f, st, s); break;
            case 5: done = filt3<5>(g, f, st, s); break;
            case 6: done = filt3<6>(g, f, st, s); break;
            default: break;
            }
            if (done) return;
        }
    }
    fline<0, double, R, R>(g, lx, 3, fs, s);     // without passes: the copy into the run's type
    if (fs.n == 0) return;
    fline<1, R, R, R>(g, ly, 3, fs, s);
    fline<2, R, R, R>(g, lz, 3, fs, s);
}

template <typename T>
void launch_filter_xz(const G3& g, const T* const in[3], T* const tmp[3], T* const out[3], const int hx[3],
                      const int hz[3], int ncomp, const FiltSeq& fs, hipStream_t s)
{
    Lines3<T, T> lx{}, lz{};
    for (int c = 0; c < ncomp; c++) {
        lx.in[c] = in[c];
        lx.out[c] = fs.n ? tmp[c] : out[c];
        lx.h[c] = hx[c];
        lz.in[c] = tmp[c];
        lz.out[c] = out[c];
        lz.h[c] = hz[c];
    }
    fline<0, T, T, T>(g, lx, ncomp, fs, s);
    if (fs.n) fline<2, T, T, T>(g, lz, ncomp, fs, s);
}
template void launch_filter_xz<float>(const G3&, const float* const*, float* const*, float* const*, const int*,
                                      const int*, int, const FiltSeq&, hipStream_t);
template void launch_filter_xz<double>(const G3&, const double* const*, double* const*, double* const*,
                                       const int*, const int*, int, const FiltSeq&, hipStream_t);

double* launch3_filter_nodal(const G3& g, double* a, double* b, double* c, const FiltSeq& fs, hipStream_t s)
{
    if (fs.n == 0) return a;
    Lines3<double, double> l0{{a, nullptr, nullptr}, {b, nullptr, nullptr}, {0, 0, 0}};
    Lines3<double, double> l1{{b, nullptr, nullptr}, {c, nullptr, nullptr}, {0, 0, 0}};
    Lines3<double, double> l2{{c, nullptr, nullptr}, {b, nullptr, nullptr}, {0, 0, 0}};
    fline<0, double, double, double>(g, l0, 1, fs, s);
    fline<1, double, double, double>(g, l1, 1, fs, s);
    fline<2, double, double, double>(g, l2, 1, fs, s);
    return b;
}

template <typename R>
void launch3_rho(const G3& g, const E3<R>& e, int ne, const I3<R>& ion, int ni, double zsh, const double* ant,
                 int na, int pol, double za, double aw, double vol_inv, double* rho, hipStream_t s)
{
    hipLaunchKernelGGL(k3_zero1, cells_grid(g), cells_block(), 0, s, g, rho);
    const long n = (long)ne + ni + na;
    if (n > 0)
        hipLaunchKernelGGL((k3_rho<R>), dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, s, g, e, ne, ion, ni, zsh,
                           ant, na, pol, za, aw, vol_inv, rho);
}

template <typename R>
void launch3_zero_j(const G3& g, const F3<R>& f, hipStream_t s)
{
    hipLaunchKernelGGL(k3_zero3, cells_grid(g), cells_block(), 0, s, g, f.J[0], f.J[1], f.J[2]);
}

template <typename R, bool MC>
void gpd_launch(const G3& g, const F3<R>& f, const E3<R>& e, const Seg3* seg, const Box3* bin, Box3* bout,
                int nseg, const Push3& pp, int pz, int* status, int* lists, int2* mis, hipStream_t s)
{
    const size_t lds = (size_t)BPL * pz * box_cell_bytes<R>();
    int *nbig = lists, *nmis = lists + 1, *big = lists + 2;
    (void)hipMemsetAsync(lists, 0, 2 * sizeof(int), s);
    (void)hipFuncSetAttribute((const void*)k3_gpd<R, MC>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((k3_gpd<R, MC>), dim3(nseg), dim3(GT), lds, s, g, f, e, seg, bin, bout, pp, pz, status, big,
                       nbig, mis, nmis);
    hipLaunchKernelGGL((k3_gpd_hbm<R, MC>), dim3(std::min(HBM_GRID, nseg)), dim3(NT), 0, s, g, f, e, seg, bout, pp,
                       status, big, nbig, mis, nmis);
}

template <typename R>
void launch3_gpd(const G3& g, const F3<R>& f, const E3<R>& e, const Seg3* seg, const Box3* bin, Box3* bout,
                 int nseg, const Push3& pp, int pz, int* status, int* lists, int2* mis, bool mc, hipStream_t s)
{
    if (nseg <= 0) return;
    if (mc) gpd_launch<R, true>(g, f, e, seg, bin, bout, nseg, pp, pz, status, lists, mis, s);
    else gpd_launch<R, false>(g, f, e, seg, bin, bout, nseg, pp, pz, status, lists, mis, s);
}

// ---- momentum-conserving gather: fields to the nodes ---------------------------------------------
// E_c at a node is the mean of its two values at -1/2 and +1/2 along c; B_c the mean of its four
// values at -+1/2 along the two other axes (B^n = (B^{n-1/2} + B^{n+1/2}) / 2); locations beyond a
// non-periodic edge read 0
template <typename R>
__global__ void __launch_bounds__(NT) k3_nodes(G3 g, F3<R> f)
{
    int q[3];
    if (!cell_of(g, q)) return;
    int lo[3];
#pragma unroll
    for (int a = 0; a < 3; a++) lo[a] = nb(q[a], -1, g.S[a], g.per[a]);
    auto at = [&](const R* A, int i, int j, int k) {
        return (i < 0 || j < 0 || k < 0) ? R(0) : A[o3(g, i, j, k)];
    };
    auto bn = [&](int c, int i, int j, int k) { return R(0.5) * (at(f.B[c], i, j, k) + at(f.Bo[c], i, j, k)); };
    const long o = o3(g, q[0], q[1], q[2]);
    f.G[0][o] = R(0.5) * (at(f.E[0], lo[0], q[1], q[2]) + at(f.E[0], q[0], q[1], q[2]));
    f.G[1][o] = R(0.5) * (at(f.E[1], q[0], lo[1], q[2]) + at(f.E[1], q[0], q[1], q[2]));
    f.G[2][o] = R(0.5) * (at(f.E[2], q[0], q[1], lo[2]) + at(f.E[2], q[0], q[1], q[2]));
    f.G[3][o] = R(0.25) * ((bn(0, q[0], lo[1], lo[2]) + bn(0, q[0], q[1], lo[2])) +
                           (bn(0, q[0], lo[1], q[2]) + bn(0, q[0], q[1], q[2])));
    f.G[4][o] = R(0.25) * ((bn(1, lo[0], q[1], lo[2]) + bn(1, q[0], q[1], lo[2])) +
                           (bn(1, lo[0], q[1], q[2]) + bn(1, q[0], q[1], q[2])));
    f.G[5][o] = R(0.25) * ((bn(2, lo[0], lo[1], q[2]) + bn(2, q[0], lo[1], q[2])) +
                           (bn(2, lo[0], q[1], q[2]) + bn(2, q[0], q[1], q[2])));
}

template <typename R>
void launch3_nodes(const G3& g, const F3<R>& f, hipStream_t s)
{
    hipLaunchKernelGGL((k3_nodes<R>), cells_grid(g), cells_block(), 0, s, g, f);
}

template <typename R>
void launch3_gpi(const G3& g, const F3<R>& f, const I3<R>& ion, const Seg3* seg, const Box3* bin, Box3* bout,
                 int nseg, double zsa, double zsb, double zsn, const Push3& pp, int pz, hipStream_t s)
{
    if (nseg <= 0) return;
    const size_t lds = (size_t)BPL * pz * 8;
    (void)hipFuncSetAttribute((const void*)k3_gpi<R>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((k3_gpi<R>), dim3(nseg), dim3(GTI), lds, s, g, f, ion, seg, bin, bout, zsa, zsb, zsn, pp, pz);
}

template <typename R>
void launch3_antenna(const G3& g, const F3<R>& f, double* xm, const double* xh, const double* yh,
                     const Antenna3& a, const Push3& pp, hipStream_t s)
{
    if (a.n <= 0) return;
    hipLaunchKernelGGL((k3_antenna<R>), dim3((a.n + 63) / 64), dim3(64), 0, s, g, f, xm, xh, yh, a, pp);
}

template <typename R>
void launch3_inject(const G3& g, const Tiles3& tl, const E3<R>& e, const I3<R>& ion, int* nused_e, int* nused_i,
                    Seg3* seg_e, Box3* box_e, Seg3* seg_i, Box3* box_i, int seg_base, const Inject3& ip,
                    int* status, hipStream_t s)
{
    const int64_t total = (int64_t)g.N[0] * g.N[1] * ip.ppc * ip.nrows;
    if (total <= 0) return;
    hipLaunchKernelGGL((k3_inject<R>), dim3((unsigned)((total + NT - 1) / NT)), dim3(NT), 0, s, g, tl, e, ion,
                       nused_e, nused_i, seg_e, box_e, seg_i, box_i, seg_base, ip, status);
    hipLaunchKernelGGL(k3_bump, dim3(1), dim3(1), 0, s, nused_e, nused_i, total, ip.cap, ip.ion_mode);
}

template <typename R>
void launch3_window(const G3& g, const F3<R>& f, const Pml3& pml, int d, hipStream_t s)
{
    (void)pml;
    if (d == 0) return;
    hipLaunchKernelGGL((k3_window<R>), cells_grid(g), cells_block(), 0, s, g, f, d);
}

template <typename R>
void launch3_sort_e(const G3& g, const Tiles3& tl, const E3<R>& src, const E3<R>& dst, int* nused, int* counts,
                    int* cursor, int* tot, Seg3* seg, Box3* box, int64_t cap, int ppc, hipStream_t s)
{
    const dim3 grid((unsigned)std::min<int64_t>(SORT_GRID, (cap + NT - 1) / NT));
    (void)hipMemsetAsync(counts, 0, sizeof(int) * tl.ntiles, s);
    hipLaunchKernelGGL((k3_sort_count_e<R>), grid, dim3(NT), 0, s, g, tl, src, nused, counts);
    hipLaunchKernelGGL(k3_sort_scan, dim3(1), dim3(1024), 0, s, g, tl, counts, cursor, seg, box, tot);
    hipLaunchKernelGGL((k3_sort_scatter_e<R>), grid, dim3(NT), 0, s, g, tl, src, dst, nused, cursor);
    hipLaunchKernelGGL((k3_sort_order_e<R>), dim3(tl.ntiles), dim3(ORD_THREADS), 0, s, g, tl, dst, src, seg, ppc);
    hipLaunchKernelGGL(k3_set_count, dim3(1), dim3(1), 0, s, nused, tot);
}

template <typename R>
void launch3_sort_i(const G3& g, const Tiles3& tl, const I3<R>& src, const I3<R>& dst, double zsh, int* nused,
                    int* counts, int* cursor, int* tot, Seg3* seg, Box3* box, int64_t cap, int ppc, hipStream_t s)
{
    const dim3 grid((unsigned)std::min<int64_t>(SORT_GRID, (cap + NT - 1) / NT));
    (void)hipMemsetAsync(counts, 0, sizeof(int) * tl.ntiles, s);
    hipLaunchKernelGGL((k3_sort_count_i<R>), grid, dim3(NT), 0, s, g, tl, src, zsh, nused, counts);
    hipLaunchKernelGGL(k3_sort_scan, dim3(1), dim3(1024), 0, s, g, tl, counts, cursor, seg, box, tot);
    hipLaunchKernelGGL((k3_sort_scatter_i<R>), grid, dim3(NT), 0, s, g, tl, src, dst, zsh, nused, cursor);
    hipLaunchKernelGGL((k3_sort_order_i<R>), dim3(tl.ntiles), dim3(ORD_THREADS), 0, s, g, tl, dst, src, seg, ppc);
    hipLaunchKernelGGL(k3_set_count, dim3(1), dim3(1), 0, s, nused, tot);
}

template <typename R>
void launch3_count_live(const R* w, int n, int* cnt, hipStream_t s)
{
    (void)hipMemsetAsync(cnt, 0, sizeof(int), s);
    if (n > 0)
        hipLaunchKernelGGL((k3_count_live<R>), dim3(std::min((n + NT - 1) / NT, SORT_GRID)), dim3(NT), 0, s, w, n, cnt);
}

template <typename R>
void launch3_stations(const G3& g, const F3<R>& f, const double* zlab, int nst, double gamma, double beta,
                      double t, double shift_cells, double* rec, int* cnt, int cap, hipStream_t s)
{
    if (nst <= 0) return;
    hipLaunchKernelGGL((k3_stations<R>), dim3(1), dim3(64), 0, s, g, f, zlab, nst, gamma, beta, t, shift_cells,
                       rec, cnt, cap);
}

#define BF3_INST(R)                                                                                           \
    template void launch3_faraday<R>(const G3&, const F3<R>&, const Pml3&, const double*, double, double,   \
                                     hipStream_t);                                                          \
    template void launch3_ampere<R>(const G3&, const F3<R>&, const R* const*, const Pml3&, double,          \
                                    hipStream_t);                                                           \
    template void launch3_filter<R>(const G3&, const F3<R>&, const FiltSeq&, const R**, hipStream_t);        \
    template void launch3_zero_j<R>(const G3&, const F3<R>&, hipStream_t);                                  \
    template void launch3_rho<R>(const G3&, const E3<R>&, int, const I3<R>&, int, double, const double*, int,   \
                                 int, double, double, double, double*, hipStream_t);                       \
    template void launch3_count_live<R>(const R*, int, int*, hipStream_t);                                  \
    template void launch3_gpd<R>(const G3&, const F3<R>&, const E3<R>&, const Seg3*, const Box3*, Box3*, int,  \
                                 const Push3&, int, int*, int*, int2*, bool, hipStream_t);                  \
    template void launch3_nodes<R>(const G3&, const F3<R>&, hipStream_t);                                   \
    template void launch3_gpi<R>(const G3&, const F3<R>&, const I3<R>&, const Seg3*, const Box3*, Box3*, int,  \
                                 double, double, double, const Push3&, int, hipStream_t);                   \
    template void launch3_antenna<R>(const G3&, const F3<R>&, double*, const double*, const double*,        \
                                     const Antenna3&, const Push3&, hipStream_t);                           \
    template void launch3_inject<R>(const G3&, const Tiles3&, const E3<R>&, const I3<R>&, int*, int*, Seg3*,   \
                                    Box3*, Seg3*, Box3*, int, const Inject3&, int*, hipStream_t);          \
    template void launch3_window<R>(const G3&, const F3<R>&, const Pml3&, int, hipStream_t);                \
    template void launch3_sort_e<R>(const G3&, const Tiles3&, const E3<R>&, const E3<R>&, int*, int*, int*,   \
                                    int*, Seg3*, Box3*, int64_t, int, hipStream_t);                         \
    template void launch3_sort_i<R>(const G3&, const Tiles3&, const I3<R>&, const I3<R>&, double, int*, int*,  \
                                    int*, int*, Seg3*, Box3*, int64_t, int, hipStream_t);                   \
    template void launch3_stations<R>(const G3&, const F3<R>&, const double*, int, double, double, double,  \
                                      double, double*, int*, int, hipStream_t);
BF3_INST(float)
BF3_INST(double)

}  // namespace bf3
