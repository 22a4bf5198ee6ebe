// bf_fields.hip -- grid kernels of the boosted-frame PIC step for gfx950.
//
//  * k_faraday: B^{n-1/2} -> B^{n+1/2} with the Cole-Karkkainen operator
//    Delta* = (alpha + beta S^1) Delta (Sec. 4.2, 2D: the y neighbours folded into the centre
//    and S^1 a full-cell transverse shift) applied to Friedman's
//    Etilde = (1+theta/4) E^n - 1/2 E^{n-1} + (1/2-theta/4) Ebar (Sec. 4.3, Eq.
//    Faraday_Friedman, indices shifted by one), split-field PML (Appendix II) on the borders.
//  * k_ampere: Yee Ampere E^{n+1} = E^n + dt (curl B^{n+1/2} - J) with the PML split.
//    k_faraday, first in the step, clears the raw current the deposit accumulates into.
//  * The current filter (Sec. 4.1) is the line filter of bf_sim3.hip (any stride mask) on the
//    grid seen with one y plane.
//  * k_window_rows: moving-window advance = ring offset change + clearing the new rows.
//  * k_stations: lab-frame stations (Sec. 3.2).
//  * k_rho: charge density for the Gauss diagnostic.
//
// Each thread owns one stored cell and writes every component there, so ping-pong targets
// receive a value for every cell (cells outside a component's update range are copied).
#include "bf_kernels.h"

namespace bf {

template <typename R>
struct Grid2 {
    Geo g;
    __device__ __forceinline__ R at(const R* a, int i, int k) const
    {
        i = swrap(i, g.Sx, g.perx);
        k = swrap(k, g.Sz, g.perz);
        if (i < 0 || k < 0) return R(0);
        return a[gofs(g, i, k)];
    }
};

template <typename R, bool FRIED>
__device__ __forceinline__ R etilde(const Grid2<R>& G, const FieldSet<R>& f, int c, int i, int k,
                                    R th)
{
    int ii = swrap(i, G.g.Sx, G.g.perx), kk = swrap(k, G.g.Sz, G.g.perz);
    if (ii < 0 || kk < 0) return R(0);
    long o = gofs(G.g, ii, kk);
    R e = f.E[c][o];
    if (!FRIED) return e;
    R eo = f.Eo[c][o], eb = f.Eb[c][o];
    R ebn = (R(1) - R(0.5) * th) * eo + R(0.5) * th * eb;
    return (R(1) + R(0.25) * th) * e - R(0.5) * eo + (R(0.5) - R(0.25) * th) * ebn;
}

// one 64 x 4 block of stored cells (bx, by), one thread per cell
template <typename R, bool FRIED>
__device__ __forceinline__ void faraday_block(const Geo& g, const FieldSet<R>& f, const PmlTab<R>& pm,
                                              R dt, R a2, R b2, R th, R idx, R idz, int bx, int by)
{
    const int i = bx * 64 + (threadIdx.x & 63);
    const int k = by * 4 + (threadIdx.x >> 6);
    if (i >= g.Sx || k >= g.Sz) return;
    Grid2<R> G{g};
    const long o = gofs(g, i, k);
    // x-difference of Etilde_c towards a target of x-stagger 1 (half): nodes i+1, i
    auto DX = [&](int c, int ii, int kk) -> R {
        return (etilde<R, FRIED>(G, f, c, ii + 1, kk, th) - etilde<R, FRIED>(G, f, c, ii, kk, th)) * idx;
    };
    auto DZ = [&](int c, int ii, int kk) -> R {
        return (etilde<R, FRIED>(G, f, c, ii, kk + 1, th) - etilde<R, FRIED>(G, f, c, ii, kk, th)) * idz;
    };
    // transverse neighbour validity (outside a non-periodic axis the term is zero)
    auto okx = [&](int ii) { return swrap(ii, g.Sx, g.perx) >= 0; };
    auto okz = [&](int kk) { return swrap(kk, g.Sz, g.perz) >= 0; };
    auto DXs = [&](int c) -> R {   // Delta*_x at (i + 1/2, k)
        R v = a2 * DX(c, i, k);
        if (b2 != R(0)) {
            R s = R(0);
            if (okz(k + 1)) s += DX(c, i, k + 1);
            if (okz(k - 1)) s += DX(c, i, k - 1);
            v += b2 * s;
        }
        return v;
    };
    auto DZs = [&](int c) -> R {   // Delta*_z at (i, k + 1/2)
        R v = a2 * DZ(c, i, k);
        if (b2 != R(0)) {
            R s = R(0);
            if (okx(i + 1)) s += DZ(c, i + 1, k);
            if (okx(i - 1)) s += DZ(c, i - 1, k);
            v += b2 * s;
        }
        return v;
    };
    const int xmax_n = smax(g.Sx, g.perx, 0), xmax_h = smax(g.Sx, g.perx, 1);
    const int zmax_n = smax(g.Sz, g.perz, 0), zmax_h = smax(g.Sz, g.perz, 1);
    // B_x (node x, half z): dB/dt = + Delta*_z E_y
    {
        R b = f.B[0][o];
        if (i <= xmax_n && k <= zmax_h) {
            R d = DZs(1);
            b = pm.xi[1][1][k] * b + pm.c[1][1][k] * d;
        }
        f.Bn[0][o] = b;
    }
    // B_z (half x, node z): dB/dt = - Delta*_x E_y
    {
        R b = f.B[2][o];
        if (i <= xmax_h && k <= zmax_n) {
            R d = -DXs(1);
            b = pm.xi[0][1][i] * b + pm.c[0][1][i] * d;
        }
        f.Bn[2][o] = b;
    }
    // B_y (half x, half z): dB/dt = + Delta*_x E_z - Delta*_z E_x, split in the PML
    {
        R b = f.B[1][o];
        if (i <= xmax_h && k <= zmax_h) {
            R dX = DXs(2);
            R dZ = -DZs(0);
            const bool sx = pm.on[0][1][i], sz = pm.on[1][1][k];
            if (!sx && !sz) {
                b = b + dt * (dX + dZ);
            } else {
                R px = f.Byx[o], pz = b - px;
                px = pm.xi[0][1][i] * px + pm.c[0][1][i] * dX;
                pz = pm.xi[1][1][k] * pz + pm.c[1][1][k] * dZ;
                f.Byx[o] = px;
                b = px + pz;
            }
        }
        f.Bn[1][o] = b;
    }
    if (FRIED) {
        for (int c = 0; c < 3; c++)
            f.Ebn[c][o] = (R(1) - R(0.5) * th) * f.Eo[c][o] + R(0.5) * th * f.Eb[c][o];
    }
    // the raw current of the previous step is cleared here, at the start of the step, so that
    // it stays readable between steps
    for (int c = 0; c < 3; c++) f.J[c][o] = R(0);
}

template <typename R, bool FRIED>
__global__ void __launch_bounds__(256) k_faraday(Geo g, FieldSet<R> f, PmlTab<R> pm, R dt, R a2,
                                                 R b2, R th, R idx, R idz)
{
    faraday_block<R, FRIED>(g, f, pm, dt, a2, b2, th, idx, idz, blockIdx.x, blockIdx.y);
}

template <typename R>
__device__ __forceinline__ void ampere_block(const Geo& g, const FieldSet<R>& f, const PmlTab<R>& pm,
                                             R dt, R idx, R idz, int bx, int by)
{
    const int i = bx * 64 + (threadIdx.x & 63);
    const int k = by * 4 + (threadIdx.x >> 6);
    if (i >= g.Sx || k >= g.Sz) return;
    Grid2<R> G{g};
    const long o = gofs(g, i, k);
    const int xlo_n = g.perx ? 0 : 1, zlo_n = g.perz ? 0 : 1;
    const int xhi = g.perx ? g.Sx - 1 : g.Sx - 2, zhi = g.perz ? g.Sz - 1 : g.Sz - 2;
    const R* By = f.Bn[1];
    // E_x (half x, node z): dE/dt = - Delta_z B_y - J_x
    {
        R e = f.E[0][o];
        if (i <= xhi && k >= zlo_n && k <= zhi) {
            R d = -(G.at(By, i, k) - G.at(By, i, k - 1)) * idz - f.Jf[0][o];
            e = pm.xi[1][0][k] * e + pm.c[1][0][k] * d;
        }
        f.Eo[0][o] = e;
    }
    // E_z (node x, half z): dE/dt = + Delta_x B_y - J_z
    {
        R e = f.E[2][o];
        if (i >= xlo_n && i <= xhi && k <= zhi) {
            R d = (G.at(By, i, k) - G.at(By, i - 1, k)) * idx - f.Jf[2][o];
            e = pm.xi[0][0][i] * e + pm.c[0][0][i] * d;
        }
        f.Eo[2][o] = e;
    }
    // E_y (node, node): dE/dt = - Delta_x B_z + Delta_z B_x - J_y, split in the PML
    {
        R e = f.E[1][o];
        if (i >= xlo_n && i <= xhi && k >= zlo_n && k <= zhi) {
            R dX = -(G.at(f.Bn[2], i, k) - G.at(f.Bn[2], i - 1, k)) * idx - f.Jf[1][o];
            R dZ = (G.at(f.Bn[0], i, k) - G.at(f.Bn[0], i, k - 1)) * idz;
            const bool sx = pm.on[0][0][i], sz = pm.on[1][0][k];
            if (!sx && !sz) {
                e = e + dt * (dX + dZ);
            } else {
                R px = f.Eyx[o], pz = e - px;
                px = pm.xi[0][0][i] * px + pm.c[0][0][i] * dX;
                pz = pm.xi[1][0][k] * pz + pm.c[1][0][k] * dZ;
                f.Eyx[o] = px;
                e = px + pz;
            }
        }
        f.Eo[1][o] = e;
    }
}

template <typename R>
__global__ void __launch_bounds__(256) k_ampere(Geo g, FieldSet<R> f, PmlTab<R> pm, R dt, R idx,
                                                R idz)
{
    ampere_block<R>(g, f, pm, dt, idx, idz, blockIdx.x, blockIdx.y);
}

// ---- momentum-conserving gather: fields to the nodes -------------------------------------
// Each component of E^n and of B^n = (B^{n-1/2} + B^{n+1/2}) / 2 becomes, at node (i, k), the
// mean of its values at the Yee locations around the node along its staggered axes: E_x (i -+
// 1/2, k), E_z (i, k -+ 1/2), B_x (i, k -+ 1/2), B_y the four (i -+ 1/2, k -+ 1/2), B_z (i -+ 1/2,
// k); E_y sits on the node.  Locations beyond a non-periodic edge read 0.
template <typename R>
__global__ void __launch_bounds__(256) k_nodes(Geo g, FieldSet<R> f)
{
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const int k = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (i >= g.Sx || k >= g.Sz) return;
    const int il = swrap(i - 1, g.Sx, g.perx), kl = swrap(k - 1, g.Sz, g.perz);
    auto at = [&](const R* a, int ii, int kk) { return (ii < 0 || kk < 0) ? R(0) : a[gofs(g, ii, kk)]; };
    auto bn = [&](int c, int ii, int kk) { return R(0.5) * (at(f.B[c], ii, kk) + at(f.Bn[c], ii, kk)); };
    const long o = gofs(g, i, k);
    f.G[0][o] = R(0.5) * (at(f.E[0], il, k) + at(f.E[0], i, k));
    f.G[1][o] = f.E[1][o];
    f.G[2][o] = R(0.5) * (at(f.E[2], i, kl) + at(f.E[2], i, k));
    f.G[3][o] = R(0.5) * (bn(0, i, kl) + bn(0, i, k));
    f.G[4][o] = R(0.25) * ((bn(1, il, kl) + bn(1, i, kl)) + (bn(1, il, k) + bn(1, i, k)));
    f.G[5][o] = R(0.5) * (bn(2, il, k) + bn(2, i, k));
}

template <typename R>
void launch_nodes(const Geo& g, const FieldSet<R>& f, hipStream_t s)
{
    dim3 grid((g.Sx + 63) / 64, (g.Sz + 3) / 4);
    hipLaunchKernelGGL((k_nodes<R>), grid, dim3(256), 0, s, g, f);
}

// ---- batched runs: one persistent launch per phase over a device work queue ----------------
template <typename R>
__global__ void __launch_bounds__(256) k_faraday_batch(const FaradayDesc<R>* __restrict__ d, QueueRef q)
{
    int r = 0;
    for (int k = 0;; k++) {
        const int it = stride_item(q, k);
        if (it < 0) return;
        r = run_of(q, it, r);
        const FaradayDesc<R>& D = d[r];
        const int local = it - q.off[r];
        if (D.fried)
            faraday_block<R, true>(D.g, D.f, D.pm, D.dt, D.a2, D.b2, D.th, D.idx, D.idz, local % D.gx,
                                   local / D.gx);
        else
            faraday_block<R, false>(D.g, D.f, D.pm, D.dt, D.a2, D.b2, D.th, D.idx, D.idz, local % D.gx,
                                    local / D.gx);
    }
}

template <typename R>
__global__ void __launch_bounds__(256) k_ampere_batch(const AmpereDesc<R>* __restrict__ d, QueueRef q)
{
    int r = 0;
    for (int k = 0;; k++) {
        const int it = stride_item(q, k);
        if (it < 0) return;
        r = run_of(q, it, r);
        const AmpereDesc<R>& D = d[r];
        const int local = it - q.off[r];
        ampere_block<R>(D.g, D.f, D.pm, D.dt, D.idx, D.idz, local % D.gx, local / D.gx);
    }
}


// ---- moving window -------------------------------------------------------------------------
// After the ring offset has moved by d rows: clear the d new rows of every array, drop the
// split x-part of rows that just left the z-PML for the interior (where no x-PML acts), and
// keep tangential E zero on the two end walls.
template <typename R>
__global__ void k_window_rows(Geo g, PtrList<R> arrays, int d, EntryRows er, FieldSet<R> f,
                              PmlTab<R> pm)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= g.Sx) return;
    const int kn0 = d > 0 ? g.Sz - d : 0, kn1 = d > 0 ? g.Sz : -d;
    for (int a = 0; a < arrays.n; a++)
        for (int k = kn0; k < kn1; k++) arrays.p[a][gofs(g, i, k)] = R(0);
    for (int q = 0; q < er.nh; q++)
        if (!pm.on[0][1][i]) f.Byx[gofs(g, i, er.h[q])] = R(0);
    for (int q = 0; q < er.nn; q++)
        if (!pm.on[0][0][i]) f.Eyx[gofs(g, i, er.n[q])] = R(0);
    const int walls[2] = {0, g.Sz - 1};
    for (int w = 0; w < 2; w++) {
        long o = gofs(g, i, walls[w]);
        f.E[0][o] = R(0); f.E[1][o] = R(0);
        f.Eo[0][o] = R(0); f.Eo[1][o] = R(0);
        f.Eb[0][o] = R(0); f.Eb[1][o] = R(0);
        f.Ebn[0][o] = R(0); f.Ebn[1][o] = R(0);
    }
}

// ---- stations ----------------------------------------------------------------------------
template <typename R>
__device__ double bilin(const Geo& g, const R* a, int hx, int hz, double xc, double zc)
{
    double xs = xc - 0.5 * hx, zs = zc - 0.5 * hz;
    int jx = (int)floor(xs), jz = (int)floor(zs);
    double fx = xs - jx, fz = zs - jz;
    double v = 0.0;
    for (int p = 0; p < 2; p++)
        for (int q = 0; q < 2; q++) {
            int i = swrap(jx + p + g.Px, g.Sx, g.perx), k = swrap(jz + q + g.Pz, g.Sz, g.perz);
            if (i < 0 || k < 0) continue;
            v += (p ? fx : 1.0 - fx) * (q ? fz : 1.0 - fz) * (double)a[gofs(g, i, k)];
        }
    return v;
}

template <typename R>
__global__ void k_stations(Geo g, FieldSet<R> f, StationParams sp, double* rec, int* counts)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= sp.n) return;
    double zb = sp.zlab[q] / sp.gamma - sp.beta * sp.t;     // boosted position
    double zc = (zb - sp.shift * sp.dz_um) / sp.dz_um;     // window cells
    int n = counts[q];
    if (zc < 0.0 || zc >= (double)g.Nz || n >= sp.cap) return;
    double xc = sp.xc;
    double E0 = bilin(g, f.E[0], 1, 0, xc, zc), E1 = bilin(g, f.E[1], 0, 0, xc, zc),
           E2 = bilin(g, f.E[2], 0, 1, xc, zc);
    double B0 = 0.5 * (bilin(g, f.B[0], 0, 1, xc, zc) + bilin(g, f.Bn[0], 0, 1, xc, zc));
    double B1 = 0.5 * (bilin(g, f.B[1], 1, 1, xc, zc) + bilin(g, f.Bn[1], 1, 1, xc, zc));
    double B2 = 0.5 * (bilin(g, f.B[2], 1, 0, xc, zc) + bilin(g, f.Bn[2], 1, 0, xc, zc));
    double ga = sp.gamma, be = sp.beta;
    double* r = rec + ((long)q * sp.cap + n) * 7;
    r[0] = ga * (sp.t + be * zb);
    r[1] = ga * (E0 + be * B1);
    r[2] = ga * (E1 - be * B0);
    r[3] = E2;
    r[4] = ga * (B0 - be * E1);
    r[5] = ga * (B1 + be * E0);
    r[6] = B2;
    counts[q] = n + 1;
}

// ---- charge density (diagnostic, FP64) -------------------------------------------------------
__device__ __forceinline__ double s3d(double r)
{
    double a = fabs(r);
    if (a < 1.0) return 2.0 / 3.0 - a * a + 0.5 * a * a * a;
    if (a < 2.0) { double b = 2.0 - a; return b * b * b / 6.0; }
    return 0.0;
}

__device__ void rho_add(const Geo& g, double* rho, double qw, double x, double z)
{
    int i0 = (int)floor(x), k0 = (int)floor(z);
    for (int a = -1; a <= 2; a++) {
        double sx = s3d(x - (i0 + a));
        int si = swrap(i0 + a + g.Px, g.Sx, g.perx);
        if (si < 0 || sx == 0.0) continue;
        for (int b = -1; b <= 2; b++) {
            double sz = s3d(z - (k0 + b));
            int sk = swrap(k0 + b + g.Pz, g.Sz, g.perz);
            if (sk < 0 || sz == 0.0) continue;
            atomicAdd(&rho[(long)sk * g.Sx + si], qw * sx * sz);
        }
    }
}

template <typename R>
__global__ void k_rho(Geo g, ElectronArrays<R> e, int ne, IonArrays<R> ion, int ni, double zsh,
                      const double* xm, int na, double xa_home0, double za, double aw,
                      double inv_cell, double* rho)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < ne) {
        double w = (double)e.w[p];
        if (w != 0.0) rho_add(g, rho, -w * inv_cell, e.x[p], e.z[p]);
    } else if (p < ne + ni) {
        int q = p - ne;
        double w = (double)ion.w[q];
        if (w != 0.0) rho_add(g, rho, w * inv_cell, ion.x[q], ion.z0[q] - zsh);
    } else if (p < ne + ni + na) {
        int q = p - ne - ni;
        rho_add(g, rho, -aw * inv_cell, xm[q], za);
        rho_add(g, rho, aw * inv_cell, xa_home0 + q, za);
    }
}

__global__ void k_fill_int(int* p, int n, int v)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---- launchers ------------------------------------------------------------------------------
template <typename R>
void launch_faraday_batch(const FaradayDesc<R>* d, const QueueRef& q, int nblocks, hipStream_t s)
{
    if (q.total > 0)
        hipLaunchKernelGGL((k_faraday_batch<R>), dim3(nblocks), dim3(256), 0, s, d, q);
}

template <typename R>
void launch_ampere_batch(const AmpereDesc<R>* d, const QueueRef& q, int nblocks, hipStream_t s)
{
    if (q.total > 0)
        hipLaunchKernelGGL((k_ampere_batch<R>), dim3(nblocks), dim3(256), 0, s, d, q);
}



template <typename R>
void launch_faraday(const Geo& g, const FieldSet<R>& f, const PmlTab<R>& pm, const SolverCoef& c,
                    hipStream_t s)
{
    dim3 grid((g.Sx + 63) / 64, (g.Sz + 3) / 4);
    if (c.theta > 0.0)
        hipLaunchKernelGGL((k_faraday<R, true>), grid, dim3(256), 0, s, g, f, pm, (R)c.dt, (R)c.a2,
                           (R)c.b2, (R)c.theta, (R)c.idx, (R)c.idz);
    else
        hipLaunchKernelGGL((k_faraday<R, false>), grid, dim3(256), 0, s, g, f, pm, (R)c.dt, (R)c.a2,
                           (R)c.b2, (R)c.theta, (R)c.idx, (R)c.idz);
}

template <typename R>
void launch_ampere(const Geo& g, const FieldSet<R>& f, const PmlTab<R>& pm, const SolverCoef& c,
                   hipStream_t s)
{
    dim3 grid((g.Sx + 63) / 64, (g.Sz + 3) / 4);
    hipLaunchKernelGGL((k_ampere<R>), grid, dim3(256), 0, s, g, f, pm, (R)c.dt, (R)c.idx, (R)c.idz);
}

template <typename R>
void launch_window_rows(const Geo& g, const PtrList<R>& arrays, int d, const EntryRows& er,
                        const FieldSet<R>& f, const PmlTab<R>& pm, hipStream_t s)
{
    hipLaunchKernelGGL((k_window_rows<R>), dim3((g.Sx + 255) / 256), dim3(256), 0, s, g, arrays, d, er,
                       f, pm);
}

template <typename R>
void launch_stations(const Geo& g, const FieldSet<R>& f, const StationParams& sp, double* rec,
                     int* counts, hipStream_t s)
{
    if (sp.n <= 0) return;
    hipLaunchKernelGGL((k_stations<R>), dim3(1), dim3(64), 0, s, g, f, sp, rec, counts);
}

template <typename R>
void launch_rho(const Geo& g, const ElectronArrays<R>& e, int ne, const IonArrays<R>& ion, int ni,
                double zsh, const double* xm, int na, double xa_home0, double za, double aw,
                double inv_cell, double* rho, hipStream_t s)
{
    int n = ne + ni + na;
    if (n <= 0) return;
    hipLaunchKernelGGL((k_rho<R>), dim3((n + 255) / 256), dim3(256), 0, s, g, e, ne, ion, ni, zsh, xm,
                       na, xa_home0, za, aw, inv_cell, rho);
}

__global__ void k_rho_beam(Geo g, BeamArrays b, int n, double inv_cell, double* rho)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n || b.state[p] == 2) return;
    const double x = b.x[p], z = b.z[p];
    if (!g.perx && (x < 0.0 || x >= (double)g.Nx)) return;
    if (!g.perz && (z < 0.0 || z >= (double)g.Nz)) return;
    rho_add(g, rho, -b.w[p] * inv_cell, x, z);
}

void launch_rho_beam(const Geo& g, const BeamArrays& b, int n, double inv_cell, double* rho, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_rho_beam, dim3((n + 255) / 256), dim3(256), 0, s, g, b, n, inv_cell, rho);
}

void launch_fill_int(int* p, int n, int v, hipStream_t s)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_int, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
}

#define BF_INST(R)                                                                                 \
    template void launch_faraday<R>(const Geo&, const FieldSet<R>&, const PmlTab<R>&,              \
                                    const SolverCoef&, hipStream_t);                               \
    template void launch_nodes<R>(const Geo&, const FieldSet<R>&, hipStream_t);                       \
    template void launch_ampere<R>(const Geo&, const FieldSet<R>&, const PmlTab<R>&,               \
                                   const SolverCoef&, hipStream_t);                                \
    template void launch_faraday_batch<R>(const FaradayDesc<R>*, const QueueRef&, int, hipStream_t); \
    template void launch_ampere_batch<R>(const AmpereDesc<R>*, const QueueRef&, int, hipStream_t);   \
    template void launch_window_rows<R>(const Geo&, const PtrList<R>&, int, const EntryRows&,      \
                                        const FieldSet<R>&, const PmlTab<R>&, hipStream_t);        \
    template void launch_stations<R>(const Geo&, const FieldSet<R>&, const StationParams&,         \
                                     double*, int*, hipStream_t);                                  \
    template void launch_rho<R>(const Geo&, const ElectronArrays<R>&, int, const IonArrays<R>&,    \
                                int, double, const double*, int, double, double, double, double,   \
                                double*, hipStream_t);
BF_INST(float)
BF_INST(double)

}  // namespace bf
