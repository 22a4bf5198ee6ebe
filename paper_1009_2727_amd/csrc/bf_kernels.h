// bf_kernels.h -- kernel parameter blocks and the host-side launch functions of the
// gfx950 kernels (definitions in bf_fields.hip and bf_particles.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "bf_device.h"

namespace bf {

// One set of field pointers for a step.  Ping-pong pairs are resolved by the host:
//   E   = E^n,        Eo  = E^{n-1} (Ampere writes E^{n+1} there)
//   Eb  = Ebar read,  Ebn = Ebar written (Friedman recursion, Sec. 4.3)
//   B   = B^{n-1/2},  Bn  = B^{n+1/2} (written by Faraday)
//   J   = raw deposit, Jf = filtered current read by Ampere (== J without filter)
//   Byx, Eyx = x-parts of the split PML components (Appendix II)
template <typename R>
struct FieldSet {
    R* E[3];
    R* Eo[3];
    R* Eb[3];
    R* Ebn[3];
    R* B[3];
    R* Bn[3];
    R* J[3];
    R* Jf[3];
    R* Byx;
    R* Eyx;
    R* G[6];    // momentum-conserving gather: E^n and B^n interpolated to the nodes (else unused)
};

// PML coefficient tables indexed [axis 0 x / 1 z][stagger 0 node / 1 half]; x tables by
// stored index, z tables by logical row.  xi = exp(-sigma dt), c = (1 - xi)/sigma (dt where
// sigma = 0), on = sigma > 0.
template <typename R>
struct PmlTab {
    const R* xi[2][2];
    const R* c[2][2];
    const uint8_t* on[2][2];
};

struct SolverCoef {
    double dt, a2, b2, theta, idx, idz;
};

// particle arrays (structure of arrays)
template <typename R>
struct ElectronArrays {
    double* x;   // cells, interior-relative, unwrapped on periodic axes between sorts
    double* z;
    R* ux;
    R* uy;
    R* uz;
    R* w;        // 0 marks a free / absorbed slot
    uint32_t* id;
};

template <typename R>
struct IonArrays {
    double* x;   // cells
    double* z0;  // cells, boosted position at t = 0 (absolute lattice coordinate)
    R* w;
    uint32_t* id;
};

struct Segment {
    int start, count;
};

// per-step particle parameters
template <typename R>
struct PushParams {
    R qdt2;            // q dt / (2 m) for electrons (q = -1, m = 1)
    R dtdx, dtdz;      // dt / dx, dt / dz  (cell units per unit velocity)
    R fjx, fjz, fjy;   // -q/(dz dt), -q/(dx dt), q/(dx dz)   (times w, v_y)
    int shift;         // window shift (cells) applied after this step
    int vay;           // 1: Vay's pusher, 0: Boris
};

struct InjectParams {
    int64_t row0;      // first lattice row to create
    int nrows, nchunks, tile_x, ppc, ion_mode;
    double beta, gamma, t, dz_um, dx_um, shift;
    double n0, ramp_start, ramp_len;   // lab profile (um, normalised density)
    double wfac;       // gamma dx dz / ppc
    double uz0;        // -gamma beta
    uint64_t seed;
    int seg_base;      // first segment slot written
    int64_t cap;
};

struct AntennaParams {
    int n;             // sheet particles per sign (one per transverse cell)
    double za, zb;     // plane position (cells) at t_n and t_{n+1}, current window frame
    double tmid;       // t_n + dt/2 (um/c)
    double gamma, e0, omega, w0, sig_t, t0, dx_um, xc_um;
    double weight;     // |q| w of each sheet particle
    double dt, dx, dz; // um
    int active;
    int pol;           // 0: the - sheet moves along x (J_x); 1: along y, out of the plane (J_y)
};

// particle beam launched through a lab-fixed plane (Sec. 3.1.1): FP64 state in the work buffer
struct BeamArrays {
    double *x, *z;        // cells, current window frame
    double *ux, *uy, *uz; // calculation-frame momenta gamma v / c
    double* w;            // macro-weight
    double* tact;         // boosted time t'* at which the particle crosses the plane (um/c)
    int* state;           // 0 frozen, 1 active, 2 lost
    double* hist;         // one record of 8 doubles per step (see BF_DIAG_BEAM)
};
struct BeamParams {
    int n;
    int deposit;          // 1: frozen and active particles deposit current
    int rec;              // history record of this step (-1: the history is full)
    double t0, t1;        // t_n, t_{n+1} (um/c)
    double vbar_cells;    // frozen move per step: vbar' dt / dz
    double gamma, beta, dz_um;
    double shift;         // window cells moved before this step (lab back-transformation)
};

struct StationParams {
    int n;
    const double* zlab;
    double gamma, beta, t, dz_um, shift;
    double xc;         // transverse centre (cells)
    int cap;
};

// ---- batched runs: per-run arguments of the persistent launch of each phase ------------
template <typename R>
struct FaradayDesc {
    Geo g;
    FieldSet<R> f;
    PmlTab<R> pm;
    R dt, a2, b2, th, idx, idz;
    int fried, gx;     // Friedman on; blocks per row of the 64 x 4 block grid
};
template <typename R>
struct AmpereDesc {
    Geo g;
    FieldSet<R> f;
    PmlTab<R> pm;
    R dt, idx, idz;
    int gx;
};
template <typename R>
struct GpdDesc {
    Geo g;
    FieldSet<R> f;
    ElectronArrays<R> e;
    const Segment* seg;
    const int4* bbin;
    int4* bbout;
    PushParams<R> pp;
    int* status;
};

template <typename R>
void launch_faraday_batch(const FaradayDesc<R>* d, const QueueRef& q, int nblocks, hipStream_t s);
template <typename R>
void launch_ampere_batch(const AmpereDesc<R>* d, const QueueRef& q, int nblocks, hipStream_t s);
template <typename R>
void launch_gpd_batch(const GpdDesc<R>* d, const QueueRef& q, int nblocks, hipStream_t s);

// ---- launchers (stream-ordered) -------------------------------------------------------
template <typename R>
void launch_faraday(const Geo& g, const FieldSet<R>& f, const PmlTab<R>& pm, const SolverCoef& c,
                    hipStream_t s);
template <typename R>
void launch_ampere(const Geo& g, const FieldSet<R>& f, const PmlTab<R>& pm, const SolverCoef& c,
                   hipStream_t s);
template <typename R>
struct PtrList {
    R* p[32];
    int n;
};
struct EntryRows {
    int h[4], nh;   // half-z rows whose split B_y x-part is dropped
    int n[4], nn;   // node-z rows whose split E_y x-part is dropped
};
template <typename R>
void launch_window_rows(const Geo& g, const PtrList<R>& arrays, int d, const EntryRows& er,
                        const FieldSet<R>& f, const PmlTab<R>& pm, hipStream_t s);
template <typename R>
void launch_stations(const Geo& g, const FieldSet<R>& f, const StationParams& sp,
                     double* rec, int* counts, hipStream_t s);
// momentum-conserving gather, first step: E^n and B^n = (B^{n-1/2} + B^{n+1/2})/2 interpolated to
// the nodes (the mean over the Yee locations around each node along the staggered axes) into f.G
template <typename R>
void launch_nodes(const Geo& g, const FieldSet<R>& f, hipStream_t s);
// gather, push and deposit; mc: the gather reads f.G with nodal weights for every component
template <typename R>
void launch_gpd(const Geo& g, const FieldSet<R>& f, const ElectronArrays<R>& e,
                const Segment* seg, const int4* bbox_in, int4* bbox_out, int nseg,
                const PushParams<R>& pp, int* status, bool mc, hipStream_t s);
template <typename R>
void launch_ions(const Geo& g, const FieldSet<R>& f, const IonArrays<R>& ion, const Segment* seg,
                 const int4* bbox_in, int4* bbox_out, int nseg, double zsh_a, double zsh_b,
                 int shift, R fjz, hipStream_t s);
template <typename R>
void launch_antenna(const Geo& g, const FieldSet<R>& f, double* xminus, const AntennaParams& ap,
                    hipStream_t s);
template <typename R>
void launch_inject(const Geo& g, const ElectronArrays<R>& e, const IonArrays<R>& ion,
                   Segment* seg_e, int4* bbox_e, Segment* seg_i, int4* bbox_i,
                   int* nused_e, int* nused_i, const InjectParams& ip, int* status,
                   hipStream_t s);
template <typename R>
void launch_sort_electrons(const Geo& g, int tile_x, int tile_z, int ntx, int ntiles,
                           const ElectronArrays<R>& src, const ElectronArrays<R>& dst,
                           const Segment* seg_old, int nseg_old, Segment* seg_new, int4* bbox_new,
                           int* counts, int* cursor, int* nused, hipStream_t s);
template <typename R>
void launch_sort_ions(const Geo& g, int tile_x, int tile_z, int ntx, int ntiles,
                      const IonArrays<R>& src, const IonArrays<R>& dst, const Segment* seg_old,
                      int nseg_old, Segment* seg_new, int4* bbox_new, double zsh, int* counts,
                      int* cursor, int* nused, hipStream_t s);
template <typename R>
void launch_rho(const Geo& g, const ElectronArrays<R>& e, int ne, const IonArrays<R>& ion,
                int ni, double zsh, const double* xm, int na, double xa_home0, double za,
                double aw, double inv_cell, double* rho, hipStream_t s);
void launch_fill_int(int* p, int n, int v, hipStream_t s);
// one step of the beam at t_n: frozen particles whose crossing time has come become active;
// frozen ones move along z at vbar', active ones are gathered (mc: from the node values f.G),
// pushed in FP64 (pp.vay: Vay, else Boris) and absorbed outside the interior; both deposit
// into f.J when bp.deposit; positions are rebased by pp.shift; the active particles' lab-frame
// sums go to record bp.rec of the history
template <typename R>
void launch_beam(const Geo& g, const FieldSet<R>& f, const BeamArrays& b, const BeamParams& bp,
                 const PushParams<double>& pp, int* status, bool mc, hipStream_t s);
// charge density of the beam's frozen and active particles inside the interior into rho
// (the layout of launch_rho)
void launch_rho_beam(const Geo& g, const BeamArrays& b, int n, double inv_cell, double* rho, hipStream_t s);

}  // namespace bf
