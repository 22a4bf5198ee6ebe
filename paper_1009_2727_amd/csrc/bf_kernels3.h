// bf_kernels3.h -- device-side types and launchers of the 3D step (x, y transverse, z the boost
// axis).  Fields are [z plane][y row][x] with a padded x pitch; the z planes form a ring buffer
// (stored plane = (plane + zoff) mod Sz) so that the moving window only moves zoff and clears
// the planes that wrap round.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace bf3 {

struct G3 {
    int N[3];          // interior cells
    int S[3];          // stored cells (N + 2 P + 1 on a non-periodic axis, N on a periodic one)
    int P[3];          // PML depth (0 on a periodic axis)
    int per[3];        // periodic flags
    long pitch, plane; // x pitch and plane stride (elements)
    int zoff;          // ring offset of the z planes
    double d[3];       // cell sizes
};

// per-axis PML coefficients at nodes (h = 0) and half nodes (h = 1): sigma, xi = exp(-sigma dt)
// and c = (1 - xi) / sigma (dt where sigma = 0); entry [axis][h] points at S[axis] values
struct Pml3 {
    const double* sig[3][2];
    const double* xi[3][2];
    const double* c[3][2];
};

template <typename R>
struct F3 {
    R* E[3];
    R* Eo[3];   // E^{n-1}
    R* Eb[3];   // Friedman average
    R* B[3];
    R* Bo[3];   // B^{n-1/2} (kept for the gather average)
    double* J[3];   // deposited current, accumulated in FP64 (the electron and ion currents
                    // nearly cancel in a plasma drifting at -beta c)
    R* Jf[3];       // filter passes ping-pong between Jf and Jg
    R* Jg[3];
    R* SE[3];   // PML split parts of E (part along the cyclic-next axis)
    R* SB[3];   // PML split parts of B
    R* T[3];    // the other Ebar buffer: Faraday writes the new Friedman average here
    R* G[6];    // momentum-conserving gather: E^n and B^n interpolated to the nodes (else null)
};

template <typename R>
struct E3 {     // electrons: positions in cells of the current window (FP64)
    double *x, *y, *z;
    R *ux, *uy, *uz, *w;
    uint32_t* id;
};

template <typename R>
struct I3 {     // rigid ions: x, y fixed, z0 the boosted position at t = 0 (cells)
    double *x, *y, *z0;
    R* w;
    uint32_t* id;
};

struct Push3 {
    double dt;          // time step
    double dtd[3];      // dt / d (cells per unit velocity)
    double jk[3];       // -q w factor of J_c: 1 / (d_a1 d_a2 dt) (times q w per particle)
    double shift;       // whole cells the window moves at the end of this step
    int vay;            // 1: Vay's pusher, 0: Boris
};

// particle segment: a contiguous index range whose particles share a cell box
struct Seg3 { int start, count; };
// cell bounding box (interior cells, inclusive); empty when lo > hi
struct Box3 { int lo[3], hi[3]; };
// tiles of the particle sort: t cells per tile along each axis, nt tiles per axis
struct Tiles3 { int t[3]; int nt[3]; int ntiles; };

// LDS box of the particle kernels: a segment's cell box widened by the stencil reach (2 cells
// below, 3 above) must fit BOX_PX x BOX_PY cells transversely and the run's plane count in z.
// Planes are BOX_PL cells apart.  The 8-byte LDS adds of the deposit are served 16 lanes at a
// time, two lanes conflicting when their word indices agree mod 16.  The particle tiles are 16
// cells wide in x, so a quarter-wave (one row of 16 cells of a lattice-ordered wave) adds to 16
// distinct slots, and the plane stride of 0 (mod 16) keeps a lane whose stencil starts one plane
// lower (a z face crossed, or a z-staggered component's lower half cell) on its own slot.
constexpr int BOX_PX = 24, BOX_PY = 10, BOX_PL = BOX_PX * BOX_PY;
// LDS bytes per box cell of the electron kernel: 6 field components in the run's type and 3
// current accumulators of 8 bytes
template <typename R> constexpr int box_cell_bytes() { return 6 * (int)sizeof(R) + 24; }

struct Inject3 {
    int64_t row0;
    int nrows, ppc, ion_mode;
    int64_t cap;
    uint64_t seed;
    double gamma, beta, t, dx, dy, dz, n0, ramp_start, ramp_len, uz0, shift;
};

struct Antenna3 {
    int n;              // transverse cells
    double za, zb;      // plane position at t_n and t_{n+1} (cells)
    double tm;          // time of the emitted field
    double e0g, w0, xc, yc, gamma, t0, sig_t, omega;
    double aw;          // macro-weight of each sheet particle
    int pol;            // axis the - sheet particle moves along: 0 x, 1 y
};

// status bits (same meaning as the 2D path)
constexpr int ST3_CAPACITY = 1, ST3_NONFINITE = 2;

// Faraday + PML, with Friedman's E-tilde (theta > 0) made from E, E^{n-1} and Ebar on the fly;
// the new Ebar is written to f.T (the caller swaps the two Ebar buffers after the step)
template <typename R>
void launch3_faraday(const G3& g, const F3<R>& f, const Pml3& pml, const double ck[3], double theta, double dt,
                     hipStream_t s);
template <typename R>
void launch3_ampere(const G3& g, const F3<R>& f, const R* const J[3], const Pml3& pml, double dt, hipStream_t s);
// The passes of the current filter along one axis (Sec. 4.1, Eqs. 3ptfilter and
// 3ptfilter_stride): for each stride of the mask in ascending order, npass passes with
// alpha = 1/2 and, when asked, one compensation pass with alpha = npass/2 + 1.  reach is the sum
// of the strides: a cell's result depends on the input within reach cells along the axis.
constexpr int FSEQ_MAX = 48;       // passes per axis
constexpr int FREACH_MAX = 128;    // reach per axis
struct FiltSeq {
    int n, reach;
    double alpha[FSEQ_MAX];
    int stride[FSEQ_MAX];
};
// builds the sequence; false when it exceeds FSEQ_MAX passes or FREACH_MAX cells of reach
bool filter_seq(int npass, int comp, int stride_mask, FiltSeq* fs);
// the whole filter on J (FP64 accumulators) into the run's type, one launch per axis for the
// three components (Jf <- J along x, Jg <- Jf along y, Jf <- Jg along z); out[] receives each
// component's result.  Without passes J is copied into Jf.
template <typename R>
void launch3_filter(const G3& g, const F3<R>& f, const FiltSeq& fs, const R* out[3], hipStream_t s);
// the filter on up to three arrays of a grid with a single y plane (the 2-1/2D layout: S[1] = 1,
// plane = the row pitch, the ring on z): in -> tmp along x, tmp -> out along z.  hx, hz: each
// array's staggers.  Without passes in is copied into out.
template <typename T>
void launch_filter_xz(const G3& g, const T* const in[3], T* const tmp[3], T* const out[3], const int hx[3],
                      const int hz[3], int ncomp, const FiltSeq& fs, hipStream_t s);
// the same filter on one FP64 array of nodal stagger (the charge density of the Gauss
// diagnostic): a -> b along x, b -> c along y, c -> b along z; returns b
double* launch3_filter_nodal(const G3& g, double* a, double* b, double* c, const FiltSeq& fs, hipStream_t s);
// charge density on the nodes (FP64, cubic shape) of the electrons, rigid ions (at z0 - zsh) and
// antenna sheets (plane at za cells; + at home, - at its moving coordinate along pol) into rho
// (cleared here); vol_inv = 1 / cell volume
template <typename R>
void launch3_rho(const G3& g, const E3<R>& e, int ne, const I3<R>& ion, int ni, double zsh, const double* ant,
                 int na, int pol, double za, double aw, double vol_inv, double* rho, hipStream_t s);
template <typename R> void launch3_zero_j(const G3& g, const F3<R>& f, hipStream_t s);
// gather, push and deposit of the electrons of nseg segments (one workgroup each); bin holds
// each segment's cell box at the start of the step, bout receives the box after the push (in
// the next window frame); pz = z planes of the LDS box
// lists: 2 + nseg ints of scratch, mis: one int2 per particle slot (particles outside their
// segment's box and segments too large for LDS are pushed in a second pass, on HBM)
template <typename R>
void launch3_gpd(const G3& g, const F3<R>& f, const E3<R>& e, const Seg3* seg, const Box3* bin, Box3* bout,
                 int nseg, const Push3& pp, int pz, int* status, int* lists, int2* mis, bool mc, hipStream_t s);
// momentum-conserving gather, first step: E^n and B^n = (B^{n-1/2} + B^{n+1/2})/2 interpolated to
// the nodes (the mean over the Yee locations around each node along the staggered axes) into f.G
template <typename R> void launch3_nodes(const G3& g, const F3<R>& f, hipStream_t s);
// rigid-ion J_z of nseg segments: z = z0 - zsa at t_n, z0 - zsb at t_{n+1}, z0 - zsn in the
// next window frame (for the boxes)
template <typename R>
void launch3_gpi(const G3& g, const F3<R>& f, const I3<R>& ion, const Seg3* seg, const Box3* bin, Box3* bout,
                 int nseg, double zsa, double zsb, double zsn, const Push3& pp, int pz, hipStream_t s);
template <typename R>
void launch3_antenna(const G3& g, const F3<R>& f, double* xm, const double* xh, const double* yh,
                     const Antenna3& a, const Push3& pp, hipStream_t s);
// lattice planes into slots nused.. of both species, laid out in transverse tile chunks; chunk
// c of plane r becomes segment seg_base + r * chunks + c (table and box of each species)
template <typename R>
void launch3_inject(const G3& g, const Tiles3& tl, const E3<R>& e, const I3<R>& ion, int* nused_e, int* nused_i,
                    Seg3* seg_e, Box3* box_e, Seg3* seg_i, Box3* box_i, int seg_base, const Inject3& ip,
                    int* status, hipStream_t s);
// window moved by d planes (zoff already advanced): clear the planes that wrapped round, drop
// split parts in planes that just left the z PML, keep tangential E zero on the end walls
template <typename R>
void launch3_window(const G3& g, const F3<R>& f, const Pml3& pml, int d, hipStream_t s);
// counting sort of the live particles (w != 0) of slots [0, *nused) of src by tile, through dst
// (scatter by tile into dst, then each tile back into src in plasma-lattice order, ppc
// particles per lattice cell):
// segment t = tile t with its cell box, *nused = live count; counts/cursor hold ntiles ints,
// tot one int of scratch.  Ions are binned at z0 - zsh.
template <typename R>
void launch3_sort_e(const G3& g, const Tiles3& tl, const E3<R>& src, const E3<R>& dst, int* nused, int* counts,
                    int* cursor, int* tot, Seg3* seg, Box3* box, int64_t cap, int ppc, hipStream_t s);
template <typename R>
void launch3_sort_i(const G3& g, const Tiles3& tl, const I3<R>& src, const I3<R>& dst, double zsh, int* nused,
                    int* counts, int* cursor, int* tot, Seg3* seg, Box3* box, int64_t cap, int ppc, hipStream_t s);
// live particles (w != 0) among n slots into *cnt (zeroed here)
template <typename R> void launch3_count_live(const R* w, int n, int* cnt, hipStream_t s);
template <typename R>
void launch3_stations(const G3& g, const F3<R>& f, const double* zlab, int nst, double gamma, double beta,
                      double t, double shift_cells, double* rec, int* cnt, int cap, hipStream_t s);

}  // namespace bf3
