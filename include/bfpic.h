/*
 * bfpic.h -- C ABI of the MI355X (gfx950) boosted-frame laser-wakefield PIC library.
 *
 * The calls follow the way the paper (Vay, Geddes, Cormier-Michel, Grote, arXiv:1009.2727)
 * states the problem: choose the frame (Sec. 2, boosted quantities), give the plasma
 * (Table "Tablephyspar2d": density, length, entrance ramp) and the laser emitted through a
 * plane (Sec. 3.1.2), give the numerical parameters (tunable solver Table "CKcoefs",
 * Friedman theta Sec. 4.3, filter passes and compensation Sec. 4.1, PML Appendix II, time
 * step at a fraction of the CFL limit Eq. cfl), step, and collect lab-frame outputs through
 * stations (Sec. 3.2), fields and particles.
 *
 * Conventions
 *  - Geometry: 2-1/2D, the plane (x, z), z the boost and laser axis.  Interior cells
 *    nx * nz; every non-periodic face carries a split-field PML of pml_cells cells.
 *  - Units at the boundary: lengths in um, durations in fs, densities in cm^-3, laser and
 *    plasma always given in the LAB frame (the library applies the boost).
 *  - Ownership: the caller owns every device byte.  bf_query_buffers() lists the device
 *    buffers a configuration needs (name, size, alignment); the caller allocates each
 *    (e.g. torch.empty on the HIP device) and passes them to bf_create().  The library never
 *    allocates or frees device memory; bf_destroy() frees host metadata only.  Buffers must
 *    stay valid until bf_destroy().  Host pointers passed to the other calls are only read
 *    or written during the call.
 *  - Streams: every launch goes to the hipStream_t given to bf_create(); bf_step() is
 *    asynchronous.  bf_diagnose(), bf_sync_status(), bf_get_state() and the particle/field
 *    copies synchronise the stream.  A handle is not thread-safe.
 *  - Errors: status codes only, no exceptions or aborts cross the ABI.  Device-side
 *    conditions (particle capacity exceeded, non-finite momentum) are sticky bits reported
 *    by the next synchronising call; after such an error the handle accepts only
 *    bf_diagnose(), bf_get_state(), bf_last_error() and bf_destroy() (BF_ESTATE otherwise).
 */
#ifndef BFPIC_H
#define BFPIC_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BF_ABI_VERSION 5u

typedef enum {
    BF_OK = 0,
    BF_EINVAL = -1,        /* malformed argument or configuration                          */
    BF_ECFL = -2,          /* time step above the (Friedman-corrected) CFL limit           */
    BF_ECAPACITY = -3,     /* particle or segment capacity exceeded on the device          */
    BF_ENONFINITE = -4,    /* non-finite particle momentum detected                        */
    BF_EDEVICE = -5,       /* HIP runtime error                                            */
    BF_ESTATE = -6,        /* call not allowed in the handle's current state               */
    BF_EUNSUPPORTED = -7   /* valid request this build does not implement                  */
} bf_status;

typedef struct bf_sim bf_sim;

/* Simulation configuration.  abi_version must be BF_ABI_VERSION and struct_size
   sizeof(bf_config). */
typedef struct {
    uint32_t abi_version, struct_size;
    int dim;                   /* 2 (x, z plane) or 3 (x, y transverse, z the boost axis)      */
    int nx, ny, nz;            /* interior cells (ny unused in 2D)                             */
    double dx_um, dy_um, dz_um;/* cell sizes in the calculation frame                          */
    int real_bytes;            /* 4: FP32 fields/momenta, 8: FP64 throughout                   */
    int shape_order;           /* 3: cubic B-spline gather and deposit (Sec. 4)                */
    double ck_alpha, ck_beta, ck_gamma; /* tunable-solver coefficients, 3D values of Table
                                           CKcoefs; 2D folds the y neighbours in            */
    double friedman_theta;     /* 0 <= theta <= 1 (Sec. 4.3)                                    */
    double cfl_fraction;       /* dt = cfl_fraction * dt*_c (Eq. cfl x sqrt((2+t)/(2+3t)))      */
    int filter_npass;          /* bilinear passes per axis (Sec. 4.1)                          */
    int filter_compensate;     /* 1: one extra pass with alpha_c = n/2 + 1                     */
    int filter_kind;           /* BF_FILTER_BILINEAR, or BF_FILTER_LEARNED (FP32 runs only;
                                  weights from bf_set_learned_filter)                         */
    int filter_strides;        /* bilinear filter strides (Eq. 3ptfilter_stride): bit s-1 set
                                  applies the npass passes (+ compensation) with stride s, in
                                  ascending order of s, e.g. 0x3 = S(1:2), 0x7 = S(1:2:3),
                                  0xB = S(1:2:4); 0 means stride 1 only.  BF_EINVAL beyond
                                  stride 16, 48 passes or a reach of 128 cells per axis       */
    int gather_kind;           /* 0: energy conserving, each field component gathered from its
                                  own Yee location (Sec. 5.1); 1: momentum conserving, the
                                  fields interpolated to the nodes first (Sec. 5.3)           */
    int pusher;                /* 0: Boris; 1: Vay (Phys. Plasmas 15, 056701, 2008)            */
    int pml_cells;             /* PML depth on non-periodic faces (Appendix II)                */
    int periodic_mask;         /* bit 0: x, bit 1: y (3D), bit 2: z periodic (no moving window) */
    double gamma_boost;        /* Lorentz factor of the calculation frame (>= 1)              */
    int moving_window;         /* 1: window follows the wake at beta_w* c (Sec. 2)             */
    int64_t particle_capacity; /* slots per species (electrons; rigid ions alike)              */
    int sort_every;            /* steps between tile sorts (0: library default, 20)            */
    int tile_x, tile_z;        /* particle tile in cells (0: library default, 26 x 8)          */
    int max_stations;          /* lab-frame stations that may be added                         */
    int station_capacity;      /* samples kept per station                                     */
    int phase_timers;          /* 1: record HIP events around every phase of bf_step          */
    uint64_t seed;             /* counter-based RNG seed for plasma loading                    */
    int64_t beam_capacity;     /* beam macro-particles bf_add_beam may load (2D runs; 0: none)  */
    int32_t beam_history;      /* per-step beam records kept (BF_DIAG_BEAM, arg 1)             */
    int32_t pml_kind;          /* 0: curl coefficient (1 - xi)/sigma; 1: the modified
                                  coefficients (Appendix II, sigma*): dt kappa(p) with
                                  kappa(p + 1/2) kappa(p) = xi(p) outwards from the layer's
                                  inner edge (kappa = 1 inside), which lets a normally incident
                                  wave at c dt = delta cross every half cell unreflected.
                                  BF_EUNSUPPORTED with a CK solver above 0.95 of its Courant
                                  limit, where this layer is unstable                          */
} bf_config;

/* Plasma given in the lab frame: zero density before start_um, linear up-ramp of ramp_um
   (0: step), then the plateau n0_cm3.  ppc macro-electrons per cell, placed uniformly at
   random in each cell by SplitMix64 keyed by (seed, lattice row, cell, index).
   ion_mode 0: immobile neutralising background (lab frame), 1: ions at rest in the lab,
   i.e. drifting rigidly at -beta c in the calculation frame and depositing current. */
typedef struct {
    double n0_cm3, ramp_um, start_um;
    int ppc;
    int ion_mode;
} bf_plasma;

/* Laser given in the lab frame (Sec. 3.1.2): wavelength, normalised amplitude a0, 1/e
   field waist, intensity FWHM duration, lab position of the emitting plane, lab time at
   which the pulse peak crosses the plane (0 selects 3 sigma_t, so nothing is emitted before
   t = 0; negative is BF_EINVAL), and the linear polarisation: 0 along x, 1 along y (in 2D
   the out-of-plane component, E_y, B_x, B_z and J_y).  Any other pol is BF_EINVAL. */
typedef struct {
    double lambda_um, a0, waist_um, fwhm_fs, z_antenna_um;
    double t_peak_fs;
    int pol;
} bf_laser;

/* Lab-frame station: fields sampled on axis at the lab position z_lab_um, back-transformed
   to the lab frame (Sec. 3.2). */
typedef struct {
    double z_lab_um;
} bf_station;

/* Device buffer descriptor / binding.  dtype is informational (0: raw bytes). */
typedef struct { const char* name; size_t bytes; size_t align; int dtype; } bf_buffer_desc;
typedef struct { const char* name; void* ptr; size_t bytes; } bf_buffer_binding;

/* Scalar run state (checkpointing). */
typedef struct {
    uint32_t abi_version, struct_size;
    int64_t step;              /* steps taken                                                  */
    double time;               /* calculation-frame time (um / c)                              */
    int64_t shift;             /* whole cells the window has moved                             */
    int64_t next_row;          /* next plasma lattice row to create                            */
    int32_t zoff;              /* ring offset of the z rows                                    */
    int32_t e_cur, b_cur, p_cur; /* which half of each ping-pong pair is current              */
    int32_t nseg_e, nseg_i;    /* particle segments in use                                     */
    int32_t since_sort;
    int32_t have_plasma, have_laser, nstations;
    int32_t have_beam, beam_test_only;  /* beam loaded; it deposits no current                 */
    int64_t beam_n, beam_records;       /* beam macro-particles; history records written      */
    double beam_vbar;                   /* boosted mean beam velocity (c = 1)                  */
} bf_state;

/* ---- set-up ---------------------------------------------------------------------------- */

/* Pure: validates cfg (BF_EINVAL, BF_ECFL) and lists the device buffers it needs.  On entry
   *n_inout is the capacity of out (may be 0 with out == NULL); on return the number of
   buffers.  Names are static strings. */
bf_status bf_query_buffers(const bf_config* cfg, bf_buffer_desc* out, int* n_inout);

/* Creates a handle over caller-owned buffers (every name from bf_query_buffers must be
   bound with at least the listed size and alignment).  hip_stream: hipStream_t or NULL for
   the default stream.  Buffers are cleared on the stream. */
bf_status bf_create(const bf_config* cfg, const bf_buffer_binding* bindings, int n,
                    void* hip_stream, bf_sim** out);

/* Loads the plasma lattice rows lying inside the window at t = 0 (Sec. 3.1.1: background
   plasma fixed in the lab, created continuously at the front plane afterwards). */
bf_status bf_init_plasma(bf_sim* sim, const bf_plasma* plasma);

/* Installs the laser antenna: one positive and one negative macro-particle per transverse
   cell on the lab-fixed plane (Sec. 3.1.2). */
bf_status bf_init_laser(bf_sim* sim, const bf_laser* laser);

/* Adds a lab-frame station; *station_id receives its index. */
bf_status bf_add_station(bf_sim* sim, const bf_station* station, int* station_id);

/* Replaces the electron set by n explicit particles (host arrays, positions in um relative
   to the interior origin, momenta u = gamma v / c, weights in the library's normalised
   units).  id may be NULL.  Ions and antenna are unchanged.  2D runs only. */
bf_status bf_load_electrons(bf_sim* sim, int64_t n, const uint32_t* id, const double* x,
                            const double* z, const double* ux, const double* uy,
                            const double* uz, const double* w);

/* The same for a 3D run (dim == 3), with the y positions. */
bf_status bf_load_electrons3(bf_sim* sim, int64_t n, const uint32_t* id, const double* x,
                             const double* y, const double* z, const double* ux, const double* uy,
                             const double* uz, const double* w);

/* Particle beam launched through a lab-fixed plane (Sec. 3.1.1, steps 1-3): the caller gives
   each macro-particle's LAB state at t = 0 (the standard synchronisation z = z' = 0 at
   t = t' = 0); the library projects it ballistically onto the plane z = z_inj_um
   (Eqs. t*, x*), Lorentz transforms the crossing event and the momentum (Eqs. tp*-vzp*, with
   each particle's own v_z, which they equal at the mean velocity), and synchronises the beam
   at t' = 0 (Eq. zp) at the boosted mean velocity vbar' = (beta_b - beta)/(1 - beta beta_b).
   Until a step starts at t_n >= t'* (the particle has crossed the plane) it is frozen: it
   moves along z at vbar' with transverse position and momentum fixed.  Then it is pushed as
   an electron (charge -1, mass 1) with the run's gather and pusher, in FP64.  Frozen and
   active particles deposit their current unless test_only (the beam of the paper's scaled
   10 GeV stages is made of test particles); a frozen particle deposits only for steps that start inside the
   interior, and one that is activated outside it, or an active one that leaves it, is lost.
   No field solve sets the initial self-field of a depositing beam. */
typedef struct {
    double beta_b;             /* mean lab velocity of the beam (c = 1), 0 < beta_b < 1         */
    double z_inj_um;           /* lab position of the injection plane                          */
    int32_t test_only;         /* 1: test particles, no current                                */
    int32_t reserved;
} bf_beam;

/* Loads a beam (replacing any previous one) from host arrays of n particles: x in um
   relative to the interior origin, z the lab position (um), ux, uy, uz the lab momenta
   gamma v / c (uz > 0), w the weights in the library's normalised units.  The history
   restarts.  Synchronous.  BF_EINVAL: n above beam_capacity, beta_b outside (0, 1), uz <= 0 or a
   non-finite value; BF_EUNSUPPORTED: a 3D run. */
bf_status bf_add_beam(bf_sim* sim, const bf_beam* beam, int64_t n, const double* x, const double* z,
                      const double* ux, const double* uy, const double* uz, const double* w);

/* ---- stepping -------------------------------------------------------------------------- */

/* Advances nsteps PIC steps (Faraday+Friedman+PML, stations, gather/push/deposit, antenna,
   filter, Ampere+PML, window and injection, periodic tile sort).  Asynchronous. */
bf_status bf_step(bf_sim* sim, int nsteps);

/* ---- diagnostics and state ------------------------------------------------------------- */

enum {
    BF_DIAG_FIELD = 0,     /* arg = field id (BF_F_*): stored_z x stored_x doubles (3D:
                              stored_z x stored_y x stored_x)                               */
    BF_DIAG_PARTICLES = 1, /* arg = species (0 e-, 1 ions): 7 arrays of n doubles (id, x, z,
                              ux, uy, uz, w), n = BF_DIAG_COUNTS value; 3D: 8 arrays (id, x,
                              y, z, ux, uy, uz, w)                                           */
    BF_DIAG_COUNTS = 2,    /* 4 int64: live electrons, live ions, slots e-, slots ions     */
    BF_DIAG_STATION = 3,   /* arg = station: int64 count then count x 7 doubles (t_lab, Ex,
                              Ey, Ez, Bx, By, Bz in the lab frame)                           */
    BF_DIAG_ENERGY = 4,    /* 3 doubles: field energy E, field energy B, kinetic energy of
                              the plasma electrons (the beam is not included)               */
    BF_DIAG_GAUSS = 5,     /* div E - F[rho] on the nodes, doubles in the field layout; 3D
                              uses the FP64 current accumulators as scratch (J_xr .. J_zr of
                              the last step are gone afterwards)                            */
    BF_DIAG_INFO = 6,      /* bf_info                                                       */
    BF_DIAG_ANTENNA = 7,   /* nx doubles (3D: nx x ny): coordinate of each moving antenna
                              particle along the polarisation, in cells (x; 3D y polarisation:
                              y; 2D y polarisation: x, which then stays at the home position) */
    BF_DIAG_TIMERS = 8,    /* BF_PHASE_COUNT x 2 doubles: accumulated ms and launches per
                              phase since the last call (phase_timers = 1); arg != 0 resets */
    BF_DIAG_PARTICLE_BLOCK = 9, /* 3D only; arg = species + 2 b: the live particles of slots
                              [b, b + 1) x BF_PARTICLE_BLOCK, as int64 n then 8 arrays of n
                              doubles (id, x, y, z, ux, uy, uz, w); a sample of a large run  */
    BF_DIAG_BEAM = 10      /* arg 0: int64 n then 8 arrays of n doubles: x, z (um, window
                              frame), ux, uy, uz (calculation frame), w, crossing time t'*
                              (um/c), state (0 frozen, 1 active, 2 lost).  arg 1: int64 count
                              then count records of 8 doubles, one per step, over the active
                              particles after the push, back-transformed to the lab frame:
                              t'_{n+1}, count, sum w, sum w z_lab, sum w t_lab, sum w gamma_lab,
                              sum w u_z,lab, sum w u_z,lab^2 (z_lab = gamma (z' + beta t'),
                              gamma_lab = gamma (gamma' + beta u'_z), the momentum taken at
                              t_{n+1/2})                                                      */
};
#define BF_PARTICLE_BLOCK 65536

/* phases of one bf_step (BF_DIAG_TIMERS rows) */
enum {
    BF_PHASE_FARADAY = 0,  /* Faraday + Friedman + PML, stations, clearing the current      */
    BF_PHASE_PUSH,         /* electrons: gather, push, deposit                              */
    BF_PHASE_IONS,         /* rigid-ion current                                             */
    BF_PHASE_ANTENNA,      /* laser antenna current                                         */
    BF_PHASE_FILTER,       /* current filter                                                */
    BF_PHASE_AMPERE,       /* Ampere + PML                                                  */
    BF_PHASE_WINDOW,       /* window shift and plasma injection                             */
    BF_PHASE_SORT,         /* tile sort                                                     */
    BF_PHASE_BEAM,         /* beam through the injection plane                              */
    BF_PHASE_COUNT
};

/* field ids (logical layout [stored_z][stored_x], x fastest).  J_x, J_y, J_z are the current
   Ampere used (filtered when a filter is on); J_xr, J_yr, J_zr the raw deposited current of
   the last step, before the filter.  B_yx, E_yx are the 2D PML split parts; in 3D every
   component has one, E_xs .. B_zs (the part along the axis cyclically next to the
   component). */
enum {
    BF_F_EX = 0, BF_F_EY, BF_F_EZ, BF_F_BX, BF_F_BY, BF_F_BZ, BF_F_JX, BF_F_JY, BF_F_JZ,
    BF_F_EXO, BF_F_EYO, BF_F_EZO, BF_F_EXB, BF_F_EYB, BF_F_EZB, BF_F_BYX, BF_F_EYX,
    BF_F_BXO, BF_F_BYO, BF_F_BZO, BF_F_JXR, BF_F_JYR, BF_F_JZR,
    BF_F_EXS, BF_F_EYS, BF_F_EZS, BF_F_BXS, BF_F_BYS, BF_F_BZS, BF_F_COUNT
};

typedef struct {
    double dt, dt_crit, beta, gamma, v_window, n0_norm, e0_norm, omega, alpha2, beta2;
    double antenna_weight;
    int32_t stored_x, stored_z, pml_x, pml_z;
    int64_t step;
    double time;
    int64_t shift, next_row;
    int32_t tile_x, tile_z, ntiles, sort_every;
    int32_t dim, stored_y, pml_y, reserved;   /* 3D: stored y extent and its PML depth      */
} bf_info;

/* Synchronises; copies the requested diagnostic (FP64, host order described above) into
   host_out of `bytes` bytes (BF_EINVAL if too small).  Allowed after a sticky error. */
bf_status bf_diagnose(bf_sim* sim, int kind, int arg, void* host_out, size_t bytes);

/* Overwrites one field array (logical layout, doubles) on the device.  Synchronous. */
bf_status bf_set_field(bf_sim* sim, int field, const double* host_in, size_t bytes);

/* Synchronises and returns the sticky device status (BF_OK, BF_ECAPACITY, BF_ENONFINITE). */
bf_status bf_sync_status(bf_sim* sim);

/* Scalar state for checkpointing (device buffers are the caller's to copy). */
bf_status bf_get_state(const bf_sim* sim, bf_state* out);
bf_status bf_set_state(bf_sim* sim, const bf_state* in);

const char* bf_status_string(bf_status s);
const char* bf_last_error(const bf_sim* sim);

/* Frees host metadata only; the caller frees its buffers afterwards. */
void bf_destroy(bf_sim* sim);

/* ---- batched independent runs -----------------------------------------------------------
   Several handles stepped together, e.g. a scan over boost factor, density, grid and time step
   (each run follows Sec. 2-4 on its own).  Faraday, the electron push and Ampere are each one
   persistent launch over a device queue of (run, work item) pairs; the other phases (stations,
   rigid ions, antenna, current filter, window shift, injection, sort) are each run's own
   launches, in phase order, spread over the batch stream and three side streams the batch
   owns (run r on stream r % 4, joined back before each persistent launch).  Results equal each
   run's
   bf_step up to the order of floating-point atomic additions.  Runs must be FP32 handles on
   the current device without a sticky error; phase timers are not recorded in batched steps. */
typedef struct bf_batch bf_batch;

/* Bytes of the device work buffer (descriptor tables) for n runs; -1 for n < 1 or > 4096. */
int64_t bf_batch_work_bytes(int nsims);

/* Creates a batch over n distinct handles (not owned).  work: device buffer of at least
   bf_batch_work_bytes(n) bytes, 256-byte aligned, owned by the caller.  hip_stream: the stream
   of the batched launches (NULL: default).  BF_EINVAL: bad arguments or a repeated handle;
   BF_EUNSUPPORTED: an FP64 or 3D handle, or one with the momentum-conserving gather, Vay's
   pusher or a beam capacity; BF_ESTATE: a handle with a sticky error;
   BF_EDEVICE: pinned staging memory, the side streams or their events could not be created. */
bf_status bf_batch_create(bf_sim* const* sims, int n, void* work, int64_t work_bytes,
                          void* hip_stream, bf_batch** out);

/* nsteps steps of every run, asynchronous on the batch stream, ordered after the work queued
   on each run's own stream and before later work there.  BF_ESTATE: a run has a sticky error
   or lacks its learned-filter parameters. */
bf_status bf_batch_step(bf_batch* batch, int nsteps);

/* Frees the batch's host resources and side streams (not the runs, not the work buffer). */
void bf_batch_destroy(bf_batch* batch);

/* ---- learned current filter ---------------------------------------------------------------
   An addition that replaces the n-pass bilinear + compensation filter of Sec. 4.1 (Eq.
   3ptfilter) when filter_kind is BF_FILTER_LEARNED; the bilinear filter stays the default and
   the reference it is judged against.  Three 5x5 convolutions, channels 1 -> 16 -> 16 -> 1,
   identity activations, no bias, one network shared by J_x, J_y, J_z, each on its own
   staggered domain with the bilinear filter's boundary rule per layer (wrap on periodic
   axes, zero outside otherwise).  It is linear and shift-invariant, so it keeps Gauss's law
   (Sec. 4.2.2) as the bilinear filter does.  Arithmetic: BF16 weights, every layer input split
   into BF16 hi + lo parts, FP32 accumulation on the matrix cores.
   Parameters (FP32, BF_LF_PARAMS values): W1[t][co] (25 x 16), then W2[t][ci][co]
   (25 x 16 x 16), then W3[t][ci] (25 x 16); tap t = 5 (dy + 2) + (dx + 2) with dy along the
   rows (z) and dx along x, and layer output(p) = sum_t W[t] . input(p + (dx, dy)). */
#define BF_FILTER_BILINEAR 0
#define BF_FILTER_LEARNED 1
#define BF_LF_PARAMS 7200

/* Loads the learned filter's parameters (host array of n = BF_LF_PARAMS floats) into the
   handle; required before bf_step when filter_kind is BF_FILTER_LEARNED.  Synchronous.
   BF_EINVAL: wrong n or null; BF_ESTATE: the handle was created with the bilinear filter. */
bf_status bf_set_learned_filter(bf_sim* sim, const float* host_params, int64_t n);

/* Standalone use on batches of device images (row-major [img][y][x], FP32, one channel):
   bytes of the device work buffer that bf_lf_apply / bf_lf_train_step need for nimg images of
   ny x nx, or -1 for invalid sizes (nimg < 1 or > 65535, ny or nx < 1, too many pixels). */
int64_t bf_lf_work_bytes(int nimg, int ny, int nx);

/* out = filter(in) per image; params, in, out and work are device pointers; periodic_x/y
   select wrap instead of zero padding.  Asynchronous on hip_stream (NULL: default stream).
   BF_EINVAL: null pointer, bad sizes or work_bytes below bf_lf_work_bytes. */
bf_status bf_lf_apply(void* work, int64_t work_bytes, const float* params, const float* in,
                      float* out, int nimg, int ny, int nx, int periodic_x, int periodic_y,
                      void* hip_stream);

/* One training step on device images: loss = mean over the pixels at least `margin` from the
   image edges of (filter(in) - target)^2; gradient by backpropagation through the three
   convolutions (the BF16 weights as used in the forward pass); then, if lr != 0, one Adam
   step (Kingma & Ba 2015, bias-corrected with step number `step` >= 1) on params using the
   device moment arrays adam_m and adam_v (BF_LF_PARAMS floats each, start at zero).
   grad_out (BF_LF_PARAMS floats) and loss_out (one double) are optional device outputs that
   receive the gradient and the loss before the update.  Asynchronous on hip_stream.
   BF_EINVAL: null pointer, bad sizes, 2 margin >= ny or nx, missing moments with lr != 0. */
bf_status bf_lf_train_step(void* work, int64_t work_bytes, float* params, float* adam_m,
                           float* adam_v, const float* in, const float* target, int nimg, int ny,
                           int nx, int margin, int periodic_x, int periodic_y, float lr,
                           float beta1, float beta2, float eps, int64_t step, float* grad_out,
                           double* loss_out, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
   loops, harnesses that forbid it): bf_lf_apply without a work buffer.  Same arguments and
   results as bf_lf_apply; the packed BF16 weights go to a 64 KiB device array inside the
   library (one per device, held until the process ends, its address looked up once per
   device on the first call made with that device current).  Allocates nothing.  All calls on
   one device share that array: calls that overlap on one device (other streams or host
   threads) race.  BF_EINVAL: null pointer or bad sizes (as bf_lf_apply; the scratch need does
   not grow with the images); BF_EDEVICE: the array's address could not be obtained. */
bf_status bf_lf_apply_noalloc(const float* params, const float* in, float* out, int nimg, int ny, int nx,
                              int periodic_x, int periodic_y, void* hip_stream);

/* Host-side: the learned-filter parameters (n = BF_LF_PARAMS floats into host_params) that
   reproduce the n-pass bilinear filter with or without the compensation pass alpha_c = n/2 + 1
   of Sec. 4.1 (Eq. 3ptfilter) exactly: along each axis the composed stencil is cut into three
   factors of at most five taps, one per layer, each layer carrying the outer product of its
   factor with itself in channel 0.  BF_EINVAL: null pointer, wrong n, npass < 0, or more passes
   than three 5-tap layers hold (npass <= 6 without compensation, <= 5 with it). */
bf_status bf_lf_bilinear_params(int npass, int compensate, float* host_params, int64_t n);

#ifdef __cplusplus
}
#endif
#endif
