/*
 * pic_oracle.h -- FP64 CPU reference of one boosted-frame laser-wakefield PIC step
 * (2-1/2D, x-z plane), used ONLY as test infrastructure: by the tests, by the smoke
 * check and by the CPU-baseline leg of the benchmark. The product path never links it.
 *
 * It is written from the paper (Vay, Geddes, Cormier-Michel, Grote, "Modeling laser
 * wakefield accelerators in a Lorentz boosted frame", arXiv:1009.2727) as plain loops:
 * no tiles, no sorting, no ring buffers, no shared code with the HIP library.
 *
 * Normalised units throughout: length unit L0 = 1 um, c = 1, eps0 = 1, electron
 * charge -1 and mass 1.  Fields: E in m c^2/(e L0), B in m c/(e L0); density in
 * eps0 m c^2/(e^2 L0^2) (so omega_p^2 = n); momenta u = gamma v / c.
 */
#ifndef PIC_ORACLE_H
#define PIC_ORACLE_H
#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_sim orc_sim;

typedef struct {
    int nx, nz;               /* interior cells along x (transverse) and z (boost axis) */
    double dx_um, dz_um;      /* cell sizes (lab or boosted-frame metres x 1e-6)       */
    int pml_cells;            /* split-field PML depth on every non-periodic face        */
    int periodic_x, periodic_z;
    double ck_alpha, ck_beta, ck_gamma;  /* Cole-Karkkainen coefficients (3D table)      */
    double theta;             /* Friedman damping parameter, 0 <= theta <= 1             */
    double cfl_fraction;      /* dt = cfl_fraction * dt*_c                               */
    int filter_npass;         /* bilinear (alpha = 1/2) passes per axis                  */
    int filter_compensate;    /* 1: add one pass with alpha_c = n/2 + 1                  */
    double gamma_boost;       /* Lorentz factor of the calculation frame                 */
    int moving_window;        /* 1: window follows the wake at beta_w* c                 */
    uint64_t seed;
    int filter_strides;       /* bit s-1 set: the n passes (+ compensation) are applied
                                 with stride s (Eq. 3ptfilter_stride), strides ascending;
                                 0 is the same as 1 (stride 1 only)                        */
    int gather_kind;          /* 0: energy conserving, each component from its own Yee
                                 location; 1: momentum conserving, the fields interpolated
                                 to the nodes first (Sec. 5.3)                              */
    int pusher;               /* 0: Boris; 1: Vay (Phys. Plasmas 15, 056701, 2008)          */
    int pml_kind;             /* 0: c = (1 - xi)/sigma; 1: the modified coefficients (the
                                 layer matched cell by cell, Appendix II's sigma*)           */
} orc_config;

typedef struct {
    double n0_cm3;            /* lab-frame plateau density                               */
    double ramp_um;           /* lab-frame linear up-ramp length (0: step)               */
    double start_um;          /* lab-frame position where the ramp starts                */
    int ppc;                  /* macro-electrons per cell                                */
    int ion_mode;             /* 0: immobile background, 1: ions rigid in the lab frame  */
} orc_plasma;

typedef struct {
    double lambda_um, a0, waist_um, fwhm_fs;
    double z_antenna_um;      /* lab-frame position of the emitting plane                */
    double t_peak_fs;         /* lab time at which the pulse peak crosses the plane;
                                 0 selects 3 sigma_t (nothing emitted before t = 0)      */
    int pol;                  /* linear polarisation: 0 along x, 1 along y               */
} orc_laser;

/* field component ids */
enum { ORC_EX = 0, ORC_EY, ORC_EZ, ORC_BX, ORC_BY, ORC_BZ, ORC_JX, ORC_JY, ORC_JZ,
       ORC_EXO, ORC_EYO, ORC_EZO, ORC_EXB, ORC_EYB, ORC_EZB, ORC_BYX, ORC_EYX,
       ORC_BXO, ORC_BYO, ORC_BZO, ORC_NFIELD };

/* species ids */
enum { ORC_ELECTRONS = 0, ORC_IONS = 1 };

orc_sim* orc_create(const orc_config* cfg);
void     orc_destroy(orc_sim* s);
int      orc_init_plasma(orc_sim* s, const orc_plasma* p);
int      orc_init_laser(orc_sim* s, const orc_laser* l);
int      orc_add_station(orc_sim* s, double z_lab_um, int capacity);
int      orc_step(orc_sim* s, int nsteps);

/* individual stages (the step is exactly these, in this order) */
void orc_stage_faraday(orc_sim* s);
void orc_stage_stations(orc_sim* s);
void orc_stage_particles(orc_sim* s);   /* gather, push, deposit, removal */
void orc_stage_filter(orc_sim* s);
void orc_stage_ampere(orc_sim* s);
void orc_stage_advance(orc_sim* s);     /* time, window shift, plasma injection */

/* derived quantities */
typedef struct {
    double dt, dt_crit, beta, gamma, v_window, n0_norm, e0_norm, omega;
    double alpha2, beta2;      /* reduced 2D CK coefficients */
    double antenna_weight;
    int stored_x, stored_z;    /* stored array extents (x fastest) */
    int pml_x, pml_z;          /* PML depth along x and z (0 on periodic axes) */
    long step; double time; long shift; long next_row;
} orc_info;
void orc_get_info(const orc_sim* s, orc_info* out);
double orc_cfl_2d(double a, double b, double g, double dx, double dz, double theta);
double orc_cfl_3d(double a, double b, double g, double dx, double dy, double dz, double theta);

/* field access in the logical layout [stored_z][stored_x] */
int  orc_get_field(const orc_sim* s, int comp, double* out);
int  orc_set_field(orc_sim* s, int comp, const double* in);

/* particle access */
long orc_num_particles(const orc_sim* s, int species);
int  orc_get_particles(const orc_sim* s, int species, uint32_t* id, double* x, double* z,
                       double* ux, double* uy, double* uz, double* w);
/* replace the electron set (tests: arbitrary states); x,z in um relative to the interior */
int  orc_set_electrons(orc_sim* s, long n, const uint32_t* id, const double* x, const double* z,
                       const double* ux, const double* uy, const double* uz, const double* w);
int  orc_set_ions(orc_sim* s, long n, const uint32_t* id, const double* x, const double* z0,
                  const double* w);
/* antenna state: x of the moving (negative) sheet particles (they stay at their home x
   when the polarisation is along y) */
int  orc_get_antenna(const orc_sim* s, double* xminus);
int  orc_set_antenna(orc_sim* s, const double* xminus);
/* scalar state: step, time, window shift count, next lattice row */
int  orc_set_clock(orc_sim* s, long step, double time, long shift, long next_row);

/* diagnostics */
void orc_energy(const orc_sim* s, double out[3]);   /* U_E, U_B, kinetic */
/* div E - F[rho] on the nodes, logical layout [stored_z][stored_x] */
int  orc_gauss_residual(const orc_sim* s, double* out);
/* rho on nodes (unfiltered), logical layout */
int  orc_charge_density(const orc_sim* s, double* out);
long orc_station_samples(const orc_sim* s, int station, double* out /* 7 per sample */, long cap);

/* Particle beam launched through a lab-fixed plane (Sec. 3.1.1): the caller gives each
   macro-particle's lab state at t = 0; the beam is projected ballistically onto the plane,
   Lorentz transformed, synchronised to t' = 0 and kept frozen (moving along z at the
   boosted mean velocity, transverse position and momentum fixed) until it crosses the
   plane, then pushed as an ordinary electron.  Beam particles have charge -1 and mass 1. */
typedef struct {
    double beta_b;            /* mean lab velocity of the beam (c = 1), 0 < beta_b < 1      */
    double z_inj_um;          /* lab position of the injection plane                        */
    int test_only;            /* 1: the beam deposits no current (test particles)          */
} orc_beam;
/* x: um relative to the interior origin; z: lab position (um); u = gamma v lab momenta;
   w: weights in normalised units.  Replaces a previous beam.  history_cap: records kept. */
int  orc_add_beam(orc_sim* s, const orc_beam* b, long n, const double* x, const double* z,
                  const double* ux, const double* uy, const double* uz, const double* w,
                  long history_cap);
/* 8 arrays of n doubles: x, z (um, window frame), ux, uy, uz (calculation frame), w,
   crossing time t'* (um/c), state (0 frozen, 1 active, 2 lost); returns n */
long orc_beam_state(const orc_sim* s, double* out);
/* one record per step of the active particles after the push, back-transformed to the lab
   frame: t'_{n+1}, count, sum w, sum w z_lab, sum w t_lab, sum w gamma_lab, sum w u_z,lab,
   sum w u_z,lab^2; returns the number of records */
long orc_beam_history(const orc_sim* s, double* out, long cap);
/* the boosted-frame quantities of one lab particle (pins): t'*, x*, z'(0), u'x, u'y, u'z */
void orc_beam_transform(const orc_sim* s, const orc_beam* b, double x, double z, double ux,
                        double uy, double uz, double out[6]);
/* one-particle helpers for pins */
/* E^n and B^n gathered at (x, z) (um, interior-relative) exactly as the particle stage does:
   out = Ex, Ey, Ez, Bx, By, Bz */
void orc_gather_at(const orc_sim* s, double x, double z, double out[6]);
double orc_shape3(double r);
void orc_boris(double q_over_m, double dt, const double E[3], const double B[3], double u[3]);
void orc_vay(double q_over_m, double dt, const double E[3], const double B[3], double u[3]);
/* Esirkepov deposit of one particle into a zeroed J (logical layout), for pins */
void orc_deposit_one(orc_sim* s, double q, double w, double x0, double z0, double x1, double z1,
                     double vy);

/* host threads of the particle stages (default 1; the result then does not depend on it
   beyond the order of the floating-point sums of the current) */
void orc_set_threads(int n);
int  orc_threads(void);

/* SplitMix64 output number k (k >= 1) from state `seed` */
uint64_t orc_splitmix64(uint64_t seed, uint64_t k);

#ifdef __cplusplus
}
#endif
#endif
