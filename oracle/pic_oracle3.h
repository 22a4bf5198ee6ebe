/*
 * pic_oracle3.h -- FP64 CPU reference of one boosted-frame laser-wakefield PIC step in full
 * 3D (x, y transverse, z the boost axis).  TEST INFRASTRUCTURE ONLY: used by the tests, the
 * smoke check and the CPU-baseline leg of the benchmark; the product library never links it.
 *
 * Same method, readings and normalised units as the 2-1/2D reference (pic_oracle.h), written
 * out for three dimensions as plain loops: the full Cole-Karkkainen operator with its beta and
 * gamma shifts in both transverse directions, split-field PML on every component, cubic gather
 * on 4x4x4 nodes, the three-dimensional Esirkepov weights, a laser sheet with one particle pair
 * per transverse cell, plane-wise plasma injection.
 */
#ifndef PIC_ORACLE3_H
#define PIC_ORACLE3_H
#include <stdint.h>
#include <stddef.h>
#include "pic_oracle.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc3_sim orc3_sim;

typedef struct {
    int nx, ny, nz;                      /* interior cells                                   */
    double dx_um, dy_um, dz_um;
    int pml_cells;                       /* split-field PML depth on every non-periodic face */
    int periodic_x, periodic_y, periodic_z;
    double ck_alpha, ck_beta, ck_gamma;  /* Cole-Karkkainen coefficients (3D table)          */
    double theta;                        /* Friedman damping parameter                       */
    double cfl_fraction;
    int filter_npass, filter_compensate;
    double gamma_boost;
    int moving_window;
    uint64_t seed;
    int filter_strides;                  /* stride mask, as in orc_config                    */
    int gather_kind, pusher;             /* as in orc_config                                 */
    int pml_kind;                        /* as in orc_config                                 */
} orc3_config;

/* field component ids; the split arrays S hold the PML part along the cyclic-next axis of the
   component (x: y part, y: z part, z: x part) */
enum { O3_EX = 0, O3_EY, O3_EZ, O3_BX, O3_BY, O3_BZ, O3_JX, O3_JY, O3_JZ,
       O3_EXO, O3_EYO, O3_EZO, O3_EXB, O3_EYB, O3_EZB,
       O3_EXS, O3_EYS, O3_EZS, O3_BXS, O3_BYS, O3_BZS,
       O3_BXO, O3_BYO, O3_BZO, O3_NFIELD };

typedef struct {
    double dt, dt_crit, beta, gamma, v_window, n0_norm, e0_norm, omega, antenna_weight;
    int stored_x, stored_y, stored_z;    /* array extents, x fastest then y then z */
    int pml_x, pml_y, pml_z;
    long step; double time; long shift; long next_row;
} orc3_info;

orc3_sim* orc3_create(const orc3_config* cfg);
void orc3_destroy(orc3_sim* s);
int  orc3_init_plasma(orc3_sim* s, const orc_plasma* p);
int  orc3_init_laser(orc3_sim* s, const orc_laser* l);
int  orc3_add_station(orc3_sim* s, double z_lab_um, int capacity);
int  orc3_step(orc3_sim* s, int nsteps);

void orc3_stage_faraday(orc3_sim* s);
void orc3_stage_stations(orc3_sim* s);
void orc3_stage_particles(orc3_sim* s);
void orc3_stage_filter(orc3_sim* s);
void orc3_stage_ampere(orc3_sim* s);
void orc3_stage_advance(orc3_sim* s);

void orc3_get_info(const orc3_sim* s, orc3_info* out);
int  orc3_get_field(const orc3_sim* s, int comp, double* out);     /* [stored_z][stored_y][stored_x] */
int  orc3_set_field(orc3_sim* s, int comp, const double* in);

long orc3_num_particles(const orc3_sim* s, int species);
int  orc3_get_particles(const orc3_sim* s, int species, uint32_t* id, double* x, double* y, double* z,
                        double* ux, double* uy, double* uz, double* w);
int  orc3_set_electrons(orc3_sim* s, long n, const uint32_t* id, const double* x, const double* y,
                        const double* z, const double* ux, const double* uy, const double* uz,
                        const double* w);
int  orc3_set_ions(orc3_sim* s, long n, const uint32_t* id, const double* x, const double* y,
                   const double* z0, const double* w);
/* antenna state: coordinate of each moving (negative) sheet particle along the polarisation
   (x, or y for y polarisation), nx * ny values, x fastest */
int  orc3_get_antenna(const orc3_sim* s, double* xminus);
int  orc3_set_antenna(orc3_sim* s, const double* xminus);
int  orc3_set_clock(orc3_sim* s, long step, double time, long shift, long next_row);

void orc3_energy(const orc3_sim* s, double out[3]);
int  orc3_charge_density(const orc3_sim* s, double* out);
int  orc3_gauss_residual(const orc3_sim* s, double* out);
long orc3_station_samples(const orc3_sim* s, int station, double* out, long cap);

/* E^n and B^n gathered at r (um, interior-relative) as the particle stage does, for pins */
void orc3_gather_at(const orc3_sim* s, const double r[3], double out[6]);

/* Esirkepov deposit of one particle into J (um, interior-relative), for pins */
void orc3_deposit_one(orc3_sim* s, double q, double w, const double r0[3], const double r1[3]);

#ifdef __cplusplus
}
#endif
#endif
