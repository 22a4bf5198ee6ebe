/*
 * pic_oracle3.c -- plain FP64 reference of the boosted-frame laser-wakefield PIC step in 3D.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes, links or calls this
 * file; only the tests, the smoke check and the CPU-baseline leg of the benchmark load it.  It
 * shares no source with the HIP path.
 *
 * The method is the one of pic_oracle.c, in three dimensions, each routine following the
 * paper (arXiv:1009.2727) in its own order and notation:
 *   - Faraday with the Cole-Karkkainen operator Delta* and Friedman damping (Sec. 4.2 Eqs.
 *     Faraday/Ampere and the Delta*, S^1, S^2 operators; Sec. 4.3 Eq. Faraday_Friedman),
 *     Ampere with plain Yee differences;
 *   - cubic B-spline gather from the staggered Yee locations (Sec. 5.1) and Esirkepov's
 *     charge-conserving deposit in 3D (Sec. 4.2.2);
 *   - n-pass bilinear filter plus compensation along each axis (Sec. 4.1 Eq. 3ptfilter);
 *   - split-field PML with xi = exp(-sigma dt) (Appendix II Eq. PML_stencil);
 *   - laser emitted by particle sheets on a lab-fixed plane (Sec. 3.1.2);
 *   - moving window at the boosted wake velocity (Sec. 2);
 *   - lab-frame stations with Lorentz back-transformation (Sec. 3.2).
 * Readings added for 3D (the 2-1/2D ones carry over unchanged):
 *   - Delta*_a = (alpha + beta S^1_a + gamma S^2_a) Delta_a with S^1_a the sum of the four
 *     one-cell shifts along the two axes transverse to a and S^2_a the sum of the four
 *     diagonal shifts (full-cell shifts, as in 2D); a shift leaving a non-periodic axis adds 0;
 *   - PML: every component is split into its two curl terms, each damped by the conductivity
 *     of its derivative's axis; the stored part is the one along the axis cyclically next to
 *     the component (x: y part, y: z part, z: x part), and it carries the current source; the
 *     split part is dropped wherever neither of its axes has a conductivity once the window
 *     has moved;
 *   - plasma: ppc particles per cell of each injected plane (lab-fixed lattice, as in 2D),
 *     the in-cell offsets drawn with counter slots 3 id + 1, 3 id + 2, 3 id + 3;
 *   - antenna: one +/- particle pair per transverse cell, polarisation along x, Gaussian in
 *     x and y around the axis.
 *
 * Parity unpinned: as in 2D (energy-conserving gather beyond exact uniform and linear
 * fields, quantitative PML reflection, the nonlinear wake), the 3D PML split convention and
 * the small static field the split layer can keep inside itself (it does not hold div E = 0
 * there; only the outflow from the interior is pinned).
 *
 * Units: L0 = 1 um, c = 1, eps0 = 1, electron charge -1 and mass 1.
 */
#include "pic_oracle3.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846

static const double C_LIGHT = 299792458.0;
static const double EPS0 = 8.8541878128e-12;
static const double M_E = 9.1093837015e-31;
static const double Q_E = 1.602176634e-19;

typedef struct {
    int N, P, periodic, S;
    double d;
} ax3_t;

typedef struct {
    double z_lab;
    long n, cap;
    double* rec;
} st3_t;

struct orc3_sim {
    orc3_config cfg;
    ax3_t a[3];
    double dt, dt_crit, beta, gamma, vw, theta;
    double n0, omega, e0, lambda;
    int have_plasma, have_laser;
    orc_plasma plasma;
    orc_laser laser;
    double* f[O3_NFIELD];
    long ncell;
    long step, shift, next_row;
    double t;
    long ne, cape;
    uint32_t* eid;
    double *ex, *ey, *ez, *eux, *euy, *euz, *ew;
    long ni, capi;
    uint32_t* iid;
    double *ix, *iy, *iz0, *iw;
    long na;
    double *ah_x, *ah_y, *am;           /* home x, y; moving particle's coordinate along pol */
    double aw, az_lab, sig_t, t0, w0;
    int pol;
    int nst;
    st3_t st[16];
};

/* Yee staggers (x, y, z) of the E (and J) and B components */
static const int STAG_E[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
static const int STAG_B[3][3] = {{0, 1, 1}, {1, 0, 1}, {1, 1, 0}};

static double u01(uint64_t seed, uint64_t k)
{
    return (double)(orc_splitmix64(seed, k) >> 11) * (1.0 / 9007199254740992.0);
}

static void axis_init(ax3_t* a, int N, int P, int periodic, double d)
{
    a->N = N; a->periodic = periodic; a->d = d;
    a->P = periodic ? 0 : P;
    a->S = periodic ? N : N + 2 * a->P + 1;
}

static long sidx(const ax3_t* a, long j)
{
    if (a->periodic) { long m = j % a->N; return m < 0 ? m + a->N : m; }
    long i = j + a->P;
    return (i < 0 || i >= a->S) ? -1 : i;
}

static long snb(const ax3_t* a, long i, long o)
{
    long j = i + o;
    if (a->periodic) { j %= a->N; if (j < 0) j += a->N; return j; }
    return (j < 0 || j >= a->S) ? -1 : j;
}

static double spos(const ax3_t* a, long i, int h) { return (double)(i - a->P) + 0.5 * h; }

static double sigma_at(const ax3_t* a, double p)
{
    if (a->periodic || a->P == 0) return 0.0;
    double d = 0.0;
    if (p < 0.0) d = -p; else if (p > (double)a->N) d = p - (double)a->N;
    if (d <= 0.0) return 0.0;
    double sm = 4.0 / a->d;
    return sm * (d / 5.0) * (d / 5.0);
}

static void pml_coef(double sig, double dt, double* xi, double* c)
{
    if (sig == 0.0) { *xi = 1.0; *c = dt; return; }
    *xi = exp(-sig * dt);
    *c = (1.0 - *xi) / sig;
}

/* Modified coefficients (Appendix II, sigma*; reading as in the 2D oracle): the curl
   coefficient of the value at half-grid position p along the layer's axis is dt kappa(p), with
   kappa(p + 1/2) kappa(p) = xi(p) walking outwards from the inner edge (kappa = 1 inside), which
   lets a normally incident wave with c dt = d cross every half cell without reflection. */
static double kappa3_at(const ax3_t* a, double p, double dt)
{
    if (sigma_at(a, p) == 0.0) return 1.0;
    double k = 1.0;
    if (p > (double)a->N) {
        for (double q = (double)a->N; q < p; q += 0.5) k = exp(-sigma_at(a, q) * dt) / k;
    } else {
        for (double q = 0.0; q > p; q -= 0.5) k = exp(-sigma_at(a, q) * dt) / k;
    }
    return k;
}

static inline long ID3(const orc3_sim* s, long i, long j, long k)
{
    return (k * s->a[1].S + j) * s->a[0].S + i;
}

static inline long IDq(const orc3_sim* s, const long q[3]) { return ID3(s, q[0], q[1], q[2]); }

/* ------------------------------------------------------------------ */
/* creation                                                            */
/* ------------------------------------------------------------------ */

static void update_window_speed(orc3_sim* s)
{
    if (!s->cfg.moving_window) { s->vw = 0.0; return; }
    double bw = 1.0;
    if (s->have_laser) {
        double wp2 = s->have_plasma ? s->n0 : 0.0;
        bw = 1.0 / sqrt(1.0 + wp2 / (s->omega * s->omega));
    }
    s->vw = (bw - s->beta) / (1.0 - bw * s->beta);
}

orc3_sim* orc3_create(const orc3_config* cfg)
{
    if (!cfg || cfg->nx <= 0 || cfg->ny <= 0 || cfg->nz <= 0) return NULL;
    if (cfg->dx_um <= 0 || cfg->dy_um <= 0 || cfg->dz_um <= 0) return NULL;
    if (cfg->gamma_boost < 1.0 || cfg->theta < 0 || cfg->theta > 1) return NULL;
    orc3_sim* s = (orc3_sim*)calloc(1, sizeof(orc3_sim));
    s->cfg = *cfg;
    axis_init(&s->a[0], cfg->nx, cfg->pml_cells, cfg->periodic_x, cfg->dx_um);
    axis_init(&s->a[1], cfg->ny, cfg->pml_cells, cfg->periodic_y, cfg->dy_um);
    axis_init(&s->a[2], cfg->nz, cfg->pml_cells, cfg->periodic_z, cfg->dz_um);
    s->theta = cfg->theta;
    s->dt_crit = orc_cfl_3d(cfg->ck_alpha, cfg->ck_beta, cfg->ck_gamma, cfg->dx_um, cfg->dy_um,
                            cfg->dz_um, cfg->theta);
    s->dt = cfg->cfl_fraction * s->dt_crit;
    s->gamma = cfg->gamma_boost;
    s->beta = sqrt(1.0 - 1.0 / (s->gamma * s->gamma));
    s->ncell = (long)s->a[0].S * s->a[1].S * s->a[2].S;
    for (int c = 0; c < O3_NFIELD; c++) s->f[c] = (double*)calloc((size_t)s->ncell, sizeof(double));
    update_window_speed(s);
    return s;
}

void orc3_destroy(orc3_sim* s)
{
    if (!s) return;
    for (int c = 0; c < O3_NFIELD; c++) free(s->f[c]);
    free(s->eid); free(s->ex); free(s->ey); free(s->ez); free(s->eux); free(s->euy); free(s->euz);
    free(s->ew);
    free(s->iid); free(s->ix); free(s->iy); free(s->iz0); free(s->iw);
    free(s->ah_x); free(s->ah_y); free(s->am);
    for (int i = 0; i < s->nst; i++) free(s->st[i].rec);
    free(s);
}

static void grow_e(orc3_sim* s, long need)
{
    if (need <= s->cape) return;
    long cap = s->cape ? s->cape : 1024;
    while (cap < need) cap *= 2;
    s->eid = (uint32_t*)realloc(s->eid, cap * sizeof(uint32_t));
    double** arr[7] = {&s->ex, &s->ey, &s->ez, &s->eux, &s->euy, &s->euz, &s->ew};
    for (int m = 0; m < 7; m++) *arr[m] = (double*)realloc(*arr[m], cap * sizeof(double));
    s->cape = cap;
}

static void grow_i(orc3_sim* s, long need)
{
    if (need <= s->capi) return;
    long cap = s->capi ? s->capi : 1024;
    while (cap < need) cap *= 2;
    s->iid = (uint32_t*)realloc(s->iid, cap * sizeof(uint32_t));
    double** arr[4] = {&s->ix, &s->iy, &s->iz0, &s->iw};
    for (int m = 0; m < 4; m++) *arr[m] = (double*)realloc(*arr[m], cap * sizeof(double));
    s->capi = cap;
}

static double n_lab(const orc3_sim* s, double z_lab)
{
    const orc_plasma* p = &s->plasma;
    if (z_lab < p->start_um) return 0.0;
    if (p->ramp_um > 0.0 && z_lab < p->start_um + p->ramp_um)
        return s->n0 * (z_lab - p->start_um) / p->ramp_um;
    return s->n0;
}

/* every lattice plane whose upper edge has entered the interior is created whole at the front
   (the lab-fixed lattice drifts at -beta c in the boosted frame, Sec. 3.1.1) */
static void inject_planes(orc3_sim* s)
{
    if (!s->have_plasma) return;
    const int Nx = s->a[0].N, Ny = s->a[1].N, ppc = s->plasma.ppc;
    const double dx = s->a[0].d, dy = s->a[1].d, dz = s->a[2].d;
    for (;;) {
        long l = s->next_row;
        double upper = (double)(l + 1) - s->beta * s->t / dz - (double)s->shift;
        if (upper > (double)s->a[2].N) break;
        for (int j = 0; j < Ny; j++)
            for (int i = 0; i < Nx; i++)
                for (int k = 0; k < ppc; k++) {
                    uint64_t id = (((uint64_t)l * (uint64_t)Ny + (uint64_t)j) * (uint64_t)Nx + (uint64_t)i) *
                                  (uint64_t)ppc + (uint64_t)k;
                    double rx = u01(s->cfg.seed, 3 * id + 1);
                    double ry = u01(s->cfg.seed, 3 * id + 2);
                    double rz = u01(s->cfg.seed, 3 * id + 3);
                    double zb = ((double)l + rz) * dz;
                    double w = s->gamma * n_lab(s, s->gamma * zb) * dx * dy * dz / (double)ppc;
                    if (w == 0.0) continue;
                    double x = ((double)i + rx) * dx, y = ((double)j + ry) * dy;
                    double z = zb - s->beta * s->t - (double)s->shift * dz;
                    grow_e(s, s->ne + 1);
                    long e = s->ne++;
                    s->eid[e] = (uint32_t)id;
                    s->ex[e] = x; s->ey[e] = y; s->ez[e] = z;
                    s->eux[e] = 0.0; s->euy[e] = 0.0; s->euz[e] = -s->gamma * s->beta;
                    s->ew[e] = w;
                    if (s->plasma.ion_mode == 1) {
                        grow_i(s, s->ni + 1);
                        long q = s->ni++;
                        s->iid[q] = (uint32_t)id; s->ix[q] = x; s->iy[q] = y; s->iz0[q] = zb; s->iw[q] = w;
                    }
                }
        s->next_row++;
    }
}

int orc3_init_plasma(orc3_sim* s, const orc_plasma* p)
{
    if (!s || !p || p->ppc <= 0 || p->n0_cm3 < 0) return -1;
    s->plasma = *p;
    double nu = EPS0 * M_E * C_LIGHT * C_LIGHT / (Q_E * Q_E * 1e-12);
    s->n0 = p->n0_cm3 * 1e6 / nu;
    s->have_plasma = 1;
    s->next_row = 0;
    update_window_speed(s);
    inject_planes(s);
    return 0;
}

int orc3_init_laser(orc3_sim* s, const orc_laser* l)
{
    if (!s || !l || l->lambda_um <= 0 || l->pol < 0 || l->pol > 1 || l->t_peak_fs < 0) return -1;
    s->laser = *l;
    s->have_laser = 1;
    s->lambda = l->lambda_um;
    s->omega = 2.0 * PI / l->lambda_um;
    s->e0 = l->a0 * s->omega;
    s->w0 = l->waist_um;
    s->sig_t = l->fwhm_fs * 1e-15 * C_LIGHT * 1e6 / (2.0 * sqrt(log(2.0)));
    s->t0 = l->t_peak_fs > 0.0 ? l->t_peak_fs * 1e-15 * C_LIGHT * 1e6 : 3.0 * s->sig_t;
    s->pol = l->pol;
    s->az_lab = l->z_antenna_um;
    s->na = (long)s->a[0].N * s->a[1].N;
    free(s->ah_x); free(s->ah_y); free(s->am);
    s->ah_x = (double*)malloc(s->na * sizeof(double));
    s->ah_y = (double*)malloc(s->na * sizeof(double));
    s->am = (double*)malloc(s->na * sizeof(double));
    for (long q = 0; q < s->na; q++) {
        long i = q % s->a[0].N, j = q / s->a[0].N;
        s->ah_x[q] = ((double)i + 0.5) * s->a[0].d;
        s->ah_y[q] = ((double)j + 0.5) * s->a[1].d;
        s->am[q] = s->pol == 0 ? s->ah_x[q] : s->ah_y[q];
    }
    /* sheet current K = -2 E_perp per unit area; the moving sheet stays below 0.01 c */
    s->aw = (2.0 * s->e0 / s->gamma) * s->a[0].d * s->a[1].d / 0.01;
    update_window_speed(s);
    return 0;
}

int orc3_add_station(orc3_sim* s, double z_lab_um, int capacity)
{
    if (!s || s->nst >= 16 || capacity <= 0) return -1;
    st3_t* t = &s->st[s->nst];
    t->z_lab = z_lab_um; t->n = 0; t->cap = capacity;
    t->rec = (double*)calloc((size_t)capacity * 7, sizeof(double));
    return s->nst++;
}

void orc3_get_info(const orc3_sim* s, orc3_info* o)
{
    memset(o, 0, sizeof(*o));
    o->dt = s->dt; o->dt_crit = s->dt_crit; o->beta = s->beta; o->gamma = s->gamma;
    o->v_window = s->vw; o->n0_norm = s->n0; o->e0_norm = s->e0; o->omega = s->omega;
    o->antenna_weight = s->aw;
    o->stored_x = s->a[0].S; o->stored_y = s->a[1].S; o->stored_z = s->a[2].S;
    o->pml_x = s->a[0].P; o->pml_y = s->a[1].P; o->pml_z = s->a[2].P;
    o->step = s->step; o->time = s->t; o->shift = s->shift; o->next_row = s->next_row;
}

/* ------------------------------------------------------------------ */
/* field solver                                                        */
/* ------------------------------------------------------------------ */

/* difference of G along axis ax towards a target with stagger ht there, at stored index q:
   right neighbour q + ht, left q + ht - 1 (a neighbour beyond a non-periodic edge is 0) */
static double dG(const orc3_sim* s, const double* G, const long q[3], int ax, int ht)
{
    long p[3] = {q[0], q[1], q[2]};
    long r = snb(&s->a[ax], q[ax], ht), l = snb(&s->a[ax], q[ax], ht - 1);
    double gr = 0.0, gl = 0.0;
    if (r >= 0) { p[ax] = r; gr = G[IDq(s, p)]; }
    if (l >= 0) { p[ax] = l; gl = G[IDq(s, p)]; }
    return (gr - gl) / s->a[ax].d;
}

/* Delta*_ax: alpha at the point, beta on the four one-cell shifts along the two transverse
   axes, gamma on the four diagonal shifts */
static double dStar(const orc3_sim* s, const double* G, const long q[3], int ax, int ht)
{
    const double A = s->cfg.ck_alpha, B = s->cfg.ck_beta, Cg = s->cfg.ck_gamma;
    double v = A * dG(s, G, q, ax, ht);
    if (B == 0.0 && Cg == 0.0) return v;
    const int t1 = (ax + 1) % 3, t2 = (ax + 2) % 3;
    for (int sg = -1; sg <= 1; sg += 2) {
        long p[3] = {q[0], q[1], q[2]};
        p[t1] = snb(&s->a[t1], q[t1], sg);
        if (p[t1] >= 0) v += B * dG(s, G, p, ax, ht);
        long r[3] = {q[0], q[1], q[2]};
        r[t2] = snb(&s->a[t2], q[t2], sg);
        if (r[t2] >= 0) v += B * dG(s, G, r, ax, ht);
    }
    if (Cg != 0.0)
        for (int s1 = -1; s1 <= 1; s1 += 2)
            for (int s2 = -1; s2 <= 1; s2 += 2) {
                long p[3] = {q[0], q[1], q[2]};
                p[t1] = snb(&s->a[t1], q[t1], s1);
                p[t2] = snb(&s->a[t2], q[t2], s2);
                if (p[t1] >= 0 && p[t2] >= 0) v += Cg * dG(s, G, p, ax, ht);
            }
    return v;
}

/* update ranges: B (last half-node beyond a wall untouched), E (walls keep tangential E = 0) */
static long b_hi(const ax3_t* a, int h) { return a->periodic ? a->S - 1 : a->S - 1 - h; }
static long e_lo(const ax3_t* a, int h) { return (a->periodic || h) ? 0 : 1; }
static long e_hi(const ax3_t* a) { return a->periodic ? a->S - 1 : a->S - 2; }

/* split update of one component from its two curl terms t1 (axis a1 at position r1, the stored
   part) and t2 (axis a2 at r2) */
static void split_update(const orc3_sim* s, double* F, double* Sp, const double* Fold, long q, double t1,
                         double t2, int a1, double r1, int a2, double r2, double dt)
{
    const double s1 = sigma_at(&s->a[a1], r1), s2 = sigma_at(&s->a[a2], r2);
    if (s1 == 0.0 && s2 == 0.0) { F[q] = Fold[q] + dt * (t1 + t2); return; }
    double xi1, c1, xi2, c2;
    pml_coef(s1, dt, &xi1, &c1);
    pml_coef(s2, dt, &xi2, &c2);
    if (s->cfg.pml_kind == 1) {
        if (s1 != 0.0) c1 = dt * kappa3_at(&s->a[a1], r1, dt);
        if (s2 != 0.0) c2 = dt * kappa3_at(&s->a[a2], r2, dt);
    }
    double p1 = Sp[q], p2 = Fold[q] - Sp[q];
    p1 = xi1 * p1 + c1 * t1;
    p2 = xi2 * p2 + c2 * t2;
    Sp[q] = p1;
    F[q] = p1 + p2;
}

void orc3_stage_faraday(orc3_sim* s)
{
    const long n = s->ncell;
    const double th = s->theta, dt = s->dt;
    double* E[3] = {s->f[O3_EX], s->f[O3_EY], s->f[O3_EZ]};
    double* Eo[3] = {s->f[O3_EXO], s->f[O3_EYO], s->f[O3_EZO]};
    double* Eb[3] = {s->f[O3_EXB], s->f[O3_EYB], s->f[O3_EZB]};
    double* Et[3];
    for (int c = 0; c < 3; c++) memcpy(s->f[O3_BXO + c], s->f[O3_BX + c], n * sizeof(double));
    if (th > 0.0) {
        for (int c = 0; c < 3; c++) {
            Et[c] = (double*)malloc(n * sizeof(double));
            for (long q = 0; q < n; q++) {
                Eb[c][q] = (1.0 - 0.5 * th) * Eo[c][q] + 0.5 * th * Eb[c][q];
                Et[c][q] = (1.0 + 0.25 * th) * E[c][q] - 0.5 * Eo[c][q] + (0.5 - 0.25 * th) * Eb[c][q];
            }
        }
    } else {
        for (int c = 0; c < 3; c++) Et[c] = E[c];
    }
    /* dB_c/dt = -(Delta*_a1 E_a2 - Delta*_a2 E_a1), (c, a1, a2) cyclic */
    for (int c = 0; c < 3; c++) {
        const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
        const int* h = STAG_B[c];
        double* B = s->f[O3_BX + c];
        double* Sp = s->f[O3_BXS + c];
        long q[3];
        for (q[2] = 0; q[2] <= b_hi(&s->a[2], h[2]); q[2]++)
            for (q[1] = 0; q[1] <= b_hi(&s->a[1], h[1]); q[1]++)
                for (q[0] = 0; q[0] <= b_hi(&s->a[0], h[0]); q[0]++) {
                    double t1 = -dStar(s, Et[a2], q, a1, h[a1]);
                    double t2 = dStar(s, Et[a1], q, a2, h[a2]);
                    split_update(s, B, Sp, B, IDq(s, q), t1, t2, a1, spos(&s->a[a1], q[a1], h[a1]), a2,
                                 spos(&s->a[a2], q[a2], h[a2]), dt);
                }
    }
    if (th > 0.0) for (int c = 0; c < 3; c++) free(Et[c]);
}

void orc3_stage_ampere(orc3_sim* s)
{
    const long n = s->ncell;
    const double dt = s->dt;
    for (int c = 0; c < 3; c++) memcpy(s->f[O3_EXO + c], s->f[O3_EX + c], n * sizeof(double));
    /* dE_c/dt = Delta_a1 B_a2 - Delta_a2 B_a1 - J_c, the source in the a1 part */
    for (int c = 0; c < 3; c++) {
        const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
        const int* h = STAG_E[c];
        double* Ef = s->f[O3_EX + c];
        const double* Eold = s->f[O3_EXO + c];
        double* Sp = s->f[O3_EXS + c];
        const double* J = s->f[O3_JX + c];
        const double* Ba1 = s->f[O3_BX + a1];
        const double* Ba2 = s->f[O3_BX + a2];
        long q[3];
        for (q[2] = e_lo(&s->a[2], h[2]); q[2] <= e_hi(&s->a[2]); q[2]++)
            for (q[1] = e_lo(&s->a[1], h[1]); q[1] <= e_hi(&s->a[1]); q[1]++)
                for (q[0] = e_lo(&s->a[0], h[0]); q[0] <= e_hi(&s->a[0]); q[0]++) {
                    long id = IDq(s, q);
                    double t1 = dG(s, Ba2, q, a1, h[a1]) - J[id];
                    double t2 = -dG(s, Ba1, q, a2, h[a2]);
                    split_update(s, Ef, Sp, Eold, id, t1, t2, a1, spos(&s->a[a1], q[a1], h[a1]), a2,
                                 spos(&s->a[a2], q[a2], h[a2]), dt);
                }
    }
}

/* ------------------------------------------------------------------ */
/* gather / push / deposit                                             */
/* ------------------------------------------------------------------ */

/* field at r (cells) from a component with staggers h, cubic weights on 4 nodes per axis */
static double gather3(const orc3_sim* s, const double* F, const int h[3], const double r[3])
{
    double w[3][4];
    long id[3][4];
    for (int d = 0; d < 3; d++) {
        double xs = r[d] - 0.5 * h[d];
        long j0 = (long)floor(xs);
        for (int m = 0; m < 4; m++) {
            long node = j0 - 1 + m;
            w[d][m] = orc_shape3(xs - (double)node);
            id[d][m] = sidx(&s->a[d], node);
        }
    }
    double sum = 0.0;
    for (int c = 0; c < 4; c++) {
        if (id[2][c] < 0) continue;
        for (int b = 0; b < 4; b++) {
            if (id[1][b] < 0) continue;
            for (int a = 0; a < 4; a++) {
                if (id[0][a] < 0) continue;
                sum += w[0][a] * w[1][b] * w[2][c] * F[ID3(s, id[0][a], id[1][b], id[2][c])];
            }
        }
    }
    return sum;
}

static void add3(orc3_sim* s, double* F, const long j[3], double v)
{
    long i = sidx(&s->a[0], j[0]), k = sidx(&s->a[1], j[1]), l = sidx(&s->a[2], j[2]);
    if (i < 0 || k < 0 || l < 0) return;
    F[ID3(s, i, k, l)] += v;
}

/* Esirkepov (2001) in 3D: with S0, S1 the shape factors at the old and new positions and
   DS = S1 - S0 on a 7-node window per axis,
     W_c = DS_c (S0_a1 S0_a2 + DS_a1 S0_a2 / 2 + S0_a1 DS_a2 / 2 + DS_a1 DS_a2 / 3),
     J_c(node + 1/2) - J_c(node - 1/2) = -q w W_c / (d_a1 d_a2 dt)    ((c, a1, a2) cyclic) */
static void deposit_into3(orc3_sim* s, double* const Jc[3], double q, double w, const double r0[3],
                          const double r1[3]);

void orc3_deposit_one(orc3_sim* s, double q, double w, const double r0[3], const double r1[3])
{
    double* const J[3] = {s->f[O3_JX], s->f[O3_JY], s->f[O3_JZ]};
    deposit_into3(s, J, q, w, r0, r1);
}

/* the same into the given current arrays (each thread of the particle stage has its own) */
static void deposit_into3(orc3_sim* s, double* const Jc[3], double q, double w, const double r0[3],
                          const double r1[3])
{
    double S0[3][7], DS[3][7];
    long base[3];
    for (int d = 0; d < 3; d++) {
        double a0 = r0[d] / s->a[d].d, a1 = r1[d] / s->a[d].d;
        base[d] = (long)floor(a0) - 3;
        for (int m = 0; m < 7; m++) {
            S0[d][m] = orc_shape3(a0 - (double)(base[d] + m));
            DS[d][m] = orc_shape3(a1 - (double)(base[d] + m)) - S0[d][m];
        }
    }
    for (int c = 0; c < 3; c++) {
        const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
        const double k = -q * w / (s->a[a1].d * s->a[a2].d * s->dt);
        double* J = Jc[c];
        for (int m1 = 0; m1 < 7; m1++)
            for (int m2 = 0; m2 < 7; m2++) {
                double T = S0[a1][m1] * S0[a2][m2] + 0.5 * DS[a1][m1] * S0[a2][m2] +
                           0.5 * S0[a1][m1] * DS[a2][m2] + DS[a1][m1] * DS[a2][m2] / 3.0;
                if (T == 0.0) continue;
                double acc = 0.0;
                for (int mc = 0; mc < 7; mc++) {
                    acc += k * DS[c][mc] * T;
                    if (acc == 0.0) continue;
                    long j[3];
                    j[c] = base[c] + mc;
                    j[a1] = base[a1] + m1;
                    j[a2] = base[a2] + m2;
                    add3(s, J, j, acc);
                }
            }
    }
}

static double antenna_z(const orc3_sim* s, double t)
{
    return s->az_lab / s->gamma - s->beta * t - (double)s->shift * s->a[2].d;
}

/* field emitted at the plane: E0/gamma f sin(omega t'/gamma) (Sec. 3.1.2), Gaussian in x, y */
static double antenna_field(const orc3_sim* s, double x, double y, double t)
{
    double xc = 0.5 * s->a[0].N * s->a[0].d, yc = 0.5 * s->a[1].N * s->a[1].d;
    double tau = t / s->gamma - s->t0;
    double r2 = (x - xc) * (x - xc) + (y - yc) * (y - yc);
    double f = exp(-r2 / (s->w0 * s->w0)) * exp(-tau * tau / (2.0 * s->sig_t * s->sig_t));
    return (s->e0 / s->gamma) * f * sin(s->omega * tau);
}

static const int NODE3[3] = {0, 0, 0};

/* Momentum-conserving gather, first step (Sec. 5.3): each component of E^n and B^n interpolated
   to the nodes, the mean of its values at the Yee locations around the node along its
   staggered axes (2 for E, 4 for B); values beyond the stored range read 0. */
static void node_fields3(orc3_sim* s, double* G[6])
{
    for (int c = 0; c < 6; c++) {
        const int* h = c < 3 ? STAG_E[c] : STAG_B[c - 3];
        const double* F = c < 3 ? s->f[O3_EX + c] : s->f[O3_BX + c - 3];
        const double* Fo = c < 3 ? NULL : s->f[O3_BXO + c - 3];
        long q[3];
        for (q[2] = 0; q[2] < s->a[2].S; q[2]++)
            for (q[1] = 0; q[1] < s->a[1].S; q[1]++)
                for (q[0] = 0; q[0] < s->a[0].S; q[0]++) {
                    double sum = 0.0;
                    int n = 0;
                    for (int m = 0; m < 8; m++) {
                        long p[3];
                        int skip = 0, ok = 1;
                        for (int d = 0; d < 3; d++) {
                            int lower = (m >> d) & 1;
                            if (lower && !h[d]) { skip = 1; break; }
                            p[d] = lower ? snb(&s->a[d], q[d], -1) : q[d];
                            if (p[d] < 0) ok = 0;
                        }
                        if (skip) continue;
                        n++;
                        if (!ok) continue;
                        double v = F[IDq(s, p)];
                        if (Fo) v = 0.5 * (v + Fo[IDq(s, p)]);
                        sum += v;
                    }
                    G[c][IDq(s, q)] = sum / (double)n;
                }
    }
}

/* E^n, B^n at rc (cells): from the staggered locations, or from the node values G */
static void gather_fields3(const orc3_sim* s, double* const G[6], const double rc[3], double E[3], double B[3])
{
    for (int c = 0; c < 3; c++) {
        if (G) {
            E[c] = gather3(s, G[c], NODE3, rc);
            B[c] = gather3(s, G[3 + c], NODE3, rc);
        } else {
            E[c] = gather3(s, s->f[O3_EX + c], STAG_E[c], rc);
            B[c] = 0.5 * (gather3(s, s->f[O3_BXO + c], STAG_B[c], rc) + gather3(s, s->f[O3_BX + c], STAG_B[c], rc));
        }
    }
}

void orc3_gather_at(const orc3_sim* s_, const double r[3], double out[6])
{
    /* the gather of the particle stage at one position (um, interior-relative) */
    orc3_sim* s = (orc3_sim*)s_;
    double rc[3] = {r[0] / s->a[0].d, r[1] / s->a[1].d, r[2] / s->a[2].d};
    double* G[6] = {NULL};
    int mc = s->cfg.gather_kind == 1;
    if (mc) {
        for (int c = 0; c < 6; c++) G[c] = (double*)malloc(s->ncell * sizeof(double));
        node_fields3(s, G);
    }
    gather_fields3(s, mc ? G : NULL, rc, out, out + 3);
    if (mc) for (int c = 0; c < 6; c++) free(G[c]);
}

void orc3_stage_particles(orc3_sim* s)
{
    const double dt = s->dt;
    double L[3];
    for (int d = 0; d < 3; d++) L[d] = s->a[d].N * s->a[d].d;
    for (int c = 0; c < 3; c++) memset(s->f[O3_JX + c], 0, s->ncell * sizeof(double));

    /* electrons, then rigid ions, split over the threads: each thread deposits into current
       arrays of its own, added to J in thread order afterwards; new states are stored first
       and compacted in particle order */
    const int nt = orc_threads();
    const size_t nc = (size_t)s->ncell;
    double* priv = (double*)calloc((size_t)nt * 3 * nc, sizeof(double));
    double* nst = (double*)malloc((size_t)(s->ne > 0 ? s->ne : 1) * 6 * sizeof(double));
    const int mc = s->cfg.gather_kind == 1;
    double* G[6] = {NULL};
    if (mc) {
        for (int c = 0; c < 6; c++) G[c] = (double*)malloc(nc * sizeof(double));
        node_fields3(s, G);
    }
#pragma omp parallel for schedule(static) num_threads(nt)
    for (long p = 0; p < s->ne; p++) {
        int th = 0;
#ifdef _OPENMP
        th = omp_get_thread_num();
#endif
        double* const Jt[3] = {priv + (size_t)th * 3 * nc, priv + ((size_t)th * 3 + 1) * nc,
                               priv + ((size_t)th * 3 + 2) * nc};
        double r0[3] = {s->ex[p], s->ey[p], s->ez[p]};
        double rc[3] = {r0[0] / s->a[0].d, r0[1] / s->a[1].d, r0[2] / s->a[2].d};
        double E[3], B[3];
        gather_fields3(s, mc ? G : NULL, rc, E, B);
        double u[3] = {s->eux[p], s->euy[p], s->euz[p]};
        if (s->cfg.pusher == 1) orc_vay(-1.0, dt, E, B, u);
        else orc_boris(-1.0, dt, E, B, u);
        double g = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        double r1[3];
        for (int d = 0; d < 3; d++) r1[d] = r0[d] + dt * u[d] / g;
        deposit_into3(s, Jt, -1.0, s->ew[p], r0, r1);
        double* o = nst + 6 * p;
        for (int d = 0; d < 3; d++) { o[d] = r1[d]; o[3 + d] = u[d]; }
    }
    long keep = 0;
    for (long p = 0; p < s->ne; p++) {
        double r1[3] = {nst[6 * p], nst[6 * p + 1], nst[6 * p + 2]};
        int out = 0;
        for (int d = 0; d < 3; d++) {
            if (s->a[d].periodic) { if (r1[d] < 0.0) r1[d] += L[d]; else if (r1[d] >= L[d]) r1[d] -= L[d]; }
            else if (r1[d] < 0.0 || r1[d] >= L[d]) out = 1;
        }
        if (out) continue;
        s->eid[keep] = s->eid[p];
        s->ex[keep] = r1[0]; s->ey[keep] = r1[1]; s->ez[keep] = r1[2];
        s->eux[keep] = nst[6 * p + 3]; s->euy[keep] = nst[6 * p + 4]; s->euz[keep] = nst[6 * p + 5];
        s->ew[keep] = s->ew[p];
        keep++;
    }
    s->ne = keep;
    free(nst);
    if (mc) for (int c = 0; c < 6; c++) free(G[c]);

    if (s->plasma.ion_mode == 1) {
        double t0 = s->t, t1 = (double)(s->step + 1) * dt;
#pragma omp parallel for schedule(static) num_threads(nt)
        for (long p = 0; p < s->ni; p++) {
            int th = 0;
#ifdef _OPENMP
            th = omp_get_thread_num();
#endif
            double* const Jt[3] = {priv + (size_t)th * 3 * nc, priv + ((size_t)th * 3 + 1) * nc,
                                   priv + ((size_t)th * 3 + 2) * nc};
            double ra[3] = {s->ix[p], s->iy[p], s->iz0[p] - s->beta * t0 - (double)s->shift * s->a[2].d};
            double rb[3] = {s->ix[p], s->iy[p], s->iz0[p] - s->beta * t1 - (double)s->shift * s->a[2].d};
            deposit_into3(s, Jt, 1.0, s->iw[p], ra, rb);
        }
        long kp = 0;
        for (long p = 0; p < s->ni; p++) {
            double zb = s->iz0[p] - s->beta * t1 - (double)s->shift * s->a[2].d;
            if (!s->a[2].periodic && (zb < 0.0 || zb >= L[2])) continue;
            s->iid[kp] = s->iid[p]; s->ix[kp] = s->ix[p]; s->iy[kp] = s->iy[p];
            s->iz0[kp] = s->iz0[p]; s->iw[kp] = s->iw[p];
            kp++;
        }
        s->ni = kp;
    }
    for (int th = 0; th < nt; th++)
        for (int c = 0; c < 3; c++) {
            const double* Jt = priv + ((size_t)th * 3 + c) * nc;
            double* J = s->f[O3_JX + c];
            for (size_t q = 0; q < nc; q++) J[q] += Jt[q];
        }
    free(priv);

    if (s->have_laser) {
        double t0 = s->t, t1 = (double)(s->step + 1) * dt;
        double za = antenna_z(s, t0), zb = antenna_z(s, t1);
        if (za >= 0.0 && za < L[2]) {
            double tm = t0 + 0.5 * dt;
            for (long q = 0; q < s->na; q++) {
                double K = -2.0 * antenna_field(s, s->ah_x[q], s->ah_y[q], tm);
                double v = K * s->a[0].d * s->a[1].d / (-1.0 * s->aw);   /* along pol */
                double ma = s->am[q], mb = ma + v * dt;
                double m0[3] = {s->ah_x[q], s->ah_y[q], za}, m1[3] = {s->ah_x[q], s->ah_y[q], zb};
                m0[s->pol] = ma;
                m1[s->pol] = mb;
                double h0[3] = {s->ah_x[q], s->ah_y[q], za}, h1[3] = {s->ah_x[q], s->ah_y[q], zb};
                orc3_deposit_one(s, -1.0, s->aw, m0, m1);
                orc3_deposit_one(s, 1.0, s->aw, h0, h1);
                s->am[q] = mb;
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* filter (Sec. 4.1)                                                   */
/* ------------------------------------------------------------------ */

/* one 3-point pass along axis ax over the stored range of a component with stagger h there;
   values beyond the range read 0 */
static void filter_pass(orc3_sim* s, double* F, int ax, int h, double alpha, int st, double* tmp)
{
    memcpy(tmp, F, s->ncell * sizeof(double));
    const long hi = b_hi(&s->a[ax], h);
    long q[3];
    for (q[2] = 0; q[2] < s->a[2].S; q[2]++)
        for (q[1] = 0; q[1] < s->a[1].S; q[1]++)
            for (q[0] = 0; q[0] < s->a[0].S; q[0]++) {
                if (q[ax] > hi) continue;
                long p[3] = {q[0], q[1], q[2]};
                long l = snb(&s->a[ax], q[ax], -st), r = snb(&s->a[ax], q[ax], st);
                double vl = 0.0, vr = 0.0;
                if (l >= 0 && l <= hi) { p[ax] = l; vl = tmp[IDq(s, p)]; }
                if (r >= 0 && r <= hi) { p[ax] = r; vr = tmp[IDq(s, p)]; }
                F[IDq(s, q)] = alpha * tmp[IDq(s, q)] + (1.0 - alpha) * 0.5 * (vl + vr);
            }
}

static void filter_array(orc3_sim* s, double* F, const int h[3])
{
    int np = s->cfg.filter_npass;
    if (np <= 0) return;
    double* tmp = (double*)malloc(s->ncell * sizeof(double));
    double ac = 0.5 * np + 1.0;
    const int mask = s->cfg.filter_strides ? s->cfg.filter_strides : 1;
    /* per axis, for each stride of the mask in ascending order: n passes + compensation of
       Eq. 3ptfilter_stride */
    for (int ax = 0; ax < 3; ax++)
        for (int st = 1; st <= 16; st++) {
            if (!(mask & (1 << (st - 1)))) continue;
            for (int p = 0; p < np; p++) filter_pass(s, F, ax, h[ax], 0.5, st, tmp);
            if (s->cfg.filter_compensate) filter_pass(s, F, ax, h[ax], ac, st, tmp);
        }
    free(tmp);
}

void orc3_stage_filter(orc3_sim* s)
{
    for (int c = 0; c < 3; c++) filter_array(s, s->f[O3_JX + c], STAG_E[c]);
}

/* ------------------------------------------------------------------ */
/* stations (Sec. 3.2)                                                 */
/* ------------------------------------------------------------------ */

static double trilin(const orc3_sim* s, const double* F, const int h[3], const double r[3])
{
    long j[3];
    double f[3];
    for (int d = 0; d < 3; d++) {
        double xs = r[d] - 0.5 * h[d];
        j[d] = (long)floor(xs);
        f[d] = xs - (double)j[d];
    }
    double v = 0.0;
    for (int c = 0; c < 2; c++)
        for (int b = 0; b < 2; b++)
            for (int a = 0; a < 2; a++) {
                long i = sidx(&s->a[0], j[0] + a), k = sidx(&s->a[1], j[1] + b), l = sidx(&s->a[2], j[2] + c);
                if (i < 0 || k < 0 || l < 0) continue;
                v += (a ? f[0] : 1.0 - f[0]) * (b ? f[1] : 1.0 - f[1]) * (c ? f[2] : 1.0 - f[2]) * F[ID3(s, i, k, l)];
            }
    return v;
}

void orc3_stage_stations(orc3_sim* s)
{
    for (int q = 0; q < s->nst; q++) {
        st3_t* st = &s->st[q];
        double zb = st->z_lab / s->gamma - s->beta * s->t;
        double zc = (zb - (double)s->shift * s->a[2].d) / s->a[2].d;
        if (zc < 0.0 || zc >= (double)s->a[2].N || st->n >= st->cap) continue;
        double r[3] = {0.5 * s->a[0].N, 0.5 * s->a[1].N, zc};
        double E[3], B[3];
        for (int c = 0; c < 3; c++) {
            E[c] = trilin(s, s->f[O3_EX + c], STAG_E[c], r);
            B[c] = 0.5 * (trilin(s, s->f[O3_BXO + c], STAG_B[c], r) + trilin(s, s->f[O3_BX + c], STAG_B[c], r));
        }
        double g = s->gamma, b = s->beta;
        double* rec = st->rec + 7 * st->n;
        rec[0] = g * (s->t + b * zb);
        rec[1] = g * (E[0] + b * B[1]);
        rec[2] = g * (E[1] - b * B[0]);
        rec[3] = E[2];
        rec[4] = g * (B[0] - b * E[1]);
        rec[5] = g * (B[1] + b * E[0]);
        rec[6] = B[2];
        st->n++;
    }
}

long orc3_station_samples(const orc3_sim* s, int q, double* out, long cap)
{
    if (q < 0 || q >= s->nst) return -1;
    long n = s->st[q].n < cap ? s->st[q].n : cap;
    if (out) memcpy(out, s->st[q].rec, n * 7 * sizeof(double));
    return s->st[q].n;
}

/* ------------------------------------------------------------------ */
/* time advance, moving window, injection                              */
/* ------------------------------------------------------------------ */

static void shift_planes(orc3_sim* s, double* F, long d)
{
    const long P = (long)s->a[0].S * s->a[1].S, Sz = s->a[2].S;
    if (d > 0) {
        for (long k = 0; k < Sz; k++) {
            if (k + d < Sz) memcpy(F + k * P, F + (k + d) * P, P * sizeof(double));
            else memset(F + k * P, 0, P * sizeof(double));
        }
    } else if (d < 0) {
        for (long k = Sz - 1; k >= 0; k--) {
            if (k + d >= 0) memcpy(F + k * P, F + (k + d) * P, P * sizeof(double));
            else memset(F + k * P, 0, P * sizeof(double));
        }
    }
}

void orc3_stage_advance(orc3_sim* s)
{
    s->step++;
    s->t = (double)s->step * s->dt;
    if (s->cfg.moving_window && !s->cfg.periodic_z) {
        double zw = s->vw * s->t;
        long sn = (long)trunc(zw / s->a[2].d);
        long d = sn - s->shift;
        if (d != 0) {
            for (int c = 0; c < O3_NFIELD; c++) shift_planes(s, s->f[c], d);
            /* split parts are meaningful only where one of their two axes has a conductivity */
            for (int c = 0; c < 6; c++) {
                const int comp = c % 3;
                const int* h = c < 3 ? STAG_E[comp] : STAG_B[comp];
                const int a1 = (comp + 1) % 3, a2 = (comp + 2) % 3;
                double* Sp = s->f[(c < 3 ? O3_EXS : O3_BXS) + comp];
                long q[3];
                for (q[2] = 0; q[2] < s->a[2].S; q[2]++)
                    for (q[1] = 0; q[1] < s->a[1].S; q[1]++)
                        for (q[0] = 0; q[0] < s->a[0].S; q[0]++)
                            if (sigma_at(&s->a[a1], spos(&s->a[a1], q[a1], h[a1])) == 0.0 &&
                                sigma_at(&s->a[a2], spos(&s->a[a2], q[a2], h[a2])) == 0.0)
                                Sp[IDq(s, q)] = 0.0;
            }
            /* tangential E stays zero on the conducting end walls */
            const long P = (long)s->a[0].S * s->a[1].S, last = s->a[2].S - 1;
            int tang[6] = {O3_EX, O3_EY, O3_EXO, O3_EYO, O3_EXB, O3_EYB};
            for (int m = 0; m < 6; m++) {
                memset(s->f[tang[m]], 0, P * sizeof(double));
                memset(s->f[tang[m]] + last * P, 0, P * sizeof(double));
            }
            for (long p = 0; p < s->ne; p++) s->ez[p] -= (double)d * s->a[2].d;
            s->shift = sn;
        }
    }
    inject_planes(s);
}

int orc3_step(orc3_sim* s, int nsteps)
{
    for (int n = 0; n < nsteps; n++) {
        orc3_stage_faraday(s);
        orc3_stage_stations(s);
        orc3_stage_particles(s);
        orc3_stage_filter(s);
        orc3_stage_ampere(s);
        orc3_stage_advance(s);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* access and diagnostics                                              */
/* ------------------------------------------------------------------ */

int orc3_get_field(const orc3_sim* s, int comp, double* out)
{
    if (comp < 0 || comp >= O3_NFIELD) return -1;
    memcpy(out, s->f[comp], s->ncell * sizeof(double));
    return 0;
}

int orc3_set_field(orc3_sim* s, int comp, const double* in)
{
    if (comp < 0 || comp >= O3_NFIELD) return -1;
    memcpy(s->f[comp], in, s->ncell * sizeof(double));
    return 0;
}

long orc3_num_particles(const orc3_sim* s, int species)
{
    return species == ORC_ELECTRONS ? s->ne : s->ni;
}

int orc3_get_particles(const orc3_sim* s, int species, uint32_t* id, double* x, double* y, double* z,
                       double* ux, double* uy, double* uz, double* w)
{
    if (species == ORC_ELECTRONS) {
        for (long p = 0; p < s->ne; p++) {
            if (id) id[p] = s->eid[p];
            if (x) x[p] = s->ex[p];
            if (y) y[p] = s->ey[p];
            if (z) z[p] = s->ez[p];
            if (ux) ux[p] = s->eux[p];
            if (uy) uy[p] = s->euy[p];
            if (uz) uz[p] = s->euz[p];
            if (w) w[p] = s->ew[p];
        }
        return 0;
    }
    for (long p = 0; p < s->ni; p++) {
        if (id) id[p] = s->iid[p];
        if (x) x[p] = s->ix[p];
        if (y) y[p] = s->iy[p];
        if (z) z[p] = s->iz0[p] - s->beta * s->t - (double)s->shift * s->a[2].d;
        if (ux) ux[p] = 0.0;
        if (uy) uy[p] = 0.0;
        if (uz) uz[p] = -s->gamma * s->beta;
        if (w) w[p] = s->iw[p];
    }
    return 0;
}

int orc3_set_electrons(orc3_sim* s, long n, const uint32_t* id, const double* x, const double* y,
                       const double* z, const double* ux, const double* uy, const double* uz,
                       const double* w)
{
    s->ne = 0;
    grow_e(s, n > 0 ? n : 1);
    for (long p = 0; p < n; p++) {
        s->eid[p] = id[p]; s->ex[p] = x[p]; s->ey[p] = y[p]; s->ez[p] = z[p];
        s->eux[p] = ux[p]; s->euy[p] = uy[p]; s->euz[p] = uz[p]; s->ew[p] = w[p];
    }
    s->ne = n;
    return 0;
}

int orc3_set_ions(orc3_sim* s, long n, const uint32_t* id, const double* x, const double* y,
                  const double* z0, const double* w)
{
    s->ni = 0;
    grow_i(s, n > 0 ? n : 1);
    for (long p = 0; p < n; p++) {
        s->iid[p] = id[p]; s->ix[p] = x[p]; s->iy[p] = y[p]; s->iz0[p] = z0[p]; s->iw[p] = w[p];
    }
    s->ni = n;
    return 0;
}

int orc3_get_antenna(const orc3_sim* s, double* xm)
{
    if (!s->have_laser) return -1;
    memcpy(xm, s->am, s->na * sizeof(double));
    return (int)s->na;
}

int orc3_set_antenna(orc3_sim* s, const double* xm)
{
    if (!s->have_laser) return -1;
    memcpy(s->am, xm, s->na * sizeof(double));
    return (int)s->na;
}

int orc3_set_clock(orc3_sim* s, long step, double time, long shift, long next_row)
{
    s->step = step; s->t = time; s->shift = shift; s->next_row = next_row;
    return 0;
}

void orc3_energy(const orc3_sim* s, double out[3])
{
    double ue = 0.0, ub = 0.0, k = 0.0, dv = s->a[0].d * s->a[1].d * s->a[2].d;
    for (long q = 0; q < s->ncell; q++)
        for (int c = 0; c < 3; c++) {
            ue += s->f[O3_EX + c][q] * s->f[O3_EX + c][q];
            ub += s->f[O3_BX + c][q] * s->f[O3_BX + c][q];
        }
    for (long p = 0; p < s->ne; p++) {
        double g = sqrt(1.0 + s->eux[p] * s->eux[p] + s->euy[p] * s->euy[p] + s->euz[p] * s->euz[p]);
        k += s->ew[p] * (g - 1.0);
    }
    out[0] = 0.5 * ue * dv; out[1] = 0.5 * ub * dv; out[2] = k;
}

static void deposit_rho(orc3_sim* s, double* rho, double q, double w, const double r[3])
{
    double S[3][4];
    long id[3][4];
    for (int d = 0; d < 3; d++) {
        double a = r[d] / s->a[d].d;
        long j0 = (long)floor(a);
        for (int m = 0; m < 4; m++) {
            S[d][m] = orc_shape3(a - (double)(j0 - 1 + m));
            id[d][m] = sidx(&s->a[d], j0 - 1 + m);
        }
    }
    const double vol = s->a[0].d * s->a[1].d * s->a[2].d;
    for (int c = 0; c < 4; c++)
        for (int b = 0; b < 4; b++)
            for (int a = 0; a < 4; a++) {
                if (id[0][a] < 0 || id[1][b] < 0 || id[2][c] < 0) continue;
                rho[ID3(s, id[0][a], id[1][b], id[2][c])] += q * w * S[0][a] * S[1][b] * S[2][c] / vol;
            }
}

int orc3_charge_density(const orc3_sim* s_, double* rho)
{
    orc3_sim* s = (orc3_sim*)s_;
    memset(rho, 0, s->ncell * sizeof(double));
    for (long p = 0; p < s->ne; p++) {
        double r[3] = {s->ex[p], s->ey[p], s->ez[p]};
        deposit_rho(s, rho, -1.0, s->ew[p], r);
    }
    if (s->plasma.ion_mode == 1)
        for (long p = 0; p < s->ni; p++) {
            double r[3] = {s->ix[p], s->iy[p], s->iz0[p] - s->beta * s->t - (double)s->shift * s->a[2].d};
            deposit_rho(s, rho, 1.0, s->iw[p], r);
        }
    if (s->have_laser) {
        double za = antenna_z(s, s->t);
        if (za >= 0.0 && za < s->a[2].N * s->a[2].d)
            for (long q = 0; q < s->na; q++) {
                double m[3] = {s->ah_x[q], s->ah_y[q], za}, h[3] = {s->ah_x[q], s->ah_y[q], za};
                m[s->pol] = s->am[q];
                deposit_rho(s, rho, -1.0, s->aw, m);
                deposit_rho(s, rho, 1.0, s->aw, h);
            }
    }
    return 0;
}

int orc3_gauss_residual(const orc3_sim* s_, double* out)
{
    orc3_sim* s = (orc3_sim*)s_;
    double* rho = (double*)malloc(s->ncell * sizeof(double));
    orc3_charge_density(s, rho);
    static const int node[3] = {0, 0, 0};
    filter_array(s, rho, node);
    long q[3];
    for (q[2] = 0; q[2] < s->a[2].S; q[2]++)
        for (q[1] = 0; q[1] < s->a[1].S; q[1]++)
            for (q[0] = 0; q[0] < s->a[0].S; q[0]++) {
                double div = 0.0;
                for (int d = 0; d < 3; d++) div += dG(s, s->f[O3_EX + d], q, d, 0);
                out[IDq(s, q)] = div - rho[IDq(s, q)];
            }
    free(rho);
    return 0;
}
