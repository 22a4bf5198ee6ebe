// bf_host.hip -- host runtime of the C ABI declared in include/bfpic.h.
//
// Owns only host metadata: device memory comes from the caller's bindings.  One bf_step()
// enqueues, per PIC step, on the bound stream:
//   Faraday + Friedman + PML -> stations -> gather/push/deposit (electrons) -> rigid-ion
//   deposit -> antenna -> filter -> Ampere + PML -> window shift -> injection -> tile sort
// The order follows the time levels of the paper: B^{n+1/2} from E^n (Sec. 4.3, indices
// shifted by one), the push at E^n and B^n = (B^{n-1/2}+B^{n+1/2})/2, J^{n+1/2} from the
// x^n -> x^{n+1} move, E^{n+1} from B^{n+1/2} and the filtered J^{n+1/2} (Sec. 4.2).
#include <hip/hip_runtime.h>
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/bfpic.h"
#include "bf_kernels.h"
#include "bf_lfilter.h"
#include "bf_batch.h"
#include "bf_kernels3.h"

using namespace bf;

namespace {

constexpr double PI = 3.14159265358979323846;
// CODATA 2018
constexpr double C_LIGHT = 299792458.0;
constexpr double EPS0 = 8.8541878128e-12;
constexpr double ME_KG = 9.1093837015e-31;
constexpr double Q_E = 1.602176634e-19;

// field arrays inside the "fields" buffer
enum {
    A_E0 = 0,   // E set 0: 3 arrays
    A_E1 = 3,   // E set 1
    A_EB0 = 6,  // Ebar set 0
    A_EB1 = 9,  // Ebar set 1
    A_B0 = 12,  // B set 0
    A_B1 = 15,  // B set 1
    A_J = 18,   // raw J
    A_JF = 21,  // filtered J
    A_BYX = 24,
    A_EYX = 25,
    A_JT = 26,  // the filter's intermediate (after the x passes)
    A_G = 29,   // momentum-conserving gather: E^n, B^n at the nodes (6 arrays)
    A_COUNT = 35
};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// keeps the first HIP error of a sequence of calls
struct Chk {
    hipError_t e = hipSuccess;
    void operator()(hipError_t r)
    {
        if (e == hipSuccess) e = r;
    }
};

struct Layout {
    int real;            // bytes
    int Sx, Sz, pitch, Px, Pz;
    size_t field_array;  // bytes per field array
    size_t fields_bytes;
    int64_t cap;
    size_t e_off[7], e_bytes;   // x z ux uy uz w id
    size_t i_off[4], i_bytes;   // x z0 w id
    int tile_x, tile_z, ntx, ntz, ntiles, nchunks, seg_cap;
    // work buffer
    size_t w_seg[2], w_bbe[2], w_segi[2], w_bbi[2], w_counts, w_cursor, w_nused, w_status,
        w_pml_r, w_pml_on, w_st_z, w_st_rec, w_st_cnt, w_ant, w_rho, w_lf_par, w_lf_pk[3], w_beam[8],
        w_bhist, w_bytes;
    int nst, stcap;
};

bool layout_of(const bf_config* c, Layout* L)
{
    const int real = c->real_bytes;
    L->real = real;
    const int perx = c->periodic_mask & 1, perz = (c->periodic_mask >> 2) & 1;
    L->Px = perx ? 0 : c->pml_cells;
    L->Pz = perz ? 0 : c->pml_cells;
    L->Sx = perx ? c->nx : c->nx + 2 * L->Px + 1;
    L->Sz = perz ? c->nz : c->nz + 2 * L->Pz + 1;
    const int pe = 256 / real;                 // 256-byte row alignment
    L->pitch = (int)align_up((size_t)L->Sx, (size_t)pe);
    L->field_array = (size_t)L->pitch * L->Sz * real;
    L->fields_bytes = L->field_array * A_COUNT;
    L->cap = c->particle_capacity;
    size_t o = 0;
    const size_t esz[7] = {8, 8, (size_t)real, (size_t)real, (size_t)real, (size_t)real, 4};
    for (int k = 0; k < 7; k++) { L->e_off[k] = o; o = align_up(o + esz[k] * L->cap, 256); }
    L->e_bytes = std::max<size_t>(o, 256);
    o = 0;
    const size_t isz[4] = {8, 8, (size_t)real, 4};
    for (int k = 0; k < 4; k++) { L->i_off[k] = o; o = align_up(o + isz[k] * L->cap, 256); }
    L->i_bytes = std::max<size_t>(o, 256);
    // default tile 26 x 8: with the LDS tile pitch of 33 cells, the cells of a tile whose
    // row-major ranks are less than 25 apart fall in distinct 8-byte bank pairs (33 = 1 mod
    // 32), so the 16 lanes an LDS atomic serves at once, spread over the tile's cells by the
    // sort, rarely conflict; 26 + the 5-cell deposit halo leaves 2 columns of slack in the
    // 33-column LDS tile for particles drifting out between sorts
    L->tile_x = c->tile_x > 0 ? c->tile_x : 26;
    L->tile_z = c->tile_z > 0 ? c->tile_z : 8;
    L->ntx = (c->nx + L->tile_x - 1) / L->tile_x;
    L->ntz = (c->nz + L->tile_z - 1) / L->tile_z;
    L->ntiles = L->ntx * L->ntz;
    L->nchunks = L->ntx;
    L->seg_cap = L->ntiles + (c->nz + 64) * L->nchunks;
    L->nst = std::max(c->max_stations, 0);
    L->stcap = std::max(c->station_capacity, 1);
    o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes, 256); return r; };
    for (int k = 0; k < 2; k++) {
        L->w_seg[k] = take(sizeof(Segment) * L->seg_cap);
        L->w_bbe[k] = take(sizeof(int4) * L->seg_cap);
        L->w_segi[k] = take(sizeof(Segment) * L->seg_cap);
        L->w_bbi[k] = take(sizeof(int4) * L->seg_cap);
    }
    L->w_counts = take(sizeof(int) * (L->ntiles + 1));
    L->w_cursor = take(sizeof(int) * (L->ntiles + 1));
    L->w_nused = take(sizeof(int) * 4);
    L->w_status = take(sizeof(int) * 4);
    L->w_pml_r = take((size_t)real * 2 * 2 * (L->Sx + L->Sz) * 2);
    L->w_pml_on = take(2 * 2 * (size_t)(L->Sx + L->Sz));
    L->w_st_z = take(sizeof(double) * std::max(L->nst, 1));
    L->w_st_rec = take(sizeof(double) * 7 * (size_t)std::max(L->nst, 1) * L->stcap);
    L->w_st_cnt = take(sizeof(int) * std::max(L->nst, 1));
    L->w_ant = take(sizeof(double) * (size_t)c->nx);
    L->w_rho = take(2 * sizeof(double) * (size_t)L->Sx * L->Sz);
    // learned filter: FP32 parameters, packed BF16 fragments of the three layers, two
    // 16-channel intermediate images of the stored grid
    const bool lfk = c->filter_kind == BF_FILTER_LEARNED;
    const int nq[3] = {lf::chunks(1), lf::chunks(lf::C), lf::chunks(lf::C)};
    L->w_lf_par = take(lfk ? sizeof(float) * lf::NPARAM : 0);
    for (int k = 0; k < 3; k++) L->w_lf_pk[k] = take(lfk ? (size_t)nq[k] * lf::CHUNK_BYTES : 0);
    // beam: x, z, ux, uy, uz, w, t'* (FP64) and the state (int) of beam_capacity particles,
    // then beam_history records of 8 doubles
    for (int k = 0; k < 8; k++) L->w_beam[k] = take((k < 7 ? 8 : 4) * (size_t)c->beam_capacity);
    L->w_bhist = take(8 * sizeof(double) * (size_t)c->beam_history);
    L->w_bytes = o;
    return true;
}

// CFL (Sec. 4.2.1 Eq. cfl): the dispersion right-hand side is multilinear in the s_d^2, so
// its maximum over the zone is on a vertex; 2D takes k_y = 0 (c_y = 1).  Friedman (Sec.
// 4.3) scales it by sqrt((2+theta)/(2+3theta)).
double cfl2d(double a, double b, double g, double dx, double dz, double theta)
{
    double best = 0.0;
    const double kx = 1.0 / (dx * dx), kz = 1.0 / (dz * dz);
    for (int v = 1; v < 4; v++) {
        const double sx = (v & 1) ? 1.0 : 0.0, sz = (v & 2) ? 1.0 : 0.0;
        const double cx = 1.0 - 2.0 * sx, cz = 1.0 - 2.0 * sz;
        const double Cx = a + 2.0 * b * (1.0 + cz) + 4.0 * g * cz;
        const double Cz = a + 2.0 * b * (cx + 1.0) + 4.0 * g * cx;
        best = std::max(best, Cx * sx * kx + Cz * sz * kz);
    }
    return std::sqrt((2.0 + theta) / (2.0 + 3.0 * theta)) / std::sqrt(best);
}

bf_status validate(const bf_config* c)
{
    if (!c) return BF_EINVAL;
    if (c->abi_version != BF_ABI_VERSION || c->struct_size != sizeof(bf_config)) return BF_EINVAL;
    if (c->dim != 2 && c->dim != 3) return BF_EUNSUPPORTED;
    if (c->nx <= 0 || c->nz <= 0 || c->dx_um <= 0 || c->dz_um <= 0) return BF_EINVAL;
    if (c->dim == 3) {
        if (c->ny <= 0 || c->dy_um <= 0) return BF_EINVAL;
        if (c->filter_kind != BF_FILTER_BILINEAR) return BF_EUNSUPPORTED;
        if (((c->periodic_mask >> 1) & 1) == 0 && c->pml_cells < 4) return BF_EINVAL;
        if ((int64_t)c->nx * c->ny > (1 << 24)) return BF_EINVAL;
    }
    if (c->real_bytes != 4 && c->real_bytes != 8) return BF_EINVAL;
    if (c->shape_order != 3) return BF_EUNSUPPORTED;
    if (c->friedman_theta < 0 || c->friedman_theta > 1) return BF_EINVAL;
    if (c->filter_npass < 0 || c->filter_npass > 10) return BF_EINVAL;
    if (c->filter_strides < 0 || c->filter_strides > 0xFFFF) return BF_EINVAL;
    if (c->gather_kind < 0 || c->gather_kind > 1 || c->pusher < 0 || c->pusher > 1) return BF_EINVAL;
    {
        bf3::FiltSeq fs;
        if (!bf3::filter_seq(c->filter_npass, c->filter_compensate, c->filter_strides, &fs)) return BF_EINVAL;
    }
    if (c->filter_kind != BF_FILTER_BILINEAR && c->filter_kind != BF_FILTER_LEARNED) return BF_EINVAL;
    if (c->filter_kind == BF_FILTER_LEARNED && c->real_bytes != 4) return BF_EUNSUPPORTED;
    if (c->pml_cells < 0 || c->pml_cells > 64) return BF_EINVAL;
    if ((c->periodic_mask & 1) == 0 && c->pml_cells < 4) return BF_EINVAL;
    if (((c->periodic_mask >> 2) & 1) == 0 && c->pml_cells < 4) return BF_EINVAL;
    if (((c->periodic_mask >> 2) & 1) && c->moving_window) return BF_EINVAL;
    if (c->gamma_boost < 1.0) return BF_EINVAL;
    if (c->particle_capacity < 0 || c->particle_capacity > (int64_t)INT32_MAX - 65536) return BF_EINVAL;
    if (c->tile_x < 0 || c->tile_z < 0 || c->tile_x > 64 || c->tile_z > 64) return BF_EINVAL;
    if (c->max_stations < 0 || c->max_stations > 64 || c->station_capacity < 0) return BF_EINVAL;
    if (c->beam_capacity < 0 || c->beam_capacity > (int64_t)INT32_MAX - 65536 || c->beam_history < 0)
        return BF_EINVAL;
    if (c->pml_kind < 0 || c->pml_kind > 1) return BF_EINVAL;
    // the modified coefficients with the extended CK stencil grow without bound near the CK
    // Courant limit (measured at 0.99; bounded at 0.95)
    if (c->pml_kind == 1 && (c->ck_beta != 0.0 || c->ck_gamma != 0.0) && c->cfl_fraction > 0.95)
        return BF_EUNSUPPORTED;
    const double a2 = c->ck_alpha + 2 * c->ck_beta;
    if (std::fabs(c->ck_alpha + 4 * c->ck_beta + 4 * c->ck_gamma - 1.0) > 1e-12) return BF_EINVAL;
    (void)a2;
    if (!(c->cfl_fraction > 0.0)) return BF_EINVAL;
    if (c->cfl_fraction > 1.0) return BF_ECFL;
    return BF_OK;
}

const char* kNames[] = {"fields", "electrons0", "electrons1", "ions0", "ions1", "work"};

}  // namespace

struct Sim3;
void sim3_free(Sim3* d);

struct bf_sim {
    bf_config cfg;
    Layout L;
    Sim3* d3 = nullptr;   // the 3D run state (dim == 3)
    hipStream_t stream = nullptr;
    void* buf[6] = {};
    Geo g;
    double dt = 0, dt_crit = 0, beta = 0, gamma = 1, a2 = 1, b2 = 0, theta = 0, vw = 0;
    double n0 = 0, omega = 0, e0 = 0, w0 = 0, sig_t = 0, t0 = 0, za_lab = 0, aw = 0;
    int pol = 0;                  // laser polarisation: 0 x, 1 y
    bf_plasma plasma{};
    int have_plasma = 0, have_laser = 0, have_lf = 0;
    int e_cur = 0, b_cur = 0, eb_cur = 0, p_cur = 0, bb_cur = 0, sg_cur = 0;
    int nseg_e = 0, nseg_i = 0;
    int64_t step = 0, shift = 0, next_row = 0;
    double t = 0;
    int since_sort = 0, sort_every = 20;
    int nst = 0;
    // particle beam (Sec. 3.1.1)
    int have_beam = 0, beam_test = 1;
    int64_t nbeam = 0, beam_rec = 0;
    double vbar = 0;
    std::vector<double> st_z;
    int err = BF_OK;
    std::string msg;
    // phase timers: HIP events recorded on the stream around each phase of a step
    struct Mark { hipEvent_t a, b; int phase; };
    std::vector<hipEvent_t> ev_pool;
    std::vector<Mark> marks;
    double tacc[BF_PHASE_COUNT] = {};
    double tcnt[BF_PHASE_COUNT] = {};

    ~bf_sim()
    {
        sim3_free(d3);
        for (auto& m : marks) { ev_pool.push_back(m.a); ev_pool.push_back(m.b); }
        for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    }
    // batched execution: while rec is set, launches are gathered into rec's phase slots
    BatchRec* rec = nullptr;
    int slot = 0, rec_run = 0;
    template <class F>
    void run(F&& f)
    {
        if (rec) rec->slots[slot].emplace_back(rec_run, std::forward<F>(f));
        else f(stream);
    }

    hipEvent_t tick()
    {
        if (!cfg.phase_timers || rec) return nullptr;
        hipEvent_t e = nullptr;
        if (!ev_pool.empty()) { e = ev_pool.back(); ev_pool.pop_back(); }
        else if (hipEventCreate(&e) != hipSuccess) return nullptr;
        (void)hipEventRecord(e, stream);
        return e;
    }
    void tock(hipEvent_t a, int phase)
    {
        if (!a) return;
        hipEvent_t b = tick();
        if (!b) { ev_pool.push_back(a); return; }
        marks.push_back(Mark{a, b, phase});
    }
    // folds recorded marks into the accumulators (synchronises the stream)
    hipError_t fold_marks()
    {
        hipError_t e = hipStreamSynchronize(stream);
        for (auto& m : marks) {
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, m.a, m.b);
            tacc[m.phase] += ms;
            tcnt[m.phase] += 1.0;
            ev_pool.push_back(m.a);
            ev_pool.push_back(m.b);
        }
        marks.clear();
        return e;
    }

    char* fields() const { return (char*)buf[0]; }
    char* work() const { return (char*)buf[5]; }
    template <typename T> T* w(size_t off) const { return reinterpret_cast<T*>(work() + off); }
    template <typename R> R* arr(int a) const { return reinterpret_cast<R*>(fields() + L.field_array * a); }
};

namespace {

bf_status fail(bf_sim* s, bf_status st, const char* m)
{
    if (s) s->msg = m;
    return st;
}

bf_status hip_check(bf_sim* s, hipError_t e, const char* where)
{
    if (e == hipSuccess) return BF_OK;
    char b[256];
    snprintf(b, sizeof b, "%s: %s", where, hipGetErrorString(e));
    if (s) { s->msg = b; s->err = BF_EDEVICE; }
    return BF_EDEVICE;
}

// the 2-1/2D grid seen as a 3D one with a single y plane (for the line filter)
bf3::G3 g3_of(const Geo& g, const bf_config& c)
{
    bf3::G3 h{};
    h.N[0] = g.Nx; h.N[1] = 1; h.N[2] = g.Nz;
    h.S[0] = g.Sx; h.S[1] = 1; h.S[2] = g.Sz;
    h.P[0] = g.Px; h.P[1] = 0; h.P[2] = g.Pz;
    h.per[0] = g.perx; h.per[1] = 1; h.per[2] = g.perz;
    h.pitch = g.pitch;
    h.plane = g.pitch;
    h.zoff = g.zoff;
    h.d[0] = c.dx_um; h.d[1] = c.dx_um; h.d[2] = c.dz_um;
    return h;
}

template <typename R>
FieldSet<R> field_set(const bf_sim* s)
{
    FieldSet<R> f;
    const int e = s->e_cur, b = s->b_cur, eb = s->eb_cur;
    for (int c = 0; c < 3; c++) {
        f.E[c] = s->arr<R>((e ? A_E1 : A_E0) + c);
        f.Eo[c] = s->arr<R>((e ? A_E0 : A_E1) + c);
        f.Eb[c] = s->arr<R>((eb ? A_EB1 : A_EB0) + c);
        f.Ebn[c] = s->arr<R>((eb ? A_EB0 : A_EB1) + c);
        f.B[c] = s->arr<R>((b ? A_B1 : A_B0) + c);
        f.Bn[c] = s->arr<R>((b ? A_B0 : A_B1) + c);
        f.J[c] = s->arr<R>(A_J + c);
        f.Jf[c] = (s->cfg.filter_npass > 0 || s->cfg.filter_kind == BF_FILTER_LEARNED)
                      ? s->arr<R>(A_JF + c) : s->arr<R>(A_J + c);
    }
    f.Byx = s->arr<R>(A_BYX);
    f.Eyx = s->arr<R>(A_EYX);
    for (int c = 0; c < 6; c++) f.G[c] = s->arr<R>(A_G + c);
    return f;
}

template <typename R>
PmlTab<R> pml_tab(const bf_sim* s)
{
    PmlTab<R> p;
    R* base = s->w<R>(s->L.w_pml_r);
    uint8_t* on = s->w<uint8_t>(s->L.w_pml_on);
    const int n[2] = {s->L.Sx, s->L.Sz};
    size_t ro = 0, oo = 0;
    for (int ax = 0; ax < 2; ax++)
        for (int h = 0; h < 2; h++) {
            p.xi[ax][h] = base + ro; ro += n[ax];
            p.c[ax][h] = base + ro; ro += n[ax];
            p.on[ax][h] = on + oo; oo += n[ax];
        }
    return p;
}

template <typename R>
ElectronArrays<R> electrons(const bf_sim* s, int set)
{
    char* b = (char*)s->buf[1 + set];
    ElectronArrays<R> e;
    e.x = (double*)(b + s->L.e_off[0]);
    e.z = (double*)(b + s->L.e_off[1]);
    e.ux = (R*)(b + s->L.e_off[2]);
    e.uy = (R*)(b + s->L.e_off[3]);
    e.uz = (R*)(b + s->L.e_off[4]);
    e.w = (R*)(b + s->L.e_off[5]);
    e.id = (uint32_t*)(b + s->L.e_off[6]);
    return e;
}

template <typename R>
IonArrays<R> ions(const bf_sim* s, int set)
{
    char* b = (char*)s->buf[3 + set];
    IonArrays<R> e;
    e.x = (double*)(b + s->L.i_off[0]);
    e.z0 = (double*)(b + s->L.i_off[1]);
    e.w = (R*)(b + s->L.i_off[2]);
    e.id = (uint32_t*)(b + s->L.i_off[3]);
    return e;
}

// PML conductivity at interior-relative position p (cells) on an axis of N interior cells:
// sigma_m (d/5)^2 with sigma_m = 4 c / delta (Appendix II test prescription), d the depth
double sigma_at(double p, int N, int P, double d)
{
    if (P == 0) return 0.0;
    double dep = 0.0;
    if (p < 0.0) dep = -p; else if (p > (double)N) dep = p - (double)N;
    if (dep <= 0.0) return 0.0;
    return (4.0 / d) * (dep / 5.0) * (dep / 5.0);
}

// curl coefficient of the layer value at half-grid position p: dt (1 - xi)/(sigma dt) for the
// standard layer; for the modified coefficients dt kappa(p), kappa walked outwards from the
// inner edge with kappa(p +- 1/2) = xi(p) / kappa(p) (kappa = 1 where sigma = 0)
double pml_c(int kind, double p, int N, int P, double d, double dt)
{
    const double sg = sigma_at(p, N, P, d);
    if (sg == 0.0) return dt;
    if (kind == 0) return (1.0 - std::exp(-sg * dt)) / sg;
    const double step = p > (double)N ? 0.5 : -0.5;
    double k = 1.0;
    for (double q = p > (double)N ? (double)N : 0.0; q != p; q += step) k = std::exp(-sigma_at(q, N, P, d) * dt) / k;
    return dt * k;
}

template <typename R>
hipError_t upload_pml(bf_sim* s)
{
    const int n[2] = {s->L.Sx, s->L.Sz};
    const int P[2] = {s->L.Px, s->L.Pz};
    const int N[2] = {s->cfg.nx, s->cfg.nz};
    const double d[2] = {s->cfg.dx_um, s->cfg.dz_um};
    std::vector<R> r;
    std::vector<uint8_t> on;
    for (int ax = 0; ax < 2; ax++)
        for (int h = 0; h < 2; h++) {
            std::vector<R> xi(n[ax]), c(n[ax]);
            for (int i = 0; i < n[ax]; i++) {
                const double p = (double)(i - P[ax]) + 0.5 * h;
                const double sg = sigma_at(p, N[ax], P[ax], d[ax]);
                double x = 1.0, cc = s->dt;
                if (sg != 0.0) { x = std::exp(-sg * s->dt); cc = pml_c(s->cfg.pml_kind, p, N[ax], P[ax], d[ax], s->dt); }
                xi[i] = (R)x;
                c[i] = (R)cc;
                on.push_back(sg != 0.0 ? 1 : 0);
            }
            r.insert(r.end(), xi.begin(), xi.end());
            r.insert(r.end(), c.begin(), c.end());
        }
    Chk ck;
    ck(hipMemcpy(s->w<char>(s->L.w_pml_r), r.data(), r.size() * sizeof(R), hipMemcpyHostToDevice));
    ck(hipMemcpy(s->w<char>(s->L.w_pml_on), on.data(), on.size(), hipMemcpyHostToDevice));
    return ck.e;
}

void update_window_speed(bf_sim* s)
{
    // beta_w = (1 + omega_p^2/omega^2)^(-1/2) (Sec. 2 Eq. 1); beta_w* = (beta_w - beta)/(1 -
    // beta_w beta) (Sec. 2); vacuum or no laser: the window moves at c
    if (!s->cfg.moving_window) { s->vw = 0.0; return; }
    double bw = 1.0;
    if (s->have_laser) {
        const double wp2 = s->have_plasma ? s->n0 : 0.0;
        bw = 1.0 / std::sqrt(1.0 + wp2 / (s->omega * s->omega));
    }
    s->vw = (bw - s->beta) / (1.0 - bw * s->beta);
}

Geo geo_of(const bf_sim* s, int zoff)
{
    Geo g;
    g.Nx = s->cfg.nx; g.Nz = s->cfg.nz;
    g.Px = s->L.Px; g.Pz = s->L.Pz;
    g.Sx = s->L.Sx; g.Sz = s->L.Sz;
    g.pitch = s->L.pitch;
    g.perx = s->cfg.periodic_mask & 1;
    g.perz = (s->cfg.periodic_mask >> 2) & 1;
    g.zoff = zoff;
    return g;
}

int* nused_e(const bf_sim* s) { return s->w<int>(s->L.w_nused); }
int* nused_i(const bf_sim* s) { return s->w<int>(s->L.w_nused) + 1; }
int* status_word(const bf_sim* s) { return s->w<int>(s->L.w_status); }
Segment* seg_e(const bf_sim* s, int k) { return s->w<Segment>(s->L.w_seg[k]); }
Segment* seg_i(const bf_sim* s, int k) { return s->w<Segment>(s->L.w_segi[k]); }
int4* bb_e(const bf_sim* s, int k) { return s->w<int4>(s->L.w_bbe[k]); }
int4* bb_i(const bf_sim* s, int k) { return s->w<int4>(s->L.w_bbi[k]); }

BeamArrays beam_arrays(const bf_sim* s)
{
    const Layout& L = s->L;
    BeamArrays b;
    b.x = s->w<double>(L.w_beam[0]);
    b.z = s->w<double>(L.w_beam[1]);
    b.ux = s->w<double>(L.w_beam[2]);
    b.uy = s->w<double>(L.w_beam[3]);
    b.uz = s->w<double>(L.w_beam[4]);
    b.w = s->w<double>(L.w_beam[5]);
    b.tact = s->w<double>(L.w_beam[6]);
    b.state = s->w<int>(L.w_beam[7]);
    b.hist = s->w<double>(L.w_bhist);
    return b;
}

double ion_shift(const bf_sim* s, double t)
{
    return s->beta * t / s->cfg.dz_um + (double)s->shift;
}

template <typename R>
void sort_now(bf_sim* s)
{
    const Geo g = geo_of(s, s->g.zoff);
    const Layout& L = s->L;
    const int k = s->sg_cur;
    {
        const ElectronArrays<R> src = electrons<R>(s, s->p_cur), dst = electrons<R>(s, 1 - s->p_cur);
        Segment *so = seg_e(s, k), *sn = seg_e(s, 1 - k);
        int4* bb = bb_e(s, s->bb_cur);
        int *cnt = s->w<int>(L.w_counts), *cur = s->w<int>(L.w_cursor), *nu = nused_e(s);
        const int tx = L.tile_x, tz = L.tile_z, ntx = L.ntx, nt = L.ntiles, ns = s->nseg_e;
        s->run([=](hipStream_t st) {
            launch_sort_electrons<R>(g, tx, tz, ntx, nt, src, dst, so, ns, sn, bb, cnt, cur, nu, st);
        });
    }
    if (s->plasma.ion_mode == 1 && s->have_plasma) {
        const IonArrays<R> src = ions<R>(s, s->p_cur), dst = ions<R>(s, 1 - s->p_cur);
        Segment *so = seg_i(s, k), *sn = seg_i(s, 1 - k);
        int4* bb = bb_i(s, s->bb_cur);
        int *cnt = s->w<int>(L.w_counts), *cur = s->w<int>(L.w_cursor), *nu = nused_i(s);
        const int tx = L.tile_x, tz = L.tile_z, ntx = L.ntx, nt = L.ntiles, ns = s->nseg_i;
        const double zsh = ion_shift(s, s->t);
        s->run([=](hipStream_t st) {
            launch_sort_ions<R>(g, tx, tz, ntx, nt, src, dst, so, ns, sn, bb, zsh, cnt, cur, nu, st);
        });
        s->nseg_i = L.ntiles;
    }
    // both species end in their current buffers (the other one is the sort's scratch)
    s->sg_cur ^= 1;
    s->nseg_e = L.ntiles;
    s->since_sort = 0;
}

// rows of the plasma lattice whose upper edge has entered the interior at the current time
// (same rule as the reference: the whole row is created at the front plane)
int64_t rows_entering(const bf_sim* s)
{
    int64_t r = s->next_row;
    for (;;) {
        const double upper = (double)(r + 1) - s->beta * s->t / s->cfg.dz_um - (double)s->shift;
        if (upper > (double)s->cfg.nz) break;
        r++;
    }
    return r - s->next_row;
}

template <typename R>
void inject(bf_sim* s, int64_t nrows)
{
    if (nrows <= 0) return;
    const Layout& L = s->L;
    if (s->nseg_e + nrows * L.nchunks > L.seg_cap) sort_now<R>(s);
    if (s->nseg_e + nrows * L.nchunks > L.seg_cap) {
        // more rows than one table holds (initial load of a tall box): split
        const int64_t per = std::max<int64_t>(1, (L.seg_cap - s->nseg_e) / L.nchunks);
        while (nrows > 0) {
            const int64_t n = std::min(nrows, per);
            inject<R>(s, n);
            nrows -= n;
            if (nrows > 0) sort_now<R>(s);
        }
        return;
    }
    InjectParams ip;
    ip.row0 = s->next_row;
    ip.nrows = (int)nrows;
    ip.nchunks = L.nchunks;
    ip.tile_x = L.tile_x;
    ip.ppc = s->plasma.ppc;
    ip.ion_mode = s->plasma.ion_mode;
    ip.beta = s->beta;
    ip.gamma = s->gamma;
    ip.t = s->t;
    ip.dz_um = s->cfg.dz_um;
    ip.dx_um = s->cfg.dx_um;
    ip.shift = (double)s->shift;
    ip.n0 = s->n0;
    ip.ramp_start = s->plasma.start_um;
    ip.ramp_len = s->plasma.ramp_um;
    ip.wfac = s->gamma * s->cfg.dx_um * s->cfg.dz_um / (double)s->plasma.ppc;
    ip.uz0 = -s->gamma * s->beta;
    ip.seed = s->cfg.seed;
    ip.seg_base = s->nseg_e;
    ip.cap = L.cap;
    const int k = s->sg_cur;
    {
        const Geo g = s->g;
        const ElectronArrays<R> e = electrons<R>(s, s->p_cur);
        const IonArrays<R> ion = ions<R>(s, s->p_cur);
        Segment *se = seg_e(s, k), *si = seg_i(s, k);
        int4 *be = bb_e(s, s->bb_cur), *bi = bb_i(s, s->bb_cur);
        int *ne = nused_e(s), *ni = nused_i(s), *stw = status_word(s);
        s->run([=](hipStream_t st) { launch_inject<R>(g, e, ion, se, be, si, bi, ne, ni, ip, stw, st); });
    }
    s->nseg_e += (int)nrows * L.nchunks;
    if (s->plasma.ion_mode == 1) s->nseg_i = s->nseg_e;
    s->next_row += nrows;
}

// the arrays whose rows move with the window (the filter's intermediate and the node values of
// the momentum-conserving gather are rewritten every step before they are read)
constexpr int A_PERSISTENT = A_JT;
static_assert(A_PERSISTENT <= 32, "PtrList holds 32 arrays");

template <typename R>
PtrList<R> all_arrays(const bf_sim* s)
{
    PtrList<R> p;
    p.n = A_PERSISTENT;
    for (int a = 0; a < A_PERSISTENT; a++) p.p[a] = s->arr<R>(a);
    return p;
}

lf::Packed lf_packed(bf_sim* s)
{
    lf::Packed p{};
    for (int k = 0; k < 3; k++) p.fwd[k] = s->w<unsigned char>(s->L.w_lf_pk[k]);
    return p;
}

// the learned filter on J_x, J_y, J_z, each on its own staggered domain (as the bilinear
// filter), reading and writing the ring-buffered rows in place
void learned_filter(bf_sim* s, const FieldSet<float>& f)
{
    const Geo g = s->g;
    const int hx[3] = {1, 0, 0}, hz[3] = {0, 0, 1};
    const lf::Packed pk = lf_packed(s);
    struct { lf::View in[3], out[3]; lf::Domain d[3]; } a;
    for (int c = 0; c < 3; c++) {
        a.d[c].nimg = 1;
        a.d[c].nx = g.perx ? g.Sx : g.Sx - hx[c];
        a.d[c].ny = g.perz ? g.Sz : g.Sz - hz[c];
        a.d[c].perx = g.perx;
        a.d[c].pery = g.perz;
        a.in[c] = lf::View{f.J[c], 0, g.pitch, 1, g.zoff, g.Sz};
        a.out[c] = lf::View{f.Jf[c], 0, g.pitch, 1, g.zoff, g.Sz};
    }
    s->run([=](hipStream_t st) { lf::forward_fused(a.in, a.out, a.d, 3, pk, st); });
}

// batched recording is FP32 only (a batch is created from FP32 runs)
template <typename R>
BatchRec* batch_rec(bf_sim* s)
{
    if constexpr (sizeof(R) == 4) return s->rec;
    else return nullptr;
}

template <typename R>
bf_status step_impl(bf_sim* s, int nsteps)
{
    const bf_config& c = s->cfg;
    const Layout& L = s->L;
    SolverCoef sc{s->dt, s->a2, s->b2, s->theta, 1.0 / c.dx_um, 1.0 / c.dz_um};
    const PmlTab<R> pm = pml_tab<R>(s);
    for (int n = 0; n < nsteps; n++) {
        const FieldSet<R> f = field_set<R>(s);
        const Geo g = s->g;
        BatchRec* rb = batch_rec<R>(s);
        // Faraday + Friedman + PML
        s->slot = SLOT_FARADAY;
        hipEvent_t t_ph = s->tick();
        if constexpr (sizeof(R) == 4) {
            if (rb) {
                const int gx = (g.Sx + 63) / 64, gz = (g.Sz + 3) / 4;
                rb->faraday.push_back(FaradayDesc<float>{g, f, pm, (float)sc.dt, (float)sc.a2, (float)sc.b2,
                                                         (float)sc.theta, (float)sc.idx, (float)sc.idz,
                                                         sc.theta > 0.0 ? 1 : 0, gx});
                rb->n_faraday.push_back(gx * gz);
            }
        }
        if (!rb) launch_faraday<R>(g, f, pm, sc, s->stream);
        // stations (E^n, B^n)
        if (s->nst > 0) {
            StationParams sp;
            sp.n = s->nst;
            sp.zlab = s->w<double>(L.w_st_z);
            sp.gamma = s->gamma; sp.beta = s->beta; sp.t = s->t; sp.dz_um = c.dz_um;
            sp.shift = (double)s->shift; sp.xc = 0.5 * c.nx; sp.cap = L.stcap;
            double* rec = s->w<double>(L.w_st_rec);
            int* cnt = s->w<int>(L.w_st_cnt);
            s->slot = SLOT_STATIONS;
            s->run([=](hipStream_t st) { launch_stations<R>(g, f, sp, rec, cnt, st); });
        }
        s->tock(t_ph, BF_PHASE_FARADAY);
        // window position after this step
        const double t1 = (double)(s->step + 1) * s->dt;
        int64_t s1 = s->shift;
        if (c.moving_window) s1 = (int64_t)std::trunc(s->vw * t1 / c.dz_um);
        const int d = (int)(s1 - s->shift);
        // electrons
        PushParams<R> pp;
        pp.qdt2 = (R)(-0.5 * s->dt);
        pp.dtdx = (R)(s->dt / c.dx_um);
        pp.dtdz = (R)(s->dt / c.dz_um);
        pp.fjx = (R)(1.0 / (c.dz_um * s->dt));    // -q/(dz dt) with q = -1 (times w)
        pp.fjz = (R)(1.0 / (c.dx_um * s->dt));
        pp.fjy = (R)(-1.0 / (c.dx_um * c.dz_um));
        pp.shift = d;
        pp.vay = c.pusher;
        s->slot = SLOT_PUSH;
        t_ph = s->tick();
        if (c.gather_kind == 1) launch_nodes<R>(g, f, s->stream);      // single runs only (not batched)
        {
            const ElectronArrays<R> e = electrons<R>(s, s->p_cur);
            const Segment* sg = seg_e(s, s->sg_cur);
            const int4* bi = bb_e(s, s->bb_cur);
            int4* bo = bb_e(s, 1 - s->bb_cur);
            if constexpr (sizeof(R) == 4) {
                if (rb && s->nseg_e > 0) {
                    rb->gpd.push_back(GpdDesc<float>{g, f, e, sg, bi, bo, pp, status_word(s)});
                    rb->n_gpd.push_back(s->nseg_e);
                }
            }
            if (!rb) launch_gpd<R>(g, f, e, sg, bi, bo, s->nseg_e, pp, status_word(s), c.gather_kind == 1, s->stream);
        }
        s->tock(t_ph, BF_PHASE_PUSH);
        // rigid ions: deposit-only J_z
        s->slot = SLOT_IONS;
        t_ph = s->tick();
        if (s->have_plasma && s->plasma.ion_mode == 1) {
            const IonArrays<R> ion = ions<R>(s, s->p_cur);
            const Segment* sg = seg_i(s, s->sg_cur);
            const int4* bi = bb_i(s, s->bb_cur);
            int4* bo = bb_i(s, 1 - s->bb_cur);
            const double za = ion_shift(s, s->t), zb = ion_shift(s, t1);
            const R fjz = (R)(-1.0 / (c.dx_um * s->dt));
            // batched runs launch their ions one run at a time too: the hardware's dispatch of
            // one workgroup per segment balances the uneven segments better than a persistent
            // launch over all runs
            const int nsi = s->nseg_i;
            s->run([=](hipStream_t st) { launch_ions<R>(g, f, ion, sg, bi, bo, nsi, za, zb, d, fjz, st); });
        }
        s->tock(t_ph, BF_PHASE_IONS);
        // beam through the injection plane (single runs only: a batch rejects beam runs)
        if (s->have_beam) {
            t_ph = s->tick();
            BeamParams bp;
            bp.n = (int)s->nbeam;
            bp.deposit = s->beam_test ? 0 : 1;
            bp.rec = s->beam_rec < c.beam_history ? (int)s->beam_rec : -1;
            bp.t0 = s->t; bp.t1 = t1;
            bp.vbar_cells = s->vbar * s->dt / c.dz_um;
            bp.gamma = s->gamma; bp.beta = s->beta; bp.dz_um = c.dz_um;
            bp.shift = (double)s->shift;
            PushParams<double> pb;
            pb.qdt2 = -0.5 * s->dt;
            pb.dtdx = s->dt / c.dx_um;
            pb.dtdz = s->dt / c.dz_um;
            pb.fjx = 1.0 / (c.dz_um * s->dt);
            pb.fjz = 1.0 / (c.dx_um * s->dt);
            pb.fjy = -1.0 / (c.dx_um * c.dz_um);
            pb.shift = d;
            pb.vay = c.pusher;
            launch_beam<R>(g, f, beam_arrays(s), bp, pb, status_word(s), c.gather_kind == 1, s->stream);
            if (bp.rec >= 0) s->beam_rec++;
            s->tock(t_ph, BF_PHASE_BEAM);
        }
        // antenna
        s->slot = SLOT_ANTENNA;
        t_ph = s->tick();
        if (s->have_laser) {
            AntennaParams ap;
            ap.n = c.nx;
            ap.za = (s->za_lab / s->gamma - s->beta * s->t) / c.dz_um - (double)s->shift;
            ap.zb = (s->za_lab / s->gamma - s->beta * t1) / c.dz_um - (double)s->shift;
            ap.tmid = s->t + 0.5 * s->dt;
            ap.gamma = s->gamma; ap.e0 = s->e0; ap.omega = s->omega; ap.w0 = s->w0;
            ap.sig_t = s->sig_t; ap.t0 = s->t0; ap.dx_um = c.dx_um; ap.xc_um = 0.5 * c.nx * c.dx_um;
            ap.weight = s->aw; ap.dt = s->dt; ap.dx = c.dx_um; ap.dz = c.dz_um;
            ap.active = (ap.za >= 0.0 && ap.za < (double)c.nz) ? 1 : 0;
            ap.pol = s->pol;
            double* xm = s->w<double>(L.w_ant);
            s->run([=](hipStream_t st) { launch_antenna<R>(g, f, xm, ap, st); });
        }
        s->tock(t_ph, BF_PHASE_ANTENNA);
        // filter
        s->slot = SLOT_FILTER;
        t_ph = s->tick();
        if (c.filter_kind == BF_FILTER_LEARNED) {
            if constexpr (sizeof(R) == 4) learned_filter(s, f);
        } else if (c.filter_npass > 0) {
            // the line filter, one run at a time also in a batch (per run it beats the batched
            // tile filter)
            bf3::FiltSeq fs;
            bf3::filter_seq(c.filter_npass, c.filter_compensate, c.filter_strides, &fs);
            const bf3::G3 g3 = g3_of(g, c);
            const FieldSet<R> ff = f;
            R* tmp0 = s->arr<R>(A_JT);
            R* tmp1 = s->arr<R>(A_JT + 1);
            R* tmp2 = s->arr<R>(A_JT + 2);
            s->run([=](hipStream_t st) {
                R* in[3] = {ff.J[0], ff.J[1], ff.J[2]};
                R* out[3] = {ff.Jf[0], ff.Jf[1], ff.Jf[2]};
                R* tmp[3] = {tmp0, tmp1, tmp2};
                const int hx[3] = {1, 0, 0}, hz[3] = {0, 0, 1};
                bf3::launch_filter_xz<R>(g3, in, tmp, out, hx, hz, 3, fs, st);
            });
        }
        s->tock(t_ph, BF_PHASE_FILTER);
        // Ampere + PML (E^{n+1} into the E^{n-1} set)
        s->slot = SLOT_AMPERE;
        t_ph = s->tick();
        if constexpr (sizeof(R) == 4) {
            if (rb) {
                const int gx = (g.Sx + 63) / 64, gz = (g.Sz + 3) / 4;
                rb->ampere.push_back(AmpereDesc<float>{g, f, pm, (float)sc.dt, (float)sc.idx, (float)sc.idz, gx});
                rb->n_ampere.push_back(gx * gz);
            }
        }
        if (!rb) launch_ampere<R>(g, f, pm, sc, s->stream);
        s->tock(t_ph, BF_PHASE_AMPERE);
        s->e_cur ^= 1;
        s->b_cur ^= 1;
        if (s->theta > 0.0) s->eb_cur ^= 1;
        s->bb_cur ^= 1;
        s->step++;
        s->t = (double)s->step * s->dt;
        // moving window: advance the ring offset and clear the new rows
        s->slot = SLOT_WINDOW;
        t_ph = s->tick();
        if (d != 0) {
            s->g.zoff = (int)(((int64_t)s->g.zoff + d) % L.Sz);
            if (s->g.zoff < 0) s->g.zoff += L.Sz;
            s->shift = s1;
            EntryRows er{};
            // rows that just left the z-PML for the interior drop their split x-part
            for (int h = 0; h < 2; h++) {
                for (int k = 0; k < L.Sz; k++) {
                    const double pk = (double)(k - L.Pz) + 0.5 * h;
                    if (sigma_at(pk, c.nz, L.Pz, c.dz_um) != 0.0) continue;
                    if (sigma_at(pk + d, c.nz, L.Pz, c.dz_um) == 0.0) continue;
                    if (h == 1 && er.nh < 4) er.h[er.nh++] = k;
                    if (h == 0 && er.nn < 4) er.n[er.nn++] = k;
                }
            }
            const FieldSet<R> f2 = field_set<R>(s);
            const Geo g2 = s->g;
            const PtrList<R> arrs = all_arrays<R>(s);
            s->run([=](hipStream_t st) { launch_window_rows<R>(g2, arrs, d, er, f2, pm, st); });
        }
        // plasma injection at the front plane
        if (s->have_plasma) inject<R>(s, rows_entering(s));
        s->tock(t_ph, BF_PHASE_WINDOW);
        s->slot = SLOT_SORT;
        t_ph = s->tick();
        if (++s->since_sort >= s->sort_every && s->have_plasma) sort_now<R>(s);
        s->tock(t_ph, BF_PHASE_SORT);
        if (s->marks.size() > 40000) {
            hipError_t e = s->fold_marks();
            if (e != hipSuccess) return hip_check(s, e, "phase timers");
        }
    }
    return BF_OK;
}

}  // namespace

// ======================================================================================
// C ABI
// ======================================================================================

// ---- 3D runs -----------------------------------------------------------------------------------
// The same C ABI drives the 3D step (bf_config.dim == 3): fields [z][y][x] with a ring of z
// planes, SoA particles with x, y, z, and the 3D kernels of bf_sim3.hip.  Particles live in one
// of two copies; every sort_every steps the live ones are sorted by tile into the other copy.

struct Sim3 {
    bf3::G3 g{};
    size_t fa = 0, fa8 = 0, fields_bytes = 0;   // bytes per array (run's type, FP64)
    size_t e_off[8] = {}, e_bytes = 0, i_off[5] = {}, i_bytes = 0;
    size_t w_status = 0, w_nused = 0, w_cnt = 0, w_pml = 0, w_ant = 0, w_st_z = 0, w_st_rec = 0, w_st_cnt = 0,
           w_seg_e = 0, w_seg_i = 0, w_box_e[2] = {}, w_box_i[2] = {}, w_counts = 0, w_cursor = 0, w_tot = 0,
           w_lists = 0, w_mis = 0,
           w_bytes = 0;
    int64_t cap = 0;
    int nst_max = 0, stcap = 1, p_cur = 0, since_sort = 0;
    bf3::Tiles3 tl{};
    int seg_cap = 0, nseg = 0, bb_cur = 0;   // segments (tiles of the last sort, then injected chunks)
    int pz = 0;                              // z planes of the LDS box
    int na = 0;
    int eb_cur = 0;                          // which of A3_EB / A3_T holds the Friedman average
};

void sim3_free(Sim3* d) { delete d; }

namespace {

// arrays in the run's type, then the three FP64 current accumulators (ids A3_J + c)
enum { A3_E = 0, A3_EO = 3, A3_EB = 6, A3_B = 9, A3_BO = 12, A3_JG = 15, A3_JF = 18, A3_SE = 21, A3_SB = 24,
       A3_T = 27, A3_COUNT = 30, A3_J = 100 };

double cfl3d(double a, double b, double g, const double d[3], double theta)
{
    double best = 0.0;
    for (int v = 1; v < 8; v++) {
        double s[3], c[3];
        for (int k = 0; k < 3; k++) { s[k] = (v >> k) & 1 ? 1.0 : 0.0; c[k] = 1.0 - 2.0 * s[k]; }
        double rhs = 0.0;
        for (int k = 0; k < 3; k++) {
            const double ck = c[(k + 1) % 3], cl = c[(k + 2) % 3];
            rhs += (a + 2.0 * b * (ck + cl) + 4.0 * g * ck * cl) * s[k] / (d[k] * d[k]);
        }
        best = std::max(best, rhs);
    }
    return std::sqrt((2.0 + theta) / (2.0 + 3.0 * theta)) / std::sqrt(best);
}

void layout3(const bf_config* c, Sim3* L)
{
    const int N[3] = {c->nx, c->ny, c->nz};
    const double d[3] = {c->dx_um, c->dy_um, c->dz_um};
    const size_t real = c->real_bytes;
    for (int a = 0; a < 3; a++) {
        L->g.N[a] = N[a];
        L->g.per[a] = (c->periodic_mask >> a) & 1;
        L->g.P[a] = L->g.per[a] ? 0 : c->pml_cells;
        L->g.S[a] = L->g.per[a] ? N[a] : N[a] + 2 * L->g.P[a] + 1;
        L->g.d[a] = d[a];
    }
    L->g.pitch = (long)align_up((size_t)L->g.S[0], 256 / real);
    L->g.plane = L->g.pitch * L->g.S[1];
    L->g.zoff = 0;
    L->fa = align_up((size_t)L->g.plane * L->g.S[2] * real, 256);
    L->fa8 = align_up((size_t)L->g.plane * L->g.S[2] * 8, 256);
    L->fields_bytes = L->fa * A3_COUNT + 3 * L->fa8;
    if (c->gather_kind == 1) L->fields_bytes += 6 * L->fa;       // node values of E^n, B^n
    L->cap = std::max<int64_t>(c->particle_capacity, 1);
    size_t o = 0;
    const size_t esz[8] = {8, 8, 8, real, real, real, real, 4};
    for (int k = 0; k < 8; k++) { L->e_off[k] = o; o = align_up(o + esz[k] * L->cap, 256); }
    L->e_bytes = std::max<size_t>(o, 256);
    o = 0;
    const size_t isz[5] = {8, 8, 8, real, 4};
    for (int k = 0; k < 5; k++) { L->i_off[k] = o; o = align_up(o + isz[k] * L->cap, 256); }
    L->i_bytes = std::max<size_t>(o, 256);
    L->nst_max = std::max(c->max_stations, 0);
    L->stcap = std::max(c->station_capacity, 1);
    // particle tiles: tx x ty transverse (the LDS box pitches leave room for the stencil reach and
    // one cell of spread) by tz cells along z
    const int tx = std::min(std::max(c->tile_x > 0 ? c->tile_x : 16, 1), bf3::BOX_PX - 8);
    const int ty = std::max(1, std::min(4, bf3::BOX_PY - 6));
    const int tz = std::max(c->tile_z > 0 ? c->tile_z : (real == 4 ? 7 : 2), 1);
    const int tv[3] = {tx, ty, tz};
    L->tl.ntiles = 1;
    for (int a = 0; a < 3; a++) {
        L->tl.t[a] = tv[a];
        L->tl.nt[a] = (N[a] + tv[a] - 1) / tv[a];
        L->tl.ntiles *= L->tl.nt[a];
    }
    const int sort_every = c->sort_every > 0 ? c->sort_every : 20;
    L->seg_cap = L->tl.ntiles + L->tl.nt[0] * L->tl.nt[1] * (3 * sort_every + 16);
    o = 0;
    auto take = [&](size_t b) { size_t r = o; o = align_up(o + b, 256); return r; };
    L->w_status = take(16);
    L->w_nused = take(16);
    L->w_cnt = take(16);
    L->w_tot = take(16);
    L->w_seg_e = take(sizeof(bf3::Seg3) * L->seg_cap);
    L->w_seg_i = take(sizeof(bf3::Seg3) * L->seg_cap);
    for (int k = 0; k < 2; k++) {
        L->w_box_e[k] = take(sizeof(bf3::Box3) * L->seg_cap);
        L->w_box_i[k] = take(sizeof(bf3::Box3) * L->seg_cap);
    }
    L->w_counts = take(sizeof(int) * L->tl.ntiles);
    L->w_lists = take(sizeof(int) * (2 + (size_t)L->seg_cap));
    L->w_mis = take(sizeof(int) * 2 * (size_t)L->cap);
    L->w_cursor = take(sizeof(int) * L->tl.ntiles);
    L->w_pml = take(sizeof(double) * 3 * 2 * 3 * (size_t)(L->g.S[0] + L->g.S[1] + L->g.S[2]));
    L->w_ant = take(sizeof(double) * 3 * (size_t)N[0] * N[1]);
    L->w_st_z = take(sizeof(double) * std::max(L->nst_max, 1));
    L->w_st_rec = take(sizeof(double) * 7 * (size_t)std::max(L->nst_max, 1) * L->stcap);
    L->w_st_cnt = take(sizeof(int) * std::max(L->nst_max, 1));
    L->w_bytes = o;
}

void sizes3(const Sim3& L, size_t out[6])
{
    out[0] = L.fields_bytes;
    out[1] = out[2] = L.e_bytes;
    out[3] = out[4] = L.i_bytes;
    out[5] = L.w_bytes;
}

template <typename T> T* w3(const bf_sim* s, size_t off) { return reinterpret_cast<T*>((char*)s->buf[5] + off); }

template <typename R>
R* arr3(const bf_sim* s, int a) { return reinterpret_cast<R*>((char*)s->buf[0] + s->d3->fa * a); }

double* jacc3(const bf_sim* s, int c)
{
    return reinterpret_cast<double*>((char*)s->buf[0] + s->d3->fa * A3_COUNT + s->d3->fa8 * c);
}

template <typename R>
bf3::F3<R> fields3(const bf_sim* s)
{
    bf3::F3<R> f;
    for (int c = 0; c < 3; c++) {
        f.E[c] = arr3<R>(s, A3_E + c); f.Eo[c] = arr3<R>(s, A3_EO + c);
        f.Eb[c] = arr3<R>(s, (s->d3->eb_cur ? A3_T : A3_EB) + c);
        f.T[c] = arr3<R>(s, (s->d3->eb_cur ? A3_EB : A3_T) + c);
        f.B[c] = arr3<R>(s, A3_B + c); f.Bo[c] = arr3<R>(s, A3_BO + c); f.J[c] = jacc3(s, c);
        f.Jf[c] = arr3<R>(s, A3_JF + c); f.Jg[c] = arr3<R>(s, A3_JG + c);
        f.SE[c] = arr3<R>(s, A3_SE + c); f.SB[c] = arr3<R>(s, A3_SB + c);
    }
    for (int c = 0; c < 6; c++)
        f.G[c] = s->cfg.gather_kind == 1
                     ? reinterpret_cast<R*>((char*)s->buf[0] + s->d3->fa * A3_COUNT + 3 * s->d3->fa8 + s->d3->fa * c)
                     : nullptr;
    return f;
}

template <typename R>
bf3::E3<R> electrons3(const bf_sim* s, int copy)
{
    char* b = (char*)s->buf[1 + copy];
    const Sim3& L = *s->d3;
    bf3::E3<R> e;
    e.x = (double*)(b + L.e_off[0]); e.y = (double*)(b + L.e_off[1]); e.z = (double*)(b + L.e_off[2]);
    e.ux = (R*)(b + L.e_off[3]); e.uy = (R*)(b + L.e_off[4]); e.uz = (R*)(b + L.e_off[5]);
    e.w = (R*)(b + L.e_off[6]); e.id = (uint32_t*)(b + L.e_off[7]);
    return e;
}

template <typename R>
bf3::I3<R> ions3(const bf_sim* s, int copy)
{
    char* b = (char*)s->buf[3 + copy];
    const Sim3& L = *s->d3;
    bf3::I3<R> ion;
    ion.x = (double*)(b + L.i_off[0]); ion.y = (double*)(b + L.i_off[1]); ion.z0 = (double*)(b + L.i_off[2]);
    ion.w = (R*)(b + L.i_off[3]); ion.id = (uint32_t*)(b + L.i_off[4]);
    return ion;
}

bf3::Pml3 pml3(const bf_sim* s)
{
    const Sim3& L = *s->d3;
    bf3::Pml3 p;
    double* base = w3<double>(s, L.w_pml);
    size_t o = 0;
    for (int a = 0; a < 3; a++)
        for (int h = 0; h < 2; h++) {
            p.sig[a][h] = base + o; o += L.g.S[a];
            p.xi[a][h] = base + o; o += L.g.S[a];
            p.c[a][h] = base + o; o += L.g.S[a];
        }
    return p;
}

hipError_t upload_pml3(bf_sim* s)
{
    const Sim3& L = *s->d3;
    std::vector<double> t;
    for (int a = 0; a < 3; a++)
        for (int h = 0; h < 2; h++) {
            std::vector<double> sg(L.g.S[a]), xi(L.g.S[a]), c(L.g.S[a]);
            for (int i = 0; i < L.g.S[a]; i++) {
                const double p = (double)(i - L.g.P[a]) + 0.5 * h;
                sg[i] = L.g.per[a] ? 0.0 : sigma_at(p, L.g.N[a], L.g.P[a], L.g.d[a]);
                xi[i] = 1.0;
                c[i] = s->dt;
                if (sg[i] != 0.0) {
                    xi[i] = std::exp(-sg[i] * s->dt);
                    c[i] = pml_c(s->cfg.pml_kind, p, L.g.N[a], L.g.P[a], L.g.d[a], s->dt);
                }
            }
            t.insert(t.end(), sg.begin(), sg.end());
            t.insert(t.end(), xi.begin(), xi.end());
            t.insert(t.end(), c.begin(), c.end());
        }
    return hipMemcpy(w3<char>(s, L.w_pml), t.data(), t.size() * 8, hipMemcpyHostToDevice);
}

bf_status create3(const bf_config* cfg, const bf_buffer_binding* b, int n, void* stream, bf_sim** out)
{
    bf_sim* s = new bf_sim();
    s->cfg = *cfg;
    s->d3 = new Sim3();
    layout3(cfg, s->d3);
    size_t sizes[6];
    sizes3(*s->d3, sizes);
    for (int k = 0; k < 6; k++) {
        for (int q = 0; q < n; q++)
            if (b[q].name && std::strcmp(b[q].name, kNames[k]) == 0) {
                if (b[q].bytes < sizes[k] || !b[q].ptr || ((uintptr_t)b[q].ptr & 255u)) { delete s; return BF_EINVAL; }
                s->buf[k] = b[q].ptr;
            }
        if (!s->buf[k]) { delete s; return BF_EINVAL; }
    }
    s->stream = (hipStream_t)stream;
    s->gamma = cfg->gamma_boost;
    s->beta = std::sqrt(1.0 - 1.0 / (s->gamma * s->gamma));
    s->theta = cfg->friedman_theta;
    const double d[3] = {cfg->dx_um, cfg->dy_um, cfg->dz_um};
    s->dt_crit = cfl3d(cfg->ck_alpha, cfg->ck_beta, cfg->ck_gamma, d, s->theta);
    s->dt = cfg->cfl_fraction * s->dt_crit;
    s->sort_every = cfg->sort_every > 0 ? cfg->sort_every : 20;
    update_window_speed(s);
    {
        // z planes of the LDS box: the tile, one cell of drift and the stencil reach, as far as
        // the workgroup's LDS allows
        int dev = 0, lds_max = 65536;
        if (hipGetDevice(&dev) == hipSuccess)
            (void)hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
        const int cell = cfg->real_bytes == 4 ? bf3::box_cell_bytes<float>() : bf3::box_cell_bytes<double>();
        const int fit = lds_max / (bf3::BOX_PL * cell);
        s->d3->pz = std::min(s->d3->tl.t[2] + 7, fit);
    }
    hipError_t e = hipSuccess;
    for (int k = 0; k < 6 && e == hipSuccess; k++) e = hipMemsetAsync(s->buf[k], 0, sizes[k], s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e == hipSuccess) e = upload_pml3(s);
    if (e != hipSuccess) { delete s; return BF_EDEVICE; }
    *out = s;
    return BF_OK;
}

template <typename R>
bf3::Seg3* seg3(const bf_sim* s, int species)
{
    return w3<bf3::Seg3>(s, species == 0 ? s->d3->w_seg_e : s->d3->w_seg_i);
}

bf3::Box3* box3(const bf_sim* s, int species, int k)
{
    return w3<bf3::Box3>(s, species == 0 ? s->d3->w_box_e[k] : s->d3->w_box_i[k]);
}

// ions' boosted position in the current window frame: z = z0 - zshift3
double zshift3(const bf_sim* s, double t)
{
    return s->beta * t / s->cfg.dz_um + (double)s->shift;
}

// counting sort of both species by tile (drops removed particles); segments = tiles.  The
// particles end in their current copy (the other one is the sort's scratch).
template <typename R>
void sort3(bf_sim* s)
{
    Sim3& L = *s->d3;
    const int a = L.p_cur, b = 1 - a;
    int* nu = w3<int>(s, L.w_nused);
    int *cnt = w3<int>(s, L.w_counts), *cur = w3<int>(s, L.w_cursor), *tot = w3<int>(s, L.w_tot);
    bf3::launch3_sort_e<R>(L.g, L.tl, electrons3<R>(s, a), electrons3<R>(s, b), nu, cnt, cur, tot, seg3<R>(s, 0),
                           box3(s, 0, L.bb_cur), L.cap, s->have_plasma ? s->plasma.ppc : 1, s->stream);
    if (s->have_plasma && s->plasma.ion_mode == 1)
        bf3::launch3_sort_i<R>(L.g, L.tl, ions3<R>(s, a), ions3<R>(s, b), zshift3(s, s->t), nu + 1, cnt, cur,
                               tot + 1, seg3<R>(s, 1), box3(s, 1, L.bb_cur), L.cap, s->plasma.ppc, s->stream);
    L.nseg = L.tl.ntiles;
    L.since_sort = 0;
}

template <typename R>
hipError_t inject3(bf_sim* s, int64_t nrows)
{
    Sim3& L = *s->d3;
    if (nrows <= 0) return hipSuccess;
    const int chunks = L.tl.nt[0] * L.tl.nt[1];
    if (L.nseg + nrows * chunks > L.seg_cap) sort3<R>(s);
    if (L.nseg + nrows * chunks > L.seg_cap) {
        // more planes than one table holds (the initial load of a long box): in parts
        const int64_t per = std::max<int64_t>(1, (L.seg_cap - L.nseg) / chunks);
        while (nrows > 0) {
            const int64_t n = std::min(nrows, per);
            hipError_t e = inject3<R>(s, n);
            if (e != hipSuccess) return e;
            nrows -= n;
            if (nrows > 0) sort3<R>(s);
        }
        return hipSuccess;
    }
    bf3::Inject3 ip;
    ip.row0 = s->next_row;
    ip.nrows = (int)nrows;
    ip.ppc = s->plasma.ppc;
    ip.ion_mode = s->plasma.ion_mode;
    ip.cap = L.cap;
    ip.seed = s->cfg.seed;
    ip.gamma = s->gamma;
    ip.beta = s->beta;
    ip.t = s->t;
    ip.dx = s->cfg.dx_um;
    ip.dy = s->cfg.dy_um;
    ip.dz = s->cfg.dz_um;
    ip.n0 = s->n0;
    ip.ramp_start = s->plasma.start_um;
    ip.ramp_len = s->plasma.ramp_um;
    ip.uz0 = -s->gamma * s->beta;
    ip.shift = (double)s->shift;
    int* nu = w3<int>(s, L.w_nused);
    bf3::launch3_inject<R>(L.g, L.tl, electrons3<R>(s, L.p_cur), ions3<R>(s, L.p_cur), nu, nu + 1, seg3<R>(s, 0),
                           box3(s, 0, L.bb_cur), seg3<R>(s, 1), box3(s, 1, L.bb_cur), L.nseg, ip,
                           w3<int>(s, L.w_status), s->stream);
    L.nseg += (int)nrows * chunks;
    s->next_row += nrows;
    return hipGetLastError();
}

// particle slots in use of a species (synchronous read of the device counter)
hipError_t slots3(bf_sim* s, int species, int64_t* n)
{
    int v = 0;
    hipError_t e = hipMemcpyAsync(&v, w3<int>(s, s->d3->w_nused) + species, sizeof(int), hipMemcpyDeviceToHost,
                                  s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    *n = v;
    return e;
}

template <typename R>
bf_status step3(bf_sim* s, int nsteps)
{
    Sim3& L = *s->d3;
    const double d[3] = {s->cfg.dx_um, s->cfg.dy_um, s->cfg.dz_um};
    const double ck[3] = {s->cfg.ck_alpha, s->cfg.ck_beta, s->cfg.ck_gamma};
    const bf3::Pml3 pml = pml3(s);
    for (int it = 0; it < nsteps; it++) {
        bf3::F3<R> f = fields3<R>(s);
        const bf3::G3 g = L.g;
        hipEvent_t ev = s->tick();
        bf3::launch3_faraday<R>(g, f, pml, ck, s->theta, s->dt, s->stream);
        if (s->theta > 0.0) {   // the new Friedman average is in the other buffer
            L.eb_cur ^= 1;
            f = fields3<R>(s);
        }
        bf3::launch3_stations<R>(g, f, w3<double>(s, L.w_st_z), s->nst, s->gamma, s->beta, s->t, (double)s->shift,
                                 w3<double>(s, L.w_st_rec), w3<int>(s, L.w_st_cnt), L.stcap, s->stream);
        bf3::launch3_zero_j<R>(g, f, s->stream);        // the current of this step starts at zero
        s->tock(ev, BF_PHASE_FARADAY);
        // the window shift at the end of this step (particles are rebased in the push)
        const double t1 = (double)(s->step + 1) * s->dt;
        int64_t sn = s->shift;
        if (s->cfg.moving_window && !L.g.per[2]) sn = (int64_t)std::trunc(s->vw * t1 / d[2]);
        const int dsh = (int)(sn - s->shift);
        bf3::Push3 pp;
        pp.dt = s->dt;
        for (int a = 0; a < 3; a++) {
            pp.dtd[a] = s->dt / d[a];
            pp.jk[a] = 1.0 / (d[(a + 1) % 3] * d[(a + 2) % 3] * s->dt);
        }
        pp.shift = (double)dsh;
        pp.vay = s->cfg.pusher;
        ev = s->tick();
        const bool mc = s->cfg.gather_kind == 1;
        if (mc) bf3::launch3_nodes<R>(g, f, s->stream);
        bf3::launch3_gpd<R>(g, f, electrons3<R>(s, L.p_cur), seg3<R>(s, 0), box3(s, 0, L.bb_cur),
                            box3(s, 0, 1 - L.bb_cur), L.nseg, pp, L.pz, w3<int>(s, L.w_status), w3<int>(s, L.w_lists),
                            w3<int2>(s, L.w_mis), mc, s->stream);
        s->tock(ev, BF_PHASE_PUSH);
        ev = s->tick();
        if (s->have_plasma && s->plasma.ion_mode == 1)
            bf3::launch3_gpi<R>(g, f, ions3<R>(s, L.p_cur), seg3<R>(s, 1), box3(s, 1, L.bb_cur),
                                box3(s, 1, 1 - L.bb_cur), L.nseg, s->beta * s->t / d[2] + (double)s->shift,
                                s->beta * t1 / d[2] + (double)s->shift, s->beta * t1 / d[2] + (double)sn, pp, L.pz,
                                s->stream);
        L.bb_cur ^= 1;
        s->tock(ev, BF_PHASE_IONS);
        ev = s->tick();
        if (s->have_laser) {
            const double za = s->za_lab / s->gamma - s->beta * s->t - (double)s->shift * d[2];
            const double zb = s->za_lab / s->gamma - s->beta * t1 - (double)s->shift * d[2];
            if (za >= 0.0 && za < L.g.N[2] * d[2]) {
                bf3::Antenna3 a;
                a.n = L.na;
                a.za = za / d[2];
                a.zb = zb / d[2];
                a.tm = s->t + 0.5 * s->dt;
                a.e0g = s->e0 / s->gamma;
                a.w0 = s->w0;
                a.xc = 0.5 * L.g.N[0] * d[0];
                a.yc = 0.5 * L.g.N[1] * d[1];
                a.gamma = s->gamma;
                a.t0 = s->t0;
                a.sig_t = s->sig_t;
                a.omega = s->omega;
                a.aw = s->aw;
                a.pol = s->pol;
                double* ant = w3<double>(s, L.w_ant);
                const size_t na = (size_t)L.na;
                bf3::launch3_antenna<R>(g, f, ant, ant + na, ant + 2 * na, a, pp, s->stream);
            }
        }
        s->tock(ev, BF_PHASE_ANTENNA);
        ev = s->tick();
        const R* jout[3];
        bf3::FiltSeq fs;
        bf3::filter_seq(s->cfg.filter_npass, s->cfg.filter_compensate, s->cfg.filter_strides, &fs);
        bf3::launch3_filter<R>(g, f, fs, jout, s->stream);
        s->tock(ev, BF_PHASE_FILTER);
        ev = s->tick();
        bf3::launch3_ampere<R>(g, f, jout, pml, s->dt, s->stream);
        s->tock(ev, BF_PHASE_AMPERE);
        ev = s->tick();
        s->step++;
        s->t = (double)s->step * s->dt;
        if (dsh != 0) {
            int z = (L.g.zoff + dsh) % L.g.S[2];
            if (z < 0) z += L.g.S[2];
            L.g.zoff = z;
            s->shift = sn;
            bf3::launch3_window<R>(L.g, f, pml, dsh, s->stream);
        }
        hipError_t e = inject3<R>(s, rows_entering(s));
        s->tock(ev, BF_PHASE_WINDOW);
        if (e != hipSuccess) return hip_check(s, e, "3D injection");
        if (++L.since_sort >= s->sort_every) {
            ev = s->tick();
            sort3<R>(s);
            s->tock(ev, BF_PHASE_SORT);
        }
    }
    return hip_check(s, hipGetLastError(), "3D step launch");
}

bf_status init_plasma3(bf_sim* s)
{
    hipError_t e = s->cfg.real_bytes == 4 ? inject3<float>(s, rows_entering(s)) : inject3<double>(s, rows_entering(s));
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    return hip_check(s, e, "3D init_plasma");
}

bf_status init_laser3(bf_sim* s)
{
    Sim3& L = *s->d3;
    L.na = L.g.N[0] * L.g.N[1];
    s->aw = (2.0 * s->e0 / s->gamma) * s->cfg.dx_um * s->cfg.dy_um / 0.01;
    std::vector<double> a(3 * (size_t)L.na);
    for (int q = 0; q < L.na; q++) {
        a[L.na + q] = (q % L.g.N[0]) + 0.5;                 // home x
        a[2 * (size_t)L.na + q] = (q / L.g.N[0]) + 0.5;     // home y
        a[q] = a[(size_t)(1 + s->pol) * L.na + q];           // moving coordinate along pol
    }
    return hip_check(s, hipMemcpy(w3<double>(s, L.w_ant), a.data(), a.size() * 8, hipMemcpyHostToDevice),
                     "3D init_laser");
}

// field id -> array (-1: none)
int array3_of(const Sim3& L, int id)
{
    switch (id) {
    case BF_F_EX: case BF_F_EY: case BF_F_EZ: return A3_E + (id - BF_F_EX);
    case BF_F_EXO: case BF_F_EYO: case BF_F_EZO: return A3_EO + (id - BF_F_EXO);
    case BF_F_EXB: case BF_F_EYB: case BF_F_EZB: return (L.eb_cur ? A3_T : A3_EB) + (id - BF_F_EXB);
    case BF_F_BX: case BF_F_BY: case BF_F_BZ: return A3_B + (id - BF_F_BX);
    case BF_F_BXO: case BF_F_BYO: case BF_F_BZO: return A3_BO + (id - BF_F_BXO);
    case BF_F_JXR: case BF_F_JYR: case BF_F_JZR: return A3_J + (id - BF_F_JXR);
    case BF_F_EXS: case BF_F_EYS: case BF_F_EZS: return A3_SE + (id - BF_F_EXS);
    case BF_F_BXS: case BF_F_BYS: case BF_F_BZS: return A3_SB + (id - BF_F_BXS);
    default: return -1;
    }
}

// the filtered current ends in Jf (x pass into Jf, y into Jg, z back into Jf; a copy into Jf
// without passes)
int filtered3(const bf_config&, int comp) { return A3_JF + comp; }

bf_status read_field3(bf_sim* s, int a, double* out)
{
    const Sim3& L = *s->d3;
    const bool acc = a >= A3_J;
    const size_t bytes = acc ? L.fa8 : L.fa;
    std::vector<char> raw(bytes);
    const char* src = acc ? (const char*)jacc3(s, a - A3_J) : (const char*)s->buf[0] + L.fa * a;
    hipError_t e = hipMemcpy(raw.data(), src, bytes, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_check(s, e, "3D read field");
    const bool f32 = s->cfg.real_bytes == 4 && !acc;
    for (int k = 0; k < L.g.S[2]; k++) {
        const int pk = (k + L.g.zoff) % L.g.S[2];
        for (int j = 0; j < L.g.S[1]; j++)
            for (int i = 0; i < L.g.S[0]; i++) {
                const size_t o = (size_t)pk * L.g.plane + (size_t)j * L.g.pitch + i;
                out[((size_t)k * L.g.S[1] + j) * L.g.S[0] + i] =
                    f32 ? (double)((float*)raw.data())[o] : ((double*)raw.data())[o];
            }
    }
    return BF_OK;
}

bf_status write_field3(bf_sim* s, int a, const double* in)
{
    const Sim3& L = *s->d3;
    const bool acc = a >= A3_J;
    const size_t bytes = acc ? L.fa8 : L.fa;
    std::vector<char> raw(bytes, 0);
    const bool f32 = s->cfg.real_bytes == 4 && !acc;
    for (int k = 0; k < L.g.S[2]; k++) {
        const int pk = (k + L.g.zoff) % L.g.S[2];
        for (int j = 0; j < L.g.S[1]; j++)
            for (int i = 0; i < L.g.S[0]; i++) {
                const size_t o = (size_t)pk * L.g.plane + (size_t)j * L.g.pitch + i;
                const double v = in[((size_t)k * L.g.S[1] + j) * L.g.S[0] + i];
                if (f32) ((float*)raw.data())[o] = (float)v;
                else ((double*)raw.data())[o] = v;
            }
    }
    char* dst = acc ? (char*)jacc3(s, a - A3_J) : (char*)s->buf[0] + L.fa * a;
    return hip_check(s, hipMemcpy(dst, raw.data(), bytes, hipMemcpyHostToDevice), "3D write field");
}

// live particles: 8 columns (id, x, y, z in um, ux, uy, uz, w)
// live particles of slots [first, first + count) of a species (count < 0: up to the slots in use)
bf_status read_particles3(bf_sim* s, int species, std::vector<double>* cols, int64_t* nlive, int64_t first = 0,
                          int64_t count = -1)
{
    const Sim3& L = *s->d3;
    int64_t used = 0;
    hipError_t e0 = slots3(s, species, &used);
    if (e0 != hipSuccess) return hip_check(s, e0, "3D read particles");
    first = std::min(std::max<int64_t>(first, 0), used);
    const int64_t n = count < 0 ? used - first : std::min(count, used - first);
    const bool f32 = s->cfg.real_bytes == 4;
    const size_t rb = s->cfg.real_bytes;
    const char* b = (const char*)s->buf[(species == 0 ? 1 : 3) + L.p_cur];
    const int ncol = species == 0 ? 8 : 5;
    std::vector<std::vector<char>> raw(ncol);
    for (int q = 0; q < ncol; q++) {
        const size_t off = species == 0 ? L.e_off[q] : L.i_off[q];
        const size_t sz = q < 3 ? 8 : (q == ncol - 1 ? 4 : rb);
        raw[q].resize(std::max<int64_t>(n, 1) * sz);
        if (n > 0) {
            hipError_t e = hipMemcpy(raw[q].data(), b + off + first * sz, n * sz, hipMemcpyDeviceToHost);
            if (e != hipSuccess) return hip_check(s, e, "3D read particles");
        }
    }
    auto rv = [&](int q, int64_t p) { return f32 ? (double)((float*)raw[q].data())[p] : ((double*)raw[q].data())[p]; };
    for (int q = 0; q < 8; q++) cols[q].clear();
    const double d[3] = {s->cfg.dx_um, s->cfg.dy_um, s->cfg.dz_um};
    for (int64_t p = 0; p < n; p++) {
        const double w = species == 0 ? rv(6, p) : rv(3, p);
        if (w == 0.0) continue;
        const double* xyz = (const double*)raw[0].data();
        const double x = xyz[p] * d[0], y = ((const double*)raw[1].data())[p] * d[1];
        double z = ((const double*)raw[2].data())[p];
        if (species == 1) z = z - (s->beta * s->t / d[2] + (double)s->shift);
        cols[0].push_back((double)((const uint32_t*)raw[ncol - 1].data())[p]);
        cols[1].push_back(x);
        cols[2].push_back(y);
        cols[3].push_back(z * d[2]);
        cols[4].push_back(species == 0 ? rv(3, p) : 0.0);
        cols[5].push_back(species == 0 ? rv(4, p) : 0.0);
        cols[6].push_back(species == 0 ? rv(5, p) : -s->gamma * s->beta);
        cols[7].push_back(w);
    }
    *nlive = (int64_t)cols[0].size();
    return BF_OK;
}

// div E - F[rho] on the nodes (Sec. 4.2.2: the charge-conserving deposit keeps it constant), rho
// from the particles with the deposit's cubic shape, filtered like the current.  The FP64 current
// accumulators serve as scratch: the raw current of the last step is gone afterwards.
template <typename R>
bf_status gauss3_impl(bf_sim* s, double* out)
{
    const Sim3& L = *s->d3;
    const double d[3] = {s->cfg.dx_um, s->cfg.dy_um, s->cfg.dz_um};
    int64_t ne = 0, ni = 0;
    hipError_t e = slots3(s, 0, &ne);
    if (e == hipSuccess) e = slots3(s, 1, &ni);
    if (e != hipSuccess) return hip_check(s, e, "3D gauss");
    if (!(s->have_plasma && s->plasma.ion_mode == 1)) ni = 0;
    double za = 0.0;
    int na = 0;
    if (s->have_laser) {
        za = (s->za_lab / s->gamma - s->beta * s->t) / d[2] - (double)s->shift;
        if (za >= 0.0 && za < L.g.N[2]) na = L.na;
    }
    double* a = jacc3(s, 0);
    bf3::launch3_rho<R>(L.g, electrons3<R>(s, L.p_cur), (int)ne, ions3<R>(s, L.p_cur), (int)ni, zshift3(s, s->t),
                        w3<double>(s, L.w_ant), na, s->pol, za, s->aw, 1.0 / (d[0] * d[1] * d[2]), a, s->stream);
    bf3::FiltSeq fs;
    bf3::filter_seq(s->cfg.filter_npass, s->cfg.filter_compensate, s->cfg.filter_strides, &fs);
    const double* res = bf3::launch3_filter_nodal(L.g, a, jacc3(s, 1), jacc3(s, 2), fs, s->stream);
    e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_check(s, e, "3D gauss");
    const size_t grid = (size_t)L.g.S[0] * L.g.S[1] * L.g.S[2];
    std::vector<double> rho(grid), E[3];
    bf_status st = read_field3(s, A3_J + (res == a ? 0 : 1), rho.data());
    for (int c = 0; c < 3 && st == BF_OK; c++) {
        E[c].resize(grid);
        st = read_field3(s, A3_E + c, E[c].data());
    }
    if (st != BF_OK) return st;
    const int S0 = L.g.S[0], S1 = L.g.S[1], S2 = L.g.S[2];
    const int Sa[3] = {S0, S1, S2};
    const size_t step[3] = {1, (size_t)S0, (size_t)S0 * S1};
    for (int k = 0; k < S2; k++)
        for (int j = 0; j < S1; j++)
            for (int i = 0; i < S0; i++) {
                const int q[3] = {i, j, k};
                const size_t o = ((size_t)k * S1 + j) * S0 + i;
                double div = 0.0;
                for (int ax = 0; ax < 3; ax++) {
                    // E_ax sits on half nodes along ax: node q lies between stored q - 1 and q
                    int ql = q[ax] - 1;
                    if (L.g.per[ax]) ql = (ql + Sa[ax]) % Sa[ax];
                    const double el = ql >= 0 ? E[ax][o - (size_t)q[ax] * step[ax] + (size_t)ql * step[ax]] : 0.0;
                    div += (E[ax][o] - el) / d[ax];
                }
                out[o] = div - rho[o];
            }
    return BF_OK;
}

bf_status diagnose3(bf_sim* s, int kind, int arg, void* host_out, size_t bytes)
{
    const Sim3& L = *s->d3;
    const size_t grid = (size_t)L.g.S[0] * L.g.S[1] * L.g.S[2];
    switch (kind) {
    case BF_DIAG_FIELD: {
        int a = (arg == BF_F_JX || arg == BF_F_JY || arg == BF_F_JZ) ? filtered3(s->cfg, arg - BF_F_JX) : array3_of(*s->d3, arg);
        if (a < 0) return fail(s, BF_EINVAL, "bad field id");
        if (bytes < grid * 8) return fail(s, BF_EINVAL, "buffer too small");
        return read_field3(s, a, (double*)host_out);
    }
    case BF_DIAG_COUNTS: {
        if (bytes < 4 * sizeof(int64_t)) return fail(s, BF_EINVAL, "buffer too small");
        // live particles counted on the device (slots of removed particles hold w = 0)
        int* cnt = w3<int>(s, L.w_cnt);
        int h[2] = {0, 0};
        const bool f32 = s->cfg.real_bytes == 4;
        for (int sp = 0; sp < 2; sp++) {
            int64_t n = 0;
            hipError_t es = slots3(s, sp, &n);
            if (es != hipSuccess) return hip_check(s, es, "3D counts");
            const char* base = (const char*)s->buf[(sp == 0 ? 1 : 3) + L.p_cur] + (sp == 0 ? L.e_off[6] : L.i_off[3]);
            if (f32) bf3::launch3_count_live<float>((const float*)base, (int)n, cnt + sp, s->stream);
            else bf3::launch3_count_live<double>((const double*)base, (int)n, cnt + sp, s->stream);
        }
        hipError_t e = hipMemcpyAsync(h, cnt, sizeof h, hipMemcpyDeviceToHost, s->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
        if (e != hipSuccess) return hip_check(s, e, "3D counts");
        const int64_t ne = h[0], ni = (s->have_plasma && s->plasma.ion_mode == 1) ? h[1] : 0;
        int64_t* o = (int64_t*)host_out;
        int64_t se = 0, si = 0;
        e = slots3(s, 0, &se);
        if (e == hipSuccess) e = slots3(s, 1, &si);
        if (e != hipSuccess) return hip_check(s, e, "3D counts");
        o[0] = ne; o[1] = ni; o[2] = se; o[3] = si;
        return BF_OK;
    }
    case BF_DIAG_PARTICLES: {
        std::vector<double> cols[8];
        int64_t n = 0;
        bf_status st = read_particles3(s, arg, cols, &n);
        if (st != BF_OK) return st;
        if (bytes < (size_t)n * 8 * 8) return fail(s, BF_EINVAL, "buffer too small");
        for (int q = 0; q < 8; q++) std::memcpy((double*)host_out + (size_t)q * n, cols[q].data(), n * 8);
        return BF_OK;
    }
    case BF_DIAG_PARTICLE_BLOCK: {
        if (arg < 0) return fail(s, BF_EINVAL, "bad particle block");
        std::vector<double> cols[8];
        int64_t n = 0;
        bf_status st = read_particles3(s, arg & 1, cols, &n, (int64_t)(arg >> 1) * BF_PARTICLE_BLOCK,
                                       BF_PARTICLE_BLOCK);
        if (st != BF_OK) return st;
        if (bytes < 8 + (size_t)n * 8 * 8) return fail(s, BF_EINVAL, "buffer too small");
        *(int64_t*)host_out = n;
        for (int q = 0; q < 8; q++) std::memcpy((double*)host_out + 1 + (size_t)q * n, cols[q].data(), n * 8);
        return BF_OK;
    }
    case BF_DIAG_STATION: {
        if (arg < 0 || arg >= s->nst) return fail(s, BF_EINVAL, "bad station");
        int cnt = 0;
        hipError_t e = hipMemcpy(&cnt, w3<int>(s, L.w_st_cnt) + arg, sizeof(int), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_check(s, e, "station");
        if (bytes < 8 + (size_t)cnt * 7 * 8) return fail(s, BF_EINVAL, "buffer too small");
        *(int64_t*)host_out = cnt;
        if (cnt > 0)
            e = hipMemcpy((char*)host_out + 8, w3<double>(s, L.w_st_rec) + (size_t)arg * L.stcap * 7,
                          (size_t)cnt * 7 * 8, hipMemcpyDeviceToHost);
        return hip_check(s, e, "station");
    }
    case BF_DIAG_ENERGY: {
        if (bytes < 3 * 8) return fail(s, BF_EINVAL, "buffer too small");
        std::vector<double> f(grid);
        double ue = 0, ub = 0;
        for (int q = 0; q < 6; q++) {
            bf_status st = read_field3(s, q < 3 ? A3_E + q : A3_B + q - 3, f.data());
            if (st != BF_OK) return st;
            double acc = 0;
            for (double v : f) acc += v * v;
            (q < 3 ? ue : ub) += acc;
        }
        std::vector<double> cols[8];
        int64_t n = 0;
        bf_status st = read_particles3(s, 0, cols, &n);
        if (st != BF_OK) return st;
        double k = 0;
        for (int64_t p = 0; p < n; p++) {
            const double ux = cols[4][p], uy = cols[5][p], uz = cols[6][p];
            k += cols[7][p] * (std::sqrt(1.0 + ux * ux + uy * uy + uz * uz) - 1.0);
        }
        const double dv = s->cfg.dx_um * s->cfg.dy_um * s->cfg.dz_um;
        double* o = (double*)host_out;
        o[0] = 0.5 * ue * dv; o[1] = 0.5 * ub * dv; o[2] = k;
        return BF_OK;
    }
    case BF_DIAG_INFO: {
        if (bytes < sizeof(bf_info)) return fail(s, BF_EINVAL, "buffer too small");
        bf_info* o = (bf_info*)host_out;
        std::memset(o, 0, sizeof *o);
        o->dt = s->dt; o->dt_crit = s->dt_crit; o->beta = s->beta; o->gamma = s->gamma;
        o->v_window = s->vw; o->n0_norm = s->n0; o->e0_norm = s->e0; o->omega = s->omega;
        o->alpha2 = s->cfg.ck_alpha; o->beta2 = s->cfg.ck_beta; o->antenna_weight = s->aw;
        o->stored_x = L.g.S[0]; o->stored_z = L.g.S[2]; o->pml_x = L.g.P[0]; o->pml_z = L.g.P[2];
        o->step = s->step; o->time = s->t; o->shift = s->shift; o->next_row = s->next_row;
        o->sort_every = s->sort_every;
        o->dim = 3; o->stored_y = L.g.S[1]; o->pml_y = L.g.P[1];
        return BF_OK;
    }
    case BF_DIAG_ANTENNA: {
        if (!s->have_laser) return fail(s, BF_EINVAL, "no laser");
        if (bytes < (size_t)L.na * 8) return fail(s, BF_EINVAL, "buffer too small");
        std::vector<double> xm(L.na);
        hipError_t e = hipMemcpy(xm.data(), w3<double>(s, L.w_ant), xm.size() * 8, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_check(s, e, "antenna");
        const double dm = s->pol == 0 ? s->cfg.dx_um : s->cfg.dy_um;
        for (int q = 0; q < L.na; q++) ((double*)host_out)[q] = xm[q] * dm;
        return BF_OK;
    }
    case BF_DIAG_GAUSS: {
        if (bytes < grid * 8) return fail(s, BF_EINVAL, "buffer too small");
        return s->cfg.real_bytes == 4 ? gauss3_impl<float>(s, (double*)host_out)
                                      : gauss3_impl<double>(s, (double*)host_out);
    }
    default:
        return fail(s, BF_EUNSUPPORTED, "diagnostic not available in 3D");
    }
}

}  // namespace

extern "C" {

const char* bf_status_string(bf_status s)
{
    switch (s) {
    case BF_OK: return "ok";
    case BF_EINVAL: return "invalid argument";
    case BF_ECFL: return "time step above the CFL limit";
    case BF_ECAPACITY: return "particle capacity exceeded";
    case BF_ENONFINITE: return "non-finite particle momentum";
    case BF_EDEVICE: return "HIP runtime error";
    case BF_ESTATE: return "call not allowed in this state";
    case BF_EUNSUPPORTED: return "unsupported configuration";
    }
    return "unknown status";
}

const char* bf_last_error(const bf_sim* s) { return s ? s->msg.c_str() : "null handle"; }

bf_status bf_query_buffers(const bf_config* cfg, bf_buffer_desc* out, int* n_inout)
{
    if (!n_inout) return BF_EINVAL;
    const bf_status v = validate(cfg);
    if (v != BF_OK) return v;
    size_t sizes[6];
    if (cfg->dim == 3) {
        Sim3 L3;
        layout3(cfg, &L3);
        sizes3(L3, sizes);
    } else {
        Layout L;
        layout_of(cfg, &L);
        const size_t s2[6] = {L.fields_bytes, L.e_bytes, L.e_bytes, L.i_bytes, L.i_bytes, L.w_bytes};
        for (int k = 0; k < 6; k++) sizes[k] = s2[k];
    }
    const int cap = *n_inout;
    *n_inout = 6;
    if (!out) return BF_OK;
    if (cap < 6) return BF_EINVAL;
    for (int k = 0; k < 6; k++) {
        out[k].name = kNames[k];
        out[k].bytes = sizes[k];
        out[k].align = 256;
        out[k].dtype = 0;
    }
    return BF_OK;
}

bf_status bf_create(const bf_config* cfg, const bf_buffer_binding* b, int n, void* stream, bf_sim** out)
{
    if (!out) return BF_EINVAL;
    *out = nullptr;
    const bf_status v = validate(cfg);
    if (v != BF_OK) return v;
    if (cfg->dim == 3) return create3(cfg, b, n, stream, out);
    bf_sim* s = new bf_sim();
    s->cfg = *cfg;
    layout_of(cfg, &s->L);
    const size_t sizes[6] = {s->L.fields_bytes, s->L.e_bytes, s->L.e_bytes, s->L.i_bytes, s->L.i_bytes,
                             s->L.w_bytes};
    for (int k = 0; k < 6; k++) {
        for (int q = 0; q < n; q++)
            if (b[q].name && std::strcmp(b[q].name, kNames[k]) == 0) {
                if (b[q].bytes < sizes[k] || !b[q].ptr || ((uintptr_t)b[q].ptr & 255u)) {
                    delete s;
                    return BF_EINVAL;
                }
                s->buf[k] = b[q].ptr;
            }
        if (!s->buf[k]) { delete s; return BF_EINVAL; }
    }
    s->stream = (hipStream_t)stream;
    s->gamma = cfg->gamma_boost;
    s->beta = std::sqrt(1.0 - 1.0 / (s->gamma * s->gamma));
    s->a2 = cfg->ck_alpha + 2.0 * cfg->ck_beta;   // 2D: k_y = 0 folds the y neighbours
    s->b2 = cfg->ck_beta + 2.0 * cfg->ck_gamma;
    s->theta = cfg->friedman_theta;
    s->dt_crit = cfl2d(cfg->ck_alpha, cfg->ck_beta, cfg->ck_gamma, cfg->dx_um, cfg->dz_um, s->theta);
    s->dt = cfg->cfl_fraction * s->dt_crit;
    s->sort_every = cfg->sort_every > 0 ? cfg->sort_every : 20;
    s->g = geo_of(s, 0);
    update_window_speed(s);
    hipError_t e = hipSuccess;
    for (int k = 0; k < 6; k++) {
        const size_t sz = k == 0 ? s->L.fields_bytes : (k == 5 ? s->L.w_bytes : (k < 3 ? s->L.e_bytes : s->L.i_bytes));
        if (e == hipSuccess) e = hipMemsetAsync(s->buf[k], 0, sz, s->stream);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) { delete s; return BF_EDEVICE; }
    e = cfg->real_bytes == 4 ? upload_pml<float>(s) : upload_pml<double>(s);
    if (e != hipSuccess) { delete s; return BF_EDEVICE; }
    // empty segment tables: all tiles empty
    *out = s;
    return BF_OK;
}

void bf_destroy(bf_sim* s) { delete s; }

static bf_status guard(bf_sim* s)
{
    if (!s) return BF_EINVAL;
    if (s->err != BF_OK) return fail(s, BF_ESTATE, "handle is in an error state");
    return BF_OK;
}

bf_status bf_init_plasma(bf_sim* s, const bf_plasma* p)
{
    bf_status st = guard(s);
    if (st != BF_OK) return st;
    if (!p || p->ppc <= 0 || p->ppc > 1024 || p->n0_cm3 < 0 || (p->ion_mode != 0 && p->ion_mode != 1))
        return fail(s, BF_EINVAL, "bad plasma");
    if (s->have_plasma) return fail(s, BF_ESTATE, "plasma already loaded");
    s->plasma = *p;
    const double nu = EPS0 * ME_KG * C_LIGHT * C_LIGHT / (Q_E * Q_E * 1e-12);   // m^-3
    s->n0 = p->n0_cm3 * 1e6 / nu;
    s->have_plasma = 1;
    s->next_row = 0;
    update_window_speed(s);
    if (s->d3) return init_plasma3(s);
    // initial rows: every lattice row inside the window at the current time
    if (s->cfg.real_bytes == 4) {
        inject<float>(s, rows_entering(s));
        sort_now<float>(s);
    } else {
        inject<double>(s, rows_entering(s));
        sort_now<double>(s);
    }
    return hip_check(s, hipStreamSynchronize(s->stream), "init_plasma");
}

bf_status bf_init_laser(bf_sim* s, const bf_laser* l)
{
    bf_status st = guard(s);
    if (st != BF_OK) return st;
    if (!l || l->lambda_um <= 0 || l->waist_um <= 0 || l->fwhm_fs <= 0) return fail(s, BF_EINVAL, "bad laser");
    if (l->pol < 0 || l->pol > 1) return fail(s, BF_EINVAL, "laser polarisation must be 0 (x) or 1 (y)");
    if (!(l->t_peak_fs >= 0)) return fail(s, BF_EINVAL, "negative laser peak time");
    s->have_laser = 1;
    s->omega = 2.0 * PI / l->lambda_um;
    s->e0 = l->a0 * s->omega;                              // a0 = e E0 / (m c omega)
    s->w0 = l->waist_um;
    s->sig_t = l->fwhm_fs * 1e-15 * C_LIGHT * 1e6 / (2.0 * std::sqrt(std::log(2.0)));
    s->t0 = l->t_peak_fs > 0 ? l->t_peak_fs * 1e-15 * C_LIGHT * 1e6 : 3.0 * s->sig_t;
    s->pol = l->pol;
    s->za_lab = l->z_antenna_um;
    if (s->d3) {
        update_window_speed(s);
        return init_laser3(s);
    }
    s->aw = (2.0 * s->e0 / s->gamma) * s->cfg.dx_um / 0.01;  // |v| of the moving sheet <= 0.01 c
    std::vector<double> xm(s->cfg.nx);
    for (int i = 0; i < s->cfg.nx; i++) xm[i] = i + 0.5;
    update_window_speed(s);
    return hip_check(s, hipMemcpy(s->w<double>(s->L.w_ant), xm.data(), xm.size() * 8, hipMemcpyHostToDevice),
                     "init_laser");
}

bf_status bf_add_station(bf_sim* s, const bf_station* st_, int* id)
{
    bf_status st = guard(s);
    if (st != BF_OK) return st;
    const int nmax = s->d3 ? s->d3->nst_max : s->L.nst;
    if (!st_ || s->nst >= nmax) return fail(s, BF_EINVAL, "no station slot left");
    s->st_z.push_back(st_->z_lab_um);
    double* dz = s->d3 ? w3<double>(s, s->d3->w_st_z) : s->w<double>(s->L.w_st_z);
    hipError_t e = hipMemcpy(dz, s->st_z.data(), s->st_z.size() * 8, hipMemcpyHostToDevice);
    if (id) *id = s->nst;
    s->nst++;
    return hip_check(s, e, "add_station");
}

bf_status bf_load_electrons(bf_sim* s, int64_t n, const uint32_t* id, const double* x, const double* z,
                            const double* ux, const double* uy, const double* uz, const double* w)
{
    bf_status st = guard(s);
    if (st != BF_OK) return st;
    if (s->d3) return fail(s, BF_EINVAL, "3D runs load electrons with bf_load_electrons3");
    if (n < 0 || n > s->L.cap || (n > 0 && (!x || !z || !ux || !uy || !uz || !w)))
        return fail(s, BF_EINVAL, "bad particle arrays");
    const bool f32 = s->cfg.real_bytes == 4;
    std::vector<double> hx(n), hz(n);
    std::vector<float> f[4];
    std::vector<double> d[4];
    std::vector<uint32_t> hid(n);
    const double* src[4] = {ux, uy, uz, w};
    for (int q = 0; q < 4; q++) { if (f32) f[q].resize(n); else d[q].resize(n); }
    for (int64_t p = 0; p < n; p++) {
        hx[p] = x[p] / s->cfg.dx_um;
        hz[p] = z[p] / s->cfg.dz_um;
        for (int q = 0; q < 4; q++) { if (f32) f[q][p] = (float)src[q][p]; else d[q][p] = src[q][p]; }
        hid[p] = id ? id[p] : (uint32_t)p;
    }
    char* b = (char*)s->buf[1 + s->p_cur];
    hipError_t e = hipSuccess;
    const size_t rb = s->cfg.real_bytes;
    if (n > 0) {
        e = hipMemcpy(b + s->L.e_off[0], hx.data(), n * 8, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(b + s->L.e_off[1], hz.data(), n * 8, hipMemcpyHostToDevice);
        for (int q = 0; q < 4 && e == hipSuccess; q++)
            e = hipMemcpy(b + s->L.e_off[2 + q], f32 ? (void*)f[q].data() : (void*)d[q].data(), n * rb,
                          hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(b + s->L.e_off[6], hid.data(), n * 4, hipMemcpyHostToDevice);
    }
    // one segment per 1024 particles, then a sort into tiles
    std::vector<Segment> sg;
    for (int64_t p = 0; p < n; p += 1024) sg.push_back(Segment{(int)p, (int)std::min<int64_t>(1024, n - p)});
    if (e == hipSuccess && !sg.empty())
        e = hipMemcpy(seg_e(s, s->sg_cur), sg.data(), sg.size() * sizeof(Segment), hipMemcpyHostToDevice);
    int nu = (int)n;
    if (e == hipSuccess) e = hipMemcpy(nused_e(s), &nu, sizeof(int), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_check(s, e, "load_electrons");
    if ((int)sg.size() > s->L.seg_cap) return fail(s, BF_EINVAL, "too many particles for the segment table");
    s->nseg_e = (int)sg.size();
    if (f32) sort_now<float>(s); else sort_now<double>(s);
    return hip_check(s, hipStreamSynchronize(s->stream), "load_electrons");
}

bf_status bf_load_electrons3(bf_sim* s, int64_t n, const uint32_t* id, const double* x, const double* y,
                             const double* z, const double* ux, const double* uy, const double* uz, const double* w)
{
    bf_status st = guard(s);
    if (st != BF_OK) return st;
    if (!s->d3) return fail(s, BF_EINVAL, "2D runs load electrons with bf_load_electrons");
    Sim3& L = *s->d3;
    if (n < 0 || n > L.cap || (n > 0 && (!x || !y || !z || !ux || !uy || !uz || !w)))
        return fail(s, BF_EINVAL, "bad particle arrays");
    const bool f32 = s->cfg.real_bytes == 4;
    const size_t rb = s->cfg.real_bytes;
    const double d[3] = {s->cfg.dx_um, s->cfg.dy_um, s->cfg.dz_um};
    const double* pos[3] = {x, y, z};
    const double* mom[4] = {ux, uy, uz, w};
    char* b = (char*)s->buf[1 + L.p_cur];
    hipError_t e = hipSuccess;
    std::vector<double> h(n);
    for (int a = 0; a < 3 && e == hipSuccess; a++) {
        for (int64_t p = 0; p < n; p++) h[p] = pos[a][p] / d[a];
        if (n > 0) e = hipMemcpy(b + L.e_off[a], h.data(), n * 8, hipMemcpyHostToDevice);
    }
    std::vector<float> hf(n);
    for (int q = 0; q < 4 && e == hipSuccess; q++) {
        if (n == 0) break;
        if (f32) {
            for (int64_t p = 0; p < n; p++) hf[p] = (float)mom[q][p];
            e = hipMemcpy(b + L.e_off[3 + q], hf.data(), n * rb, hipMemcpyHostToDevice);
        } else {
            e = hipMemcpy(b + L.e_off[3 + q], mom[q], n * rb, hipMemcpyHostToDevice);
        }
    }
    std::vector<uint32_t> hid(n);
    for (int64_t p = 0; p < n; p++) hid[p] = id ? id[p] : (uint32_t)p;
    if (e == hipSuccess && n > 0) e = hipMemcpy(b + L.e_off[7], hid.data(), n * 4, hipMemcpyHostToDevice);
    const int nu = (int)n;
    if (e == hipSuccess) e = hipMemcpy(w3<int>(s, L.w_nused), &nu, sizeof nu, hipMemcpyHostToDevice);
    // bin the loaded particles (and any plasma) by tile
    if (e == hipSuccess) {
        if (f32) sort3<float>(s); else sort3<double>(s);
        e = hipStreamSynchronize(s->stream);
    }
    return hip_check(s, e, "load_electrons3");
}

// Sec. 3.1.1: (1) ballistic projection onto the plane, t* = (z - z_inj)/v_z, x* = x - v_x t*;
// (2) the crossing event (t = -t*, z = z_inj) and the momentum in the calculation frame,
// t'* = gamma (-t* - beta z_inj), z'* = gamma (z_inj + beta t*), u'_z = gamma (u_z - beta gamma_p),
// u'_perp = u_perp; (3) the synchronised position z'(0) = z'* - vbar' t'*, advanced to the
// current time at vbar' since the beam is frozen until it crosses.
bf_status bf_add_beam(bf_sim* s, const bf_beam* bm, int64_t n, const double* x, const double* z, const double* ux,
                      const double* uy, const double* uz, const double* w)
{
    bf_status st = guard(s);
    if (st != BF_OK) return st;
    if (s->d3) return fail(s, BF_EUNSUPPORTED, "the beam is available in 2D runs");
    if (!bm || n < 0 || n > s->cfg.beam_capacity || (n > 0 && (!x || !z || !ux || !uy || !uz || !w)))
        return fail(s, BF_EINVAL, "bad beam arrays or n above beam_capacity");
    if (!(bm->beta_b > 0.0 && bm->beta_b < 1.0) || !std::isfinite(bm->z_inj_um))
        return fail(s, BF_EINVAL, "beta_b must lie in (0, 1)");
    const double g = s->gamma, b = s->beta, zi = bm->z_inj_um;
    const double vbar = (bm->beta_b - b) / (1.0 - b * bm->beta_b);
    const double dx = s->cfg.dx_um, dz = s->cfg.dz_um;
    const int perx = s->cfg.periodic_mask & 1, perz = (s->cfg.periodic_mask >> 2) & 1;
    std::vector<double> col[7];
    for (auto& v : col) v.resize((size_t)n);
    for (int64_t p = 0; p < n; p++) {
        const double vals[6] = {x[p], z[p], ux[p], uy[p], uz[p], w[p]};
        for (double v : vals)
            if (!std::isfinite(v)) return fail(s, BF_EINVAL, "non-finite beam value");
        if (!(uz[p] > 0.0)) return fail(s, BF_EINVAL, "every beam particle must move forward (uz > 0)");
        const double gp = std::sqrt(1.0 + ux[p] * ux[p] + uy[p] * uy[p] + uz[p] * uz[p]);
        const double tstar = (z[p] - zi) * gp / uz[p];
        const double xstar = x[p] - ux[p] / gp * tstar;
        const double tcross = g * (-tstar - b * zi);
        const double zcross = g * (zi + b * tstar);
        double xc = xstar / dx;
        double zc = (zcross - vbar * tcross + vbar * s->t) / dz - (double)s->shift;
        if (perx) xc -= s->cfg.nx * std::floor(xc / s->cfg.nx);
        if (perz) zc -= s->cfg.nz * std::floor(zc / s->cfg.nz);
        col[0][p] = xc;
        col[1][p] = zc;
        col[2][p] = ux[p];
        col[3][p] = uy[p];
        col[4][p] = g * (uz[p] - b * gp);
        col[5][p] = w[p];
        col[6][p] = tcross;
    }
    const Layout& L = s->L;
    hipError_t e = hipStreamSynchronize(s->stream);   // earlier steps may still use the arrays
    for (int k = 0; k < 7 && e == hipSuccess && n > 0; k++)
        e = hipMemcpy(s->w<double>(L.w_beam[k]), col[k].data(), 8 * (size_t)n, hipMemcpyHostToDevice);
    if (e == hipSuccess && n > 0) e = hipMemset(s->w<int>(L.w_beam[7]), 0, 4 * (size_t)n);
    if (e == hipSuccess && s->cfg.beam_history > 0)
        e = hipMemset(s->w<double>(L.w_bhist), 0, 64 * (size_t)s->cfg.beam_history);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_check(s, e, "add_beam");
    s->have_beam = 1;
    s->beam_test = bm->test_only ? 1 : 0;
    s->nbeam = n;
    s->beam_rec = 0;
    s->vbar = vbar;
    return BF_OK;
}

bf_status bf_step(bf_sim* s, int nsteps)
{
    bf_status st = guard(s);
    if (st != BF_OK) return st;
    if (nsteps < 0) return fail(s, BF_EINVAL, "negative step count");
    if (s->cfg.filter_kind == BF_FILTER_LEARNED && !s->have_lf)
        return fail(s, BF_ESTATE, "learned filter selected but its parameters are not loaded");
    if (s->d3) return s->cfg.real_bytes == 4 ? step3<float>(s, nsteps) : step3<double>(s, nsteps);
    if (s->cfg.real_bytes == 4) st = step_impl<float>(s, nsteps);
    else st = step_impl<double>(s, nsteps);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_check(s, e, "step launch");
    return st;
}

// ---- batched runs ----------------------------------------------------------------------------

}  // extern "C"

namespace {

constexpr int BATCH_RING = 4;   // descriptor tables in flight
constexpr int BATCH_LANES = 4;  // streams the runs' own launches are spread over

size_t al256(size_t v) { return (v + 255) / 256 * 256; }

// bytes of one descriptor table for n runs: counters, then per batched phase its
// descriptors and its item offsets
size_t batch_table_bytes(int n)
{
    const size_t m = (size_t)n;
    return 256 + al256(m * sizeof(FaradayDesc<float>)) + al256((m + 1) * 4) +
           al256(m * sizeof(AmpereDesc<float>)) + al256((m + 1) * 4) +
           al256(m * sizeof(GpdDesc<float>)) + al256((m + 1) * 4);
}

}  // namespace

struct bf_batch {
    std::vector<bf_sim*> sims;
    hipStream_t stream = nullptr;
    unsigned char* dev = nullptr;
    size_t table = 0;
    unsigned char* host[BATCH_RING] = {};
    hipEvent_t ev[BATCH_RING] = {};
    bool used[BATCH_RING] = {};
    hipEvent_t join = nullptr;
    // the runs' own launches between two batched launches go to BATCH_LANES lanes (the batch
    // stream and side streams at the default priority), run r on lane r % BATCH_LANES
    hipStream_t side[BATCH_LANES - 1] = {};
    hipEvent_t fork = nullptr, lane_done[BATCH_LANES - 1] = {};
    int ring = 0, cus = 256;
    BatchRec rec;
    ~bf_batch()
    {
        for (int r = 0; r < BATCH_RING; r++) {
            if (host[r]) (void)hipHostFree(host[r]);
            if (ev[r]) (void)hipEventDestroy(ev[r]);
        }
        if (join) (void)hipEventDestroy(join);
        if (fork) (void)hipEventDestroy(fork);
        for (int k = 0; k < BATCH_LANES - 1; k++) {
            if (lane_done[k]) (void)hipEventDestroy(lane_done[k]);
            if (side[k]) (void)hipStreamDestroy(side[k]);
        }
    }
};

namespace {

// copies one phase's descriptors and item offsets into the staging table; returns the queue
// as seen from the device
template <typename D>
QueueRef stage_phase(unsigned char* H, unsigned char* Dv, size_t& o, const std::vector<D>& descs,
                     const std::vector<int>& items, int* counter_dev, const D** dev_descs)
{
    const size_t n = descs.size();
    std::memcpy(H + o, descs.data(), n * sizeof(D));
    *dev_descs = reinterpret_cast<const D*>(Dv + o);
    o = al256(o + n * sizeof(D));
    int* off = reinterpret_cast<int*>(H + o);
    int total = 0;
    for (size_t r = 0; r < n; r++) { off[r] = total; total += items[r]; }
    off[n] = total;
    QueueRef q{reinterpret_cast<const int*>(Dv + o), (int)n, total, counter_dev};
    o = al256(o + (n + 1) * 4);
    return q;
}

bf_status batch_one_step(bf_batch* b)
{
    BatchRec& rec = b->rec;
    rec.clear();
    for (size_t q = 0; q < b->sims.size(); q++) {
        bf_sim* s = b->sims[q];
        s->rec = &rec;
        s->rec_run = (int)q;
        const bf_status st = step_impl<float>(s, 1);
        s->rec = nullptr;
        if (st != BF_OK) return st;
    }
    const int r = b->ring;
    b->ring = (b->ring + 1) % BATCH_RING;
    if (b->used[r] && hipEventSynchronize(b->ev[r]) != hipSuccess) return BF_EDEVICE;
    unsigned char* H = b->host[r];
    unsigned char* Dv = b->dev + (size_t)r * b->table;
    std::memset(H, 0, 256);
    int* cnt = reinterpret_cast<int*>(Dv);
    size_t o = 256;
    const FaradayDesc<float>* dfar;
    const AmpereDesc<float>* damp;
    const GpdDesc<float>* dgpd;
    const QueueRef qf = stage_phase(H, Dv, o, rec.faraday, rec.n_faraday, cnt + 0, &dfar);
    const QueueRef qa = stage_phase(H, Dv, o, rec.ampere, rec.n_ampere, cnt + 1, &damp);
    const QueueRef qg = stage_phase(H, Dv, o, rec.gpd, rec.n_gpd, cnt + 2, &dgpd);
    hipStream_t st = b->stream;
    if (hipMemcpyAsync(Dv, H, o, hipMemcpyHostToDevice, st) != hipSuccess) return BF_EDEVICE;
    auto grid = [&](const QueueRef& q, int per_cu) { return std::max(1, std::min(q.total, per_cu * b->cus)); };
    // the runs' own launches of consecutive slots, run r on lane r % BATCH_LANES: the lanes
    // start after the batch stream's last launch and the batch stream waits for all of them,
    // so each run's launches keep their order and the runs overlap one another
    bool ok = true;
    auto closures = [&](std::initializer_list<int> slots) {
        size_t n = 0;
        for (int sl : slots) n += rec.slots[sl].size();
        if (n == 0) return;
        ok = ok && hipEventRecord(b->fork, st) == hipSuccess;
        for (int k = 0; k < BATCH_LANES - 1; k++) ok = ok && hipStreamWaitEvent(b->side[k], b->fork, 0) == hipSuccess;
        for (int sl : slots)
            for (auto& rf : rec.slots[sl]) {
                const int lane = rf.first % BATCH_LANES;
                rf.second(lane == 0 ? st : b->side[lane - 1]);
            }
        for (int k = 0; k < BATCH_LANES - 1; k++) {
            ok = ok && hipEventRecord(b->lane_done[k], b->side[k]) == hipSuccess;
            ok = ok && hipStreamWaitEvent(st, b->lane_done[k], 0) == hipSuccess;
        }
    };
    launch_faraday_batch<float>(dfar, qf, grid(qf, 8), st);
    closures({SLOT_FARADAY, SLOT_STATIONS});
    launch_gpd_batch<float>(dgpd, qg, grid(qg, 3), st);
    closures({SLOT_PUSH, SLOT_IONS, SLOT_ANTENNA, SLOT_FILTER});
    launch_ampere_batch<float>(damp, qa, grid(qa, 8), st);
    closures({SLOT_AMPERE, SLOT_WINDOW, SLOT_SORT});
    if (!ok) return BF_EDEVICE;
    if (hipEventRecord(b->ev[r], st) != hipSuccess) return BF_EDEVICE;
    b->used[r] = true;
    return hipGetLastError() == hipSuccess ? BF_OK : BF_EDEVICE;
}

}  // namespace

extern "C" {

int64_t bf_batch_work_bytes(int nsims)
{
    if (nsims < 1 || nsims > 4096) return -1;
    return (int64_t)(BATCH_RING * batch_table_bytes(nsims));
}

bf_status bf_batch_create(bf_sim* const* sims, int n, void* work, int64_t work_bytes, void* hip_stream,
                          bf_batch** out)
{
    if (!sims || !out || !work || n < 1 || n > 4096) return BF_EINVAL;
    if (work_bytes < bf_batch_work_bytes(n)) return BF_EINVAL;
    for (int q = 0; q < n; q++) {
        if (!sims[q] || sims[q]->cfg.real_bytes != 4 || sims[q]->d3) return BF_EUNSUPPORTED;
        // the batched push runs the energy-conserving gather and Boris; the beam has no batched
        // phase
        if (sims[q]->cfg.gather_kind || sims[q]->cfg.pusher || sims[q]->cfg.beam_capacity > 0)
            return BF_EUNSUPPORTED;
        if (sims[q]->err != BF_OK) return BF_ESTATE;
        for (int p = 0; p < q; p++)
            if (sims[p] == sims[q]) return BF_EINVAL;
    }
    bf_batch* b = new bf_batch();
    b->sims.assign(sims, sims + n);
    b->stream = reinterpret_cast<hipStream_t>(hip_stream);
    b->dev = static_cast<unsigned char*>(work);
    b->table = batch_table_bytes(n);
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
        b->cus = cus;
    bool ok = hipEventCreateWithFlags(&b->join, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) == hipSuccess;
    for (int k = 0; ok && k < BATCH_LANES - 1; k++)
        ok = hipStreamCreateWithFlags(&b->side[k], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&b->lane_done[k], hipEventDisableTiming) == hipSuccess;
    for (int r = 0; ok && r < BATCH_RING; r++) {
        ok = hipHostMalloc(reinterpret_cast<void**>(&b->host[r]), b->table, hipHostMallocDefault) == hipSuccess &&
             hipEventCreateWithFlags(&b->ev[r], hipEventDisableTiming) == hipSuccess;
    }
    if (!ok) { delete b; return BF_EDEVICE; }
    *out = b;
    return BF_OK;
}

bf_status bf_batch_step(bf_batch* b, int nsteps)
{
    if (!b || nsteps < 0) return BF_EINVAL;
    for (bf_sim* s : b->sims) {
        if (s->err != BF_OK) return BF_ESTATE;
        if (s->cfg.filter_kind == BF_FILTER_LEARNED && !s->have_lf) return BF_ESTATE;
        // work already queued on a run's own stream comes first
        if (hipEventRecord(b->join, s->stream) != hipSuccess || hipStreamWaitEvent(b->stream, b->join, 0) != hipSuccess)
            return BF_EDEVICE;
    }
    for (int q = 0; q < nsteps; q++) {
        const bf_status st = batch_one_step(b);
        if (st != BF_OK) return st;
    }
    // later calls on a run's own stream follow the batch
    if (hipEventRecord(b->join, b->stream) != hipSuccess) return BF_EDEVICE;
    for (bf_sim* s : b->sims)
        if (hipStreamWaitEvent(s->stream, b->join, 0) != hipSuccess) return BF_EDEVICE;
    return BF_OK;
}

void bf_batch_destroy(bf_batch* b) { delete b; }

bf_status bf_set_learned_filter(bf_sim* s, const float* host_params, int64_t n)
{
    if (!s || !host_params || n != lf::NPARAM) return BF_EINVAL;
    if (s->cfg.filter_kind != BF_FILTER_LEARNED) return fail(s, BF_ESTATE, "handle uses the bilinear filter");
    float* dev = s->w<float>(s->L.w_lf_par);
    hipError_t e = hipMemcpyAsync(dev, host_params, sizeof(float) * lf::NPARAM, hipMemcpyHostToDevice, s->stream);
    if (e != hipSuccess) return hip_check(s, e, "learned filter parameters");
    lf::pack_forward(dev, lf_packed(s), s->stream);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_check(s, e, "learned filter packing");
    s->have_lf = 1;
    return BF_OK;
}

bf_status bf_sync_status(bf_sim* s)
{
    if (!s) return BF_EINVAL;
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_check(s, e, "sync");
    int word = 0;
    e = hipMemcpy(&word, s->d3 ? w3<int>(s, s->d3->w_status) : status_word(s), sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_check(s, e, "sync");
    if (word & ST_CAPACITY) { s->err = BF_ECAPACITY; s->msg = "particle capacity exceeded"; return BF_ECAPACITY; }
    if (word & ST_NONFINITE) { s->err = BF_ENONFINITE; s->msg = "non-finite particle momentum"; return BF_ENONFINITE; }
    return s->err == BF_OK ? BF_OK : (bf_status)s->err;
}

}  // extern "C"

// ---- diagnostics ----------------------------------------------------------------------------

static void field_ptr_of(const bf_sim* s, int id, int* arr_index)
{
    const int e = s->e_cur, b = s->b_cur, eb = s->eb_cur;
    int a = -1;
    switch (id) {
    case BF_F_EX: case BF_F_EY: case BF_F_EZ: a = (e ? A_E1 : A_E0) + (id - BF_F_EX); break;
    case BF_F_EXO: case BF_F_EYO: case BF_F_EZO: a = (e ? A_E0 : A_E1) + (id - BF_F_EXO); break;
    case BF_F_BX: case BF_F_BY: case BF_F_BZ: a = (b ? A_B1 : A_B0) + (id - BF_F_BX); break;
    case BF_F_BXO: case BF_F_BYO: case BF_F_BZO: a = (b ? A_B0 : A_B1) + (id - BF_F_BXO); break;
    case BF_F_EXB: case BF_F_EYB: case BF_F_EZB: a = (eb ? A_EB1 : A_EB0) + (id - BF_F_EXB); break;
    case BF_F_JX: case BF_F_JY: case BF_F_JZ:
        a = (s->cfg.filter_npass > 0 || s->cfg.filter_kind == BF_FILTER_LEARNED ? A_JF : A_J) + (id - BF_F_JX);
        break;
    case BF_F_JXR: case BF_F_JYR: case BF_F_JZR:
        a = A_J + (id - BF_F_JXR); break;
    case BF_F_BYX: a = A_BYX; break;
    case BF_F_EYX: a = A_EYX; break;
    default: a = -1;
    }
    *arr_index = a;
}

static bf_status read_field(bf_sim* s, int a, double* out)
{
    const Layout& L = s->L;
    std::vector<char> raw(L.field_array);
    hipError_t e = hipMemcpy(raw.data(), s->fields() + L.field_array * a, L.field_array, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_check(s, e, "read field");
    for (int k = 0; k < L.Sz; k++) {
        const int pr = (k + s->g.zoff) % L.Sz;
        for (int i = 0; i < L.Sx; i++) {
            const size_t o = (size_t)pr * L.pitch + i;
            out[(size_t)k * L.Sx + i] = L.real == 4 ? (double)((float*)raw.data())[o] : ((double*)raw.data())[o];
        }
    }
    return BF_OK;
}

static bf_status read_particles(bf_sim* s, int species, std::vector<double>* cols, int64_t* nlive)
{
    const Layout& L = s->L;
    int nu[2] = {0, 0};
    hipError_t e = hipMemcpy(nu, nused_e(s), 2 * sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_check(s, e, "read counts");
    const int n = std::min<int64_t>(species == 0 ? nu[0] : nu[1], L.cap);
    const bool f32 = L.real == 4;
    char* b = (char*)s->buf[(species == 0 ? 1 : 3) + s->p_cur];
    std::vector<double> x(n), z(n);
    std::vector<char> w(n * (size_t)L.real);
    std::vector<uint32_t> id(n);
    std::vector<char> u[3];
    Chk ck;
    if (n > 0) {
        ck(hipMemcpy(x.data(), b + (species == 0 ? L.e_off[0] : L.i_off[0]), n * 8, hipMemcpyDeviceToHost));
        ck(hipMemcpy(z.data(), b + (species == 0 ? L.e_off[1] : L.i_off[1]), n * 8, hipMemcpyDeviceToHost));
        ck(hipMemcpy(w.data(), b + (species == 0 ? L.e_off[5] : L.i_off[2]), n * (size_t)L.real,
                     hipMemcpyDeviceToHost));
        ck(hipMemcpy(id.data(), b + (species == 0 ? L.e_off[6] : L.i_off[3]), n * 4, hipMemcpyDeviceToHost));
        if (species == 0)
            for (int q = 0; q < 3; q++) {
                u[q].resize(n * (size_t)L.real);
                ck(hipMemcpy(u[q].data(), b + L.e_off[2 + q], n * (size_t)L.real, hipMemcpyDeviceToHost));
            }
    }
    e = ck.e;
    if (e != hipSuccess) return hip_check(s, e, "read particles");
    auto rd = [&](const std::vector<char>& v, int p) {
        return f32 ? (double)((const float*)v.data())[p] : ((const double*)v.data())[p];
    };
    for (int q = 0; q < 7; q++) cols[q].clear();
    const double zsh = ion_shift(s, s->t);
    const int Nx = s->cfg.nx, Nz = s->cfg.nz;
    const bool perx = s->cfg.periodic_mask & 1, perz = (s->cfg.periodic_mask >> 2) & 1;
    for (int p = 0; p < n; p++) {
        const double wv = rd(w, p);
        if (wv == 0.0) continue;
        double xc = x[p], zc = species == 0 ? z[p] : z[p] - zsh;
        if (perx) { xc = std::fmod(xc, (double)Nx); if (xc < 0) xc += Nx; if (xc >= Nx) xc -= Nx; }
        if (perz) { zc = std::fmod(zc, (double)Nz); if (zc < 0) zc += Nz; if (zc >= Nz) zc -= Nz; }
        cols[0].push_back((double)id[p]);
        cols[1].push_back(xc * s->cfg.dx_um);
        cols[2].push_back(zc * s->cfg.dz_um);
        if (species == 0) {
            cols[3].push_back(rd(u[0], p));
            cols[4].push_back(rd(u[1], p));
            cols[5].push_back(rd(u[2], p));
        } else {
            cols[3].push_back(0.0);
            cols[4].push_back(0.0);
            cols[5].push_back(-s->gamma * s->beta);
        }
        cols[6].push_back(wv);
    }
    *nlive = (int64_t)cols[0].size();
    return BF_OK;
}

template <typename R>
static bf_status gauss_impl(bf_sim* s, double* out)
{
    const Layout& L = s->L;
    const size_t grid = (size_t)L.Sx * L.Sz;
    double* rho = s->w<double>(L.w_rho);
    double* rhof = rho + grid;
    Chk ck;
    ck(hipMemsetAsync(rho, 0, sizeof(double) * grid, s->stream));
    int nu[2] = {0, 0};
    ck(hipMemcpy(nu, nused_e(s), 2 * sizeof(int), hipMemcpyDeviceToHost));
    if (ck.e != hipSuccess) return hip_check(s, ck.e, "gauss");
    Geo g0 = s->g;
    g0.zoff = 0;
    g0.pitch = L.Sx;
    const double inv_cell = 1.0 / (s->cfg.dx_um * s->cfg.dz_um);
    const int ni = (s->have_plasma && s->plasma.ion_mode == 1) ? nu[1] : 0;
    double za = 0.0;
    int na = 0;
    if (s->have_laser) {
        za = (s->za_lab / s->gamma - s->beta * s->t) / s->cfg.dz_um - (double)s->shift;
        if (za >= 0.0 && za < s->cfg.nz) na = s->cfg.nx;
    }
    launch_rho<R>(g0, electrons<R>(s, s->p_cur), nu[0], ions<R>(s, s->p_cur), ni, ion_shift(s, s->t),
                  s->w<double>(L.w_ant), na, 0.5, za, s->aw, inv_cell, rho, s->stream);
    if (s->have_beam && !s->beam_test) launch_rho_beam(g0, beam_arrays(s), (int)s->nbeam, inv_cell, rho, s->stream);
    double* res = rho;
    if (s->cfg.filter_npass > 0) {
        // the step's filter on the nodal charge density: rho -> rhof along x, back along z
        bf3::FiltSeq fs;
        bf3::filter_seq(s->cfg.filter_npass, s->cfg.filter_compensate, s->cfg.filter_strides, &fs);
        double* in[3] = {rho, nullptr, nullptr};
        double* tmp[3] = {rhof, nullptr, nullptr};
        double* o3[3] = {rho, nullptr, nullptr};
        const int hx[3] = {0, 0, 0}, hz[3] = {0, 0, 0};
        bf3::launch_filter_xz<double>(g3_of(g0, s->cfg), in, tmp, o3, hx, hz, 1, fs, s->stream);
    }
    ck(hipStreamSynchronize(s->stream));
    std::vector<double> r(grid), ex(grid), ez(grid);
    ck(hipMemcpy(r.data(), res, grid * 8, hipMemcpyDeviceToHost));
    if (ck.e != hipSuccess) return hip_check(s, ck.e, "gauss");
    int a;
    field_ptr_of(s, BF_F_EX, &a);
    bf_status st = read_field(s, a, ex.data());
    if (st != BF_OK) return st;
    field_ptr_of(s, BF_F_EZ, &a);
    st = read_field(s, a, ez.data());
    if (st != BF_OK) return st;
    const bool perx = s->cfg.periodic_mask & 1, perz = (s->cfg.periodic_mask >> 2) & 1;
    for (int k = 0; k < L.Sz; k++)
        for (int i = 0; i < L.Sx; i++) {
            int il = i - 1, kl = k - 1;
            if (perx) il = (il + L.Sx) % L.Sx;
            if (perz) kl = (kl + L.Sz) % L.Sz;
            const double exl = il >= 0 ? ex[(size_t)k * L.Sx + il] : 0.0;
            const double ezl = kl >= 0 ? ez[(size_t)kl * L.Sx + i] : 0.0;
            const double div = (ex[(size_t)k * L.Sx + i] - exl) / s->cfg.dx_um +
                               (ez[(size_t)k * L.Sx + i] - ezl) / s->cfg.dz_um;
            out[(size_t)k * L.Sx + i] = div - r[(size_t)k * L.Sx + i];
        }
    return hip_check(s, hipGetLastError(), "gauss");
}

extern "C" {

bf_status bf_diagnose(bf_sim* s, int kind, int arg, void* host_out, size_t bytes)
{
    if (!s || !host_out) return BF_EINVAL;
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_check(s, e, "diagnose");
    if (s->d3 && kind != BF_DIAG_TIMERS) return diagnose3(s, kind, arg, host_out, bytes);
    const Layout& L = s->L;
    const size_t grid = (size_t)L.Sx * L.Sz;
    switch (kind) {
    case BF_DIAG_FIELD: {
        int a;
        field_ptr_of(s, arg, &a);
        if (a < 0) return fail(s, BF_EINVAL, "bad field id");
        if (bytes < grid * 8) return fail(s, BF_EINVAL, "buffer too small");
        return read_field(s, a, (double*)host_out);
    }
    case BF_DIAG_COUNTS: {
        if (bytes < 4 * sizeof(int64_t)) return fail(s, BF_EINVAL, "buffer too small");
        std::vector<double> cols[7];
        int64_t ne = 0, ni = 0;
        bf_status st = read_particles(s, 0, cols, &ne);
        if (st != BF_OK) return st;
        if (s->have_plasma && s->plasma.ion_mode == 1) {
            st = read_particles(s, 1, cols, &ni);
            if (st != BF_OK) return st;
        }
        int nu[2] = {0, 0};
        e = hipMemcpy(nu, nused_e(s), 2 * sizeof(int), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_check(s, e, "counts");
        int64_t* o = (int64_t*)host_out;
        o[0] = ne; o[1] = ni; o[2] = nu[0]; o[3] = nu[1];
        return BF_OK;
    }
    case BF_DIAG_PARTICLES: {
        std::vector<double> cols[7];
        int64_t n = 0;
        bf_status st = read_particles(s, arg, cols, &n);
        if (st != BF_OK) return st;
        if (bytes < (size_t)n * 7 * 8) return fail(s, BF_EINVAL, "buffer too small");
        double* o = (double*)host_out;
        for (int q = 0; q < 7; q++) std::memcpy(o + (size_t)q * n, cols[q].data(), n * 8);
        return BF_OK;
    }
    case BF_DIAG_STATION: {
        if (arg < 0 || arg >= s->nst) return fail(s, BF_EINVAL, "bad station");
        int cnt = 0;
        e = hipMemcpy(&cnt, s->w<int>(L.w_st_cnt) + arg, sizeof(int), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_check(s, e, "station");
        if (bytes < 8 + (size_t)cnt * 7 * 8) return fail(s, BF_EINVAL, "buffer too small");
        *(int64_t*)host_out = cnt;
        if (cnt > 0)
            e = hipMemcpy((char*)host_out + 8, s->w<double>(L.w_st_rec) + (size_t)arg * L.stcap * 7,
                          (size_t)cnt * 7 * 8, hipMemcpyDeviceToHost);
        return hip_check(s, e, "station");
    }
    case BF_DIAG_ENERGY: {
        if (bytes < 3 * 8) return fail(s, BF_EINVAL, "buffer too small");
        std::vector<double> f(grid);
        double ue = 0, ub = 0;
        const int ids[6] = {BF_F_EX, BF_F_EY, BF_F_EZ, BF_F_BX, BF_F_BY, BF_F_BZ};
        for (int q = 0; q < 6; q++) {
            int a;
            field_ptr_of(s, ids[q], &a);
            bf_status st = read_field(s, a, f.data());
            if (st != BF_OK) return st;
            double acc = 0;
            for (double v : f) acc += v * v;
            (q < 3 ? ue : ub) += acc;
        }
        std::vector<double> cols[7];
        int64_t n = 0;
        bf_status st = read_particles(s, 0, cols, &n);
        if (st != BF_OK) return st;
        double k = 0;
        for (int64_t p = 0; p < n; p++) {
            const double ux = cols[3][p], uy = cols[4][p], uz = cols[5][p];
            k += cols[6][p] * (std::sqrt(1.0 + ux * ux + uy * uy + uz * uz) - 1.0);
        }
        const double dv = s->cfg.dx_um * s->cfg.dz_um;
        double* o = (double*)host_out;
        o[0] = 0.5 * ue * dv; o[1] = 0.5 * ub * dv; o[2] = k;
        return BF_OK;
    }
    case BF_DIAG_GAUSS: {
        if (bytes < grid * 8) return fail(s, BF_EINVAL, "buffer too small");
        return L.real == 4 ? gauss_impl<float>(s, (double*)host_out) : gauss_impl<double>(s, (double*)host_out);
    }
    case BF_DIAG_INFO: {
        if (bytes < sizeof(bf_info)) return fail(s, BF_EINVAL, "buffer too small");
        bf_info* o = (bf_info*)host_out;
        std::memset(o, 0, sizeof *o);
        o->dt = s->dt; o->dt_crit = s->dt_crit; o->beta = s->beta; o->gamma = s->gamma;
        o->v_window = s->vw; o->n0_norm = s->n0; o->e0_norm = s->e0; o->omega = s->omega;
        o->alpha2 = s->a2; o->beta2 = s->b2; o->antenna_weight = s->aw;
        o->stored_x = L.Sx; o->stored_z = L.Sz; o->pml_x = L.Px; o->pml_z = L.Pz;
        o->step = s->step; o->time = s->t; o->shift = s->shift; o->next_row = s->next_row;
        o->tile_x = L.tile_x; o->tile_z = L.tile_z; o->ntiles = L.ntiles; o->sort_every = s->sort_every;
        return BF_OK;
    }
    case BF_DIAG_ANTENNA: {
        if (!s->have_laser) return fail(s, BF_EINVAL, "no laser");
        if (bytes < (size_t)s->cfg.nx * 8) return fail(s, BF_EINVAL, "buffer too small");
        std::vector<double> xm(s->cfg.nx);
        e = hipMemcpy(xm.data(), s->w<double>(L.w_ant), xm.size() * 8, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_check(s, e, "antenna");
        for (int i = 0; i < s->cfg.nx; i++) ((double*)host_out)[i] = xm[i] * s->cfg.dx_um;
        return BF_OK;
    }
    case BF_DIAG_TIMERS: {
        if (bytes < sizeof(double) * 2 * BF_PHASE_COUNT) return fail(s, BF_EINVAL, "buffer too small");
        e = s->fold_marks();
        if (e != hipSuccess) return hip_check(s, e, "timers");
        double* o = (double*)host_out;
        for (int q = 0; q < BF_PHASE_COUNT; q++) { o[2 * q] = s->tacc[q]; o[2 * q + 1] = s->tcnt[q]; }
        if (arg) for (int q = 0; q < BF_PHASE_COUNT; q++) { s->tacc[q] = 0.0; s->tcnt[q] = 0.0; }
        return BF_OK;
    }
    case BF_DIAG_BEAM: {
        if (arg != 0 && arg != 1) return fail(s, BF_EINVAL, "beam diagnostic: arg 0 or 1");
        const BeamArrays b = beam_arrays(s);
        const int64_t n = s->have_beam ? s->nbeam : 0;
        int64_t* o64 = (int64_t*)host_out;
        double* o = (double*)host_out + 1;
        if (arg == 0) {
            if (bytes < 8 + 64 * (size_t)n) return fail(s, BF_EINVAL, "buffer too small");
            o64[0] = n;
            if (n == 0) return BF_OK;
            double* const src[7] = {b.x, b.z, b.ux, b.uy, b.uz, b.w, b.tact};
            for (int k = 0; k < 7; k++) {
                e = hipMemcpy(o + k * n, src[k], 8 * (size_t)n, hipMemcpyDeviceToHost);
                if (e != hipSuccess) return hip_check(s, e, "beam");
            }
            std::vector<int> st((size_t)n);
            e = hipMemcpy(st.data(), b.state, 4 * (size_t)n, hipMemcpyDeviceToHost);
            if (e != hipSuccess) return hip_check(s, e, "beam");
            for (int64_t p = 0; p < n; p++) {
                o[p] *= s->cfg.dx_um;
                o[n + p] *= s->cfg.dz_um;
                o[7 * n + p] = (double)st[p];
            }
            return BF_OK;
        }
        const int64_t m = s->have_beam ? s->beam_rec : 0;
        if (bytes < 8 + 64 * (size_t)m) return fail(s, BF_EINVAL, "buffer too small");
        o64[0] = m;
        if (m > 0) {
            e = hipMemcpy(o, b.hist, 64 * (size_t)m, hipMemcpyDeviceToHost);
            if (e != hipSuccess) return hip_check(s, e, "beam history");
        }
        return BF_OK;
    }
    default:
        return fail(s, BF_EINVAL, "unknown diagnostic");
    }
}

bf_status bf_set_field(bf_sim* s, int field, const double* in, size_t bytes)
{
    bf_status st = guard(s);
    if (st != BF_OK) return st;
    if (s->d3) {
        const Sim3& L3 = *s->d3;
        const int a = (field == BF_F_JX || field == BF_F_JY || field == BF_F_JZ) ? filtered3(s->cfg, field - BF_F_JX)
                                                                                : array3_of(*s->d3, field);
        if (a < 0) return fail(s, BF_EINVAL, "bad field id");
        if (!in || bytes < (size_t)L3.g.S[0] * L3.g.S[1] * L3.g.S[2] * 8) return fail(s, BF_EINVAL, "buffer too small");
        hipError_t e3 = hipStreamSynchronize(s->stream);
        if (e3 != hipSuccess) return hip_check(s, e3, "set_field");
        return write_field3(s, a, in);
    }
    const Layout& L = s->L;
    if (!in || bytes < (size_t)L.Sx * L.Sz * 8) return fail(s, BF_EINVAL, "buffer too small");
    int a;
    field_ptr_of(s, field, &a);
    if (a < 0) return fail(s, BF_EINVAL, "bad field id");
    hipError_t e = hipStreamSynchronize(s->stream);
    std::vector<char> raw(L.field_array, 0);
    for (int k = 0; k < L.Sz; k++) {
        const int pr = (k + s->g.zoff) % L.Sz;
        for (int i = 0; i < L.Sx; i++) {
            const size_t o = (size_t)pr * L.pitch + i;
            const double v = in[(size_t)k * L.Sx + i];
            if (L.real == 4) ((float*)raw.data())[o] = (float)v;
            else ((double*)raw.data())[o] = v;
        }
    }
    if (e == hipSuccess)
        e = hipMemcpy(s->fields() + L.field_array * a, raw.data(), L.field_array, hipMemcpyHostToDevice);
    return hip_check(s, e, "set_field");
}

bf_status bf_get_state(const bf_sim* s, bf_state* o)
{
    if (!s || !o) return BF_EINVAL;
    if (hipStreamSynchronize(s->stream) != hipSuccess) return BF_EDEVICE;
    std::memset(o, 0, sizeof *o);
    o->abi_version = BF_ABI_VERSION;
    o->struct_size = sizeof(bf_state);
    o->step = s->step; o->time = s->t; o->shift = s->shift; o->next_row = s->next_row;
    o->zoff = s->g.zoff;
    o->e_cur = s->e_cur | (s->eb_cur << 1) | (s->bb_cur << 2) | (s->sg_cur << 3);
    o->b_cur = s->b_cur;
    o->p_cur = s->p_cur;
    o->nseg_e = s->nseg_e; o->nseg_i = s->nseg_i; o->since_sort = s->since_sort;
    o->have_plasma = s->have_plasma; o->have_laser = s->have_laser; o->nstations = s->nst;
    o->have_beam = s->have_beam; o->beam_test_only = s->beam_test; o->beam_n = s->nbeam;
    o->beam_records = s->beam_rec; o->beam_vbar = s->vbar;
    if (s->d3) {   // 3D: one segment table per species, both of nseg segments
        o->zoff = s->d3->g.zoff; o->p_cur = s->d3->p_cur; o->since_sort = s->d3->since_sort;
        o->nseg_e = o->nseg_i = s->d3->nseg;
        o->e_cur = (s->d3->bb_cur << 2) | (s->d3->eb_cur << 1);
    }
    return BF_OK;
}

bf_status bf_set_state(bf_sim* s, const bf_state* in)
{
    if (!s || !in || in->abi_version != BF_ABI_VERSION || in->struct_size != sizeof(bf_state)) return BF_EINVAL;
    if (s->d3) {
        Sim3& L3 = *s->d3;
        if (in->zoff < 0 || in->zoff >= L3.g.S[2] || in->nseg_e < 0 || in->nseg_e > L3.seg_cap ||
            in->nseg_i != in->nseg_e)
            return BF_EINVAL;
        s->step = in->step; s->t = in->time; s->shift = in->shift; s->next_row = in->next_row;
        L3.g.zoff = in->zoff; L3.p_cur = in->p_cur & 1; L3.since_sort = in->since_sort;
        L3.nseg = in->nseg_e; L3.bb_cur = (in->e_cur >> 2) & 1; L3.eb_cur = (in->e_cur >> 1) & 1;
        return BF_OK;
    }
    if (in->zoff < 0 || in->zoff >= s->L.Sz || in->nseg_e < 0 || in->nseg_e > s->L.seg_cap) return BF_EINVAL;
    if (in->have_beam && (in->beam_n < 0 || in->beam_n > s->cfg.beam_capacity || in->beam_records < 0 ||
                          in->beam_records > s->cfg.beam_history))
        return BF_EINVAL;
    s->have_beam = in->have_beam ? 1 : 0; s->beam_test = in->beam_test_only ? 1 : 0;
    s->nbeam = in->have_beam ? in->beam_n : 0; s->beam_rec = in->have_beam ? in->beam_records : 0;
    s->vbar = in->beam_vbar;
    s->step = in->step; s->t = in->time; s->shift = in->shift; s->next_row = in->next_row;
    s->g.zoff = in->zoff;
    s->e_cur = in->e_cur & 1; s->eb_cur = (in->e_cur >> 1) & 1; s->bb_cur = (in->e_cur >> 2) & 1;
    s->sg_cur = (in->e_cur >> 3) & 1;
    s->b_cur = in->b_cur & 1; s->p_cur = in->p_cur & 1;
    s->nseg_e = in->nseg_e; s->nseg_i = in->nseg_i; s->since_sort = in->since_sort;
    return BF_OK;
}

}  // extern "C"
