"""Workload recipes and seeded input generators shared by the tests, the benchmark, the
HIP binding and the oracle wrapper.

This module holds parameters only -- sizes, physical inputs, coefficient sets supplied by
the user, and seeded random states for unit tests.  It contains none of the PIC method's
arithmetic; both implementations derive everything else (time step, window speed,
normalisation, loading) themselves.

Physical inputs are in the units the C interfaces take: um, fs, cm^-3, Lorentz factor.
"""
from __future__ import annotations

import copy
import math

import numpy as np

# Coefficient sets of the tunable solver, Table "CKcoefs" of Sec. 4.2.1 (alpha, beta, gamma).
CK_SETS = {
    "yee": (1.0, 0.0, 0.0),
    "ck": (7.0 / 12.0, 1.0 / 12.0, 1.0 / 48.0),
    "ck2": (19.0 / 24.0, 1.0 / 24.0, 1.0 / 96.0),
    "ck3": (11.0 / 12.0, 1.0 / 24.0, -1.0 / 48.0),
    "ck4": (3.0 / 4.0, 1.0 / 16.0, 0.0),
    "ck5": (5.0 / 8.0, 3.0 / 40.0, 3.0 / 160.0),
}

LAMBDA_UM = 0.8


def _beta(gamma: float) -> float:
    return math.sqrt(1.0 - 1.0 / (gamma * gamma))


def boosted_cell(gamma: float, frac: float = 1.0 / 32.0, lam: float = LAMBDA_UM) -> float:
    """Cell size as a fixed fraction of the Doppler-stretched wavelength (1+beta) gamma lambda
    (Sec. 5.1 keeps dz a constant fraction of the boosted laser wavelength)."""
    return frac * (1.0 + _beta(gamma)) * gamma * lam


def make_config(nx, nz, dx_um, dz_um, *, pml_cells=10, periodic_x=0, periodic_z=0, ck="yee",
                theta=0.0, cfl_fraction=0.95, filter_npass=0, filter_compensate=0,
                gamma_boost=1.0, moving_window=0, seed=1009, real="f64", filter_strides=1,
                gather_kind=0, pusher=0, pml_kind=0):
    """filter_strides: mask of the filter strides (bit s-1: stride s), e.g. 0b11 = S(1:2),
    0b111 = S(1:2:3), 0b1011 = S(1:2:4); gather_kind 0 energy conserving, 1 momentum
    conserving; pusher 0 Boris, 1 Vay."""
    a, b, g = CK_SETS[ck] if isinstance(ck, str) else ck
    return dict(nx=int(nx), nz=int(nz), dx_um=float(dx_um), dz_um=float(dz_um),
                pml_cells=int(pml_cells), periodic_x=int(periodic_x), periodic_z=int(periodic_z),
                ck_alpha=a, ck_beta=b, ck_gamma=g, theta=float(theta),
                cfl_fraction=float(cfl_fraction), filter_npass=int(filter_npass),
                filter_compensate=int(filter_compensate), gamma_boost=float(gamma_boost),
                moving_window=int(moving_window), seed=int(seed), real=real,
                filter_strides=int(filter_strides), gather_kind=int(gather_kind), pusher=int(pusher),
                pml_kind=int(pml_kind))


def plasma(n0_cm3, ppc, *, ramp_um=0.0, start_um=0.0, ion_mode=0):
    return dict(n0_cm3=float(n0_cm3), ramp_um=float(ramp_um), start_um=float(start_um),
                ppc=int(ppc), ion_mode=int(ion_mode))


def laser(a0, waist_um, fwhm_fs, z_antenna_um, lambda_um=LAMBDA_UM, t_peak_fs=0.0, pol=0):
    """pol: 0 along x, 1 along y; t_peak_fs: lab time the peak crosses the plane (0: 3 sigma_t)."""
    return dict(lambda_um=float(lambda_um), a0=float(a0), waist_um=float(waist_um),
                fwhm_fs=float(fwhm_fs), z_antenna_um=float(z_antenna_um), t_peak_fs=float(t_peak_fs),
                pol=int(pol))


# ---------------------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------------------

def c1(real="f64", nx=64, nz=512, ppc=4):
    """2D lab frame: 64x512 Yee grid, 0.05 um cells, 4 ppc at 1e19 cm^-3 flat from z=1 um,
    immobile ions, laser 0.8 um a0=1 waist 8 um 10 fs from z=0.5 um, CFL 0.95, one bilinear
    pass, x periodic, 10-cell PML at the z ends, 200 steps."""
    return dict(
        name=f"2D lab frame {nx}x{nz}, {ppc} ppc, 1e19 cm^-3, a0=1, Yee, 1-pass bilinear",
        config=make_config(nx, nz, 0.05, 0.05, pml_cells=10, periodic_x=1, ck="yee",
                           theta=0.0, cfl_fraction=0.95, filter_npass=1, filter_compensate=0,
                           gamma_boost=1.0, moving_window=0, seed=1010, real=real),
        plasma=plasma(1e19, ppc, start_um=1.0, ion_mode=0),
        laser=laser(1.0, 8.0, 10.0, 0.5),
        steps=200,
    )


def c2(real="f32", nx=256, nz=4096, ppc=16, preload=False, gamma=13.0):
    """2D boosted frame gamma=13: 256x4096, 16 ppc, lab density 1e18 cm^-3 with a 20 um
    linear up-ramp starting 2 um ahead of the antenna, laser a0=2 waist 20 um, CK2 solver,
    Friedman theta=0.1, 4 bilinear passes + compensation, 10-cell PML on every face, moving
    window, rigid ions, 20000 steps.  preload=True fills the whole window with the plateau
    density (throughput runs start from the filled state)."""
    d = boosted_cell(gamma)
    z_ant = gamma * 0.6 * nz * d              # lab position whose boosted image sits at 60%
    start = -1e30 if preload else z_ant + 2.0
    ramp = 0.0 if preload else 20.0
    # laser FWHM = half a plasma wavelength at 1e18 cm^-3 (lambda_p = 33.39 um)
    fwhm = 0.5 * 33.39 / 0.299792458
    return dict(
        name=(f"2D boosted gamma={gamma:g} {nx}x{nz}, {ppc} ppc, 1e18 cm^-3"
              f"{' (pre-loaded window)' if preload else ''}, a0=2, CK2 + Friedman 0.1,"
              " 4-pass bilinear + compensation, 10-cell PML, moving window"),
        config=make_config(nx, nz, d, d, pml_cells=10, periodic_x=0, ck="ck2", theta=0.1,
                           cfl_fraction=0.95, filter_npass=4, filter_compensate=1,
                           gamma_boost=gamma, moving_window=1, seed=1011, real=real),
        plasma=plasma(1e18, ppc, ramp_um=ramp, start_um=start, ion_mode=1),
        laser=laser(2.0, 20.0, fwhm, z_ant),
        steps=20000,
    )


def c4(nruns=64, seed=10094, scale=1.0, real="f32"):
    """The batched scan: independent 2D boosted runs with parameters drawn per run --
    N_x ~ U{128..256}, N_z ~ U{1024..4096}, gamma = exp(U[ln 5, ln 100]),
    n0 = exp(U[ln 1e17, ln 1e19]) cm^-3, ppc ~ U{4..16}, time step 0.95 (1 + u) of the
    Friedman-corrected CFL limit with u ~ U[-0.1, 0.1] clamped at 0.999 -- and fixed square cells
    of 1/32 of the boosted wavelength, CK2, theta = 0.1, 4 passes + compensation, 10-cell PML,
    window at the wake velocity (backward when gamma exceeds gamma_w), laser a0 = 2, waist
    20 um sqrt(1e18 / n0), 30 fs, pre-loaded plasma, 2000 steps each.  scale < 1 shrinks the
    grids (parity-size batches)."""
    rng = np.random.default_rng(seed)
    runs = []
    for q in range(nruns):
        nx = int(rng.integers(128, 257) * scale)
        nz = int(rng.integers(1024, 4097) * scale)
        gamma = float(np.exp(rng.uniform(np.log(5.0), np.log(100.0))))
        n0 = float(np.exp(rng.uniform(np.log(1e17), np.log(1e19))))
        ppc = int(rng.integers(4, 17))
        cfl = min(0.95 * (1.0 + rng.uniform(-0.1, 0.1)), 0.999)
        d = boosted_cell(gamma)
        z_ant = gamma * 0.6 * nz * d
        runs.append(dict(
            name=f"scan run {q}: gamma={gamma:.3g} n0={n0:.3g} {nx}x{nz} ppc={ppc} cfl={cfl:.3f}",
            config=make_config(nx, nz, d, d, pml_cells=10, ck="ck2", theta=0.1, cfl_fraction=cfl,
                               filter_npass=4, filter_compensate=1, gamma_boost=gamma,
                               moving_window=1, seed=seed + q, real=real),
            plasma=plasma(n0, ppc, start_um=-1e30, ion_mode=1),
            laser=laser(2.0, 20.0 * np.sqrt(1e18 / n0), 30.0, z_ant),
            steps=2000,
        ))
    return runs


def c5_wake(real="f32", nx=64, nz=512, ppc=4, seed=1015, refine=1):
    """Learned-filter wake family: the lab-frame stage of c1 (0.05 um cells, 4 ppc at 1e19 cm^-3,
    a0 = 1, 10 fs) with the 4-pass + compensation filter, run 700 steps so the pulse crosses the
    box and the wake forms behind it.  refine = 2 halves the cells and the time step (same box,
    twice the steps): the reference run, unfiltered, in FP64."""
    w = c1(real, nx=nx * refine, nz=nz * refine, ppc=ppc)
    d = 0.05 / refine
    w["config"].update(make_config(nx * refine, nz * refine, d, d, pml_cells=10 * refine, periodic_x=1,
                                   ck="yee", cfl_fraction=0.95, filter_npass=4 if refine == 1 else 0,
                                   filter_compensate=1 if refine == 1 else 0, seed=seed, real=real))
    w["name"] = f"wake family {nx * refine}x{nz * refine}"
    w["steps"] = 700 * refine
    return w


def c5_growth(real="f32", nx=64, nz=512, ppc=4, gamma=13.0, n0=1e19, npass=4, comp=1, seed=1016):
    """Instability family: boosted frame gamma = 13, square cells of 1/32 of the boosted
    wavelength (0.649 um), plasma at 1e19 cm^-3 filling the moving window and streaming through it
    at -beta c with paired rigid ions, no laser: the numerical instabilities of Sec. 4 grow from
    the particle noise.  npass = 0: no filter."""
    d = boosted_cell(gamma)
    return dict(
        name=f"instability family gamma={gamma:g} {nx}x{nz}, {ppc} ppc, {n0:g} cm^-3",
        config=make_config(nx, nz, d, d, pml_cells=10, ck="ck2", theta=0.1, cfl_fraction=0.95,
                           filter_npass=npass, filter_compensate=comp, gamma_boost=gamma,
                           moving_window=1, seed=seed, real=real),
        plasma=plasma(n0, ppc, start_um=-1e30, ion_mode=1),
        laser=None,
        steps=600,
    )


def c5_growth_lab(real="f32", nx=64, nz=512, ppc=4, npass=4, comp=1, seed=1018):
    """Lab-frame instability family: the wake family's laser-plasma run (0.05 um cells, 4 ppc at
    1e19 cm^-3, a0 = 1, 10 fs) with the Cole-Karkkainen solver at 0.95 of its Courant limit
    (c dt = 0.95 dz, where its Nyquist modes are nearly stationary, App. I) instead of Yee, 600
    steps.  npass = 0: no filter."""
    w = c1(real, nx=nx, nz=nz, ppc=ppc)
    w["config"].update(make_config(nx, nz, 0.05, 0.05, pml_cells=10, periodic_x=1, ck="ck",
                                   cfl_fraction=0.95, filter_npass=npass, filter_compensate=comp,
                                   seed=seed, real=real))
    w["name"] = f"lab-frame CK instability family {nx}x{nz}, {ppc} ppc"
    w["steps"] = 600
    return w


def stage_10gev(real="f32", nx=128, nz=2048, ppc=4, gamma=130.0, cfl=0.7071, ck="ck", gather_kind=0,
                seed=1017):
    """A full-scale 10 GeV class stage in the wake frame (Sec. 5.2, 5.3): lab density 1e17 cm^-3
    (gamma_w ~ 132) with a 20 um up-ramp starting just ahead of the box, so the plasma enters at
    the front and streams through; boosted frame gamma = 130 with square cells of 6.5 um (lambda*/32);
    laser a0 = 1, waist 50 um, FWHM half a plasma wavelength (176 fs), the antenna at 60% of the box;
    CK solver without damping or filter (the high-frequency instability of Sec. 4 left free), c dt /
    dz = cfl (the 2D CK limit is c dt = dz); moving window; rigid ions."""
    d = boosted_cell(gamma)
    z_ant = gamma * 0.6 * nz * d
    fwhm = 0.5 * 105.6 / 0.299792458
    return dict(
        name=f"10 GeV stage gamma={gamma:g} {nx}x{nz}, {ppc} ppc, 1e17 cm^-3, c dt/dz={cfl:.4g}",
        config=make_config(nx, nz, d, d, pml_cells=10, ck=ck, theta=0.0, cfl_fraction=cfl, filter_npass=0,
                           filter_compensate=0, gamma_boost=gamma, moving_window=1, seed=seed, real=real,
                           gather_kind=gather_kind),
        plasma=plasma(1e17, ppc, ramp_um=20.0, start_um=gamma * (nz + 2) * d, ion_mode=1),
        laser=laser(1.0, 50.0, fwhm, z_ant),
        steps=0,
    )


def small_lab(real="f64", nx=24, nz=96, ppc=4, seed=77, npass=1, comp=0, ck="yee", theta=0.0):
    """A C1-shaped lab-frame case the oracle finishes in seconds (several tiles + ragged tail)."""
    w = c1(real, nx=nx, nz=nz, ppc=ppc)
    w["config"].update(make_config(nx, nz, 0.05, 0.05, pml_cells=10, periodic_x=1, ck=ck,
                                   theta=theta, filter_npass=npass, filter_compensate=comp,
                                   seed=seed, real=real))
    w["name"] = f"small lab {nx}x{nz}"
    return w


def small_boosted(real="f64", nx=40, nz=150, ppc=4, seed=78, gamma=13.0, preload=False):
    """A C2-shaped boosted case (window, PML on all faces, CK2 + Friedman, 4+comp filter,
    rigid ions, antenna) small enough for the oracle."""
    w = c2(real, nx=nx, nz=nz, ppc=ppc, preload=preload, gamma=gamma)
    w["config"]["seed"] = seed
    w["name"] = f"small boosted {nx}x{nz}"
    return w


# ---------------------------------------------------------------------------------------
# Three dimensions
# ---------------------------------------------------------------------------------------

def make_config3(nx, ny, nz, dx_um, dy_um, dz_um, *, pml_cells=10, periodic_x=0, periodic_y=0,
                 periodic_z=0, ck="yee", theta=0.0, cfl_fraction=0.95, filter_npass=0,
                 filter_compensate=0, gamma_boost=1.0, moving_window=0, seed=1009, real="f64",
                 filter_strides=1, gather_kind=0, pusher=0, pml_kind=0):
    a, b, g = CK_SETS[ck] if isinstance(ck, str) else ck
    return dict(dim=3, filter_strides=int(filter_strides), gather_kind=int(gather_kind), pusher=int(pusher),
                pml_kind=int(pml_kind), nx=int(nx), ny=int(ny), nz=int(nz), dx_um=float(dx_um), dy_um=float(dy_um),
                dz_um=float(dz_um), pml_cells=int(pml_cells), periodic_x=int(periodic_x),
                periodic_y=int(periodic_y), periodic_z=int(periodic_z), ck_alpha=a, ck_beta=b,
                ck_gamma=g, theta=float(theta), cfl_fraction=float(cfl_fraction),
                filter_npass=int(filter_npass), filter_compensate=int(filter_compensate),
                gamma_boost=float(gamma_boost), moving_window=int(moving_window), seed=int(seed),
                real=real)


def c3(real="f32", nx=128, ny=128, nz=1024, ppc=8, preload=False, gamma=30.0):
    """3D boosted frame gamma=30: 128x128x1024 cubic cells of (1+beta) gamma lambda / 16 (so
    that the stretched pulse and the antenna's path fit the box), 8 ppc (134M electrons when
    filled), lab density 1e17 cm^-3 with a 20 um linear up-ramp starting 2 um ahead of the
    antenna, laser a0=2 waist 50 um 30 fs, CK2 solver, Friedman theta=0.1, 4 bilinear passes
    + compensation, 10-cell PML on every face, moving window, rigid ions, 5000 steps."""
    d = boosted_cell(gamma, frac=1.0 / 16.0)
    z_ant = gamma * 0.6 * nz * d
    start = -1e30 if preload else z_ant + 2.0
    ramp = 0.0 if preload else 20.0
    fwhm = 30.0
    return dict(
        name=(f"3D boosted gamma={gamma:g} {nx}x{ny}x{nz}, {ppc} ppc, 1e17 cm^-3"
              f"{' (pre-loaded window)' if preload else ''}, a0=2, CK2 + Friedman 0.1,"
              " 4-pass bilinear + compensation, 10-cell PML, moving window"),
        config=make_config3(nx, ny, nz, d, d, d, pml_cells=10, ck="ck2", theta=0.1,
                            cfl_fraction=0.95, filter_npass=4, filter_compensate=1,
                            gamma_boost=gamma, moving_window=1, seed=1012, real=real),
        plasma=plasma(1e17, ppc, ramp_um=ramp, start_um=start, ion_mode=1),
        laser=laser(2.0, 50.0, fwhm, z_ant),
        steps=5000,
    )


def small_boosted3(real="f64", nx=12, ny=10, nz=48, ppc=2, seed=79, gamma=30.0, preload=False):
    """A C3-shaped case (window, PML on all faces, CK2 + Friedman, 4+comp filter, rigid ions,
    antenna) small enough for the 3D oracle; the laser waist is scaled to the box."""
    w = c3(real, nx=nx, ny=ny, nz=nz, ppc=ppc, preload=preload, gamma=gamma)
    w["config"]["seed"] = seed
    w["laser"]["waist_um"] = 0.3 * nx * w["config"]["dx_um"]
    w["name"] = f"small boosted 3D {nx}x{ny}x{nz}"
    return w


def random_electrons3(n, nx, ny, nz, d, seed, umax=1.0, margin=3.0):
    r = np.random.default_rng(seed)
    x = (margin + r.random(n) * (nx - 2 * margin)) * d[0]
    y = (margin + r.random(n) * (ny - 2 * margin)) * d[1]
    z = (margin + r.random(n) * (nz - 2 * margin)) * d[2]
    u = (2.0 * r.random((3, n)) - 1.0) * umax
    w = 0.5 + r.random(n)
    ids = np.arange(n, dtype=np.uint32)
    return dict(id=ids, x=x, y=y, z=z, ux=u[0], uy=u[1], uz=u[2], w=w)


def copy_workload(w):
    return copy.deepcopy(w)


# ---------------------------------------------------------------------------------------
# Seeded random states for unit tests
# ---------------------------------------------------------------------------------------

def random_electrons(n, nx, nz, dx, dz, seed, umax=1.0, margin=3.0):
    """n electrons uniformly placed at least `margin` cells inside the interior, with
    momenta uniform in [-umax, umax]^3 and weights in [0.5, 1.5] x 1e-3."""
    r = np.random.default_rng(seed)
    x = (margin + r.random(n) * (nx - 2 * margin)) * dx
    z = (margin + r.random(n) * (nz - 2 * margin)) * dz
    u = (2.0 * r.random((3, n)) - 1.0) * umax
    w = (0.5 + r.random(n)) * 1e-3
    ids = np.arange(n, dtype=np.uint32)
    return dict(id=ids, x=x, z=z, ux=u[0], uy=u[1], uz=u[2], w=w)


def random_field(shape, seed, amp=0.1):
    r = np.random.default_rng(seed)
    return amp * (2.0 * r.random(shape) - 1.0)


# Beam of the scaled 10 GeV stages (Table "Tablephyspar2d"): radius R_b = 82.5 nm with the
# transverse profile exp(-r^2 / 8 R_b^2) (a Gaussian of rms 2 R_b), length L_b = 85 nm with
# exp(-z^2 / 2 L_b^2).  The table gives no energy or spread; they are parameters here.
BEAM_RB_UM = 0.0825
BEAM_LB_UM = 0.085


def beam_lab(n, *, x_center_um, z_center_um, gamma_b, seed, rb_um=BEAM_RB_UM, lb_um=BEAM_LB_UM,
             energy_spread=0.0, angle_rms=0.0, weight=1e-6):
    """n test macro-particles of a lab-frame beam at t = 0: x (um), z (lab um), ux, uy, uz, w.
    Momenta gamma_b (1 + energy_spread N(0,1)) along z with transverse angles N(0, angle_rms)."""
    r = np.random.default_rng(seed)
    g = gamma_b * (1.0 + energy_spread * r.standard_normal(n))
    u = np.sqrt(g * g - 1.0)
    tx = np.tan(angle_rms * r.standard_normal(n))
    ty = np.tan(angle_rms * r.standard_normal(n))
    norm = np.sqrt(1.0 + tx * tx + ty * ty)
    return {
        "x": x_center_um + 2.0 * rb_um * r.standard_normal(n),
        "z": z_center_um + lb_um * r.standard_normal(n),
        "ux": u * tx / norm, "uy": u * ty / norm, "uz": u / norm,
        "w": np.full(n, weight),
    }


def scaled_stage(gamma, real="f32", ppc=1, seed=1018):
    """The scaled 10 GeV stage of Table "Tablephyspar2d" in the frame gamma: lab density 1e19 cm^-3,
    flat after a 4 um linear entrance ramp (the table's half-sinus read as linear), laser 0.8 um,
    a0 = 1, FWHM 10.08 um (33.6 fs; the table's sine profile replaced by the antenna's Gaussian),
    waist 12.6 um (the table's commented size sigma = 8.91 um as exp(-r^2/2 sigma^2)); 75 cells of
    0.65 um across and dz = lambda/32 in the lab (so (1 + beta) gamma lambda / 32 here); 1 electron +
    1 rigid ion per cell; Yee at 0.99 of its Courant limit, 4 passes + compensation, 10-cell PML.
    The window holds the emitted pulse and one plasma wavelength behind its peak, both stretched by
    the boost, with 30% to spare, and at least the table's lab-frame 1691 cells; the antenna sits at
    90% of it so the pulse, emitted while the lab-fixed plane sweeps backwards, stays inside."""
    d = boosted_cell(gamma)
    beta = _beta(gamma)
    t0 = 3.0 * (10.08 / (2.0 * math.sqrt(math.log(2.0))))          # 3 sigma_t of the field envelope, um
    lam_p = 2.0 * math.pi * 299792458e6 / (5.64e4 * math.sqrt(1e19))  # plasma wavelength at 1e19, um
    span = beta * gamma * t0 + lam_p * gamma * (1.0 + beta) + 10.0
    nz = max(1691, int(math.ceil(1.3 * span / d)))
    z_ant = gamma * 0.9 * nz * d
    return dict(
        name=f"scaled 10 GeV stage gamma={gamma:g} 75x{nz}, {ppc} ppc, 1e19 cm^-3, a0=1, Yee",
        config=make_config(75, nz, 0.65, d, pml_cells=10, periodic_x=1, ck="yee", theta=0.0, cfl_fraction=0.99,
                           filter_npass=4, filter_compensate=1, gamma_boost=gamma, moving_window=1,
                           seed=seed, real=real),
        plasma=plasma(1e19, ppc, ramp_um=4.0, start_um=z_ant + 2.0, ion_mode=1),
        laser=laser(1.0, 12.6, 10.08 / 0.299792458, z_ant),
        steps=0,
    )
