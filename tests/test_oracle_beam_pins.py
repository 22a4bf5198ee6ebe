"""Pins of the oracle's particle beam launched through a lab-fixed plane (Sec. 3.1.1).

The checks come from relativity and mechanics, not from the oracle's own formulas: the
paper's velocity transformation (Eqs. vxp*, vzp*) against the oracle's four-momentum form,
the inverse Lorentz transformation of the crossing event, the world line of the plane,
straight lab-frame trajectories of a field-free monoenergetic beam, the lab-frame
work-energy theorem in a uniform longitudinal field, and charge conservation through the
frozen-to-active transition.
"""
import math

import numpy as np
import pytest

import pic_inputs as pi
from oracle import Oracle

GAMMA = 5.0
BETA = math.sqrt(1.0 - 1.0 / GAMMA ** 2)


def _beta(g):
    return math.sqrt(1.0 - 1.0 / (g * g))


def beam_scene(*, n=64, gamma_b=50.0, z_inj=25.0, t_cross=1.5, spread=0.0, angle=0.0, seed=5,
               nx=16, nz=96, d=0.1, periodic=False, test_only=1, weight=1e-6, **cfg_kw):
    """A boosted box (gamma = 5, cells of d um) and a lab beam whose centre crosses the
    plane at z_inj at boosted time t_cross (the lab centre z_c solves
    t'* = gamma ((z_inj - z_c)/beta_b - beta z_inj) = t_cross)."""
    bb = _beta(gamma_b)
    z_c = z_inj - bb * (t_cross / GAMMA + BETA * z_inj)
    per = 1 if periodic else 0
    cfg = pi.make_config(nx, nz, d, d, pml_cells=0 if periodic else 8, periodic_x=1, periodic_z=per,
                         gamma_boost=GAMMA, **cfg_kw)
    parts = pi.beam_lab(n, x_center_um=0.5 * nx * d, z_center_um=z_c, gamma_b=gamma_b, seed=seed,
                        energy_spread=spread, angle_rms=angle, weight=weight)
    beam = dict(beta_b=bb, z_inj_um=z_inj, test_only=test_only)
    return cfg, beam, parts


# ---------------------------------------------------------------------------------------
# the transformation of Sec. 3.1.1, steps 1-3
# ---------------------------------------------------------------------------------------

def test_transform_matches_the_papers_velocity_form_at_the_mean_velocity():
    # for a particle moving at the mean beam velocity the paper's Eqs. vxp*, vyp*, vzp*
    # (written with beta_b) are exact; the oracle uses the four-momentum transformation
    cfg, beam, _ = beam_scene()
    o = Oracle(cfg)
    g, b = GAMMA, BETA
    bb = beam["beta_b"]
    gb = 1.0 / math.sqrt(1.0 - bb * bb)
    rng = np.random.default_rng(3)
    for _ in range(10):
        # a velocity of magnitude beta_b at a small angle: v_z differs from beta_b, so build
        # v_z = beta_b exactly and a transverse part on top
        vz = bb
        vx, vy = rng.normal(0, 1e-3, 2)
        gp = 1.0 / math.sqrt(1.0 - vx * vx - vy * vy - vz * vz)
        x, z = rng.uniform(0.5, 1.0), rng.uniform(10.0, 20.0)
        q = o.beam_transform(beam, x, z, gp * vx, gp * vy, gp * vz)
        gq = math.sqrt(1.0 + q[3] ** 2 + q[4] ** 2 + q[5] ** 2)
        # Eqs. vxp*, vyp*, vzp* with v_z = beta_b
        assert q[3] / gq == pytest.approx(vx / (g * (1.0 - b * bb)), rel=1e-11)
        assert q[4] / gq == pytest.approx(vy / (g * (1.0 - b * bb)), rel=1e-11)
        assert q[5] / gq == pytest.approx((vz - b) / (1.0 - b * bb), rel=1e-11)
    del gb


def test_crossing_event_maps_back_to_the_plane_and_the_ballistic_line():
    # inverse Lorentz transformation of (t'*, z'*) must give the lab event (t_c, z_inj) on
    # the particle's straight lab trajectory; z'* is where the synchronised frozen particle
    # stands at t'*: z'(0) + vbar' t'*
    cfg, beam, parts = beam_scene(spread=0.02, angle=1e-3, n=40)
    o = Oracle(cfg)
    bb = beam["beta_b"]
    vbar = (bb - BETA) / (1.0 - BETA * bb)    # relativistic velocity addition
    for p in range(40):
        x, z = parts["x"][p], parts["z"][p]
        ux, uy, uz = parts["ux"][p], parts["uy"][p], parts["uz"][p]
        gp = math.sqrt(1 + ux * ux + uy * uy + uz * uz)
        tp, xs, z0, *_ = o.beam_transform(beam, x, z, ux, uy, uz)
        zs = z0 + vbar * tp
        t_lab = GAMMA * (tp + BETA * zs)
        z_lab = GAMMA * (zs + BETA * tp)
        assert z_lab == pytest.approx(beam["z_inj_um"], abs=1e-11)
        # lab ballistics: the particle at z at t = 0 is at z + v_z t_lab
        assert z + uz / gp * t_lab == pytest.approx(beam["z_inj_um"], abs=1e-11)
        assert xs == pytest.approx(x + ux / gp * t_lab, abs=1e-12)
        # the plane's world line in the boosted frame: z' = z_inj / gamma - beta t'
        assert zs == pytest.approx(beam["z_inj_um"] / GAMMA - BETA * tp, abs=1e-11)


# ---------------------------------------------------------------------------------------
# field-free propagation: straight lab trajectories and the activation rule
# ---------------------------------------------------------------------------------------

def test_field_free_monoenergetic_beam_follows_its_lab_trajectory():
    cfg, beam, parts = beam_scene(n=64)
    o = Oracle(cfg)
    o.add_beam(beam, parts)
    bb = beam["beta_b"]
    vbar = (bb - BETA) / (1.0 - BETA * bb)
    dt = o.info()["dt"]
    seen_frozen = seen_active = False
    for k in range(1, 61):
        o.step(1)
        s = o.beam()
        tnow = k * dt
        # the activation rule: active once a step started at t_n >= t'*
        assert np.array_equal(s["state"] >= 1, s["t_act"] <= (k - 1) * dt)
        for p in range(64):
            zl = GAMMA * (s["z"][p] + BETA * tnow)
            tl = GAMMA * (tnow + BETA * s["z"][p])
            if s["state"][p] == 0:
                # a frozen particle has not reached the plane in the lab before t'*; one that
                # crossed during this step is at most one step of its lab speed beyond it
                # (dz_lab/dt' = gamma (vbar' + beta) while frozen)
                ahead = 0.0 if s["t_act"][p] > tnow else GAMMA * (vbar + BETA) * dt
                assert zl < beam["z_inj_um"] + ahead + 1e-12
                seen_frozen = True
            elif s["state"][p] == 1:
                # active: on the straight lab line z0 + beta_b t
                assert zl == pytest.approx(parts["z"][p] + bb * tl, abs=1e-10)
                seen_active = True
    assert seen_frozen and seen_active
    # momenta unchanged in zero field
    s = o.beam()
    ug = GAMMA * (parts["uz"][0] - BETA * math.sqrt(1 + parts["uz"][0] ** 2))
    assert np.allclose(s["uz"], ug, rtol=1e-13)


def test_history_is_the_lab_frame_mean_of_a_field_free_beam():
    cfg, beam, parts = beam_scene(n=64, gamma_b=40.0)
    o = Oracle(cfg)
    o.add_beam(beam, parts)
    o.step(50)
    h = o.beam_history()
    assert h.shape == (50, 8)
    bb = beam["beta_b"]
    rows = h[h[:, 1] > 0]
    assert len(rows) > 10
    for r in rows:
        n, sw, swz, swt, swg, swu, swu2 = r[1:]
        assert sw == pytest.approx(n * 1e-6, rel=1e-12)
        assert swg / sw == pytest.approx(40.0, rel=1e-12)              # gamma_lab = gamma_b
        assert swu / sw == pytest.approx(40.0 * bb, rel=1e-12)
        assert swu2 / sw - (swu / sw) ** 2 == pytest.approx(0.0, abs=1e-8)
    # once every particle is active the means lie on the mean lab line <z0> + beta_b <t>
    last = h[-1]
    assert last[1] == 64
    assert last[3] / last[2] == pytest.approx(parts["z"].mean() + bb * last[4] / last[2], abs=1e-9)


# ---------------------------------------------------------------------------------------
# uniform longitudinal field: the lab-frame work-energy theorem
# ---------------------------------------------------------------------------------------

def test_uniform_field_energy_gain_follows_the_lab_work_energy_theorem():
    # E_z along the boost is the same in both frames; the force on an electron (q = -1) is
    # -E_z, so in the lab d gamma / d z = -E_z along its path from the activation event
    ez = -0.5
    cfg, beam, parts = beam_scene(n=48, periodic=True)
    o = Oracle(cfg)
    o.set_field("Ez", np.full(o.shape, ez))
    o.add_beam(beam, parts)
    dt = o.info()["dt"]
    nsteps = 55
    o.step(nsteps)
    assert np.allclose(o.field("Ez"), ez, atol=1e-14)
    s = o.beam()
    bb = beam["beta_b"]
    gb = 50.0
    tN = nsteps * dt
    checked = 0
    for p in range(48):
        if s["state"][p] != 1:
            continue
        na = max(0, math.ceil(s["t_act"][p] / dt - 1e-12))
        if na >= nsteps - 5:
            continue
        # activation event: boosted time na dt on the lab line z0 + beta_b t
        z0 = parts["z"][p]
        ta_lab = (na * dt / GAMMA + BETA * z0) / (1.0 - BETA * bb)
        za_lab = z0 + bb * ta_lab
        gq = math.sqrt(1 + s["ux"][p] ** 2 + s["uy"][p] ** 2 + s["uz"][p] ** 2)
        g_lab = GAMMA * (gq + BETA * s["uz"][p])
        z_lab = GAMMA * (s["z"][p] + BETA * tN)
        gain = g_lab - gb
        expect = -ez * (z_lab - za_lab)
        assert gain > 1.0
        # u lags the position by half a step: at most one boosted step of work, GAMMA (1 +
        # BETA) |E_z| dt in the lab
        assert abs(gain - expect) <= GAMMA * (1 + BETA) * abs(ez) * dt
        checked += 1
    assert checked >= 10


# ---------------------------------------------------------------------------------------
# deposit of frozen and active particles (Sec. 3.1.1: the current comes from both)
# ---------------------------------------------------------------------------------------

def test_frozen_and_active_deposit_conserves_charge():
    cfg, beam, parts = beam_scene(n=48, periodic=True, test_only=0, weight=0.02, spread=0.01, angle=2e-3,
                                  filter_npass=2, filter_compensate=1)
    o = Oracle(cfg)
    o.add_beam(beam, parts)
    r0 = o.gauss_residual()
    scale = np.abs(r0).max()
    assert scale > 0.0
    states = set()
    for _ in range(6):
        o.step(8)
        states |= set(o.beam()["state"].astype(int).tolist())
        drift = np.abs(o.gauss_residual() - r0).max()
        assert drift <= 1e-11 * scale
    assert {0, 1} <= states
    assert np.abs(o.field("Jz")).max() > 0.0


def test_test_beam_leaves_the_fields_untouched():
    # test particles only (the paper's LPA runs): with a plasma and a laser, a test beam
    # changes no field value
    w = pi.small_boosted(real="f64")
    runs = []
    for with_beam in (False, True):
        o = Oracle.from_workload(w)
        if with_beam:
            parts = pi.beam_lab(32, x_center_um=0.5 * w["config"]["nx"] * w["config"]["dx_um"],
                                z_center_um=-5.0, gamma_b=30.0, seed=9)
            o.add_beam(dict(beta_b=_beta(30.0), z_inj_um=5.0, test_only=1), parts)
        o.step(12)
        runs.append([o.field(f) for f in ("Ex", "Ez", "By", "Jx", "Jz")])
    for a, b in zip(*runs):
        assert np.array_equal(a, b)
