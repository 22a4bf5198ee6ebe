"""GPU beam through a lab-fixed plane (Sec. 3.1.1) against the FP64 oracle, through the C ABI.

The beam's state (positions, momenta, crossing times, frozen/active/lost) and its lab-frame
history are compared particle by particle.  Bars: FP64 runs 1e-9 (positions in um, momenta
relative to the largest) -- only the summation order of the field arrays differs; FP32 runs
(fields in FP32, the beam in FP64) 1e-4 of the momentum scale after the stated horizon.
"""
import math

import numpy as np
import pytest

import pic_inputs as pi
from oracle import Oracle

gpu = pytest.mark.gpu

GAMMA = 5.0
BETA = math.sqrt(1.0 - 1.0 / GAMMA ** 2)
KEYS = ("x", "z", "ux", "uy", "uz", "w", "t_act", "state")


def _beta(g):
    return math.sqrt(1.0 - 1.0 / (g * g))


def _sim(w, **kw):
    from paper_1009_2727_amd import Sim
    return Sim.from_workload(w, **kw)


def _field_free(n=64, periodic=False, test_only=1, weight=1e-6, spread=0.0, angle=0.0, real="f64"):
    """gamma = 5 box of 16 x 96 cells of 0.1 um; the beam centre crosses the plane at
    z_inj = 25 um at boosted time 1.5 um/c."""
    gb, z_inj, t_cross = 50.0, 25.0, 1.5
    bb = _beta(gb)
    z_c = z_inj - bb * (t_cross / GAMMA + BETA * z_inj)
    cfg = pi.make_config(16, 96, 0.1, 0.1, pml_cells=0 if periodic else 8, periodic_x=1,
                         periodic_z=1 if periodic else 0, gamma_boost=GAMMA, real=real,
                         filter_npass=2, filter_compensate=1)
    cfg.update(beam_capacity=n + 7, beam_history=200)
    parts = pi.beam_lab(n, x_center_um=0.8, z_center_um=z_c, gamma_b=gb, seed=11, energy_spread=spread,
                        angle_rms=angle, weight=weight)
    return dict(config=cfg, plasma=None, laser=None), dict(beta_b=bb, z_inj_um=z_inj, test_only=test_only), parts


def _wake(real="f64", gather_kind=0, pusher=0, n=96, test_only=1):
    """The small boosted wake case (gamma = 13, window, CK2 + Friedman, filter, PML, rigid
    ions, antenna) with a gamma_b = 50 beam whose plane starts at 70% of the window and whose
    centre crosses it at boosted time 15 um/c."""
    w = pi.small_boosted(real=real)
    cfg = w["config"]
    cfg.update(gather_kind=gather_kind, pusher=pusher, beam_capacity=n, beam_history=400)
    g = cfg["gamma_boost"]
    b = _beta(g)
    lz = cfg["nz"] * cfg["dz_um"]
    z_inj = g * 0.7 * lz
    gb, t_cross = 50.0, 15.0
    bb = _beta(gb)
    z_c = z_inj - bb * (t_cross / g + b * z_inj)
    parts = pi.beam_lab(n, x_center_um=0.5 * cfg["nx"] * cfg["dx_um"], z_center_um=z_c, gamma_b=gb, seed=12,
                        energy_spread=0.01, angle_rms=1e-3, weight=1e-4)
    return w, dict(beta_b=bb, z_inj_um=z_inj, test_only=test_only), parts


def _pair(w, beam, parts):
    sim = _sim(w)
    ref = Oracle.from_workload(w)
    sim.add_beam(beam, parts)
    ref.add_beam(beam, parts, history_cap=w["config"]["beam_history"])
    return sim, ref


def compare_beam(sim, ref, xtol, utol, htol):
    a, b = sim.beam(), ref.beam()
    assert len(a["x"]) == len(b["x"])
    np.testing.assert_array_equal(a["state"], b["state"])
    np.testing.assert_allclose(a["t_act"], b["t_act"], rtol=1e-13, atol=1e-12)
    live = b["state"] != 2
    for k in ("x", "z"):
        d = np.abs(a[k] - b[k])[live]
        assert d.max(initial=0.0) <= xtol, (k, d.max())
    us = max(np.abs(b["uz"]).max(), 1.0)
    for k in ("ux", "uy", "uz"):
        d = np.abs(a[k] - b[k])
        assert d.max() <= utol * us, (k, d.max() / us)
    ha, hb = sim.beam_history(), ref.beam_history()
    assert ha.shape == hb.shape
    np.testing.assert_array_equal(ha[:, 1], hb[:, 1])
    for c in range(2, 8):
        sc = max(np.abs(hb[:, c]).max(), 1e-300)
        d = np.abs(ha[:, c] - hb[:, c]).max() / sc
        assert d <= htol, (c, d)
    return a


@gpu
def test_field_free_beam_matches_oracle():
    w, beam, parts = _field_free()
    sim, ref = _pair(w, beam, parts)
    seen = set()
    for n in (5, 20, 35):
        sim.step(n)
        ref.step(n)
        a = compare_beam(sim, ref, 1e-9, 1e-12, 1e-12)
        seen |= set(a["state"].astype(int).tolist())
    assert {0, 1} <= seen
    assert np.abs(sim.field("Jz")).max() == 0.0      # test particles deposit nothing
    assert sim.sync_status() == 0


@gpu
def test_depositing_beam_matches_oracle_and_conserves_charge():
    w, beam, parts = _field_free(n=48, periodic=True, test_only=0, weight=0.02, spread=0.01, angle=2e-3)
    sim, ref = _pair(w, beam, parts)
    r0 = sim.gauss_residual()
    np.testing.assert_allclose(r0, ref.gauss_residual(), rtol=0, atol=1e-12 * np.abs(r0).max())
    for n in (8, 16, 24):
        sim.step(n)
        ref.step(n)
        compare_beam(sim, ref, 1e-9, 1e-11, 1e-11)
        for f in ("Ex", "Ez", "By", "Jx", "Jz", "Jy"):
            b = ref.field(f)
            sc = max(np.abs(b).max(), 1e-30)
            assert np.abs(sim.field(f) - b).max() <= 1e-10 * sc, f
        drift = np.abs(sim.gauss_residual() - r0).max()
        assert drift <= 1e-10 * np.abs(r0).max()


@gpu
@pytest.mark.parametrize("gather_kind,pusher", [(0, 0), (1, 1)])
def test_wake_test_beam_matches_oracle(gather_kind, pusher):
    w, beam, parts = _wake(gather_kind=gather_kind, pusher=pusher)
    sim, ref = _pair(w, beam, parts)
    for n in (30, 40):
        sim.step(n)
        ref.step(n)
        a = compare_beam(sim, ref, 1e-9, 1e-9, 1e-9)
    assert (a["state"] == 1).sum() > 40
    # the beam saw a field: its momenta moved off the injected values
    assert np.abs(a["ux"]).max() > 0.0
    assert sim.sync_status() == 0


@gpu
def test_wake_test_beam_fp32_fields():
    w, beam, parts = _wake(real="f32")
    sim, ref = _pair(w, beam, parts)
    sim.step(70)
    ref.step(70)
    compare_beam(sim, ref, 1e-5, 1e-4, 1e-4)


@gpu
def test_beam_argument_errors():
    from paper_1009_2727_amd import BfError, Sim
    w, beam, parts = _field_free(n=8)
    sim = Sim.from_workload(w)
    big = {k: np.concatenate([v] * 2) for k, v in parts.items()}   # 16 > capacity 15
    with pytest.raises(BfError):
        sim.add_beam(beam, big)
    bad = dict(parts)
    bad["uz"] = -parts["uz"]
    with pytest.raises(BfError):
        sim.add_beam(beam, bad)
    with pytest.raises(BfError):
        sim.add_beam(dict(beam, beta_b=1.0), parts)
    sim2 = Sim.from_workload(w)
    sim2.add_beam(beam, parts)     # a rejected call left the first handle usable
    sim.add_beam(beam, parts)
    assert len(sim.beam()["x"]) == 8
