"""Host-side pieces of the learned filter's training set (no GPU): the patch power spectrum that
shapes the spectral term, and which current components a 2D run never deposits."""
import numpy as np

import pic_inputs as pi
from paper_1009_2727_amd import filter_training as ft


def test_patch_spectrum_of_a_plane_wave_sits_on_its_mode():
    P = ft.PATCH
    z, x = np.meshgrid(np.arange(3 * P + 5), np.arange(2 * P + 7), indexing="ij")
    f = np.cos(2 * np.pi * (5 * z + 3 * x) / P + 0.3)
    s = ft.patch_spectrum(f)
    assert s.shape == (P, P)
    peak = {(5, 3), (P - 5, P - 3)}
    off = [s[k, i] for k in range(P) for i in range(P) if (k, i) not in peak]
    assert max(off) < 1e-18 * s.max()
    # Parseval: each window holds P^2 / 2 of cos^2, so the mean spectrum sums to P^4 / 2
    np.testing.assert_allclose(s.sum(), P ** 4 / 2, rtol=1e-12)
    np.testing.assert_allclose(s[5, 3], s[P - 5, P - 3], rtol=1e-12)


def test_patch_spectrum_ignores_the_ragged_edge():
    P = ft.PATCH
    rng = np.random.default_rng(4)
    f = rng.normal(size=(2 * P, 2 * P))
    g = np.pad(f, ((0, P - 1), (0, 5)), constant_values=1e6)
    np.testing.assert_array_equal(ft.patch_spectrum(f), ft.patch_spectrum(g))


def test_zero_current_components():
    assert ft._zero_component(pi.c5_wake(), "y")          # x-polarised laser
    assert ft._zero_component(pi.c5_growth(), "y")        # no laser
    assert not ft._zero_component(pi.c5_wake(), "x")
    w = pi.c5_wake()
    w["laser"]["pol"] = 1
    assert not ft._zero_component(w, "y")


def test_lab_growth_family_is_the_wake_run_on_the_ck_solver():
    w, g = pi.c5_wake(), pi.c5_growth_lab()
    assert (g["config"]["ck_alpha"], g["config"]["ck_beta"]) == pi.CK_SETS["ck"][:2]
    assert w["config"]["ck_beta"] == 0.0
    for k in ("nx", "nz", "dx_um", "dz_um", "cfl_fraction", "gamma_boost", "filter_npass"):
        assert g["config"][k] == w["config"][k], k
    assert g["plasma"] == w["plasma"] and g["laser"] == w["laser"] and g["steps"] == 600


def test_linear_phase_ends_where_the_log_rise_saturates():
    # exponential growth at 0.08 per step from step 20 to 320, then flat: the window starts at the
    # second sample and ends at the first sample past 80% of the rise
    t = np.arange(20.0, 601.0, 20.0)
    le = np.where(t <= 320, -9.0 + 0.08 * (t - 20), -9.0 + 0.08 * 300)
    lo, hi = ft.linear_phase(t, le)
    assert lo == t[1]
    rise = 0.08 * 300
    first = t[np.argmax(le >= le.min() + 0.8 * rise)]
    assert hi == first and 240.0 <= hi <= 320.0
    sel = (t >= lo) & (t <= hi)
    np.testing.assert_allclose(np.polyfit(t[sel], le[sel], 1)[0], 0.08, rtol=1e-12)


def test_linear_phase_of_a_flat_record_keeps_a_minimal_window():
    t = np.arange(20.0, 201.0, 20.0)
    lo, hi = ft.linear_phase(t, np.full(t.shape, 3.0))
    assert lo == t[1] and hi == t[3]
