"""GPU (HIP, gfx950) 3D path against the 3D FP64 oracle, element by element, through the C ABI.

Errors are measured as in the 2D parity tests: max |GPU - oracle| over the grid divided by
the physical scale of the field group (the emitted laser amplitude for E and B, the larger
of the plasma and antenna-sheet current densities for J), never below the field's own
maximum.  Tolerances: FP64 1e-10 (summation order of the atomics only), FP32 1e-5.
"""
import numpy as np
import pytest

import pic_inputs as pi
from oracle.pic3 import Oracle3

gpu = pytest.mark.gpu
FIELDS = ["Ex", "Ey", "Ez", "Bx", "By", "Bz", "Jx", "Jy", "Jz"]


def _sim(w, **kw):
    from paper_1009_2727_amd import Sim
    return Sim.from_workload(w, **kw)


def field_scales(ref):
    i = ref.info()
    cfg = ref.config
    g, b = i["gamma"], i["beta"]
    e_emit = i["e0_norm"] / ((1 + b) * g) if i["e0_norm"] else 0.0
    j_plasma = i["n0_norm"] * g
    j_ant = 2 * i["e0_norm"] / g / cfg["dz_um"] if i["e0_norm"] else 0.0
    return {"E": e_emit, "B": e_emit, "J": max(j_plasma, j_ant)}


def compare_fields3(sim, ref, tol, names=FIELDS):
    floor = field_scales(ref)
    a = {n: sim.field(n) for n in names}
    b = {n: ref.field(n) for n in names}
    scale = {}
    for n in names:
        scale[n[0]] = max(scale.get(n[0], 0.0), np.abs(b[n]).max(), floor[n[0]])
    errs = {n: float(np.abs(a[n] - b[n]).max() / scale[n[0]]) if scale[n[0]] > 0 else float(np.abs(a[n]).max())
            for n in names}
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, f"field mismatch above {tol:g}: {bad} (all: {errs})"
    return errs


def compare_particles3(sim, ref, xtol, utol):
    a, b = sim.particles(0), ref.particles(0)
    assert len(a["id"]) == len(b["id"]), (len(a["id"]), len(b["id"]))
    ia, ib = np.argsort(a["id"], kind="stable"), np.argsort(b["id"], kind="stable")
    np.testing.assert_array_equal(a["id"][ia], b["id"][ib])
    for k, tol in (("x", xtol), ("y", xtol), ("z", xtol), ("ux", utol), ("uy", utol), ("uz", utol)):
        d = np.abs(a[k][ia] - b[k][ib])
        scale = 1.0 if k in ("x", "y", "z") else max(np.abs(b[k]).max(), 1.0)
        assert d.max() <= tol * scale, (k, d.max())


@gpu
def test_3d_initial_plasma_bitwise():
    w = pi.small_boosted3(real="f64", nx=10, ny=8, nz=40, ppc=2, preload=True)
    sim, ref = _sim(w), Oracle3.from_workload(w)
    a, b = sim.particles(0), ref.particles(0)
    ia, ib = np.argsort(a["id"]), np.argsort(b["id"])
    np.testing.assert_array_equal(a["id"][ia], b["id"][ib])
    for k in ("x", "y", "w"):
        np.testing.assert_array_equal(a[k][ia], b[k][ib])
    np.testing.assert_allclose(a["z"][ia], b["z"][ib], rtol=0, atol=1e-12)


@gpu
@pytest.mark.parametrize("real,tol,xtol", [("f64", 1e-10, 1e-9), ("f32", 1e-5, 1e-5)])
def test_3d_boosted_matches_oracle(real, tol, xtol):
    # C3-shaped: boosted gamma = 30, window, PML on every face, CK2 + Friedman, 4 + comp filter,
    # rigid ions, antenna, on a grid smaller than one particle tile
    w = pi.small_boosted3(real=real, nx=10, ny=8, nz=40, ppc=2)
    sim, ref = _sim(w, sort_every=7), Oracle3.from_workload(w)
    sim.step(24)
    ref.step(24)
    assert sim.sync_status() == 0
    assert sim.info()["shift"] == ref.info()["shift"] > 0
    compare_fields3(sim, ref, tol)
    compare_particles3(sim, ref, xtol, xtol)


@gpu
@pytest.mark.parametrize("real,tol", [("f64", 1e-12), ("f32", 2e-6)])
def test_3d_random_state_single_step(real, tol):
    nx, ny, nz = 11, 9, 13   # ragged
    d = (0.1, 0.12, 0.09)
    cfg = pi.make_config3(nx, ny, nz, *d, periodic_x=1, periodic_y=1, periodic_z=1, pml_cells=0,
                          ck="ck2", theta=0.3, filter_npass=2, filter_compensate=1, real=real, seed=5)
    from paper_1009_2727_amd import Sim
    sim = Sim(cfg, capacity=4000)
    ref = Oracle3(cfg)
    for k, name in enumerate(["Ex", "Ey", "Ez", "Bx", "By", "Bz", "Exo", "Eyo", "Ezo", "Exb", "Eyb", "Ezb"]):
        f = pi.random_field(ref.shape, seed=100 + k, amp=0.5)
        ref.set_field(name, f)
        sim.set_field(name, f)
    p = pi.random_electrons3(3000, nx, ny, nz, d, seed=11, umax=3.0, margin=0.0)
    ref.set_electrons(p)
    sim.load_electrons(p)
    ref.step(1)
    sim.step(1)
    for n in FIELDS:
        a, b = sim.field(n), ref.field(n)
        assert np.abs(a - b).max() <= tol * max(np.abs(b).max(), 1.0), n
    compare_particles3(sim, ref, 1e-9 if real == "f64" else 1e-5, 1e-10 if real == "f64" else 1e-5)


@gpu
def test_3d_vacuum_pml_matches_oracle():
    # fields only: a solenoidal pulse through the split PML on all faces
    w = pi.small_boosted3(real="f64", nx=10, ny=8, nz=30)
    sim, ref = _sim(w, plasma=False, laser=False), Oracle3.from_workload(w, plasma=False, laser=False)
    Sz, Sy, Sx = ref.shape
    Z, Y, X = np.meshgrid(np.arange(Sz), np.arange(Sy), np.arange(Sx), indexing="ij")
    f = np.exp(-((X - Sx / 2) ** 2 + (Z - Sz / 2) ** 2) / 8.0)
    for o in (sim, ref):
        o.set_field("By", f)
    sim.step(40)
    ref.step(40)
    for n in ("Ex", "Ey", "Ez", "Bx", "By", "Bz"):
        a, b = sim.field(n), ref.field(n)
        assert np.abs(a - b).max() <= 1e-11 * np.abs(f).max(), n


@gpu
@pytest.mark.parametrize("real,tol", [("f64", 1e-11), ("f32", 1e-5)])
def test_3d_spreading_segments_match_oracle(real, tol):
    # fast random electrons on a periodic box with no re-sort: the segments' boxes grow each
    # step until they exceed the LDS box, and particles wrapping round a periodic face widen
    # theirs at once, so both the staged and the HBM forms of the push run
    nx, ny, nz = 12, 10, 22
    d = (0.1, 0.11, 0.09)
    cfg = pi.make_config3(nx, ny, nz, *d, periodic_x=1, periodic_y=1, periodic_z=1, pml_cells=0,
                          ck="ck2", theta=0.2, filter_npass=1, filter_compensate=1, real=real, seed=6)
    from paper_1009_2727_amd import Sim
    sim = Sim(cfg, capacity=6000, sort_every=1000)
    ref = Oracle3(cfg)
    for k, name in enumerate(["Ex", "Ey", "Ez", "Bx", "By", "Bz"]):
        f = pi.random_field(ref.shape, seed=300 + k, amp=0.2)
        ref.set_field(name, f)
        sim.set_field(name, f)
    p = pi.random_electrons3(5000, nx, ny, nz, d, seed=12, umax=4.0, margin=0.0)
    ref.set_electrons(p)
    sim.load_electrons(p)
    ref.step(8)
    sim.step(8)
    assert sim.sync_status() == 0
    for n in FIELDS:
        a, b = sim.field(n), ref.field(n)
        assert np.abs(a - b).max() <= tol * max(np.abs(b).max(), 1.0), n
    compare_particles3(sim, ref, 1e-9 if real == "f64" else 2e-5, 1e-9 if real == "f64" else 2e-5)


@gpu
def test_3d_full_size_faraday_and_sampled_electrons_match_oracle():
    # The 3D workload at its full size (128x128x1024, 8 ppc, 134 M electrons) in the benchmark's
    # launch configuration (default tiles, sort every 80 steps).  After three steps the fields
    # are replaced by random ones (both sides), one more step is taken, and the oracle repeats
    # it from the same state: every cell of B^{n+1/2} (Faraday with Friedman and the split PML)
    # and a block of 65536 electron slots from the middle of the window (gather and push) are
    # compared.  The current, which sums all 134 M electrons, is covered by the smaller cases.
    from paper_1009_2727_amd import Sim, PARTICLE_BLOCK
    w = pi.c3(real="f32", preload=True)
    sim = Sim.from_workload(w, sort_every=80)
    sim.step(3)
    i0 = sim.info()
    ref = Oracle3(w["config"])
    ref.set_clock(i0["step"], i0["time"], i0["shift"], i0["next_row"])
    for k, name in enumerate(["Ex", "Ey", "Ez", "Bx", "By", "Bz", "Exo", "Eyo", "Ezo", "Exb", "Eyb", "Ezb"]):
        f = pi.random_field(ref.shape, seed=500 + k, amp=1.0)
        sim.set_field(name, f)
        ref.set_field(name, f)
        del f
    for name in ["Exs", "Eys", "Ezs", "Bxs", "Bys", "Bzs"]:
        ref.set_field(name, sim.field(name))
    blk = int(sim.counts()[2]) // PARTICLE_BLOCK // 2
    before = sim.particle_block(0, blk)
    assert len(before["id"]) > PARTICLE_BLOCK // 2
    ref.set_electrons(before)
    sim.step(1)
    assert sim.sync_status() == 0
    d = int(sim.info()["shift"] - i0["shift"])
    after = sim.particle_block(0, blk)
    ref.stage("faraday")
    ref.stage("particles")
    assert d >= 0
    for name in ("Bx", "By", "Bz"):
        # the GPU's step ends with the window shift: its plane k is the oracle's plane k + d
        a, b = sim.field(name), ref.field(name)
        a, b = a[:a.shape[0] - d], b[d:]
        assert np.abs(a - b).max() <= 1e-5 * np.abs(b).max(), name
        del a, b
    got = ref.particles(0)
    ia, ib = np.argsort(after["id"], kind="stable"), np.argsort(got["id"], kind="stable")
    np.testing.assert_array_equal(after["id"][ia], got["id"][ib])
    dz = w["config"]["dz_um"]
    after["z"] = after["z"] + d * dz           # the GPU's positions are rebased into the next window
    for k in ("x", "y", "z"):
        cell = w["config"]["d" + k + "_um"]
        assert np.abs(after[k][ia] - got[k][ib]).max() <= 1e-5 * cell, k
    for k in ("ux", "uy", "uz"):
        scale = max(np.abs(got[k]).max(), 1.0)
        assert np.abs(after[k][ia] - got[k][ib]).max() <= 1e-5 * scale, k


# ---------------------------------------------------------------------------------------
# diagnostics and options of the 3D path against the oracle
# ---------------------------------------------------------------------------------------

@gpu
def test_3d_gauss_residual_matches_oracle_and_holds():
    # div E - F[rho] with the deposit's shape and the step's filter (Sec. 4.2.2): the GPU's
    # residual equals the oracle's, and the charge-conserving deposit keeps it constant
    w = pi.small_boosted3(real="f64", nx=12, ny=10, nz=48, ppc=2)
    sim, ref = _sim(w, sort_every=5), Oracle3.from_workload(w)
    # scale: the charge density of one antenna sheet (the neutral pairs cancel at t = 0)
    rho = ref.info()["antenna_weight"] / w["config"]["dx_um"] ** 3
    g0 = sim.gauss_residual()
    np.testing.assert_allclose(g0, ref.gauss_residual(), rtol=0, atol=1e-11 * rho)
    sim.step(20)
    ref.step(20)
    assert ref.info()["shift"] > 5
    g1, r1 = sim.gauss_residual(), ref.gauss_residual()
    np.testing.assert_allclose(g1, r1, rtol=0, atol=1e-10 * rho)
    P = 10      # nodes clear of the non-periodic edges by the shape and filter reach
    inner = (slice(P + 10, P + 48 - 10), slice(P + 3, P + 10 - 3), slice(P + 3, P + 12 - 3))
    assert np.abs(g1 - g0)[inner].max() <= 1e-11 * rho
    assert np.abs(sim.field("Ez")).max() > 0


@gpu
def test_3d_gauss_fp32():
    w = pi.small_boosted3(real="f32", nx=12, ny=10, nz=48, ppc=2)
    ref = Oracle3.from_workload(pi.small_boosted3(real="f64", nx=12, ny=10, nz=48, ppc=2))
    sim = _sim(w, sort_every=5)
    g0 = sim.gauss_residual()
    sim.step(24)
    ref.step(24)
    g1 = sim.gauss_residual()
    rho = ref.info()["antenna_weight"] / w["config"]["dx_um"] ** 3
    P = 10
    inner = (slice(P + 10, P + 48 - 10), slice(P + 3, P + 10 - 3), slice(P + 3, P + 12 - 3))
    assert np.abs(g1 - g0)[inner].max() <= 1e-5 * rho


@gpu
def test_3d_stations_and_energy_match_oracle():
    w = pi.small_boosted3(real="f64", nx=12, ny=10, nz=48, ppc=2)
    g, d = w["config"]["gamma_boost"], w["config"]["dz_um"]
    zs = [g * 20 * d, g * 30 * d]
    sim = _sim(w, stations=zs)
    ref = Oracle3.from_workload(w, stations=zs)
    sim.step(24)
    ref.step(24)
    for q in range(2):
        a, b = sim.station(q), ref.station(q)
        assert a.shape == b.shape and a.shape[0] > 5
        np.testing.assert_allclose(a, b, rtol=1e-9, atol=1e-12 * max(np.abs(b).max(), 1))
    np.testing.assert_allclose(sim.energy(), ref.energy(), rtol=1e-10)


@gpu
@pytest.mark.parametrize("real,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_3d_stride_filter_and_y_polarisation(real, tol):
    w = pi.small_boosted3(real=real, nx=12, ny=10, nz=48, ppc=2)
    w["config"]["filter_strides"] = 0b11                         # S(1:2)
    w["laser"]["pol"] = 1
    sim, ref = _sim(w, sort_every=7), Oracle3.from_workload(w)
    sim.step(20)
    ref.step(20)
    assert np.abs(ref.field("Ey")).max() > np.abs(ref.field("Ex")).max()
    compare_fields3(sim, ref, tol)
    np.testing.assert_allclose(sim.antenna(), ref.antenna(), atol=1e-12)


@gpu
@pytest.mark.parametrize("real,tol", [("f64", 1e-10), ("f32", 1e-5)])
def test_3d_momentum_gather_and_vay_match_oracle(real, tol):
    w = pi.small_boosted3(real=real, nx=12, ny=10, nz=48, ppc=2)
    w["config"]["gather_kind"] = 1
    w["config"]["pusher"] = 1
    sim, ref = _sim(w, sort_every=7), Oracle3.from_workload(w)
    sim.step(20)
    ref.step(20)
    compare_fields3(sim, ref, tol)
    if real == "f64":
        compare_particles3(sim, ref, 1e-9, 1e-9)


@gpu
def test_3d_variants_random_state_single_step():
    nx, ny, nz = 11, 9, 13
    d = (0.1, 0.12, 0.09)
    cfg = pi.make_config3(nx, ny, nz, *d, periodic_x=1, periodic_y=1, periodic_z=1, pml_cells=0, ck="ck2",
                          theta=0.3, filter_npass=2, filter_compensate=1, real="f64", seed=5, gather_kind=1,
                          pusher=1)
    from paper_1009_2727_amd import Sim
    sim = Sim(cfg, capacity=4000)
    ref = Oracle3(cfg)
    for k, name in enumerate(["Ex", "Ey", "Ez", "Bx", "By", "Bz", "Exo", "Eyo", "Ezo", "Exb", "Eyb", "Ezb"]):
        f = pi.random_field(ref.shape, seed=400 + k, amp=0.5)
        ref.set_field(name, f)
        sim.set_field(name, f)
    p = pi.random_electrons3(3000, nx, ny, nz, d, seed=14, umax=3.0, margin=0.0)
    ref.set_electrons(p)
    sim.load_electrons(p)
    ref.step(1)
    sim.step(1)
    for n in FIELDS:
        a, b = sim.field(n), ref.field(n)
        assert np.abs(a - b).max() <= 1e-12 * max(np.abs(b).max(), 1.0), n
    compare_particles3(sim, ref, 1e-9, 1e-10)


@gpu
def test_3d_modified_pml_coefficients_match_oracle():
    # the vacuum pulse through the layer with the modified coefficients (Appendix II sigma*)
    w = pi.small_boosted3(real="f64", nx=10, ny=8, nz=30)
    w["config"]["pml_kind"] = 1
    sim, ref = _sim(w, plasma=False, laser=False), Oracle3.from_workload(w, plasma=False, laser=False)
    Sz, Sy, Sx = ref.shape
    Z, Y, X = np.meshgrid(np.arange(Sz), np.arange(Sy), np.arange(Sx), indexing="ij")
    f = np.exp(-((X - Sx / 2) ** 2 + (Z - Sz / 2) ** 2) / 8.0)
    for o in (sim, ref):
        o.set_field("By", f)
    sim.step(40)
    ref.step(40)
    for n in ("Ex", "Ey", "Ez", "Bx", "By", "Bz"):
        a, b = sim.field(n), ref.field(n)
        assert np.abs(a - b).max() <= 1e-11 * np.abs(f).max(), n
