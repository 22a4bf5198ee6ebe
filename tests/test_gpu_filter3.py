"""The 3D current filter against the FP64 oracle at every reach the one-launch kernel takes.

The n-pass bilinear filter with or without compensation (Sec. 4.1) is applied along x, y and z;
with unit strides and a reach of 1..6 the GPU runs it as one launch (the composed stencil on the
oddly continued line, a register ring along z), and on boxes shorter than 2 reach + 3 cells along
a non-periodic axis it keeps the pass-by-pass line kernels.  One step from random fields and
random electrons, then E, B and the filtered current are compared cell by cell: on a box with
PML on every face (non-periodic, every component's last half node copied), on a periodic box, and
on a box whose x axis is too short for the larger reaches.  Tolerances as in the other 3D parity
tests (FP64 1e-11, FP32 2e-6 of the field scale).
"""
import numpy as np
import pytest

import pic_inputs as pi
from oracle.pic3 import Oracle3

gpu = pytest.mark.gpu
NAMES = ["Ex", "Ey", "Ez", "Bx", "By", "Bz", "Jx", "Jy", "Jz"]

GEOMETRIES = {
    # (nx, ny, nz), pml cells, periodic flags
    "pml": ((12, 10, 18), 4, (0, 0, 0)),
    "periodic": ((11, 9, 13), 0, (1, 1, 1)),
    # stored x cells 2 + 2*4 + 1 = 11: reaches 1..4 fused, 5 and 6 (11 < 2 reach + 3) by the line kernels
    "short": ((2, 10, 16), 4, (0, 1, 0)),
}
MARGIN = {"pml": 1.5, "periodic": 0.0, "short": 0.3}


def _case(geom, npass, comp, real):
    (nx, ny, nz), pml, per = GEOMETRIES[geom]
    d = (0.1, 0.12, 0.09)
    cfg = pi.make_config3(nx, ny, nz, *d, pml_cells=pml, periodic_x=per[0], periodic_y=per[1],
                          periodic_z=per[2], ck="ck2", theta=0.2, filter_npass=npass,
                          filter_compensate=comp, real=real, seed=21)
    from paper_1009_2727_amd import Sim
    sim = Sim(cfg, capacity=6000)
    ref = Oracle3(cfg)
    for k, name in enumerate(["Ex", "Ey", "Ez", "Bx", "By", "Bz", "Exo", "Eyo", "Ezo", "Exb", "Eyb", "Ezb"]):
        f = pi.random_field(ref.shape, seed=700 + k, amp=0.4)
        ref.set_field(name, f)
        sim.set_field(name, f)
    p = pi.random_electrons3(4000, nx, ny, nz, d, seed=23, umax=3.0, margin=MARGIN[geom])
    ref.set_electrons(p)
    sim.load_electrons(p)
    return sim, ref


@gpu
@pytest.mark.parametrize("geom", list(GEOMETRIES))
@pytest.mark.parametrize("npass,comp", [(1, 0), (2, 1), (3, 1), (4, 1), (5, 1), (6, 0)])
def test_3d_filter_reaches_match_oracle(geom, npass, comp):
    sim, ref = _case(geom, npass, comp, "f64")
    ref.step(1)
    sim.step(1)
    assert sim.sync_status() == 0
    for n in NAMES:
        a, b = sim.field(n), ref.field(n)
        assert np.abs(a - b).max() <= 1e-11 * max(np.abs(b).max(), 1.0), (n, float(np.abs(a - b).max()))


@gpu
@pytest.mark.parametrize("geom", ["pml", "periodic"])
def test_3d_filter_fp32_matches_oracle(geom):
    sim, ref = _case(geom, 4, 1, "f32")
    ref.step(1)
    sim.step(1)
    assert sim.sync_status() == 0
    for n in NAMES:
        a, b = sim.field(n), ref.field(n)
        assert np.abs(a - b).max() <= 2e-6 * max(np.abs(b).max(), 1.0), (n, float(np.abs(a - b).max()))
