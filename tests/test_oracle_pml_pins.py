"""Pins of the PML coefficients (Appendix II): the standard layer and the modified
coefficients sigma*.

The paper prints sigma*_i = (xi_{i+1/2} - 1/xi_i)/delta, which is negative wherever sigma > 0, so
the formula is garbled.  The oracle reads the modified coefficients as the layer matched half cell
by half cell: the curl coefficient of the value at half-grid position p is dt kappa(p) with
kappa(p + 1/2) kappa(p) = xi(p) walking outwards (kappa = 1 inside).  That reading is pinned by
what defines it and by what the paper reports for it:
  * at normal incidence and c dt = delta the matched layer reflects nothing (the standard one
    does), which is the property the recursion is derived from;
  * in the paper's test -- a pulse with the Harris profile against an 8-cell layer with
    sigma = (4/delta)(i/5)^2 -- the modified coefficients reflect much less than the standard ones
    (the paper reports an order of magnitude);
  * where sigma = 0 both layers are the same scheme.
"""
import numpy as np
import pytest

import pic_inputs as pi
from oracle import Oracle


def _plane_wave_residue(kind):
    # x-uniform pulse E_x = B_y = f(z - t) towards the upper layer; dx >> dz puts the 2D Courant
    # limit at c dt = dz (to 5e-9)
    dz, nz = 0.1, 160
    cfg = pi.make_config(4, nz, 1e4 * dz, dz, pml_cells=10, periodic_x=1, periodic_z=0, cfl_fraction=1.0,
                         pml_kind=kind)
    o = Oracle(cfg)
    i = o.info()
    dt, P = i["dt"], i["pml_z"]
    Sz, Sx = o.shape
    z_node = (np.arange(Sz) - P) * dz
    f = lambda z: np.exp(-((z - 8.0) / 1.0) ** 2)  # noqa: E731  far from both layers at t = 0
    o.set_field("Ex", np.repeat(f(z_node)[:, None], Sx, 1))
    # B^{-1/2} at the half nodes: the same pulse half a step earlier
    o.set_field("By", np.repeat(f(z_node + 0.5 * dz + 0.5 * dt)[:, None], Sx, 1))
    o.step(206)          # the pulse has entered the layer; a reflection would be back inside
    return np.abs(o.field("Ex")[P:P + nz]).max()


def test_matched_layer_reflects_nothing_at_normal_incidence():
    std, mod = _plane_wave_residue(0), _plane_wave_residue(1)
    assert std > 1e-5          # the standard graded layer reflects
    assert mod < 1e-10         # the matched one only round-off


def _harris_run(kind, ck, n, cfl, steps=220, P=8, L=25.0):
    cfg = pi.make_config(n, n, 1.0, 1.0, pml_cells=P, periodic_x=0, periodic_z=0, ck=ck, cfl_fraction=cfl,
                         pml_kind=kind)
    o = Oracle(cfg)
    Sz, Sx = o.shape
    x = np.arange(Sx) - P
    X, Z = np.meshgrid(x, x)
    r = np.hypot(X - n / 2, Z - n / 2)
    s = 0.5 + r / L
    # the Harris profile (10 - 15 cos 2 pi s + 6 cos 4 pi s - cos 6 pi s)/32 as a radial bump
    h = (10 - 15 * np.cos(2 * np.pi * s) + 6 * np.cos(4 * np.pi * s) - np.cos(6 * np.pi * s)) / 32
    h[r >= L / 2] = 0.0
    o.set_field("Ey", h)
    o.step(steps)
    return o.field("Ey")


@pytest.mark.parametrize("ck,cfl,gain", [("yee", 0.99, 3.0), ("ck", 0.95, 10.0)])
def test_modified_coefficients_reflect_less_in_the_papers_pml_test(ck, cfl, gain):
    # a 200 x 200 box against a 500 x 500 reference whose layer is still out of reach.  CK runs at
    # 0.95 of its Courant limit: at 0.99 the modified layer grows without bound after ~500 steps
    # (the library rejects that combination)
    n, big, P = 200, 500, 8
    ref = _harris_run(0, ck, big, cfl)
    off = (big - n) // 2
    sub = ref[off:off + n + 2 * P + 1, off:off + n + 2 * P + 1][P:P + n, P:P + n]
    res = [np.abs(_harris_run(k, ck, n, cfl)[P:P + n, P:P + n] - sub).max() for k in (0, 1)]
    assert res[0] > 1e-5
    assert res[0] / res[1] >= gain, res


def test_layers_agree_where_sigma_vanishes():
    # a periodic box (no layer anywhere) from a random field state: both kinds step identically
    cfg = pi.make_config(24, 40, 0.1, 0.1, pml_cells=0, periodic_x=1, periodic_z=1, ck="ck", theta=0.1)
    runs = []
    for kind in (0, 1):
        o = Oracle(dict(cfg, pml_kind=kind))
        for q, name in enumerate(("Ex", "Ey", "Ez", "Bx", "By", "Bz")):
            o.set_field(name, pi.random_field(o.shape, 30 + q))
        o.step(5)
        runs.append([o.field(n) for n in ("Ex", "Ey", "Ez", "Bx", "By", "Bz")])
    for a, b in zip(*runs):
        assert np.abs(a).max() > 1e-3
        assert np.array_equal(a, b)
