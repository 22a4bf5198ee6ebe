"""Pins of the learned-filter oracle (oracle/lfilter.py) against what does not depend on it:
the closed-form gain of the bilinear filter (Sec. 4.1), the C oracle's bilinear filter, direct
2D convolution of the layer kernels, finite differences and the Adam recursion."""
import math

import numpy as np
import pytest

import pic_inputs as pi
from oracle import Oracle
from oracle import lfilter as L


def _g(alpha, k):
    # gain of one 3-point pass phi <- alpha phi + (1 - alpha)(phi_-1 + phi_+1)/2 (Sec. 4.1)
    return alpha + (1 - alpha) * np.cos(k)


@pytest.mark.parametrize("npass,comp", [(4, True), (1, False), (2, True), (5, False)])
def test_plain_factorisation_has_the_bilinear_gain(npass, comp):
    p = L.plain_filter_params(npass, comp)
    k = np.linspace(-math.pi, math.pi, 41)
    kx, ky = np.meshgrid(k, k)
    G = L.transfer(p, kx, ky)
    g1 = lambda kk: _g(0.5, kk) ** npass * (_g(npass / 2 + 1, kk) if comp else 1.0)  # noqa: E731
    assert np.abs(G - g1(kx) * g1(ky)).max() < 1e-14


def test_plain_factorisation_matches_the_c_oracle_filter():
    # the C oracle's own 4-pass + compensation filter on a periodic grid
    cfg = pi.make_config(24, 40, 0.1, 0.1, periodic_x=1, periodic_z=1, pml_cells=0,
                         filter_npass=4, filter_compensate=1, real="f64", seed=3)
    o = Oracle(cfg)
    rng = np.random.default_rng(5)
    j = rng.normal(size=o.shape)
    o.set_field("Jy", j)
    o.stage("filter")
    ref = o.field("Jy")
    out = L.forward(L.plain_filter_params(4, True), j[None], periodic=(True, True))[0]
    assert np.abs(out - ref).max() < 1e-13 * np.abs(ref).max()


def test_impulse_response_is_the_composed_kernel():
    rng = np.random.default_rng(1)
    p = rng.normal(scale=0.2, size=L.NPARAM).astype(np.float32)
    img = np.zeros((1, 32, 32))
    img[0, 16, 16] = 1.0
    out = L.forward(p, img, periodic=(True, True))[0]
    K = L.composed_kernel(p)
    # out(p) = sum_o K[o] in(p + o): the delta at c lands at p = c - o
    resp = np.zeros((13, 13))
    for dy in range(-6, 7):
        for dx in range(-6, 7):
            resp[dy + 6, dx + 6] = out[16 - dy, 16 - dx]
    assert np.abs(resp - K).max() < 1e-12 * np.abs(K).max()
    mask = np.ones((32, 32), bool)
    mask[10:23, 10:23] = False
    assert np.abs(out[mask]).max() == 0.0


def test_linear_and_shift_invariant():
    rng = np.random.default_rng(2)
    p = rng.normal(scale=0.2, size=L.NPARAM).astype(np.float32)
    a, b = rng.normal(size=(2, 1, 20, 28))
    f = lambda x: L.forward(p, x, periodic=(True, True))  # noqa: E731
    assert np.allclose(f(2.0 * a - 3.0 * b), 2.0 * f(a) - 3.0 * f(b), rtol=0, atol=1e-12)
    assert np.allclose(f(np.roll(a, (3, -5), axis=(1, 2))), np.roll(f(a), (3, -5), axis=(1, 2)),
                       rtol=0, atol=1e-12)


@pytest.mark.parametrize("periodic", [(False, False), (True, False), (True, True)])
def test_gradient_matches_finite_differences(periodic):
    rng = np.random.default_rng(3)
    p = rng.normal(scale=0.3, size=L.NPARAM)
    x = rng.normal(size=(2, 9, 11))
    y = rng.normal(size=(2, 9, 11))
    loss, g = L.loss_and_grad(p, x, y, margin=1, periodic=periodic, quantize=False)
    idx = rng.choice(L.NPARAM, 40, replace=False)
    h = 1e-3
    for i in idx:
        e = np.zeros(L.NPARAM)
        e[i] = h
        lp = L.loss_and_grad(p.astype(np.float64) + e, x, y, 1, periodic, quantize=False)[0]
        lm = L.loss_and_grad(p.astype(np.float64) - e, x, y, 1, periodic, quantize=False)[0]
        assert g[i] == pytest.approx((lp - lm) / (2 * h), rel=2e-4, abs=1e-9)
    assert loss > 0


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(4)
    w = rng.normal(size=50)
    g = rng.normal(size=50)
    w1, m, v = L.adam(w, np.zeros(50), np.zeros(50), g, 1, lr=0.01, eps=1e-8)
    # bias-corrected first moments are g and g^2: the step is -lr g / (|g| + eps)
    assert np.allclose(w1 - w, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    w2, m2, v2 = L.adam(w1, m, v, g, 2, lr=0.01, eps=0.0)
    assert np.allclose(w2 - w1, -0.01 * np.sign(g), rtol=1e-12, atol=0)   # same g: same step


def test_bf16_rounding_is_round_to_nearest_even():
    # values on and around the 8-bit significand grid of [1, 2): spacing 2^-7
    ulp = 2.0 ** -7
    x = np.array([1.0, 1.0 + ulp / 2, 1.0 + 3 * ulp / 2, 1.0 + ulp / 2 + 2 ** -20, -1.0 - ulp / 4])
    assert list(L.bf16(x)) == [1.0, 1.0, 1.0 + 2 * ulp, 1.0 + ulp, -1.0]


def test_any_weights_commute_with_the_staggered_divergence():
    # Gauss's law survives filtering (Sec. 4.2.2) when div(F J) = F(div J): J_x lives on
    # (i+1/2, k), J_z on (i, k+1/2), div J on nodes; periodic grid, random weights
    rng = np.random.default_rng(6)
    p = rng.normal(scale=0.2, size=L.NPARAM).astype(np.float32)
    jx, jz = rng.normal(size=(2, 1, 24, 30))            # [img, z, x]
    div = lambda ax, az: (ax - np.roll(ax, 1, axis=2)) + (az - np.roll(az, 1, axis=1))  # noqa: E731
    f = lambda a: L.forward(p, a, periodic=(True, True))  # noqa: E731
    lhs = div(f(jx), f(jz))
    rhs = f(div(jx, jz))
    assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(rhs).max()


@pytest.mark.parametrize("npass,comp", [(4, True), (1, False), (2, True)])
def test_library_factorisation_equals_the_oracle_one(npass, comp):
    # the package computes the same parameters on its own (it may not import the oracle)
    import paper_1009_2727_amd as P
    assert np.array_equal(P.bilinear_factor_params(npass, comp), L.plain_filter_params(npass, comp))
