"""GPU parity of the learned current filter (MFMA kernels through the C ABI) against the FP64
oracle in oracle/lfilter.py, and of a PIC run using it against the bilinear-filter run.

Tolerance of the forward pass, derived from the arithmetic: each layer input x is carried as
BF16 hi + lo, |x - hi - lo| <= 2^-18 |x|; products with BF16 weights are exact in FP32 and a
K-term FP32 sum errs by at most (K - 1) 2^-24 sum|terms| (K = 50, 800, 800 for the three
layers).  Propagated through the layers the error is below (3 2^-18 + 1650 2^-24) A < 1.1e-4 A,
with A the same network evaluated on |weights| and |input|."""
import numpy as np
import pytest

import pic_inputs as pi
from oracle import Oracle
from oracle import lfilter as L

gpu = pytest.mark.gpu
FWD_TOL = 1.1e-4


def _torch():
    import torch
    return torch


def _rand_params(seed, scale=0.25):
    return np.random.default_rng(seed).normal(scale=scale, size=L.NPARAM).astype(np.float32)


def _abs_net(params, x, periodic):
    return L.forward(np.abs(params), np.abs(x), periodic=periodic)


@gpu
@pytest.mark.parametrize("periodic", [(False, False), (True, True), (True, False)])
@pytest.mark.parametrize("shape", [(3, 37, 83), (1, 4, 64), (2, 61, 130)])
def test_forward_matches_oracle(periodic, shape):
    torch = _torch()
    from paper_1009_2727_amd import LearnedFilter
    p = _rand_params(11)
    x = np.random.default_rng(12).normal(size=shape).astype(np.float32)
    lf = LearnedFilter(p)
    out = lf.apply(torch.tensor(x, device="cuda"), periodic=periodic).cpu().numpy()
    ref = L.forward(p, x, periodic=periodic)
    bound = FWD_TOL * _abs_net(p, x, periodic) + 1e-30
    assert np.all(np.abs(out - ref) <= bound), float((np.abs(out - ref) / bound).max())


@gpu
def test_plain_weights_reproduce_the_bilinear_filter():
    torch = _torch()
    from paper_1009_2727_amd import LearnedFilter
    p = L.plain_filter_params(4, True)
    x = np.random.default_rng(13).normal(size=(2, 40, 70)).astype(np.float32)
    out = LearnedFilter(p).apply(torch.tensor(x, device="cuda"), periodic=(True, True)).cpu().numpy()
    ref = L.forward(p, x, periodic=(True, True))
    assert np.abs(out - ref).max() <= FWD_TOL * np.abs(_abs_net(p, x, (True, True))).max()


@gpu
@pytest.mark.parametrize("periodic", [(False, False), (True, True)])
def test_gradient_and_loss_match_oracle(periodic):
    torch = _torch()
    from paper_1009_2727_amd import LearnedFilter
    p = _rand_params(21, 0.2)
    rng = np.random.default_rng(22)
    x = rng.normal(size=(4, 32, 32)).astype(np.float32)
    y = L.forward(L.plain_filter_params(4, True), x, periodic=periodic).astype(np.float32)
    lf = LearnedFilter(p)
    loss, grad = lf.train_step(torch.tensor(x, device="cuda"), torch.tensor(y, device="cuda"), margin=6,
                               lr=0.0, periodic=periodic, want_grad=True)
    ref_loss, ref_grad = L.loss_and_grad(p, x, y, 6, periodic)
    assert float(loss.cpu()) == pytest.approx(ref_loss, rel=5e-4)
    g = grad.cpu().numpy().astype(np.float64)
    for a, b in ((L.OFF_W1, L.OFF_W2), (L.OFF_W2, L.OFF_W3), (L.OFF_W3, L.NPARAM)):
        scale = np.abs(ref_grad[a:b]).max()
        assert np.abs(g[a:b] - ref_grad[a:b]).max() <= 2e-3 * scale
    assert np.array_equal(lf.params.cpu().numpy(), p)      # lr = 0: no update


@gpu
def test_adam_update_matches_oracle():
    torch = _torch()
    from paper_1009_2727_amd import LearnedFilter
    p = _rand_params(31, 0.2)
    rng = np.random.default_rng(32)
    x = torch.tensor(rng.normal(size=(2, 24, 40)).astype(np.float32), device="cuda")
    y = torch.tensor(rng.normal(size=(2, 24, 40)).astype(np.float32), device="cuda")
    lf = LearnedFilter(p)
    w = p.astype(np.float64)
    m = np.zeros(L.NPARAM)
    v = np.zeros(L.NPARAM)
    for t in (1, 2, 3):
        _, g = lf.train_step(x, y, margin=2, lr=1e-3, want_grad=True)
        w, m, v = L.adam(w, m, v, g.cpu().numpy().astype(np.float64), t, 1e-3)
        assert np.abs(lf.params.cpu().numpy() - w).max() <= 1e-6
        assert np.abs(lf.m.cpu().numpy() - m).max() <= 1e-6 * max(np.abs(m).max(), 1e-30)


@gpu
def test_training_fits_the_bilinear_filter():
    torch = _torch()
    from paper_1009_2727_amd import LearnedFilter
    rng = np.random.default_rng(41)
    x = rng.normal(size=(64, 32, 32)).astype(np.float32)
    y = L.forward(L.plain_filter_params(4, True), x).astype(np.float32)
    xt, yt = torch.tensor(x, device="cuda"), torch.tensor(y, device="cuda")
    lf = LearnedFilter(_rand_params(42, 0.05))
    first = float(lf.train_step(xt, yt, margin=6, lr=0.0)[0].cpu())
    for _ in range(400):
        lf.train_step(xt, yt, margin=6, lr=3e-3)
    last = float(lf.train_step(xt, yt, margin=6, lr=0.0)[0].cpu())
    assert last < 0.05 * first


@gpu
@pytest.mark.parametrize("real_case", ["lab", "boosted"])
def test_pic_with_plain_weights_matches_bilinear_run(real_case):
    from paper_1009_2727_amd import Sim
    from test_gpu_parity import field_scales
    if real_case == "lab":
        w = pi.small_lab(real="f32", nx=24, nz=96, ppc=4, npass=4, comp=1)
        steps = 40
    else:
        w = pi.small_boosted(real="f32", nx=40, nz=150, ppc=2)
        steps = 60
    a = Sim.from_workload(w)
    w2 = pi.copy_workload(w)
    w2["config"]["filter_kind"] = 1
    b = Sim.from_workload(w2)
    b.set_learned_filter(L.plain_filter_params(w["config"]["filter_npass"],
                                               bool(w["config"]["filter_compensate"])))
    a.step(steps)
    b.step(steps)
    sc = field_scales(Oracle.from_workload(w))   # the physical field scales only
    for n in ["Ex", "Ey", "Ez", "Bx", "By", "Bz", "Jx", "Jy", "Jz"]:
        fa, fb = a.field(n), b.field(n)
        s = max(np.abs(fa).max(), sc[n[0]])
        assert np.abs(fa - fb).max() <= 1e-5 * s, n
