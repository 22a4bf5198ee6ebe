"""Training data, training and evaluation of the learned current filter.

* Pairs (raw current, current after the 4-pass + compensation bilinear filter of Sec. 4.1) come
  from the method itself: GPU runs read back J_r (deposited) and J (filtered) after a step.
* A spectral term: band-limited random patches whose spectrum lies in the high-k band where the
  numerical instabilities of Sec. 4 grow; their targets are the bilinear filter's output, and
  their weight sets how strongly the learned gain is held to the plain one in that band.
* Training is Adam through the library's MFMA kernels (LearnedFilter.train_step).
* Evaluation: the learned transfer function against the plain one, the growth rate of the
  high-k field energy in an unstable run, and the on-axis wake field against a reference.
"""
from __future__ import annotations

import copy

import numpy as np

from . import FILTER_LEARNED, LF_PARAMS, LearnedFilter, Sim, bilinear_factor_params

PATCH = 32
MARGIN = 6          # receptive field radius of three 5x5 layers


def current_pairs(workload, steps, every, per_component=48, seed=0, patch=PATCH, sort_every=0):
    """Runs `workload` on the GPU with its bilinear filter and returns normalised patch pairs
    (inputs, targets), each (n, patch, patch) float32, cut at random from J_r and J of every
    component every `every` steps."""
    sim = Sim.from_workload(workload, sort_every=sort_every)
    rng = np.random.default_rng(seed)
    xs, ys = [], []
    for s in range(1, steps + 1):
        sim.step(1)
        if s % every:
            continue
        for c in "xyz":
            raw, filt = sim.field("J" + c + "r"), sim.field("J" + c)
            nz, nx = raw.shape
            if nz < patch or nx < patch:
                raise ValueError("grid smaller than a patch")
            for _ in range(per_component):
                k0, i0 = rng.integers(0, nz - patch + 1), rng.integers(0, nx - patch + 1)
                a = raw[k0:k0 + patch, i0:i0 + patch]
                b = filt[k0:k0 + patch, i0:i0 + patch]
                r = np.sqrt(np.mean(a * a))
                if r == 0.0:
                    continue
                xs.append(a / r)
                ys.append(b / r)
    return np.asarray(xs, np.float32), np.asarray(ys, np.float32)


def band_probes(n, kmin_frac=0.5, seed=1, patch=PATCH):
    """Random patches with all their energy at |k| > kmin_frac * pi (grid units), and the
    bilinear filter's output on them (computed with the exact factorisation on the device)."""
    import torch
    rng = np.random.default_rng(seed)
    k = 2 * np.pi * np.fft.fftfreq(patch)
    kk = np.sqrt(k[:, None] ** 2 + k[None, :] ** 2)
    x = np.fft.ifft2(np.fft.fft2(rng.normal(size=(n, patch, patch))) * (kk > kmin_frac * np.pi)).real
    x /= np.sqrt(np.mean(x * x, axis=(1, 2), keepdims=True))
    x = x.astype(np.float32)
    plain = LearnedFilter(bilinear_factor_params(4, True))
    y = plain.apply(torch.tensor(x, device=plain.device), periodic=(True, True)).cpu().numpy()
    return x, y


def train(inputs, targets, probes=None, probe_weight=1.0, params0=None, steps=2000, lr=2e-3,
          batch=64, seed=2, log_every=0):
    """Adam on the mean squared error of the patch pairs (plus the weighted probe pairs).
    Returns (LearnedFilter, loss history)."""
    import torch
    rng = np.random.default_rng(seed)
    if params0 is None:
        params0 = rng.normal(scale=0.05, size=LF_PARAMS).astype(np.float32)
    lf = LearnedFilter(params0)
    X, Y = inputs, targets
    if probes is not None:
        s = np.float32(np.sqrt(probe_weight))
        X = np.concatenate([X, probes[0] * s])
        Y = np.concatenate([Y, probes[1] * s])
    Xd = torch.tensor(X, device=lf.device)
    Yd = torch.tensor(Y, device=lf.device)
    hist = []
    for it in range(steps):
        idx = torch.tensor(rng.integers(0, len(X), batch), device=lf.device)
        loss, _ = lf.train_step(Xd[idx].contiguous(), Yd[idx].contiguous(), MARGIN, lr)
        if log_every and it % log_every == 0:
            hist.append((it, float(loss.cpu())))
    return lf, hist


def composed_kernel(params):
    """The 13 x 13 kernel of the (linear) network, K[dy + 6, dx + 6], from its BF16 weights."""
    from scipy.signal import convolve2d
    p = np.asarray(params, np.float32)
    q = (p.view(np.uint32).astype(np.uint64) + 0x7FFF + ((p.view(np.uint32) >> 16) & 1)) & 0xFFFF0000
    w = q.astype(np.uint32).view(np.float32).astype(np.float64)
    w1 = w[:400].reshape(25, 16)
    w2 = w[400:6800].reshape(25, 16, 16)
    w3 = w[6800:].reshape(25, 16)
    h = [sum(convolve2d(w2[:, a, b].reshape(5, 5), w1[:, a].reshape(5, 5)) for a in range(16))
         for b in range(16)]
    return sum(convolve2d(w3[:, b].reshape(5, 5), h[b]) for b in range(16))


def gain(params, kx, kz):
    K = composed_kernel(params)
    d = np.arange(-6, 7)
    ph = np.exp(1j * (np.multiply.outer(kz, d)[..., :, None] + np.multiply.outer(kx, d)[..., None, :]))
    return (ph * K).sum(axis=(-1, -2)).real


def plain_gain(kx, kz, npass=4, comp=True):
    g = lambda a, k: a + (1 - a) * np.cos(k)   # noqa: E731  (3-point pass, Sec. 4.1)
    one = lambda k: g(0.5, k) ** npass * (g(npass / 2 + 1, k) if comp else 1.0)  # noqa: E731
    return one(kx) * one(kz)


def gain_error(params, kmax):
    """max |G_learned - G_plain| over |k| < kmax (grid units)."""
    k = np.linspace(-kmax, kmax, 81)
    kx, kz = np.meshgrid(k, k)
    inside = kx ** 2 + kz ** 2 < kmax ** 2
    return float(np.abs(gain(params, kx, kz) - plain_gain(kx, kz))[inside].max())


def highk_energy(field, frac=0.5):
    """sum of |E^(k)|^2 over |k| > frac * k_max."""
    f = np.fft.fft2(field)
    kz = np.fft.fftfreq(field.shape[0])[:, None]
    kx = np.fft.fftfreq(field.shape[1])[None, :]
    band = np.sqrt(kx ** 2 + kz ** 2) > frac * 0.5
    return float((np.abs(f[band]) ** 2).sum())


def growth_rate(workload, params=None, steps=400, every=10, field="Ez"):
    """Growth rate (per step) of the high-k energy of `field`: the slope of its logarithm over
    the stretch where it grows steadily (least squares over the second half of the samples
    above the noise floor).  params None: the workload's own filter."""
    w = copy.deepcopy(workload)
    if params is not None:
        w["config"]["filter_kind"] = FILTER_LEARNED
    sim = Sim.from_workload(w)
    if params is not None:
        sim.set_learned_filter(params)
    t, e = [], []
    for s in range(every, steps + 1, every):
        sim.step(every)
        t.append(s)
        e.append(highk_energy(sim.field(field)))
    t, le = np.asarray(t, float), np.log(np.maximum(np.asarray(e), 1e-300))
    h = len(t) // 2
    slope = np.polyfit(t[h:], le[h:], 1)[0]
    return float(slope), t, le
