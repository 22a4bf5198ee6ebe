"""Training data, training and evaluation of the learned current filter.

* Pairs (raw current, current after the 4-pass + compensation bilinear filter of Sec. 4.1) come
  from the method itself: GPU runs read back J_r (deposited) and J (filtered) after a step.
* A spectral term: random patches whose power spectrum is the growth spectrum measured in
  unfiltered unstable runs (the band where the numerical instabilities of Sec. 4 grow), or a flat
  high-k band; their targets are the bilinear filter's output, so the learned gain is held to the
  plain one where the instabilities grow, weighted by how fast they grow there.
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


def training_set(runs, n_total, seed=0, patch=PATCH):
    """Patch pairs from several runs: `runs` is a list of (workload, steps, every); each run is
    asked for about n_total / len(runs) pairs from its non-zero current components (patches with
    no current at all are dropped, so a short harvest is cut again with more patches per frame),
    and the union is cut to exactly n_total pairs at random (seeded).  Returns (inputs, targets,
    pairs per run)."""
    scale = 1.05
    for _ in range(4):
        xs, ys, per_run = [], [], []
        for r, (w, steps, every) in enumerate(runs):
            frames = steps // every
            comps = 3 - sum(1 for c in "xyz" if _zero_component(w, c))
            per = int(np.ceil(scale * n_total / (len(runs) * frames * comps)))
            x, y = current_pairs(w, steps, every, per_component=per, seed=seed + 7919 * r, patch=patch)
            xs.append(x)
            ys.append(y)
            per_run.append(len(x))
        X, Y = np.concatenate(xs), np.concatenate(ys)
        if len(X) >= n_total:
            break
        if len(X) == 0:
            raise RuntimeError("the runs deposited no current: no patch pairs to cut")
        scale *= 1.1 * n_total / len(X)
    if len(X) < n_total:
        raise RuntimeError(f"{len(X)} pairs from the runs, fewer than {n_total}")
    keep = np.sort(np.random.default_rng(seed).choice(len(X), n_total, replace=False))
    return X[keep], Y[keep], per_run


def _zero_component(workload, c):
    """True for the current component a 2D run never deposits: J_y without a y-polarised laser
    (no force along y acts on particles that start with u_y = 0)."""
    las = workload.get("laser")
    return c == "y" and (las is None or las.get("pol", 0) == 0)


def patch_spectrum(field, patch=PATCH):
    """Mean power spectrum |F(k)|^2 of the non-overlapping patch x patch windows of a 2D field,
    on the patch's own frequency grid (numpy FFT order)."""
    nz, nx = field.shape
    w = field[:nz - nz % patch, :nx - nx % patch].reshape(nz // patch, patch, nx // patch, patch)
    return (np.abs(np.fft.fft2(w.transpose(0, 2, 1, 3))) ** 2).mean(axis=(0, 1))


def growth_spectrum(workload, steps, early, field="Ez", patch=PATCH):
    """Per-step growth rate of each patch mode of `field` in an unfiltered copy of `workload`:
    ln(P_end(k) / P_early(k)) / (steps - early), negative rates clipped to zero."""
    w = copy.deepcopy(workload)
    w["config"]["filter_npass"], w["config"]["filter_compensate"] = 0, 0
    sim = Sim.from_workload(w)
    sim.step(early)
    p0 = patch_spectrum(sim.field(field), patch)
    sim.step(steps - early)
    p1 = patch_spectrum(sim.field(field), patch)
    tiny = 1e-300
    return np.maximum(np.log((p1 + tiny) / (p0 + tiny)), 0.0) / (steps - early)


def band_probes(n, kmin_frac=0.5, seed=1, patch=PATCH, weight=None):
    """Random patches and the bilinear filter's output on them (computed with the exact
    factorisation on the device).  weight None: all their energy at |k| > kmin_frac * pi (grid
    units); else their power spectrum is `weight` (patch x patch, numpy FFT order)."""
    import torch
    rng = np.random.default_rng(seed)
    k = 2 * np.pi * np.fft.fftfreq(patch)
    kk = np.sqrt(k[:, None] ** 2 + k[None, :] ** 2)
    shape = (kk > kmin_frac * np.pi).astype(float) if weight is None else np.sqrt(np.asarray(weight, float))
    x = np.fft.ifft2(np.fft.fft2(rng.normal(size=(n, patch, patch))) * shape).real
    x /= np.sqrt(np.mean(x * x, axis=(1, 2), keepdims=True))
    x = x.astype(np.float32)
    plain = LearnedFilter(bilinear_factor_params(4, True))
    y = plain.apply(torch.tensor(x, device=plain.device), periodic=(True, True)).cpu().numpy()
    return x, y


def train(inputs, targets, probes=None, probe_weight=1.0, params0=None, steps=2000, lr=2e-3,
          batch=64, seed=2, log_every=0, lr_final=None):
    """Adam on the mean squared error of the patch pairs (plus the weighted probe pairs); with
    lr_final the step size falls from lr to lr_final along a half cosine.  Returns
    (LearnedFilter, loss history)."""
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
        a = lr if lr_final is None else lr_final + 0.5 * (lr - lr_final) * (1 + np.cos(np.pi * it / steps))
        loss, _ = lf.train_step(Xd[idx].contiguous(), Yd[idx].contiguous(), MARGIN, float(a))
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


def growth_rate(workload, params=None, steps=400, every=10, field="Ez", window=None):
    """Growth rate (per step) of the high-k energy of `field`: the least-squares slope of its
    logarithm over the samples at steps in `window` = (first, last), or over the second half of
    the samples when no window is given.  params None: the workload's own filter."""
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
    sel = (t >= window[0]) & (t <= window[1]) if window is not None else np.arange(len(t)) >= len(t) // 2
    slope = np.polyfit(t[sel], le[sel], 1)[0]
    return float(slope), t, le


def linear_phase(t, le, frac=0.8):
    """The stretch of an unfiltered run's log high-k energy where the instability grows: from
    the second sample (the first holds the start-up transient) to the first sample that has
    covered `frac` of the rise from the minimum to the maximum (where saturation begins)."""
    lo, hi = le.min(), le.max()
    k1 = int(np.argmax(le >= lo + frac * (hi - lo)))
    k1 = max(k1, 3)
    return float(t[1]), float(t[k1])
