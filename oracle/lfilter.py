"""FP64 reference of the learned current filter (plain numpy).

TEST INFRASTRUCTURE ONLY: imported by tests/ and by the training/evaluation helpers of the
tests; the product package never imports it.  It shares no code with the HIP kernels.

The filter replaces the n-pass bilinear + compensation filter of the paper's Sec. 4.1 (Eq.
3ptfilter).  It is three 5x5 convolutions, channels 1 -> 16 -> 16 -> 1, with identity
activations and no bias.  One network is shared by J_x, J_y and J_z.  Every layer reads its
input with zero padding outside the domain, or wraps on a periodic axis:

    out(p, co) = sum_{t, ci} W[t, ci, co] * in(p + o_t, ci),
    o_t = (dy, dx),  t = 5 (dy + 2) + (dx + 2),  dy along the image rows.

The weights are BF16, round to nearest even of the FP32 master values.  Inputs are exact here;
the device splits them into BF16 hi + lo parts.  Parameters are a flat FP32 vector:
W1[t][co] (25 x 16), then W2[t][ci][co] (25 x 16 x 16), then W3[t][ci] (25 x 16).

Training uses the mean squared error over the pixels at least `margin` from the image edges.
Backpropagation goes through the convolutions with the weights as used, i.e. BF16.  The update
is Adam, Kingma & Ba (2015), with bias correction.

Pins: the network's transfer function against the closed-form gain of the bilinear filter
(Sec. 4.1); forward passes against the C oracle's bilinear filter; impulse response against the
kernel composed by direct 2D convolution; gradients against central finite differences; Adam
against its first-step closed form.
"""
from __future__ import annotations

import numpy as np

C = 16
TAPS = 25
OFF_W1 = 0
OFF_W2 = TAPS * C
OFF_W3 = OFF_W2 + TAPS * C * C
NPARAM = OFF_W3 + TAPS * C
OFFSETS = [(t // 5 - 2, t % 5 - 2) for t in range(TAPS)]   # (dy, dx) of tap t


def bf16(x):
    """Round FP32 values to BF16 (8-bit significand), round to nearest even; returned as FP64."""
    u = np.ascontiguousarray(np.asarray(x, dtype=np.float32)).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(params, quantize=True):
    p = np.asarray(params, dtype=np.float32).ravel()
    assert p.size == NPARAM
    q = bf16(p) if quantize else p.astype(np.float64)
    w1 = q[OFF_W1:OFF_W2].reshape(TAPS, 1, C)
    w2 = q[OFF_W2:OFF_W3].reshape(TAPS, C, C)
    w3 = q[OFF_W3:].reshape(TAPS, C, 1)
    return w1, w2, w3


def pack(w1, w2, w3):
    return np.concatenate([np.ravel(w1), np.ravel(w2), np.ravel(w3)]).astype(np.float32)


def _shifted(x, dy, dx, periodic):
    """x[n, y + dy, x + dx, c] with the boundary rule (zero or wrap) per axis."""
    n, ny, nx, c = x.shape
    ys = np.arange(ny) + dy
    xs = np.arange(nx) + dx
    if periodic[1]:
        ys %= ny
    if periodic[0]:
        xs %= nx
    oky = (ys >= 0) & (ys < ny)
    okx = (xs >= 0) & (xs < nx)
    out = np.zeros_like(x)
    out[:, np.nonzero(oky)[0][:, None], np.nonzero(okx)[0][None, :]] = x[:, ys[oky]][:, :, xs[okx]]
    return out


def conv(x, w, periodic=(False, False)):
    """One layer: x [n, ny, nx, cin], w [25, cin, cout] -> [n, ny, nx, cout]."""
    out = np.zeros(x.shape[:3] + (w.shape[2],))
    for t, (dy, dx) in enumerate(OFFSETS):
        out += np.tensordot(_shifted(x, dy, dx, periodic), w[t], axes=([3], [0]))
    return out


def conv_adjoint(g, w, periodic=(False, False)):
    """Adjoint of conv with respect to its input: g [n, ny, nx, cout] -> [n, ny, nx, cin]."""
    out = np.zeros(g.shape[:3] + (w.shape[1],))
    for t, (dy, dx) in enumerate(OFFSETS):
        out += np.tensordot(_shifted(g, -dy, -dx, periodic), w[t], axes=([3], [1]))
    return out


def conv_wgrad(x, g, periodic=(False, False)):
    """Gradient of sum(g * conv(x, w)) with respect to w: [25, cin, cout]."""
    return np.stack([np.tensordot(_shifted(x, dy, dx, periodic), g, axes=([0, 1, 2], [0, 1, 2]))
                     for dy, dx in OFFSETS])


def forward(params, images, periodic=(False, False), quantize=True, keep=False):
    """images [nimg, ny, nx] -> filtered [nimg, ny, nx] (FP64)."""
    w1, w2, w3 = unpack(params, quantize)
    x = np.asarray(images, dtype=np.float64)[..., None]
    h1 = conv(x, w1, periodic)
    h2 = conv(h1, w2, periodic)
    out = conv(h2, w3, periodic)[..., 0]
    return (out, (x, h1, h2)) if keep else out


def loss_and_grad(params, images, targets, margin, periodic=(False, False), quantize=True):
    """Mean squared error over the pixels at least `margin` from the edges, and its gradient
    with respect to the parameters (backpropagation through the three convolutions)."""
    w1, w2, w3 = unpack(params, quantize)
    out, (x, h1, h2) = forward(params, images, periodic, quantize, keep=True)
    n, ny, nx = out.shape
    mask = np.zeros((ny, nx))
    mask[margin:ny - margin, margin:nx - margin] = 1.0
    count = n * mask.sum()
    e = (out - np.asarray(targets, dtype=np.float64)) * mask
    loss = float((e * e).sum() / count)
    g3 = (2.0 * e / count)[..., None]
    dw3 = conv_wgrad(h2, g3, periodic)
    gh2 = conv_adjoint(g3, w3, periodic)
    dw2 = conv_wgrad(h1, gh2, periodic)
    gh1 = conv_adjoint(gh2, w2, periodic)
    dw1 = conv_wgrad(x, gh1, periodic)
    return loss, pack(dw1, dw2, dw3).astype(np.float64)


def adam(params, m, v, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2015); returns new (params, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def plain_filter_params(npass=4, compensate=True):
    """Parameters for which the network is exactly the n-pass bilinear filter (+ compensation
    with alpha_c = n/2 + 1): per axis the 1D kernel is ((1 + z)^2 / 4)^n times the compensation
    stencil, split into three factors of at most 5 taps; channel 0 carries it."""
    factors = []
    powers = 2 * npass                    # (1 + z)^(2n) / 4^n: 2n factors (1 + z)/2
    room = [4, 4, 2 if compensate else 4]
    for L in range(3):
        p = min(room[L], powers)
        powers -= p
        f = np.array([1.0])
        for _ in range(p):
            f = np.convolve(f, [0.5, 0.5])
        factors.append(f)
    if powers:
        raise ValueError("more passes than three 5-tap layers can hold")
    if compensate:
        ac = npass / 2 + 1
        factors[2] = np.convolve(factors[2], [(1 - ac) / 2, ac, (1 - ac) / 2])
    ws = []
    for L, f in enumerate(factors):
        f5 = np.zeros(5)
        off = (5 - len(f)) // 2
        f5[off:off + len(f)] = f
        k2 = np.outer(f5, f5).ravel()     # [dy, dx] -> tap
        cin = 1 if L == 0 else C
        cout = 1 if L == 2 else C
        w = np.zeros((TAPS, cin, cout))
        w[:, 0, 0] = k2
        ws.append(w)
    return pack(*ws)


def composed_kernel(params, quantize=True):
    """The network's 13 x 13 kernel K[dy + 6, dx + 6] by direct 2D convolution of the layers'
    5 x 5 kernels summed over the hidden channels (out(p) = sum K[o] in(p + o))."""
    from scipy.signal import convolve2d
    w1, w2, w3 = unpack(params, quantize)
    k1 = [w1[:, 0, c].reshape(5, 5) for c in range(C)]
    k2 = [[w2[:, a, b].reshape(5, 5) for b in range(C)] for a in range(C)]
    k3 = [w3[:, c, 0].reshape(5, 5) for c in range(C)]
    # out(p) = sum_o K[o] in(p + o) is a correlation; composing correlations = correlation with
    # the convolution of the kernels
    h = [sum(convolve2d(k2[a][b], k1[a]) for a in range(C)) for b in range(C)]   # 9 x 9
    return sum(convolve2d(k3[b], h[b]) for b in range(C))                         # 13 x 13


def transfer(params, kx, ky, quantize=True):
    """Fourier gain G(kx, ky) = sum_o K[o] exp(i (kx dx + ky dy)) (grid units)."""
    K = composed_kernel(params, quantize)
    d = np.arange(-6, 7)
    ph = np.exp(1j * (np.multiply.outer(ky, d)[..., :, None] + np.multiply.outer(kx, d)[..., None, :]))
    return (ph * K).sum(axis=(-1, -2))
