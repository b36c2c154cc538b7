"""FP64 CPU reference of the surrogate network's operations.

TEST INFRASTRUCTURE (see the package docstring).  Plain NumPy from the
definitions, no blocking: a 3x3 cross-correlation over NHWC frames that are
periodic in x and zero-padded in y, its input and weight gradients, the bias
gradient, one Adam step, the squared-error loss, and the whole residual network
(forward and backward).  BF16 storage is emulated by rounding to the nearest
BF16 value (ties to even) wherever the GPU stores BF16, so the GPU results can
be compared within FP32 accumulation-order error.

Taps are ordered t = 3 (dy + 1) + (dx + 1); weights are [co][t][ci].
"""
from __future__ import annotations

import numpy as np

TAPS = [(t // 3 - 1, t % 3 - 1) for t in range(9)]


def bf16_round(a) -> np.ndarray:
    """Nearest BF16 value of each element (ties to even), returned as float64."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def fp32_round(a) -> np.ndarray:
    """Nearest FP32 value of each element, returned as float64."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def shifted(a: np.ndarray, dy: int, dx: int) -> np.ndarray:
    """out[n, y, x] = a[n, y + dy, (x + dx) mod W], zero where y + dy is outside."""
    out = np.zeros_like(a)
    H = a.shape[1]
    if abs(dy) >= H:
        return out
    rolled = np.roll(a, -dx, axis=2)
    if dy >= 0:
        out[:, :H - dy] = rolled[:, dy:]
    else:
        out[:, -dy:] = rolled[:, :H + dy]
    return out


def conv(a: np.ndarray, w: np.ndarray, bias=None, dil: int = 1) -> np.ndarray:
    """out[n, y, x, co] = sum_{t, ci} a[n, y + d dy_t, x + d dx_t, ci] w[co, t, ci] (+ bias[co]),
    d the dilation."""
    a = np.asarray(a, np.float64)
    w = np.asarray(w, np.float64)
    out = np.zeros(a.shape[:3] + (w.shape[0],))
    for t, (dy, dx) in enumerate(TAPS):
        out += shifted(a, dil * dy, dil * dx) @ w[:, t, :].T
    if bias is not None:
        out += np.asarray(bias, np.float64)
    return out


def conv_input_grad(g: np.ndarray, w: np.ndarray, dil: int = 1) -> np.ndarray:
    """Gradient of sum(conv(a, w, dil=dil) * g) with respect to a."""
    g = np.asarray(g, np.float64)
    w = np.asarray(w, np.float64)
    out = np.zeros(g.shape[:3] + (w.shape[2],))
    for t, (dy, dx) in enumerate(TAPS):
        out += shifted(g @ w[:, t, :], -dil * dy, -dil * dx)
    return out


def conv_weight_grad(g: np.ndarray, a: np.ndarray, dil: int = 1) -> np.ndarray:
    """Gradient of sum(conv(a, w, dil=dil) * g) with respect to w: [co, t, ci]."""
    g = np.asarray(g, np.float64)
    a = np.asarray(a, np.float64)
    co, ci = g.shape[3], a.shape[3]
    out = np.zeros((co, 9, ci))
    gf = g.reshape(-1, co)
    for t, (dy, dx) in enumerate(TAPS):
        out[:, t, :] = gf.T @ shifted(a, dil * dy, dil * dx).reshape(-1, ci)
    return out


def adam(p, g, m1, m2, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam step; returns (p, m1, m2)."""
    m1 = b1 * m1 + (1 - b1) * g
    m2 = b2 * m2 + (1 - b2) * g * g
    p = p - lr * (m1 / (1 - b1 ** t)) / (np.sqrt(m2 / (1 - b2 ** t)) + eps)
    return p, m1, m2


def relu(a):
    return np.maximum(a, 0.0)


class NetRef:
    """The surrogate network in FP64 with BF16 storage emulated:

        h0 = conv(x, W0) + b0                      (x: 8 input channels)
        h_r = h_{r-1} + conv(relu(h_{r-1}), W_r) + b_r,   r = 1..4
        delta = conv(relu(h_4), W5) + b5           (channels 0..nout-1 used)
        loss = sum over pixels and channels c < nout of (delta_c - target_c)^2
    with nout the number of target channels.

    Weights: W0 [32, 9, 8], W1..W4 [32, 9, 32], W5 [32, 9, 32] (rows >= nout zero);
    biases [32]; layer r's taps dilated by dil[r].  Activations h_r are stored
    as BF16; delta is kept in FP32.
    """

    def __init__(self, weights, biases, dil=(1, 1, 1, 1, 1, 1)):
        self.W = [bf16_round(w) for w in weights]
        self.b = [np.asarray(b, np.float64) for b in biases]
        self.d = tuple(int(v) for v in dil)

    def forward(self, x):
        x = bf16_round(x)
        d = self.d
        hs = [bf16_round(conv(x, self.W[0], self.b[0], d[0]))]
        for r in range(1, 5):
            hs.append(bf16_round(hs[-1] + conv(relu(hs[-1]), self.W[r], self.b[r], d[r])))
        delta = fp32_round(conv(relu(hs[-1]), self.W[5], self.b[5], d[5]))
        return x, hs, delta

    def loss_and_grads(self, x, target, scale):
        x, hs, delta = self.forward(x)
        nout = target.shape[-1]
        e = delta[..., :nout] - target
        loss = float(np.sum(e * e))
        gd = np.zeros_like(delta)
        gd[..., :nout] = 2.0 * e * scale
        gd = bf16_round(gd)
        gW, gb = self.grads_from(x, hs, gd)
        return loss, gW, gb, delta

    def grads_from(self, x, hs, gd):
        """The backward pass alone: weight and bias gradients from the
        network input x, the stored activations h0..h4 and the BF16 gradient
        gd of the loss with respect to delta (all as given)."""
        x = bf16_round(x)
        gW = [None] * 6
        gb = [None] * 6
        d = self.d
        gW[5] = conv_weight_grad(gd, relu(hs[4]), d[5])
        gb[5] = gd.sum(axis=(0, 1, 2))
        gh = bf16_round(conv_input_grad(gd, self.W[5], d[5]) * (hs[4] > 0))
        for r in range(4, 0, -1):
            gW[r] = conv_weight_grad(gh, relu(hs[r - 1]), d[r])
            gb[r] = gh.sum(axis=(0, 1, 2))
            gh = bf16_round(gh + conv_input_grad(gh, self.W[r], d[r]) * (hs[r - 1] > 0))
        gW[0] = conv_weight_grad(gh, x, d[0])
        gb[0] = gh.sum(axis=(0, 1, 2))
        return gW, gb
