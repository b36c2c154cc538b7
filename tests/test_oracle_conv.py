"""Pins of the FP64 reference of the surrogate's convolution (CPU)."""
import numpy as np
import pytest
from scipy import signal

from oracle import conv_ref as cr


def test_bf16_rounding():
    """Nearest BF16 (8 significant bits), ties to even; exact values pass."""
    assert cr.bf16_round(1.0) == 1.0 and cr.bf16_round(-2.5) == -2.5
    assert cr.bf16_round(1.0 + 2 ** -8) == 1.0            # tie -> even
    assert cr.bf16_round(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6  # tie -> even (up)
    assert cr.bf16_round(1.0 + 2 ** -8 + 2 ** -12) == 1.0 + 2 ** -7
    x = np.random.default_rng(0).standard_normal(1000)
    assert np.all(np.abs(cr.bf16_round(x) - x) <= np.abs(x) * 2 ** -8 * (1 + 1e-12))


def test_conv_matches_scipy_correlate():
    """Per channel pair the convolution is scipy's 2-D cross-correlation of the
    frame padded periodically in x and with zeros in y."""
    rng = np.random.default_rng(1)
    a = rng.standard_normal((2, 5, 7, 3))
    w = rng.standard_normal((4, 9, 3))
    out = cr.conv(a, w)
    for n in range(2):
        for co in range(4):
            acc = np.zeros((5, 7))
            for ci in range(3):
                fr = np.pad(a[n, :, :, ci], ((1, 1), (0, 0)))
                fr = np.concatenate([fr[:, -1:], fr, fr[:, :1]], axis=1)
                k = w[co, :, ci].reshape(3, 3)
                acc += signal.correlate2d(fr, k, mode="valid")
            assert np.allclose(out[n, :, :, co], acc, atol=1e-12)


@pytest.mark.parametrize("dil", [2, 3])
def test_dilated_conv_matches_scipy_correlate(dil):
    """A dilation d is the cross-correlation with the 3x3 kernel spread onto a
    (2d+1) x (2d+1) grid of zeros, on the frame padded by d rows of zeros and
    wrapped by d columns."""
    rng = np.random.default_rng(4 + dil)
    a = rng.standard_normal((1, 6, 8, 2))
    w = rng.standard_normal((3, 9, 2))
    out = cr.conv(a, w, dil=dil)
    for co in range(3):
        acc = np.zeros((6, 8))
        for ci in range(2):
            fr = np.pad(a[0, :, :, ci], ((dil, dil), (0, 0)))
            fr = np.concatenate([fr[:, -dil:], fr, fr[:, :dil]], axis=1)
            k = np.zeros((2 * dil + 1, 2 * dil + 1))
            k[::dil, ::dil] = w[co, :, ci].reshape(3, 3)
            acc += signal.correlate2d(fr, k, mode="valid")
        assert np.allclose(out[0, :, :, co], acc, atol=1e-12)


@pytest.mark.parametrize("dil", [1, 2])
def test_conv_gradients_by_linearity(dil):
    """The input and weight gradients are exact for the bilinear form
    <conv(a, w), g>: checked by directional derivatives (exact for a linear map)."""
    rng = np.random.default_rng(2)
    a = rng.standard_normal((1, 4, 6, 3))
    w = rng.standard_normal((5, 9, 3))
    g = rng.standard_normal((1, 4, 6, 5))
    da = rng.standard_normal(a.shape)
    dw = rng.standard_normal(w.shape)
    f = lambda aa, ww: np.sum(cr.conv(aa, ww, dil=dil) * g)  # noqa: E731
    assert np.isclose(f(a + da, w) - f(a, w), np.sum(cr.conv_input_grad(g, w, dil) * da), rtol=1e-11)
    assert np.isclose(f(a, w + dw) - f(a, w), np.sum(cr.conv_weight_grad(g, a, dil) * dw), rtol=1e-11)


def test_net_gradients_finite_difference():
    """Gradients of the reference network match central differences of its
    loss (BF16 storage switched off by exact-in-BF16 inputs is not possible, so
    the check uses a tiny step on an FP64 copy without rounding)."""
    rng = np.random.default_rng(3)
    W = [0.1 * rng.standard_normal((32, 9, 8))] + [0.05 * rng.standard_normal((32, 9, 32)) for _ in range(4)]
    w5 = np.zeros((32, 9, 32))
    w5[:4] = 0.05 * rng.standard_normal((4, 9, 32))
    W.append(w5)
    b = [0.01 * rng.standard_normal(32) for _ in range(6)]
    x = np.zeros((1, 3, 32, 8))
    x[..., :4] = rng.standard_normal((1, 3, 32, 4))
    target = rng.standard_normal((1, 3, 32, 4))
    saved = cr.bf16_round, cr.fp32_round
    cr.bf16_round = cr.fp32_round = lambda v: np.asarray(v, np.float64)  # exact storage for the check
    try:
        dil = (1, 2, 1, 3, 1, 2)
        net = cr.NetRef(W, b, dil)
        loss, gW, gb, _ = net.loss_and_grads(x, target, 1.0)
        for layer, (co, t, ci) in ((0, (3, 4, 2)), (2, (7, 0, 11)), (5, (1, 8, 30))):
            e = 1e-6
            Wp = [w.copy() for w in W]
            Wp[layer][co, t, ci] += e
            Wm = [w.copy() for w in W]
            Wm[layer][co, t, ci] -= e
            lp = cr.NetRef(Wp, b, dil).loss_and_grads(x, target, 1.0)[0]
            lm = cr.NetRef(Wm, b, dil).loss_and_grads(x, target, 1.0)[0]
            assert np.isclose((lp - lm) / (2 * e), gW[layer][co, t, ci], rtol=1e-5, atol=1e-9)
        bp = [v.copy() for v in b]
        bp[3][5] += 1e-6
        bm = [v.copy() for v in b]
        bm[3][5] -= 1e-6
        d = (cr.NetRef(W, bp, dil).loss_and_grads(x, target, 1.0)[0]
             - cr.NetRef(W, bm, dil).loss_and_grads(x, target, 1.0)[0]) / 2e-6
        assert np.isclose(d, gb[3][5], rtol=1e-5, atol=1e-9)
    finally:
        cr.bf16_round, cr.fp32_round = saved


def test_adam_matches_closed_form_first_step():
    """The first bias-corrected Adam step moves each weight by lr * sign(g)
    (up to eps)."""
    g = np.array([0.3, -2.0, 1e-3])
    p, _, _ = cr.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=1e-12)
    assert np.allclose(p, -0.01 * np.sign(g), rtol=1e-6)


def check_adam_constant_gradient(adam, steps=40):
    """Under a constant gradient the bias-corrected moments equal g and g^2 at
    every step, so each step moves a weight by lr * sign(g) (up to eps): after
    t steps the weight has moved t * lr * sign(g)."""
    g = np.array([0.3, -2.0, 1e-3])
    lr = 0.01
    p, m1, m2 = np.zeros(3), np.zeros(3), np.zeros(3)
    for t in range(1, steps + 1):
        p, m1, m2 = adam(p, g, m1, m2, t, lr=lr, eps=1e-12)
        assert np.allclose(p, -lr * t * np.sign(g), rtol=1e-6, atol=0), t


def check_adam_impulse_response(adam, steps=30, b1=0.9, b2=0.999):
    """A single gradient g at step 1 and none afterwards: the moments decay
    geometrically, m_t = b1^(t-1) (1 - b1) g and v_t = b2^(t-1) (1 - b2) g^2, so
    step t moves a weight by lr m_t/(1 - b1^t) / (sqrt(v_t/(1 - b2^t)) + eps)."""
    g = np.array([0.3, -2.0, 1e-3])
    lr, eps = 0.01, 1e-12
    p, m1, m2 = np.zeros(3), np.zeros(3), np.zeros(3)
    for t in range(1, steps + 1):
        gt = g if t == 1 else np.zeros(3)
        q, m1, m2 = adam(p, gt, m1, m2, t, lr=lr, b1=b1, b2=b2, eps=eps)
        mt = b1 ** (t - 1) * (1 - b1) * g
        vt = b2 ** (t - 1) * (1 - b2) * g * g
        want = -lr * (mt / (1 - b1 ** t)) / (np.sqrt(vt / (1 - b2 ** t)) + eps)
        assert np.allclose(q - p, want, rtol=1e-9, atol=0), t
        p = q


def test_adam_constant_gradient():
    check_adam_constant_gradient(cr.adam)


def test_adam_impulse_response():
    check_adam_impulse_response(cr.adam)


def test_adam_scale_invariant():
    """Adam's step does not depend on the scale of the gradients (up to eps)."""
    rng = np.random.default_rng(3)
    gs = rng.standard_normal((12, 5))
    out = []
    for s in (1.0, 1e3):
        p, m1, m2 = np.zeros(5), np.zeros(5), np.zeros(5)
        for t, g in enumerate(gs, start=1):
            p, m1, m2 = cr.adam(p, s * g, m1, m2, t, lr=0.01, eps=1e-14)
        out.append(p)
    assert np.allclose(out[0], out[1], rtol=1e-9, atol=0)
