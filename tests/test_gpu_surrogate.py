"""Surrogate kernels (BF16 matrix cores, FP32 accumulation) against the FP64
CPU reference with BF16 storage emulated (oracle/conv_ref.py).

State-side kernels (packing, increments, state update, volume and judge
reductions) are checked against their definitions in NumPy, and the hybrid
rollout's bookkeeping against the plain lattice update.

Tolerances: FP32 outputs within 2e-5 relative (max error over max magnitude)
-- FP32 accumulation of <= 288 products per output, or of sums over <= 1e4
pixels for gradients; BF16 outputs within one BF16 step (2^-7 relative) of the
reference rounded to BF16; whole-network gradients within 3e-2 relative L2 per
layer, since an FP32-versus-FP64 difference can flip the BF16 rounding of an
intermediate activation.
"""
import numpy as np
import pytest

from oracle import conv_ref as cr
from tests.conftest import announce

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
sur = pytest.importorskip("paper_2306_11320_amd.surrogate")


def t_bf16(a, dev="cuda"):
    return torch.tensor(np.asarray(a, np.float32), device=dev).to(torch.bfloat16).contiguous()


def t_f32(a, dev="cuda"):
    return torch.tensor(np.asarray(a, np.float32), device=dev).contiguous()


def host(t):
    return t.float().cpu().numpy().astype(np.float64)


def dev(stream, *tensors):
    """Orders work on `stream` after the creation of the given device tensors
    (made on torch's current stream).  The caller keeps the returned tensors
    referenced until `stream` is synchronized: the caching allocator would
    otherwise hand their memory to the next allocation while a kernel on
    `stream` still reads it."""
    stream.wait_stream(torch.cuda.current_stream())
    return tensors


def relmax(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))


@pytest.fixture(scope="module")
def stream():
    return torch.cuda.Stream()


@pytest.mark.parametrize("cin", [8, 32])
@pytest.mark.parametrize("relu_in", [False, True])
@pytest.mark.parametrize("dil,W", [(1, 64), (3, 64), (1, 256), (3, 256), (16, 256), (2, 128),
                                   (1, 129), (3, 200), (16, 41), (1, 7), (20, 64), (17, 45)])
def test_conv_forward(cin, relu_in, dil, W, stream):
    """Frame widths of one to eight 32-pixel segments per row (periodic wrap at
    both ends of the row), ragged widths whose last segment is partly outside
    the row, and dilations up to 16 (32 input channels: the kernel by columns
    with staged input rows) and beyond (the kernel by segments)."""
    rng = np.random.default_rng(cin + relu_in + 10 * dil + W)
    N, H = 2, 5
    announce("conv_forward", cin, relu_in, dil, W)
    x = cr.bf16_round(rng.standard_normal((N, H, W, cin)))
    w = cr.bf16_round(0.2 * rng.standard_normal((32, 9, cin)))
    b = rng.standard_normal(32).astype(np.float32)
    res = rng.standard_normal((N, H, W, 32)).astype(np.float32)
    out = torch.empty((N, H, W, 32), device="cuda")
    xd, wd, bd, rd = dev(stream, t_bf16(x), t_bf16(w), t_f32(b), t_f32(res))
    sur.sur_conv3x3(xd, cin, wd, bd, rd, None, out, relu_in, stream, dil)
    stream.synchronize()
    a = cr.relu(x) if relu_in else x
    ref = cr.conv(a, w, b, dil) + res
    assert relmax(host(out), ref) <= 2e-5
    # BF16 output with a mask
    mask = cr.bf16_round(rng.standard_normal((N, H, W, 32)))
    outb = torch.empty((N, H, W, 32), dtype=torch.bfloat16, device="cuda")
    (md,) = dev(stream, t_bf16(mask))
    sur.sur_conv3x3(xd, cin, wd, bd, None, md, outb, relu_in, stream, dil)
    stream.synchronize()
    refb = cr.bf16_round(cr.conv(a, w, b, dil) * (mask > 0))
    got = host(outb)
    assert np.all(np.abs(got - refb) <= 2 ** -7 * np.abs(refb) + 1e-6)


@pytest.mark.parametrize("dil", [2, 4, 5, 8])
def test_conv_columns_many_items(dil, stream):
    """The hidden layer as the network runs it (ReLU on the input, the input as
    a BF16 residual, BF16 output) on 8 frames of 128 x 256: more column groups
    than resident workgroups, so each workgroup walks several of them; on
    both sides of the switch between the 40-pixel staging window (dilation
    <= 4, three workgroups per CU) and the 64-pixel one.  Within one BF16 step
    of the reference rounded to BF16."""
    rng = np.random.default_rng(40 + dil)
    N, H, W = 8, 128, 256
    announce("conv_columns_many_items", dil)
    x = cr.bf16_round(rng.standard_normal((N, H, W, 32)))
    w = cr.bf16_round(0.2 * rng.standard_normal((32, 9, 32)))
    b = rng.standard_normal(32).astype(np.float32)
    xd, wd, bd = dev(stream, t_bf16(x), t_bf16(w), t_f32(b))
    out = torch.empty((N, H, W, 32), dtype=torch.bfloat16, device="cuda")
    sur.sur_conv3x3(xd, 32, wd, bd, xd, None, out, True, stream, dil)
    stream.synchronize()
    ref = cr.bf16_round(cr.conv(cr.relu(x), w, b, dil) + x)
    got = host(out)
    assert np.all(np.abs(got - ref) <= 2 ** -7 * np.abs(ref) + 1e-6)


def test_adjoint_input_gradient(stream):
    rng = np.random.default_rng(7)
    N, H = 1, 6
    announce("adjoint")
    for cin, dil, W in ((8, 1, 32), (32, 1, 32), (32, 2, 32), (8, 5, 32), (32, 4, 128), (8, 16, 256), (32, 3, 200),
                        (8, 2, 45)):
        w = cr.bf16_round(0.2 * rng.standard_normal((32, 9, cin)))
        g = cr.bf16_round(rng.standard_normal((N, H, W, 32)))
        wt = torch.empty((32, 9, 32), dtype=torch.bfloat16, device="cuda")
        wd, gd = dev(stream, t_bf16(w), t_bf16(g))
        sur.sur_adjoint_weights(wd, cin, wt, stream)
        out = torch.empty((N, H, W, 32), device="cuda")
        sur.sur_conv3x3(gd, 32, wt, None, None, None, out, False, stream, dil)
        stream.synchronize()
        ref = cr.conv_input_grad(g, w, dil)
        got = host(out)[..., :cin]
        assert relmax(got, ref) <= 2e-5
        if cin < 32:
            assert np.abs(host(out)[..., cin:]).max() == 0.0


@pytest.mark.parametrize("cin", [8, 32])
@pytest.mark.parametrize("dil", [1, 4])
@pytest.mark.parametrize("W", [96, 129])
def test_weight_and_bias_gradient(cin, dil, W, stream):
    rng = np.random.default_rng(11 + cin + dil + W)
    N, H = 2, 7
    announce("wgrad", cin, dil, W)
    a = cr.bf16_round(rng.standard_normal((N, H, W, cin)))
    g = cr.bf16_round(rng.standard_normal((N, H, W, 32)))
    for relu_in in (False, True):
        groups = 13
        part = torch.empty(groups * 32 * 9 * cin, device="cuda")
        out = torch.empty((32, 9, cin), device="cuda")
        gd, ad = dev(stream, t_bf16(g), t_bf16(a))
        sur.sur_weight_grad(gd, ad, cin, relu_in, part, groups, out, stream, dil)
        stream.synchronize()
        ref = cr.conv_weight_grad(g, cr.relu(a) if relu_in else a, dil)
        assert relmax(host(out), ref) <= 2e-5
    bpart = torch.empty(5 * 32, device="cuda")
    bout = torch.empty(32, device="cuda")
    (gd,) = dev(stream, t_bf16(g))
    sur.sur_bias_grad(gd, bpart, 5, bout, stream)
    stream.synchronize()
    assert relmax(host(bout), g.sum(axis=(0, 1, 2))) <= 2e-5


def test_adam_and_mse(stream):
    rng = np.random.default_rng(3)
    announce("adam_mse")
    p = rng.standard_normal(1000)
    gr = rng.standard_normal(1000)
    m1 = np.zeros(1000)
    m2 = np.zeros(1000)
    tp, tg, tm1, tm2 = t_f32(p), t_f32(gr), t_f32(m1), t_f32(m2)
    pb = torch.empty(1000, dtype=torch.bfloat16, device="cuda")
    dev(stream, tp, tg, tm1, tm2, pb)
    for t in (1, 2, 3):
        sur.sur_adam(tp, tg, tm1, tm2, pb, 1e-2, t, stream)
        p, m1, m2 = cr.adam(p, gr, m1, m2, t, lr=1e-2)
    stream.synchronize()
    assert relmax(host(tp), p) <= 1e-6
    assert np.array_equal(host(pb), cr.bf16_round(host(tp)))
    N, H, W = 1, 3, 32
    d = rng.standard_normal((N, H, W, 32)).astype(np.float32)
    tg4 = rng.standard_normal((N, H, W, 4)).astype(np.float32)
    grad = torch.empty((N, H, W, 32), dtype=torch.bfloat16, device="cuda")
    part = torch.empty(7, device="cuda")
    dd, td = dev(stream, t_f32(d), t_f32(tg4))
    sur.sur_mse(dd, td, 0.25, grad, part, stream)
    stream.synchronize()
    e = d[..., :4].astype(np.float64) - tg4
    assert abs(float(part.sum()) - np.sum(e * e)) <= 1e-5 * np.sum(e * e)
    gref = np.zeros((N, H, W, 32))
    gref[..., :4] = 0.5 * e
    assert np.all(np.abs(host(grad) - cr.bf16_round(gref)) <= 2 ** -7 * np.abs(gref) + 1e-7)


def test_network_gradients_vs_reference():
    """Whole-network loss, output and gradients against the FP64 reference
    with BF16 storage emulated.  End to end the gradients agree within 3e-2:
    an FP32-versus-FP64 difference in a sum can round a stored BF16
    activation to the neighbouring value (a flip of one BF16 step, 2^-8
    relative), and the flips of the forward pass change the backward's inputs.
    The flips are counted, and given the GPU's own activations and output
    gradient the reference backward pass agrees with the GPU's within 1e-4 per
    layer (measured: at most 1.8e-5; flips in 4e-5 to 3e-3 of the activations
    per layer)."""
    announce("network_gradients")
    net = sur.Surrogate(seed=3)
    rng = np.random.default_rng(5)
    N, H, W = 2, 40, 64
    x = np.zeros((N, H, W, 8))
    x[..., :6] = rng.standard_normal((N, H, W, 6))
    x = cr.bf16_round(x)
    target = rng.standard_normal((N, H, W, 4)).astype(np.float32)
    loss, gW, gb, delta = net.gradients(t_bf16(x), t_f32(target))
    ref = cr.NetRef([w.cpu().numpy() for w in net.W], [b.cpu().numpy() for b in net.b], net.dil)
    rloss, rgW, rgb, rdelta = ref.loss_and_grads(x, target.astype(np.float64), 1.0)
    assert abs(loss - rloss) <= 1e-3 * rloss
    assert relmax(host(delta)[..., :4], rdelta[..., :4]) <= 2e-2
    for i in range(6):
        g, r = host(gW[i]), rgW[i]
        e = np.linalg.norm(g - r) / max(np.linalg.norm(r), 1e-30)
        assert e <= 3e-2, (i, e)
        e = np.linalg.norm(host(gb[i]) - rgb[i]) / max(np.linalg.norm(rgb[i]), 1e-30)
        assert e <= 3e-2, (i, "bias", e)
    # BF16 flips of the forward activations, and the backward pass from the GPU's own activations
    hs_gpu = [host(net._buf[f"h{r}"]) for r in range(5)]
    gd_gpu = host(net._buf["gd"])
    _, hs_ref, _ = ref.forward(x)
    flips = [float(np.mean(hs_gpu[r] != hs_ref[r])) for r in range(5)]
    # differences beyond one BF16 step of the larger value: a flip carried through a residual
    # connection into a smaller activation
    big = []
    for r in range(5):
        a, b = hs_gpu[r], hs_ref[r]
        m = np.maximum(np.abs(a), np.abs(b))
        step = np.exp2(np.floor(np.log2(np.maximum(m, 1e-30))) - 7)
        big.append(float(np.mean((np.abs(a - b) > step) & (m > 1e-3 * np.abs(b).max()))))
    print(f"[grad] activations differing from the reference (fraction per layer): {flips}; "
          f"by more than one BF16 step: {big}", flush=True)
    assert max(flips) <= 0.01 and max(big) <= 2e-3
    sgW, sgb = ref.grads_from(x, hs_gpu, gd_gpu)
    errs = []
    for i in range(6):
        e = np.linalg.norm(host(gW[i]) - sgW[i]) / max(np.linalg.norm(sgW[i]), 1e-30)
        eb = np.linalg.norm(host(gb[i]) - sgb[i]) / max(np.linalg.norm(sgb[i]), 1e-30)
        errs.append((e, eb))
    print(f"[grad] given the GPU's activations, per-layer relative error (weights, bias): {errs}", flush=True)
    assert all(e <= 1e-4 and eb <= 1e-4 for e, eb in errs), errs


def test_training_fits_a_shift():
    """The GPU training loop learns a fixed map: the state shifted by one node
    in x (a pure transport over K steps), with the loss falling 10x."""
    announce("training_fits_shift")
    net = sur.Surrogate(seed=1)
    rng = np.random.default_rng(2)
    P, H, W = 32, 8, 64
    x = np.zeros((P, H, W, 8))
    yy, xx = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    for p in range(P):
        k = rng.integers(1, 4)
        ph = rng.uniform(0, 6.28)
        x[p, :, :, 0] = np.sin(2 * np.pi * k * xx / W + ph) * np.cos(np.pi * yy / H)
        x[p, :, :, 1] = 0.5 * np.cos(2 * np.pi * k * xx / W + ph)
    x = cr.bf16_round(x)
    y = (np.roll(x[..., :4], 1, axis=2) - x[..., :4]).astype(np.float32)
    X, Y = t_bf16(x), t_f32(y)
    hist = sur.train(net, X, Y, iters=300, batch=8, lr=3e-3, seed=0)
    assert np.mean(hist[-20:]) < 0.1 * np.mean(hist[:5]), (hist[:5], hist[-5:])


# ---- state-side kernels ------------------------------------------------------

def _cfg_scales():
    from paper_2306_11320_amd import workloads as wl
    cfg, _ = wl.sweep_instance(64, 256, 12.0, 3.0, 1.5)
    return cfg


def _rand_state(rng, h, w):
    return {k: torch.tensor(rng.standard_normal((h, w)).astype(np.float32), device="cuda").contiguous()
            for k in sur.FIELDS}


def test_pack_target_and_advance(stream):
    """sur_pack against its definition (BF16 rounding of the scaled fields);
    sur_advance(sur_pack_target(f0, f1)) takes f0 to f1 within FP32 rounding."""
    announce("pack_target_advance")
    rng = np.random.default_rng(21)
    cfg = _cfg_scales()
    sc = sur.scales_of(cfg, (0.01, 0.02, 0.03, 0.04, 0.05))
    h, w = 9, 64
    f0, f1 = _rand_state(rng, h, w), _rand_state(rng, h, w)
    x = torch.empty((h, w, 8), dtype=torch.bfloat16, device="cuda")
    dev(stream)
    sur.sur_pack(f0, sc, x, stream)
    t = torch.empty((h, w, 5), device="cuda")
    sur.sur_pack_target(f0, f1, sc, t, stream)
    stream.synchronize()
    H = {k: v.cpu().numpy().astype(np.float64) for k, v in f0.items()}
    y = np.arange(h, dtype=np.float64)[:, None]
    want = np.zeros((h, w, 8))
    want[..., 0] = H["phi"]
    want[..., 1] = H["ux"] / sc.u
    want[..., 2] = H["uy"] / sc.u
    want[..., 3] = (H["T"] - (sc.t_a + sc.t_b * y)) / sc.dT
    want[..., 4] = sc.c4
    want[..., 5] = sc.c5
    want[..., 6] = (H["p"] - sc.P * 0.5 * (1.0 - H["phi"])) / sc.P
    got = host(x)
    assert np.all(np.abs(got - cr.bf16_round(want)) <= 2 ** -8 * np.abs(want) + 1e-6)
    inc = np.array([sc.inc[c] for c in range(5)])
    tt = host(t)
    for c, k in enumerate(sur.FIELDS):
        d = (f1[k].double() - f0[k].double()).cpu().numpy() / inc[c]
        assert np.allclose(tt[..., c], d, rtol=2e-6, atol=1e-6 / inc[c])
    delta = torch.zeros((h, w, 32), device="cuda")
    delta[..., :5] = t
    g = {k: v.clone() for k, v in f0.items()}
    torch.cuda.synchronize()
    sur.sur_advance(delta, sc, g, stream)
    stream.synchronize()
    for k in sur.FIELDS:
        assert torch.allclose(g[k], f1[k], rtol=1e-5, atol=1e-5), k


@pytest.mark.parametrize("relu_in", [False, True])
@pytest.mark.parametrize("dil,W", [(1, 64), (16, 256), (3, 200), (2, 45), (1, 7), (20, 64)])
def test_conv_advance_fused(relu_in, dil, W, stream):
    """The output layer with the state update fused (sur_conv3x3_advance) is
    bitwise equal to the convolution into an FP32 buffer followed by
    sur_advance, on frames with whole and ragged last segments; and that
    update matches the FP64 reference convolution."""
    announce("conv_advance_fused", relu_in, dil, W)
    rng = np.random.default_rng(7 + relu_in + 10 * dil + W)
    H = 37
    cfg = _cfg_scales()
    sc = sur.scales_of(cfg, (0.01, 0.02, 0.03, 0.04, 0.05))
    x = cr.bf16_round(rng.standard_normal((1, H, W, 32)))
    w = cr.bf16_round(0.2 * rng.standard_normal((32, 9, 32)))
    b = rng.standard_normal(32).astype(np.float32)
    f0 = _rand_state(rng, H, W)
    xd, wd, bd = dev(stream, t_bf16(x), t_bf16(w), t_f32(b))
    g1 = {k: v.clone() for k, v in f0.items()}
    g2 = {k: v.clone() for k, v in f0.items()}
    delta = torch.empty((1, H, W, 32), device="cuda")
    dev(stream, delta, *g1.values(), *g2.values())
    sur.sur_conv3x3(xd, 32, wd, bd, None, None, delta, relu_in, stream, dil)
    sur.sur_advance(delta, sc, g1, stream)
    sur.sur_conv3x3_advance(xd, wd, bd, relu_in, sc, g2, stream, dil)
    stream.synchronize()
    for k in sur.FIELDS:
        assert torch.equal(g1[k], g2[k]), k
    a = cr.relu(x) if relu_in else x
    ref = cr.conv(a, w, b, dil)[0]
    for c, k in enumerate(sur.FIELDS):
        want = f0[k].double().cpu().numpy() + ref[..., c] * sc.inc[c]
        got = g2[k].double().cpu().numpy()
        assert np.abs(got - want).max() <= 1e-5 * (np.abs(want).max() + 1.0), k


@pytest.mark.parametrize("H,W,dil", [(37, 45, 1), (64, 96, 4), (200, 64, 16), (1024, 256, 1)])
def test_conv_advance_volume(H, W, dil, stream):
    """The output layer that also sums the light-phase volume
    (sur_conv3x3_advance_volume) leaves the state bitwise as
    sur_conv3x3_advance does and writes sur_light_volume's value of the
    updated phi within 1e-13 relative (FP64 sums in another order); on
    ragged and whole segments and on the largest grid (256 x 1024: one
    partial per resident workgroup).  Two calls in a row on one partials
    buffer, the second on a smaller frame, and the second again: the same sum,
    bitwise."""
    announce("conv_advance_volume", H, W, dil)
    rng = np.random.default_rng(H + W + dil)
    cfg = _cfg_scales()
    sc = sur.scales_of(cfg, (0.01, 0.02, 0.03, 0.04, 0.05))
    x = cr.bf16_round(rng.standard_normal((1, H, W, 32)))
    w = cr.bf16_round(0.2 * rng.standard_normal((32, 9, 32)))
    b = rng.standard_normal(32).astype(np.float32)
    f0 = _rand_state(rng, H, W)
    xd, wd, bd = dev(stream, t_bf16(x), t_bf16(w), t_f32(b))
    part = torch.empty(8 * sur.VOLUME_PARTS, dtype=torch.float64, device="cuda")
    lpart = torch.empty(8 * 256, dtype=torch.float64, device="cuda")
    vol = torch.zeros(4, dtype=torch.float64, device="cuda")
    small = {k: v[:H // 2].clone() for k, v in f0.items()}
    xs = xd[:, :H // 2].contiguous()
    g1 = {k: v.clone() for k, v in f0.items()}
    g2 = {k: v.clone() for k, v in f0.items()}
    s1 = {k: v.clone() for k, v in small.items()}
    s2 = {k: v.clone() for k, v in small.items()}
    dev(stream, part, lpart, vol, xs, *g1.values(), *g2.values(), *s1.values(), *s2.values())
    sur.sur_conv3x3_advance(xd, wd, bd, True, sc, g1, stream, dil)
    sur.sur_conv3x3_advance_volume(xd, wd, bd, True, sc, g2, part, vol[0:1], stream, dil)
    sur.sur_light_volume(g1["phi"], lpart, vol[1:2], stream)
    sur.sur_conv3x3_advance(xs, wd, bd, True, sc, s1, stream, dil)
    sur.sur_conv3x3_advance_volume(xs, wd, bd, True, sc, s2, part, vol[2:3], stream, dil)
    sur.sur_light_volume(s1["phi"], lpart, vol[3:4], stream)
    stream.synchronize()
    for k in sur.FIELDS:
        assert torch.equal(g1[k], g2[k]), k
        assert torch.equal(s1[k], s2[k]), k
    v = vol.cpu().numpy()
    assert abs(v[0] - v[1]) <= 1e-13 * abs(v[1]), (v[0], v[1])
    assert abs(v[2] - v[3]) <= 1e-13 * abs(v[3]), (v[2], v[3])
    # the same call again on the same input gives the same sum, bitwise
    s3 = {k: v.clone() for k, v in small.items()}
    dev(stream, *s3.values())
    sur.sur_conv3x3_advance_volume(xs, wd, bd, True, sc, s3, part, vol[0:1], stream, dil)
    stream.synchronize()
    assert vol[0].item() == v[2]


def test_generate_pairs_uneven_equals_single_lattices():
    """Training pairs from the batched generator (autotuned launch on lattices
    of uneven size) equal, bitwise, the pairs built from each lattice stepped
    on its own: states at the start times and their increments K steps later."""
    from paper_2306_11320_amd import lbm, workloads as wl
    announce("generate_pairs_uneven")
    items = wl.sweep(3, seed=9, nx_range=(64, 96), laplace_p=True)
    K, starts = 10, [20, 40]
    Xs, Ys = sur.generate_pairs_uneven(items, K, starts)
    for k, (cfg, f0) in enumerate(items):
        lat = lbm.Lattice(cfg, f0, lbm.FP32_DEV)
        sc = sur.scales_of(cfg)
        st = lat.stream
        ny, nx = lat.shapes[0]
        a = {key: torch.empty((ny, nx), device="cuda") for key in sur.FIELDS}
        b = {key: torch.empty((ny, nx), device="cuda") for key in sur.FIELDS}
        x = torch.empty((ny, nx, 8), dtype=torch.bfloat16, device="cuda")
        y = torch.empty((ny, nx, sur.N_OUT), device="cuda")
        torch.cuda.synchronize()
        t = 0
        for q, s0 in enumerate(starts):
            lat.step(s0 - t)
            lat.fields(0, out="f32", into=a)
            sur.sur_pack(a, sc, x, st)
            lat.step(K)
            t = s0 + K
            lat.fields(0, out="f32", into=b)
            sur.sur_pack_target(a, b, sc, y, st)
            st.synchronize()
            assert torch.equal(Xs[k][q].view(torch.int16), x.view(torch.int16)), (k, q)
            assert torch.equal(Ys[k][q], y), (k, q)
        lat.close()


def test_light_volume_and_judge(stream):
    announce("volume_judge")
    rng = np.random.default_rng(22)
    cfg = _cfg_scales()
    sc = sur.scales_of(cfg)
    h, w = 37, 64
    a, b = _rand_state(rng, h, w), _rand_state(rng, h, w)
    part = torch.empty(8 * 13, dtype=torch.float64, device="cuda")
    out = torch.full((8,), -7.0, dtype=torch.float64, device="cuda")
    dev(stream)
    sur.sur_light_volume(a["phi"], part, out[:1], stream)
    stream.synchronize()
    phi = a["phi"].double().cpu().numpy()
    assert abs(float(out[0]) - np.sum(0.5 * (1 - phi))) <= 1e-12 * np.sum(np.abs(phi)) * 10
    assert torch.all(out[1:] == -7.0)       # exactly one value written
    sur.sur_judge(a, b, sc, part, out, stream)
    stream.synchronize()
    A = {k: v.double().cpu().numpy() for k, v in a.items()}
    B = {k: v.double().cpu().numpy() for k, v in b.items()}
    y = np.arange(h, dtype=np.float64)[:, None]
    rest = {"phi": 1.0, "ux": 0.0, "uy": 0.0, "T": float(sc.t_a) + float(sc.t_b) * y}
    o = out.cpu().numpy()
    for c, k in enumerate(("phi", "ux", "uy", "T")):
        assert np.isclose(o[2 * c], np.sum((A[k] - B[k]) ** 2), rtol=1e-12)
        assert np.isclose(o[2 * c + 1], np.sum((B[k] - rest[k]) ** 2), rtol=1e-12)


def test_hybrid_bookkeeping():
    """With a zero tolerance every judged block falls back and the lattice
    update carries on from its own result: judging every block is then the
    plain lattice update, bitwise.  With a huge tolerance an untrained network
    runs undisturbed between judged blocks, and with a tiny one the judged
    blocks hand the following blocks to the lattice update."""
    from paper_2306_11320_amd import lbm, workloads as wl
    announce("hybrid_bookkeeping")
    cfg, f0 = wl.sweep_instance(64, 256, 12.0, 3.0, 1.5, laplace_p=True)
    ref = lbm.Lattice(cfg, f0, lbm.FP32_DEV)
    ref.step(300)
    fr = ref.fields(0, out="f32", to_host=False)
    lat = lbm.Lattice(cfg, f0, lbm.FP32_DEV)
    net = sur.Surrogate(seed=2, stream=lat.stream)
    h = sur.Hybrid(net, lat, cfg, K=100, check_every=1, tol_check=0.0, fallback_blocks=0)
    st = h.run(3)
    assert st["lbm_blocks"] == 3 and st["net_blocks"] == 0 and st["judged"] == 3 and st["fallbacks"] == 3
    for k in sur.FIELDS:
        assert torch.equal(h.s[k], fr[k]), k
    lat2 = lbm.Lattice(cfg, f0, lbm.FP32_DEV)
    net.stream = lat2.stream
    h2 = sur.Hybrid(net, lat2, cfg, K=100, check_every=4, tol_check=1e9, tol_vol=1e9, tol_check_u=1e9)
    st2 = h2.run(8)
    assert (st2["net_blocks"], st2["lbm_blocks"], st2["fallbacks"], st2["judged"]) == (6, 2, 0, 2)
    lat3 = lbm.Lattice(cfg, f0, lbm.FP32_DEV)
    net.stream = lat3.stream
    h3 = sur.Hybrid(net, lat3, cfg, K=100, check_every=4, tol_check=0.0, fallback_blocks=2)
    st3 = h3.run(10)
    # 3 network + 1 judged, 2 fallback, 3 network + 1 judged -> 10 blocks
    assert (st3["net_blocks"], st3["lbm_blocks"], st3["fallbacks"]) == (6, 4, 2)
    for L in (ref, lat, lat2, lat3):
        L.close()


def test_hybrid_graph_replay_equals_eager():
    """The network blocks between judged blocks replayed from a captured HIP
    graph give bitwise the state, volumes and judged errors of the same blocks
    launched one by one: undisturbed (four replays, with the judged blocks'
    own launches and synchronisations between them) and with every judged
    block falling back, so that the state buffers swap and the second buffer's
    graph is captured on its first use."""
    import os
    from paper_2306_11320_amd import lbm, workloads as wl
    announce("hybrid_graph_replay")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    net = sur.Surrogate.load(os.path.join(root, "paper_2306_11320_amd", "weights", "surrogate_k100_sweep2000.npz"))
    cfg, f0 = wl.sweep_instance(96, 256, 12.0, 3.0, 1.5, laplace_p=True)
    for kw, runs in ((dict(check_every=4, tol_check=1e9, tol_vol=1e9, tol_check_u=1e9), 4),
                     (dict(check_every=3, tol_check=0.0, fallback_blocks=1), 3)):
        # 4 blocks a run: 3 network + 1 judged, or 2 network (graph) + 1 judged (falls back) + 1 lattice
        hs, lats = [], []
        for graph in (False, True):
            lat = lbm.Lattice(cfg, f0, lbm.FP32_DEV)
            lat.step(200)
            net.stream = lat.stream
            hs.append(sur.Hybrid(net, lat, cfg, K=100, **kw, graph=graph))
            lats.append(lat)
        for r in range(runs):
            for h in hs:
                h.net.stream = h.lat.stream
                h.run(4)
            e, g = hs
            for k in sur.FIELDS:
                assert torch.equal(e.s[k], g.s[k]), (kw, r, k)
            assert torch.equal(e.vol, g.vol), (kw, r)
            assert e.stats["judge_errors"] == g.stats["judge_errors"], (kw, r)
            assert (e.stats["net_blocks"], e.stats["fallbacks"]) == (g.stats["net_blocks"], g.stats["fallbacks"])
        assert len(hs[1]._graphs) == (1 if kw["tol_check"] > 1 else 2)
        assert hs[0].stats["fallbacks"] == (0 if kw["tol_check"] > 1 else runs)
        for L in lats:
            L.close()


def test_trained_network_gain():
    """The earlier network, trained on 64 fixed 256 x 1024 lattices
    (weights/surrogate_k100.npz), against the plain FP32 lattice update on
    two fresh droplet lattices (sweep parameters, seed 55), 10 blocks of 100
    steps after 30000 steps of warm-up: the hybrid is at least twice as fast
    and needs no fallback; every field stays within 1 % of the lattice
    update; phi and T are at least 4 times closer to it than the state they
    started from (persistence); the velocity, whose per-block change is mostly
    the lattice's weakly damped sound waves, is closer than persistence."""
    import os
    from paper_2306_11320_amd.train_surrogate import sweep_items
    announce("trained_network_gain")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    net = sur.Surrogate.load(os.path.join(root, "paper_2306_11320_amd", "weights", "surrogate_k100.npz"))
    res = sur.evaluate(net, sweep_items(2, 55, 256, 1024), warm=30000, blocks=10, chunk=10, log=None)
    for r in res:
        eh, ep = r["err_hybrid"][-1], r["err_persistence"][-1]
        speedup = sum(r["t_ref_ms"]) / sum(r["t_hybrid_ms"])
        print(f"speedup {speedup:.2f} hybrid {eh} persistence {ep}", flush=True)
        assert speedup >= 2.0
        assert r["fallbacks"] == 0
        for k in ("phi", "T"):
            assert eh[k] <= 0.01 and eh[k] <= 0.25 * ep[k], k
        for k in ("ux", "uy"):
            assert eh[k] <= 0.01 and eh[k] < ep[k], k


@pytest.mark.parametrize("lattices", ["256x1024", "uneven"])
def test_sweep_trained_network_gain(lattices):
    """The production network, trained on 2000 trajectories of the batched-sweep
    generator (weights/surrogate_k100_sweep2000.npz), against the plain FP32
    lattice update on two fresh lattices (seed 55): 256 x 1024 lattices drawn
    with the sweep's parameters, or the generator's own lattices of uneven
    size; 10 blocks of 100 steps after 30000 steps of warm-up.  The hybrid is
    at least twice as fast and needs no fallback; every field stays within 1 %
    of the lattice update; phi and T are at least 4 times closer to it than
    persistence, the velocity closer than persistence.  (Measured: 0.51-0.95 %
    worst field, persistence 3.2-4.0 %.)"""
    import os
    from paper_2306_11320_amd import workloads as wl
    from paper_2306_11320_amd.train_surrogate import sweep_items
    announce("sweep_trained_network_gain", lattices)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    net = sur.Surrogate.load(os.path.join(root, "paper_2306_11320_amd", "weights", "surrogate_k100_sweep2000.npz"))
    items = sweep_items(2, 55, 256, 1024) if lattices == "256x1024" else wl.sweep(2, seed=55, laplace_p=True)
    res = sur.evaluate(net, items, warm=30000, blocks=10, chunk=10, log=None)
    for r in res:
        eh, ep = r["err_hybrid"][-1], r["err_persistence"][-1]
        speedup = sum(r["t_ref_ms"]) / sum(r["t_hybrid_ms"])
        print(f"speedup {speedup:.2f} hybrid {eh} persistence {ep}", flush=True)
        assert speedup >= 2.0
        assert r["fallbacks"] == 0
        for k in ("phi", "T"):
            assert eh[k] <= 0.01 and eh[k] <= 0.25 * ep[k], k
        for k in ("ux", "uy"):
            assert eh[k] <= 0.01 and eh[k] < ep[k], k
