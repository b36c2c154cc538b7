"""Learned surrogate of the lattice update: a residual network of 3x3
convolutions that advances the macroscopic state of a thermocapillary
droplet-migration lattice by K lattice time steps at once, with the lattice
Boltzmann update as its fallback and as the judge of its error.  Not part of
the paper's method; built beside it.

Every tensor operation of the network runs in the HIP kernels declared in
``include/surrogate.h`` (BF16 matrix-core convolutions with FP32 accumulation,
weight/bias gradient reductions, Adam, squared error, packing, state update,
volume and error reductions); this module allocates buffers with PyTorch,
marshals pointers and sequences the calls.

State of a frame: five FP32 fields phi, ux, uy, T and the pressure p.  The
pressure rides along so that a hand-back to the lattice update restarts at the
right pressure: a restart at p = 0 emits a pressure wave that spoils the
velocity field by tens of per cent.

Network (6 convolutions, 32 channels):
    h0 = conv(x, W0) + b0                      x: 8 channels (phi, ux/U, uy/U,
                                               (T - T_rest)/dT, c4, c5, p_dyn/P, 0)
    h_r = h_{r-1} + conv(relu(h_{r-1}), W_r) + b_r,   r = 1..4
    delta = conv(relu(h_4), W5) + b5           5 used output channels
with 3x3 taps dilated by DIL = (1, 2, 4, 8, 16, 1) per layer (receptive field
of radius 32 nodes, about half the distance sound travels in K = 100 steps)
and p_dyn = p - P (1 - phi) / 2 the pressure less its Young-Laplace part.
    f_c(t + K) = f_c(t) + delta_c inc_c        (FP32 state, c = phi, ux, uy, T, p)
Input scales per lattice: U the characteristic thermocapillary velocity,
dT = |grad T| R, P = sigma_ref / R (the Laplace pressure), T_rest the
conduction profile; conditioning c4 = log10(Ma) / 2, c5 = lambda_r - 1.
Output units inc_c = kappa_c * (1, U, U, dT, P), kappa fixed from the training
set (1 % of the rms deviation of each field from rest; 0.1 % for phi, 0.3 % for
T), so the loss weighs the fields by the relative error the judge measures,
phi and T more.
"""
from __future__ import annotations

import ctypes as C
import math
import time

import numpy as np

from . import lbm as _lbm

CIN = (8, 32, 32, 32, 32, 32)
DIL = (1, 2, 4, 8, 16, 1)       # dilation of each layer's 3x3 taps
N_IN = 7            # used input channels
N_OUT = 5           # phi, ux, uy, T, p
FIELDS = ("phi", "ux", "uy", "T", "p")

_sur = None


class SurScales(C.Structure):
    _fields_ = [("u", C.c_float), ("dT", C.c_float), ("t_a", C.c_float), ("t_b", C.c_float), ("P", C.c_float),
                ("c4", C.c_float), ("c5", C.c_float), ("inc", C.c_float * 5)]


def lib():
    global _sur
    if _sur is None:
        L = _lbm.lib()
        vp, ip, i64, f = C.c_void_p, C.c_int, C.c_int64, C.c_float
        sp = C.POINTER(SurScales)
        pp = C.POINTER(vp)
        L.sur_conv3x3.argtypes = [vp, ip, vp, vp, vp, vp, vp, ip, ip, ip, ip, ip, ip, vp]
        L.sur_adjoint_weights.argtypes = [vp, ip, vp, vp]
        L.sur_weight_grad.argtypes = [vp, vp, ip, ip, ip, ip, ip, ip, vp, ip, vp, vp]
        L.sur_wgrad_scratch_floats.restype = C.c_size_t
        L.sur_wgrad_scratch_floats.argtypes = [ip, ip]
        L.sur_bias_grad.argtypes = [vp, i64, vp, ip, vp, vp]
        L.sur_adam.argtypes = [vp, vp, vp, vp, vp, i64, f, f, f, f, ip, vp]
        L.sur_mse.argtypes = [vp, vp, i64, ip, f, vp, vp, ip, vp]
        L.sur_pack.argtypes = [pp, ip, ip, sp, vp, vp]
        L.sur_pack_target.argtypes = [pp, pp, i64, sp, vp, vp]
        L.sur_advance.argtypes = [vp, i64, sp, pp, vp]
        L.sur_conv3x3_advance.argtypes = [vp, vp, vp, ip, ip, ip, ip, sp, pp, vp]
        L.sur_conv3x3_advance_volume.argtypes = [vp, vp, vp, ip, ip, ip, ip, sp, pp, vp, vp, vp]
        L.sur_light_volume.argtypes = [vp, ip, ip, vp, ip, vp, vp]
        L.sur_judge.argtypes = [pp, pp, ip, ip, sp, vp, ip, vp, vp]
        L.sur_judge_noscratch.argtypes = [pp, pp, ip, ip, sp, ip, vp, vp]
        L.sur_last_error.restype = C.c_char_p
        _sur = L
    return _sur


def _ck(rc):
    if rc != 0:
        raise RuntimeError(f"surrogate kernel error {rc}: {lib().sur_last_error().decode()}")


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _s(stream):
    return C.c_void_p(stream.cuda_stream)


def _state(f):
    return (C.c_void_p * 5)(*[f[k].data_ptr() for k in FIELDS])


# ---- thin wrappers with the names of the C ABI -----------------------------

def sur_conv3x3(x, cin, w, bias, res, mask, out, relu_in, stream, dil=1):
    n, h, wd = x.shape[0], x.shape[1], x.shape[2]
    _ck(lib().sur_conv3x3(_p(x), cin, _p(w), _p(bias), _p(res), _p(mask), _p(out), int(out.element_size() == 4),
                          int(relu_in), int(dil), n, h, wd, _s(stream)))


def sur_adjoint_weights(w, cin, wt, stream):
    _ck(lib().sur_adjoint_weights(_p(w), cin, _p(wt), _s(stream)))


def sur_weight_grad(dy, x, cin, relu_in, part, groups, out, stream, dil=1):
    n, h, wd = dy.shape[0], dy.shape[1], dy.shape[2]
    _ck(lib().sur_weight_grad(_p(dy), _p(x), cin, int(relu_in), int(dil), n, h, wd, _p(part), groups, _p(out),
                              _s(stream)))


def sur_bias_grad(dy, part, groups, out, stream):
    npix = dy.numel() // 32
    _ck(lib().sur_bias_grad(_p(dy), npix, _p(part), groups, _p(out), _s(stream)))


def sur_adam(p, g, m1, m2, pb, lr, t, stream, b1=0.9, b2=0.999, eps=1e-8):
    _ck(lib().sur_adam(_p(p), _p(g), _p(m1), _p(m2), _p(pb), p.numel(), lr, b1, b2, eps, int(t), _s(stream)))


def sur_mse(delta, target, scale, grad, part, stream):
    nout = target.shape[-1]
    npix = target.numel() // nout
    _ck(lib().sur_mse(_p(delta), _p(target), npix, nout, scale, _p(grad), _p(part), part.numel(), _s(stream)))


def sur_pack(f, sc: SurScales, x, stream):
    h, w = f["phi"].shape
    _ck(lib().sur_pack(_state(f), h, w, C.byref(sc), _p(x), _s(stream)))


def sur_pack_target(f0, f1, sc: SurScales, t, stream):
    _ck(lib().sur_pack_target(_state(f0), _state(f1), f0["phi"].numel(), C.byref(sc), _p(t), _s(stream)))


def sur_advance(delta, sc: SurScales, f, stream):
    _ck(lib().sur_advance(_p(delta), f["phi"].numel(), C.byref(sc), _state(f), _s(stream)))


def sur_conv3x3_advance(x, w, bias, relu_in, sc: SurScales, f, stream, dil=1):
    h, wd = f["phi"].shape
    _ck(lib().sur_conv3x3_advance(_p(x), _p(w), _p(bias), int(relu_in), int(dil), h, wd, C.byref(sc), _state(f),
                                  _s(stream)))


VOLUME_PARTS = 512   # SUR_VOLUME_PARTS


def sur_conv3x3_advance_volume(x, w, bias, relu_in, sc: SurScales, f, part, vol, stream, dil=1):
    h, wd = f["phi"].shape
    _ck(lib().sur_conv3x3_advance_volume(_p(x), _p(w), _p(bias), int(relu_in), int(dil), h, wd, C.byref(sc),
                                         _state(f), _p(part), _p(vol), _s(stream)))


def sur_light_volume(phi, part, out, stream):
    h, w = phi.shape
    _ck(lib().sur_light_volume(_p(phi), h, w, _p(part), part.numel() // 8, _p(out), _s(stream)))


def sur_judge(a, b, sc: SurScales, part, out, stream):
    h, w = a["phi"].shape
    _ck(lib().sur_judge(_state(a), _state(b), h, w, C.byref(sc), _p(part), part.numel() // 8, _p(out), _s(stream)))


def sur_judge_noscratch(a, b, sc: SurScales, groups, out, stream):
    h, w = a["phi"].shape
    _ck(lib().sur_judge_noscratch(_state(a), _state(b), h, w, C.byref(sc), int(groups), _p(out), _s(stream)))


# ---- scaling of a lattice's state -----------------------------------------

KAPPA_UNIT = (1.0, 1.0, 1.0, 1.0, 1.0)


def scales_of(cfg: dict, kappa=KAPPA_UNIT) -> SurScales:
    """Scales of a droplet-migration lattice (periodic in x, walls in y at
    T = 0 and gradT * ny)."""
    m = cfg["meta"]
    U = float(m["U"])
    R = float(m["R"])
    gradT = float(m["gradT"])
    dT = gradT * R
    Ma = float(m.get("Ma", 1.0))
    lr = float(m.get("lambda_r", cfg["lambda_l"] / cfg["lambda_h"]))
    P = float(cfg["sigma_ref"]) / R
    unit = (1.0, U, U, dT, P)
    return SurScales(U, dT, 0.5 * gradT, gradT, P, math.log10(max(Ma, 1e-3)) / 2.0, lr - 1.0,
                     (C.c_float * 5)(*[float(k) * u for k, u in zip(kappa, unit)]))


class Surrogate:
    """Parameters, Adam state and work buffers of the network on one device."""

    def __init__(self, device="cuda:0", seed=5, stream=None, kappa=KAPPA_UNIT, dil=DIL):
        import torch
        self.torch = torch
        self.dil = tuple(int(d) for d in dil)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self.kappa = tuple(float(k) for k in kappa)
        g = torch.Generator().manual_seed(seed)
        self.W, self.Wb, self.b = [], [], []
        for layer, cin in enumerate(CIN):
            fan_in = 9 * (cin if layer else N_IN)
            std = math.sqrt(2.0 / fan_in) * (0.2 if 0 < layer < 5 else (0.05 if layer == 5 else 1.0))
            w = torch.randn((32, 9, cin), generator=g) * std
            if layer == 0:
                w[:, :, N_IN:] = 0.0
            if layer == 5:
                w[N_OUT:] = 0.0
            w = w.to(self.device)
            self.W.append(w.contiguous())
            self.Wb.append(w.to(torch.bfloat16).contiguous())
            self.b.append(torch.zeros(32, device=self.device))
        self.step_count = 0
        self.adam = {}
        for name, ts in (("W", self.W), ("b", self.b)):
            self.adam[name] = [(torch.zeros_like(t), torch.zeros_like(t)) for t in ts]
        self.Wt = [torch.empty((32, 9, 32), dtype=torch.bfloat16, device=self.device) for _ in CIN]
        self._buf = {}

    @staticmethod
    def n_params() -> int:
        """Trainable parameters: N_IN used input channels in layer 0, N_OUT outputs in layer 5."""
        return (32 * 9 * N_IN + 32) + 4 * (32 * 9 * 32 + 32) + (N_OUT * 9 * 32 + N_OUT)

    @staticmethod
    def flops_per_pixel() -> int:
        """2 x multiply-adds of one forward pass per pixel as computed (32
        output channels in every layer, 8 input channels in the first)."""
        return 2 * 9 * 32 * (8 + 5 * 32)

    def _get(self, name, shape, dtype):
        t = self._buf.get(name)
        if t is None or tuple(t.shape) != tuple(shape) or t.dtype != dtype:
            t = self.torch.empty(shape, dtype=dtype, device=self.device)
            self._buf[name] = t
        return t

    # ---- network ----
    def _hidden(self, x, keep: bool):
        """Layers 0..4 on x (BF16 [N, H, W, 8]): the last hidden activation and,
        if keep, all five."""
        N, H, W, _ = x.shape
        bf = self.torch.bfloat16
        hs = []
        h = self._get("h0", (N, H, W, 32), bf)
        d = self.dil
        sur_conv3x3(x, 8, self.Wb[0], self.b[0], None, None, h, False, self.stream, d[0])
        hs.append(h)
        for r in range(1, 5):
            hn = self._get(f"h{r}" if keep else f"hp{r % 2}", (N, H, W, 32), bf)
            sur_conv3x3(h, 32, self.Wb[r], self.b[r], h, None, hn, True, self.stream, d[r])
            h = hn
            hs.append(h)
        return h, hs

    def forward(self, x, keep: bool = False):
        """x: BF16 [N, H, W, 8].  Returns delta (FP32 [N, H, W, 32]) and, if
        keep, the BF16 activations h0..h4 for the backward pass."""
        N, H, W, _ = x.shape
        h, hs = self._hidden(x, keep)
        delta = self._get("delta", (N, H, W, 32), self.torch.float32)
        sur_conv3x3(h, 32, self.Wb[5], self.b[5], None, None, delta, True, self.stream, self.dil[5])
        return delta, (hs if keep else None)

    def _backward(self, x, hs, gd, gW, gb, wpart, bpart, groups):
        torch = self.torch
        N, H, W, _ = x.shape
        d = self.dil
        sur_weight_grad(gd, hs[4], 32, True, wpart, groups, gW[5], self.stream, d[5])
        sur_bias_grad(gd, bpart, groups, gb[5], self.stream)
        sur_adjoint_weights(self.Wb[5], 32, self.Wt[5], self.stream)
        gh = self._get("gh0", (N, H, W, 32), torch.bfloat16)
        sur_conv3x3(gd, 32, self.Wt[5], None, None, hs[4], gh, False, self.stream, d[5])
        for r in range(4, 0, -1):
            sur_weight_grad(gh, hs[r - 1], 32, True, wpart, groups, gW[r], self.stream, d[r])
            sur_bias_grad(gh, bpart, groups, gb[r], self.stream)
            sur_adjoint_weights(self.Wb[r], 32, self.Wt[r], self.stream)
            gn = self._get(f"gh{r % 2 + 1}", (N, H, W, 32), torch.bfloat16)
            sur_conv3x3(gh, 32, self.Wt[r], None, gh, hs[r - 1], gn, False, self.stream, d[r])
            gh = gn
        sur_weight_grad(gh, x, 8, False, wpart, groups, gW[0], self.stream, d[0])
        sur_bias_grad(gh, bpart, groups, gb[0], self.stream)

    def train_step(self, x, target, lr: float, groups: int = 256) -> float:
        """One Adam step on the mean squared error of delta[..., :N_OUT]
        against the target increment (FP32 [N, H, W, N_OUT], in units of inc).
        Returns the mean squared error before the step."""
        torch = self.torch
        N, H, W, _ = x.shape
        npix = N * H * W
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        delta, hs = self.forward(x, keep=True)
        gd = self._get("gd", (N, H, W, 32), torch.bfloat16)
        part = self._get("mse_part", (256,), torch.float32)
        sur_mse(delta, target, 1.0 / (npix * N_OUT), gd, part, self.stream)
        gW = [self._get(f"gW{i}", tuple(w.shape), torch.float32) for i, w in enumerate(self.W)]
        gb = [self._get(f"gb{i}", (32,), torch.float32) for i in range(6)]
        wpart = self._get("wpart", (groups * 32 * 9 * 32,), torch.float32)
        bpart = self._get("bpart", (groups * 32,), torch.float32)
        self._backward(x, hs, gd, gW, gb, wpart, bpart, groups)
        self.step_count += 1
        for i in range(6):
            m1, m2 = self.adam["W"][i]
            sur_adam(self.W[i], gW[i], m1, m2, self.Wb[i], lr, self.step_count, self.stream)
            m1, m2 = self.adam["b"][i]
            bb = self._get(f"bb{i}", (32,), torch.bfloat16)
            sur_adam(self.b[i], gb[i], m1, m2, bb, lr, self.step_count, self.stream)
        torch.cuda.current_stream(self.device).wait_stream(self.stream)
        return float(part.sum().item()) / (npix * N_OUT)

    def gradients(self, x, target, groups: int = 64):
        """Loss (sum of squares over the N_OUT channels) and gradients, without
        an update (for checks)."""
        torch = self.torch
        N, H, W, _ = x.shape
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        delta, hs = self.forward(x, keep=True)
        gd = self._get("gd", (N, H, W, 32), torch.bfloat16)
        part = self._get("mse_part", (256,), torch.float32)
        sur_mse(delta, target, 1.0, gd, part, self.stream)
        gW = [torch.empty_like(w) for w in self.W]
        gb = [torch.empty(32, device=self.device) for _ in range(6)]
        wpart = torch.empty(groups * 32 * 9 * 32, device=self.device)
        bpart = torch.empty(groups * 32, device=self.device)
        self._backward(x, hs, gd, gW, gb, wpart, bpart, groups)
        self.stream.synchronize()
        return float(part.sum().item()), gW, gb, delta

    def state_dict(self) -> dict:
        out = {f"W{i}": self.W[i].cpu().numpy() for i in range(6)}
        out.update({f"b{i}": self.b[i].cpu().numpy() for i in range(6)})
        out["kappa"] = np.asarray(self.kappa, np.float64)
        out["dil"] = np.asarray(self.dil, np.int64)
        return out

    def load_state_dict(self, sd: dict) -> None:
        torch = self.torch
        for i in range(6):
            self.W[i].copy_(torch.as_tensor(np.asarray(sd[f"W{i}"], np.float32)).to(self.device))
            self.Wb[i].copy_(self.W[i].to(torch.bfloat16))
            self.b[i].copy_(torch.as_tensor(np.asarray(sd[f"b{i}"], np.float32)).to(self.device))
        self.kappa = tuple(float(k) for k in np.asarray(sd["kappa"]).reshape(-1))
        self.dil = tuple(int(d) for d in np.asarray(sd["dil"]).reshape(-1))

    def save(self, path: str) -> None:
        np.savez(path, **self.state_dict())

    @classmethod
    def load(cls, path: str, device="cuda:0", stream=None) -> "Surrogate":
        with np.load(path, allow_pickle=False) as z:
            sd = {k: z[k] for k in z.files}
        net = cls(device=device, stream=stream)
        net.load_state_dict(sd)
        return net

    # ---- one block of K lattice steps on a state ----
    def advance(self, state: dict, sc: SurScales, part=None, vol=None) -> None:
        """state (five FP32 (ny, nx) device tensors) += the predicted increment,
        on self.stream.  With part and vol (FP64 device tensors of
        8 * VOLUME_PARTS elements and of one element) the
        output layer also writes the light-phase volume of the updated phi
        into vol (output-layer dilation <= 16)."""
        ny, nx = state["phi"].shape
        x = self._get("x1", (1, ny, nx, 8), self.torch.bfloat16)
        sur_pack(state, sc, x, self.stream)
        h, _ = self._hidden(x, False)
        # the output layer adds its increment to the state directly
        if vol is None:
            sur_conv3x3_advance(h, self.Wb[5], self.b[5], True, sc, state, self.stream, self.dil[5])
        else:
            sur_conv3x3_advance_volume(h, self.Wb[5], self.b[5], True, sc, state, part, vol, self.stream, self.dil[5])


# ---- data from the lattice Boltzmann update --------------------------------

def _tuned_batch(items, device):
    """The batched FP32 lattice of `items` with the autotuner's launch
    configuration, chosen on a throwaway copy (trial steps advance the state
    they run on; the choice does not change the results, which are bitwise
    independent of the tile shape and grid)."""
    probe = _lbm.Lattice.batch(items, _lbm.FP32_DEV, device=device)
    try:
        tuned = probe.autotune(steps_per_trial=4)
    finally:
        probe.close()
    lat = _lbm.Lattice.batch(items, _lbm.FP32_DEV, device=device)
    lat.set_tile(tuned["tile"])
    lat.set_grid(tuned["grid"])
    return lat


def generate_pairs(items, K: int, starts, device="cuda:0"):
    """Runs the batched FP32 lattice update over `items` (all of one size) and
    returns network inputs X (BF16 [P, H, W, 8]) and target increments Y (FP32
    [P, H, W, N_OUT], in units of (1, U, U, dT, P)) of the states K steps
    later, for every start time in `starts` and every lattice."""
    import torch
    lat = _tuned_batch(items, device)
    ny, nx = lat.shapes[0]
    n = len(items)
    P = n * len(starts)
    X = torch.empty((P, ny, nx, 8), dtype=torch.bfloat16, device=device)
    Y = torch.empty((P, ny, nx, N_OUT), dtype=torch.float32, device=device)
    sc = [scales_of(c) for c, _ in items]
    st = lat.stream
    f0 = [{k: torch.empty((ny, nx), device=device) for k in FIELDS} for _ in range(n)]
    f1 = {k: torch.empty((ny, nx), device=device) for k in FIELDS}
    t = 0
    for q, s in enumerate(sorted(starts)):
        if s < t:
            raise ValueError("start times must be at least K apart")
        lat.step(s - t)
        for k in range(n):
            lat.fields(k, out="f32", into=f0[k])
            sur_pack(f0[k], sc[k], X[q * n + k], st)
        lat.step(K)
        t = s + K
        for k in range(n):
            lat.fields(k, out="f32", into=f1)
            sur_pack_target(f0[k], f1, sc[k], Y[q * n + k], st)
    st.synchronize()
    lat.close()
    return X, Y


def generate_pairs_uneven(items, K: int, starts, device="cuda:0"):
    """As generate_pairs for lattices of any sizes (one batched launch per
    step): returns per-lattice lists Xs[l] (BF16 [S, H_l, W_l, 8]) and Ys[l]
    (FP32 [S, H_l, W_l, N_OUT]), S = len(starts)."""
    import torch
    lat = _tuned_batch(items, device)
    n = len(items)
    S = len(starts)
    Xs = [torch.empty((S, ny, nx, 8), dtype=torch.bfloat16, device=device) for ny, nx in lat.shapes]
    Ys = [torch.empty((S, ny, nx, N_OUT), dtype=torch.float32, device=device) for ny, nx in lat.shapes]
    sc = [scales_of(c) for c, _ in items]
    st = lat.stream
    f0 = [{k: torch.empty(shp, device=device) for k in FIELDS} for shp in lat.shapes]
    f1 = [{k: torch.empty(shp, device=device) for k in FIELDS} for shp in lat.shapes]
    t = 0
    for q, s in enumerate(sorted(starts)):
        if s < t:
            raise ValueError("start times must be at least K apart")
        lat.step(s - t)
        for k in range(n):
            lat.fields(k, out="f32", into=f0[k])
            sur_pack(f0[k], sc[k], Xs[k][q], st)
        lat.step(K)
        t = s + K
        for k in range(n):
            lat.fields(k, out="f32", into=f1[k])
            sur_pack_target(f0[k], f1[k], sc[k], Ys[k][q], st)
    st.synchronize()
    lat.close()
    return Xs, Ys


def dataset_kappa_uneven(Xs, frac=(0.001, 0.01, 0.01, 0.003, 0.01)) -> tuple:
    """dataset_kappa over frames of several sizes (mean squares weighted by
    pixel count)."""
    import torch
    tot = sum(x[..., 0].numel() for x in Xs)

    def ms(f):
        return sum(float(torch.sum(f(x).float() ** 2).item()) for x in Xs) / tot
    k_u = math.sqrt(0.5 * (ms(lambda x: x[..., 1]) + ms(lambda x: x[..., 2])))
    rms = (math.sqrt(ms(lambda x: x[..., 0].float() - 1.0)), k_u, k_u, math.sqrt(ms(lambda x: x[..., 3])),
           math.sqrt(ms(lambda x: x[..., 6].float() + 0.5 * (1.0 - x[..., 0].float()))))
    return tuple(f * v for f, v in zip(frac, rms))


def train_streamed(net: "Surrogate", batches, K: int, starts, iters_per_batch: int, frames: int,
                   crop_rows: int, lr: float = 1e-3, seed: int = 5, log=print, on_batch=None) -> list:
    """Trains on lattice trajectories generated batch by batch and discarded
    after use: for each batch of lattice items (any sizes), the batched FP32
    lattice update produces the pairs of every start time, then
    `iters_per_batch` Adam steps each take `frames` pairs of one randomly
    chosen lattice of the batch (one frame size per step), cut to a random
    band of `crop_rows` rows at full width (frames are periodic in x).  The
    learning rate decays by a cosine over all steps.  The network's kappa is
    set from the first batch.  Returns the loss history."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    total = iters_per_batch * len(batches)
    hist, it = [], 0
    for bi, items in enumerate(batches):
        t0 = time.perf_counter()
        Xs, Ys = generate_pairs_uneven(items, K, starts, device=net.device)
        if bi == 0 and net.kappa == KAPPA_UNIT:
            net.kappa = dataset_kappa_uneven(Xs)
        for Y in Ys:
            for c in range(N_OUT):
                Y[..., c] /= net.kappa[c]
        t_gen = time.perf_counter() - t0
        t0 = time.perf_counter()
        S = len(starts)
        for _ in range(iters_per_batch):
            li = int(torch.randint(0, len(Xs), (1,), generator=g))
            X, Y = Xs[li], Ys[li]
            idx = torch.randint(0, S, (frames,), generator=g).to(X.device)
            xb, yb = X.index_select(0, idx), Y.index_select(0, idx)
            H = X.shape[1]
            if crop_rows < H:
                y0 = int(torch.randint(0, H - crop_rows + 1, (1,), generator=g))
                xb, yb = xb[:, y0:y0 + crop_rows], yb[:, y0:y0 + crop_rows]
            lr_t = lr * 0.5 * (1 + math.cos(math.pi * it / max(1, total)))
            hist.append(net.train_step(xb.contiguous(), yb.contiguous(), lr_t))
            it += 1
        torch.cuda.synchronize(net.device)
        t_train = time.perf_counter() - t0
        if log:
            log(f"[stream] batch {bi + 1}/{len(batches)}: {len(items)} lattices, {len(items) * S} pairs generated in "
                f"{t_gen:.1f} s, {iters_per_batch} steps in {t_train:.1f} s, loss {np.mean(hist[-iters_per_batch:]):.3e}")
        if on_batch:
            on_batch(bi, hist)
        del Xs, Ys
    return hist


def dataset_kappa(X, frac=(0.001, 0.01, 0.01, 0.003, 0.01)) -> tuple:
    """kappa_c = frac_c x the rms deviation from rest of field c over the
    inputs X (scaled units: phi - 1, u / U, (T - T_rest) / dT, p / P).  phi
    and T get finer units: their increments are smooth in time and local, so
    learnable, while those of u and p carry the lattice's weakly damped sound
    waves; and phi errors are what a restart of the lattice update from the
    network's state is most sensitive to (the chemical potential holds its
    second derivative)."""
    import torch

    def ms(a):
        return float(torch.mean(a.float() ** 2).item())
    k_u = math.sqrt(0.5 * (ms(X[..., 1]) + ms(X[..., 2])))
    p_over_P = X[..., 6].float() + 0.5 * (1.0 - X[..., 0].float())
    rms = (math.sqrt(ms(X[..., 0] - 1.0)), k_u, k_u, math.sqrt(ms(X[..., 3])), math.sqrt(ms(p_over_P)))
    return tuple(f * v for f, v in zip(frac, rms))


def train(net: Surrogate, X, Y, iters: int, batch: int, lr: float = 1e-3, seed: int = 5, log_every: int = 0,
          crop_rows: int | None = None):
    """Adam on random mini-batches (optionally random bands of crop_rows
    rows at full width, since frames are periodic in x) with a cosine
    learning-rate decay.  Returns the loss history."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    P, H = X.shape[0], X.shape[1]
    hist = []
    for it in range(iters):
        idx = torch.randint(0, P, (batch,), generator=g).to(X.device)
        xb = X.index_select(0, idx)
        yb = Y.index_select(0, idx)
        if crop_rows is not None and crop_rows < H:
            y0 = int(torch.randint(0, H - crop_rows + 1, (1,), generator=g))
            xb, yb = xb[:, y0:y0 + crop_rows], yb[:, y0:y0 + crop_rows]
        lr_t = lr * 0.5 * (1 + math.cos(math.pi * it / max(1, iters)))
        loss = net.train_step(xb.contiguous(), yb.contiguous(), lr_t)
        hist.append(loss)
        if log_every and (it % log_every == 0 or it == iters - 1):
            print(f"[train] iter {it} loss {loss:.4e}", flush=True)
    return hist


# ---- rollout with the lattice update as fallback and judge -----------------

class Hybrid:
    """Advances one FP32 lattice by blocks of K steps with the network, the
    lattice update judging every `check_every`-th block and taking over when
    the network fails.

    A judged block runs the lattice update for one block from the network's
    state (a shift restart: the populations' non-equilibrium part is kept, the
    equilibria move to the network's fields, pressure included) beside the
    network's own prediction of that block, and compares the two (relative L2
    on deviations from rest).  phi and T trigger above `tol_check`.  Right
    after a restart the lattice's velocity carries a capillary transient (the
    network's small phi errors change the interface's chemical potential), so
    the judged velocity error overstates the network's own (measured: 0.9-2.1 %
    judged where the velocity is 0.5-1.0 % off the plain lattice update); the
    velocity triggers above `tol_check_u`, set above that transient.  A
    trigger, or a light-phase volume drift above `tol_vol` since the start,
    hands the following `fallback_blocks` blocks to the lattice update, which
    continues from its judged result; otherwise the network's state
    continues.

    With graph=True the run of check_every - 1 network blocks between judged
    blocks (packing, six layers and the volume reduction per block) is
    captured once per state buffer into a HIP graph and replayed: one launch
    instead of ~8 per block, for small lattices whose kernels take less time
    than their launches (at 256 x 1024 the launches keep ahead of the GPU and
    the replay measured 1-3 % slower per 10 blocks).  The graph holds the
    network's weights and buffers as they were at capture: load other weights
    into the network, or use it on a lattice of another size, only through a
    new Hybrid."""

    TRIGGER = (0, 3)            # phi, T
    TRIGGER_U = (1, 2)          # ux, uy

    def __init__(self, net: Surrogate, lat, cfg: dict, K: int = 100, check_every: int = 10,
                 tol_check: float = 0.01, tol_vol: float = 0.01, fallback_blocks: int | None = None,
                 tol_check_u: float = 0.03, graph: bool = False):
        import torch
        self._torch = torch
        if net.stream is not lat.stream:
            raise ValueError("the network must run on the lattice's stream")
        if check_every < 1:
            raise ValueError("check_every must be >= 1")
        self.net, self.lat, self.K = net, lat, int(K)
        self.C = int(check_every)
        self.tol_check, self.tol_vol = float(tol_check), float(tol_vol)
        self.tol_check_u = float(tol_check_u)
        self.fallback_blocks = self.C if fallback_blocks is None else int(fallback_blocks)
        self.sc = scales_of(cfg, net.kappa)
        ny, nx = lat.shapes[0]
        dev = lat.device
        self.s = {k: torch.empty((ny, nx), device=dev) for k in FIELDS}
        self.s_lbm = {k: torch.empty((ny, nx), device=dev) for k in FIELDS}
        self.part = torch.empty(8 * 256, dtype=torch.float64, device=dev)
        # the judge's sums, then the light-phase volumes after each network block (and at the start, last):
        # one buffer, read back by one copy into pinned memory per judged block
        self.red = torch.zeros(8 + self.C + 1, dtype=torch.float64, device=dev)
        self.judge_out, self.vol = self.red[:8], self.red[8:]
        self.red_host = torch.empty(8 + self.C + 1, dtype=torch.float64, pin_memory=True)
        # the output layer sums the volume's partials itself when its dilation allows
        self.vpart = torch.empty(8 * VOLUME_PARTS, dtype=torch.float64, device=dev) if net.dil[5] <= 16 else None
        lat.set_graph_steps(self.K)
        lat.fields(0, out="f32", into=self.s)
        sur_light_volume(self.s["phi"], self.part, self.vol[self.C:], lat.stream)
        lat.stream.synchronize()
        self.vol0 = float(self.vol[self.C].item())
        self.stats = dict(blocks=0, net_blocks=0, lbm_blocks=0, judged=0, fallbacks=0, max_judge=0.0,
                          max_judge_u=0.0, max_drift=0.0, judge_errors=[])
        self.lat_current = True     # the lattice holds self.s
        self.fallback_left = 0
        self.graph = bool(graph)
        self._graphs = {}           # state buffer (phi's address) -> (graph, tensors it reads or writes)
        if self.graph and self.C > 1:
            # captured here, outside any timing; the other buffer's graph on its first use (after a fallback)
            self._graphs[self.s["phi"].data_ptr()] = self._capture(self.C - 1)

    def _net_run(self, n: int):
        """n network blocks on self.s; the light-phase volume after block i
        into self.vol[i]."""
        st = self.lat.stream
        if self.graph and n == self.C - 1:
            key = self.s["phi"].data_ptr()
            g = self._graphs.get(key)
            if g is None:
                g = self._graphs[key] = self._capture(n)
            with self._torch.cuda.stream(st):      # replay() launches on the current stream
                g[0].replay()
            return
        for i in range(n):
            self._net_block(self.s, i)

    def _net_block(self, s: dict, i: int):
        """One network block on s, the light-phase volume after it into self.vol[i]."""
        if self.vpart is not None:
            self.net.advance(s, self.sc, self.vpart, self.vol[i:i + 1])
        else:
            self.net.advance(s, self.sc)
            sur_light_volume(s["phi"], self.part, self.vol[i:i + 1], self.lat.stream)

    def _capture(self, n: int):
        import torch
        st = self.lat.stream
        # first-call work (the network's buffers) outside the capture, on a copy
        with torch.cuda.stream(st):
            tmp = {k: v.clone() for k, v in self.s.items()}
        self._net_block(tmp, 0)
        st.synchronize()
        del tmp
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=st):
            for i in range(n):
                self._net_block(self.s, i)
        keep = [*self.s.values(), self.part, self.vol, self.vpart, *self.net._buf.values(), *self.net.Wb, *self.net.b]
        return g, keep

    def _lbm_block(self, lat_current: bool):
        if not lat_current:
            self.lat.reinit_fields(self.s, shift=True, sync_free=True)
        self.lat.step(self.K)
        self.lat.fields(0, out="f32", into=self.s)
        self.stats["lbm_blocks"] += 1

    def run(self, blocks: int) -> dict:
        """Advances `blocks` blocks (calls may follow one another)."""
        st = self.lat.stream
        if self.net.stream is not st:
            raise ValueError("the network must run on the lattice's stream")
        lat_current = self.lat_current
        fallback_left = self.fallback_left
        b = 0
        while b < blocks:
            if fallback_left > 0:
                self._lbm_block(lat_current)
                lat_current = True
                fallback_left -= 1
                b += 1
                continue
            n_net = min(self.C - 1, blocks - b - 1)
            if n_net:
                self._net_run(n_net)
                lat_current = False
                self.stats["net_blocks"] += n_net
            b += n_net
            # judged block: the lattice update and the network from one state
            if not lat_current:
                self.lat.reinit_fields(self.s, shift=True, sync_free=True)
            self.lat.step(self.K)
            self.lat.fields(0, out="f32", into=self.s_lbm)
            self.net.advance(self.s, self.sc)
            sur_judge(self.s, self.s_lbm, self.sc, self.part, self.judge_out, st)
            with self._torch.cuda.stream(st):
                self.red_host.copy_(self.red, non_blocking=True)
            self.stats["judged"] += 1
            self.stats["lbm_blocks"] += 1
            b += 1
            st.synchronize()
            j = self.red_host[:8].numpy()
            err = [math.sqrt(j[2 * c] / j[2 * c + 1]) if j[2 * c + 1] > 0 else math.sqrt(j[2 * c]) for c in range(4)]
            self.stats["judge_errors"].append(err)
            drift = 0.0
            if n_net:
                vols = self.red_host[8:8 + n_net].numpy()
                drift = float(np.max(np.abs(vols - self.vol0)) / self.vol0)
            trig = max(err[c] for c in self.TRIGGER)
            trig_u = max(err[c] for c in self.TRIGGER_U)
            self.stats["max_judge"] = max(self.stats["max_judge"], trig)
            self.stats["max_judge_u"] = max(self.stats["max_judge_u"], trig_u)
            self.stats["max_drift"] = max(self.stats["max_drift"], drift)
            if not (trig <= self.tol_check and trig_u <= self.tol_check_u and drift <= self.tol_vol):  # NaN fails
                self.stats["fallbacks"] += 1
                fallback_left = self.fallback_blocks
                self.s, self.s_lbm = self.s_lbm, self.s
                lat_current = True
            else:
                lat_current = False
        self.lat_current, self.fallback_left = lat_current, fallback_left
        self.stats["blocks"] += blocks
        st.synchronize()
        return self.stats


def rel_err(a: dict, b: dict, cfg: dict) -> dict:
    """Relative L2 error of fields a against b, each on the deviation of b
    from rest (phi = 1, u = 0, T = conduction profile)."""
    import torch
    gradT = float(cfg["meta"]["gradT"])
    ny = b["phi"].shape[0]
    y = torch.arange(ny, dtype=torch.float64, device=b["phi"].device).unsqueeze(1)
    rest = {"phi": 1.0, "ux": 0.0, "uy": 0.0, "T": gradT * (y + 0.5)}
    out = {}
    for k in ("phi", "ux", "uy", "T"):
        bb = b[k].double()
        d = (a[k].double() - bb).norm().item()
        r = (bb - rest[k]).norm().item()
        out[k] = d / r if r > 0 else d
    return out


def evaluate(net: Surrogate, items, warm: int, blocks: int, K: int = 100, check_every: int = 10,
             tol_check: float = 0.01, chunk: int = 10, device="cuda:0", log=print) -> list[dict]:
    """For each lattice: warm it up with the lattice update, then advance it
    `blocks` blocks of K steps, in chunks of `chunk` blocks, (a) by the plain
    FP32 lattice update (the reference), (b) by the hybrid, (c) by the network
    alone and (d) not at all (persistence).  Reports the errors of (b)-(d)
    against (a) after every chunk and the times of (a) and (b) per chunk (each
    chunk bracketed by device synchronisations; the field extractions between
    chunks are outside the timings)."""
    import torch
    if blocks % chunk:
        raise ValueError("blocks must be a multiple of chunk")
    out = []
    for cfg, f0 in items:
        ref = _lbm.Lattice(cfg, f0, _lbm.FP32_DEV, device=device)
        ref.set_graph_steps(K)
        ref.step(warm)
        snap = ref.get_state(0)
        start = {k: v.clone() for k, v in ref.fields(0, out="f32", to_host=False).items()}
        ref.step(K)                      # graph capture outside the timed region
        ref.set_state(0, **snap)
        traj, t_ref = [], []
        for c in range(blocks // chunk):
            ref.synchronize()
            t0 = time.perf_counter()
            ref.step(chunk * K)
            ref.synchronize()
            t_ref.append(time.perf_counter() - t0)
            traj.append({k: v.clone() for k, v in ref.fields(0, out="f32", to_host=False).items()})

        hyb = _lbm.Lattice(cfg, f0, _lbm.FP32_DEV, device=device)
        hyb.set_graph_steps(K)
        hyb.step(K)                      # graph capture outside the timed region
        hyb.set_state(0, **snap)
        net.stream = hyb.stream
        h = Hybrid(net, hyb, cfg, K=K, check_every=check_every, tol_check=tol_check)
        warm_s = {k: v.clone() for k, v in h.s.items()}
        torch.cuda.synchronize(hyb.device)
        net.advance(warm_s, h.sc)        # first-call costs outside the timing
        hyb.synchronize()
        t_hyb, e_h = [], []
        for c in range(blocks // chunk):
            t0 = time.perf_counter()
            h.run(chunk)
            t_hyb.append(time.perf_counter() - t0)
            e_h.append(rel_err(h.s, traj[c], cfg))
        stats = h.stats

        s = {k: v.clone() for k, v in start.items()}
        torch.cuda.synchronize(hyb.device)
        e_n, e_i = [], []
        for c in range(blocks // chunk):
            for _ in range(chunk):
                net.advance(s, h.sc)
            net.stream.synchronize()
            e_n.append(rel_err(s, traj[c], cfg))
            e_i.append(rel_err(start, traj[c], cfg))
        r = dict(Ma=cfg["meta"]["Ma"], lambda_r=cfg["meta"]["lambda_r"], R=cfg["meta"]["R"], chunk=chunk,
                 t_ref_ms=[1e3 * t for t in t_ref], t_hybrid_ms=[1e3 * t for t in t_hyb],
                 err_hybrid=e_h, err_net_only=e_n, err_persistence=e_i,
                 **{k: v for k, v in stats.items() if k != "judge_errors"})
        if log:
            for c in range(blocks // chunk):
                n = (c + 1) * chunk
                sp = sum(t_ref[:c + 1]) / sum(t_hyb[:c + 1])
                log(f"[eval] Ma={r['Ma']:.2f} lr={r['lambda_r']:.2f} R={r['R']:.1f} blocks {n}: speedup {sp:.2f} "
                    f"hybrid {max(e_h[c].values()):.4f} net-only {max(e_n[c].values()):.4f} "
                    f"persistence {max(e_i[c].values()):.4f}")
            log(f"[eval]   fallbacks {stats['fallbacks']} judged {stats['judged']} max judge {stats['max_judge']:.4f} "
                f"(u {stats['max_judge_u']:.4f}) drift {stats['max_drift']:.2e}")
        out.append(r)
        ref.close()
        hyb.close()
    return out
