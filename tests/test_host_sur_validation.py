"""Host-side argument checks of the surrogate's C ABI (include/surrogate.h):
every rejected call returns -1 before any launch and sur_last_error names the
cause.  The device addresses passed are placeholders that no kernel may
touch; each case is rejected by a check on sizes, alignment, NULL entries or
scales, so no GPU is used (the module is skipped where a GPU device node
exists, so that a check that wrongly passed could not launch on them)."""
import ctypes as C
import os
import re

import pytest

sur = pytest.importorskip("paper_2306_11320_amd.surrogate")

pytestmark = pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="placeholder addresses: host-only test")

A = C.c_void_p(0x100000)         # 16-byte aligned placeholder
MIS = C.c_void_p(0x100008)       # 8-byte aligned placeholder


def _lib():
    try:
        return sur.lib()
    except RuntimeError as e:
        pytest.fail(str(e))


def _scales(**over):
    s = sur.SurScales(u=1e-3, dT=1.0, t_a=0.0, t_b=0.0, P=1e-3, c4=0.0, c5=0.0)
    for c in range(5):
        s.inc[c] = 1e-3
    for k, v in over.items():
        if k == "inc0":
            s.inc[0] = v
        else:
            setattr(s, k, v)
    return s


def _state(null_at=None):
    vals = [0x200000 + 0x1000 * c for c in range(5)]
    if null_at is not None:
        vals[null_at] = 0
    return (C.c_void_p * 5)(*vals)


def _rejects(rc, words):
    msg = _lib().sur_last_error().decode()
    assert rc == -1, (rc, msg)
    assert words in msg, msg


@pytest.mark.parametrize("args,words", [
    (dict(d_in=None), "NULL tensor"),
    (dict(cin=16), "cin must be 8 or 32"),
    (dict(n=0), "need n, h, w >= 1"),
    (dict(w=0), "need n, h, w >= 1"),
    (dict(dil=0), "1 <= dil <= w"),
    (dict(dil=65, w=64), "1 <= dil <= w"),
    (dict(n=1, h=1 << 30, w=32), "2^30 segments"),
    (dict(n=4, h=1 << 23, w=1024), "2^30 segments"),
    (dict(d_in=MIS), "16-byte aligned"),
    (dict(d_res=MIS), "16-byte aligned"),
    (dict(d_out=MIS), "16-byte aligned"),
])
def test_conv3x3_rejects(args, words):
    a = dict(d_in=A, cin=32, d_w=A, d_bias=None, d_res=None, d_mask=None, d_out=A, out_f32=0, relu_in=1, dil=1, n=1,
             h=8, w=64)
    a.update(args)
    rc = _lib().sur_conv3x3(a["d_in"], a["cin"], a["d_w"], a["d_bias"], a["d_res"], a["d_mask"], a["d_out"],
                            a["out_f32"], a["relu_in"], a["dil"], a["n"], a["h"], a["w"], None)
    _rejects(rc, words)


@pytest.mark.parametrize("args,words", [
    (dict(state=_state(2)), "bad arguments"),
    (dict(scales=_scales(u=0.0)), "bad arguments"),
    (dict(scales=_scales(inc0=-1.0)), "bad arguments"),
    (dict(h=0), "need h, w >= 1"),
    (dict(dil=33, w=32), "1 <= dil <= w"),
    (dict(h=1 << 30, w=32), "2^30 segments"),
    (dict(d_in=MIS), "16-byte aligned"),
])
def test_conv3x3_advance_rejects(args, words):
    a = dict(d_in=A, d_w=A, dil=1, h=8, w=64, scales=_scales(), state=_state())
    a.update(args)
    sc = a["scales"]
    rc = _lib().sur_conv3x3_advance(a["d_in"], a["d_w"], None, 1, a["dil"], a["h"], a["w"], C.byref(sc), a["state"],
                                    None)
    _rejects(rc, words)


@pytest.mark.parametrize("args,words", [
    (dict(part=None), "bad arguments"),
    (dict(vol=None), "bad arguments"),
    (dict(dil=17, w=64), "1 <= dil <= min(w, 16)"),
    (dict(part=C.c_void_p(0x100004)), "8-byte aligned"),
])
def test_conv3x3_advance_volume_rejects(args, words):
    a = dict(d_in=A, d_w=A, dil=1, h=8, w=64, part=A, vol=A)
    a.update(args)
    sc = _scales()
    rc = _lib().sur_conv3x3_advance_volume(a["d_in"], a["d_w"], None, 1, a["dil"], a["h"], a["w"], C.byref(sc),
                                           _state(), a["part"], a["vol"], None)
    _rejects(rc, words)


def judge_max_groups():
    """SUR_JUDGE_MAX_GROUPS as the header defines it."""
    hdr = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "surrogate.h")
    return int(re.search(r"#define\s+SUR_JUDGE_MAX_GROUPS\s+(\d+)", open(hdr).read()).group(1))


def test_judge_noscratch_group_limit():
    L = _lib()
    sc = _scales()
    gmax = judge_max_groups()
    for groups in (0, gmax + 1):
        rc = L.sur_judge_noscratch(_state(), _state(), 8, 64, C.byref(sc), groups, A, None)
        _rejects(rc, f"groups {groups} outside [1, {gmax}]")


def test_other_entry_points_reject():
    L = _lib()
    sc = _scales()
    _rejects(L.sur_adjoint_weights(A, 16, A, None), "cin must be 8 or 32")
    _rejects(L.sur_weight_grad(A, A, 32, 1, 1, 1, 8, 64, A, 0, A, None), "bad sizes")
    _rejects(L.sur_weight_grad(A, A, 32, 1, 65, 1, 8, 64, A, 4, A, None), "1 <= dil <= w")
    _rejects(L.sur_bias_grad(A, 0, A, 4, A, None), "bad arguments")
    _rejects(L.sur_adam(A, A, A, A, A, 10, 1e-3, 0.9, 0.999, 1e-8, 0, None), "bad arguments")
    _rejects(L.sur_mse(A, A, 100, 33, 1.0, A, A, 4, None), "bad arguments")
    _rejects(L.sur_pack(_state(0), 8, 64, C.byref(sc), A, None), "bad arguments")
    _rejects(L.sur_pack(_state(), 8, 64, C.byref(_scales(dT=0.0)), A, None), "bad arguments")
    _rejects(L.sur_pack_target(_state(), _state(4), 512, C.byref(sc), A, None), "bad arguments")
    _rejects(L.sur_advance(A, 0, C.byref(sc), _state(), None), "bad arguments")
    _rejects(L.sur_light_volume(A, 8, 64, A, 0, A, None), "bad arguments")
    _rejects(L.sur_judge(_state(), _state(), 8, 64, C.byref(_scales(P=-1.0)), A, 4, A, None), "bad arguments")
