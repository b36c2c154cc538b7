"""Host-side error behaviour of the lattice C ABI (include/lbm.h) that needs no
GPU: every entry point that takes a context rejects a NULL one with
LBM_EINVAL and a message; the NULL-safe queries return their documented
values; lbm_init and lbm_init_batch reject bad workspaces and arguments before
touching the device; the copy probe rejects bad sizes and alignment; the
per-update byte counts are the algorithmic 58 words per node.  Device
addresses passed are placeholders that every case rejects before use (the
module is skipped where a GPU device node exists)."""
import ctypes as C
import os

import numpy as np
import pytest

from paper_2306_11320_amd import workloads as wl

lbm = pytest.importorskip("paper_2306_11320_amd.lbm")

pytestmark = pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="placeholder addresses: host-only test")

EINVAL, ENOSPACE = -1, -2
WS = C.c_void_p(0x10000000)      # 256-byte aligned placeholder


def _lib():
    try:
        return lbm.lib()
    except RuntimeError as e:
        pytest.fail(str(e))


def _err(rc, code, words):
    msg = _lib().lbm_last_error().decode()
    assert rc == code, (rc, msg)
    assert words in msg, msg


def test_null_context_rejected():
    L = _lib()
    d = lbm.Diag()
    buf = (C.c_char * 16)()
    dp = C.POINTER(C.c_double)()
    step = C.c_int64(0)
    ti, tg, tm = C.c_int(0), C.c_int(0), C.c_float(0)
    calls = [
        lambda: L.lbm_step(None, 1),
        lambda: L.lbm_fields(None, WS, WS, WS, WS, None, 0),
        lambda: L.lbm_fields_instance(None, 0, WS, WS, WS, WS, None, 0),
        lambda: L.lbm_diagnostics(None, C.byref(d)),
        lambda: L.lbm_diagnostics_instance(None, 0, C.byref(d)),
        lambda: L.lbm_reinit_fields(None, 0, WS, WS, WS, WS, None, 0, 0),
        lambda: L.lbm_get_state(None, 0, dp, dp, dp, dp, C.byref(step)),
        lambda: L.lbm_set_state(None, 0, dp, dp, dp, dp, 0),
        lambda: L.lbm_set_tile(None, 0),
        lambda: L.lbm_set_graph_steps(None, 2),
        lambda: L.lbm_set_grid(None, 1),
        lambda: L.lbm_autotune(None, 4, C.byref(ti), C.byref(tg), C.byref(tm)),
    ]
    for call in calls:
        _err(call(), EINVAL, "context is NULL")
    for call in (lambda: L.lbm_checkpoint_save(None, buf, 16), lambda: L.lbm_checkpoint_load(None, buf, 16)):
        _err(call(), EINVAL, "NULL argument")


def test_null_safe_queries():
    L = _lib()
    assert L.lbm_destroy(None) == 0
    assert L.lbm_instances(None) == 0
    assert L.lbm_get_tile(None) == -1
    assert L.lbm_get_grid(None) == -1
    assert L.lbm_checkpoint_bytes(None) == 0


def test_tile_shapes_and_bytes_per_update():
    L = _lib()
    n = L.lbm_tile_count()
    assert n == len(lbm.tile_shapes())
    tx, ty = C.c_int(0), C.c_int(0)
    for bad in (-1, n):
        _err(L.lbm_tile_shape(bad, C.byref(tx), C.byref(ty)), EINVAL, "out of range")
    for t in range(n):
        assert L.lbm_tile_shape(t, C.byref(tx), C.byref(ty)) == 0
        assert tx.value > 0 and ty.value >= 0
    # 27 populations read and written plus (phi u) of the previous step read and written
    assert L.lbm_bytes_per_update(lbm.FP64) == 58 * 8
    assert L.lbm_bytes_per_update(lbm.FP32_DEV) == 58 * 4


@pytest.mark.parametrize("src,dst,nbytes,words", [
    (None, WS, 1024, "bad arguments"),
    (WS, WS, 0, "bad arguments"),
    (WS, WS, 1000, "bad arguments"),
    (C.c_void_p(0x10000008), WS, 1024, "16-byte aligned"),
])
def test_copy_probe_rejects(src, dst, nbytes, words):
    _err(_lib().lbm_copy_probe(src, dst, nbytes, None), EINVAL, words)


def _init_args(prec=lbm.FP32_DEV):
    cfg, f0 = wl.tiny(40, 24, bc=wl.ALL_BCS[1], seed=1)
    p = lbm.make_params(cfg, prec)
    fields = [np.ascontiguousarray(f0[k], np.float64) for k in ("phi", "ux", "uy", "T")]
    return p, fields


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def test_init_rejects_before_the_device():
    L = _lib()
    p, fl = _init_args()
    need = L.lbm_workspace_bytes(C.byref(p))
    assert need > 0
    out = C.c_void_p()
    ptrs = [_dp(a) for a in fl]
    _err(L.lbm_init(C.byref(p), *ptrs, WS, need, None, None), EINVAL, "out is NULL")
    _err(L.lbm_init(C.byref(p), *ptrs, C.c_void_p(0x10000080), need, None, C.byref(out)), EINVAL, "256-byte aligned")
    _err(L.lbm_init(C.byref(p), ptrs[0], None, ptrs[2], ptrs[3], WS, need, None, C.byref(out)), EINVAL, "NULL")
    _err(L.lbm_init(C.byref(p), *ptrs, None, need, None, C.byref(out)), EINVAL, "NULL")
    _err(L.lbm_init(C.byref(p), *ptrs, WS, need - 1, None, C.byref(out)), ENOSPACE, "needed")
    assert out.value is None


def test_init_batch_rejects_before_the_device():
    L = _lib()
    p32, fl = _init_args(lbm.FP32_DEV)
    p64, _ = _init_args(lbm.FP64)
    out = C.c_void_p()
    P2 = lbm.Params * 2
    PP = C.POINTER(C.c_double) * 2
    f = [PP(_dp(a), _dp(a)) for a in fl]
    _err(L.lbm_init_batch(0, P2(p32, p32), *f, WS, 1 << 30, None, C.byref(out)), EINVAL, "n < 1")
    _err(L.lbm_init_batch(2, P2(p32, p64), *f, WS, 1 << 30, None, C.byref(out)), EINVAL, "precision differs")
    fnull = [PP(_dp(a), None) if i == 3 else PP(_dp(a), _dp(a)) for i, a in enumerate(fl)]
    _err(L.lbm_init_batch(2, P2(p32, p32), *fnull, WS, 1 << 30, None, C.byref(out)), EINVAL, "lattice 1: NULL field")
    need = L.lbm_workspace_bytes_batch(P2(p32, p32), 2)
    assert need > 0
    _err(L.lbm_init_batch(2, P2(p32, p32), *f, WS, need - 1, None, C.byref(out)), ENOSPACE, "needed")
    assert out.value is None
