"""The allocation-free judge (sur_judge_noscratch, include/surrogate.h) against
sur_judge, whose partial sums live in a caller-allocated buffer: the same
kernels in the same order, so the sums must agree bitwise.  Two calls in a
row, the second on a smaller frame with fewer partials (the static scratch
keeps the first call's partials, none of which the second may read), and both
against FP64 sums computed on the host.  The group limit is rejected on the
host before any GPU work."""
import ctypes as C

import numpy as np
import pytest

from tests.conftest import announce

sur = pytest.importorskip("paper_2306_11320_amd.surrogate")
torch = pytest.importorskip("torch")

FIELDS = ("phi", "ux", "uy", "T", "p")


def _scales():
    sc = sur.SurScales()
    sc.u, sc.dT, sc.P = 1e-3, 0.5, 2e-4
    sc.t_a, sc.t_b = 0.25, 0.01
    for c in range(5):
        sc.inc[c] = 1.0
    return sc


def _frames(h, w, seed, dev):
    rng = np.random.default_rng(seed)
    a = {k: rng.standard_normal((h, w)).astype(np.float32) for k in FIELDS}
    b = {k: (a[k] + 0.01 * rng.standard_normal((h, w))).astype(np.float32) for k in FIELDS}
    to = lambda d: {k: torch.tensor(v, device=dev) for k, v in d.items()}  # noqa: E731
    return a, b, to(a), to(b)


def _host_sums(a, b, sc, h, w):
    rest = [np.ones((h, w)), np.zeros((h, w)), np.zeros((h, w)),
            np.float64(sc.t_a) + np.float64(sc.t_b) * np.arange(h, dtype=np.float64)[:, None] * np.ones((1, w))]
    out = []
    for c, k in enumerate(FIELDS[:4]):
        av, bv = a[k].astype(np.float64), b[k].astype(np.float64)
        out += [np.sum((av - bv) ** 2), np.sum((bv - rest[c]) ** 2)]
    return np.array(out)


def test_rejects_groups_beyond_the_static_scratch():
    L = sur.lib()
    sc = _scales()
    z = (C.c_void_p * 5)(*([C.c_void_p(16)] * 5))
    for g in (0, 1025):
        rc = L.sur_judge_noscratch(z, z, 4, 32, C.byref(sc), g, C.c_void_p(16), None)
        assert rc == -1
        assert "groups" in L.sur_last_error().decode()


@pytest.mark.gpu
def test_noscratch_judge_equals_judge():
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    sc = _scales()
    for call, (h, w, groups) in enumerate(((160, 224, 1024), (40, 96, 37))):
        announce("noscratch_judge", call, h, w, groups)
        a, b, ad, bd = _frames(h, w, 7 + call, dev)
        part = torch.empty(8 * groups, dtype=torch.float64, device=dev)
        ref = torch.zeros(8, dtype=torch.float64, device=dev)
        out = torch.zeros(8, dtype=torch.float64, device=dev)
        stream.wait_stream(torch.cuda.current_stream(dev))
        sur.sur_judge(ad, bd, sc, part, ref, stream)
        sur.sur_judge_noscratch(ad, bd, sc, groups, out, stream)
        stream.synchronize()
        r, o = ref.cpu().numpy(), out.cpu().numpy()
        assert np.array_equal(o, r), (call, o, r)
        host = _host_sums(a, b, sc, h, w)
        assert np.allclose(o, host, rtol=1e-12, atol=0), (call, o, host)
