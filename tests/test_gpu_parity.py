"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

FP64 tolerances: one step on small lattices, max |difference| <= 2e-13 times
the largest magnitude of the population family (f, g, h) -- a few hundred
roundings of FMA-contracted versus plain arithmetic; after many steps, relative
L2 <= 1e-10 per macroscopic field.  Launch-shape changes (tile shape, graph
capture, batching) must leave results bitwise identical.
"""
import numpy as np
import pytest

import oracle
from paper_2306_11320_amd import workloads as wl
from tests.conftest import announce

pytestmark = pytest.mark.gpu

lbm = pytest.importorskip("paper_2306_11320_amd.lbm")

ONE_STEP_TOL = 2e-13
MULTI_STEP_TOL = 1e-10


def perturbed_state(cfg, f0, seed):
    """Equilibrium state of the oracle plus random non-equilibrium parts."""
    o = oracle.Oracle(cfg, f0)
    st = o.get_state()
    d = wl.perturbation(cfg["nx"], cfg["ny"], seed=seed)
    st = {k: st[k] + d[k] for k in ("f", "g", "h", "jprev")}
    o.set_state(**st, step=0)
    return o, st


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.sqrt(np.sum(b * b))
    return float(np.sqrt(np.sum((a - b) ** 2)) / (den if den > 0 else 1.0))


def compare_pops(gpu_st, orc_st, tol):
    for fam in ("f", "g", "h", "jprev"):
        ref = orc_st[fam]
        scale = max(np.abs(ref).max(), 1e-300)
        err = np.abs(gpu_st[fam] - ref).max() / scale
        assert err <= tol, f"{fam}: max rel diff {err:.3e} > {tol:.1e}"


@pytest.mark.parametrize("bcs", wl.ALL_BCS, ids=lambda b: "bc" + "".join(map(str, b)))
@pytest.mark.parametrize("shape", [(70, 13), (5, 4), (133, 41)], ids=lambda s: f"{s[0]}x{s[1]}")
@pytest.mark.parametrize("grad_mode", [0, 1])
def test_one_step_fp64(bcs, shape, grad_mode):
    nx, ny = shape
    cfg, f0 = wl.tiny(nx, ny, bc=bcs, seed=nx + ny)
    cfg["grad_mode"] = grad_mode
    announce("one_step_fp64", bcs, shape, grad_mode)
    o, st = perturbed_state(cfg, f0, seed=7)
    lat = lbm.Lattice(cfg, f0, lbm.FP64)
    lat.set_state(0, **st, step=0)
    o.step(1)
    lat.step(1)
    compare_pops(lat.get_state(), o.get_state(), ONE_STEP_TOL)


def test_full_size_one_step_fp64():
    """One step at the droplet workload's full size (256 x 1024) from a
    perturbed equilibrium, every population compared."""
    cfg, f0 = wl.droplet(Ma=1.0, ratio=0.5)
    announce("full_size_one_step", cfg["nx"], cfg["ny"])
    o, st = perturbed_state(cfg, f0, seed=3)
    lat = lbm.Lattice(cfg, f0, lbm.FP64)
    lat.set_state(0, **st, step=0)
    o.step(1)
    lat.step(1)
    compare_pops(lat.get_state(), o.get_state(), ONE_STEP_TOL)


@pytest.mark.parametrize("bcs", [wl.ALL_BCS[1], wl.ALL_BCS[4]], ids=["channel", "inlet"])
def test_multistep_fp64(bcs):
    cfg, f0 = wl.tiny(96, 72, bc=bcs, seed=5)
    announce("multistep_fp64", bcs)
    o = oracle.Oracle(cfg, f0)
    lat = lbm.Lattice(cfg, f0, lbm.FP64)
    for _ in range(3):
        o.step(100)
        lat.step(100)
        ref, got = o.fields(), lat.fields()
        for k in ("phi", "ux", "uy", "T", "p"):
            e = rel_l2(got[k], ref[k])
            assert e <= MULTI_STEP_TOL, f"{k}: rel L2 {e:.3e}"


def test_diagnostics_fp64():
    cfg, f0 = wl.tiny(80, 60, seed=11)
    announce("diagnostics_fp64")
    o = oracle.Oracle(cfg, f0)
    lat = lbm.Lattice(cfg, f0, lbm.FP64)
    o.step(50)
    lat.step(50)
    a, b = lat.diagnostics(), o.diagnostics()
    for k in ("mass_phi", "vol_light", "heat", "sum_neg", "u_r", "ux_r", "xc", "yc", "max_u"):
        assert abs(a[k] - b[k]) <= 1e-10 * max(abs(b[k]), 1e-12), (k, a[k], b[k])
    assert a["n_neg"] == b["n_neg"] and a["n_nonfinite"] == 0
    for q in range(1):
        assert abs(a["bub_x"][q] - b["bub_x"][q]) < 1e-9 and abs(a["bub_uy"][q] - b["bub_uy"][q]) < 1e-12


def test_tile_shapes_bitwise():
    cfg, f0 = wl.tiny(150, 45, bc=wl.ALL_BCS[4], seed=2)
    announce("tile_shapes_bitwise")
    ref = None
    for t in range(len(lbm.tile_shapes())):
        lat = lbm.Lattice(cfg, f0, lbm.FP64)
        lat.set_tile(t)
        lat.step(21)
        st = lat.get_state()
        if ref is None:
            ref = st
        else:
            for k in ("f", "g", "h", "jprev"):
                assert np.array_equal(st[k], ref[k]), f"tile {t}: {k} differs"


@pytest.mark.parametrize("prec", ["FP64", "FP32_DEV"])
@pytest.mark.parametrize("bcs,ny", [(wl.ALL_BCS[1], 40), (wl.ALL_BCS[0], 42)])
def test_tile_shapes_bitwise_periodic_x(prec, bcs, ny):
    """Interior tiles (periodic wrap at both ends of a tile row) give bitwise
    the same state for every tile shape.  nx = 320: whole tiles and tiles cut
    by the lattice's end in x (interior when x is periodic); with ny = 42 and
    y periodic, also tiles cut in y."""
    cfg, f0 = wl.tiny(320, ny, bc=bcs, seed=6)
    announce("tile_shapes_bitwise_periodic_x", prec, bcs, ny)
    ref = None
    for t in range(len(lbm.tile_shapes())):
        lat = lbm.Lattice(cfg, f0, getattr(lbm, prec))
        lat.set_tile(t)
        lat.step(21)
        st = lat.get_state()
        lat.close()
        if ref is None:
            ref = st
        else:
            for k in ("f", "g", "h", "jprev"):
                assert np.array_equal(st[k], ref[k]), f"tile {t}: {k} differs"


def test_graph_capture_bitwise():
    cfg, f0 = wl.tiny(64, 40, seed=4)
    announce("graph_capture_bitwise")
    a = lbm.Lattice(cfg, f0, lbm.FP64)
    a.set_graph_steps(0)
    b = lbm.Lattice(cfg, f0, lbm.FP64)
    b.set_graph_steps(16)
    for n in (3, 40, 17):
        a.step(n)
        b.step(n)
    sa, sb = a.get_state(), b.get_state()
    for k in ("f", "g", "h", "jprev"):
        assert np.array_equal(sa[k], sb[k]), k
    assert sa["step"] == sb["step"] == 60


def test_heated_channel_fp64_full():
    """Heated microchannel, 64 x 32, 20000 steps, both conductivity ratios."""
    for lr in (1.0, 2.0):
        cfg, f0 = wl.heated_channel(lr)
        announce("heated_channel_fp64", lr)
        o = oracle.Oracle(cfg, f0)
        lat = lbm.Lattice(cfg, f0, lbm.FP64)
        o.step(20000)
        lat.step(20000)
        ref, got = o.fields(), lat.fields()
        for k in ("phi", "ux", "uy", "T", "p"):
            e = rel_l2(got[k], ref[k])
            assert e <= MULTI_STEP_TOL, f"lambda_r={lr} {k}: rel L2 {e:.3e}"


def test_checkpoint_resume_bitwise():
    cfg, f0 = wl.tiny(70, 50, seed=9)
    announce("checkpoint_resume")
    a = lbm.Lattice(cfg, f0, lbm.FP64)
    a.step(31)
    ck = a.checkpoint()
    a.step(40)
    b = lbm.Lattice(cfg, f0, lbm.FP64)
    b.restore(ck)
    b.step(40)
    sa, sb = a.get_state(), b.get_state()
    for k in ("f", "g", "h", "jprev"):
        assert np.array_equal(sa[k], sb[k]), k
    assert sb["step"] == 71
    # a checkpoint of another storage layout (format tag) or other parameters is refused
    bad = bytearray(ck)
    bad[7] ^= 1
    with pytest.raises(lbm.LbmError):
        b.restore(bytes(bad))
    other = dict(cfg, mobility=cfg["mobility"] * 1.5)
    c = lbm.Lattice(other, f0, lbm.FP64)
    with pytest.raises(lbm.LbmError):
        c.restore(ck)


# ---- two-relaxation-time collision -------------------------------------------

@pytest.mark.parametrize("bcs", [wl.ALL_BCS[0], wl.ALL_BCS[1], wl.ALL_BCS[4]], ids=["periodic", "channel", "inlet"])
@pytest.mark.parametrize("magic", [3.0 / 16.0, 0.25])
def test_one_step_trt_fp64(bcs, magic):
    cfg, f0 = wl.tiny(70, 13, bc=bcs, seed=17)
    cfg.update(collision=1, trt_magic=magic)
    announce("one_step_trt", bcs, magic)
    o, st = perturbed_state(cfg, f0, seed=8)
    lat = lbm.Lattice(cfg, f0, lbm.FP64)
    lat.set_state(0, **st, step=0)
    o.step(1)
    lat.step(1)
    compare_pops(lat.get_state(), o.get_state(), ONE_STEP_TOL)


def test_multistep_trt_fp64():
    cfg, f0 = wl.tiny(96, 72, bc=wl.ALL_BCS[1], seed=6)
    cfg.update(collision=1)
    announce("multistep_trt")
    o = oracle.Oracle(cfg, f0)
    lat = lbm.Lattice(cfg, f0, lbm.FP64)
    o.step(300)
    lat.step(300)
    ref, got = o.fields(), lat.fields()
    for k in ("phi", "ux", "uy", "T", "p"):
        e = rel_l2(got[k], ref[k])
        assert e <= MULTI_STEP_TOL, f"{k}: rel L2 {e:.3e}"


@pytest.mark.parametrize("prec,tol", [(lbm.FP64, 1e-12), (lbm.FP32_DEV, 1e-4)], ids=["fp64", "fp32dev"])
def test_trt_poiseuille_exact(prec, tol):
    """The GPU reproduces the exactness of the two-relaxation-time collision
    (magic 3/16) for plane Poiseuille flow that pins the oracle."""
    ny, mu, G = 32, 0.5, 1e-6
    cfg, f0 = wl.body_force_channel(ny, mu, G, collision=1, nx=64)
    announce("trt_poiseuille", prec)
    lat = lbm.Lattice(cfg, f0, prec)
    lat.step(40000)
    ux = lat.fields()["ux"]
    y = np.arange(ny)
    exact = G / (2 * mu) * (y + 0.5) * (ny - 0.5 - y)
    assert np.abs(ux - exact[:, None]).max() <= tol * exact.max()


def test_full_size_bubbles_one_step_fp64():
    """One step at the two-bubble workload's full size (512 x 2048, walls in x,
    inflow and outflow in y, parabolic sigma(T), density ratio 10) from a
    perturbed equilibrium, every population compared."""
    cfg, f0 = wl.two_bubbles(sigma_TT=0.2)
    announce("full_size_bubbles_one_step", cfg["nx"], cfg["ny"])
    o, st = perturbed_state(cfg, f0, seed=4)
    lat = lbm.Lattice(cfg, f0, lbm.FP64)
    lat.set_state(0, **st, step=0)
    o.step(1)
    lat.step(1)
    compare_pops(lat.get_state(), o.get_state(), ONE_STEP_TOL)
