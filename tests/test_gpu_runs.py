"""Runs: the tile ids that step lattices periodic in x with 64 <= nx <= 256 in
runs of 512 or 256 consecutive nodes (x-fastest order), one workgroup per run.

The per-node arithmetic is that of the tiles, so the state after any number
of steps is bitwise the same as with the TX x TY tiles; checked from a
perturbed state (random non-equilibrium parts on every population) across
widths that put the periodic seam anywhere in a run (64 to 256, odd widths,
a last run cut by the lattice's end), boundary sets whose y sides are
periodic, walls or inlet/outlet, both precisions, both normal modes, two
relaxation times, and batches that mix run lattices with tile lattices.  One
step from the same perturbed state also matches the FP64 oracle at the
one-step tolerance of the tile path (2e-13 of the population family's
largest magnitude).
"""
import numpy as np
import pytest

import oracle
from paper_2306_11320_amd import workloads as wl
from tests.conftest import announce

pytestmark = pytest.mark.gpu

lbm = pytest.importorskip("paper_2306_11320_amd.lbm")

P, WT, WA, IN, OUT = wl.PERIODIC, wl.WALL_T, wl.WALL_ADIABATIC, wl.INLET, wl.OUTLET
Y_SIDES = [(P, P), (WT, WT), (WA, WT), (IN, OUT)]
WIDTHS = [(64, 9), (97, 23), (130, 40), (221, 31), (256, 12)]


def _run_ids():
    ids = [t for t, (_, ty) in enumerate(lbm.tile_shapes()) if ty == 0]
    assert sorted(lbm.tile_shapes()[t][0] for t in ids) == [256, 512]
    return ids


def _perturbed(cfg, f0, prec, seed):
    lat = lbm.Lattice(cfg, f0, prec)
    st = lat.get_state()
    lat.close()
    d = wl.perturbation(cfg["nx"], cfg["ny"], seed=seed)
    return {k: st[k] + d[k] for k in ("f", "g", "h", "jprev")}


def _after(cfg, f0, prec, tile, st, steps):
    lat = lbm.Lattice(cfg, f0, prec)
    lat.set_tile(tile)
    lat.set_state(0, **st, step=0)
    lat.step(steps)
    out = lat.get_state()
    lat.close()
    return out


def _same(a, b, what):
    for k in ("f", "g", "h", "jprev"):
        assert np.array_equal(a[k], b[k]), f"{what}: {k} differs"


@pytest.mark.parametrize("prec", ["FP64", "FP32_DEV"])
@pytest.mark.parametrize("ysides", Y_SIDES, ids=lambda s: "y" + "".join(map(str, s)))
@pytest.mark.parametrize("shape", WIDTHS, ids=lambda s: f"{s[0]}x{s[1]}")
def test_runs_bitwise_vs_tiles(prec, ysides, shape):
    nx, ny = shape
    cfg, f0 = wl.tiny(nx, ny, bc=(P, P) + ysides, seed=nx + ny)
    announce("runs_bitwise_vs_tiles", prec, ysides, shape)
    p = getattr(lbm, prec)
    st = _perturbed(cfg, f0, p, seed=nx)
    ref = _after(cfg, f0, p, 5, st, 13)
    for t in _run_ids():
        _same(_after(cfg, f0, p, t, st, 13), ref, f"{lbm.tile_name(t)} vs 128x4")
    _same(_after(cfg, f0, p, 0, st, 13), ref, "64x4 vs 128x4")


@pytest.mark.parametrize("variant", ["trt", "stencil_normal"])
def test_runs_bitwise_variants(variant):
    cfg, f0 = wl.tiny(221, 31, bc=wl.ALL_BCS[1], seed=3)
    if variant == "trt":
        cfg["collision"] = lbm.TRT
        cfg["trt_magic"] = 0.25
    else:
        cfg["grad_mode"] = 1
    announce("runs_bitwise_variants", variant)
    for prec in (lbm.FP64, lbm.FP32_DEV):
        st = _perturbed(cfg, f0, prec, seed=5)
        ref = _after(cfg, f0, prec, 5, st, 11)
        for t in _run_ids():
            _same(_after(cfg, f0, prec, t, st, 11), ref, f"{variant}, {lbm.tile_name(t)}")


@pytest.mark.parametrize("prec", ["FP64", "FP32_DEV"])
def test_runs_batched_mixed(prec):
    """A batch of run lattices (periodic x, 64 <= nx <= 256) and tile lattices
    (nx = 300; x walls) gives each lattice's single-lattice state bitwise."""
    items = [wl.tiny(97, 23, bc=wl.ALL_BCS[1], seed=1), wl.tiny(300, 20, bc=wl.ALL_BCS[0], seed=2),
             wl.tiny(80, 30, bc=wl.ALL_BCS[3], seed=3), wl.tiny(256, 11, bc=wl.ALL_BCS[2], seed=4),
             wl.tiny(64, 17, bc=wl.ALL_BCS[0], seed=5)]
    announce("runs_batched_mixed", prec)
    p = getattr(lbm, prec)
    refs = []
    for cfg, f0 in items:
        lat = lbm.Lattice(cfg, f0, p)
        lat.set_tile(5)
        lat.step(14)
        refs.append(lat.get_state())
        lat.close()
    for t in _run_ids():
        b = lbm.Lattice.batch(items, p)
        b.set_tile(t)
        b.step(14)
        for k in range(len(items)):
            _same(b.get_state(k), refs[k], f"{lbm.tile_name(t)}, lattice {k}")
        b.close()


@pytest.mark.parametrize("bcs", wl.ALL_BCS[:3], ids=lambda b: "bc" + "".join(map(str, b)))
@pytest.mark.parametrize("shape", [(97, 23), (256, 12)], ids=lambda s: f"{s[0]}x{s[1]}")
@pytest.mark.parametrize("grad_mode", [0, 1])
def test_runs_one_step_fp64_vs_oracle(bcs, shape, grad_mode):
    nx, ny = shape
    cfg, f0 = wl.tiny(nx, ny, bc=bcs, seed=nx + ny)
    cfg["grad_mode"] = grad_mode
    announce("runs_one_step_fp64", bcs, shape, grad_mode)
    o = oracle.Oracle(cfg, f0)
    st = o.get_state()
    d = wl.perturbation(nx, ny, seed=7)
    st = {k: st[k] + d[k] for k in ("f", "g", "h", "jprev")}
    o.set_state(**st, step=0)
    o.step(1)
    ref = o.get_state()
    for t in _run_ids():
        got = _after(cfg, f0, lbm.FP64, t, st, 1)
        for fam in ("f", "g", "h", "jprev"):
            scale = max(np.abs(ref[fam]).max(), 1e-300)
            err = np.abs(got[fam] - ref[fam]).max() / scale
            assert err <= 2e-13, f"{lbm.tile_name(t)}, {fam}: max rel diff {err:.3e}"


def test_autotune_skips_runs_without_run_lattices():
    """A context with no lattice that runs can step (walls in x; nx > 256)
    never times, and so never keeps, a run id; with a run lattice it may."""
    items = [wl.tiny(70, 90, bc=wl.ALL_BCS[4], seed=2), wl.tiny(300, 20, bc=wl.ALL_BCS[0], seed=3)]
    announce("autotune_skips_runs")
    for _ in range(2):
        b = lbm.Lattice.batch(items, lbm.FP32_DEV)
        res = b.autotune(steps_per_trial=2)
        assert res["tile"] not in _run_ids(), res
        b.close()
