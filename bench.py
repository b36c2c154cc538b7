"""Throughput of the fused lattice Boltzmann step on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload sweep|bubbles|droplet|channel]
                    [--precision fp32|fp64] [--only] [--no-cpu] [--surrogate N] [--potential]

A step is one time step of the three coupled D2Q9 LBEs over every node of the
workload (one fused kernel launch).  The headline workload is the largest
single-GPU configuration: 64 droplet-migration lattices of uneven size
(NX in 128..256, NY = 4 NX, 10.43 M nodes, 2.3 GB of populations) advanced
together by one persistent launch per step in FP32 deviation storage, tiles
chosen by the autotuner.  The same JSON line also carries:
* the batched launch against the same 64 lattices advanced one after another;
* the same 64 lattices in FP64 (4.7 GB);
* the two-bubble channel of Sec. 4.3 (512 x 2048) in FP64 (470 MB, streamed
  from HBM) and FP32 (235 MB, at the edge of the 256 MB Infinity Cache);
* the 256 x 1024 droplet (cache-resident: 59 MB FP32, 117 MB FP64);
* for each timed workload the error against the FP64 oracle after a 200-step
  window from the initial state (three lattices of the sweep);
* the learned surrogate (trained on 2000 trajectories of the batched-sweep
  generator) against the plain FP32 lattice update, on 256 x 1024 lattices
  and on the generator's uneven lattices, and its convolution against the
  BF16 dense peak;
* the oracle on the host cores, all cores and one thread.
Working-set bytes are reported next to every number.  --only times just the
named workload and precision, --conv-only just the surrogate's convolution
timings (profiling runs).  Every timed workload takes
the autotuner's tile (and, for batches, grid) choice.  Only one GPU is used;
--gpus above 1 is refused.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS (3 coupled D2Q9 LBEs) FP64 vs FP32; surrogate speedup at ≤1% L2 err"
HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SRC = os.path.join(ROOT, "paper_2306_11320_amd", "csrc", "lbm_kernels.hip")
WORKLOADS = {"sweep": "batched_droplet_sweep_64", "bubbles": "two_bubbles_512x2048",
             "droplet": "droplet_migration_256x1024", "channel": "heated_channel_64x32"}


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def stored_traffic(workload: str, prec: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(PROFILES, f"lbm_step_{workload}_{prec}_counters.txt")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", txt)
    t = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not m or not t or m.group(1) != kernel_hash():
        return None
    return float(t.group(1))


def make_workload(name: str):
    from paper_2306_11320_amd import workloads as wl
    if name == "droplet":
        cfg, f0 = wl.droplet(Ma=1.0, ratio=0.5)
        return [(cfg, f0)], dict(workload=WORKLOADS[name], nx=256, ny=1024, Ma=1.0, ratio=0.5)
    if name == "bubbles":
        cfg, f0 = wl.two_bubbles(sigma_TT=0.2)
        return [(cfg, f0)], dict(workload=WORKLOADS[name], nx=512, ny=2048, sigma_TT=0.2)
    if name == "channel":
        cfg, f0 = wl.heated_channel(2.0)
        return [(cfg, f0)], dict(workload=WORKLOADS[name], nx=64, ny=32, lambda_ratio=2.0)
    if name == "sweep":
        items = wl.sweep(64, seed=4)
        nodes = sum(c["nx"] * c["ny"] for c, _ in items)
        return items, dict(workload=WORKLOADS[name], instances=64, nodes=nodes, seed=4)
    raise SystemExit(f"unknown workload {name}")


def prewarm(seconds: float = 0.3):
    """Brings the GPU out of its idle clocks before anything is timed."""
    import torch
    x = torch.ones(1 << 24, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(20):
            x.mul_(1.0000001)
        torch.cuda.synchronize()


def time_gpu(items, prec, steps, warmup, tile=None, autotune=False, tune_cache=None):
    """Times `steps` steps after `warmup` untimed ones.  The events are
    recorded on the lattice's own stream, which every step kernel runs on, so
    their interval is the step kernels' time."""
    import torch
    from paper_2306_11320_amd import lbm
    if len(items) == 1:
        lat = lbm.Lattice(items[0][0], items[0][1], prec)
    else:
        lat = lbm.Lattice.batch(items, prec)
    tuned = None
    if tile is not None:
        lat.set_tile(tile)
    elif autotune:
        # single lattices step in ~10-120 us: 50 steps a trial keep launch noise out of the choice
        tuned = lat.autotune(steps_per_trial=50 if len(items) == 1 else max(2, min(50, warmup // 20 or 2)),
                             cache=tune_cache)
    lat.step(warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(lat.stream)
    t0 = time.perf_counter()
    lat.step(steps)
    ev1.record(lat.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    d = lat.diagnostics()
    nodes = sum(c["nx"] * c["ny"] for c, _ in items)
    tile_used = lbm.tile_name(lat.tile())
    lat.close()
    return dict(ms_total=ms, wall_s=wall, ms_per_step=ms / steps, nodes=nodes, tuned=tuned, tile=tile_used,
                mlups=nodes * steps / (ms * 1e-3) / 1e6, finite=d["n_nonfinite"] == 0, max_u=d["max_u"])


def lbm_leg(name, prec_name, steps, warmup, tile=None, potential=False, tune_cache=None):
    """MLUPS and the roofline of the step kernel for one workload and precision."""
    from paper_2306_11320_amd import lbm
    items, desc = make_workload(name)
    if potential:
        for cfg, _ in items:
            cfg["force_form"] = lbm.FORCE_POTENTIAL
        desc["force_form"] = "potential"
    prec = lbm.FP32_DEV if prec_name == "fp32" else lbm.FP64
    log(f"{desc['workload']}: {prec_name}, {steps} steps")
    r = time_gpu(items, prec, steps, warmup, tile, autotune=tile is None, tune_cache=tune_cache)
    if not r["finite"]:
        raise SystemExit(f"{desc['workload']} {prec_name}: non-finite state after the timed steps")
    word = 4 if prec_name == "fp32" else 8
    per_launch = lbm.bytes_per_update(prec) * r["nodes"]
    achieved = per_launch / (r["ms_per_step"] * 1e-3) / 1e9
    out = {"workload": desc["workload"], "value": round(r["mlups"], 1), "unit": "MLUPS",
           "ms_per_step": round(r["ms_per_step"], 5), "precision": "fp32_deviation" if word == 4 else "fp64",
           "tile": r["tile"], "nodes": r["nodes"], "working_set_bytes": (2 * 27 + 2) * word * r["nodes"],
           "algorithmic_bytes_per_launch": per_launch,
           "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4),
                        "traffic": None if potential else stored_traffic(name, prec_name)}}
    if r["tuned"] is not None:
        out["autotuned"] = r["tuned"]
    return out, items, desc


def time_sequential(items, prec, steps, warmup):
    """The lattices of a batch advanced one after another, each by the
    single-lattice kernel (one launch per step) with the autotuner's choice
    for that lattice: the baseline of batching."""
    import torch
    from paper_2306_11320_amd import lbm
    total_ms = 0.0
    for cfg, f0 in items:
        lat = lbm.Lattice(cfg, f0, prec)
        lat.autotune(steps_per_trial=50)
        lat.step(warmup)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(lat.stream)
        lat.step(steps)
        e1.record(lat.stream)
        torch.cuda.synchronize()
        total_ms += e0.elapsed_time(e1)
        lat.close()
    return total_ms / steps


def _field_errors(got: dict, ref: dict, T0: float) -> dict:
    """Relative L2 of phi and of T - T0, and the rms error of u over max |u|."""
    import numpy as np
    out = {}
    for k in ("phi", "T"):
        a, b = got[k], ref[k]
        if k == "T":
            a, b = a - T0, b - T0
        out[k] = float(np.sqrt(np.sum((a - b) ** 2) / max(np.sum(b ** 2), 1e-300)))
    umax = max(float(np.abs(ref["ux"]).max()), float(np.abs(ref["uy"]).max()), 1e-300)
    for k in ("ux", "uy"):
        out[k] = float(np.sqrt(np.mean((got[k] - ref[k]) ** 2)) / umax)
    return out


def oracle_error(name: str, prec_name: str, steps: int = 200, lattices=(0, 1, 2), tile=None):
    """The GPU path against the FP64 oracle on the timed workload: both take
    `steps` steps from the initial state (for the sweep, lattices `lattices`
    of the batch, stepped inside the batch), then the fields are compared.
    `tile`: the tile id the timed run used (else the default)."""
    import oracle
    from paper_2306_11320_amd import lbm
    items, _ = make_workload(name)
    prec = lbm.FP32_DEV if prec_name == "fp32" else lbm.FP64
    if len(items) > 1:
        lat = lbm.Lattice.batch(items, prec)
        which = list(lattices)
    else:
        lat = lbm.Lattice(items[0][0], items[0][1], prec)
        which = [0]
    if tile is not None:
        lat.set_tile(tile)
    lat.step(steps)
    worst = {}
    for k in which:
        cfg, f0 = items[k]
        o = oracle.Oracle(cfg, f0)
        o.step(steps)
        e = _field_errors(lat.fields(k), o.fields(), float(cfg.get("T_ref", 0.0)))
        worst = {q: max(worst.get(q, 0.0), v) for q, v in e.items()}
    lat_tile = lat.tile()
    lat.close()
    return {"steps": steps, "lattices": which if len(items) > 1 else None, "tile": lbm.tile_name(lat_tile),
            "rel_l2": {k: float(f"{v:.3e}") for k, v in worst.items()}}


def cpu_baseline(items, budget_s: float = 12.0):
    """The FP64 oracle as it stands, on the first lattice of the workload from
    its initial state: steps are added until about budget_s of CPU work, once
    on every host core (OpenMP) and once on one thread."""
    import oracle
    cfg, f0 = items[0]
    nodes = cfg["nx"] * cfg["ny"]

    def run(threads):
        o = oracle.Oracle(cfg, f0, threads=threads)
        used = oracle.Oracle.threads()
        t0 = time.perf_counter()
        o.step(2)
        dt = time.perf_counter() - t0
        n = max(2, int(budget_s / max(dt / 2, 1e-6)))
        t0 = time.perf_counter()
        o.step(n)
        dt = time.perf_counter() - t0
        return nodes * n / dt / 1e6, used, n, dt

    # OpenMP's default thread count (OMP_NUM_THREADS where set): the host
    # cores this process may use
    all_cores = oracle.Oracle.threads()
    va, ca, na, da = run(all_cores)
    v1, c1, n1, d1 = run(1)
    oracle.Oracle(cfg, f0, threads=all_cores)
    sample = f"{cfg['nx']}x{cfg['ny']} lattice of the workload (lattice 0), FP64 steps from the initial state"
    return dict(value=round(va, 2), unit="MLUPS", cores=ca, kind="oracle",
                sample=f"{sample}: {na} steps in {da:.1f} s on {ca} OpenMP threads",
                single_thread={"value": round(v1, 2), "unit": "MLUPS", "cores": c1,
                               "sample": f"{sample}: {n1} steps in {d1:.1f} s on one thread"})


def surrogate_leg(n: int, blocks: int = 10, warm: int = 30000, weights: str = "surrogate_k100_sweep2000.npz",
                  lattices: str = "256x1024"):
    """Hybrid rollout of a trained surrogate against the plain FP32 lattice
    update: speedup and relative L2 errors over `blocks` blocks of 100 steps,
    on fresh 256 x 1024 droplet lattices drawn with the sweep's parameters
    (lattices="256x1024") or on lattices of the batched-sweep generator
    (lattices="sweep", uneven sizes); seed 55 for both."""
    from paper_2306_11320_amd import surrogate as S
    from paper_2306_11320_amd import workloads as wl
    from paper_2306_11320_amd.train_surrogate import sweep_items
    wpath = os.path.join(ROOT, "paper_2306_11320_amd", "weights", weights)
    net = S.Surrogate.load(wpath)
    items = sweep_items(n, 55, 256, 1024) if lattices == "256x1024" else wl.sweep(n, seed=55, laplace_p=True)
    res = S.evaluate(net, items, warm=warm, blocks=blocks, K=100, check_every=10, chunk=blocks,
                     log=lambda m: print(m, file=sys.stderr, flush=True))
    sp = [sum(r["t_ref_ms"]) / sum(r["t_hybrid_ms"]) for r in res]
    err = [max(r["err_hybrid"][-1].values()) for r in res]
    ok = [s_ for s_, e in zip(sp, err) if e <= 0.01]
    srt = sorted(ok)
    return {
        "workload": "droplet_sweep_256x1024" if lattices == "256x1024" else "batched_sweep_generator_uneven",
        "K": 100, "blocks": blocks, "warm_steps": warm,
        "instances": n, "weights": f"paper_2306_11320_amd/weights/{weights}",
        "speedup": [round(v, 3) for v in sp],
        "max_rel_l2": [round(v, 5) for v in err],
        "max_rel_l2_net_only": [round(max(r["err_net_only"][-1].values()), 5) for r in res],
        "max_rel_l2_persistence": [round(max(r["err_persistence"][-1].values()), 5) for r in res],
        "rel_l2_by_field": [{k: round(v, 5) for k, v in r["err_hybrid"][-1].items()} for r in res],
        "fallbacks": [r["fallbacks"] for r in res],
        "instances_within_1pct": len(ok),
        "speedup_at_le_1pct_median": round(srt[len(srt) // 2], 3) if srt else None,
        "lbm_ms": [round(sum(r["t_ref_ms"]), 3) for r in res],
        "hybrid_ms": [round(sum(r["t_hybrid_ms"]), 3) for r in res],
    }


def conv_leg(reps: int = 50) -> dict:
    """The surrogate's convolutions on one 256 x 1024 frame, timed with HIP
    events on the network's stream: a hidden layer (32 channels, dilation 4,
    input ReLU and residual, BF16 out) against the BF16 dense peak, and a
    whole network block (packing, six layers, the fused state update)."""
    import torch
    from paper_2306_11320_amd import surrogate as S
    from paper_2306_11320_amd.train_surrogate import sweep_items
    net = S.Surrogate.load(os.path.join(ROOT, "paper_2306_11320_amd", "weights", "surrogate_k100_sweep2000.npz"))
    st = torch.cuda.Stream()
    net.stream = st
    H, W = 1024, 256
    g = torch.Generator(device="cpu").manual_seed(0)
    x = (0.5 * torch.randn((1, H, W, 32), generator=g)).to(torch.bfloat16).to("cuda")
    out = torch.empty_like(x)
    cfg, _ = sweep_items(1, 55, W, H)[0]
    sc = S.scales_of(cfg, net.kappa)
    state = {k: torch.zeros((H, W), device="cuda") for k in S.FIELDS}
    state["phi"].fill_(1.0)
    torch.cuda.synchronize()

    def timed(fn):
        for _ in range(5):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            fn()
        e1.record(st)
        st.synchronize()
        return e0.elapsed_time(e1) / reps * 1e3  # us

    layer_us = timed(lambda: S.sur_conv3x3(x, 32, net.Wb[2], net.b[2], x, None, out, True, st, 4))
    block_us = timed(lambda: net.advance(state, sc))
    flop = 2 * 9 * 32 * 32 * H * W
    return {"frame": "256x1024", "hidden_layer_us": round(layer_us, 2),
            "hidden_layer_tflops": round(flop / layer_us / 1e6, 1),
            "hidden_layer_frac_of_bf16_dense_peak": round(flop / layer_us / 1e6 / 2500.0, 4),
            "network_block_us": round(block_us, 1), "flop_per_hidden_layer": flop}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2048)
    ap.add_argument("--warmup", type=int, default=256)
    ap.add_argument("--workload", default="sweep", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--only", action="store_true", help="time only --workload in --precision")
    ap.add_argument("--tile", type=int, default=None)
    ap.add_argument("--tune-cache", default=None, metavar="JSON",
                    help="reuse (or store) the autotuner's choice for a batch in this file")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-error", action="store_true", help="skip the oracle error windows")
    ap.add_argument("--surrogate", type=int, default=4, metavar="N",
                    help="lattices for the surrogate leg (0 skips it)")
    ap.add_argument("--surrogate-only", action="store_true",
                    help="run only the surrogate leg on --surrogate lattices (profiling runs)")
    ap.add_argument("--conv-only", action="store_true",
                    help="run only the surrogate's convolution timings (profiling runs)")
    ap.add_argument("--potential", action="store_true",
                    help="potential form of the capillary force (-phi grad mu_phi) instead of Eq. 11's")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run the plain copy kernel on MIB MiB, 20 times (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the lattice update runs on one GPU "
              "and is not sharded across GPUs", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2306_11320_amd import lbm
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        n = args.calibrate_copy << 20
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        st = torch.cuda.Stream()
        for _ in range(3):
            lbm.copy_probe(src, dst, st)
        st.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(20):
            lbm.copy_probe(src, dst, st)
        e1.record(st)
        st.synchronize()
        ms = e0.elapsed_time(e1) / 20
        print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "ms_per_copy": ms,
                          "copy_GBps": 2 * n / (ms * 1e-3) / 1e9}), flush=True)
        return
    if args.conv_only:
        print(json.dumps({"surrogate_conv": conv_leg()}), flush=True)
        return
    prewarm()
    if args.surrogate_only:
        print(json.dumps({"surrogate": surrogate_leg(max(1, args.surrogate))}), flush=True)
        return
    head, items, desc = lbm_leg(args.workload, args.precision, args.steps, args.warmup, args.tile, args.potential,
                                args.tune_cache)
    cfg_out = dict(desc, precision=head["precision"], parallelism="single_gpu", tile=head["tile"],
                   working_set_bytes=head["working_set_bytes"],
                   algorithmic_bytes_per_launch=head["algorithmic_bytes_per_launch"])
    if "autotuned" in head:
        cfg_out["autotuned"] = head["autotuned"]
    out = {
        "metric": METRIC, "value": head["value"], "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64", "data": "synthetic", "config": cfg_out,
        "roofline": head["roofline"],
    }
    if not args.only:
        if len(items) > 1:
            log("sequential single-lattice baseline of the batch")
            seq_ms = time_sequential(items, lbm.FP32_DEV if args.precision == "fp32" else lbm.FP64,
                                     max(16, args.steps // 8), max(4, args.warmup // 8))
            out["batched"] = {"sequential_ms_per_step": round(seq_ms, 5),
                              "batched_ms_per_step": head["ms_per_step"],
                              "speedup_over_sequential": round(seq_ms / head["ms_per_step"], 3),
                              "error": "bitwise equal to the sequential runs (tested)"}
        extra = []
        for name, prec in (("sweep", "fp64"), ("bubbles", "fp64"), ("bubbles", "fp32"), ("droplet", "fp32"),
                           ("droplet", "fp64")):
            if (name, prec) != (args.workload, args.precision):
                extra.append((name, prec))
        out["other_workloads"] = []
        # tile id each timed workload ran with: its error window runs with it too
        timed_tile = {(args.workload, args.precision): (head.get("autotuned") or {}).get("tile", args.tile)}
        for name, prec in extra:
            leg, _, _ = lbm_leg(name, prec, args.steps, args.warmup, None, args.potential)
            leg["cache_resident"] = leg["working_set_bytes"] <= 256 * 2 ** 20
            timed_tile[(name, prec)] = (leg.get("autotuned") or {}).get("tile")
            out["other_workloads"].append(leg)
        if not args.no_error:
            log("errors against the FP64 oracle (200-step windows)")
            out["oracle_error"] = {}
            for name, prec in ((args.workload, args.precision), ("sweep", "fp64"), ("bubbles", "fp64"),
                               ("bubbles", "fp32")):
                key = f"{name}_{prec}"
                if key not in out["oracle_error"]:
                    out["oracle_error"][key] = oracle_error(name, prec, tile=timed_tile.get((name, prec)))
        if args.surrogate > 0:
            # the network trained on 2000 trajectories of the batched-sweep
            # generator, on 256 x 1024 lattices and on the generator's own
            # uneven lattices; beside it the earlier network trained on 64
            # fixed 256 x 1024 lattices
            log("surrogate")
            out["surrogate"] = surrogate_leg(args.surrogate)
            out["surrogate_conv"] = conv_leg()
            log("surrogate on lattices of the batched-sweep generator")
            out["surrogate_uneven"] = surrogate_leg(2, lattices="sweep")
            log("surrogate trained on 64 fixed lattices")
            out["surrogate_fixed64"] = surrogate_leg(2, weights="surrogate_k100.npz")
    if not args.no_cpu:
        log("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(items)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
