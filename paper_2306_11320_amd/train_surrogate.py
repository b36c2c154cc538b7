"""Trains the learned surrogate on trajectories of the FP32 lattice update and
evaluates the hybrid rollout on fresh lattices.

    python -m paper_2306_11320_amd.train_surrogate --out weights.npz [--report r.json] [--source sweep]

--source sweep (the default): --n-traj trajectories from the batched-sweep
generator (NX uniform in 128..256, NY = 4 NX, R in [16, 40], Ma in [0.1, 50],
lambda_r in [0.5, 2]; seed --seed), started with the Laplace pressure and run
--batch-lattices at a time by the batched FP32 lattice update; each batch
yields a pair (state at t, increment to t + K) per lattice every --stride
steps from --t0 to --t1, trains --iters-per-batch Adam steps (each on --frames
pairs of one lattice, a random band of --crop rows at full width) and is then
discarded.  --source fixed: --n-train lattices of --nx x --ny, all pairs held
in memory, --iters Adam steps.  Both use a cosine learning-rate decay.
Evaluation: --n-eval fresh lattices from the same generator (seed
--eval-seed) warmed up for --warm steps, then --blocks blocks of K steps.

The committed weights: weights/surrogate_k100_sweep2000.npz (the production
network) from the defaults, i.e. 2000 trajectories, pairs every 500 steps
from t = 28000 to 36000, 700 Adam steps per batch of 64 lattices (17 min on
one MI355X); weights/surrogate_k100.npz (the earlier network) from
--source fixed --t0 20000 --t1 45000 --n-eval 8 --blocks 30.  Each has a
report beside it with the arguments of its run.
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np


def sweep_items(n: int, seed: int, nx: int, ny: int):
    from . import workloads as wl
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        R = float(rng.uniform(16.0, 40.0))
        Ma = float(rng.uniform(0.1, 50.0))
        lr = float(rng.uniform(0.5, 2.0))
        out.append(wl.sweep_instance(nx, ny, R, Ma, lr, laplace_p=True))
    return out


def eval_items(source: str, n: int, seed: int, nx: int, ny: int):
    from . import workloads as wl
    if source == "sweep":
        return wl.sweep(n, seed=seed, laplace_p=True)
    return sweep_items(n, seed, nx, ny)


def main(argv=None) -> dict:
    import torch
    from . import surrogate as S
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", required=True)
    ap.add_argument("--report", default=None)
    ap.add_argument("--nx", type=int, default=256)
    ap.add_argument("--ny", type=int, default=1024)
    ap.add_argument("--n-train", type=int, default=64)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--K", type=int, default=100)
    ap.add_argument("--t0", type=int, default=28000)
    ap.add_argument("--t1", type=int, default=36000)
    ap.add_argument("--stride", type=int, default=500)
    ap.add_argument("--iters", type=int, default=12000)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--crop", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--n-eval", type=int, default=4)
    ap.add_argument("--eval-seed", type=int, default=55)
    ap.add_argument("--warm", type=int, default=30000)
    ap.add_argument("--blocks", type=int, default=20)
    ap.add_argument("--check-every", type=int, default=10)
    ap.add_argument("--tol-check", type=float, default=0.01)
    ap.add_argument("--source", default="sweep", choices=["sweep", "fixed"])
    ap.add_argument("--n-traj", type=int, default=2000)
    ap.add_argument("--batch-lattices", type=int, default=64)
    ap.add_argument("--iters-per-batch", type=int, default=700)
    ap.add_argument("--frames", type=int, default=8)
    ap.add_argument("--checkpoint", default=None, help="save the weights here after every 4 batches")
    ap.add_argument("--init", default=None, help="start from these weights (and their kappa) instead of random ones")
    a = ap.parse_args(argv)
    rep = {"args": vars(a)}
    if a.source == "sweep":
        return main_streamed(a, rep)

    t = time.perf_counter()
    items = sweep_items(a.n_train, a.seed, a.nx, a.ny)
    starts = list(range(a.t0, a.t1 + 1, a.stride))
    X, Y = S.generate_pairs(items, a.K, starts)
    torch.cuda.synchronize()
    rep["pairs"] = int(X.shape[0])
    rep["t_generate_s"] = time.perf_counter() - t
    print(f"[data] {X.shape[0]} pairs in {rep['t_generate_s']:.1f} s", flush=True)
    kappa = S.dataset_kappa(X)
    rep["kappa"] = kappa
    for c in range(S.N_OUT):
        Y[..., c] /= kappa[c]
    rep["target_rms"] = [float(torch.sqrt(torch.mean(Y[..., c] ** 2)).item()) for c in range(S.N_OUT)]
    print(f"[data] kappa {kappa} target rms {rep['target_rms']}", flush=True)

    net = S.Surrogate(seed=a.seed, kappa=kappa)
    t = time.perf_counter()
    hist = S.train(net, X, Y, a.iters, a.batch, lr=a.lr, seed=a.seed, log_every=max(1, a.iters // 20),
                   crop_rows=a.crop)
    torch.cuda.synchronize()
    rep["t_train_s"] = time.perf_counter() - t
    rep["loss_first"] = float(np.mean(hist[:20]))
    rep["loss_last"] = float(np.mean(hist[-100:]))
    print(f"[train] {a.iters} iterations in {rep['t_train_s']:.1f} s, loss {rep['loss_first']:.3e} -> "
          f"{rep['loss_last']:.3e}", flush=True)
    net.save(a.out)
    del X, Y
    torch.cuda.empty_cache()

    ev = eval_items(a.source, a.n_eval, a.eval_seed, a.nx, a.ny)
    res = S.evaluate(net, ev, warm=a.warm, blocks=a.blocks, K=a.K, check_every=a.check_every,
                     tol_check=a.tol_check, log=lambda m: print(m, flush=True))
    rep["eval"] = res
    if a.report:
        with open(a.report, "w") as f:
            json.dump(rep, f, indent=1)
    return rep


def main_streamed(a, rep: dict) -> dict:
    """Trajectories of the batched-sweep generator, generated batch by batch
    and streamed into training."""
    import torch
    from . import surrogate as S
    from . import workloads as wl
    items = wl.sweep(a.n_traj, seed=a.seed, laplace_p=True)
    batches = [items[i:i + a.batch_lattices] for i in range(0, len(items), a.batch_lattices)]
    starts = list(range(a.t0, a.t1 + 1, a.stride))
    rep["trajectories"] = len(items)
    rep["nodes_per_trajectory_mean"] = float(np.mean([c["nx"] * c["ny"] for c, _ in items]))
    rep["pairs"] = len(items) * len(starts)
    net = S.Surrogate.load(a.init) if a.init else S.Surrogate(seed=a.seed)
    if a.init:
        rep["init"] = a.init

    def on_batch(bi, hist):
        if a.checkpoint and (bi + 1) % 4 == 0:
            net.save(a.checkpoint)

    t = time.perf_counter()
    hist = S.train_streamed(net, batches, a.K, starts, a.iters_per_batch, a.frames, a.crop, lr=a.lr, seed=a.seed,
                            log=lambda m: print(m, flush=True), on_batch=on_batch)
    torch.cuda.synchronize()
    rep["t_generate_and_train_s"] = time.perf_counter() - t
    rep["kappa"] = list(net.kappa)
    rep["iters"] = len(hist)
    rep["loss_first"] = float(np.mean(hist[:20]))
    rep["loss_last"] = float(np.mean(hist[-100:]))
    print(f"[train] {len(hist)} steps over {len(items)} trajectories in {rep['t_generate_and_train_s']:.1f} s, "
          f"loss {rep['loss_first']:.3e} -> {rep['loss_last']:.3e}", flush=True)
    net.save(a.out)
    torch.cuda.empty_cache()
    ev = eval_items("sweep", a.n_eval, a.eval_seed, a.nx, a.ny)
    res = S.evaluate(net, ev, warm=a.warm, blocks=a.blocks, K=a.K, check_every=a.check_every,
                     tol_check=a.tol_check, log=lambda m: print(m, flush=True))
    rep["eval"] = res
    if a.report:
        with open(a.report, "w") as f:
            json.dump(rep, f, indent=1)
    return rep


if __name__ == "__main__":
    main()
