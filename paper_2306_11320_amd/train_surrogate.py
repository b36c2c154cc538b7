"""Trains the learned surrogate on trajectories of the FP32 lattice update and
evaluates the hybrid rollout on fresh lattices.

    python -m paper_2306_11320_amd.train_surrogate --out weights.npz [--report r.json]

Data: droplet-migration lattices of nx x ny nodes drawn like the parameter
sweep (R in [16, 40], Ma in [0.1, 50], lambda_r in [0.5, 2]; seed --seed),
started with the Laplace pressure, advanced by the batched FP32 lattice update;
a pair (state at t, increment to t + K) every --stride steps from --t0 to --t1.
Training: Adam with a cosine learning-rate decay on bands of --crop rows at
full width.  Evaluation: --n-eval fresh lattices (seed --eval-seed) warmed up
for --warm steps, then --blocks blocks of K steps.
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
    ap.add_argument("--t0", type=int, default=20000)
    ap.add_argument("--t1", type=int, default=45000)
    ap.add_argument("--stride", type=int, default=500)
    ap.add_argument("--iters", type=int, default=12000)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--crop", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--n-eval", type=int, default=8)
    ap.add_argument("--eval-seed", type=int, default=55)
    ap.add_argument("--warm", type=int, default=30000)
    ap.add_argument("--blocks", type=int, default=30)
    ap.add_argument("--check-every", type=int, default=10)
    ap.add_argument("--tol-check", type=float, default=0.01)
    a = ap.parse_args(argv)
    rep = {"args": vars(a)}

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

    ev = sweep_items(a.n_eval, a.eval_seed, a.nx, a.ny)
    res = S.evaluate(net, ev, warm=a.warm, blocks=a.blocks, K=a.K, check_every=a.check_every,
                     tol_check=a.tol_check, log=lambda m: print(m, flush=True))
    rep["eval"] = res
    if a.report:
        with open(a.report, "w") as f:
            json.dump(rep, f, indent=1)
    return rep


if __name__ == "__main__":
    main()
