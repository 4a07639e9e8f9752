"""Train the learned initial guess on trajectories the solver generates itself.

    python -m paper_1208_2643_amd.train_guess [--out PATH] [--iters N] ...

1. Data: `--trajectories` runs of the second-order scheme with the 1024^2
   benchmark's parameters (h = pi/4, eps = 0.025, beta = 0.9, M = 1, dt = 0.05)
   on `--grid`^2 grids, each from 0.07 liquid with three one-mode
   crystallites of radius 20 h (seeds 100, 101, ...; the benchmark's
   evaluation uses seed 5), `--steps` steps each, all advanced together by the
   batched solver in FP64 to residual 1e-10.  Every state stays on the GPU;
   a training sample is (phi^{n-1}, phi^n, psi^n, phi^{n+1}) of one run.
   The last `--holdout` runs are kept for validation.
2. Scale: out_scale is set so that the target (phi^{n+1} - 2 phi^n +
   phi^{n-1}) / (out_scale sigma1) has unit mean square over the data (the
   loss of the zero-output network, measured with the library's kernels).
3. Training: Adam on random batches, learning rate `--lr` with a cosine decay
   to 1 % over `--iters` iterations; all passes run in the library's kernels.
4. Output: the blob (float32) and a JSON file next to it with the settings,
   the loss curve and the validation loss (1.0 = extrapolation).

The losses are normalised so that 1.0 is the error of plain extrapolation.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np


def parse(argv=None):
    from . import guess_net
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", default=guess_net.DEFAULT_WEIGHTS)
    ap.add_argument("--grid", type=int, default=256)
    ap.add_argument("--trajectories", type=int, default=18)
    ap.add_argument("--holdout", type=int, default=2)
    ap.add_argument("--steps", type=int, default=1250)
    ap.add_argument("--iters", type=int, default=4000)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=1)
    return ap.parse_args(argv)


def log(msg):
    print(f"[train_guess] {msg}", file=sys.stderr, flush=True)


def generate(args, torch, api, inputs, dev):
    """States phi and psi of every run: tensors (runs, steps + 1, n, m) on the GPU
    (psi[r, k] = psi^k, the input of step k)."""
    N = args.grid
    h = math.pi / 4
    params = api.Params(eps=0.025, beta=0.9, M=1.0, h=h, dt=0.05, scheme=2)
    R = args.trajectories
    store = torch.empty((R, args.steps + 1, N, N), dtype=torch.float64, device=dev)
    pstore = torch.zeros((R, args.steps + 1, N, N), dtype=torch.float64, device=dev)
    for r in range(R):
        store[r, 0] = torch.from_numpy(inputs.crystallites(N, N, h, seed=100 + r)).to(dev)
    b = api.Batch([(N, N, params)] * R, tol=1e-10, precision=0)
    cycles = 0
    t0 = time.perf_counter()
    for k in range(args.steps):
        prev = [store[r, max(k - 1, 0)] for r in range(R)]
        pstore[:, k + 1].copy_(pstore[:, k])
        infos = b.step([store[r, k] for r in range(R)], prev, [pstore[r, k + 1] for r in range(R)],
                       [store[r, k + 1] for r in range(R)], history=False)
        cycles += sum(i.n_cycles for i in infos)
        if (k + 1) % 250 == 0:
            log(f"data: {k + 1}/{args.steps} steps ({time.perf_counter() - t0:.1f} s)")
    b.close()
    torch.cuda.synchronize()
    return store, pstore, cycles / (R * args.steps)


def batches(data, runs, steps, batch, rng):
    """Random samples (run, n) with 1 <= n < steps (phi^{n-1} != phi^n)."""
    store, pstore = data
    rr = rng.choice(runs, size=batch)
    nn = rng.integers(1, steps, size=batch)
    return ([store[r, n - 1] for r, n in zip(rr, nn)], [store[r, n] for r, n in zip(rr, nn)],
            [pstore[r, n] for r, n in zip(rr, nn)], [store[r, n + 1] for r, n in zip(rr, nn)])


def mean_loss(tr, data, runs, steps, batch, count, seed):
    rng = np.random.default_rng(seed)
    return float(np.mean([tr.step(*batches(data, runs, steps, batch, rng), update=False)
                          for _ in range(count)]))


def main(argv=None):
    args = parse(argv)
    import torch
    from . import api, guess_net, inputs
    dev = torch.device("cuda:0")
    t_start = time.perf_counter()
    store, pstore, cyc = generate(args, torch, api, inputs, dev)
    data = (store, pstore)
    t_data = time.perf_counter() - t_start
    N = args.grid
    train_runs = np.arange(args.trajectories - args.holdout)
    val_runs = np.arange(args.trajectories - args.holdout, args.trajectories)
    log(f"data: {args.trajectories} runs x {args.steps} steps of {N}^2 in {t_data:.1f} s, "
        f"{cyc:.2f} V-cycles per step")

    blob = guess_net.initial_blob(args.seed, 0.05, out_scale=1.0)
    tr = api.CnnTrainer(N, N, args.batch, blob, lr=args.lr)
    ms = mean_loss(tr, data, train_runs, args.steps, args.batch, 16, args.seed + 1)
    tr.close()
    out_scale = math.sqrt(ms)
    blob = guess_net.with_out_scale(blob, out_scale)
    log(f"out_scale = {out_scale:.4g}")

    tr = api.CnnTrainer(N, N, args.batch, blob, lr=args.lr)
    rng = np.random.default_rng(args.seed + 2)
    curve = []
    t0 = time.perf_counter()
    run_loss = 0.0
    for it in range(args.iters):
        lr = args.lr * (0.01 + 0.99 * 0.5 * (1 + math.cos(math.pi * it / args.iters)))
        tr.set_lr(lr)
        loss = tr.step(*batches(data, train_runs, args.steps, args.batch, rng))
        if not math.isfinite(loss):
            raise RuntimeError(f"training diverged at iteration {it}")
        run_loss += loss
        if (it + 1) % 200 == 0:
            curve.append([it + 1, run_loss / 200])
            log(f"iter {it + 1}/{args.iters}: loss {run_loss / 200:.4f} (lr {lr:.2e}, "
                f"{time.perf_counter() - t0:.1f} s)")
            run_loss = 0.0
    t_train = time.perf_counter() - t0
    val = mean_loss(tr, data, val_runs, args.steps, args.batch, 32, args.seed + 3)
    trained = tr.blob()
    tr.close()
    log(f"validation loss {val:.4f} (extrapolation = 1)")
    meta = {
        "network": "4 x conv3x3 (3-32-32-32-1), tanh-GELU, circular padding, BF16/FP32",
        "data": {"grid": N, "runs": args.trajectories, "holdout": args.holdout,
                 "steps": args.steps, "seeds": [100, 100 + args.trajectories - 1],
                 "params": "scheme 2, h=pi/4, eps=0.025, beta=0.9, M=1, dt=0.05, "
                           "0.07 liquid + 3 crystallites of radius 20h",
                 "vcycles_per_step": cyc, "seconds": t_data},
        "training": {"iters": args.iters, "batch": args.batch, "lr": args.lr,
                     "schedule": "cosine to 1%", "optimizer": "Adam(0.9, 0.999, 1e-8)",
                     "seed": args.seed, "seconds": t_train, "curve": curve},
        "out_scale": out_scale, "in_scale": float(trained[4]),
        "validation_loss": val,
    }
    guess_net.save(trained, args.out, meta)
    log(f"wrote {args.out}")
    print(json.dumps({"validation_loss": val, "out_scale": out_scale, "data_s": t_data,
                      "train_s": t_train}), flush=True)


if __name__ == "__main__":
    main()
