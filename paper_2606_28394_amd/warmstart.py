"""Training data and training of the learned PGS warm start, on the GPU.

Data: episodes of the 450-tower removal batch (other seeds than the evaluation batch) stepped
with the plain solver at many iterations (converged impulses), recording every contact point's
24 features, k_n, k_t1, k_t2 and solved impulses (jg_query_features).  Targets are the
change of the dimensionless impulses lambda_d k_d / (|g| dt) from the previous step's.

Training: mean squared error, AdamW (learning rate 3e-4 and weight decay 1e-4 by default, the
paper's optimiser settings), forward and backward in the library's own matrix-core kernels
(jg_mlp_grad, jg_mlp_adamw).  Features are z-scored with the training set's statistics.

    python -m paper_2606_28394_amd.warmstart --out paper_2606_28394_amd/data/warmstart_mlp.npy

(the shipped network: 10^7 records from plain solves at 100 iterations, 20 epochs, batch 8192,
learning rate 1e-3 on a cosine, weight decay 1e-4, targets clipped to +-0.5, seed 0)
"""
from __future__ import annotations

import argparse
import math
import time

import numpy as np

from . import jenga as J
from . import workloads as W

N_FEAT = 24


def targets_of(records: np.ndarray, gravity_norm: float, dt: float, clip: float | None = 0.5) -> np.ndarray:
    """Network targets from records (n x 30: features, k[3], impulses[3]): the change of the
    dimensionless impulses lambda_d k_d / (|g| dt) from the previous step's (features 12..14),
    clipped to +-clip.  Impact transients, which no warm start can anticipate, would otherwise
    dominate the squared error.  The clip also keeps the network's corrections small: the
    previous impulses are already a good start, and the corrections are added to every contact.
    On the removal batch, the median residual after 4 sweeps was lowest at clip 0.5 among
    10, 2, 1 and 0.5."""
    r = records.astype(np.float64)
    t = r[:, 27:30] * r[:, 24:27] / (gravity_norm * dt) - r[:, 12:15]
    return t if clip is None else np.clip(t, -clip, clip)


def generate(n_records: int, iters: int = 100, episodes_seed: int = 1, every: int = 50, n_per_mu: int = 50,
             max_steps: int = 2000, log=print) -> np.ndarray:
    """Records from plain solves at `iters` iterations over removal episodes, one snapshot of
    every tower every `every` steps, until n_records are collected."""
    out, total, seed = [], 0, episodes_seed
    while total < n_records:
        sc = W.cfg2(seed=seed, n_per_mu=n_per_mu, n_steps=max_steps)
        p = dict(sc["params"])
        p["iters"] = iters
        world = J.World(sc, record_features=True, params=p)
        steps = 0
        while steps < max_steps and total < n_records:
            world.step(every)
            steps += every
            rec = world.features(-1)
            out.append(rec)
            total += len(rec)
        log(f"  episode seed {seed}: {steps} steps, {total} records")
        world.close()
        seed += 1
    return np.concatenate(out)[:n_records]


def init_params(features: np.ndarray, seed: int = 0) -> np.ndarray:
    """Initial weights and the feature normalisation.  A feature's scale is its standard
    deviation, but at least 1% of its RMS value: a feature that barely varies in the training
    set (the relative orientation of upright blocks) must not turn small changes into huge
    network inputs."""
    flat = W.mlp_init(seed)
    mean = features.mean(axis=0)
    sd = features.std(axis=0)
    rms = np.sqrt(mean ** 2 + sd ** 2)
    flat[-2 * N_FEAT:-N_FEAT] = mean
    flat[-N_FEAT:] = np.maximum(np.maximum(sd, 1e-2 * rms), 1e-9)
    return flat


def fit(features: np.ndarray, targets: np.ndarray, epochs: int = 4, batch: int = 16384, lr: float = 3e-4,
        weight_decay: float = 1e-4, seed: int = 0, lr_floor: float = 1 / 20, log=print):
    """Train on the GPU; returns (parameters as float32, per-epoch mean losses).  The learning
    rate follows a cosine from lr down to lr * lr_floor over the run."""
    import torch
    dev = "cuda"
    F = torch.as_tensor(np.ascontiguousarray(features, np.float32), device=dev)
    T = torch.as_tensor(np.ascontiguousarray(targets, np.float32), device=dev)
    n = F.shape[0]
    net = J.Mlp(init_params(features, seed))
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    steps_per_epoch = max(1, n // batch)
    total_steps = epochs * steps_per_epoch
    losses = []
    step = 0
    for ep in range(epochs):
        perm = torch.randperm(n, device=dev, generator=gen)
        acc = torch.zeros((), device=dev)
        for b in range(steps_per_epoch):
            idx = perm[b * batch:(b + 1) * batch]
            cur = lr * (lr_floor + (1 - lr_floor) * 0.5 * (1 + math.cos(math.pi * step / max(1, total_steps))))
            acc += net.train_step(F[idx].contiguous(), T[idx].contiguous(), lr=cur, weight_decay=weight_decay)[0]
            step += 1
        losses.append(float(acc.item()) / steps_per_epoch)
        log(f"  epoch {ep}: mse {losses[-1]:.5f}")
    return net.params.cpu().numpy(), losses


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--out", required=True)
    ap.add_argument("--records", type=float, default=1e7)
    ap.add_argument("--iters", type=int, default=100)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--weight-decay", type=float, default=1e-4)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--clip", type=float, default=0.5)
    args = ap.parse_args()
    J.load_library()
    t0 = time.time()
    rec = generate(int(args.records), iters=args.iters)
    g = math.sqrt(sum(x * x for x in W.default_params()["gravity"]))
    dt = W.default_params()["dt"]
    feats, tg = rec[:, :N_FEAT].astype(np.float64), targets_of(rec, g, dt, args.clip)
    print(f"data: {len(rec)} records in {time.time() - t0:.1f} s", flush=True)
    t0 = time.time()
    params, losses = fit(feats, tg, epochs=args.epochs, batch=args.batch, lr=args.lr,
                         weight_decay=args.weight_decay, seed=args.seed)
    print(f"training: {time.time() - t0:.1f} s, mse {losses[0]:.5f} -> {losses[-1]:.5f}", flush=True)
    np.save(args.out, params.astype(np.float32))
    print(f"saved {args.out}", flush=True)


if __name__ == "__main__":
    main()
