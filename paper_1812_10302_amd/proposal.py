"""Training data and training loop of the learned block ordering.

The ordering network learns log1p(DTW / m) of a (query, candidate) pair from their PAA
features.  Training pairs are drawn from a separate series: noisy cuts of it serve as queries,
half of each query's candidates are random windows and half lie within +-m of the query's
source.  Labels come from this library's own banded DTW kernel (exact values, no abandoning)
and features from its PAA kernel; the updates run in its forward/backward/Adam kernels.  This
module only draws the pairs and drives the loop.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import workloads as W


def make_pairs(ctx, T_host: np.ndarray, m: int, r: int, n_queries: int, per_query: int, seed: int,
               noise_std: float = 0.1):
    """Feature rows X (n x 32) and targets y* = log1p(DTW / m) (n), as CUDA tensors."""
    import torch
    dev = torch.device("cuda", ctx.device)
    rng = np.random.default_rng(seed)
    n = T_host.size
    Td = torch.from_numpy(T_host).to(dev)
    Xs, Ys = [], []
    half = per_query // 2
    for k in range(n_queries):
        src = int(rng.integers(0, n - m))
        Q = W.noisy_cut(T_host, src, m, noise_std, seed * 100_003 + k)
        Qd = torch.from_numpy(Q).to(dev)
        near = np.clip(src + rng.integers(-m, m + 1, half), 0, n - m)
        far = rng.integers(0, n - m + 1, per_query - half)
        starts = torch.from_numpy(np.concatenate([near, far]).astype(np.int64)).to(dev)
        d = ctx.dtw_band(Td, Qd, r, starts)
        qf = ctx.paa(Qd, m, torch.zeros(1, dtype=torch.int64, device=dev))
        cf = ctx.paa(Td, m, starts)
        Xs.append(torch.cat([qf.expand(starts.numel(), 16), cf], dim=1))
        Ys.append(torch.log1p(d / m))
    return torch.cat(Xs).contiguous(), torch.cat(Ys).contiguous()


def train(ctx, X, Y, epochs: int = 3, batch: int = 4096, lr: float = 1e-3, seed: int = 0, init: bool = True,
          log=None):
    """Adam on mean squared error; returns the per-epoch mean training loss."""
    import torch
    if init:
        ctx.model_init(seed)
    g = torch.Generator(device="cpu").manual_seed(seed)
    n = X.shape[0]
    curve = []
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(X.device)
        Xp, Yp = X[perm].contiguous(), Y[perm].contiguous()
        tot, cnt = 0.0, 0
        t0 = time.time()
        for a in range(0, n - batch + 1, batch):
            want = (a // batch) % 16 == 0
            loss = ctx.model_train_step(Xp[a:a + batch], Yp[a:a + batch], lr, want_loss=want)
            if want:
                tot += loss
                cnt += 1
        curve.append(tot / max(cnt, 1))
        if log:
            log(f"epoch {ep}: loss {curve[-1]:.5f} ({time.time() - t0:.2f}s)")
    return curve


def train_default(ctx, n: int = 10_000_000, m: int = 256, frac: float = 0.05, pairs: int = 1_000_000,
                  epochs: int = 3, seed: int = 8, log=None):
    """The default recipe: sinusoid/random-walk mixture of n points (seed 8), queries of length m,
    band frac*m, `pairs` labelled pairs (half near the source, half random)."""
    T = W.sinusoid_mix(n, seed)
    r = int(math.floor(frac * m))
    per_query = 1000
    X, Y = make_pairs(ctx, T, m, r, max(1, pairs // per_query), per_query, seed)
    return train(ctx, X, Y, epochs=epochs, seed=seed, log=log)
