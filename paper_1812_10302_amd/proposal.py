"""Training data and training loop of the learned block ordering.

The ordering network learns y* = log(DTW / m + 1e-4) of a (query, candidate) pair from their PAA
features; the offset spreads out the small distances that decide which block is visited first.
Training pairs are drawn from a separate series.  Three in four queries are noisy cuts of it (noise
std 0.5, 1 or 2 times noise_std) and one in four an independent random walk.  A query's
candidates are its proposals over the whole training series (the per-quarter-block PAA-nearest
starts that the learned order scores at search time), starts within +-m/4 and within +-2 proposal
strides of the query's source, and uniform random starts.  Labels come from
this library's banded DTW kernel (exact values, no abandoning), features from its PAA and proposal
kernels, and the updates run in its forward/backward/Adam kernels.  This module only draws the
pairs and drives the loop.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import workloads as W

TARGET_EPS = 1e-4


def target(d, m: int):
    """Training target of a DTW distance d of a length-m pair."""
    import torch
    return torch.log(d / m + TARGET_EPS)


def make_pairs(ctx, T_host: np.ndarray, m: int, r: int, n_queries: int, seed: int, near: int = 32,
               random: int = 256, noise_std: float = 0.1):
    """Feature rows X (rows x 32) and targets y* (rows) for n_queries training queries, as CUDA
    tensors; about n / 1024 + 2 near + random rows per query for a series of n points."""
    import torch
    dev = torch.device("cuda", ctx.device)
    rng = np.random.default_rng(seed)
    n = T_host.size
    Td = torch.from_numpy(T_host).to(dev)
    zero = torch.zeros(1, dtype=torch.int64, device=dev)
    Xs, Ys = [], []
    for k in range(n_queries):
        if k % 4 == 3:
            src = None
            Q = W.random_walk(m, seed * 100_003 + k)
        else:
            src = int(rng.integers(0, n - m))
            Q = W.noisy_cut(T_host, src, m, noise_std * (0.5, 1.0, 2.0)[k % 3], seed * 100_003 + k)
        Qd = torch.from_numpy(Q).to(dev)
        ps, px = ctx.propose(Td, Qd)
        keep = ps >= 0
        ps, px = ps[keep], px[keep]
        extra = [rng.integers(0, n - m + 1, random)]
        if src is not None:
            stride = m // 64 if m >= 128 else 1
            extra.append(np.clip(src + rng.integers(-(m // 4), m // 4 + 1, near), 0, n - m))
            extra.append(np.clip(src + rng.integers(-2 * stride, 2 * stride + 1, near), 0, n - m))
        es = torch.from_numpy(np.concatenate(extra).astype(np.int64)).to(dev)
        qf = ctx.paa(Qd, m, zero)
        ex = torch.cat([qf.expand(es.numel(), 16), ctx.paa(Td, m, es)], dim=1)
        starts = torch.cat([ps, es]).contiguous()
        d = ctx.dtw_band(Td, Qd, r, starts)
        Xs.append(torch.cat([px, ex]))
        Ys.append(target(d, m))
    return torch.cat(Xs).contiguous(), torch.cat(Ys).contiguous()


def train(ctx, X, Y, epochs: int = 3, batch: int = 4096, lr: float = 1e-3, seed: int = 0, init: bool = True,
          log=None, lr_final: float | None = None):
    """Adam on mean squared error, learning rate decayed linearly from lr to lr_final (default lr / 10)
    over the epochs; returns the per-epoch mean training loss."""
    import torch
    if init:
        ctx.model_init(seed)
    g = torch.Generator(device="cpu").manual_seed(seed)
    n = X.shape[0]
    curve = []
    lr_final = lr / 10 if lr_final is None else lr_final
    for ep in range(epochs):
        lr_ep = lr + (lr_final - lr) * (ep / max(epochs - 1, 1))
        perm = torch.randperm(n, generator=g).to(X.device)
        Xp, Yp = X[perm].contiguous(), Y[perm].contiguous()
        tot, cnt = 0.0, 0
        t0 = time.time()
        for a in range(0, n - batch + 1, batch):
            want = (a // batch) % 16 == 0
            loss = ctx.model_train_step(Xp[a:a + batch], Yp[a:a + batch], lr_ep, want_loss=want)
            if want:
                tot += loss
                cnt += 1
        curve.append(tot / max(cnt, 1))
        if log:
            log(f"epoch {ep}: loss {curve[-1]:.5f} ({time.time() - t0:.2f}s)")
    return curve


def train_default(ctx, n: int = 10_000_000, m: int = 256, frac: float = 0.05, pairs: int = 1_000_000,
                  epochs: int = 12, seed: int = 8, log=None):
    """The default recipe: sinusoid/random-walk mixture of n points (seed 8), queries of length m,
    band floor(frac m), about `pairs` labelled pairs."""
    T = W.sinusoid_mix(n, seed)
    r = int(math.floor(frac * m))
    per_query = n // 1024 + 320
    X, Y = make_pairs(ctx, T, m, r, max(1, pairs // per_query), seed)
    return train(ctx, X, Y, epochs=epochs, seed=seed, log=log)
