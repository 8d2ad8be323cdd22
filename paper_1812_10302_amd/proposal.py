"""Training recipes of the learned block ordering.

The training itself runs in the library (Context.model_train -> dtws_model_train): query
generation, the candidates (the proposals the learned order scores, near-source and random
starts), the exact DTW labels, the target log(DTW / m + 1e-4), shuffling and the Adam epochs are
HIP kernels.  This module only uploads a training series and picks the recipe's numbers.
"""
from __future__ import annotations

import math

import numpy as np

from . import workloads as W

TARGET_EPS = 1e-4


def rows_per_query(n: int, block: int = 4096, random: int = 256, near: int = 32) -> int:
    """Pairs one training query yields on a series of n points (upper bound): one proposal per
    quarter block plus the extra candidates."""
    return 4 * -(-n // block) + random + 2 * near


def _device_series(ctx, T):
    import torch
    if isinstance(T, np.ndarray):
        return torch.from_numpy(np.ascontiguousarray(T, dtype=np.float32)).to(torch.device("cuda", ctx.device))
    return T


def train(ctx, T_train, shapes, queries_per_shape: int = 24, epochs: int = 12, seed: int = 90, log=None, **kw):
    """Train the ordering network on a training series (numpy array or float32 CUDA tensor) for the
    given (m, r) shapes, with the context's current block.  Returns (per-epoch mean loss, pairs)."""
    Td = _device_series(ctx, T_train)
    curve, pairs = ctx.model_train(Td, shapes, queries_per_shape, epochs, seed=seed, **kw)
    if log:
        for ep, v in enumerate(curve):
            log(f"epoch {ep}: loss {v:.5f}")
    return curve, pairs


def queries_for_pairs(n: int, pairs: int, shapes: int = 1, block: int = 4096) -> int:
    """Training queries per shape that give about `pairs` pairs in all on a series of n points."""
    return max(1, pairs // (rows_per_query(n, block) * shapes))


def train_default(ctx, n: int = 10_000_000, m: int = 256, frac: float = 0.05, pairs: int = 1_000_000,
                  epochs: int = 12, seed: int = 8, log=None):
    """The default recipe: sinusoid/random-walk mixture of n points (seed 8), queries of length m,
    band floor(frac m), about `pairs` labelled pairs."""
    T = W.sinusoid_mix(n, seed)
    r = int(math.floor(frac * m))
    block = ctx.get_schedule()["block"]
    return train(ctx, T, [(m, r)], queries_for_pairs(n, pairs, 1, block), epochs, seed, log)
