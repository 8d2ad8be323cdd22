"""FP64 reference of the learned block-ordering model.

TEST INFRASTRUCTURE (see the package docstring).

The model is not part of the paper's method: it only orders the work, while the exact lower
bounds and exact DTW decide every result.  Its inputs are Piecewise Aggregate Approximations
(PAA): the means of 16 consecutive segments of the z-normalised query and of the z-normalised
candidate, segment s covering positions [floor(s*m/16), floor((s+1)*m/16)).

Network: y = w3 . relu(W2^T relu(W1^T x + b1) + b2) + b3 + log(d(x) / 16 + 1e-4) with x in R^32
(query PAA, then candidate PAA), hidden widths 256 and 256, and d(x) = sum_t (x_t - x_{t+16})^2 the
squared distance of the two PAAs: the network learns a correction to the logarithm of the PAA
distance (a model with a zero output layer orders exactly as the PAA distance does).  Loss: mean squared error against given targets (the
training recipe uses log(DTW / m + 1e-4)).  Parameters are kept as one flat FP32 vector in the order
W1 (32 x 256, row = input), b1 (256), W2 (256 x 256, row = layer-1 unit), b2 (256), w3 (256), b3 (1).

With bf16=True the reference rounds to bfloat16 exactly where the GPU kernels do: the inputs x,
W1 and W2, the layer-1 activations before layer 2, and the back-propagated pre-activation
gradients before they enter a matrix product.  Everything else is FP64.
"""
from __future__ import annotations

import numpy as np

D_IN, H1, H2 = 32, 256, 256
SHAPES = [("W1", (D_IN, H1)), ("b1", (H1,)), ("W2", (H1, H2)), ("b2", (H2,)), ("w3", (H2,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unflatten(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, k = {}, 0
    for name, shape in SHAPES:
        size = int(np.prod(shape))
        out[name] = theta[k:k + size].reshape(shape)
        k += size
    return out


def flatten(p) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def bf16(x) -> np.ndarray:
    """Round to bfloat16 (round to nearest, ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    r = np.where(np.isnan(f), u, r)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _q(x, on):
    return bf16(x) if on else np.asarray(x, dtype=np.float64)


def paa(xhat, segments: int = 16) -> np.ndarray:
    """Segment means of a normalised sequence."""
    x = np.asarray(xhat, dtype=np.float64)
    m = x.size
    b = [(s * m) // segments for s in range(segments + 1)]
    return np.array([x[b[s]:b[s + 1]].mean() for s in range(segments)])


def proposals(T, Q, block: int = 4096, quarters: int = 4):
    """The candidates the learned order scores: the candidates 0 .. n-m are cut into quarter blocks
    of block/quarters starts; within each, every ps-th start (ps = m // 64 for m >= 128, else 1)
    is compared with the query by the squared Euclidean distance of their PAAs (both windows
    z-normalised, flat ones to zero), and the nearest is proposed, the lowest start on ties.
    Returns (starts, distances) per quarter; -1 / inf past the last candidate."""
    from .reference import normalized_windows, znorm
    T = np.asarray(T, dtype=np.float64)
    m = len(Q)
    N = T.size - m + 1
    ps = m // 64 if m >= 128 else 1
    qp = paa(znorm(Q))
    quarter = block // quarters
    rows = -(-N // block) * quarters
    starts = np.full(rows, -1, dtype=np.int64)
    dists = np.full(rows, np.inf)
    for k in range(rows):
        lo, hi = k * quarter, min((k + 1) * quarter, N)
        if lo >= hi:
            continue
        cand = np.arange(lo, hi, ps)
        C = normalized_windows(T, m, cand)
        F = np.stack([C[:, (t * m) // 16:((t + 1) * m) // 16].mean(axis=1) for t in range(16)], axis=1)
        d = ((F - qp) ** 2).sum(axis=1)
        j = int(np.argmin(d))
        starts[k], dists[k] = cand[j], d[j]
    return starts, dists


def paa_skip(X) -> np.ndarray:
    """log(d / 16 + 1e-4) per row, d = squared distance of the query half to the candidate half."""
    X = np.asarray(X, dtype=np.float64)
    d = ((X[:, :16] - X[:, 16:]) ** 2).sum(axis=1)
    return np.log(d / 16.0 + 1e-4)


def forward(theta, X, bf16_ops: bool = False):
    """Returns (y, cache) for inputs X of shape (R, 32)."""
    p = unflatten(theta)
    Xq = _q(X, bf16_ops)
    A1 = Xq @ _q(p["W1"], bf16_ops) + p["b1"]
    Hl1 = np.maximum(A1, 0.0)
    Hq = _q(Hl1, bf16_ops)
    A2 = Hq @ _q(p["W2"], bf16_ops) + p["b2"]
    Hl2 = np.maximum(A2, 0.0)
    y = Hl2 @ p["w3"] + p["b3"][0] + paa_skip(X)
    return y, (Xq, A1, Hq, A2, Hl2, p)


def loss_and_grads(theta, X, target, bf16_ops: bool = False):
    """Mean squared error and its gradient with respect to the flat parameter vector."""
    y, (Xq, A1, Hq, A2, Hl2, p) = forward(theta, X, bf16_ops)
    R = X.shape[0]
    diff = y - np.asarray(target, dtype=np.float64)
    loss = float(np.mean(diff ** 2))
    dy = 2.0 * diff / R
    g = {"w3": Hl2.T @ dy, "b3": np.array([dy.sum()])}
    dA2 = np.outer(dy, p["w3"]) * (A2 > 0)
    g["b2"] = dA2.sum(axis=0)
    dA2q = _q(dA2, bf16_ops)
    g["W2"] = Hq.T @ dA2q
    dH1 = dA2q @ _q(p["W2"], bf16_ops).T
    dA1 = dH1 * (A1 > 0)
    g["b1"] = dA1.sum(axis=0)
    g["W1"] = Xq.T @ _q(dA1, bf16_ops)
    return loss, flatten(g)


def adam(theta, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, 2015) with bias correction; returns (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed: int) -> np.ndarray:
    """He-normal weights, zero biases (reference initialisation for CPU tests)."""
    rng = np.random.default_rng(seed)
    p = {"W1": rng.normal(0, np.sqrt(2 / D_IN), (D_IN, H1)), "b1": np.zeros(H1),
         "W2": rng.normal(0, np.sqrt(2 / H1), (H1, H2)), "b2": np.zeros(H2),
         "w3": rng.normal(0, np.sqrt(1 / H2), H2), "b3": np.zeros(1)}
    return flatten(p)
