"""Seeded synthetic inputs for best-match DTW search.

This module only draws numbers: it holds none of the search arithmetic
(no normalisation, no bounds, no DTW), so that the oracle and the HIP path
can both be fed from it without sharing any of the method's code.

Shapes follow the paper's experiments (Section 4): a float32 random-walk
series (the paper's "Random Walk" data set) and queries that are noisy cuts
of the series or independent walks.  The paper's real data sets (EPG, ECG)
are not available; the sinusoid mixture below stands in for their
quasi-periodic shape.  Every array is a deterministic function of its seed.

All generators return float32 numpy arrays on the host.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

CHUNK = 1 << 24  # points drawn per normal() call when building long walks


def band(m: int, frac: float) -> int:
    """Sakoe-Chiba band in points for a band given as a fraction of the query length."""
    return int(math.floor(frac * m))


def random_walk(n: int, seed: int) -> np.ndarray:
    """Cumulative sum of N(0,1) steps (float64 carried across chunks), cast to float32."""
    rng = np.random.default_rng(seed)
    out = np.empty(n, dtype=np.float32)
    carry = 0.0
    for a in range(0, n, CHUNK):
        b = min(n, a + CHUNK)
        steps = rng.standard_normal(b - a)
        walk = np.cumsum(steps) + carry
        carry = float(walk[-1])
        out[a:b] = walk.astype(np.float32)
    return out


def noisy_cut(T: np.ndarray, start: int, m: int, noise_std: float, seed: int) -> np.ndarray:
    """T[start:start+m] plus N(0, noise_std) noise (noise drawn in float64, result float32)."""
    rng = np.random.default_rng(seed)
    q = T[start:start + m].astype(np.float64) + rng.normal(0.0, noise_std, m)
    return q.astype(np.float32)


def sinusoid_mix(n: int, seed: int, seg: int = 1 << 20, noise_std: float = 0.2) -> np.ndarray:
    """Series of consecutive segments, each a random-walk continuation or a sum of three
    sinusoids (periods log-uniform in [50, 5000], amplitudes U[0.5,2], phases U[0,2pi)),
    level-matched at each seam, plus N(0, noise_std) everywhere."""
    rng = np.random.default_rng(seed)
    out = np.empty(n, dtype=np.float64)
    level = 0.0
    for a in range(0, n, seg):
        b = min(n, a + seg)
        L = b - a
        if rng.random() < 0.5:
            x = np.cumsum(rng.standard_normal(L))
        else:
            t = np.arange(L, dtype=np.float64)
            x = np.zeros(L)
            for _ in range(3):
                period = math.exp(rng.uniform(math.log(50.0), math.log(5000.0)))
                amp = rng.uniform(0.5, 2.0)
                phase = rng.uniform(0.0, 2.0 * math.pi)
                x += amp * np.sin(2.0 * math.pi * t / period + phase)
        out[a:b] = x - x[0] + level
        level = float(out[b - 1])
    out += rng.normal(0.0, noise_std, n)
    return out.astype(np.float32)


@dataclass
class Workload:
    """One series plus a list of queries with their bands."""
    name: str
    T: np.ndarray
    queries: list = field(default_factory=list)   # float32 arrays
    bands: list = field(default_factory=list)     # int r per query
    sources: list = field(default_factory=list)   # start the query was cut at, or -1
    note: str = ""


def single_query_small() -> Workload:
    """Random walk n=262,144 (seed 0); one query T[100000:100128] + N(0,0.1) (seed 1); r=6."""
    T = random_walk(262_144, 0)
    q = noisy_cut(T, 100_000, 128, 0.1, 1)
    return Workload("rw262144_m128_r6", T, [q], [band(128, 0.05)], [100_000],
                    "random walk n=262144, one query m=128, band 5% (6 points)")


def three_queries_large(n: int = 100_000_000) -> Workload:
    """Random walk n=1e8 (seed 0); queries m=128/512/1024 cut at starts drawn from
    default_rng(2) plus N(0,0.1) noise (seeds 3,4,5); bands 5% of m."""
    T = random_walk(n, 0)
    rng = np.random.default_rng(2)
    qs, rs, src = [], [], []
    for k, m in enumerate((128, 512, 1024)):
        s = int(rng.integers(0, n - m))
        qs.append(noisy_cut(T, s, m, 0.1, 3 + k))
        rs.append(band(m, 0.05))
        src.append(s)
    return Workload(f"rw{n}_m128-512-1024_r5pct", T, qs, rs, src,
                    f"random walk n={n}, queries m=128/512/1024, band 5%")


def batched_queries(T: np.ndarray, nq: int = 256, seed: int = 6) -> Workload:
    """nq queries with m ~ U{64..2048} and band fraction ~ U[0, 0.10): the first half cut from
    T at seeded starts plus N(0,0.1) noise, the second half independent random walks."""
    n = T.size
    rng = np.random.default_rng(seed)
    ms = rng.integers(64, 2049, nq)
    fr = rng.uniform(0.0, 0.10, nq)
    qs, rs, src = [], [], []
    for j in range(nq):
        m = int(ms[j])
        if j < nq // 2:
            s = int(rng.integers(0, n - m))
            qs.append(noisy_cut(T, s, m, 0.1, 10_000 + j))
            src.append(s)
        else:
            qs.append(random_walk(m, 1000 + j))
            src.append(-1)
        rs.append(band(m, float(fr[j])))
    return Workload(f"batched{nq}", T, qs, rs, src,
                    f"{nq} queries, m in 64..2048, band 0-10%")


def mixed_queries(T: np.ndarray, nq: int = 64, m: int = 256, seed: int = 9000) -> Workload:
    """nq queries of length m on a sinusoid-mixture series: half cut from T plus N(0,0.1),
    half fresh mixture snippets; band 5%."""
    n = T.size
    rng = np.random.default_rng(seed)
    qs, rs, src = [], [], []
    for j in range(nq):
        if j < nq // 2:
            s = int(rng.integers(0, n - m))
            qs.append(noisy_cut(T, s, m, 0.1, seed + 1 + j))
            src.append(s)
        else:
            qs.append(sinusoid_mix(m, seed + 100 + j, seg=m, noise_std=0.2))
            src.append(-1)
        rs.append(band(m, 0.05))
    return Workload(f"mix{n}_{nq}q_m{m}", T, qs, rs, src, "sinusoid/random-walk mixture")


def tiny_random(n: int, m: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """A short random walk and an independent random-walk query, for exhaustive checks."""
    rng = np.random.default_rng(seed)
    T = np.cumsum(rng.standard_normal(n)).astype(np.float32)
    Q = np.cumsum(rng.standard_normal(m)).astype(np.float32)
    return T, Q


def motif_shapes(m: int = 1024) -> list[np.ndarray]:
    """Ten z-normalised shapes of length m: five random walks (seeds 100..104) and five sums of
    two or three sinusoids and Gaussian bumps (seeds 200..204)."""
    out = []
    for k in range(5):
        out.append(random_walk(m, 100 + k).astype(np.float64))
    t = np.arange(m, dtype=np.float64)
    for k in range(5):
        rng = np.random.default_rng(200 + k)
        x = np.zeros(m)
        for _ in range(int(rng.integers(2, 4))):
            if rng.random() < 0.5:
                x += rng.uniform(0.5, 2.0) * np.sin(2 * math.pi * t / rng.uniform(m / 8, m) + rng.uniform(0, 2 * math.pi))
            else:
                c, w = rng.uniform(0, m), rng.uniform(m / 40, m / 6)
                x += rng.uniform(1.0, 4.0) * np.exp(-0.5 * ((t - c) / w) ** 2)
        out.append(x)
    return [(x - x.mean()) / x.std() for x in out]


def planted_motifs(n: int = 1_000_000_000, m: int = 1024, copies: int = 100, seed: int = 0) -> Workload:
    """Random walk of n points (seed) with copies x 10 planted motifs: shape k = motif_shapes()[k]
    is written at non-overlapping seeded starts p as T[p + j] = T[p] + a S_k[j] + N(0, 0.1),
    a ~ U[0.5, 5].  Queries (128): a_q S_{q mod 10} + N(0, 0.1), band 10% of m.  Workload.src
    holds, per query, the shape index; the plant positions and shapes are in note."""
    shapes = motif_shapes(m)
    T = random_walk(n, seed)
    rng = np.random.default_rng(300)
    total = copies * len(shapes)
    seg = (n - m) // total
    pos = np.arange(total, dtype=np.int64) * seg + rng.integers(0, seg - m, total)
    kind = rng.permutation(np.repeat(np.arange(len(shapes)), copies))
    amp = rng.uniform(0.5, 5.0, total)
    for p, k, a in zip(pos, kind, amp):
        noise = rng.normal(0.0, 0.1, m)
        T[p:p + m] = (float(T[p]) + a * shapes[k] + noise).astype(np.float32)
    qrng = np.random.default_rng(500)
    qs, rs, src = [], [], []
    for q in range(128):
        a = qrng.uniform(0.5, 5.0)
        qs.append((a * shapes[q % 10] + np.random.default_rng(400 + q).normal(0.0, 0.1, m)).astype(np.float32))
        rs.append(band(m, 0.10))
        src.append(q % 10)
    wl = Workload(f"motifs{n}_128q_m{m}", T, qs, rs, src, {"positions": pos, "shapes": kind})
    return wl
