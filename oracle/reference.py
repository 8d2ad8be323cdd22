"""FP64 NumPy oracle for best-match subsequence search under banded DTW.

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module; the search library
never does, and this module imports nothing from the library.

Every function follows a definition of Kraeva & Zymbler, "The Use of MPI and
OpenMP Technologies for Subsequence Similarity Search in Very Large Time
Series ..." (arXiv:1812.10302), Section 2 (problem statement) and Section 3.1
(fragmentation).  Notation: the series T has length n, the query Q length m
(the paper swaps the two letters between its definitions), the band is r
points, and candidate starts are 0-based, i in [0, n-m].

Readings taken where the paper is silent or garbled (each also listed in the
design notes):
  * band (Section 2.1 prose): cell (i, j) is inside iff |i - j| <= r;
    r >= m-1 is unconstrained DTW.
  * z-normalisation (eq. Normalization1): population sigma, computed two-pass
    (mean first, then mean squared deviation) - mathematically the paper's
    E[t^2] - mu^2, numerically stable.  A window whose sigma <= SIGMA_FLAT is
    flat and normalises to all zeros.
  * LB_KimFL (eq. LB_Kim) uses squared differences of the first and of the
    last pair; the unsquared form printed is not a bound of squared DTW.
  * envelope windows (eq. envelope) are clipped to the sequence.
  * LB_Keogh names: the paper's "EC" bound compares the candidate with the
    query envelope (here lb_keogh_q), its "EQ" bound the query with the
    candidate envelope (here lb_keogh_d).
  * ties between equal distances resolve to the lowest start index.
"""
from __future__ import annotations

import itertools

import numpy as np

SIGMA_FLAT = 1e-8


# ---------------------------------------------------------------- normalisation
def znorm(x) -> np.ndarray:
    """eq. (Normalization1): t_hat = (t - mu) / sigma, population sigma, two-pass."""
    x = np.asarray(x, dtype=np.float64)
    mu = x.mean()
    dev = x - mu
    sigma = np.sqrt((dev * dev).mean())
    if sigma <= SIGMA_FLAT:
        return np.zeros_like(x)
    return dev / sigma


def window_stats(T, m: int) -> tuple[np.ndarray, np.ndarray]:
    """Two-pass mean and population sigma of every length-m window of T (FP64)."""
    W = np.lib.stride_tricks.sliding_window_view(np.asarray(T, dtype=np.float64), m)
    mu = W.mean(axis=1)
    dev = W - mu[:, None]
    sigma = np.sqrt((dev * dev).mean(axis=1))
    return mu, sigma


def normalized_windows(T, m: int, starts) -> np.ndarray:
    """z-normalised candidates T[i:i+m] for the given starts, shape (len(starts), m)."""
    T = np.asarray(T, dtype=np.float64)
    starts = np.asarray(starts, dtype=np.int64)
    W = T[starts[:, None] + np.arange(m)[None, :]]
    mu = W.mean(axis=1, keepdims=True)
    dev = W - mu
    sigma = np.sqrt((dev * dev).mean(axis=1, keepdims=True))
    flat = sigma[:, 0] <= SIGMA_FLAT
    out = np.where(flat[:, None], 0.0, dev / np.where(flat[:, None], 1.0, sigma))
    return out


# ---------------------------------------------------------------------- DTW
def dtw(x, y, r: int) -> float:
    """eq. (dtw) with the Sakoe-Chiba band of Section 2.1, written with the paper's 1-based d:
    d(0,0)=0, d(i,0)=d(0,j)=inf, d(i,j) = (x_i-y_j)^2 + min(d(i-1,j), d(i,j-1), d(i-1,j-1)),
    and d(i,j)=inf for |i-j| > r.  Returns d(m,m)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    m = x.size
    assert y.size == m
    r = max(0, min(int(r), m - 1))
    d = np.full((m + 1, m + 1), np.inf)
    d[0, 0] = 0.0
    for i in range(1, m + 1):
        for j in range(max(1, i - r), min(m, i + r) + 1):
            cost = (x[i - 1] - y[j - 1]) ** 2
            d[i, j] = cost + min(d[i - 1, j], d[i, j - 1], d[i - 1, j - 1])
    return float(d[m, m])


def dtw_many(xhat, C, r: int) -> np.ndarray:
    """The same recurrence as dtw(), evaluated for many second operands at once.
    C has shape (m, B): column b is one candidate.  Returns B distances."""
    x = np.asarray(xhat, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    m, B = C.shape
    assert x.size == m
    r = max(0, min(int(r), m - 1))
    prev = np.full((m + 1, B), np.inf)   # row i-1 of d, indexed by j
    prev[0, :] = 0.0
    cur = np.empty_like(prev)
    for i in range(1, m + 1):
        cur.fill(np.inf)
        for j in range(max(1, i - r), min(m, i + r) + 1):
            cost = (x[i - 1] - C[j - 1]) ** 2
            cur[j] = cost + np.minimum(np.minimum(prev[j], cur[j - 1]), prev[j - 1])
        prev, cur = cur, prev
    return prev[m].copy()


def dtw_allpaths(x, y, r: int) -> float:
    """Minimum cost over every warping path (Section 2.1): a sequence of cells from (0,0) to
    (m-1,m-1), each step to an adjacent cell (i+1,j), (i,j+1) or (i+1,j+1), every cell inside
    the band.  Exhaustive enumeration; only for tiny m."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    m = x.size
    best = np.inf

    def walk(i, j, acc):
        nonlocal best
        acc = acc + (x[i] - y[j]) ** 2
        if i == m - 1 and j == m - 1:
            best = min(best, acc)
            return
        for di, dj in ((1, 0), (0, 1), (1, 1)):
            a, b = i + di, j + dj
            if a < m and b < m and abs(a - b) <= r:
                walk(a, b, acc)

    walk(0, 0, 0.0)
    return float(best)


# ------------------------------------------------------------- lower bounds
def envelope(x, r: int) -> tuple[np.ndarray, np.ndarray]:
    """eq. (envelope): u_i = max(x_{i-r..i+r}), l_i = min(...), windows clipped to the sequence."""
    x = np.asarray(x, dtype=np.float64)
    m = x.size
    U = np.empty(m)
    L = np.empty(m)
    for i in range(m):
        a, b = max(0, i - r), min(m, i + r + 1)
        U[i] = x[a:b].max()
        L[i] = x[a:b].min()
    return U, L


def lb_kim_fl(qhat, chat) -> float:
    """eq. (LB_Kim), read with squared differences: first pair plus last pair."""
    q = np.asarray(qhat, dtype=np.float64)
    c = np.asarray(chat, dtype=np.float64)
    if q.size == 1:
        return float((q[0] - c[0]) ** 2)
    return float((q[0] - c[0]) ** 2 + (q[-1] - c[-1]) ** 2)


def lb_keogh(x, U, L) -> float:
    """eq. (LBKeoghEC): sum of squared excursions of x outside the envelope [L, U]."""
    x = np.asarray(x, dtype=np.float64)
    above = np.where(x > U, (x - U) ** 2, 0.0)
    below = np.where(x < L, (x - L) ** 2, 0.0)
    return float((above + below).sum())


def lb_keogh_q(qhat, chat, r: int) -> float:
    """The paper's LB_Keogh EC: the candidate against the query envelope."""
    U, L = envelope(qhat, r)
    return lb_keogh(chat, U, L)


def lb_keogh_d(qhat, chat, r: int) -> float:
    """The paper's LB_Keogh EQ (roles swapped): the query against the candidate envelope,
    the envelope taken over the candidate alone."""
    U, L = envelope(chat, r)
    return lb_keogh(qhat, U, L)


def series_envelope(T, r: int) -> tuple[np.ndarray, np.ndarray]:
    """Envelope of the raw series: max/min of T over [k-r, k+r] clipped to [0, n)."""
    return envelope(T, r)


def lb_keogh_d_series(T, i: int, m: int, r: int, qhat) -> float:
    """Query against the series-level envelope of the raw series, mapped through candidate i's
    normalisation.  A candidate's own envelope is contained in this one (its windows are
    subsets), so this bound is looser than lb_keogh_d and still a lower bound of DTW."""
    T = np.asarray(T, dtype=np.float64)
    n = T.size
    seg = T[max(0, i - r):min(n, i + m + r)]
    off = i - max(0, i - r)
    U, L = envelope(seg, r)
    U, L = U[off:off + m], L[off:off + m]
    w = T[i:i + m]
    mu = w.mean()
    sigma = np.sqrt(((w - mu) ** 2).mean())
    if sigma <= SIGMA_FLAT:
        Un, Ln = np.zeros(m), np.zeros(m)
    else:
        Un, Ln = (U - mu) / sigma, (L - mu) / sigma
    return lb_keogh(qhat, Un, Ln)


# ------------------------------------------------------------- best match
def all_distances(T, Q, r: int, chunk: int = 8192) -> np.ndarray:
    """DTW(Q_hat, C_hat_i) for every start i in [0, n-m] (the quantity minimised in the
    best-match definition, Section 2.1)."""
    T = np.asarray(T, dtype=np.float64)
    m = len(Q)
    N = T.size - m + 1
    qh = znorm(Q)
    out = np.empty(N)
    for a in range(0, N, chunk):
        b = min(N, a + chunk)
        C = normalized_windows(T, m, np.arange(a, b)).T
        out[a:b] = dtw_many(qh, C, r)
    return out


def best_match(T, Q, r: int, chunk: int = 8192) -> tuple[int, float]:
    """Best match (Section 2.1): the start i minimising DTW(Q_hat, C_hat_i); lowest i on ties."""
    D = all_distances(T, Q, r, chunk)
    i = int(np.argmin(D))          # argmin returns the first minimum: lowest index
    return i, float(D[i])


def distances_at(T, Q, r: int, starts) -> np.ndarray:
    """DTW of the normalised query against the normalised candidates at the given starts."""
    starts = np.asarray(starts, dtype=np.int64)
    m = len(Q)
    C = normalized_windows(T, m, starts).T
    return dtw_many(znorm(Q), C, r)


# ------------------------------------------------------------- fragmentation
def fragments(N: int, F: int, m: int) -> list[tuple[int, int]]:
    """eq. (OverlapPartitioning), 0-based: fragment k starts at k*floor(N/F) and holds
    floor(N/F) + m - 1 points, the last one also the N mod F remainder."""
    base = N // F
    out = []
    for k in range(F):
        start = k * base
        length = base + m - 1 + (N % F if k == F - 1 else 0)
        out.append((start, length))
    return out


def best_match_fragmented(T, Q, r: int, F: int) -> tuple[int, float]:
    """Best match computed fragment by fragment and reduced by minimum distance, lowest global
    index on ties (the reduction of Algorithm 1 over fragments)."""
    T = np.asarray(T)
    m = len(Q)
    N = T.size - m + 1
    best = (np.inf, -1)
    for start, length in fragments(N, F, m):
        i, d = best_match(T[start:start + length], Q, r)
        cand = (d, start + i)
        if cand < best:
            best = cand
    return best[1], best[0]


def warping_path_count(m: int, r: int) -> int:
    """Number of warping paths on an m x m grid inside the band (for documenting tests)."""
    count = {(0, 0): 1}
    for s in range(1, 2 * m - 1):
        for i, j in itertools.product(range(m), range(m)):
            if i + j != s or abs(i - j) > r:
                continue
            count[(i, j)] = (count.get((i - 1, j), 0) + count.get((i, j - 1), 0)
                             + count.get((i - 1, j - 1), 0))
    return count.get((m - 1, m - 1), 0)
