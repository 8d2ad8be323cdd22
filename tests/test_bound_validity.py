"""The bound the GPU path adds to the paper's early abandoning of DTW is a lower bound of the banded
DTW distance (eq. (dtw) with the band of Section 2.1), checked here in FP64 against the oracle's DTW
on random and adversarial small inputs: after column j of the DP over the candidate, the band
minimum of that column plus the query-envelope LB_Keogh terms (eq. (LBKeoghEC)) of the later
columns.  This checks the mathematics the lane DTW kernels rely on; the kernels themselves are
covered by the GPU parity tests, which would miss matches if the bound overshot."""
import numpy as np

from oracle import reference as R


def dp_columns(q, c, r):
    """Banded DP swept over the candidate index j (the GPU's column order): column j holds
    D(i, j) for every query index i (inf outside the band)."""
    m = len(q)
    D = np.full((m, m), np.inf)
    for j in range(m):
        for i in range(max(0, j - r), min(m, j + r + 1)):
            best = 0.0 if i == 0 and j == 0 else min(
                D[i - 1, j - 1] if i and j else np.inf, D[i, j - 1] if j else np.inf, D[i - 1, j] if i else np.inf)
            D[i, j] = (q[i] - c[j]) ** 2 + best
    return D


def cases(seed, count):
    rng = np.random.default_rng(seed)
    for k in range(count):
        m = int(rng.integers(6, 40))
        r = int(rng.integers(0, m))
        kind = k % 3
        if kind == 0:
            q, c = rng.normal(size=m), rng.normal(size=m)
        elif kind == 1:                       # near-identical: the bounds are nearly tight
            q = np.cumsum(rng.normal(size=m))
            c = q + rng.normal(scale=1e-3, size=m)
        else:                                 # a shifted copy (warping pays off)
            base = np.cumsum(rng.normal(size=m + 3))
            q, c = base[:m], base[3:]
        yield R.znorm(q), R.znorm(c), r


def test_suffix_bound_after_every_column():
    for q, c, r in cases(8, 300):
        m = len(q)
        d = R.dtw(q, c, r)
        U, L = R.envelope(q, r)
        terms = np.maximum(c - U, 0.0) ** 2 + np.maximum(L - c, 0.0) ** 2
        D = dp_columns(q, c, r)
        assert abs(D[m - 1, m - 1] - d) <= 1e-9 * max(d, 1.0)
        for j in range(m):
            lb = D[:, j].min() + terms[j + 1:].sum()
            assert lb <= d * (1 + 1e-12) + 1e-12, (m, r, j, lb, d)


def test_the_check_catches_an_overshooting_bound():
    """Counting column j's own term as well (off by one) overshoots DTW on some case, and the check
    above would fail on it."""
    bad = 0
    for q, c, r in cases(9, 200):
        U, L = R.envelope(q, r)
        terms = np.maximum(c - U, 0.0) ** 2 + np.maximum(L - c, 0.0) ** 2
        D = dp_columns(q, c, r)
        d = R.dtw(q, c, r)
        bad += any(D[:, j].min() + terms[j:].sum() > d * (1 + 1e-9) + 1e-9 for j in range(len(q)))
    assert bad > 0
