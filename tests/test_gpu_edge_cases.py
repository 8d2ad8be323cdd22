"""Degenerate inputs through the C ABI, against the CPU oracle: flat stretches in the series, flat
queries (population sigma <= 1e-8 normalises to all zeros, the reading the oracle takes for the
case eq. (Normalization1) leaves open), many exact ties, and near-best or survivor lists that
overflow.

A list that overflows must never give a wrong index: the plain search scans the series again in
list-sized chunks under the final best-so-far and certifies each chunk, and the batched search hands
the affected queries to the plain search.  The list capacity is lowered through the schedule to
reach those paths at small sizes; one test reaches the full-size near-best limit (2^20 entries)
with a flat stretch of 1.2 million windows.

Where several starts share the minimum FP64 distance (exact ties), the answer is the lowest of them,
which both sides compute exactly.  A flat query against a series without flat windows ties every
candidate at distance m up to rounding, so there only the distance and the validity of the index
are compared.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1812_10302_amd as dtws
from paper_1812_10302_amd import workloads as W
from oracle import reference as R
from oracle import Cascade

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


@pytest.fixture(scope="module")
def ctx():
    c = dtws.Context(0, max_n=2_000_000, max_m=512, max_queries=8)
    yield c
    c.close()


@pytest.fixture(scope="module")
def casc():
    return Cascade()


@pytest.fixture
def small_lists(ctx):
    """Near-best and survivor lists cut to 64 entries for the duration of a test."""
    keep = ctx.get_schedule()
    ctx.set_schedule(list_cap=64)
    yield
    ctx.set_schedule(**keep)


def flat_series(n=60_000, seed=61):
    T = W.random_walk(n, seed)
    T[10_000:10_700] = np.float32(4.5)       # 700 points: 700 - m + 1 flat windows
    T[40_000:40_300] = np.float32(-2.0)
    return T


def exact(got, ref):
    assert got[0] == ref[0], (got, ref)
    assert abs(got[1] - ref[1]) <= 1e-9 * ref[1] + 1e-12, (got, ref)


@pytest.mark.parametrize("m,r", [(64, 3), (200, 20)])
def test_series_with_flat_stretches(ctx, casc, m, r):
    T = flat_series()
    Q = W.noisy_cut(T, 25_000, m, 0.1, 62)
    ref = R.best_match(T, Q, r)
    print(f"flat-stretch series, m={m} r={r}: oracle {ref}", flush=True)
    exact(ctx.search(dev(T), dev(Q), r, seed=1), ref)
    exact(ctx.search_batch(dev(T), dtws.PackedQueries([dev(Q)]), [r])[0], ref)
    # a query that is itself a cut across the start of a flat stretch
    Q2 = W.noisy_cut(T, 10_700 - m // 2, m, 0.05, 63)
    ref2 = casc.search(T, Q2, r)[:2]
    exact(ctx.search(dev(T), dev(Q2), r, seed=2), ref2)


@pytest.mark.parametrize("m,r", [(64, 3), (128, 0), (300, 30)])
def test_flat_query_finds_lowest_flat_window(ctx, casc, m, r):
    """A flat query normalises to zeros; a flat window does too, so its distance is exactly 0 and the
    answer is the lowest flat window (the first of the 10_000 stretch)."""
    T = flat_series()
    Q = np.full(m, 3.0, np.float32)
    ref = casc.search(T, Q, r)[:2]
    assert ref == (10_000, 0.0)
    exact(ctx.search(dev(T), dev(Q), r, seed=3), ref)
    got = ctx.search_batch(dev(T), dtws.PackedQueries([dev(Q), dev(W.noisy_cut(T, 3_000, m, 0.1, 64))]), [r, r])
    exact(got[0], ref)
    exact(got[1], casc.search(T, W.noisy_cut(T, 3_000, m, 0.1, 64), r)[:2])


def test_flat_query_without_flat_windows(ctx, casc):
    """Every candidate then lies at distance m (each column of the DP is visited once, by the
    diagonal path, and the normalised candidate has squared norm m): the minimum is m up to
    rounding and the returned start must be a valid one at that distance."""
    T = W.random_walk(30_000, 65)
    m, r = 96, 5
    Q = np.full(m, -1.25, np.float32)
    i, d = ctx.search(dev(T), dev(Q), r, seed=4)
    assert 0 <= i <= T.size - m
    assert d == pytest.approx(m, rel=1e-9)
    assert casc.dtw_starts(T, Q, r, np.array([i]))[0] == pytest.approx(d, rel=1e-12)


@pytest.mark.parametrize("order", ["natural", "random"])
def test_exact_ties_overflow_near_best_list(ctx, casc, small_lists, order):
    """A periodic series repeats every window exactly every 100 points, so the best distance is
    shared by hundreds of identical windows: far more than the 64-entry near-best list holds.  The
    plain search recovers by chunked re-certification and returns the lowest of them."""
    base = W.random_walk(100, 66)
    T = np.tile(base, 600).astype(np.float32)
    m, r = 64, 4
    Q = W.noisy_cut(T, 1_234, m, 0.05, 67)
    ref = casc.search(T, Q, r)[:2]
    assert ref[0] < 100          # the lowest copy of the tie class
    print(f"periodic series: oracle {ref}", flush=True)
    flags = dtws.ORDER_NATURAL if order == "natural" else dtws.ORDER_RANDOM
    exact(ctx.search(dev(T), dev(Q), r, flags=flags, seed=5), ref)
    assert ctx.counters()["certified"] > 64


def test_batched_survivor_overflow_falls_back(ctx, casc, small_lists):
    """With 64 survivor slots the batched cascade overflows at once; every query of the batch must
    still come back with the oracle's answer (through the plain search)."""
    T = flat_series(40_000, 68)
    qs = [W.noisy_cut(T, s, m, 0.1, 69 + k) for k, (s, m) in enumerate(((1_000, 64), (22_000, 128), (35_000, 64)))]
    rs = [3, 12, 0]
    got = ctx.search_batch(dev(T), dtws.PackedQueries([dev(q) for q in qs]), rs)
    for g, q, r in zip(got, qs, rs):
        exact(g, casc.search(T, q, r)[:2])


def test_flat_stretch_beyond_full_near_best_list(ctx, casc):
    """1.2 million windows of one flat stretch against a flat query: every one of them is an exact
    tie at distance 0, more than the full 2^20-entry near-best list.  The answer is the stretch's
    first window."""
    n, m, r = 1_500_000, 16, 2
    T = W.random_walk(n, 70)
    T[200_000:200_000 + 1_200_000 + m - 1] = np.float32(-7.0)
    Q = np.full(m, 0.5, np.float32)
    ref = casc.search(T, Q, r)[:2]
    assert ref == (200_000, 0.0)
    exact(ctx.search(dev(T), dev(Q), r, seed=6), ref)
    exact(ctx.search_batch(dev(T), dtws.PackedQueries([dev(Q)]), [r])[0], ref)
