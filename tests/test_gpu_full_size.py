"""Parity at the full workload sizes, through the C ABI, in the configuration the benchmark times.

The FP64 cascade oracle (oracle/cascade.c, all host threads) gives the exact answer of a seeded
subset of every workload's queries; the other queries are checked by properties that hold at any
size, computed by the oracle one candidate at a time: the returned distance is the FP64 DTW at the
returned start, and no other candidate examined (the query's source position, seeded random
starts) is better.  Parity is claimed only for the oracle-checked queries.

  * random walk n = 1e8, queries m = 128/512/1024 (5% band): all three exact, for the plain
    (series order and LB-sorted order), batched (series order) and learned-order paths;
  * the same series, 256 queries m ~ U{64..2048}, band 0-10%: 16 exact (every r = 0 query up to
    four, the longest and the widest-band noisy cut, the rest seeded among m <= 1024), properties
    for all, learned order = series order;
  * sinusoid/random-walk mixture n = 1e8, 64 queries m = 256 (r = 12): 8 exact (four cuts, four
    fresh snippets), properties for all;
  * random walk n = 1e9 with 1000 planted motifs, 128 queries m = 1024 (r = 102): 4 exact, of four
    different shapes, properties for all, and the answers are reported against the planted
    positions of each query's shape.
"""
import math
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1812_10302_amd as dtws
from paper_1812_10302_amd import proposal
from paper_1812_10302_amd import workloads as W
from oracle import Cascade

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


@pytest.fixture(scope="module")
def casc():
    return Cascade()


@pytest.fixture(scope="module")
def rw():
    wl = W.three_queries_large(100_000_000)
    return wl, dev(wl.T)


@pytest.fixture(scope="module")
def ctx():
    c = dtws.Context(0, max_n=100_000_000, max_m=2048, max_queries=256)
    yield c
    c.close()


def train_order(ctx, T_train, shapes, queries_per_shape=24, epochs=12, seed=90):
    curve, pairs = proposal.train(ctx, T_train, shapes, queries_per_shape, epochs, seed)
    print(f"ordering network: {pairs} pairs, loss {curve[0]:.4f} -> {curve[-1]:.4f}", flush=True)


def check_properties(casc, T, queries, rs, got, sources=None, samples=64, seed=0):
    """got[k] = (index, distance) must be the FP64 DTW at that start, and no better than any
    sampled start or the query's source (ties: the returned start is the lowest)."""
    rng = np.random.default_rng(seed)
    for k, (q, r) in enumerate(zip(queries, rs)):
        i, d = got[k]
        N = T.size - q.size + 1
        at = casc.dtw_starts(T, q, r, np.array([i]))[0]
        assert abs(at - d) <= 1e-9 * max(d, 1e-300), (k, i, d, at)
        starts = rng.integers(0, N, samples)
        if sources is not None and sources[k] >= 0:
            s = sources[k]
            starts = np.concatenate([starts, np.arange(max(0, s - 3), min(N, s + 4))])
        dd = casc.dtw_starts(T, q, r, starts)
        assert np.all(dd >= d * (1 - 1e-12)), (k, d, float(dd.min()))
        tie = dd == d
        assert np.all(starts[tie] >= i), (k, i, starts[tie])


def say(*a):
    print(*a, flush=True)


def oracle_each(casc, T, queries, rs, label):
    """Oracle answers one query at a time, with a progress line per query."""
    out = []
    for k, (q, r) in enumerate(zip(queries, rs)):
        t0 = time.time()
        out.append(casc.search(T, q, r)[:2])
        say(f"{label}: oracle query {k} (m={q.size}, r={r}) {out[-1]} in {time.time() - t0:.1f}s")
    return out


def check_exact(got, ref):
    assert len(got) == len(ref)
    for k, ((gi, gd), (ri, rd)) in enumerate(zip(got, ref)):
        assert gi == ri, (k, gi, ri, gd, rd)
        assert abs(gd - rd) <= 1e-9 * rd + 1e-12, (k, gd, rd)


def test_random_walk_1e8_three_queries_exact(ctx, rw, casc):
    wl, Td = rw
    ref = oracle_each(casc, wl.T, wl.queries, wl.bands, "1e8 three queries")
    Qd = [dev(q) for q in wl.queries]
    plain = [ctx.search(Td, q, r, seed=7) for q, r in zip(Qd, wl.bands)]
    check_exact(plain, ref)
    check_exact([ctx.search(Td, q, r, flags=dtws.LB_SORTED, seed=7) for q, r in zip(Qd, wl.bands)], ref)
    pq = dtws.PackedQueries(Qd)
    check_exact(ctx.search_batch(Td, pq, wl.bands), ref)
    train_order(ctx, W.random_walk(10_000_000, 8), list(zip([q.size for q in wl.queries], wl.bands)))
    check_exact(ctx.search_batch(Td, pq, wl.bands, flags=dtws.ORDER_LEARNED, seed=7), ref)


def c3_subset(b, count=16, seed=66):
    """Seeded, stratified subset of the 256 mixed queries: the r = 0 queries (up to four), the
    longest and the widest-band query among the noisy cuts (the first half), then seeded picks of
    queries with m <= 1024 until `count` (the oracle's time grows with m; the largest m and r are
    already in)."""
    nq = len(b.queries)
    ms = np.array([q.size for q in b.queries])
    rs = np.array(b.bands)
    cut = np.arange(nq) < nq // 2
    pick = [int(k) for k in np.flatnonzero(rs == 0)[:4]]
    for k in (int(np.argmax(np.where(cut, ms, 0))), int(np.argmax(np.where(cut, rs, -1)))):
        if k not in pick:
            pick.append(k)
    rng = np.random.default_rng(seed)
    for k in rng.permutation(nq):
        if len(pick) >= count:
            break
        if int(k) not in pick and ms[k] <= 1024:
            pick.append(int(k))
    return sorted(pick)


def test_random_walk_1e8_256_mixed_queries(ctx, rw, casc):
    wl, Td = rw
    b = W.batched_queries(wl.T, 256, seed=6)
    pq = dtws.PackedQueries([dev(q) for q in b.queries])
    t0 = time.time()
    natural = ctx.search_batch(Td, pq, b.bands)
    say(f"256 mixed queries: batched, series order, {time.time() - t0:.2f}s")
    train_order(ctx, W.random_walk(10_000_000, 8), [(128, 6), (512, 25), (1024, 51), (2048, 102)],
                queries_per_shape=12, epochs=8)
    learned = ctx.search_batch(Td, pq, b.bands, flags=dtws.ORDER_LEARNED, seed=3)
    assert learned == natural
    say("256 mixed queries: learned order = series order")
    check_properties(casc, wl.T, b.queries, b.bands, natural, b.sources, samples=32, seed=1)
    say("256 mixed queries: properties hold")
    sub = c3_subset(b)
    assert len(sub) == 16 and any(b.bands[k] == 0 for k in sub)
    ref = oracle_each(casc, wl.T, [b.queries[k] for k in sub], [b.bands[k] for k in sub], "256 mixed queries")
    check_exact([natural[k] for k in sub], ref)
    for k in (0, 200):
        check_exact([ctx.search(Td, dev(b.queries[k]), b.bands[k], seed=5)], [natural[k]])


def test_mixture_1e8_64_queries(ctx, casc):
    T = W.sinusoid_mix(100_000_000, 7)
    wl = W.mixed_queries(T, 64, 256, seed=9000)
    Td = dev(T)
    pq = dtws.PackedQueries([dev(q) for q in wl.queries])
    natural = ctx.search_batch(Td, pq, wl.bands)
    say("mixture: batched, series order")
    train_order(ctx, W.sinusoid_mix(10_000_000, 8), [(256, 12)], queries_per_shape=96)
    learned = ctx.search_batch(Td, pq, wl.bands, flags=dtws.ORDER_LEARNED, seed=3)
    assert learned == natural
    check_properties(casc, T, wl.queries, wl.bands, natural, wl.sources, samples=64, seed=2)
    say("mixture: learned order = series order, properties hold")
    sub = [0, 9, 18, 27, 32, 41, 50, 63]     # four cuts of the series, four fresh snippets
    t0 = time.time()
    ref, _ = casc.search_many(T, [wl.queries[k] for k in sub], [wl.bands[k] for k in sub])
    print(f"mixture: oracle on queries {sub} took {time.time() - t0:.1f}s", flush=True)
    check_exact([natural[k] for k in sub], ref)


C5_SUBSET = [0, 13, 26, 77]                 # shapes 0, 3, 6, 7: random-walk and sinusoid/bump shapes


def test_random_walk_1e9_planted_motifs(casc):
    t0 = time.time()
    wl = W.planted_motifs(1_000_000_000)
    say(f"planted motifs: generated in {time.time() - t0:.1f}s")
    c = dtws.Context(0, max_n=wl.T.size, max_m=1024, max_queries=128)
    try:
        Td = dev(wl.T)
        pq = dtws.PackedQueries([dev(q) for q in wl.queries])
        c.set_schedule(block=16384)
        train_order(c, W.sinusoid_mix(10_000_000, 8), [(1024, 102)], queries_per_shape=48, epochs=10)
        t0 = time.time()
        learned = c.search_batch(Td, pq, wl.bands, flags=dtws.ORDER_LEARNED, seed=3)
        say(f"planted motifs: batched, learned order, {time.time() - t0:.2f}s, counters {c.counters()}")
        check_properties(casc, wl.T, wl.queries, wl.bands, learned, None, samples=16, seed=3)
        say("planted motifs: properties hold")
        check_exact([c.search(Td, dev(wl.queries[k]), wl.bands[k], seed=5) for k in (0, 77)],
                    [learned[0], learned[77]])
        say("planted motifs: plain = batched on queries 0 and 77")
        say(f"planted motifs: oracle on queries {C5_SUBSET} (scans sharing the window moments) ...")
        t0 = time.time()
        # four scans over quarters of the starts (each with the m - 1 points after it), so that
        # progress shows; the best over the quarters, ties to the lowest start, is the whole answer
        m = wl.queries[C5_SUBSET[0]].size
        assert all(wl.queries[k].size == m for k in C5_SUBSET)
        N = wl.T.size - m + 1
        cuts = [N * j // 4 for j in range(5)]
        best = [None] * len(C5_SUBSET)
        for j in range(4):
            a, b = cuts[j], cuts[j + 1]
            part, _ = casc.search_many(wl.T[a:b + m - 1], [wl.queries[k] for k in C5_SUBSET],
                                       [wl.bands[k] for k in C5_SUBSET])
            for t, (i, d) in enumerate(part):
                if best[t] is None or (d, i + a) < best[t]:
                    best[t] = (d, i + a)
            say(f"planted motifs: oracle, starts {a}..{b - 1} done at {time.time() - t0:.1f}s")
        ref = [(i, d) for d, i in best]
        say(f"planted motifs: oracle {ref} in {time.time() - t0:.1f}s")
        check_exact([learned[k] for k in C5_SUBSET], ref)
        # expected, not guaranteed: each answer is a planted copy of the query's own shape
        pos, kind = wl.note["positions"], wl.note["shapes"]
        hits = 0
        for k, (i, _) in enumerate(learned):
            near = np.abs(pos - i) <= 16
            hits += bool(np.any(kind[near] == wl.sources[k]))
        print(f"answers at a planted copy of the query's shape: {hits}/{len(learned)}")
        assert hits >= int(0.9 * len(learned))
        del Td
    finally:
        c.close()
        torch.cuda.empty_cache()
