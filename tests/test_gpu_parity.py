"""Parity of the HIP path (called through the C ABI) with the CPU oracle, element by element.

Tolerances: FP32 device arithmetic against the FP64 oracle.
  * window statistics: FP64 on both sides (anchored prefix sums vs two-pass): mu to 1e-12
    relative to the window's magnitude, sigma to 1e-9 relative.
  * bounds and FP32 DTW values: |gpu - ref| <= 1e-4 * ref + 1e-5 (FP32 accumulation over at
    most 2m terms of O(1) size; the distance tolerance stated for the method is 1e-4).
  * search results: identical index; distance certified in FP64, so within 1e-9 relative.
"""
import math

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


def close_rel(gpu, ref, rtol=1e-4, atol=1e-5):
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    bad = np.abs(gpu - ref) > rtol * np.abs(ref) + atol
    assert not bad.any(), f"{bad.sum()} mismatches, first at {np.argmax(bad)}: {gpu[bad][:5]} vs {ref[bad][:5]}"


@pytest.fixture(scope="module")
def ctx():
    c = dtws.Context(0, max_n=3_000_000, max_m=2048, max_queries=16)
    yield c
    c.close()


@pytest.fixture(scope="module")
def casc():
    return Cascade()


@pytest.fixture(scope="module")
def small_wl():
    wl = W.single_query_small()
    D = R.all_distances(wl.T, wl.queries[0], wl.bands[0], chunk=16384)
    return wl, D


# --------------------------------------------------------------------- statistics
def oracle_stats(T, m, chunk=100_000):
    N = T.size - m + 1
    mu = np.empty(N)
    sg = np.empty(N)
    for a in range(0, N, chunk):
        b = min(N, a + chunk)
        mu[a:b], sg[a:b] = R.window_stats(T[a:b + m - 1], m)
    return mu, sg


@pytest.mark.parametrize("n,m,offset", [(300_000, 128, 0.0), (123_457, 2, 0.0), (50_001, 1500, 0.0),
                                        (1_000_003, 1024, 2.0e4), (2100, 2048, -7.5)])
def test_znorm_stats(ctx, n, m, offset):
    T = (W.random_walk(n, 5) + np.float32(offset)).astype(np.float32)
    mu, sg = ctx.znorm_stats(dev(T), m)
    mu_r, sg_r = oracle_stats(T, m)
    scale = np.maximum(1.0, np.abs(mu_r))
    assert np.max(np.abs(mu.cpu().numpy() - mu_r) / scale) < 1e-12
    assert np.all(np.abs(sg.cpu().numpy() - sg_r) <= 1e-9 * sg_r + 1e-12)


def test_znorm_stats_flat_windows(ctx):
    T = W.random_walk(10_000, 6)
    T[3000:3400] = np.float32(17.25)          # constant stretch: windows inside are flat
    T[6000:6100] = np.float32(0.0)
    mu, sg = ctx.znorm_stats(dev(T), 64)
    mu_r, sg_r = oracle_stats(T, 64)
    sg = sg.cpu().numpy()
    flat = sg_r <= R.SIGMA_FLAT
    assert flat.sum() == (400 - 63) + (100 - 63)
    assert np.all(sg[flat] <= R.SIGMA_FLAT)
    assert np.all(np.abs(sg[~flat] - sg_r[~flat]) <= 1e-9 * sg_r[~flat])


# --------------------------------------------------------------------- bounds
@pytest.mark.parametrize("m,r", [(128, 6), (128, 0), (77, 40), (16, 15)])
def test_lb_values(ctx, m, r):
    T = W.random_walk(20_011, 9)
    Q = W.noisy_cut(T, 5_000, m, 0.1, 10)
    out = ctx.lb_cascade(dev(T), dev(Q), r)
    kim, kq, kd = (out[k].cpu().numpy() for k in ("kim", "keogh_q", "keogh_d"))
    N = T.size - m + 1
    qh = R.znorm(Q)
    C = R.normalized_windows(T, m, np.arange(N))
    kim_r = (qh[0] - C[:, 0]) ** 2 + (qh[-1] - C[:, -1]) ** 2
    close_rel(kim, kim_r)
    rng = np.random.default_rng(m + r)
    sample = np.unique(np.concatenate([rng.integers(0, N, 250), [0, 1, N - 2, N - 1], np.arange(4990, 5010)]))
    kq_r = [R.lb_keogh_q(qh, C[i], r) for i in sample]
    kd_r = [R.lb_keogh_d_series(T, int(i), m, r, qh) for i in sample]
    close_rel(kq[sample], kq_r, rtol=2e-4, atol=2e-4)
    close_rel(kd[sample], kd_r, rtol=2e-4, atol=2e-4)


def test_lb_survivors(ctx):
    T = W.random_walk(50_000, 11)
    Q = W.noisy_cut(T, 20_000, 128, 0.1, 12)
    vals = ctx.lb_cascade(dev(T), dev(Q), 6)
    mx = np.maximum(np.maximum(vals["kim"].cpu().numpy(), vals["keogh_q"].cpu().numpy()),
                    vals["keogh_d"].cpu().numpy())
    thr = float(np.quantile(mx, 0.01))
    out = ctx.lb_cascade(dev(T), dev(Q), 6, values=False, threshold=thr, survivors=True)
    got = np.sort(out["survivors"].cpu().numpy())
    want = np.nonzero(mx <= np.float32(thr))[0]
    np.testing.assert_array_equal(got, want)
    assert 20_000 in set(got.tolist()) or mx[20_000] > thr


# --------------------------------------------------------------------- DTW
def test_dtw_band_all_candidates_small_workload(ctx, small_wl):
    wl, D = small_wl
    N = D.size
    got = ctx.dtw_band(dev(wl.T), dev(wl.queries[0]), wl.bands[0],
                       torch.arange(N, dtype=torch.int64, device=DEV)).cpu().numpy()
    close_rel(got, D)


@pytest.mark.parametrize("n,m,r", [(400, 2, 0), (400, 2, 1), (900, 3, 1), (2500, 17, 4), (2000, 100, 0),
                                   (1500, 100, 99), (1200, 128, 111), (1200, 128, 112), (1100, 300, 150),
                                   (700, 64, 63), (333, 333, 20)])
def test_dtw_band_shapes(ctx, n, m, r):
    T, Q = W.tiny_random(n, m, n + m + r)
    N = n - m + 1
    starts = np.arange(N, dtype=np.int64)
    got = ctx.dtw_band(dev(T), dev(Q), r, dev(starts)).cpu().numpy()
    ref = R.distances_at(T, Q, r, starts)
    close_rel(got, ref)


def test_dtw_band_abandon_and_invalid_starts(ctx, small_wl):
    wl, D = small_wl
    thr = float(np.quantile(D, 0.05))
    rng = np.random.default_rng(3)
    starts = rng.integers(0, D.size, 5000)
    got = ctx.dtw_band(dev(wl.T), dev(wl.queries[0]), wl.bands[0], dev(starts), abandon_at=thr).cpu().numpy()
    fin = np.isfinite(got)
    close_rel(got[fin], D[starts[fin]])
    assert np.all(D[starts[~fin]] > thr * (1 - 1e-5))
    bad = np.array([-1, D.size, 10 ** 9, 0], dtype=np.int64)
    g = ctx.dtw_band(dev(wl.T), dev(wl.queries[0]), wl.bands[0], dev(bad)).cpu().numpy()
    assert np.isnan(g[:3]).all() and np.isfinite(g[3])


# --------------------------------------------------------------------- best-so-far
def test_bsf_update_contention(ctx):
    rng = np.random.default_rng(4)
    n = 1 << 20
    d = rng.choice(np.array([3.5, 1.25, 1.25, 7.0, 2.0], np.float32), n)
    idx = rng.permutation(n).astype(np.int64) + 17
    keys = torch.full((1,), -1, dtype=torch.int64, device=DEV)     # all ones = +inf key
    ctx.bsf_update(keys, dev(d), dev(idx))
    k = int(keys.cpu().numpy().view(np.uint64)[0])
    dist, i = dtws.unpack_key(k)
    assert dist == 1.25 and i == int(idx[d == np.float32(1.25)].min())


# --------------------------------------------------------------------- search
def test_search_single_query_workload(ctx, small_wl):
    wl, D = small_wl
    i_ref = int(np.argmin(D))
    for seed in (0, 1, 2):
        idx, dist = ctx.search(dev(wl.T), dev(wl.queries[0]), wl.bands[0], seed=seed)
        assert idx == i_ref
        assert abs(dist - D[i_ref]) <= 1e-9 * D[i_ref]
    c = ctx.counters()
    assert c["candidates"] == D.size and c["certified"] >= 1
    idx, dist = ctx.search(dev(wl.T), dev(wl.queries[0]), wl.bands[0], flags=dtws.NO_LOWER_BOUNDS)
    assert idx == i_ref and abs(dist - D[i_ref]) <= 1e-9 * D[i_ref]


@pytest.mark.parametrize("n,m,r,seed", [(64, 64, 3, 1), (65, 64, 63, 2), (500, 16, 0, 3), (3000, 40, 4, 4),
                                        (3000, 200, 30, 5), (2000, 128, 127, 6), (5000, 2, 1, 7),
                                        (4000, 500, 120, 8)])
def test_search_small_shapes(ctx, n, m, r, seed):
    T, Q = W.tiny_random(n, m, seed)
    i_ref, d_ref = R.best_match(T, Q, r)
    idx, dist = ctx.search(dev(T), dev(Q), r, seed=seed)
    assert idx == i_ref, (idx, i_ref, dist, d_ref)
    assert abs(dist - d_ref) <= 1e-9 * d_ref + 1e-12


def test_search_exact_copies_lowest_index(ctx):
    T, _ = W.tiny_random(5000, 8, 21)
    T = T.copy()
    T[4000:4050] = T[1000:1050]       # bit-identical second copy at a higher index
    T[2500:2550] = T[1000:1050]
    Q = (T[1000:1050].astype(np.float64) * 0.25 - 1.0).astype(np.float32)
    idx, dist = ctx.search(dev(T), dev(Q), 5)
    i_ref, d_ref = R.best_match(T, Q, 5)
    assert idx == i_ref == 1000
    assert dist < 1e-9


def test_search_batch_equals_single(ctx):
    T = W.random_walk(200_000, 13)
    qs, rs = [], []
    for k, (m, fr) in enumerate([(64, 0.05), (300, 0.1), (128, 0.0), (1000, 0.02), (64, 0.5)]):
        qs.append(W.noisy_cut(T, 1000 + 37_000 * k, m, 0.1, 40 + k))
        rs.append(dtws.band(m, fr))
    Td = dev(T)
    batch = ctx.search_batch(Td, [dev(q) for q in qs], rs)
    for q, r, got in zip(qs, rs, batch):
        single = ctx.search(Td, dev(q), r)
        assert got[0] == single[0] and got[1] == pytest.approx(single[1], rel=1e-12)


# --------------------------------------------------------------------- batched search
def _cascade_refs(casc, T, qs, rs):
    return [casc.search(T, q, r)[:2] for q, r in zip(qs, rs)]


def _check_batch(got, ref):
    for k, ((gi, gd), (ri, rd)) in enumerate(zip(got, ref)):
        assert gi == ri, (k, gi, ri, gd, rd)
        assert abs(gd - rd) <= 1e-9 * rd + 1e-12, (k, gd, rd)


def test_batch_mixed_lengths_and_bands(ctx, casc):
    """Different m per query: window statistics from the blocked prefix; one wide band (r > 111)."""
    T = W.random_walk(150_001, 31)
    specs = [(16, 1), (40, 0), (64, 6), (100, 10), (128, 6), (200, 20), (300, 150), (512, 25), (65, 64), (128, 0),
             (777, 38), (2048, 102)]
    qs, rs = [], []
    for k, (m, r) in enumerate(specs):
        src = (9_973 * (k + 1)) % (T.size - m)
        qs.append(W.noisy_cut(T, src, m, 0.1, 500 + k) if k % 3 else W.random_walk(m, 600 + k))
        rs.append(r)
    got = ctx.search_batch(dev(T), [dev(q) for q in qs], rs)
    _check_batch(got, _cascade_refs(casc, T, qs, rs))


@pytest.mark.parametrize("n", [1 << 18, (1 << 18) + 1])
def test_batch_prefix_matches_at_series_end(ctx, casc, n):
    """Different m per query, each cut from the very end of the series, so the best window ends at
    n: the prefix entry at n (the sentinel after the last block when n is a whole number of blocks,
    an odd entry completed from the last point otherwise) decides the statistics of the match."""
    T = W.random_walk(n, 37)
    specs = [(64, 3), (128, 6), (130, 7), (200, 10), (512, 25), (1024, 51)]
    qs = [W.noisy_cut(T, n - m, m, 0.02, 1_000 + k) for k, (m, _) in enumerate(specs)]
    rs = [r for _, r in specs]
    got = ctx.search_batch(dev(T), [dev(q) for q in qs], rs)
    _check_batch(got, _cascade_refs(casc, T, qs, rs))
    assert [i for i, _ in got] == [n - m for m, _ in specs]


def test_batch_contexts_in_flight_from_threads(casc):
    """Several batches in flight: two contexts, each searched repeatedly from its own host thread
    (each replays its own graph on its own stream), agree with the oracle on every call."""
    import threading
    T = W.random_walk(300_001, 38)
    specs = [(64, 3), (128, 6), (200, 10), (512, 25)]
    qs = [W.noisy_cut(T, 17_000 + 61_000 * k, m, 0.1, 1_100 + k) for k, (m, _) in enumerate(specs)]
    rs = [r for _, r in specs]
    ref = _cascade_refs(casc, T, qs, rs)
    Td = dev(T)
    pq = dtws.PackedQueries([dev(q) for q in qs])
    ctxs = [dtws.Context(0, max_n=T.size, max_m=512, max_queries=len(qs)) for _ in range(2)]
    outs = [[] for _ in ctxs]
    errors = []

    def work(k):
        try:
            for _ in range(4):
                outs[k].append(ctxs[k].search_batch(Td, pq, rs, flags=dtws.ORDER_NATURAL, seed=7))
        except Exception as e:   # reported below; the thread itself must not raise
            errors.append(e)

    try:
        threads = [threading.Thread(target=work, args=(k,)) for k in range(len(ctxs))]
        for th in threads:
            th.start()
        for th in threads:
            th.join()
        assert not errors, errors
        for got_list in outs:
            assert len(got_list) == 4
            for got in got_list:
                _check_batch(got, ref)
    finally:
        for c in ctxs:
            c.close()


def test_wide_bands_plain_and_batched(ctx, casc):
    """Bands from 256 up to unconstrained DTW (r = m - 1) and r = 1023: the wide one-wave
    instances in the plain search (DTW and FP64 certification) and in the batched search."""
    T = W.random_walk(12_001, 39)
    specs = [(400, 256), (600, 599), (1024, 819), (128, 6)]
    qs = [W.noisy_cut(T, 900 + 2_500 * k, m, 0.1, 1_200 + k) if k % 2 == 0 else W.random_walk(m, 1_300 + k)
          for k, (m, _) in enumerate(specs)]
    rs = [r for _, r in specs]
    ref = _cascade_refs(casc, T, qs, rs)
    for q, r, (ri, rd) in zip(qs, rs, ref):
        gi, gd = ctx.search(dev(T), dev(q), r, seed=7)
        assert gi == ri and abs(gd - rd) <= 1e-9 * rd + 1e-12, (len(q), r, gi, ri, gd, rd)
    _check_batch(ctx.search_batch(dev(T), [dev(q) for q in qs], rs), ref)


def test_batch_shared_length(ctx, casc):
    """All queries of one length: per-window statistics arrays shared by the batch."""
    T = W.random_walk(300_000, 32)
    qs = [W.noisy_cut(T, 1_000 + 29_000 * k, 128, 0.1, 700 + k) for k in range(10)]
    rs = [6] * 10
    got = ctx.search_batch(dev(T), [dev(q) for q in qs], rs)
    _check_batch(got, _cascade_refs(casc, T, qs, rs))


def test_batch_order_invariance(ctx):
    """Natural order and seeded random block orders give identical results."""
    T = W.random_walk(400_000, 33)
    qs = [W.noisy_cut(T, 3_000 + 51_000 * k, m, 0.1, 800 + k) for k, m in enumerate((64, 128, 256, 128, 512))]
    rs = [3, 6, 12, 0, 25]
    Td = dev(T)
    Qd = [dev(q) for q in qs]
    base = ctx.search_batch(Td, Qd, rs)
    for seed in (1, 2, 3):
        assert ctx.search_batch(Td, Qd, rs, flags=dtws.ORDER_RANDOM, seed=seed) == base


def test_batch_graph_replays_match_eager(ctx, casc):
    """The batched pipeline replays a captured graph when called again with the same inputs; every
    replay, with eager work in between, must equal the eagerly enqueued result and the oracle."""
    T = W.random_walk(250_000, 34)
    qs = [W.noisy_cut(T, 5_000 + 40_000 * k, m, 0.1, 900 + k) for k, m in enumerate((96, 256, 640))]
    rs = [4, 12, 32]
    Td = dev(T)
    pq = dtws.PackedQueries([dev(q) for q in qs])
    eager = ctx.search_batch(Td, pq, rs, flags=dtws.NO_GRAPH)
    _check_batch(eager, _cascade_refs(casc, T, qs, rs))
    for rep in range(4):
        assert ctx.search_batch(Td, pq, rs) == eager, rep
        ctx.search(Td, dev(qs[rep % 3]), rs[rep % 3])            # eager work between replays
        torch.cuda.synchronize()


# --------------------------------------------------------------------- schedules
@pytest.mark.parametrize("n,m,r", [(400, 2, 0), (400, 2, 1), (900, 3, 2), (2500, 17, 4), (2000, 100, 0),
                                   (3000, 130, 63), (3000, 130, 64), (2000, 300, 127), (2100, 300, 128),
                                   (1500, 400, 255), (4200, 2048, 102), (2048, 2048, 255), (1200, 256, 255),
                                   (1500, 400, 256), (2200, 700, 399), (1800, 600, 599), (2000, 1024, 819),
                                   (2200, 2048, 1023)])
def test_dtw_band_wave_schedule(ctx, n, m, r):
    """One wave per candidate along anti-diagonals (odd / even bands, one to four slot registers,
    and the wide instance's six to sixteen up to r = 1023; r = 0, r = m - 1 clamped, unconstrained
    DTW, n = m) against the oracle, and against the lane schedule."""
    T, Q = W.tiny_random(n, m, 7 * n + m + r)
    N = n - m + 1
    starts = np.arange(0, N, max(1, N // 600), dtype=np.int64)
    ref = R.distances_at(T, Q, r, starts)
    try:
        ctx.set_schedule(band_lanes=64)
        got = ctx.dtw_band(dev(T), dev(Q), r, dev(starts)).cpu().numpy()
        ctx.set_schedule(band_lanes=1)
        lane = ctx.dtw_band(dev(T), dev(Q), r, dev(starts)).cpu().numpy()
    finally:
        ctx.set_schedule(band_lanes=0)
    close_rel(got, ref)
    close_rel(got, lane)


def test_dtw_band_wave_schedule_abandon_and_invalid(ctx, small_wl):
    wl, D = small_wl
    thr = float(np.quantile(D, 0.05))
    starts = np.random.default_rng(5).integers(0, D.size, 3000)
    try:
        ctx.set_schedule(band_lanes=64)
        got = ctx.dtw_band(dev(wl.T), dev(wl.queries[0]), wl.bands[0], dev(starts), abandon_at=thr).cpu().numpy()
        bad = np.array([-1, D.size, 5], dtype=np.int64)
        g = ctx.dtw_band(dev(wl.T), dev(wl.queries[0]), wl.bands[0], dev(bad)).cpu().numpy()
    finally:
        ctx.set_schedule(band_lanes=0)
    fin = np.isfinite(got)
    close_rel(got[fin], D[starts[fin]])
    assert np.all(D[starts[~fin]] > thr * (1 - 1e-5))
    assert np.all(fin[D[starts] <= thr * 0.999])
    assert np.isnan(g[:2]).all() and abs(g[2] - D[5]) <= 1e-4 * D[5] + 1e-5


def test_schedules_give_identical_results(ctx, casc):
    """Every DTW schedule (lane only, wave only, the default split) and every block size returns
    the oracle's matches, for the plain and the batched search."""
    T = W.random_walk(200_003, 35)
    specs = [(64, 3), (128, 6), (200, 20), (300, 150), (512, 25), (1000, 255), (777, 0)]
    qs = [W.noisy_cut(T, 7_000 + 27_000 * k, m, 0.1, 950 + k) if k % 2 == 0 else W.random_walk(m, 960 + k)
          for k, (m, r) in enumerate(specs)]
    rs = [r for _, r in specs]
    ref = _cascade_refs(casc, T, qs, rs)
    Td = dev(T)
    Qd = [dev(q) for q in qs]
    default = ctx.get_schedule()
    try:
        for sched in ({"diag_max": 0}, {"diag_max": 1 << 24}, {"diag_max": 8192, "block": 2048},
                      {"diag_max": 64, "block": 16384, "lb_blocks_per_cu": 2, "dtw_blocks_per_cu": 1},
                      {"diag_max": 8192, "block": 4096, "stats_prefix": 1, "data_envelope": 0},
                      {"rounds": 1, "block": 8192}, {"rounds": 2, "stats_prefix": 1}):
            ctx.set_schedule(**sched)
            _check_batch(ctx.search_batch(Td, Qd, rs), ref)
            _check_batch([ctx.search(Td, q, r, seed=3) for q, r in zip(Qd, rs)], ref)
    finally:
        ctx.set_schedule(**default)


def test_dtw_suffix_bound_and_refilling_rows_same_matches(ctx, casc):
    """The lane DTW with and without the suffix bound of the columns still to come, and the batched
    lane DTW with whole waves and with refilling 16-lane rows: the oracle's matches every way, for the
    plain and the batched search on the lane schedule, with bands of 4 to 14 chunks (m = 2048 takes
    bound blocks of 32 columns), lengths that are not multiples of 16 and queries of several lengths
    in one bucket; the bound can only abandon earlier, so it computes fewer DTW cells (up to the
    timing of best-so-far updates)."""
    T = W.random_walk(400_009, 44)
    specs = [(512, 51), (300, 60), (1024, 102), (2048, 111), (1000, 99), (777, 70), (200, 30), (130, 31),
             (1001, 50)]
    qs = [W.noisy_cut(T, (9_000 + 61_000 * k) % (T.size - m), m, 0.2, 1100 + k) if k % 2 == 0
          else W.random_walk(m, 1110 + k) for k, (m, _) in enumerate(specs)]
    rs = [r for _, r in specs]
    ref = _cascade_refs(casc, T, qs, rs)
    Td = dev(T)
    Qd = [dev(q) for q in qs]
    default = ctx.get_schedule()
    cells = {}
    try:
        for rows in (0, 1):
            for bound in (0, 1):
                ctx.set_schedule(diag_max=0, dtw_bound=bound, dtw_rows=rows)
                print("suffix bound", bound, "refilling rows", rows, flush=True)
                _check_batch(ctx.search_batch(Td, Qd, rs, seed=5), ref)
                cells[rows, bound] = ctx.counters()["dtw_cells"]
                _check_batch([ctx.search(Td, q, r, seed=5) for q, r in zip(Qd, rs)], ref)
            for order in (dtws.ORDER_RANDOM, dtws.ORDER_NATURAL):
                ctx.set_schedule(diag_max=0, rounds=1, block=2048, dtw_rows=rows)
                _check_batch(ctx.search_batch(Td, Qd, rs, flags=order, seed=6), ref)
    finally:
        ctx.set_schedule(**default)
    print(f"DTW cells, batched (rows, bound): {cells}")
    assert cells[0, 1] <= 1.1 * cells[0, 0]


def test_dtw_eviction_same_matches(ctx, casc):
    """Rows of the batched lane DTW that move their last few live candidates out and resume them in
    full rows (dtw_evict): the oracle's matches for thresholds 0 (off), 1, 6 and 15, with bands of 4
    to 14 chunks, several lengths per bucket, and in the random, natural and PAA orders; rows did
    move candidates (counter dtw_evicted) whenever the threshold is on."""
    T = W.random_walk(400_009, 45)
    specs = [(512, 51), (300, 60), (1024, 102), (2048, 111), (1000, 99), (777, 70), (200, 30), (130, 31),
             (1001, 50), (1024, 100)]
    qs = [W.noisy_cut(T, (7_000 + 53_000 * k) % (T.size - m), m, 0.3, 1200 + k) if k % 2 == 0
          else W.random_walk(m, 1210 + k) for k, (m, _) in enumerate(specs)]
    rs = [r for _, r in specs]
    ref = _cascade_refs(casc, T, qs, rs)
    Td = dev(T)
    Qd = [dev(q) for q in qs]
    default = ctx.get_schedule()
    moved = {}
    try:
        for ev in (0, 1, 6, 15):
            for order in (dtws.ORDER_RANDOM, dtws.ORDER_NATURAL, dtws.ORDER_PAA):
                ctx.set_schedule(diag_max=0, dtw_rows=1, dtw_bound=1, dtw_evict=ev, rounds=4, block=4096)
                print("dtw_evict", ev, "order", order, flush=True)
                _check_batch(ctx.search_batch(Td, Qd, rs, flags=order, seed=8), ref)
                moved[ev, order] = ctx.counters()["dtw_evicted"]
    finally:
        ctx.set_schedule(**default)
    print(f"candidates moved: {moved}")
    assert all(v == 0 for (ev, _), v in moved.items() if ev == 0)
    assert all(v > 0 for (ev, _), v in moved.items() if ev > 0)


def test_series_order_xcd_sub_queues(casc):
    """A series-order round large enough for the eight XCD sub-queues (at least 64 work items per
    wave: 128 queries x 977 blocks of 2048 candidates for 1024 waves), in series order and as the
    last round of the random and PAA orders (with its skip of the blocks visited before): the
    oracle's matches, and every (query, candidate) pair visited exactly once."""
    n, m = 2_000_000, 64
    T = W.random_walk(n, 46)
    qs = [W.noisy_cut(T, (7_919 * (k + 1) * 13) % (n - m), m, 0.2, 1200 + k) if k % 2 == 0
          else W.random_walk(m, 1300 + k) for k in range(128)]
    rs = [3 + (k % 4) for k in range(128)]
    ref, _ = casc.search_many(T, qs, rs)
    c = dtws.Context(0, max_n=n, max_m=m, max_queries=128)
    try:
        Td = dev(T)
        pq = dtws.PackedQueries([dev(q) for q in qs])
        for sched, order in (({"rounds": 1}, dtws.ORDER_NATURAL), ({"rounds": 4}, dtws.ORDER_NATURAL),
                             ({"rounds": 2}, dtws.ORDER_RANDOM), ({"rounds": 2}, dtws.ORDER_PAA)):
            c.set_schedule(block=2048, lb_blocks_per_cu=1, lb_tile=0, **sched)
            print("sub-queues", sched, order, flush=True)
            _check_batch(c.search_batch(Td, pq, rs, flags=order, seed=4), ref)
            cn = c.counters()
            # every pair ends in one bound or in a DTW; the seeding adds its own DTWs (one random
            # candidate per query, or 256 around the best proposals)
            visited = cn["pruned_kim"] + cn["pruned_keogh_q"] + cn["pruned_keogh_d"] + cn["dtw_started"]
            assert cn["fallbacks"] == 0
            assert visited - 128 * (n - m + 1) in (128, 128 * 256), (visited, cn)
    finally:
        c.close()


def test_tiled_cascade_equals_per_query_items(ctx, casc):
    """The tiled cascade (one LDS-staged series tile shared by every query of a length) against the
    per-query work items and the oracle: seven queries in four length groups (the longest, m = 2048,
    with a 2047-point halo), a series that ends inside a tile, statistics from the per-length arrays
    and from the prefix, the data envelope on and off, four rounds and one, series and random order."""
    n = 7 * 2048 * 9 + 1_234
    T = W.random_walk(n, 38)
    specs = [(64, 3), (64, 0), (64, 12), (200, 20), (200, 5), (2048, 102), (1000, 255)]
    qs = [W.noisy_cut(T, (13_331 * (k + 1)) % (n - m), m, 0.1, 980 + k) if k % 3 else W.random_walk(m, 990 + k)
          for k, (m, _) in enumerate(specs)]
    qs.append(W.noisy_cut(T, n - 64, 64, 0.01, 999))            # a match at the very end of the series
    specs.append((64, 3))
    rs = [r for _, r in specs]
    ref = _cascade_refs(casc, T, qs, rs)
    Td = dev(T)
    Qd = [dev(q) for q in qs]
    default = ctx.get_schedule()
    try:
        for sched in ({"lb_tile": 1}, {"lb_tile": 0}, {"lb_tile": 1, "stats_prefix": 1},
                      {"lb_tile": 1, "data_envelope": 0}, {"lb_tile": 1, "rounds": 1, "block": 2048},
                      {"lb_tile": 1, "rounds": 2, "block": 16384, "stats_prefix": 1, "data_envelope": 0}):
            ctx.set_schedule(**sched)
            print("tiled cascade schedule", sched, flush=True)
            for order in (dtws.ORDER_NATURAL, dtws.ORDER_RANDOM):
                _check_batch(ctx.search_batch(Td, Qd, rs, flags=order, seed=9), ref)
            assert ctx.counters()["fallbacks"] == 0
    finally:
        ctx.set_schedule(**default)
    ctx.search_batch(Td, Qd, rs)
    c = ctx.counters()
    assert c["lb_terms"] > 0 and c["pruned_kim"] + c["pruned_keogh_q"] + c["pruned_keogh_d"] > 0


@pytest.mark.parametrize("n,m,r,seed", [(3000, 40, 4, 41), (5000, 128, 0, 42), (4000, 200, 199, 43),
                                        (20_000, 512, 25, 44), (64, 64, 3, 45)])
def test_lb_sorted_order_matches_oracle(ctx, n, m, r, seed):
    """The Prepare / Improve scheme with the candidates in ascending order of their bound returns the
    oracle's match (plain, and batched query by query)."""
    T, Q = W.tiny_random(n, m, seed)
    i_ref, d_ref = R.best_match(T, Q, r)
    idx, dist = ctx.search(dev(T), dev(Q), r, flags=dtws.LB_SORTED, seed=seed)
    assert idx == i_ref, (idx, i_ref, dist, d_ref)
    assert abs(dist - d_ref) <= 1e-9 * d_ref + 1e-12
    got = ctx.search_batch(dev(T), [dev(Q), dev(Q)], [r, 0], flags=dtws.LB_SORTED)
    assert got[0] == (idx, dist)
    i0, d0 = R.best_match(T, Q, 0)
    assert got[1][0] == i0 and abs(got[1][1] - d0) <= 1e-9 * d0 + 1e-12


def test_lb_sorted_order_single_query_workload(ctx, small_wl):
    """n = 262,144, m = 128, r = 6: the LB-sorted order against the brute-force oracle, with the
    DTW count it needs (the bound's order reaches the best match among the first candidates)."""
    wl, D = small_wl
    i_ref = int(np.argmin(D))
    idx, dist = ctx.search(dev(wl.T), dev(wl.queries[0]), wl.bands[0], flags=dtws.LB_SORTED, seed=4)
    assert idx == i_ref and abs(dist - D[i_ref]) <= 1e-9 * D[i_ref]
    sorted_dtw = ctx.counters()["dtw_started"]
    ctx.search(dev(wl.T), dev(wl.queries[0]), wl.bands[0], seed=4)
    print(f"DTW started: LB-sorted {sorted_dtw}, series order {ctx.counters()['dtw_started']}")
    assert sorted_dtw <= ctx.counters()["dtw_started"]


def test_set_schedule_rejects_bad_fields(ctx):
    default = ctx.get_schedule()
    for bad in ({"block": 3000}, {"diag_max": -2}, {"band_lanes": 2}, {"lb_blocks_per_cu": 65},
                {"stats_prefix": 2}, {"data_envelope": -1}, {"rounds": 3}, {"list_cap": 63}, {"lb_tile": 2},
                {"dtw_bound": 2}, {"dtw_rows": -1}, {"dtw_evict": -1}, {"dtw_evict": 16}):
        with pytest.raises(dtws.DtwsError):
            ctx.set_schedule(**bad)
        assert ctx.get_schedule() == default


def test_autotune_installs_a_candidate_schedule(ctx, casc):
    T = W.random_walk(300_000, 36)
    qs = [W.noisy_cut(T, 11_000 + 61_000 * k, m, 0.1, 970 + k) for k, m in enumerate((128, 256, 512))]
    rs = [6, 12, 25]
    default = ctx.get_schedule()
    try:
        pq = dtws.PackedQueries([dev(q) for q in qs])
        best, ms = ctx.autotune_batch(dev(T), pq, rs, reps=2)
        assert ms > 0
        assert best["block"] in (2048, 4096, 8192, 16384) and best["diag_max"] in (0, 2048, 16384, 65536)
        assert best["lb_blocks_per_cu"] in (4, 8, 16, 32) and best["dtw_blocks_per_cu"] in (2, 4, 8)
        assert best["stats_prefix"] in (0, 1) and best["data_envelope"] in (0, 1) and best["rounds"] in (1, 2, 4)
        assert ctx.get_schedule() == best
        _check_batch(ctx.search_batch(dev(T), pq, rs), _cascade_refs(casc, T, qs, rs))
    finally:
        ctx.set_schedule(**default)
