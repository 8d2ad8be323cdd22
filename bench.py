"""Benchmark: exact best-match DTW search on one MI355X.

One step = the whole search path (window statistics, data envelope, bound cascade, banded DTW
with the device best-so-far, FP64 certification) for every query of the workload, with the
series already resident in HBM.  The timed path is the batched search with the learned block
order (one graph replay per step), with three batches in flight by default: three library
contexts, each replaying its graph on its own stream from its own host thread, so that one batch's
latency-bound phases overlap the other's streaming kernels (every step still runs the whole path
on its batch; the rate with one batch in flight is reported beside it).  The plain per-query
search and the batched search in series order are timed beside it.  The ordering network is trained before timing (seeded).  Default workload: float32 random walk of n = 1e8 points and
three queries (m = 128, 512, 1024, cut from the series plus N(0, 0.1) noise, band 5%).

Prints one JSON line.  value = seconds per query (lower is better).  The roofline object is
for the kernel class with the largest total time, timed with HIP events recorded on the
launch stream inside the library (DTWS_PROFILE) over a separate profiled pass.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "search s/query and DTW GCUPS (frac. VALU peak), batched+learned vs plain, 1 GPU"
# MI355X peaks (public figures): HBM3E 8 TB/s; FP32 VALU lane-ops: 256 CU x 4 SIMD x 16 lanes x
# 2.4 GHz = 39.3e12 /s (no packed math); DTW needs 3 lane-ops per cell -> 13,107 GCUPS.
HBM_PEAK_GBS = 8000.0
VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9
DTW_PEAK_GCUPS = VALU_LANE_OPS / 3 / 1e9


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# sources that define each kernel whose HBM traffic is recorded (profiles/hbm_traffic.md)
# (keyed by the kernel's name without template arguments)
KERNEL_SOURCES = {
    "k_lb_batch": ["batch.hip", "batch_stats.h", "device.h", "dtws_internal.h"],
    "k_prefix": ["batch.hip", "dtws_internal.h"],
    "k_propose": ["mlp.hip", "device.h", "dtws_internal.h"],
}


def kernel_source_hash(kernel: str) -> str:
    """SHA-256 over the sources of `kernel`, to tell whether recorded counters still describe it."""
    import hashlib
    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_1812_10302_amd", "csrc")
    for f in KERNEL_SOURCES.get(kernel.split("<")[0], []):
        with open(os.path.join(src, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()


def traffic_of(kernel: str, launches: int, algorithmic: float):
    """HBM bytes per launch of `kernel` recorded from rocprofv3 FETCH_SIZE / WRITE_SIZE runs
    (profiles/hbm_traffic.md), or None when none is recorded for the kernel's current sources."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.md")
    if not os.path.exists(path) or kernel.split("<")[0] not in KERNEL_SOURCES:
        return None
    cur = kernel_source_hash(kernel)
    for line in open(path):
        if line.startswith("| `" + kernel + "`"):
            cols = [c.strip().strip("`") for c in line.strip().strip("|").split("|")]
            # | kernel | sources sha256 | bytes per launch (calibrated) | ...
            if cols[1] == cur:
                return float(cols[2])
    return None


def cells(m: int, r: int) -> int:
    r = min(r, m - 1)
    return m * (2 * r + 1) - r * (r + 1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=100_000_000)
    ap.add_argument("--cpu-sample", type=int, default=1 << 26, help="series points for the CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--train-n", type=int, default=10_000_000, help="training series length (ordering network)")
    ap.add_argument("--train-pairs", type=int, default=999_000)
    ap.add_argument("--train-epochs", type=int, default=20)
    ap.add_argument("--only-learned", action="store_true",
                    help="time only the batched search in learned order (profiling runs)")
    ap.add_argument("--schedule", default="",
                    help="comma-separated schedule fields (k=v) to use instead of the autotuner")
    ap.add_argument("--inflight", type=int, default=3,
                    help="learned batches in flight: one library context, stream and host thread each")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="after timing, copy this many MiB on the device (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the search shards by "
              "series fragment across GPUs but this build runs and times a single GPU.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1812_10302_amd as dtws
    from paper_1812_10302_amd import workloads as W

    t0 = time.time()
    wl = W.three_queries_large(args.n)
    log(f"workload {wl.name}: generated in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    T = torch.from_numpy(wl.T).to(dev)
    Qs = [torch.from_numpy(q).to(dev) for q in wl.queries]
    ms = [q.size for q in wl.queries]
    rs = list(wl.bands)
    nq = len(Qs)
    ctx = dtws.Context(0, max_n=wl.T.size, max_m=max(ms), max_queries=nq)
    torch.cuda.synchronize()

    # ---------------------------------------------------------------- plain: one query at a time
    def plain_step(flags=0):
        return [ctx.search(T, q, r, flags=flags, seed=7) for q, r in zip(Qs, rs)]

    per_query = []
    plain_s, plain_results = None, None
    if not args.only_learned:
        for _ in range(args.warmup):
            plain_step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            for q, r in zip(Qs, rs):
                a = time.perf_counter()
                ctx.search(T, q, r, seed=7)
                per_query.append(time.perf_counter() - a)
        torch.cuda.synchronize()
        plain_s = (time.perf_counter() - t1) / args.steps / nq
        plain_results = plain_step()

    # ---------------------------------------------------------------- ordering network (untimed)
    from paper_1812_10302_amd import proposal
    t0 = time.time()
    train_T = W.random_walk(args.train_n, 8)
    Xs, Ys = [], []
    for k, (m, r) in enumerate(zip(ms, rs)):
        rows_per_query = args.train_n // 1024 + 320
        X, Y = proposal.make_pairs(ctx, train_T, m, r, max(1, args.train_pairs // (rows_per_query * nq)),
                                   seed=80 + k)
        Xs.append(X)
        Ys.append(Y)
    curve = proposal.train(ctx, torch.cat(Xs).contiguous(), torch.cat(Ys).contiguous(), epochs=args.train_epochs,
                           seed=9, log=log)
    train_s = time.time() - t0
    log(f"ordering network trained in {train_s:.1f}s, loss {curve[0]:.4f} -> {curve[-1]:.4f}")

    # ---------------------------------------------------------------- batched: all queries, graph replay
    pq = dtws.PackedQueries(Qs)

    def batch_step(order, flags=0):
        return ctx.search_batch(T, pq, rs, flags=order | flags, seed=7)

    def time_batched(order):
        for _ in range(max(1, args.warmup)):
            batch_step(order)        # the first call captures the graph
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            res = batch_step(order)
        torch.cuda.synchronize()
        return (time.perf_counter() - t1) / args.steps, res

    natural_step_s, natural_results = (None, None) if args.only_learned else time_batched(dtws.ORDER_NATURAL)
    if args.schedule:
        ctx.set_schedule(**{k: int(v) for k, v in (kv.split("=") for kv in args.schedule.split(","))})
        schedule = ctx.get_schedule()
        log(f"schedule {schedule} (given)")
    else:
        # launch schedule for the learned batch picked by the library's autotuner (untimed)
        t0 = time.time()
        schedule, tune_ms = ctx.autotune_batch(T, pq, rs, flags=dtws.ORDER_LEARNED, seed=7, reps=3)
        log(f"autotuned schedule {schedule} ({tune_ms:.2f} ms per batch, tuning took {time.time() - t0:.1f}s)")
    single_step_s, results = time_batched(dtws.ORDER_LEARNED)
    elapsed_step = single_step_s
    if args.inflight > 1:
        # several batches in flight: each context runs whole steps on its own stream from its own
        # host thread, so one batch's latency-bound phases (DTW, certification, host round trips)
        # overlap another's streaming kernels; every step still runs the whole path on its batch
        import threading
        params = ctx.model_get()
        ctxs = [ctx]
        for _ in range(args.inflight - 1):
            c2 = dtws.Context(0, max_n=wl.T.size, max_m=max(ms), max_queries=nq)
            c2.model_set(params)
            c2.set_schedule(**schedule)
            ctxs.append(c2)
        for c in ctxs:
            for _ in range(max(1, args.warmup)):
                assert c.search_batch(T, pq, rs, flags=dtws.ORDER_LEARNED, seed=7) == results
        torch.cuda.synchronize()
        share = [args.steps // len(ctxs) + (1 if k < args.steps % len(ctxs) else 0) for k in range(len(ctxs))]
        outs = [None] * len(ctxs)
        start = threading.Barrier(len(ctxs) + 1)

        def worker(k):
            start.wait()
            for _ in range(share[k]):
                outs[k] = ctxs[k].search_batch(T, pq, rs, flags=dtws.ORDER_LEARNED, seed=7)

        threads = [threading.Thread(target=worker, args=(k,)) for k in range(len(ctxs))]
        for th in threads:
            th.start()
        torch.cuda.synchronize()
        start.wait()
        t1 = time.perf_counter()
        for th in threads:
            th.join()
        torch.cuda.synchronize()
        elapsed_step = (time.perf_counter() - t1) / args.steps
        assert all(o == results for o, k in zip(outs, share) if k > 0), "batches in flight disagree"
    ms_per_step = elapsed_step * 1e3
    s_per_query = elapsed_step / nq
    log("plain:", plain_results)
    log("batched natural:", natural_results)
    log("batched learned:", results)
    if not args.only_learned:
        assert results == natural_results, "learned and natural orders disagree"
        assert [i for i, _ in results] == [i for i, _ in plain_results], "batched and plain disagree"
    if args.copy_calibration_mib > 0:
        # a plain device copy of known size: its HBM counters calibrate the traffic of the others
        nb = args.copy_calibration_mib << 20
        src_buf = torch.empty(nb // 4, dtype=torch.float32, device=dev).fill_(1.0)
        dst_buf = torch.empty_like(src_buf)
        torch.cuda.synchronize()
        dst_buf.copy_(src_buf)
        torch.cuda.synchronize()
        del src_buf, dst_buf

    def batch_step_learned(flags=0):
        return batch_step(dtws.ORDER_LEARNED, flags)

    # ---------------------------------------------------------------- profiled passes
    def profiled(run):
        run()
        p = ctx.profile()
        return {k: [v[0], v[1]] for k, v in p.items()}, ctx.counters()

    prof_total, cnt_total = {k: [0.0, 0] for k in dtws.KERNEL_CLASSES}, {}
    per_query_prof = []
    if not args.no_profile:
        prof_total, cnt_total = profiled(lambda: batch_step_learned(dtws.PROFILE))
        for q, r in ([] if args.only_learned else zip(Qs, rs)):
            kp, c = profiled(lambda: ctx.search(T, q, r, flags=dtws.PROFILE, seed=7))
            per_query_prof.append({"m": int(q.numel()), "r": int(r),
                                   "plain_kernel_ms": {k: round(v[0], 4) for k, v in kp.items()}, "counters": c})
    dtw_cells = cnt_total.get("dtw_cells", 0)
    lb_candidates = cnt_total.get("candidates", 0)
    roofline = None
    if not args.no_profile:
        dominant = max(prof_total, key=lambda k: prof_total[k][0])
        t_ms, nl = prof_total[dominant]
        if dominant == "lb":
            # per candidate the cascade must read its series point (4 B) and its window statistics:
            # half a stored (sum, sum of squares) prefix entry (8 B: even entries only, an odd lane
            # completes the even one before it with a point it reads anyway) or the three
            # per-window values (12 B)
            per_cand = 12 if schedule["stats_prefix"] else 16
            kernel = "k_lb_batch<%s, %s>" % ("true" if schedule["stats_prefix"] else "false",
                                              "true" if schedule["data_envelope"] else "false")
            units = lb_candidates
        elif dominant == "stats":
            # blocked prefix: read 4 B, write 8 B per series point (a 16-byte entry at every
            # second point; one pass for the batch)
            per_cand, kernel, units = 12, "k_prefix", wl.T.size
        else:
            per_cand, kernel, units = None, f"class {dominant}", None
        if per_cand is not None:
            ach = units * per_cand / (t_ms * 1e-3) / 1e9
            roofline = {"bound": "hbm", "kernel": kernel, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                        "traffic": traffic_of(kernel, nl, units * per_cand / max(nl, 1)),
                        "algorithmic_bytes_per_launch": round(units * per_cand / max(nl, 1)),
                        "bytes_per_unit": per_cand, "avg_launch_ms": round(t_ms / max(nl, 1), 4), "launches": nl}
        else:
            roofline = {"bound": "latency", "kernel": kernel, "achieved": None, "peak": None, "unit": None,
                        "frac": None, "traffic": None, "avg_launch_ms": round(t_ms / max(nl, 1), 4),
                        "launches": nl}

    # ---------------------------------------------------------------- DTW kernel throughput
    # exact banded DTW (no abandoning) of many random candidates per query shape, default schedule:
    # the rate of the DTW kernel itself, which the pruned search above hardly exercises
    dtw_rate = []
    if not args.no_profile:
        rng = np.random.default_rng(11)
        # the bench queries' bands, plus the longest query with a band of 0.8 m (the wide-band
        # regime: one wave per candidate, 13 slot registers per lane)
        shapes = list(zip(Qs, ms, rs)) + [(Qs[-1], ms[-1], int(0.8 * ms[-1]))]
        for q, m, r in shapes:
            count = (1 << 20) if m <= 256 else ((1 << 18) if r <= 111 else (1 << 14))
            st = torch.from_numpy(rng.integers(0, wl.T.size - m + 1, count)).to(dev)
            ctx.dtw_band(T, q, r, st)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                ctx.dtw_band(T, q, r, st)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / 3
            g = count * cells(m, r) / dt / 1e9
            dtw_rate.append({"m": m, "r": r, "candidates": count, "ms": round(dt * 1e3, 3), "gcups": round(g, 1),
                             "frac_valu_peak": round(g / DTW_PEAK_GCUPS, 4)})

    # ---------------------------------------------------------------- CPU baseline (oracle)
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import Cascade
        casc = Cascade()
        ns = min(args.cpu_sample, wl.T.size)
        Ts = wl.T[:ns]
        t = time.perf_counter()
        for q, r in zip(wl.queries, rs):
            casc.search(Ts, q, r)
        dt = time.perf_counter() - t
        scale = (wl.T.size - np.mean(ms) + 1) / (ns - np.mean(ms) + 1)
        cpu = {"value": round(dt / nq * scale, 4), "unit": "s/query", "cores": casc.num_threads(), "kind": "oracle",
               "sample": f"C FP64 cascade oracle on the first {ns} points for each of the {nq} queries "
                         f"({dt:.2f}s), scaled linearly to n={wl.T.size}"}

    out = {
        "metric": METRIC,
        "value": round(s_per_query, 6),
        "unit": "s/query",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "n": int(wl.T.size), "m": ms, "r": rs, "mode": "batched+learned",
                   "note": wl.note},
        "batches_in_flight": args.inflight,
        "learned_one_in_flight_s_per_query": round(single_step_s / nq, 6),
        "batched_natural_s_per_query": round(natural_step_s / nq, 6) if natural_step_s else None,
        "ordering_network": {"train_series": f"random walk n={args.train_n} seed 8", "pairs": int(sum(x.shape[0] for x in Xs)),
                             "epochs": args.train_epochs, "loss_curve": [round(v, 5) for v in curve],
                             "train_s": round(train_s, 2)},
        "schedule": schedule,
        "plain_s_per_query": round(plain_s, 6) if plain_s else None,
        "batched_over_plain": round(s_per_query / plain_s, 4) if plain_s else None,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "plain_per_query_s": [round(float(np.median(per_query[i::nq])), 6) for i in range(nq)] if per_query else None,
        "batched_kernel_ms": {k: [round(v[0], 4), v[1]] for k, v in prof_total.items()},
        "dtw_throughput": dtw_rate,
        "dtw_gcups": max((d["gcups"] for d in dtw_rate), default=None),
        "dtw_frac_valu_peak": max((d["frac_valu_peak"] for d in dtw_rate), default=None),
        "search_dtw_gcups": round(dtw_cells / (prof_total["dtw"][0] * 1e-3) / 1e9, 2)
        if prof_total["dtw"][0] > 0 else None,
        "counters": cnt_total,
        "plain_profile": per_query_prof,
        "results": [[int(i), float(d)] for i, d in results],
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
