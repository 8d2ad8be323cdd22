"""The allocation-free banded DTW (dtws_dtw_band_noalloc) against the context's dtws_dtw_band, through
the C ABI: two calls in a row on one device, the second with a smaller input, each compared with
the context call and with the oracle on a sample.  FP32 DTW values: |gpu - ref| <= 1e-4 ref + 1e-5."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1812_10302_amd as dtws
from paper_1812_10302_amd import workloads as W
from oracle import reference as R

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def close(gpu, ref):
    gpu, ref = np.asarray(gpu, np.float64), np.asarray(ref, np.float64)
    bad = np.abs(gpu - ref) > 1e-4 * np.abs(ref) + 1e-5
    assert not bad.any(), (int(bad.sum()), gpu[bad][:4], ref[bad][:4])


def test_noalloc_matches_context_call_twice():
    rng = np.random.default_rng(91)
    cases = [(400_000, 1024, 102, 40_000), (50_000, 96, 5, 3_000)]   # the second call is smaller
    with dtws.Context(0, max_n=400_000, max_m=1024) as ctx:
        for n, m, r, count in cases:
            print(f"noalloc case n={n} m={m} r={r} count={count}", flush=True)
            T = W.random_walk(n, 92 + m)
            Q = W.noisy_cut(T, n // 3, m, 0.1, 93)
            st = rng.integers(0, n - m + 1, count)
            st[:3] = [0, n - m, n // 3]
            Td, Qd, sd = dev(T), dev(Q), dev(st.astype(np.int64))
            out = torch.full((count,), -1.0, dtype=torch.float32, device=DEV)
            dtws.dtw_band_noalloc(Td, Qd, r, sd, out)
            want = ctx.dtw_band(Td, Qd, r, sd)
            got = out.cpu().numpy()
            close(got, want.cpu().numpy())
            pick = np.arange(0, count, max(1, count // 16))
            close(got[pick], R.distances_at(T, Q, r, st[pick]))
    assert dtws.dtw_band_noalloc is not None


def test_noalloc_rejects_over_limits():
    T = dev(W.random_walk(5_000, 94))
    Q = dev(W.random_walk(2_049, 95)[:2049])
    st = dev(np.zeros(4, np.int64))
    out = torch.empty(4, dtype=torch.float32, device=DEV)
    with pytest.raises(dtws.DtwsError):
        dtws.dtw_band_noalloc(T, Q, 10, st, out)            # m > 2048
