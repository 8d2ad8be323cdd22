"""Exact best-match subsequence search under banded, z-normalised, squared DTW on AMD MI355X.

Thin ctypes binding over the C ABI of libdtws.so (include/dtws.h).  Every step of the search
runs in the library's HIP kernels; this module only marshals arguments.  PyTorch supplies
device memory (tensors) and the current HIP stream.  There is no CPU fallback: if the library
is missing the calls raise.

    import torch, paper_1812_10302_amd as dtws
    ctx = dtws.Context(max_n=T.numel(), max_m=1024)
    index, distance = ctx.search(T_gpu, Q_gpu, r)
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdtws.so")

OK, EINVAL, ENOMEM, ENODEV, EHIP, EOVERFLOW, ENOMODEL = 0, -1, -2, -3, -4, -5, -6
ORDER_NATURAL, ORDER_RANDOM, ORDER_LEARNED, ORDER_PAA = 0, 1, 2, 3
NO_LOWER_BOUNDS = 4
PROFILE = 8
NO_GRAPH = 16
LB_SORTED = 32
KERNEL_CLASSES = ("prep", "stats", "env", "lb", "dtw", "cert", "other", "score", "dtw_wave")
MODEL_PARAMS = 74497
TRAIN_MAX_SHAPES = 8
MODEL_MAX_ROWS = 65536
MAX_M = 2048

COUNTER_FIELDS = ("candidates", "pruned_kim", "pruned_keogh_q", "pruned_keogh_d", "dtw_started",
                  "dtw_abandoned", "dtw_cells", "certified", "dtw_lane_cells", "lb_terms", "fallbacks",
                  "dtw_wave_cells", "dtw_evicted")


class Match(ctypes.Structure):
    _fields_ = [("index", ctypes.c_int64), ("distance", ctypes.c_double), ("status", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Counters(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in COUNTER_FIELDS]


class Schedule(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int64), ("lb_blocks_per_cu", ctypes.c_int32),
                ("dtw_blocks_per_cu", ctypes.c_int32), ("diag_max", ctypes.c_int32), ("band_lanes", ctypes.c_int32),
                ("stats_prefix", ctypes.c_int32), ("data_envelope", ctypes.c_int32), ("rounds", ctypes.c_int32),
                ("list_cap", ctypes.c_int32), ("lb_tile", ctypes.c_int32), ("dtw_bound", ctypes.c_int32),
                ("dtw_rows", ctypes.c_int32), ("dtw_evict", ctypes.c_int32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class TrainCfg(ctypes.Structure):
    _fields_ = [("shapes", ctypes.c_int32), ("m", ctypes.c_int32 * 8), ("r", ctypes.c_int32 * 8),
                ("queries_per_shape", ctypes.c_int32), ("random_per_query", ctypes.c_int32),
                ("near_per_query", ctypes.c_int32), ("epochs", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("init", ctypes.c_int32), ("lr", ctypes.c_float), ("lr_final", ctypes.c_float),
                ("noise_std", ctypes.c_float), ("reserved", ctypes.c_int32), ("seed", ctypes.c_uint64)]


class DtwsError(RuntimeError):
    def __init__(self, code: int, what: str, detail: str = ""):
        self.code = code
        msg = f"{what}: {_strerror(code)} ({code})"
        if detail:
            msg += f" -- {detail}"
        super().__init__(msg)


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1812_10302_amd.build`")
    # PyTorch ships its own HIP runtime under the same soname (libamdhip64.so.7).  Loading torch
    # first makes libdtws.so bind to that runtime, so the process holds a single HIP runtime and
    # torch's streams and allocations are valid in the library's calls.  Loading the library
    # first would bring in a second runtime that then hides the GPU from torch.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64, U32, U64, F32 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                  ctypes.c_uint64, ctypes.c_float)
    sig = {
        "dtws_create": ([ctypes.c_int, I64, I32, I32, ctypes.POINTER(P)], ctypes.c_int),
        "dtws_destroy": ([P], None),
        "dtws_strerror": ([ctypes.c_int], ctypes.c_char_p),
        "dtws_last_error": ([P], ctypes.c_char_p),
        "dtws_device_count": ([], ctypes.c_int),
        "dtws_get_counters": ([P, ctypes.POINTER(Counters)], ctypes.c_int),
        "dtws_get_profile": ([P, P, P], ctypes.c_int),
        "dtws_search": ([P, P, I64, P, I32, I32, U32, U64, P, ctypes.POINTER(Match)], ctypes.c_int),
        "dtws_search_batch": ([P, P, I64, P, P, P, P, I32, U32, U64, P, P], ctypes.c_int),
        "dtws_znorm_stats": ([P, P, I64, I32, P, P, P], ctypes.c_int),
        "dtws_lb_cascade": ([P, P, I64, P, I32, I32, F32, P, P, P, P, ctypes.POINTER(I64), P], ctypes.c_int),
        "dtws_dtw_band": ([P, P, I64, P, I32, I32, P, I64, F32, P, P], ctypes.c_int),
        "dtws_dtw_band_noalloc": ([P, I64, P, I32, I32, P, I64, F32, P, P], ctypes.c_int),
        "dtws_bsf_update": ([P, P, P, P, I64, P], ctypes.c_int),
        "dtws_model_init": ([P, U64], ctypes.c_int),
        "dtws_model_get": ([P, P, I64], ctypes.c_int),
        "dtws_model_set": ([P, P, I64], ctypes.c_int),
        "dtws_model_forward": ([P, P, I64, P, P], ctypes.c_int),
        "dtws_model_grad": ([P, P, P, I64, P, P, P], ctypes.c_int),
        "dtws_model_train_step": ([P, P, P, I64, F32, P, P], ctypes.c_int),
        "dtws_model_train": ([P, P, I64, ctypes.POINTER(TrainCfg), P, P, ctypes.POINTER(I64)], ctypes.c_int),
        "dtws_model_save": ([P, P, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "dtws_model_load": ([P, P, ctypes.c_size_t], ctypes.c_int),
        "dtws_paa": ([P, P, I64, I32, P, I64, P, P], ctypes.c_int),
        "dtws_propose": ([P, P, I64, P, I32, P, P, I64, ctypes.POINTER(I64), P], ctypes.c_int),
        "dtws_get_schedule": ([P, ctypes.POINTER(Schedule)], ctypes.c_int),
        "dtws_set_schedule": ([P, ctypes.POINTER(Schedule)], ctypes.c_int),
        "dtws_autotune_batch": ([P, P, I64, P, P, P, P, I32, U32, U64, P, I32, ctypes.POINTER(Schedule),
                                 ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def library():
    """The loaded ctypes library (raises ImportError when it has not been built)."""
    return _load()


def _strerror(code: int) -> str:
    try:
        return _load().dtws_strerror(code).decode()
    except ImportError:
        return "error"


def device_count() -> int:
    return int(_load().dtws_device_count())


def dtw_band_noalloc(T, Q, r: int, starts, out, abandon_at: float = math.inf):
    """dtws_dtw_band_noalloc: FP32 banded DTW of the normalised query against the candidates at
    `starts` (int64 CUDA tensor) into `out` (float32 CUDA tensor, caller-allocated), on T's device,
    without a context and without device allocation."""
    torch = _torch()
    _dev_f32(T, "T")
    _dev_f32(Q, "Q")
    _dev_f32(out, "out")
    if starts.dtype != torch.int64 or not starts.is_cuda or not starts.is_contiguous():
        raise TypeError("starts must be a contiguous int64 CUDA tensor")
    if out.numel() < starts.numel():
        raise ValueError("out holds fewer values than starts")
    with torch.cuda.device(T.device):
        rc = _load().dtws_dtw_band_noalloc(T.data_ptr(), T.numel(), Q.data_ptr(), Q.numel(), int(r), starts.data_ptr(),
                                           starts.numel(), float(abandon_at), out.data_ptr(), _stream(T))
    if rc != OK:
        raise DtwsError(rc, "dtws_dtw_band_noalloc")
    return out


def band(m: int, frac: float) -> int:
    """Band in points for a band given as a fraction of the query length (floor)."""
    return int(math.floor(frac * m))


def _torch():
    import torch
    return torch


def _dev_f32(x, name):
    torch = _torch()
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if x.dtype != torch.float32 or not x.is_contiguous() or x.dim() != 1:
        raise TypeError(f"{name} must be a contiguous 1-D float32 tensor")
    return x


def _stream(t):
    return ctypes.c_void_p(_torch().cuda.current_stream(t.device).cuda_stream)


class PackedQueries:
    """Queries packed back to back in one device tensor.  Reusing the same object in repeated
    batched calls keeps every pointer stable, so the library replays its captured graph."""

    def __init__(self, queries):
        torch = _torch()
        qs = [q.reshape(-1) for q in queries]
        self.packed = torch.cat(qs).contiguous()
        _dev_f32(self.packed, "queries")
        self.ms = np.array([q.numel() for q in qs], np.int32)
        self.offsets = np.zeros(len(qs), np.int64)
        self.offsets[1:] = np.cumsum(self.ms.astype(np.int64))[:-1]

    def __len__(self):
        return int(self.ms.size)


class Context:
    """A search context on one GPU; owns all device scratch (sized by max_n, max_m, max_queries)."""

    def __init__(self, device: int = 0, max_n: int = 1 << 20, max_m: int = MAX_M, max_queries: int = 1):
        L = _load()
        h = ctypes.c_void_p()
        rc = L.dtws_create(int(device), int(max_n), int(max_m), int(max_queries), ctypes.byref(h))
        if rc != OK:
            raise DtwsError(rc, "dtws_create")
        self._h = h
        self.device, self.max_n, self.max_m, self.max_queries = device, max_n, max_m, max_queries

    def close(self):
        if getattr(self, "_h", None):
            _load().dtws_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _check(self, rc: int, what: str):
        if rc != OK:
            raise DtwsError(rc, what, _load().dtws_last_error(self._h).decode())

    # ------------------------------------------------------------------ search
    def search(self, T, Q, r: int, flags: int = ORDER_NATURAL, seed: int = 0):
        """Best match of Q in T with band r: (0-based start, squared z-normalised DTW distance)."""
        _dev_f32(T, "T")
        _dev_f32(Q, "Q")
        out = Match()
        rc = _load().dtws_search(self._h, T.data_ptr(), T.numel(), Q.data_ptr(), Q.numel(), int(r), int(flags),
                                 int(seed), _stream(T), ctypes.byref(out))
        self._check(rc, "dtws_search")
        return int(out.index), float(out.distance)

    def search_batch(self, T, queries, rs, flags: int = ORDER_NATURAL, seed: int = 0):
        """Best matches of several queries (a list of 1-D float32 tensors, or PackedQueries) in one
        batched search; returns a list of (index, distance) pairs."""
        _dev_f32(T, "T")
        pq = queries if isinstance(queries, PackedQueries) else PackedQueries(queries)
        nq = len(pq)
        rr = np.array([int(x) for x in rs], np.int32)
        if rr.size != nq:
            raise ValueError("one band per query")
        out = (Match * nq)()
        rc = _load().dtws_search_batch(self._h, T.data_ptr(), T.numel(), pq.packed.data_ptr(), pq.offsets.ctypes.data,
                                       pq.ms.ctypes.data, rr.ctypes.data, nq, int(flags), int(seed), _stream(T),
                                       ctypes.cast(out, ctypes.c_void_p))
        self._check(rc, "dtws_search_batch")
        return [(int(o.index), float(o.distance)) for o in out]

    def counters(self) -> dict:
        c = Counters()
        self._check(_load().dtws_get_counters(self._h, ctypes.byref(c)), "dtws_get_counters")
        return {f: int(getattr(c, f)) for f in COUNTER_FIELDS}

    def profile(self) -> dict:
        """{class: (milliseconds, launches)} of the last search run with the PROFILE flag."""
        ms = np.zeros(len(KERNEL_CLASSES), np.float64)
        nl = np.zeros(len(KERNEL_CLASSES), np.int64)
        self._check(_load().dtws_get_profile(self._h, ms.ctypes.data, nl.ctypes.data), "dtws_get_profile")
        return {k: (float(ms[i]), int(nl[i])) for i, k in enumerate(KERNEL_CLASSES)}

    # ------------------------------------------------------------------ stages
    def znorm_stats(self, T, m: int):
        """(mu, sigma) of every length-m window, FP64 tensors of n-m+1 elements."""
        torch = _torch()
        _dev_f32(T, "T")
        N = T.numel() - m + 1
        mu = torch.empty(max(N, 1), dtype=torch.float64, device=T.device)
        sg = torch.empty_like(mu)
        rc = _load().dtws_znorm_stats(self._h, T.data_ptr(), T.numel(), int(m), mu.data_ptr(), sg.data_ptr(),
                                      _stream(T))
        self._check(rc, "dtws_znorm_stats")
        return mu[:N], sg[:N]

    def lb_cascade(self, T, Q, r: int, values: bool = True, threshold: float = math.inf, survivors: bool = False):
        """Bound values (kim, keogh_q, keogh_d) of every candidate and/or the survivors' starts."""
        torch = _torch()
        _dev_f32(T, "T")
        _dev_f32(Q, "Q")
        N = T.numel() - Q.numel() + 1
        kim = kq = kd = None
        ptrs = [None, None, None]
        if values:
            kim, kq, kd = (torch.empty(max(N, 1), dtype=torch.float32, device=T.device) for _ in range(3))
            ptrs = [kim.data_ptr(), kq.data_ptr(), kd.data_ptr()]
        surv = None
        nsurv = ctypes.c_int64(0)
        if survivors:
            surv = torch.empty(max(N, 1), dtype=torch.int32, device=T.device)
        rc = _load().dtws_lb_cascade(self._h, T.data_ptr(), T.numel(), Q.data_ptr(), Q.numel(), int(r),
                                     float(threshold), *ptrs, surv.data_ptr() if survivors else None,
                                     ctypes.byref(nsurv) if survivors else None, _stream(T))
        self._check(rc, "dtws_lb_cascade")
        res = {}
        if values:
            res.update(kim=kim[:N], keogh_q=kq[:N], keogh_d=kd[:N])
        if survivors:
            res["survivors"] = surv[:nsurv.value]
        return res

    def dtw_band(self, T, Q, r: int, starts, abandon_at: float = math.inf):
        """FP32 banded DTW of the normalised query against the candidates at `starts` (int64 tensor)."""
        torch = _torch()
        _dev_f32(T, "T")
        _dev_f32(Q, "Q")
        if starts.dtype != torch.int64 or not starts.is_cuda or not starts.is_contiguous():
            raise TypeError("starts must be a contiguous int64 CUDA tensor")
        out = torch.empty(max(starts.numel(), 1), dtype=torch.float32, device=T.device)
        rc = _load().dtws_dtw_band(self._h, T.data_ptr(), T.numel(), Q.data_ptr(), Q.numel(), int(r),
                                   starts.data_ptr(), starts.numel(), float(abandon_at), out.data_ptr(),
                                   _stream(T))
        self._check(rc, "dtws_dtw_band")
        return out[:starts.numel()]

    # ------------------------------------------------------------------ ordering network
    def model_init(self, seed: int = 0):
        self._check(_load().dtws_model_init(self._h, int(seed)), "dtws_model_init")

    def model_get(self) -> np.ndarray:
        out = np.empty(MODEL_PARAMS, np.float32)
        self._check(_load().dtws_model_get(self._h, out.ctypes.data, MODEL_PARAMS), "dtws_model_get")
        return out

    def model_set(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != MODEL_PARAMS:
            raise ValueError(f"expected {MODEL_PARAMS} parameters")
        self._check(_load().dtws_model_set(self._h, p.ctypes.data, MODEL_PARAMS), "dtws_model_set")

    def model_forward(self, X):
        """Predictions for feature rows X (float32 CUDA tensor, rows x 32)."""
        torch = _torch()
        X = X.contiguous()
        y = torch.empty(max(X.shape[0], 1), dtype=torch.float32, device=X.device)
        self._check(_load().dtws_model_forward(self._h, X.data_ptr(), X.shape[0], y.data_ptr(), _stream(X)),
                    "dtws_model_forward")
        return y[:X.shape[0]]

    def model_grad(self, X, t):
        """(gradient of the mean squared error as a CUDA tensor, loss)."""
        torch = _torch()
        X, t = X.contiguous(), t.contiguous()
        g = torch.empty(MODEL_PARAMS, dtype=torch.float32, device=X.device)
        loss = ctypes.c_float(0.0)
        self._check(_load().dtws_model_grad(self._h, X.data_ptr(), t.data_ptr(), X.shape[0], g.data_ptr(),
                                            ctypes.byref(loss), _stream(X)), "dtws_model_grad")
        return g, float(loss.value)

    def model_train_step(self, X, t, lr: float, want_loss: bool = True):
        loss = ctypes.c_float(0.0)
        self._check(_load().dtws_model_train_step(self._h, X.data_ptr(), t.data_ptr(), X.shape[0], float(lr),
                                                  ctypes.byref(loss) if want_loss else None, _stream(X)),
                    "dtws_model_train_step")
        return float(loss.value) if want_loss else None

    def model_train(self, T, shapes, queries_per_shape: int, epochs: int, seed: int = 0, random_per_query: int = 256,
                    near_per_query: int = 32, batch: int = 4096, lr: float = 1e-3, lr_final: float | None = None,
                    noise_std: float = 0.1, init: bool = True):
        """Train the ordering network in the library (dtws_model_train) on pairs drawn from the
        training series T (float32 CUDA tensor) for the (m, r) shapes; returns (per-epoch mean
        loss, number of pairs)."""
        _dev_f32(T, "T")
        shapes = list(shapes)
        if not 1 <= len(shapes) <= TRAIN_MAX_SHAPES:
            raise ValueError(f"1 to {TRAIN_MAX_SHAPES} (m, r) shapes")
        cfg = TrainCfg()
        cfg.shapes = len(shapes)
        for k, (m, r) in enumerate(shapes):
            cfg.m[k], cfg.r[k] = int(m), int(r)
        cfg.queries_per_shape, cfg.random_per_query, cfg.near_per_query = int(queries_per_shape), int(
            random_per_query), int(near_per_query)
        cfg.epochs, cfg.batch, cfg.init = int(epochs), int(batch), 1 if init else 0
        cfg.lr, cfg.lr_final = float(lr), float(lr / 10 if lr_final is None else lr_final)
        cfg.noise_std, cfg.seed = float(noise_std), int(seed)
        curve = np.zeros(max(int(epochs), 1), np.float32)
        pairs = ctypes.c_int64(0)
        self._check(_load().dtws_model_train(self._h, T.data_ptr(), T.numel(), ctypes.byref(cfg), _stream(T),
                                             curve.ctypes.data, ctypes.byref(pairs)), "dtws_model_train")
        return [float(v) for v in curve[:int(epochs)]], int(pairs.value)

    def model_save(self) -> bytes:
        """The trained model as bytes (header with a content hash, then the FP32 parameters)."""
        size = ctypes.c_size_t(0)
        lib = _load()
        self._check(lib.dtws_model_save(self._h, None, ctypes.byref(size)), "dtws_model_save")
        buf = ctypes.create_string_buffer(size.value)
        self._check(lib.dtws_model_save(self._h, ctypes.cast(buf, ctypes.c_void_p), ctypes.byref(size)),
                    "dtws_model_save")
        return buf.raw[:size.value]

    def model_load(self, blob: bytes):
        buf = ctypes.create_string_buffer(bytes(blob), len(blob))
        self._check(_load().dtws_model_load(self._h, ctypes.cast(buf, ctypes.c_void_p), len(blob)), "dtws_model_load")

    def paa(self, T, m: int, starts):
        """16-segment PAA of the normalised windows T[s:s+m] (rows x 16 float32 CUDA tensor)."""
        torch = _torch()
        _dev_f32(T, "T")
        out = torch.empty((max(starts.numel(), 1), 16), dtype=torch.float32, device=T.device)
        self._check(_load().dtws_paa(self._h, T.data_ptr(), T.numel(), int(m), starts.data_ptr(), starts.numel(),
                                     out.data_ptr(), _stream(T)), "dtws_paa")
        return out[:starts.numel()]

    def propose(self, T, Q):
        """Proposals of every quarter block for query Q: (starts int64, features rows x 32)."""
        torch = _torch()
        _dev_f32(T, "T")
        _dev_f32(Q, "Q")
        rows = ctypes.c_int64(0)
        lib = _load()
        self._check(lib.dtws_propose(self._h, T.data_ptr(), T.numel(), Q.data_ptr(), Q.numel(), None, None, 0,
                                     ctypes.byref(rows), _stream(T)), "dtws_propose")
        starts = torch.empty(max(rows.value, 1), dtype=torch.int64, device=T.device)
        X = torch.empty((max(rows.value, 1), 32), dtype=torch.float32, device=T.device)
        self._check(lib.dtws_propose(self._h, T.data_ptr(), T.numel(), Q.data_ptr(), Q.numel(), starts.data_ptr(),
                                     X.data_ptr(), rows.value, ctypes.byref(rows), _stream(T)), "dtws_propose")
        return starts[:rows.value], X[:rows.value]

    def get_schedule(self) -> dict:
        """Launch schedule in effect (block, lb_blocks_per_cu, dtw_blocks_per_cu, diag_max, band_lanes)."""
        sc = Schedule()
        self._check(_load().dtws_get_schedule(self._h, ctypes.byref(sc)), "dtws_get_schedule")
        return sc.as_dict()

    def set_schedule(self, **fields):
        """Change some schedule fields (the others keep their current values)."""
        cur = self.get_schedule()
        unknown = set(fields) - set(cur)
        if unknown:
            raise ValueError(f"unknown schedule fields {sorted(unknown)}")
        cur.update(fields)
        sc = Schedule(**cur)
        self._check(_load().dtws_set_schedule(self._h, ctypes.byref(sc)), "dtws_set_schedule")

    def autotune_batch(self, T, queries, rs, flags: int = ORDER_NATURAL, seed: int = 0, reps: int = 3):
        """Pick and install the fastest schedule for this batch; returns (schedule dict, ms per call)."""
        _dev_f32(T, "T")
        pq = queries if isinstance(queries, PackedQueries) else PackedQueries(queries)
        rr = np.array([int(x) for x in rs], np.int32)
        if rr.size != len(pq):
            raise ValueError("one band per query")
        sc = Schedule()
        ms = ctypes.c_double(0.0)
        self._check(_load().dtws_autotune_batch(self._h, T.data_ptr(), T.numel(), pq.packed.data_ptr(),
                                                pq.offsets.ctypes.data, pq.ms.ctypes.data, rr.ctypes.data,
                                                len(pq), int(flags), int(seed), _stream(T), int(reps),
                                                ctypes.byref(sc), ctypes.byref(ms)), "dtws_autotune_batch")
        return sc.as_dict(), float(ms.value)

    def bsf_update(self, keys, d, idx):
        """Atomically lower keys[0] to the minimum packed (distance, index) key."""
        rc = _load().dtws_bsf_update(self._h, keys.data_ptr(), d.data_ptr(), idx.data_ptr(), d.numel(),
                                     _stream(d))
        self._check(rc, "dtws_bsf_update")
        return keys


def unpack_key(key: int):
    """(distance, index) of a packed best-so-far key."""
    d = np.array([key >> 32], dtype=np.uint32).view(np.float32)[0]
    return float(d), int(key & 0xFFFFFFFF)
