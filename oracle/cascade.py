"""ctypes wrapper and gcc build step for the C cascade oracle (cascade.c).

TEST INFRASTRUCTURE (see the package docstring).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cascade.c")


def cascade_path() -> str:
    return os.path.join(_HERE, "liboracle_cascade.so")


def build_cascade() -> str:
    """Compile cascade.c with gcc (-O2, OpenMP).  Always recompiles."""
    out = cascade_path()
    tmp = out + ".tmp"
    subprocess.run(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-o", tmp, _SRC, "-lm"],
                   check=True)
    os.replace(tmp, out)
    return out


class Cascade:
    """Loaded C oracle.  Builds the library first if it is missing."""

    def __init__(self):
        path = cascade_path()
        if not os.path.exists(path):
            build_cascade()
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        lib.oc_search.argtypes = [P, ctypes.c_int64, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                  P, P, P]
        lib.oc_search.restype = ctypes.c_int
        lib.oc_dtw_starts.argtypes = [P, ctypes.c_int64, P, ctypes.c_int32, ctypes.c_int32, P,
                                      ctypes.c_int64, ctypes.c_int32, P]
        lib.oc_dtw_starts.restype = ctypes.c_int
        lib.oc_search_many.argtypes = [P, ctypes.c_int64, P, ctypes.c_int32, P, ctypes.c_int32, ctypes.c_int32,
                                       P, P, P]
        lib.oc_search_many.restype = ctypes.c_int
        lib.oc_num_threads.restype = ctypes.c_int
        self.lib = lib

    def num_threads(self) -> int:
        return int(self.lib.oc_num_threads())

    def search(self, T, Q, r: int, nthreads: int = 0):
        """Returns (index, distance, counters) with counters = candidates, pruned by LB_Kim,
        by the query-envelope bound, by the candidate-envelope bound, DTW abandoned, DTW done."""
        T = np.ascontiguousarray(T, dtype=np.float32)
        Q = np.ascontiguousarray(Q, dtype=np.float32)
        idx = ctypes.c_int64(-1)
        dist = ctypes.c_double(0.0)
        cnt = np.zeros(6, dtype=np.int64)
        rc = self.lib.oc_search(T.ctypes.data, T.size, Q.ctypes.data, Q.size, int(r), int(nthreads),
                                ctypes.addressof(idx), ctypes.addressof(dist), cnt.ctypes.data)
        if rc != 0:
            raise ValueError("oc_search rejected its arguments")
        return int(idx.value), float(dist.value), cnt

    def search_many(self, T, queries, rs, nthreads: int = 0):
        """The searches of several queries of one length in one scan of the series (each window's
        moments shared); returns [(index, distance)] in query order and the summed counters."""
        T = np.ascontiguousarray(T, dtype=np.float32)
        m = int(np.asarray(queries[0]).size)
        if any(np.asarray(q).size != m for q in queries):
            raise ValueError("search_many needs queries of one length")
        Q = np.ascontiguousarray(np.concatenate([np.asarray(q, np.float32) for q in queries]))
        r = np.ascontiguousarray(np.asarray(rs, dtype=np.int32))
        nq = len(queries)
        idx = np.empty(nq, dtype=np.int64)
        dist = np.empty(nq, dtype=np.float64)
        cnt = np.zeros(6, dtype=np.int64)
        rc = self.lib.oc_search_many(T.ctypes.data, T.size, Q.ctypes.data, m, r.ctypes.data, nq, int(nthreads),
                                     idx.ctypes.data, dist.ctypes.data, cnt.ctypes.data)
        if rc != 0:
            raise ValueError("oc_search_many rejected its arguments")
        return [(int(i), float(d)) for i, d in zip(idx, dist)], cnt

    def dtw_starts(self, T, Q, r: int, starts, nthreads: int = 0) -> np.ndarray:
        T = np.ascontiguousarray(T, dtype=np.float32)
        Q = np.ascontiguousarray(Q, dtype=np.float32)
        starts = np.ascontiguousarray(starts, dtype=np.int64)
        out = np.empty(starts.size, dtype=np.float64)
        rc = self.lib.oc_dtw_starts(T.ctypes.data, T.size, Q.ctypes.data, Q.size, int(r), starts.ctypes.data,
                                    starts.size, int(nthreads), out.ctypes.data)
        if rc != 0:
            raise ValueError("oc_dtw_starts rejected its arguments")
        return out
