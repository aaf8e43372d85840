"""CPU oracle for graph best-first search with a relaxed fetch schedule.

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The oracle is plain C (``oracle.c``,
built with gcc into ``liboracle.so``) behind this ctypes wrapper; it shares no
code with the GPU library and never imports it.

What it computes is stated in ``oracle.c``: the strict best-first search of
paper section 4.1.1 and the dependency-relaxed schedule of section 4.1.2 with
an exact staleness ``delay``, (distance, id) keys, exact visited set, squared
L2 in int64 (u8/i8) or fp64 (f32).  Distances are returned as float64 for
every dtype (exact for the integer types).

With ``codebooks`` the search uses compressed navigation (paper section 2.2):
product-quantisation distances order the candidate list, and the answer is
the first k expanded nodes by exact distance.  The PQ arithmetic is fp32 in
the fixed order stated in ``oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

DTYPES = {np.dtype(np.uint8): 1, np.dtype(np.int8): 2, np.dtype(np.float32): 3}

_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (no GPU involved).  Returns the .so path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-pthread", _SRC, "-o", tmp, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


def bind(path: str):
    """Load an oracle shared library and declare its C signatures."""
    lib = ctypes.CDLL(path)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.oracle_distances.argtypes = [vp, i64, i32, i32, vp, vp]
    lib.oracle_distances.restype = ctypes.c_int
    lib.oracle_bruteforce.argtypes = [vp, i64, i32, i32, vp, i64, i32, i32, vp, vp]
    lib.oracle_bruteforce.restype = ctypes.c_int
    lib.oracle_search.argtypes = [vp, i64, i32, i32, vp, i32, i32, vp, i64,
                                  i32, i32, i32, i32, i32, i32, vp, vp, vp, vp, vp, i32]
    lib.oracle_search.restype = ctypes.c_int
    lib.oracle_search_pq.argtypes = lib.oracle_search.argtypes + [vp, i32]
    lib.oracle_search_pq.restype = ctypes.c_int
    lib.oracle_pq_encode.argtypes = [vp, i64, i32, i32, vp, i32, vp]
    lib.oracle_pq_encode.restype = ctypes.c_int
    lib.oracle_pq_table.argtypes = [vp, i32, i32, vp, i32, vp]
    lib.oracle_pq_table.restype = ctypes.c_int
    return lib


def use_library(path: str) -> None:
    """Route every call of this module through the library at ``path``."""
    global _lib
    _lib = bind(path)


def _load():
    global _lib
    if _lib is None:
        _lib = bind(build())
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check_vectors(base, queries):
    base = np.ascontiguousarray(base)
    if base.dtype not in DTYPES or base.ndim != 2:
        raise ValueError("base must be a 2-D uint8, int8 or float32 array")
    queries = np.ascontiguousarray(queries, dtype=base.dtype)
    if queries.ndim == 1:
        queries = queries.reshape(1, -1)
    if queries.shape[1] != base.shape[1]:
        raise ValueError("query dimension does not match base")
    return base, queries


def distances(base: np.ndarray, query: np.ndarray) -> np.ndarray:
    """Squared L2 distance of one query to every base row (float64)."""
    base, q = _check_vectors(base, query)
    out = np.empty(base.shape[0], dtype=np.float64)
    rc = _load().oracle_distances(_ptr(base), base.shape[0], base.shape[1],
                                  DTYPES[base.dtype], _ptr(q[0]), _ptr(out))
    if rc != 0:
        raise ValueError("oracle_distances failed: %d" % rc)
    return out


def bruteforce(base: np.ndarray, queries: np.ndarray, k: int, threads: int = 0):
    """Exact top-k by full scan.  Returns (ids int32 [nq,k], dists float64 [nq,k])."""
    base, queries = _check_vectors(base, queries)
    nq = queries.shape[0]
    ids = np.empty((nq, k), dtype=np.int32)
    dists = np.empty((nq, k), dtype=np.float64)
    threads = threads or (os.cpu_count() or 1)
    rc = _load().oracle_bruteforce(_ptr(base), base.shape[0], base.shape[1], DTYPES[base.dtype],
                                   _ptr(queries), nq, k, threads, _ptr(ids), _ptr(dists))
    if rc != 0:
        raise ValueError("oracle_bruteforce failed: %d" % rc)
    return ids, dists


def _check_codebooks(codebooks, d):
    cb = np.ascontiguousarray(codebooks, dtype=np.float32)
    if cb.ndim != 3 or cb.shape[1] != 256 or cb.shape[0] * cb.shape[2] != d:
        raise ValueError("codebooks must be [M, 256, d / M] float32")
    return cb


def pq_encode(base: np.ndarray, codebooks: np.ndarray) -> np.ndarray:
    """PQ codes [n, M] uint8 of every base row (nearest centroid per subspace)."""
    base, _ = _check_vectors(base, base[:1])
    cb = _check_codebooks(codebooks, base.shape[1])
    codes = np.empty((base.shape[0], cb.shape[0]), dtype=np.uint8)
    rc = _load().oracle_pq_encode(_ptr(base), base.shape[0], base.shape[1], DTYPES[base.dtype],
                                  _ptr(cb), cb.shape[0], _ptr(codes))
    if rc != 0:
        raise ValueError("oracle_pq_encode failed: %d" % rc)
    return codes


def pq_table(query: np.ndarray, codebooks: np.ndarray, dtype=None) -> np.ndarray:
    """Distance table [M, 256] float32 of one query."""
    q = np.ascontiguousarray(query if dtype is None else np.asarray(query, dtype=dtype))
    if q.dtype not in DTYPES or q.ndim != 1:
        raise ValueError("query must be a 1-D uint8, int8 or float32 array")
    cb = _check_codebooks(codebooks, q.shape[0])
    tab = np.empty((cb.shape[0], 256), dtype=np.float32)
    rc = _load().oracle_pq_table(_ptr(q), q.shape[0], DTYPES[q.dtype], _ptr(cb), cb.shape[0],
                                 _ptr(tab))
    if rc != 0:
        raise ValueError("oracle_pq_table failed: %d" % rc)
    return tab


def search(base: np.ndarray, adj: np.ndarray, entry: int, queries: np.ndarray, k: int,
           L: int, R: int | None = None, delay: int = 1, beam: int = 1, threads: int = 0,
           trace_cap: int = 0, codebooks: np.ndarray | None = None):
    """Best-first search, strict (delay=0) or dependency-relaxed (delay>=1).

    With ``codebooks`` ([M, 256, d/M] float32) navigation uses PQ distances and
    the answer is re-ranked by exact distance (theta then holds PQ distances).

    Returns a dict with ids [nq,k] int32, dists [nq,k] float64, steps [nq] uint32
    and, when trace_cap > 0, trace [nq,trace_cap] int32 (selected ids, -1
    padded) and theta [nq,trace_cap] float64 (L-th distance after each
    processed node; nan past the end).
    """
    base, queries = _check_vectors(base, queries)
    adj = np.ascontiguousarray(adj, dtype=np.int32)
    if adj.ndim != 2 or adj.shape[0] != base.shape[0]:
        raise ValueError("adj must be [n, stride] int32")
    R = adj.shape[1] if R is None else R
    nq = queries.shape[0]
    ids = np.empty((nq, k), dtype=np.int32)
    dists = np.empty((nq, k), dtype=np.float64)
    steps = np.empty(nq, dtype=np.uint32)
    trace = theta = None
    if trace_cap > 0:
        trace = np.empty((nq, trace_cap), dtype=np.int32)
        theta = np.empty((nq, trace_cap), dtype=np.float64)
    threads = threads or (os.cpu_count() or 1)
    args = (_ptr(base), base.shape[0], base.shape[1], DTYPES[base.dtype], _ptr(adj),
            adj.shape[1], int(entry), _ptr(queries), nq, k, L, R, delay, beam, threads,
            _ptr(ids), _ptr(dists), _ptr(steps), _ptr(trace), _ptr(theta), trace_cap)
    if codebooks is None:
        rc = _load().oracle_search(*args)
    else:
        cb = _check_codebooks(codebooks, base.shape[1])
        rc = _load().oracle_search_pq(*args, _ptr(cb), cb.shape[0])
    if rc != 0:
        raise ValueError("oracle_search failed: %d" % rc)
    out = {"ids": ids, "dists": dists, "steps": steps}
    if trace_cap > 0:
        out["trace"] = trace
        out["theta"] = theta
    return out
