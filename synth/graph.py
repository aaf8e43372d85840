"""Python side of the graph builder (``csrc/graph_build.cpp``, built with g++).

Index construction is input generation here: the paper inherits DiskANN-style
graphs and does not describe how they are built, so both the oracle and the
GPU search simply consume the adjacency produced below.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "graph_build.cpp")
_LIB = os.path.join(_HERE, "libsynth.so")
_DT = {np.dtype(np.uint8): 1, np.dtype(np.int8): 2, np.dtype(np.float32): 3}
_lib = None


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O3", "-std=c++17", "-mavx2", "-mfma", "-shared", "-fPIC",
                               "-pthread", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        vp, i64, i32, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64
        lib.synth_build_graph.argtypes = [vp, i64, i32, i32, i32, u64, i32, i32, ctypes.c_float,
                                          i32, i64, i32, i32, vp, vp]
        lib.synth_build_graph.restype = ctypes.c_int
        lib.synth_random_graph.argtypes = [i64, i32, u64, vp]
        lib.synth_random_graph.restype = ctypes.c_int
        lib.synth_medoid.argtypes = [vp, i64, i32, i32]
        lib.synth_medoid.restype = ctypes.c_int64
        _lib = lib
    return _lib


REFINE_PASSES = 1


def _threads(t):
    return t or min(16, os.cpu_count() or 1)


def build_graph(base: np.ndarray, R: int, seed: int, threads: int = 0, pool: int | None = None,
                alpha: float = 1.2, n_hubs: int | None = None, exact_limit: int = 20000,
                passes: int = REFINE_PASSES, L_build: int | None = None):
    """Degree-R proximity graph over ``base``.  Returns (adj int32 [n, R], entry).

    `passes` Vamana-style refinement passes (greedy search of each point's own
    vector with list size `L_build`, default max(64, 3R/2), then pruning of
    the expanded nodes with alpha = 1) follow the pool-based construction;
    `alpha` applies to the initial pool pruning."""
    base = np.ascontiguousarray(base)
    n, d = base.shape
    pool = pool or max(2 * R, 64)
    if n_hubs is None:
        n_hubs = int(min(max(64, n // 1000), 4096))
    L_build = L_build or max(64, (3 * R) // 2)
    adj = np.empty((n, R), dtype=np.int32)
    entry = ctypes.c_int32(-1)
    rc = _load().synth_build_graph(base.ctypes.data_as(ctypes.c_void_p), n, d, _DT[base.dtype],
                                   R, seed, _threads(threads), pool, alpha, n_hubs, exact_limit,
                                   passes, L_build,
                                   adj.ctypes.data_as(ctypes.c_void_p), ctypes.byref(entry))
    if rc != 0:
        raise ValueError("synth_build_graph failed: %d" % rc)
    return adj, int(entry.value)


def random_graph(n: int, R: int, seed: int) -> np.ndarray:
    """Random-link graph: R distinct non-self neighbours per node."""
    adj = np.empty((n, R), dtype=np.int32)
    rc = _load().synth_random_graph(n, R, seed, adj.ctypes.data_as(ctypes.c_void_p))
    if rc != 0:
        raise ValueError("synth_random_graph failed: %d" % rc)
    return adj


def medoid(base: np.ndarray) -> int:
    base = np.ascontiguousarray(base)
    return int(_load().synth_medoid(base.ctypes.data_as(ctypes.c_void_p), base.shape[0],
                                    base.shape[1], _DT[base.dtype]))
