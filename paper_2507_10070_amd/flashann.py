"""ctypes binding of ``libflashann.so`` (C ABI in ``include/flashann.h``).

Argument marshalling only: every step of the search runs in the HIP
kernels.  PyTorch provides device memory and the current stream.  If the
library is missing, every entry point raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libflashann.so")

ANN_ERRORS = {0: "ANN_OK", -5: "ANN_EIO", -12: "ANN_ENOMEM", -16: "ANN_EBUSY",
              -19: "ANN_ENODEV", -22: "ANN_EINVAL", -95: "ANN_ENOTSUP", -110: "ANN_ETIMEDOUT"}
DTYPE_CODES = {np.dtype(np.uint8): 1, np.dtype(np.int8): 2, np.dtype(np.float32): 3}
TIER_HBM, TIER_HOST, TIER_FILE = 0, 1, 2

TRANSPORT_AUTO, TRANSPORT_DIRECT, TRANSPORT_AGENT = 0, 1, 2
SYNC_QUERY, SYNC_KERNEL = 0, 1
NAV_FULL, NAV_PQ = 0, 1
PQ_AUTO, PQ_TABLE, PQ_CACHE = 0, 1, 2
PQ_DROP_NAV = 1

EXPORTED = ["ann_index_create", "ann_index_info_get", "ann_search", "ann_index_free",
            "ann_last_error", "ann_device_clock_khz", "ann_save_index", "ann_build_index",
            "ann_load_records", "ann_agent_configure", "ann_agent_stats", "ann_search_graph",
            "ann_graph_launch", "ann_graph_free", "ann_server_open", "ann_server_submit",
            "ann_server_poll", "ann_server_stats_get", "ann_server_close", "ann_clock_us",
            "ann_server_submit_batch", "ann_server_poll_into", "ann_index_set_pq",
            "ann_index_pq_codes", "ann_search_noalloc", "ann_save_records_striped",
            "ann_load_records_striped", "ann_agent_profile_get", "ann_index_set_record_cache"]


class AnnError(RuntimeError):
    def __init__(self, code, message):
        super().__init__("%s (%d): %s" % (ANN_ERRORS.get(code, "?"), code, message))
        self.code = code


class SearchOptions(ctypes.Structure):
    _fields_ = [("delay", ctypes.c_int32), ("beam_width", ctypes.c_int32),
                ("hash_bits", ctypes.c_int32), ("waves_per_block", ctypes.c_int32),
                ("d_stats", ctypes.c_void_p), ("d_trace", ctypes.c_void_p),
                ("trace_cap", ctypes.c_int32), ("d_times", ctypes.c_void_p),
                ("d_phases", ctypes.c_void_p), ("transport", ctypes.c_int32),
                ("spin_limit", ctypes.c_uint32), ("d_L", ctypes.c_void_p),
                ("d_k", ctypes.c_void_p), ("d_order", ctypes.c_void_p),
                ("persistent", ctypes.c_int32), ("sync_grain", ctypes.c_int32),
                ("navigation", ctypes.c_int32), ("pq_scoring", ctypes.c_int32),
                ("poll_backoff", ctypes.c_int32), ("query_lanes", ctypes.c_int32)]


class IndexInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("d", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("R", ctypes.c_int32), ("entry", ctypes.c_int32), ("slot_bytes", ctypes.c_int32),
                ("tier", ctypes.c_int32), ("nav_stride", ctypes.c_int32),
                ("rec_bytes", ctypes.c_int32), ("hbm_bytes", ctypes.c_int64),
                ("direct_io", ctypes.c_int32), ("pq_m", ctypes.c_int32),
                ("nav_full", ctypes.c_int32), ("stripes", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("cached_records", ctypes.c_int64)]


class AgentProfile(ctypes.Structure):
    _fields_ = [(f, ctypes.c_uint64) for f in ("requests", "bytes", "errors", "passes",
                                                "busy_passes", "scan_ns", "copy_ns", "io_ns",
                                                "max_batch")] + \
               [("threads", ctypes.c_int32), ("async_io", ctypes.c_int32),
                ("stripes", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("stripe_requests", ctypes.c_uint64 * 16)]


class ServerOptions(ctypes.Structure):
    _fields_ = [("k_max", ctypes.c_int32), ("L_max", ctypes.c_int32), ("delay", ctypes.c_int32),
                ("waves_per_block", ctypes.c_int32), ("hash_bits", ctypes.c_int32),
                ("queue_cap", ctypes.c_int32), ("idle_polls", ctypes.c_int32),
                ("beam_width", ctypes.c_int32), ("transport", ctypes.c_int32),
                ("spin_limit", ctypes.c_uint32),
                ("navigation", ctypes.c_int32), ("pq_scoring", ctypes.c_int32),
                ("first_ticket", ctypes.c_uint64)]


class Result(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int32), ("k", ctypes.c_int32),
                ("ids", ctypes.c_void_p), ("dists", ctypes.c_void_p), ("steps", ctypes.c_uint32),
                ("submit_us", ctypes.c_double), ("done_us", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("admitted", ctypes.c_uint64),
                ("completed", ctypes.c_uint64), ("relaunches", ctypes.c_uint64),
                ("max_inflight", ctypes.c_int64), ("slots", ctypes.c_int64),
                ("resident_waves", ctypes.c_int64)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("%s is not built: run __graft_entry__.build() first" % path)
    lib = ctypes.CDLL(path)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.ann_index_create.argtypes = [vp, vp, i64, i32, i32, i32, i32, i32, i32,
                                     ctypes.POINTER(vp)]
    lib.ann_index_create.restype = ctypes.c_int
    lib.ann_index_info_get.argtypes = [vp, ctypes.POINTER(IndexInfo)]
    lib.ann_index_info_get.restype = ctypes.c_int
    lib.ann_search.argtypes = [vp, vp, i64, i32, i32, i32, ctypes.POINTER(SearchOptions),
                               vp, vp, vp, vp]
    lib.ann_search.restype = ctypes.c_int
    lib.ann_search_noalloc.argtypes = lib.ann_search.argtypes
    lib.ann_search_noalloc.restype = ctypes.c_int
    lib.ann_index_free.argtypes = [vp]
    lib.ann_index_free.restype = ctypes.c_int
    cp, u64p = ctypes.c_char_p, ctypes.POINTER(ctypes.c_uint64)
    lib.ann_save_index.argtypes = [cp, vp, vp, i64, i32, i32, i32, i32, i32]
    lib.ann_save_index.restype = ctypes.c_int
    lib.ann_build_index.argtypes = [vp, i64, i32, i32, i32, i32, ctypes.c_uint64, cp]
    lib.ann_build_index.restype = ctypes.c_int
    lib.ann_load_records.argtypes = [cp, i32, cp, ctypes.POINTER(vp)]
    lib.ann_load_records.restype = ctypes.c_int
    lib.ann_agent_configure.argtypes = [vp, i32, i32, i32, i32, i32]
    lib.ann_agent_configure.restype = ctypes.c_int
    lib.ann_agent_stats.argtypes = [vp, u64p, u64p, u64p]
    lib.ann_agent_stats.restype = ctypes.c_int
    lib.ann_agent_profile_get.argtypes = [vp, ctypes.POINTER(AgentProfile)]
    lib.ann_agent_profile_get.restype = ctypes.c_int
    lib.ann_save_records_striped.argtypes = [vp, vp, i64, i32, i32, i32, i32,
                                             ctypes.POINTER(cp), i32]
    lib.ann_save_records_striped.restype = ctypes.c_int
    lib.ann_load_records_striped.argtypes = [cp, i32, ctypes.POINTER(cp), i32, ctypes.POINTER(vp)]
    lib.ann_load_records_striped.restype = ctypes.c_int
    lib.ann_index_set_pq.argtypes = [vp, vp, i32, i32]
    lib.ann_index_set_pq.restype = ctypes.c_int
    lib.ann_index_set_record_cache.argtypes = [vp, vp, i64]
    lib.ann_index_set_record_cache.restype = ctypes.c_int
    lib.ann_index_pq_codes.argtypes = [vp, vp]
    lib.ann_index_pq_codes.restype = ctypes.c_int
    lib.ann_search_graph.argtypes = [vp, vp, i64, i32, i32, i32, ctypes.POINTER(SearchOptions),
                                     vp, vp, vp, vp, ctypes.POINTER(vp)]
    lib.ann_search_graph.restype = ctypes.c_int
    lib.ann_graph_launch.argtypes = [vp, vp]
    lib.ann_graph_launch.restype = ctypes.c_int
    lib.ann_graph_free.argtypes = [vp]
    lib.ann_graph_free.restype = ctypes.c_int
    lib.ann_server_open.argtypes = [vp, ctypes.c_size_t, ctypes.POINTER(ServerOptions),
                                    ctypes.POINTER(vp)]
    lib.ann_server_open.restype = ctypes.c_int
    lib.ann_server_submit.argtypes = [vp, vp, i32, i32, ctypes.c_uint64]
    lib.ann_server_submit.restype = ctypes.c_int
    lib.ann_server_submit_batch.argtypes = [vp, vp, i64, vp, vp, vp, vp]
    lib.ann_server_submit_batch.restype = ctypes.c_int
    lib.ann_server_poll_into.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp,
                                         ctypes.POINTER(i32), i32]
    lib.ann_server_poll_into.restype = ctypes.c_int
    lib.ann_server_poll.argtypes = [vp, ctypes.POINTER(Result), i32, ctypes.POINTER(i32), i32]
    lib.ann_server_poll.restype = ctypes.c_int
    lib.ann_server_stats_get.argtypes = [vp, ctypes.POINTER(ServerStats)]
    lib.ann_server_stats_get.restype = ctypes.c_int
    lib.ann_server_close.argtypes = [vp]
    lib.ann_server_close.restype = ctypes.c_int
    lib.ann_clock_us.argtypes = []
    lib.ann_clock_us.restype = ctypes.c_double
    lib.ann_device_clock_khz.argtypes = [ctypes.POINTER(ctypes.c_int32)]
    lib.ann_device_clock_khz.restype = ctypes.c_int
    lib.ann_last_error.argtypes = []
    lib.ann_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(rc):
    if rc != 0:
        raise AnnError(rc, load_library().ann_last_error().decode(errors="replace"))


def device_clock_khz() -> int:
    """Frequency of the device wall clock that stamps per-query times."""
    v = ctypes.c_int32()
    _check(load_library().ann_device_clock_khz(ctypes.byref(v)))
    return v.value


def save_index(path: str, vectors: np.ndarray, adjacency: np.ndarray, entry: int,
               slot_bytes: int) -> None:
    """ann_save_index: write meta.json, vectors.bin and records.bin."""
    vectors = np.ascontiguousarray(vectors)
    adjacency = np.ascontiguousarray(adjacency, dtype=np.int32)
    _check(load_library().ann_save_index(path.encode(), vectors.ctypes.data, adjacency.ctypes.data,
                                         vectors.shape[0], vectors.shape[1],
                                         DTYPE_CODES[vectors.dtype], adjacency.shape[1], int(entry),
                                         int(slot_bytes)))


def save_records_striped(vectors: np.ndarray, adjacency: np.ndarray, slot_bytes: int,
                         stripe_paths) -> None:
    """ann_save_records_striped: record v goes to slot v // S of file v % S."""
    vectors = np.ascontiguousarray(vectors)
    adjacency = np.ascontiguousarray(adjacency, dtype=np.int32)
    arr = (ctypes.c_char_p * len(stripe_paths))(*[p.encode() for p in stripe_paths])
    _check(load_library().ann_save_records_striped(
        vectors.ctypes.data, adjacency.ctypes.data, vectors.shape[0], vectors.shape[1],
        DTYPE_CODES[vectors.dtype], adjacency.shape[1], int(slot_bytes), arr, len(stripe_paths)))


def build_index(path: str, vectors: np.ndarray, R: int, slot_bytes: int, seed: int) -> None:
    """ann_build_index: construct the graph and write the index directory."""
    vectors = np.ascontiguousarray(vectors)
    _check(load_library().ann_build_index(vectors.ctypes.data, vectors.shape[0], vectors.shape[1],
                                          DTYPE_CODES[vectors.dtype], int(R), int(slot_bytes),
                                          int(seed), path.encode()))


_CODE_DTYPES = {v: k for k, v in DTYPE_CODES.items()}


class Index:
    """A searchable index: navigation copy in HBM plus records in a tier."""

    @classmethod
    def load(cls, path: str, tier: int = TIER_HBM, records_path: str | None = None) -> "Index":
        """ann_load_records: open an index directory written by save/build_index."""
        self = cls.__new__(cls)
        self._h = None
        h = ctypes.c_void_p()
        _check(load_library().ann_load_records(path.encode(), int(tier),
                                               records_path.encode() if records_path else None,
                                               ctypes.byref(h)))
        self._h = h
        info = self.info()
        self.dtype = _CODE_DTYPES[info["dtype"]]
        self.d = info["d"]
        return self

    def configure_agent(self, threads: int = 0, delay_node: int = -1, delay_us: int = 0,
                        fail_node: int = -1, drop_node: int = -1) -> None:
        _check(load_library().ann_agent_configure(self.handle, threads, delay_node, delay_us,
                                                  fail_node, drop_node))

    def agent_stats(self) -> dict:
        r, b, e = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        _check(load_library().ann_agent_stats(self.handle, ctypes.byref(r), ctypes.byref(b),
                                              ctypes.byref(e)))
        return {"requests": r.value, "bytes": b.value, "errors": e.value}

    def agent_profile(self) -> dict:
        """ann_agent_profile_get: counters and time split of the agent threads."""
        p = AgentProfile()
        _check(load_library().ann_agent_profile_get(self.handle, ctypes.byref(p)))
        out = {f: getattr(p, f) for f, _ in AgentProfile._fields_
               if f not in ("reserved", "stripe_requests")}
        out["stripe_requests"] = list(p.stripe_requests)[:max(1, p.stripes)]
        return out

    @classmethod
    def load_striped(cls, path: str, stripe_paths, tier: int = TIER_FILE) -> "Index":
        """ann_load_records_striped: an index directory whose records are
        striped over the files `stripe_paths` (record v in file v % S)."""
        self = cls.__new__(cls)
        self._h = None
        arr = (ctypes.c_char_p * len(stripe_paths))(*[p.encode() for p in stripe_paths])
        h = ctypes.c_void_p()
        _check(load_library().ann_load_records_striped(path.encode(), int(tier), arr,
                                                       len(stripe_paths), ctypes.byref(h)))
        self._h = h
        info = self.info()
        self.dtype = _CODE_DTYPES[info["dtype"]]
        self.d = info["d"]
        return self

    def __init__(self, vectors: np.ndarray, adjacency: np.ndarray, entry: int,
                 slot_bytes: int, tier: int = TIER_HBM):
        lib = load_library()
        vectors = np.ascontiguousarray(vectors)
        adjacency = np.ascontiguousarray(adjacency, dtype=np.int32)
        if vectors.dtype not in DTYPE_CODES or vectors.ndim != 2:
            raise ValueError("vectors must be a 2-D uint8, int8 or float32 array")
        if adjacency.ndim != 2 or adjacency.shape[0] != vectors.shape[0]:
            raise ValueError("adjacency must be [n, R] int32")
        self.dtype = vectors.dtype
        self.d = vectors.shape[1]
        h = ctypes.c_void_p()
        _check(lib.ann_index_create(vectors.ctypes.data, adjacency.ctypes.data,
                                    vectors.shape[0], vectors.shape[1], DTYPE_CODES[vectors.dtype],
                                    adjacency.shape[1], int(entry), int(slot_bytes), int(tier),
                                    ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("index is closed")
        return self._h

    def set_pq(self, codebooks: np.ndarray, drop_nav: bool = False) -> None:
        """ann_index_set_pq: encode the base with `codebooks` ([M, 256, d/M]
        float32) into PQ codes in HBM, for searches with navigation=NAV_PQ."""
        cb = np.ascontiguousarray(codebooks, dtype=np.float32)
        if cb.ndim != 3 or cb.shape[1] != 256 or cb.shape[0] * cb.shape[2] != self.d:
            raise ValueError("codebooks must be [M, 256, d / M] float32")
        _check(load_library().ann_index_set_pq(self.handle, cb.ctypes.data, cb.shape[0],
                                               PQ_DROP_NAV if drop_nav else 0))

    def set_record_cache(self, ids) -> None:
        """ann_index_set_record_cache: keep copies of the records of nodes
        `ids` (distinct, host int array) in device memory; batch searches
        read those records there (the agents get no request for them).
        Results do not change.  An empty array releases the cache."""
        a = np.ascontiguousarray(np.asarray(ids).reshape(-1), dtype=np.int32)
        _check(load_library().ann_index_set_record_cache(self.handle,
                                                         a.ctypes.data if a.size else None,
                                                         int(a.size)))

    def pq_codes(self) -> np.ndarray:
        """ann_index_pq_codes: the PQ codes, [n, M] uint8 on the host."""
        info = self.info()
        out = np.empty((info["n"], info["pq_m"]), dtype=np.uint8)
        _check(load_library().ann_index_pq_codes(self.handle, out.ctypes.data))
        return out

    def info(self) -> dict:
        out = IndexInfo()
        _check(load_library().ann_index_info_get(self.handle, ctypes.byref(out)))
        return {f: getattr(out, f) for f, _ in IndexInfo._fields_}

    def close(self):
        """Release the index; AnnError (ANN_EBUSY) while a server on it is open."""
        if getattr(self, "_h", None) is not None:
            _check(load_library().ann_index_free(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass  # still in use by an open server: the server keeps a reference

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def _ptr(t):
    return t.data_ptr() if t is not None else None


def _check_buffer(name, t, dtypes, numel, dev):
    if t.dtype not in dtypes or not t.is_cuda or t.device != dev or not t.is_contiguous() \
            or t.numel() != numel:
        raise ValueError("%s must be a contiguous %s tensor of %d elements on %s (got %s %s on %s)"
                         % (name, "/".join(str(d) for d in dtypes), numel, dev, t.dtype,
                            tuple(t.shape), t.device))


def _prepare(index, queries, k, L, R, delay, beam_width, hash_bits, waves_per_block, stats,
             trace, times, phases, transport, spin_limit, L_per_query, k_per_query, order,
             persistent, out, sync_grain=0, navigation=NAV_FULL, pq_scoring=PQ_AUTO,
             poll_backoff=0, query_lanes=0):
    import torch

    if queries.dim() != 2 or queries.shape[1] != index.d:
        raise ValueError("queries must be [nq, %d]" % index.d)
    want = {np.dtype(np.uint8): torch.uint8, np.dtype(np.int8): torch.int8,
            np.dtype(np.float32): torch.float32}[index.dtype]
    if queries.dtype != want or not queries.is_cuda or not queries.is_contiguous():
        raise ValueError("queries must be a contiguous CUDA %s tensor" % want)
    for name, t in (("L_per_query", L_per_query), ("k_per_query", k_per_query),
                    ("order", order)):
        if t is not None and (t.dtype != torch.int32 or not t.is_cuda or t.numel() != queries.shape[0]):
            raise ValueError("%s must be a CUDA int32 tensor of nq entries" % name)
    nq = queries.shape[0]
    dev = queries.device
    dist_dtype = torch.float32 if index.dtype == np.float32 else torch.int32
    if out is None:
        ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
        dists = torch.empty((nq, k), dtype=dist_dtype, device=dev)
        steps = torch.empty((nq,), dtype=torch.int32, device=dev)
    else:
        ids, dists, steps = out
    # every caller-supplied device buffer is written by the kernel: its
    # dtype, device, contiguity and size must match what the launch assumes
    _check_buffer("ids", ids, (torch.int32,), nq * k, dev)
    _check_buffer("dists", dists, (dist_dtype,), nq * k, dev)
    if steps is not None:
        _check_buffer("steps", steps, (torch.int32,), nq, dev)
    if stats is not None:
        _check_buffer("stats", stats, (torch.int64,), 3, dev)
    if trace is not None:
        if trace.dim() != 2 or trace.shape[0] != nq or trace.shape[1] < 1:
            raise ValueError("trace must be [nq, cap >= 1]")
        _check_buffer("trace", trace, (torch.int32,), trace.numel(), dev)
    if times is not None:
        _check_buffer("times", times, (torch.int64,), 2 * nq, dev)
    if phases is not None:
        _check_buffer("phases", phases, (torch.int64,), 2 * nq, dev)
    opts = SearchOptions(delay, beam_width, hash_bits, waves_per_block, _ptr(stats), _ptr(trace),
                         trace.shape[1] if trace is not None else 0, _ptr(times), _ptr(phases),
                         transport, spin_limit, _ptr(L_per_query), _ptr(k_per_query), _ptr(order),
                         1 if persistent else 0, int(sync_grain), int(navigation),
                         int(pq_scoring), int(poll_backoff), int(query_lanes))
    return nq, ids, dists, steps, opts


def search(index: Index, queries, k: int, L: int, R: int = 0, delay: int = 1,
           beam_width: int = 1, hash_bits: int = 0, waves_per_block: int = 0, stats=None,
           trace=None, times=None, phases=None, transport: int = TRANSPORT_AUTO,
           spin_limit: int = 0, L_per_query=None, k_per_query=None, order=None,
           persistent: bool = False, stream=None, out=None, sync_grain: int = SYNC_QUERY,
           navigation: int = NAV_FULL, pq_scoring: int = PQ_AUTO, poll_backoff: int = 0,
           query_lanes: int = 0):
    """ann_search on torch CUDA tensors.

    queries: [nq, d] device tensor of the index dtype (uint8/int8/float32).
    stats: optional int64 device tensor of 3 counters (accumulated);
    trace: optional int32 device tensor [nq, cap] receiving expanded ids;
    times: optional int64 device tensor [nq, 2] receiving start/end stamps;
    phases: optional int64 device tensor [nq, 2] (strict only): summed fetch and
    compute ticks per query;
    L_per_query / k_per_query / order: optional int32 device tensors [nq]
    (uneven batches; L and k are then the batch maxima).
    sync_grain: SYNC_QUERY (default) or SYNC_KERNEL (lockstep rounds with
    grid-wide barriers; strict schedule only).
    navigation: NAV_FULL, or NAV_PQ (PQ codes from Index.set_pq order the
    list; results re-ranked by exact distance from the records).
    pq_scoring: PQ_AUTO, PQ_TABLE (per-query LDS table) or PQ_CACHE
    (centroids from the cache); the results are the same.
    query_lanes: 0/64 (one query per wave64) or 32 (two queries per wave;
    direct transport, full navigation, delay <= 1, beam 1, records <= 512 B);
    the results are the same.
    Returns (ids int32 [nq,k], dists [nq,k] int32-viewed uint32 or float32,
    steps int32-viewed uint32 [nq]), all on the device.
    """
    import torch

    nq, ids, dists, steps, opts = _prepare(index, queries, k, L, R, delay, beam_width, hash_bits,
                                           waves_per_block, stats, trace, times, phases,
                                           transport, spin_limit, L_per_query, k_per_query,
                                           order, persistent, out, sync_grain, navigation,
                                           pq_scoring, poll_backoff, query_lanes)
    st = stream if stream is not None else torch.cuda.current_stream(queries.device)
    _check(load_library().ann_search(index.handle, queries.data_ptr(), nq, k, L, R,
                                     ctypes.byref(opts), ids.data_ptr(), dists.data_ptr(),
                                     steps.data_ptr() if steps is not None else None,
                                     st.cuda_stream))
    return ids, dists, steps


def search_noalloc(index: Index, queries, k: int, L: int, out, R: int = 0, delay: int = 1,
                   beam_width: int = 1, hash_bits: int = 0, waves_per_block: int = 0,
                   stats=None, trace=None, times=None, L_per_query=None, k_per_query=None,
                   order=None, persistent: bool = False, stream=None,
                   sync_grain: int = SYNC_QUERY, spin_limit: int = 0, navigation: int = NAV_FULL,
                   pq_scoring: int = PQ_AUTO):
    """ann_search_noalloc: the search without any allocation in the call.
    `out` = (ids, dists, steps) device tensors are required (the binding
    allocates nothing either); records are read directly (HBM or host tier)."""
    import torch

    if out is None:
        raise ValueError("search_noalloc writes into caller-owned out=(ids, dists, steps)")
    nq, ids, dists, steps, opts = _prepare(index, queries, k, L, R, delay, beam_width, hash_bits,
                                           waves_per_block, stats, trace, times, None,
                                           TRANSPORT_DIRECT, spin_limit, L_per_query, k_per_query,
                                           order, persistent, out, sync_grain, navigation,
                                           pq_scoring)
    st = stream if stream is not None else torch.cuda.current_stream(queries.device)
    _check(load_library().ann_search_noalloc(index.handle, queries.data_ptr(), nq, k, L, R,
                                             ctypes.byref(opts), ids.data_ptr(), dists.data_ptr(),
                                             steps.data_ptr() if steps is not None else None,
                                             st.cuda_stream))
    return ids, dists, steps


class SearchGraph:
    """ann_search_graph: one persistent search captured in a HIP graph.

    The graph keeps the tensors it was recorded with; rewrite their contents
    and call launch() to replay.  `stream` must not be the default stream.
    """

    def __init__(self, index: Index, queries, k: int, L: int, stream, R: int = 0,
                 delay: int = 1, hash_bits: int = 0, waves_per_block: int = 0,
                 L_per_query=None, k_per_query=None, order=None, out=None, beam_width: int = 1,
                 navigation: int = NAV_FULL, query_lanes: int = 0):
        nq, ids, dists, steps, opts = _prepare(index, queries, k, L, R, delay, beam_width, hash_bits,
                                               waves_per_block, None, None, None, None,
                                               TRANSPORT_DIRECT, 0, L_per_query, k_per_query,
                                               order, True, out, 0, navigation,
                                               query_lanes=query_lanes)
        self._keep = (index, queries, ids, dists, steps, L_per_query, k_per_query, order)
        self.ids, self.dists, self.steps = ids, dists, steps
        self.stream = stream
        g = ctypes.c_void_p()
        _check(load_library().ann_search_graph(index.handle, queries.data_ptr(), nq, k, L, R,
                                               ctypes.byref(opts), ids.data_ptr(),
                                               dists.data_ptr(), steps.data_ptr(),
                                               stream.cuda_stream, ctypes.byref(g)))
        self._g = g

    def launch(self, stream=None):
        st = stream if stream is not None else self.stream
        _check(load_library().ann_graph_launch(self._g, st.cuda_stream))
        return self.ids, self.dists, self.steps

    def close(self):
        if getattr(self, "_g", None) is not None:
            load_library().ann_graph_free(self._g)
            self._g = None

    __del__ = close


def clock_us() -> float:
    """The host clock (microseconds) of the server's result stamps."""
    return load_library().ann_clock_us()


class Server:
    """ann_server_*: continuous-batching search service over an index."""

    def __init__(self, index: Index, hbm_budget_bytes: int, k_max: int = 100, L_max: int = 256,
                 delay: int = 1, waves_per_block: int = 0, hash_bits: int = 0,
                 queue_cap: int = 0, idle_polls: int = 0, beam_width: int = 1,
                 transport: int = TRANSPORT_AUTO, spin_limit: int = 0,
                 navigation: int = NAV_FULL, pq_scoring: int = PQ_AUTO,
                 first_ticket: int = 0):
        self.index = index
        self.dtype = index.dtype
        self.d = index.d
        self.k_max = k_max
        opts = ServerOptions(k_max, L_max, delay, waves_per_block, hash_bits, queue_cap,
                             idle_polls, beam_width, transport, spin_limit, navigation,
                             pq_scoring, first_ticket)
        h = ctypes.c_void_p()
        _check(load_library().ann_server_open(index.handle, int(hbm_budget_bytes),
                                              ctypes.byref(opts), ctypes.byref(h)))
        self._h = h
        self._buf = (Result * 4096)()

    def submit(self, query: np.ndarray, k: int, L: int, tag: int) -> None:
        q = np.ascontiguousarray(query, dtype=self.dtype).reshape(-1)
        if q.shape[0] != self.d:
            raise ValueError("query must have %d elements" % self.d)
        _check(load_library().ann_server_submit(self._h, q.ctypes.data, int(k), int(L), int(tag)))

    def submit_batch(self, queries: np.ndarray, ks, Ls, tags, arrival_us=None) -> None:
        """Queue many queries; optional non-decreasing arrival times (clock_us())."""
        q = np.ascontiguousarray(queries, dtype=self.dtype)
        n = q.shape[0]
        ks = np.ascontiguousarray(ks, dtype=np.int32)
        Ls = np.ascontiguousarray(Ls, dtype=np.int32)
        tags = np.ascontiguousarray(tags, dtype=np.uint64)
        arr = None if arrival_us is None else np.ascontiguousarray(arrival_us, dtype=np.float64)
        _check(load_library().ann_server_submit_batch(
            self._h, q.ctypes.data, n, ks.ctypes.data, Ls.ctypes.data, tags.ctypes.data,
            arr.ctypes.data if arr is not None else None))

    def poll(self, max_results: int = 4096, timeout_us: int = 0):
        """Completed results: list of dicts (ids, dists copied to numpy)."""
        n = ctypes.c_int32()
        m = min(max_results, len(self._buf))
        _check(load_library().ann_server_poll(self._h, self._buf, m, ctypes.byref(n), timeout_us))
        dt = np.float32 if self.dtype == np.float32 else np.uint32
        out = []
        for i in range(n.value):
            r = self._buf[i]
            ids = np.ctypeslib.as_array(ctypes.cast(r.ids, ctypes.POINTER(ctypes.c_int32)),
                                        shape=(r.k,)).copy()
            raw = np.ctypeslib.as_array(ctypes.cast(r.dists, ctypes.POINTER(ctypes.c_uint32)),
                                        shape=(r.k,)).copy()
            out.append({"tag": r.tag, "status": r.status, "ids": ids, "dists": raw.view(dt),
                        "steps": r.steps, "submit_us": r.submit_us, "done_us": r.done_us})
        return out

    def drain(self, n_expected: int, timeout_s: float = 120.0, chunk: int = 8192):
        """Collect n_expected results with the bulk poll; returns numpy arrays
        (tags, ks, ids [n, k_max], dists [n, k_max], steps, submit_us, done_us,
        status: 0, or -5 / -110 for a failed or timed-out record read)."""
        import time

        dt = np.float32 if self.dtype == np.float32 else np.uint32
        out = {"tags": np.zeros(n_expected, np.uint64), "ks": np.zeros(n_expected, np.int32),
               "ids": np.zeros((n_expected, self.k_max), np.int32),
               "dists": np.zeros((n_expected, self.k_max), np.uint32),
               "steps": np.zeros(n_expected, np.uint32),
               "submit_us": np.zeros(n_expected), "done_us": np.zeros(n_expected),
               "status": np.zeros(n_expected, np.int32)}
        got = 0
        nn = ctypes.c_int32()
        end = time.time() + timeout_s
        lib = load_library()
        while got < n_expected and time.time() < end:
            m = min(chunk, n_expected - got)
            _check(lib.ann_server_poll_into(
                self._h, m, out["tags"][got:].ctypes.data, out["ks"][got:].ctypes.data,
                out["ids"][got:].ctypes.data, out["dists"][got:].ctypes.data,
                out["steps"][got:].ctypes.data, out["submit_us"][got:].ctypes.data,
                out["done_us"][got:].ctypes.data, out["status"][got:].ctypes.data,
                ctypes.byref(nn), 2000))
            got += nn.value
        for key in out:
            out[key] = out[key][:got]
        out["dists"] = out["dists"].view(dt)
        return out

    def stats(self) -> dict:
        st = ServerStats()
        _check(load_library().ann_server_stats_get(self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None:
            h, self._h = self._h, None
            _check(load_library().ann_server_close(h))

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
