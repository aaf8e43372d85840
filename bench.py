#!/usr/bin/env python3
"""Benchmark of the search hot path on one MI355X.

Metric: QPS at recall@10 >= 0.95 for the dependency-relaxed pipeline (delay 1)
against the strict best-first search (delay 0), plus per-query latency
percentiles.  Default workload: 1M uint8 vectors, d = 128, from a
256-component Gaussian mixture, degree-64 graph, 512 B records in pinned host
DRAM read by the GPU over the host link, 10,000 queries, k = 10, L swept over
32..256 (synthetic stand-in for SIFT1B, which is not available).

A "step" is one ann_search launch over the whole query batch with the index
resident (navigation copy in HBM, records in pinned host memory, queries in
HBM).  Prints exactly one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
L_SWEEP = (32, 36, 40, 44, 48, 52, 56, 60, 64, 96, 128, 192, 256)
# (delta, W) pairs of the schedule sweep; (delta + 1) * W <= 8
SCHEDULES = ((0, 1), (1, 1), (2, 1), (3, 1), (0, 2), (1, 2), (3, 2), (0, 4), (1, 4), (0, 8))


def log(msg):
    print("[bench %7.1fs] %s" % (time.time() - T0, msg), file=sys.stderr, flush=True)


T0 = time.time()


def ground_truth(base, queries, k, torch, dev):
    """Exact k-th neighbour distance per query (paper_2507_10070_amd.recall:
    a GPU full scan in int32-indexable chunks, spot-checked on the CPU)."""
    from paper_2507_10070_amd.recall import exact_kth

    return exact_kth(base, queries, k, dev)


def recall_at(dists_u32, kth):
    import numpy as np

    hits = np.minimum((dists_u32.astype(np.float64) <= kth[:, None]).sum(1), 10)
    return float(hits.mean() / 10.0)


def host_cpu():
    """CPU model and SMT state of this host (for the CPU baseline)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    smt = None
    try:
        with open("/sys/devices/system/cpu/smt/active") as f:
            smt = f.read().strip() == "1"
    except OSError:
        pass
    return {"model": model, "smt": smt, "online": os.cpu_count()}


def _code_only(src: bytes) -> bytes:
    """C++ source without // comments and blank lines (the code it compiles)."""
    out = []
    for line in src.split(b"\n"):
        i = line.find(b"//")
        if i >= 0:
            line = line[:i]
        line = line.rstrip()
        if line:
            out.append(line)
    return b"\n".join(out)


def kernel_source_hash():
    """Hash of everything the profiled search kernel is compiled from: the
    kernel header, search_kernel.hip up to the end of the search kernel
    itself (the lockstep and server kernels and the host launchers follow it
    and do not change the profiled code), the units that instantiate it for
    each element type, and the compiler flags; comments and blank lines are
    left out of the sources."""
    from paper_2507_10070_amd import build as hip_build

    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2507_10070_amd", "csrc")
    with open(os.path.join(csrc, "search_kernel.h"), "rb") as fh:
        h.update(_code_only(fh.read()))
    with open(os.path.join(csrc, "search_kernel.hip"), "rb") as fh:
        src = fh.read()
    end = src.find(b"__global__ void reset_work(")
    h.update(_code_only(src if end < 0 else src[:end]))
    for unit in sorted(u for u in hip_build.SOURCES if os.path.basename(u).startswith("search_")
                       and u != "search_kernel.hip"):
        with open(os.path.join(csrc, unit), "rb") as fh:
            h.update(_code_only(fh.read()))
    h.update(" ".join(hip_build.FLAGS).encode())
    return h.hexdigest()[:16]


def stored_traffic(workload, L):
    """HBM traffic per launch measured by rocprofv3 counters, if the kernel
    and the operating L have not changed since (profiles/search_traffic.json)."""
    p = os.path.join(ROOT, "profiles", "search_traffic.json")
    try:
        with open(p) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    h = kernel_source_hash()
    for e in t.get("entries", [t]):
        if e.get("kernel_hash") == h and e.get("workload") == workload and e.get("L") == L:
            return e.get("traffic_bytes_per_launch")
    return None


def serving_leg(fa, ix, queries, kth, budget, L_op):
    """Continuous batching under open-loop Poisson arrivals.

    The operating mix draws k from {10, 100} and L from the swept values with
    L >= max(k, L_op), L_op being the smallest L whose recall@10 reaches 0.95,
    so every request runs at the target recall.  Saturation throughput comes
    from a 200k-query burst; then Poisson arrivals at fractions of it, with
    latency from intended arrival to result.  The wide mix (L in
    {32, 64, 128, 256} with L >= k) is measured at saturation only."""
    import numpy as np

    rng = np.random.default_rng(5)
    nq = queries.shape[0]

    def mix(m, Lset):
        ks = rng.choice(np.array([10, 100], np.int32), m)
        Ls = np.array([rng.choice([L for L in Lset if L >= k]) for k in ks], np.int32)
        return ks, Ls

    def recall(res):
        qi = (res["tags"] % nq).astype(np.int64)
        d10 = res["dists"][:, :10].astype(np.float64)
        hit = np.minimum((d10 <= kth[qi][:, None]).sum(1), 10) / 10.0
        return float(hit.mean())

    op_set = [L for L in L_SWEEP if L >= L_op]
    wide_set = [32, 64, 128, 256]
    out = {"workload": "1M u8/128 index, pinned host DRAM records, k in {10, 100}, "
                       "L in %s with L >= k" % op_set,
           "budget_bytes": budget}

    def saturate(srv, Lset, m0=200000):
        ks, Ls = mix(m0, Lset)
        idx = np.arange(m0) % nq
        t0 = fa.clock_us()
        srv.submit_batch(queries[idx], ks, Ls, np.arange(m0, dtype=np.uint64))
        res = srv.drain(m0)
        return (round(m0 / ((res["done_us"].max() - t0) / 1e6), 1), round(recall(res), 4),
                float(np.mean(Ls)))

    with fa.Server(ix, hbm_budget_bytes=budget) as srv:
        st = srv.stats()
        out["slots"], out["resident_waves"] = st["slots"], st["resident_waves"]
        qmax, rec, _ = saturate(srv, op_set)
        out["saturation_qps"], out["saturation_recall@10"] = qmax, rec
        rates = []
        for frac in (0.25, 0.5, 0.75, 0.9):
            lam = frac * qmax
            m = int(min(max(3000, lam * 0.5), 150000))
            ks, Ls = mix(m, op_set)
            idx = rng.integers(0, nq, m)
            start = fa.clock_us() + 20000.0
            arr = start + np.cumsum(rng.exponential(1e6 / lam, m))
            srv.submit_batch(queries[idx], ks, Ls, idx.astype(np.uint64), arr)
            res = srv.drain(m)
            lat = (res["done_us"] - res["submit_us"]) / 1e3
            rates.append({"offered_qps": round(lam, 1), "queries": int(len(lat)),
                          "achieved_qps": round(len(lat) / ((res["done_us"].max() - start) / 1e6), 1),
                          "latency_ms_p50": round(float(np.percentile(lat, 50)), 3),
                          "latency_ms_p99": round(float(np.percentile(lat, 99)), 3),
                          "recall@10": round(recall(res), 4)})
            log("serving at %.0f QPS offered: %s" % (lam, rates[-1]))
        out["rates"] = rates
        wq, wr, wl = saturate(srv, wide_set)
        out["wide_mix"] = {"L": wide_set, "mean_L": round(wl, 1), "saturation_qps": wq,
                           "recall@10": wr}
        st = srv.stats()
        out["relaunches"] = st["relaunches"]
        out["max_inflight"] = st["max_inflight"]
    return out


def serving_burst(fa, ix, queries, kth, L_op, m=2000, where="records in a file", **server_kw):
    """Continuous batching measured briefly: the operating mix of the serving
    leg (L >= L_op), saturation from an m-query burst, then Poisson arrivals
    at half of it.  With records in a file the server's own host agents read
    them (O_DIRECT), one request line per resident wave; `server_kw` passes
    server options (e.g. compressed navigation)."""
    import numpy as np

    rng = np.random.default_rng(23)
    nq = queries.shape[0]
    Lset = [L for L in L_SWEEP if L >= L_op]
    ks = rng.choice(np.array([10, 100], np.int32), 2 * m)
    Ls = np.array([rng.choice([L for L in Lset if L >= k]) for k in ks], np.int32)

    def recall(res):
        qi = (res["tags"] % nq).astype(np.int64)
        d10 = res["dists"][:, :10].astype(np.float64)
        return float((np.minimum((d10 <= kth[qi][:, None]).sum(1), 10) / 10.0).mean())

    out = {"workload": "%s, k in {10, 100}, L in %s with L >= k" % (where, Lset)}
    with fa.Server(ix, hbm_budget_bytes=256 << 20, **server_kw) as srv:
        idx = np.arange(m) % nq
        t0 = fa.clock_us()
        srv.submit_batch(queries[idx], ks[:m], Ls[:m], idx.astype(np.uint64))
        res = srv.drain(m)
        qmax = m / ((res["done_us"].max() - t0) / 1e6)
        out["saturation_qps"] = round(qmax, 1)
        out["failed_reads"] = int((res["status"] != 0).sum())
        lam = 0.5 * qmax
        idx = rng.integers(0, nq, m)
        start = fa.clock_us() + 20000.0
        arr = start + np.cumsum(rng.exponential(1e6 / lam, m))
        srv.submit_batch(queries[idx], ks[m:], Ls[m:], idx.astype(np.uint64), arr)
        res = srv.drain(m)
        lat = (res["done_us"] - res["submit_us"]) / 1e3
        out["half_load"] = {"offered_qps": round(lam, 1), "queries": int(len(lat)),
                            "latency_ms_p50": round(float(np.percentile(lat, 50)), 3),
                            "latency_ms_p99": round(float(np.percentile(lat, 99)), 3),
                            "recall@10": round(recall(res), 4)}
    log("serving (%s): %s" % (where, out))
    return out


def pq_leg(fa, torch, dev, base, adj, entry, cfg, ix, qd, kth, L_full, stream, subspaces,
           queries_host=None):
    """Compressed navigation (paper section 2.2): PQ codes in HBM order the
    candidate list, expanded nodes are re-ranked exactly from their records.
    Per number of subspaces M: codebook training and GPU encoding time, the
    recall sweep (up to the first L with recall@10 >= 0.95), and at that L
    the throughput (records in host DRAM and in HBM, relaxed and strict) and
    the HBM bytes of navigation per launch against those of the
    full-precision copy.  L_full None: the full-precision operating L is
    swept here too."""
    import numpy as np

    import synth

    nq, k = qd.shape[0], cfg.k
    info = ix.info()
    full_sweep = None
    if L_full is None:
        full_sweep = []
        for L in L_SWEEP:
            ids_, d_, s_ = fa.search(ix, qd, k=k, L=L, delay=1, stream=stream)
            torch.cuda.synchronize()
            rec = recall_at(d_.cpu().numpy().view(np.uint32), kth)
            full_sweep.append({"L": L, "recall@10": round(rec, 4)})
            if rec >= 0.95:
                L_full = L
                break
        L_full = L_full or L_SWEEP[-1]
    out = (torch.empty((nq, k), dtype=torch.int32, device=dev),
           torch.empty((nq, k), dtype=torch.int32, device=dev),
           torch.empty((nq,), dtype=torch.int32, device=dev))

    def timed(index, L, delay, reps=5, **kw):
        fa.search(index, qd, k=k, L=L, delay=delay, out=out, stream=stream, **kw)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(stream)
        for _ in range(reps):
            fa.search(index, qd, k=k, L=L, delay=delay, out=out, stream=stream, **kw)
        ev[1].record(stream)
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / reps

    def stats_at(index, L, delay, **kw):
        st = torch.zeros(3, dtype=torch.int64, device=dev)
        fa.search(index, qd, k=k, L=L, delay=delay, out=out, stream=stream, stats=st, **kw)
        torch.cuda.synchronize()
        return st.cpu().numpy()

    res = {"workload": cfg.name, "full_navigation": {
        "L": L_full, "nav_hbm_bytes": info["n"] * info["nav_stride"],
        "relaxed_qps": round(nq / (timed(ix, L_full, 1) / 1e3), 1)}}
    if full_sweep is not None:
        res["full_navigation"]["sweep"] = full_sweep
    s_full = stats_at(ix, L_full, 1)
    res["full_navigation"]["nav_bytes_per_launch"] = int(s_full[1]) * info["nav_stride"]
    hix = fa.Index(base, adj, entry, cfg.slot, fa.TIER_HBM)
    try:
        res["full_navigation"]["records_in_hbm_qps"] = round(nq / (timed(hix, L_full, 1) / 1e3), 1)
        for M in subspaces:
            t = time.time()
            cb = synth.train_codebooks(base, M, iters=8, sample=20000, seed=50 + M)
            t_train = time.time() - t
            t = time.time()
            ix.set_pq(cb)
            t_enc = time.time() - t
            hix.set_pq(cb)
            nav = {"navigation": fa.NAV_PQ}
            sweep, L_op = [], None
            for L in L_SWEEP + (384, 512):
                fa.search(ix, qd, k=k, L=L, delay=1, out=out, stream=stream, **nav)
                torch.cuda.synchronize()
                rec = recall_at(out[1].cpu().numpy().view(np.uint32), kth)
                sweep.append({"L": L, "recall@10": round(rec, 4),
                              "mean_steps": round(float(out[2].cpu().numpy().mean()), 2)})
                if rec >= 0.95:
                    L_op = L
                    break
            reached = L_op is not None
            if L_op is None:  # timed at the largest L of the regular sweep
                L_op = L_SWEEP[-1]
            s = stats_at(ix, L_op, 1, **nav)
            ms_r = timed(ix, L_op, 1, **nav)
            ms_s = timed(ix, L_op, 0, **nav)
            ms_h = timed(hix, L_op, 1, **nav)
            # the two ways of forming PQ distances (same results)
            by_scoring = {}
            for name, sc in (("table", fa.PQ_TABLE), ("cache", fa.PQ_CACHE)):
                by_scoring[name] = {
                    "relaxed_qps": round(nq / (timed(ix, L_op, 1, pq_scoring=sc, **nav) / 1e3), 1),
                    "records_in_hbm_qps": round(
                        nq / (timed(hix, L_op, 1, pq_scoring=sc, **nav) / 1e3), 1)}
            res["M%d" % M] = {
                "train_s": round(t_train, 1), "encode_s": round(t_enc, 2),
                "code_hbm_bytes": info["n"] * 32, "code_bytes_per_node": M,
                "L": L_op, "recall_target_reached": reached, "sweep": sweep,
                "by_scoring": by_scoring,
                "relaxed_qps": round(nq / (ms_r / 1e3), 1),
                "strict_qps": round(nq / (ms_s / 1e3), 1),
                "records_in_hbm_qps": round(nq / (ms_h / 1e3), 1),
                "expansions": int(s[0]), "codes_scored": int(s[1]),
                "nav_bytes_per_launch": int(s[1]) * M,
                "nav_bytes_loaded_per_launch": int(s[1]) * 32,
                "host_link_bytes_per_launch": int(s[0]) * info["rec_bytes"],
                # records in HBM: algorithmic bytes (codes + records) per second
                "records_in_hbm_GBps": round((int(s[1]) * M + int(s[0]) * info["rec_bytes"]) /
                                             (ms_h / 1e3) / 1e9, 1)}
            log("PQ M=%d: %s" % (M, {kk: v for kk, v in res["M%d" % M].items() if kk != "sweep"}))
            if reached and queries_host is not None:
                res["M%d" % M]["serving"] = serving_burst(
                    fa, ix, queries_host, kth, L_op, m=50000,
                    where="PQ navigation (M = %d), records in host DRAM" % M,
                    navigation=fa.NAV_PQ)
    finally:
        hix.close()
    return res


def pq_kernel_run(fa, torch, dev, steps):
    """One compressed-navigation configuration alone, for profiling its kernel:
    the 1M u8/128 workload of intrinsic dimension 16 with records in HBM, PQ
    codes with M = 32 scored from the cache, relaxed schedule, L = 64 (its
    recall@10 >= 0.95 point); `steps` timed launches of 10k queries.  Prints
    one JSON line with the kernel's algorithmic bytes and rate."""
    import numpy as np

    import synth

    cfg = synth.WORKLOADS["1m-u8-128-latent16"]
    base, q = synth.make_dataset(cfg)
    adj, entry = synth.build_graph(base, cfg.R, 3000 + cfg.seed_offset,
                                   threads=min(16, os.cpu_count() or 1))
    kth = ground_truth(base, q, cfg.k, torch, dev)
    cb = synth.train_codebooks(base, 32, iters=8, sample=20000, seed=50 + 32)
    stream = torch.cuda.current_stream(dev)
    qd = torch.from_numpy(q).to(dev)
    L, M = 64, 32
    with fa.Index(base, adj, entry, cfg.slot, fa.TIER_HBM) as ix:
        ix.set_pq(cb)
        info = ix.info()
        kw = dict(k=cfg.k, L=L, delay=1, navigation=fa.NAV_PQ, pq_scoring=fa.PQ_CACHE,
                  stream=stream)
        st = torch.zeros(3, dtype=torch.int64, device=dev)
        ids, dists, steps_ = fa.search(ix, qd, stats=st, **kw)
        torch.cuda.synchronize()
        rec = recall_at(dists.cpu().numpy().view(np.uint32), kth)
        s = st.cpu().numpy()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(stream)
        for _ in range(steps):
            fa.search(ix, qd, **kw)
        ev[1].record(stream)
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1]) / steps
    byt = int(s[1]) * M + int(s[0]) * info["rec_bytes"] + len(q) * (cfg.d + 8 * cfg.k + 4)
    print(json.dumps({"pq_kernel": {"workload": "1M u8/128 of intrinsic dimension 16, records in HBM",
                                    "M": M, "L": L, "scoring": "cache",
                                    "recall@10": round(rec, 4), "ms_per_launch": round(ms, 4),
                                    "qps": round(len(q) / (ms / 1e3), 1),
                                    "expansions": int(s[0]), "codes_scored": int(s[1]),
                                    "algorithmic_bytes_per_launch": byt,
                                    "algorithmic_GBps": round(byt / (ms / 1e3) / 1e9, 1),
                                    "hbm_frac": round(byt / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}}),
          flush=True)


def pq_scale_run(fa, torch, dev, n):
    """Compressed against full-precision navigation at a larger size: the
    workload of intrinsic dimension 16 with n vectors, records in pinned host
    DRAM, PQ M = 32 (the pq_navigation leg on that index).  Prints one JSON
    line."""
    import synth

    cfg = synth.WORKLOADS["1m-u8-128-latent16"]
    log("generating %d x %d u8 vectors of intrinsic dimension %d" % (n, cfg.d, cfg.latent))
    base, q = synth.make_dataset(cfg, n=n)
    os.environ["FLASHANN_BUILD_PROGRESS"] = "1"
    t = time.time()
    adj, entry = synth.build_graph(base, cfg.R, 3000 + cfg.seed_offset,
                                   threads=min(16, os.cpu_count() or 1))
    log("graph R=%d built in %.1fs" % (cfg.R, time.time() - t))
    kth = ground_truth(base, q, cfg.k, torch, dev)
    log("ground truth done")
    stream = torch.cuda.current_stream(dev)
    with fa.Index(base, adj, entry, cfg.slot, fa.TIER_HOST) as ix:
        res = pq_leg(fa, torch, dev, base, adj, entry, cfg, ix, torch.from_numpy(q).to(dev), kth,
                     None, stream, (32,), queries_host=q)
    res["workload"] = "%d x u8/128 of intrinsic dimension 16, records in pinned host DRAM" % n
    res["n"] = n
    print(json.dumps({"pq_scale": res}, default=float), flush=True)


def f32_file_leg(fa, torch, dev, n, R_values, nq, L, keep_dir=None, tier="file"):
    """The f32/96 workload with 4 KB record slots in a file: n unit vectors
    from a 1,024-component mixture (sigma 0.1 before normalisation), nq
    queries, k = 10, list size L; per degree R, a real graph, the index files
    (records padded to 4,096 B, read with O_DIRECT by the host agents),
    relaxed and strict QPS with recall@10, and the per-expansion fetch and
    compute times T_f, T_c of the strict schedule (the two stages Eq. 6 of
    the degree selection balances).  With keep_dir, the last degree's index
    directory, graph and queries stay there for the sampled oracle check
    (tests/fullsize_f32_parity.py).  tier "host" or "hbm" keeps the same 4 KB
    slots in pinned DRAM or in HBM instead (the kernel without the disk)."""
    import shutil
    import tempfile

    import numpy as np

    import synth
    from paper_2507_10070_amd import degree_selector

    cfg = synth.WORKLOADS["10m-f32-96"]
    t = time.time()
    base, q = synth.make_dataset(cfg, n=n, nq=nq)
    log("f32-file: %d x 96 f32 vectors, %d queries in %.1fs" % (n, nq, time.time() - t))
    # exact 10th-neighbour distances (fp32 GEMM expansion; recall allows the
    # expansion's rounding, 1e-5 relative, as the parity tolerance does)
    kth = ground_truth(base, q, 10, torch, dev)
    qd = torch.from_numpy(q).to(dev)
    khz = fa.device_clock_khz()
    os.environ["FLASHANN_BUILD_PROGRESS"] = "1"
    rows = []
    for R in R_values:
        t = time.time()
        adj, entry = synth.build_graph(base, R, 3003, threads=min(16, os.cpu_count() or 1))
        t_graph = time.time() - t
        log("f32-file: graph R=%d in %.1fs" % (R, t_graph))
        last = keep_dir is not None and R == R_values[-1]
        tmpd = keep_dir if last else tempfile.mkdtemp(
            prefix="flashann_f32_", dir=os.environ.get("TMPDIR", "/tmp"))
        try:
            t = time.time()
            fa.save_index(tmpd, base, adj, entry, 4096)
            t_save = time.time() - t
            if last:
                np.save(os.path.join(tmpd, "adj.npy"), adj)
                np.save(os.path.join(tmpd, "queries.npy"), q)
            del adj
            log("f32-file: R=%d index files (%.1f GB of records) written in %.1fs"
                % (R, n * 4096 / 1e9, t_save))
            t_tier = {"file": fa.TIER_FILE, "host": fa.TIER_HOST, "hbm": fa.TIER_HBM}[tier]
            with fa.Index.load(tmpd, t_tier) as ix:
                row = {"R": R, "L": L, "tier": tier, "graph_build_s": round(t_graph, 1),
                       "write_s": round(t_save, 1), "direct_io": ix.info()["direct_io"]}
                fa.search(ix, qd[:500].contiguous(), k=10, L=L, delay=1)  # warm-up
                for name, delay in (("relaxed", 1), ("strict", 0)):
                    p0 = ix.agent_profile()
                    reps = 1 if tier == "file" else 5
                    t = time.perf_counter()
                    for _ in range(reps):
                        _, dist, steps = fa.search(ix, qd, k=10, L=L, delay=delay)
                    torch.cuda.synchronize()
                    el = (time.perf_counter() - t) / reps
                    p1 = ix.agent_profile()
                    dv = dist.cpu().numpy().astype(np.float64)
                    rec = float(np.minimum((dv <= kth[:, None] * (1 + 1e-5)).sum(1), 10).mean() / 10)
                    row[name] = {"qps": round(nq / el, 1), "recall@10": round(rec, 4),
                                 "mean_steps": round(float(steps.cpu().numpy().view(np.uint32).mean()), 2),
                                 "reads_per_s": round((p1["requests"] - p0["requests"]) / el / reps, 1)}
                # algorithmic bytes of one relaxed launch (the kernel's own
                # counters): rows scored x row stride from HBM, expansions x
                # record bytes from the record tier
                st = torch.zeros(3, dtype=torch.int64, device=dev)
                fa.search(ix, qd, k=10, L=L, delay=1, stats=st)
                torch.cuda.synchronize()
                stv = st.cpu().numpy()
                info = ix.info()
                row["nav_bytes_per_launch"] = int(stv[1]) * info["nav_stride"]
                row["record_bytes_per_launch"] = int(stv[0]) * info["rec_bytes"]
                sec = nq / row["relaxed"]["qps"]
                row["relaxed"]["algorithmic_GBps"] = round(
                    (row["nav_bytes_per_launch"] + row["record_bytes_per_launch"]) / sec / 1e9, 1)
                # stage times of Eq. 6 on this graph: strict schedule, stamps,
                # median of three runs (their spread is the noise the
                # degree selector's fit allows for)
                tf, tc = [], []
                for _ in range(3):
                    phases = torch.zeros((nq, 2), dtype=torch.int64, device=dev)
                    _, _, steps = fa.search(ix, qd, k=10, L=L, delay=0, phases=phases)
                    torch.cuda.synchronize()
                    ph = phases.cpu().numpy().sum(0).astype(np.float64)
                    ns = float(steps.cpu().numpy().view(np.uint32).astype(np.int64).sum())
                    tf.append(ph[0] / ns / khz * 1e3)
                    tc.append(ph[1] / ns / khz * 1e3)
                row["T_f_us"] = round(float(np.median(tf)), 3)
                row["T_c_us"] = round(float(np.median(tc)), 3)
                row["T_f_spread_us"] = round(float(np.ptp(tf)), 3)
            rows.append(row)
            log("f32-file: %s" % row)
        finally:
            if not last:
                shutil.rmtree(tmpd, ignore_errors=True)
    out = {"workload": "%d x 96 f32 (1,024-component mixture), 4,096 B record slots, %s tier"
           % (n, tier), "queries": nq, "k": 10, "L": L, "rows": rows}
    if len(rows) > 1:
        out["selected_R"], out["fit"] = degree_selector.select_fitted(rows)
        out["selected_R_raw"] = degree_selector.select(rows)
    return out


def serving_file_leg(fa, torch, dev, n, nq=10000, m=2000, cache_fraction=0.0):
    """The serving form with records in a file: n u8/128 vectors of the
    4,096-component mixture, degree-64 graph, 512 B records in a file read
    with O_DIRECT by the server's own host agents; requests draw k from
    {10, 100} and L from the swept values with L >= max(k, L_op), L_op the
    smallest L whose recall@10 reaches 0.95 on a 2,000-query sample.
    Saturation from an m-query burst, then open-loop Poisson arrivals at
    0.25, 0.5, 0.75 and 0.9 of it (m queries each), latency from the
    intended arrival to the result.  With cache_fraction > 0 the same
    requests are first served with that share of the records in the
    hot-record cache (most-expanded nodes of 10,000 training queries of
    another seed), then without it."""
    import shutil
    import tempfile

    import numpy as np

    import synth

    cfg = synth.WORKLOADS["100m-u8-128"]
    t = time.time()
    base, q = synth.make_dataset(cfg, n=n, nq=nq)
    log("serving-file: %d x 128 u8 vectors, %d queries in %.1fs" % (n, nq, time.time() - t))
    kth = ground_truth(base, q, 10, torch, dev)
    os.environ["FLASHANN_BUILD_PROGRESS"] = "1"
    t = time.time()
    adj, entry = synth.build_graph(base, cfg.R, 3000 + cfg.seed_offset,
                                   threads=min(16, os.cpu_count() or 1))
    t_graph = time.time() - t
    log("serving-file: graph R=%d in %.1fs" % (cfg.R, t_graph))
    tmpd = tempfile.mkdtemp(prefix="flashann_serve_", dir=os.environ.get("TMPDIR", "/tmp"))
    try:
        t = time.time()
        fa.save_index(tmpd, base, adj, entry, cfg.slot)
        t_save = time.time() - t
        del adj
        out = {"workload": "%d x 128 u8 (4,096-component mixture), R=64, 512 B records in a "
                           "file (O_DIRECT), served by the server's own agents" % n,
               "graph_build_s": round(t_graph, 1), "write_s": round(t_save, 1)}
        with fa.Index.load(tmpd, fa.TIER_FILE) as ix:
            out["direct_io"] = ix.info()["direct_io"]
            qs = torch.from_numpy(q[:2000]).to(dev)
            L_op = L_SWEEP[-1]
            sweep = []
            for L in L_SWEEP:
                _, d_, s_ = fa.search(ix, qs, k=10, L=L, delay=1)
                torch.cuda.synchronize()
                rec = recall_at(d_.cpu().numpy().view(np.uint32), kth[:2000])
                sweep.append({"L": L, "recall@10": round(rec, 4)})
                if rec >= 0.95:
                    L_op = L
                    break
            out["L_op"], out["sweep"] = L_op, sweep
            log("serving-file: L_op %d (%s)" % (L_op, sweep))
            Lset = [L for L in L_SWEEP if L >= L_op]

            def recall(res):
                qi = (res["tags"] % nq).astype(np.int64)
                d10 = res["dists"][:, :10].astype(np.float64)
                return float((np.minimum((d10 <= kth[qi][:, None]).sum(1), 10) / 10.0).mean())

            def serve():
                rng = np.random.default_rng(29)

                def mix(cnt):
                    ks = rng.choice(np.array([10, 100], np.int32), cnt)
                    return ks, np.array([rng.choice([L for L in Lset if L >= k]) for k in ks],
                                        np.int32)

                res_out = {}
                with fa.Server(ix, hbm_budget_bytes=256 << 20) as srv:
                    ks, Ls = mix(m)
                    # queries the L sweep did not touch: their records are cold,
                    # as they are for the arrivals that follow
                    idx = 2000 + rng.integers(0, nq - 2000, m)
                    t0 = fa.clock_us()
                    srv.submit_batch(q[idx], ks, Ls, idx.astype(np.uint64))
                    res = srv.drain(m, timeout_s=300)
                    qmax = m / ((res["done_us"].max() - t0) / 1e6)
                    res_out["saturation_qps"] = round(qmax, 1)
                    res_out["saturation_recall@10"] = round(recall(res), 4)
                    res_out["failed_reads"] = int((res["status"] != 0).sum())
                    rates = []
                    for frac in (0.25, 0.5, 0.75, 0.9):
                        lam = frac * qmax
                        ks, Ls = mix(m)
                        idx = 2000 + rng.integers(0, nq - 2000, m)
                        start = fa.clock_us() + 20000.0
                        arr = start + np.cumsum(rng.exponential(1e6 / lam, m))
                        srv.submit_batch(q[idx], ks, Ls, idx.astype(np.uint64), arr)
                        res = srv.drain(m, timeout_s=300)
                        lat = (res["done_us"] - res["submit_us"]) / 1e3
                        rates.append({"offered_qps": round(lam, 1), "queries": int(len(lat)),
                                      "latency_ms_p50": round(float(np.percentile(lat, 50)), 3),
                                      "latency_ms_p99": round(float(np.percentile(lat, 99)), 3),
                                      "recall@10": round(recall(res), 4),
                                      "failed_reads": int((res["status"] != 0).sum())})
                        log("serving-file at %.0f QPS offered: %s" % (lam, rates[-1]))
                    res_out["rates"] = rates
                return res_out

            if cache_fraction > 0:
                # hot set from training queries of another seed, traced at L_op
                qt = torch.from_numpy(synth.gmm.make_queries(10000, cfg.d, cfg.dtype, cfg.components,
                                                             1000 + cfg.seed_offset,
                                                             7000 + cfg.seed_offset)).to(dev)
                tr = torch.full((qt.shape[0], 600), -1, dtype=torch.int32, device=dev)
                t = time.time()
                fa.search(ix, qt, k=10, L=max(L_op, 64), trace=tr)
                torch.cuda.synchronize()
                visits = torch.bincount(tr[tr >= 0].long(), minlength=n)
                hot = torch.argsort(visits, descending=True, stable=True)[:int(cache_fraction * n)]
                t_hot = time.time() - t
                t = time.time()
                ix.set_record_cache(hot.cpu().numpy())
                t_fill = time.time() - t
                cached = serve()
                ix.set_record_cache([])
                cached.update({"fraction": cache_fraction, "records": int(hot.numel()),
                               "hot_set_s": round(t_hot, 1), "fill_s": round(t_fill, 1)})
                out["hot_cache"] = cached
                log("serving-file with %.0f%% of the records cached: %s"
                    % (100 * cache_fraction, cached))
            out.update(serve())
            prof = ix.agent_profile()
            out["agent"] = {"threads": prof["threads"], "async_io": prof["async_io"]}
    finally:
        shutil.rmtree(tmpd, ignore_errors=True)
    log("serving-file: %s" % out)
    return out


def batched_file_leg(fa, torch, dev, n, nq_total, cache_fraction=0.0):
    """Batched form at scale: n int8 vectors of d = 100 (4,096-component
    mixture), degree-48 graph, 512 B records in a file read with O_DIRECT by
    the host agents, nq_total queries with L uniform over {32, 64, 128, 256}
    in one persistent launch; schedule and tiles chosen by the autotuner on a
    10,000-query sample.  Recall@10 on the first 1,000 queries.

    With cache_fraction > 0 the same launch also runs with that share of the
    records in the hot-record cache (the most-expanded nodes of 10,000
    training queries of another seed, traced at L = 128).  The cached launch
    runs first, so the disk has seen its records less often than those of
    the uncached launch that follows; both must return identical results."""
    import shutil
    import tempfile

    import numpy as np

    import synth
    from paper_2507_10070_amd import autotune

    t = time.time()
    base = synth.make_base(n, 100, "i8", 4096, 1004)
    q = synth.make_queries(nq_total, 100, "i8", 4096, 1004, 2004)
    log("batched-file: %d x 100 i8 vectors, %d queries in %.1fs" % (n, nq_total, time.time() - t))
    os.environ["FLASHANN_BUILD_PROGRESS"] = "1"
    t = time.time()
    adj, entry = synth.build_graph(base, 48, 3004, threads=min(16, os.cpu_count() or 1))
    t_graph = time.time() - t
    log("batched-file: graph R=48 in %.1fs" % t_graph)
    # exact 10th-neighbour distance of the first 1,000 queries
    kth = ground_truth(base, q[:1000], 10, torch, dev)
    tmpd = tempfile.mkdtemp(prefix="flashann_batched_", dir=os.environ.get("TMPDIR", "/tmp"))
    try:
        t = time.time()
        fa.save_index(tmpd, base, adj, entry, 512)
        t_save = time.time() - t
        del adj
        log("batched-file: index files written in %.1fs" % t_save)
        ix = fa.Index.load(tmpd, fa.TIER_FILE)
        qd = torch.from_numpy(q).to(dev)
        Lq = np.random.default_rng(19).choice(np.array([32, 64, 128, 256], np.int32), nq_total)
        Lt = torch.from_numpy(Lq).to(dev)

        def score(i_, d_, s_):
            return recall_at(d_[:1000].cpu().numpy().view(np.uint32), kth)

        ns = min(10000, nq_total)
        t = time.time()
        tuned = autotune.tune(ix, qd[:ns].contiguous(), 10, 256, cache_path=None, reps=1,
                              passes=1, score=score,
                              space={"delay": (0, 1, 2), "beam_width": (1, 2),
                                     "persistent": (False, True)},
                              progress=lambda row: log("batched-file tune %s" % row),
                              L_per_query=Lt[:ns].contiguous())
        t_tune = time.time() - t
        kw = autotune.search_kwargs(tuned["params"], {"L_per_query": Lt})
        cached = None
        if cache_fraction > 0:
            qt = torch.from_numpy(synth.make_queries(10000, 100, "i8", 4096, 1004, 7004)).to(dev)
            tr = torch.full((qt.shape[0], 600), -1, dtype=torch.int32, device=dev)
            t = time.time()
            fa.search(ix, qt, k=10, L=128, trace=tr)
            torch.cuda.synchronize()
            visits = torch.bincount(tr[tr >= 0].long(), minlength=n)
            hot = torch.argsort(visits, descending=True, stable=True)[:int(cache_fraction * n)]
            t_hot = time.time() - t
            t = time.time()
            ix.set_record_cache(hot.cpu().numpy())
            t_fill = time.time() - t
            t = time.perf_counter()
            c_ids, c_dists, c_steps = fa.search(ix, qd, k=10, L=256, **kw)
            torch.cuda.synchronize()
            el_c = time.perf_counter() - t
            ix.set_record_cache([])
            cached = {"fraction": cache_fraction, "records": int(hot.numel()),
                      "cache_MB": round(int(hot.numel()) * 512 / 1e6, 1),
                      "hot_set_s": round(t_hot, 1), "fill_s": round(t_fill, 1),
                      "qps": round(nq_total / el_c, 1), "seconds": round(el_c, 2)}
            log("batched-file with %.0f%% of the records cached: %s" % (100 * cache_fraction, cached))
        t = time.perf_counter()
        ids, dists, steps = fa.search(ix, qd, k=10, L=256, **kw)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        if cached is not None:
            cached["identical_results"] = bool(torch.equal(ids, c_ids) and torch.equal(dists, c_dists)
                                               and torch.equal(steps, c_steps))
        out = {"workload": "%d x 100 i8, R=48, 512 B records in a file (O_DIRECT)" % n,
               "queries": nq_total, "L": [32, 64, 128, 256], "k": 10,
               "params": tuned["params"], "qps": round(nq_total / el, 1),
               "seconds": round(el, 2),
               "recall@10_first_1000": round(score(ids, dists, steps), 4),
               "mean_steps": round(float(steps.cpu().numpy().view(np.uint32).mean()), 1),
               "default_sample_qps": round(ns / (tuned["default"]["ms"] / 1e3), 1),
               "tuned_sample_qps": round(ns / (tuned["ms"] / 1e3), 1),
               "tune_s": round(t_tune, 1), "graph_build_s": round(t_graph, 1),
               "write_s": round(t_save, 1), "direct_io": ix.info()["direct_io"]}
        if cached is not None:
            out["hot_cache"] = cached
        ix.close()
    finally:
        shutil.rmtree(tmpd, ignore_errors=True)
    log("batched-file: %s" % out)
    return out


def hot_cache_leg(fa, torch, dev, ix, qd, cfg, k, op, info, out, stream,
                  fractions=(0.01, 0.05, 0.1, 0.2), n_train=10000):
    """Headline index and queries with a hot-record cache in HBM.  The hot
    set is the most-expanded nodes of n_train training queries drawn from the
    same mixture with another seed (never the timed queries).  Per cache size:
    the share of the timed queries' expansions it serves (from traces), QPS of
    both schedules at their operating L, and the record bytes per second that
    still cross the host link."""
    import numpy as np

    import synth

    n = info["n"]
    qt = synth.gmm.make_queries(n_train, cfg.d, cfg.dtype, cfg.components, 1000 + cfg.seed_offset,
                                7000 + cfg.seed_offset)
    qtd = torch.from_numpy(qt).to(dev)
    cap = 512

    def visits(queries, L):
        tr = torch.full((queries.shape[0], cap), -1, dtype=torch.int32, device=dev)
        fa.search(ix, queries, k=k, L=L, delay=1, trace=tr, stream=stream)
        torch.cuda.synchronize()
        t = tr[tr >= 0].long()
        return torch.bincount(t, minlength=n)

    hot_order = torch.argsort(visits(qtd, op[1]), descending=True, stable=True).cpu().numpy()
    test_visits = visits(qd, op[1])
    total = float(test_visits.sum().item())

    def timed(L, delay, reps=10):
        fa.search(ix, qd, k=k, L=L, delay=delay, out=out, stream=stream)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(stream)
        for _ in range(reps):
            fa.search(ix, qd, k=k, L=L, delay=delay, out=out, stream=stream)
        ev[1].record(stream)
        torch.cuda.synchronize()
        return ev[0].elapsed_time(ev[1]) / reps

    rows = []
    try:
        for f in fractions:
            m = int(f * n)
            ids = hot_order[:m]
            ix.set_record_cache(ids)
            covered = float(test_visits[torch.from_numpy(ids).to(dev).long()].sum().item()) / total
            ms = {d: timed(op[d], d) for d in (0, 1)}
            link = (1.0 - covered) * total * info["rec_bytes"]
            rows.append({"fraction": f, "records": m,
                         "cache_MB": round(m * info["slot_bytes"] / 1e6, 1),
                         "expansions_served": round(covered, 4),
                         "relaxed_qps": round(qd.shape[0] / (ms[1] / 1e3), 1),
                         "strict_qps": round(qd.shape[0] / (ms[0] / 1e3), 1),
                         "link_GBps_relaxed": round(link / (ms[1] / 1e3) / 1e9, 2)})
    finally:
        ix.set_record_cache([])
    return ({"hot_set": "most-expanded nodes of %d training queries (another seed), relaxed, L=%d"
                        % (n_train, op[1]), "rows": rows}, hot_order)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=None, help="base vectors (default: workload size)")
    ap.add_argument("--nq", type=int, default=None, help="queries (default: workload size)")
    ap.add_argument("--tier", choices=("host", "hbm"), default="host")
    ap.add_argument("--L", type=int, default=0, help="fixed L (skip the sweep)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=10000,
                    help="queries per oracle pass in the CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="repeat oracle passes until this much CPU time has elapsed")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the continuous-batching serving measurement")
    ap.add_argument("--serving-budget-mb", type=int, default=256,
                    help="HBM budget of the serving admission")
    ap.add_argument("--no-schedule-sweep", action="store_true",
                    help="skip the (delay, beam width) sweep")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the autotuned uneven-L batch")
    ap.add_argument("--batched-queries", type=int, default=100000)
    ap.add_argument("--serving-file-cache", type=float, default=0.0,
                    help="with --serving-file-n: also serve with this share of the records in "
                         "the hot-record cache")
    ap.add_argument("--batched-file-cache", type=float, default=0.0,
                    help="with --batched-file-n: also run with this share of the records in "
                         "the hot-record cache")
    ap.add_argument("--batched-file-n", type=int, default=0,
                    help="also run the batched form at scale: this many int8/100 vectors, "
                         "records in a file (off by default: minutes of graph build)")
    ap.add_argument("--serving-file-n", type=int, default=0,
                    help="opt-in: the serving form with records in a file at this size "
                         "(u8/128, 4,096-component mixture, R=64); with --serving-file-only "
                         "nothing else runs")
    ap.add_argument("--serving-file-only", action="store_true")
    ap.add_argument("--f32-file-n", type=int, default=0,
                    help="opt-in: the f32/96 workload with 4 KB record slots in a file at this "
                         "size (10M = 41 GB of records), one real graph per --f32-R degree")
    ap.add_argument("--f32-R", type=int, nargs="+", default=[32, 48, 64, 96])
    ap.add_argument("--f32-L", type=int, default=128)
    ap.add_argument("--f32-nq", type=int, default=10000)
    ap.add_argument("--f32-keep", default=None,
                    help="keep the last degree's index directory here (for the sampled "
                         "oracle check)")
    ap.add_argument("--f32-tier", choices=("file", "host", "hbm"), default="file")
    ap.add_argument("--f32-only", action="store_true",
                    help="run only the f32 file leg and print its JSON")
    ap.add_argument("--no-hot-cache", action="store_true",
                    help="skip the hot-record cache measurement")
    ap.add_argument("--no-hbm-tier", action="store_true",
                    help="skip the same search with the records in HBM")
    ap.add_argument("--no-transports", action="store_true",
                    help="skip the agent-transport and file-tier measurements")
    ap.add_argument("--file-queries", type=int, default=1000,
                    help="queries of the file-tier measurement (records read with O_DIRECT)")
    ap.add_argument("--no-pq", action="store_true",
                    help="skip the compressed (PQ) navigation leg")
    ap.add_argument("--pq-kernel-only", action="store_true",
                    help="run only one compressed-navigation configuration (for profiling)")
    ap.add_argument("--pq-n", type=int, default=0,
                    help="run only the compressed-navigation leg on an n-vector index of "
                         "intrinsic dimension 16 (e.g. 10000000)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 256 MiB device-to-device copy (scale reference "
                         "for memory counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported "
              "(across GPUs the search would shard by query, each GPU holding its own "
              "navigation copy)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    import paper_2507_10070_amd as fa

    fa.load_library()
    dev = torch.device("cuda:0")
    if args.pq_kernel_only:
        pq_kernel_run(fa, torch, dev, args.steps)
        return
    if args.pq_n:
        pq_scale_run(fa, torch, dev, args.pq_n)
        return
    if args.serving_file_only:
        if not args.serving_file_n:
            sys.exit("--serving-file-only needs --serving-file-n")
        print(json.dumps({"serving_file": serving_file_leg(
            fa, torch, dev, args.serving_file_n, cache_fraction=args.serving_file_cache)}),
              flush=True)
        return
    if args.f32_only:
        if not args.f32_file_n:
            sys.exit("--f32-only needs --f32-file-n")
        res = f32_file_leg(fa, torch, dev, args.f32_file_n, args.f32_R, args.f32_nq, args.f32_L,
                           args.f32_keep, args.f32_tier)
        print(json.dumps({"f32_file": res}), flush=True)
        return
    cfg = synth.WORKLOADS["1m-u8-128"]
    n = args.n or cfg.n
    nq = args.nq or cfg.nq
    k = cfg.k

    log("generating %d x %d %s mixture vectors, %d queries" % (n, cfg.d, cfg.dtype, nq))
    base, queries = synth.make_dataset(cfg, n=n, nq=nq)
    t = time.time()
    threads = min(16, os.cpu_count() or 1)
    adj, entry = synth.build_graph(base, cfg.R, 3000 + cfg.seed_offset, threads=threads)
    t_graph = time.time() - t
    log("graph R=%d built in %.1fs (entry %d)" % (cfg.R, t_graph, entry))
    kth = ground_truth(base, queries, k, torch, dev)
    log("ground truth done")
    tier = fa.TIER_HOST if args.tier == "host" else fa.TIER_HBM
    ix = fa.Index(base, adj, entry, cfg.slot, tier)
    info = ix.info()
    qd = torch.from_numpy(queries).to(dev)
    ids = torch.empty((nq, k), dtype=torch.int32, device=dev)
    dists = torch.empty((nq, k), dtype=torch.int32, device=dev)
    steps = torch.empty((nq,), dtype=torch.int32, device=dev)
    out = (ids, dists, steps)
    stream = torch.cuda.current_stream(dev)

    def run(L, delay, **kw):
        return fa.search(ix, qd, k=k, L=L, delay=delay, out=out, stream=stream, **kw)

    # ---- operating points: smallest L with recall@10 >= 0.95 per schedule
    sweep = {}
    op = {}
    for delay in (0, 1):
        for L in ((args.L,) if args.L else L_SWEEP):
            run(L, delay)
            torch.cuda.synchronize()
            rec = recall_at(dists.cpu().numpy().view(np.uint32), kth)
            sweep.setdefault(delay, []).append({"L": L, "recall@10": round(rec, 4),
                                                "mean_steps": float(steps.cpu().numpy().mean())})
            if rec >= 0.95 and delay not in op:
                op[delay] = L
        op.setdefault(delay, sweep[delay][-1]["L"])
        log("delay %d sweep: %s" % (delay, sweep[delay]))

    # ---- per-query latency, counters and steps at each operating point
    khz = fa.device_clock_khz()
    detail = {}
    for delay in (0, 1):
        L = op[delay]
        stats = torch.zeros(3, dtype=torch.int64, device=dev)
        times = torch.zeros((nq, 2), dtype=torch.int64, device=dev)
        run(L, delay, stats=stats, times=times)
        torch.cuda.synchronize()
        tt = times.cpu().numpy()
        lat_ms = (tt[:, 1] - tt[:, 0]) / khz
        s = stats.cpu().numpy()
        detail[delay] = {"L": L, "expansions": int(s[0]), "rows_scored": int(s[1]),
                         "record_mismatches": int(s[2]),
                         "recall@10": recall_at(dists.cpu().numpy().view(np.uint32), kth),
                         "query_latency_ms_p50": float(np.percentile(lat_ms, 50)),
                         "query_latency_ms_p99": float(np.percentile(lat_ms, 99))}

    # ---- timed region: K launches per schedule, HIP events on the launch stream
    def timed(L, delay, steps_=None, warmup_=None, **kw):
        steps_ = args.steps if steps_ is None else steps_
        for _ in range(args.warmup if warmup_ is None else warmup_):
            run(L, delay, **kw)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps_ + 1)]
        ev[0].record(stream)
        for i in range(steps_):
            run(L, delay, **kw)
            ev[i + 1].record(stream)
        torch.cuda.synchronize()
        per = [ev[i].elapsed_time(ev[i + 1]) for i in range(steps_)]
        return sum(per) / len(per)

    log("timing strict at L=%d and relaxed at L=%d" % (op[0], op[1]))
    ms = {d: timed(op[d], d) for d in (0, 1)}
    ms_equal_L = timed(op[1], 0) if op[0] != op[1] else ms[0]
    qps = {d: nq / (ms[d] / 1e3) for d in (0, 1)}
    log("ms/launch strict %.3f relaxed %.3f" % (ms[0], ms[1]))

    # ---- roofline of the search kernel (algorithmic bytes per launch)
    d1 = detail[1]
    sec = ms[1] / 1e3
    link_bytes = d1["expansions"] * info["rec_bytes"]
    hbm_bytes = d1["rows_scored"] * info["nav_stride"] + nq * (cfg.d + 8 * k + 4)
    if tier == fa.TIER_HBM:
        hbm_bytes += link_bytes
        link_bytes = 0
    # host-link probe: a large pinned host -> device copy
    src = torch.empty(1 << 30, dtype=torch.uint8).pin_memory()
    dst = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    dst.copy_(src, non_blocking=True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(4):
        dst.copy_(src, non_blocking=True)
    e1.record(stream)
    torch.cuda.synchronize()
    link_peak = 4 * (1 << 30) / (e0.elapsed_time(e1) / 1e3) / 1e9
    del src, dst
    workload = "custom"
    if (n, nq) == (cfg.n, cfg.nq):
        workload = "1M-u8-128-R64-512B-%s-10kq" % ("host" if tier == fa.TIER_HOST else "hbm")
    hbm_ach = hbm_bytes / sec / 1e9
    roofline = {"bound": "hbm", "binding": "host_link" if link_bytes else "hbm",
                "achieved": round(hbm_ach, 2), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(hbm_ach / HBM_PEAK_GBS, 5),
                "traffic": stored_traffic(workload, op[1]),
                "algorithmic_bytes_per_launch": hbm_bytes,
                "host_link": {"achieved": round(link_bytes / sec / 1e9, 2),
                              "peak_probe": round(link_peak, 2), "unit": "GB/s",
                              "frac": round(link_bytes / sec / 1e9 / link_peak, 4),
                              "bytes_per_launch": link_bytes}}

    # ---- relaxed vs strict as the batch shrinks: with fewer queries in flight
    # the host link is no longer saturated and each query's fetch latency is
    # exposed, which is where the relaxed pipeline pays (section 4.1)
    concurrency = None
    if not args.no_schedule_sweep:
        concurrency = []
        for nb in (128, 512, 2048, nq):
            qsub = qd[:nb].contiguous()
            ob = (torch.empty((nb, k), dtype=torch.int32, device=dev),
                  torch.empty((nb, k), dtype=torch.int32, device=dev),
                  torch.empty((nb,), dtype=torch.int32, device=dev))
            row = {"queries": nb}
            for name, delay in (("strict", 0), ("relaxed", 1)):
                for _ in range(2):
                    fa.search(ix, qsub, k=k, L=op[1], delay=delay, out=ob, stream=stream)
                ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
                reps_c = 10
                ev[0].record(stream)
                for _ in range(reps_c):
                    fa.search(ix, qsub, k=k, L=op[1], delay=delay, out=ob, stream=stream)
                ev[1].record(stream)
                torch.cuda.synchronize()
                row[name + "_qps"] = round(nb / (ev[0].elapsed_time(ev[1]) / reps_c / 1e3), 1)
            row["relaxed_vs_strict"] = round(row["relaxed_qps"] / row["strict_qps"], 4)
            concurrency.append(row)
            log("concurrency %s" % row)

    # ---- staleness delta and beam width W at the relaxed operating L: steps,
    # recall and throughput of each schedule (direct loads; agent transport
    # too when records are in host DRAM)
    schedules = None
    if not args.no_schedule_sweep:
        schedules = []
        Lr = op[1]
        for delay, beam in SCHEDULES:
            run(Lr, delay, beam_width=beam)
            torch.cuda.synchronize()
            row = {"delay": delay, "W": beam,
                   "recall@10": round(recall_at(dists.cpu().numpy().view(np.uint32), kth), 4),
                   "mean_steps": round(float(steps.cpu().numpy().mean()), 2)}
            row["qps"] = round(nq / (timed(Lr, delay, 3, 1, beam_width=beam) / 1e3), 1)
            if tier == fa.TIER_HOST and not args.no_transports:
                t = time.perf_counter()
                run(Lr, delay, beam_width=beam, transport=fa.TRANSPORT_AGENT)
                row["agent_qps"] = round(nq / (time.perf_counter() - t), 1)
            schedules.append(row)
            log("schedule %s" % row)

    # ---- batched form: 100k searches with L uniform over {32, 64, 128, 256}
    # in one launch, tiles and schedule chosen by the autotuner
    batched = None
    if not args.no_batched:
        from paper_2507_10070_amd import autotune

        nb = args.batched_queries
        rng = np.random.default_rng(17)
        rows = rng.integers(0, nq, nb)
        qb = qd[torch.from_numpy(rows).to(dev)].contiguous()
        Lq = rng.choice(np.array([32, 64, 128, 256], np.int32), nb)
        Lt = torch.from_numpy(Lq).to(dev)
        kthb = kth[rows]

        def score(i_, d_, s_):
            return recall_at(d_.cpu().numpy().view(np.uint32), kthb)

        t = time.time()
        tuned = autotune.tune(ix, qb, k, 256, score=score, cache_path=None, reps=2,
                              L_per_query=Lt)
        t_tune = time.time() - t
        kw = autotune.search_kwargs(tuned["params"], {"L_per_query": Lt})
        ob = (torch.empty((nb, k), dtype=torch.int32, device=dev),
              torch.empty((nb, k), dtype=torch.int32, device=dev),
              torch.empty((nb,), dtype=torch.int32, device=dev))
        fa.search(ix, qb, k=k, L=256, out=ob, stream=stream, **kw)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(stream)
        reps_b = 3
        for _ in range(reps_b):
            fa.search(ix, qb, k=k, L=256, out=ob, stream=stream, **kw)
        ev[1].record(stream)
        torch.cuda.synchronize()
        ms_b = ev[0].elapsed_time(ev[1]) / reps_b
        batched = {"queries": nb, "L": [32, 64, 128, 256], "k": k,
                   "tuned": {"params": tuned["params"], "qps": round(nb / (ms_b / 1e3), 1),
                             "ms_per_launch": round(ms_b, 3),
                             "recall@10": round(score(*ob), 4)},
                   "default": {"params": tuned["default"]["params"],
                               "qps": round(nb / (tuned["default"]["ms"] / 1e3), 1),
                               "recall@10": round(tuned["default"]["score"], 4)},
                   "settings_tried": len(tuned["table"]), "tune_s": round(t_tune, 1)}
        log("batched: %s" % batched)
        del qb, ob

    batched_file = None
    if args.batched_file_n:
        batched_file = batched_file_leg(fa, torch, dev, args.batched_file_n, args.batched_queries,
                                        args.batched_file_cache)
    serving_file = None
    if args.serving_file_n:
        serving_file = serving_file_leg(fa, torch, dev, args.serving_file_n,
                                        cache_fraction=args.serving_file_cache)
    f32_file = None
    if args.f32_file_n:
        f32_file = f32_file_leg(fa, torch, dev, args.f32_file_n, args.f32_R, args.f32_nq,
                                args.f32_L, args.f32_keep, args.f32_tier)

    # ---- the same index with its records in HBM: the kernel without the host
    # link in the way (where the HBM roofline applies)
    # Both threads-per-query tiles: one query per wave64 (the keys "strict"
    # and "relaxed") and two queries per wave ("two_per_wave", at the default
    # 2^10-slot hash and at 2^9, which lets more queries share a CU's LDS).
    hbm_tier = None
    if tier == fa.TIER_HOST and not args.no_hbm_tier:
        with fa.Index(base, adj, entry, cfg.slot, fa.TIER_HBM) as hix:
            def hbm_measure(delay, **kw):
                st_ = torch.zeros(3, dtype=torch.int64, device=dev)
                fa.search(hix, qd, k=k, L=op[1], delay=delay, out=out, stream=stream, stats=st_,
                          **kw)
                torch.cuda.synchronize()
                s_ = st_.cpu().numpy()
                ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
                ev[0].record(stream)
                for _ in range(5):
                    fa.search(hix, qd, k=k, L=op[1], delay=delay, out=out, stream=stream, **kw)
                ev[1].record(stream)
                torch.cuda.synchronize()
                ms_h = ev[0].elapsed_time(ev[1]) / 5
                byt = int(s_[0]) * info["rec_bytes"] + int(s_[1]) * info["nav_stride"] + \
                    nq * (cfg.d + 8 * k + 4)
                return {"qps": round(nq / (ms_h / 1e3), 1), "ms_per_step": round(ms_h, 4),
                        "algorithmic_GBps": round(byt / (ms_h / 1e3) / 1e9, 1),
                        "hbm_frac": round(byt / (ms_h / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}

            hbm_tier = {}
            for name, delay in (("strict", 0), ("relaxed", 1)):
                hbm_tier[name] = hbm_measure(delay)
            pair = {}
            for name, delay in (("strict", 0), ("relaxed", 1)):
                for hb in (10, 9):
                    pair["%s_hash%d" % (name, hb)] = hbm_measure(delay, query_lanes=32,
                                                                 hash_bits=hb)
            hbm_tier["two_per_wave"] = pair
            log("records in HBM: %s" % hbm_tier)
        # the same choice with records in host DRAM (bound by the host link)
        t0 = time.time()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        fa.search(ix, qd, k=k, L=op[1], delay=1, out=out, stream=stream, query_lanes=32)
        ev[0].record(stream)
        for _ in range(5):
            fa.search(ix, qd, k=k, L=op[1], delay=1, out=out, stream=stream, query_lanes=32)
        ev[1].record(stream)
        torch.cuda.synchronize()
        hbm_tier["two_per_wave_host_relaxed_qps"] = round(nq / (ev[0].elapsed_time(ev[1]) / 5e3), 1)
        log("two queries per wave, records in DRAM: %.0f QPS (%.1fs)"
            % (hbm_tier["two_per_wave_host_relaxed_qps"], time.time() - t0))

    # ---- hot-record cache: the most-visited records of a separate sample of
    # training queries copied into HBM, the rest read over the host link
    hot_cache = hot_order = None
    if tier == fa.TIER_HOST and not args.no_hot_cache:
        hot_cache, hot_order = hot_cache_leg(fa, torch, dev, ix, qd, cfg, k, op, info, out, stream)
        log("hot-record cache: %s" % hot_cache)

    # ---- compressed navigation: PQ codes in HBM, exact re-rank from records,
    # on this workload (isotropic clusters: the hard case for PQ) and on one of
    # intrinsic dimension 16 (the structure of real descriptors)
    pq = None
    if not args.no_pq and tier == fa.TIER_HOST:
        pq = {"isotropic": pq_leg(fa, torch, dev, base, adj, entry, cfg, ix, qd, kth, op[1],
                                  stream, (16, 32))}
        lcfg = synth.WORKLOADS["1m-u8-128-latent16"]
        lbase, lq = synth.make_dataset(lcfg, n=n, nq=nq)
        ladj, lentry = synth.build_graph(lbase, lcfg.R, 3000 + lcfg.seed_offset, threads=threads)
        lkth = ground_truth(lbase, lq, k, torch, dev)
        log("latent-16 workload ready")
        with fa.Index(lbase, ladj, lentry, lcfg.slot, tier) as lix:
            pq["latent16"] = pq_leg(fa, torch, dev, lbase, ladj, lentry, lcfg, lix,
                                    torch.from_numpy(lq).to(dev), lkth, None, stream, (16, 32),
                                    queries_host=lq)
        del lbase, ladj

    # ---- the paper's query-grained I/O stack on the same workload: agent
    # transport from pinned DRAM (all queries) and from a file (O_DIRECT)
    transports = None
    if not args.no_transports:
        import tempfile

        transports = {}

        def measure(index, qsub, L, delay, reps, **kw):
            outs = (torch.empty((qsub.shape[0], k), dtype=torch.int32, device=dev),
                    torch.empty((qsub.shape[0], k), dtype=torch.int32, device=dev),
                    torch.empty((qsub.shape[0],), dtype=torch.int32, device=dev))
            times = torch.zeros((qsub.shape[0], 2), dtype=torch.int64, device=dev)
            fa.search(index, qsub, k=k, L=L, delay=delay, transport=fa.TRANSPORT_AGENT, out=outs,
                      times=times, **kw)
            tt = times.cpu().numpy()
            lat = (tt[:, 1] - tt[:, 0]) / khz
            p0 = index.agent_profile()
            t = time.perf_counter()
            for _ in range(reps):
                fa.search(index, qsub, k=k, L=L, delay=delay, transport=fa.TRANSPORT_AGENT,
                          out=outs, **kw)
            el = (time.perf_counter() - t) / reps
            p1 = index.agent_profile()
            out = {"qps": round(qsub.shape[0] / el, 1), "ms_per_step": round(el * 1e3, 3),
                   "query_latency_ms_p50": round(float(np.percentile(lat, 50)), 3),
                   "query_latency_ms_p99": round(float(np.percentile(lat, 99)), 3)}
            out.update(agent_split(p0, p1, el * reps))
            return out

        def agent_split(p0, p1, wall_s):
            """Where the agent threads' time went over a timed region: requests
            per second, the fraction of the threads' wall time spent scanning
            request lines, copying records or doing file I/O, and requests per
            busy scan (the batch one pass serves)."""
            d = {key: p1[key] - p0[key] for key in ("requests", "passes", "busy_passes",
                                                    "scan_ns", "copy_ns", "io_ns")}
            thr_s = max(1e-9, wall_s * p1["threads"])
            return {"agent": {"threads": p1["threads"], "async_io": p1["async_io"],
                              "requests_per_s": round(d["requests"] / wall_s, 1),
                              "scan_frac": round(d["scan_ns"] / 1e9 / thr_s, 3),
                              "copy_frac": round(d["copy_ns"] / 1e9 / thr_s, 3),
                              "io_frac": round(d["io_ns"] / 1e9 / thr_s, 3),
                              "requests_per_busy_pass": round(d["requests"] / max(1, d["busy_passes"]), 1),
                              "passes_per_s_per_thread": round(d["passes"] / thr_s, 1)}}

        # query-grained (each query waits for its own records; relaxed and
        # strict) against kernel-grained (lockstep rounds, strict)
        modes = (("relaxed", 1, {}), ("strict", 0, {}),
                 ("kernel_grained", 0, {"sync_grain": fa.SYNC_KERNEL}))

        def compare(index, qsub, reps, rounds):
            res = {m: [] for m, _, _ in modes}
            for _ in range(rounds):  # alternate the modes so drift hits all alike
                for m, delay, kw in modes:
                    res[m].append(measure(index, qsub, op[1], delay, reps, **kw))
            def mean_rows(rows):
                return {key: (mean_rows([r[key] for r in rows]) if isinstance(rows[0][key], dict)
                              else round(float(np.mean([r[key] for r in rows])), 3))
                        for key in rows[0]}

            return {m: mean_rows(rows) for m, rows in res.items()}

        if tier == fa.TIER_HOST:
            reps = max(1, min(args.steps, 3))
            transports["agent_host"] = {"queries": nq, "L": op[1], **compare(ix, qd, reps, 1)}
            st = ix.agent_stats()
            transports["agent_host"]["agent_threads_requests"] = st["requests"]
            # the GPU's completion polls share the host link with the staged
            # records: the pause between polls, short (4 units, ~1.7 us) and
            # the default (32 units, ~14 us)
            transports["agent_host"]["poll_backoff"] = {
                str(pb): measure(ix, qd, op[1], 1, reps, poll_backoff=pb)["qps"] for pb in (4, 32, 128)}
            if hot_order is not None:
                # the same with the hottest 10 % of the records in HBM: the
                # agents get no request for those nodes
                ix.set_record_cache(hot_order[:n // 10])
                try:
                    transports["agent_host"]["hot_cache_10pct"] = compare(ix, qd, reps, 1)
                finally:
                    ix.set_record_cache([])
            log("agent transport: %s" % transports["agent_host"])
            # the relaxed pipeline where fetch latency, not bandwidth, binds:
            # fewer queries in flight through the agents
            conc = {}
            for m in (256, 1024, 4096):
                qm = qd[:m].contiguous()
                conc[str(m)] = {name: measure(ix, qm, op[1], delay, max(reps, 3))["qps"]
                                for name, delay in (("relaxed", 1), ("strict", 0))}
                conc[str(m)]["relaxed_vs_strict"] = round(conc[str(m)]["relaxed"] /
                                                          conc[str(m)]["strict"], 3)
            transports["agent_host"]["concurrency"] = conc
            log("agent transport by queries in flight: %s" % conc)
            if not args.no_serving:
                # the server with its own host agents over the same DRAM records
                transports["agent_host"]["serving"] = serving_burst(
                    fa, ix, queries, kth, op[1], m=20000, where="records in pinned host DRAM, "
                    "served through the host agents", transport=fa.TRANSPORT_AGENT)
            kg = timed(op[1], 0, 3, 1, sync_grain=fa.SYNC_KERNEL)
            transports["direct_host"] = {
                "queries": nq, "L": op[1],
                "relaxed": {"qps": round(nq / (ms[1] / 1e3), 1)},
                "strict": {"qps": round(nq / (ms_equal_L / 1e3), 1)},
                "kernel_grained": {"qps": round(nq / (kg / 1e3), 1)}}
            log("direct transport: %s" % transports["direct_host"])
        tmpd = tempfile.mkdtemp(prefix="flashann_", dir=os.environ.get("TMPDIR", "/tmp"))
        try:
            t = time.time()
            fa.save_index(tmpd, base, adj, entry, cfg.slot)
            t_save = time.time() - t
            fix = fa.Index.load(tmpd, fa.TIER_FILE)
            mq = min(args.file_queries, nq)
            qsub = qd[:mq].contiguous()
            fa.search(fix, qsub, k=k, L=op[1])  # warm-up pass
            transports["file"] = {"queries": mq, "L": op[1], "direct_io": fix.info()["direct_io"],
                                  "write_s": round(t_save, 1), **compare(fix, qsub, 1, 2)}
            if hot_order is not None:
                # the hottest 10 % of the records in HBM, read from the file
                # once: the disk serves only the other nodes' records
                t = time.time()
                fix.set_record_cache(hot_order[:n // 10])
                transports["file"]["hot_cache_10pct"] = {"fill_s": round(time.time() - t, 2),
                                                         **compare(fix, qsub, 1, 2)}
                fix.set_record_cache([])
            if not args.no_serving:
                transports["file"]["serving"] = serving_burst(fa, fix, queries, kth, op[1])
            fix.close()
            log("file tier: %s" % transports["file"])
        finally:
            import shutil

            shutil.rmtree(tmpd, ignore_errors=True)

    # ---- serving: continuous batching under open-loop Poisson arrivals, at
    # the relaxed operating L and above
    serving = None
    if not args.no_serving and tier == fa.TIER_HOST:
        serving = serving_leg(fa, ix, queries, kth, args.serving_budget_mb << 20, op[1])
        log("serving: %s" % json.dumps(serving))

    # ---- CPU baseline: the oracle on this host's cores, bounded sample
    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        m = min(args.cpu_sample, nq)
        thr = os.cpu_count() or 1
        passes = 0
        t = time.time()
        while True:
            oracle.search(base, adj, entry, queries[:m], k, op[1], delay=1, threads=thr)
            passes += 1
            if time.time() - t >= args.cpu_seconds or passes >= 100:
                break
        el = time.time() - t
        cpu = {"value": round(passes * m / el, 1), "unit": "queries/s", "cores": thr,
               "kind": "oracle", "cpu": host_cpu(),
               "sample": "%d passes over the first %d of the %d queries (%.1f s), L=%d, "
                         "delay 1, records in DRAM" % (passes, m, nq, el, op[1])}
        log("oracle: %d x %d queries in %.1fs on %d threads" % (passes, m, el, thr))

    if args.copy_calibration:
        a = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log("copy calibration: 268435456 B device-to-device")

    line = {
        "metric": "QPS at recall@10>=0.95 (relaxed vs strict, 1 GPU); p50/p99 query latency",
        "value": round(qps[1], 1),
        "unit": "queries/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms[1], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8", "data": "synthetic",
        "config": {"workload": workload, "n": n, "d": cfg.d, "R": cfg.R, "slot_bytes": cfg.slot,
                   "tier": args.tier, "queries": nq, "k": k, "L_relaxed": op[1],
                   "L_strict": op[0], "graph_build_s": round(t_graph, 1)},
        "strict": {"qps": round(qps[0], 1), "ms_per_step": round(ms[0], 4), "L": op[0],
                   "qps_at_relaxed_L": round(nq / (ms_equal_L / 1e3), 1)},
        "relaxed_vs_strict": round(qps[1] / qps[0], 4),
        "latency_ms": {name: {"p50": round(detail[d]["query_latency_ms_p50"], 4),
                              "p99": round(detail[d]["query_latency_ms_p99"], 4)}
                       for name, d in (("relaxed", 1), ("strict", 0))},
        "detail": {"strict": detail[0], "relaxed": detail[1]},
        "sweep": {"strict": sweep[0], "relaxed": sweep[1]},
        "roofline": roofline,
        "concurrency": concurrency,
        "schedules": schedules,
        "batched": batched,
        "batched_file": batched_file,
        "f32_file": f32_file,
        "serving_file": serving_file,
        "records_in_hbm": hbm_tier,
        "hot_record_cache": hot_cache,
        "pq_navigation": pq,
        "transports": transports,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    ix.close()


if __name__ == "__main__":
    main()
