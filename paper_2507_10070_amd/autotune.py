"""Autotuner for search launches.

Tiles that do not change results -- queries per workgroup, visited-hash size,
persistent or one-shot grid -- and the prefetch depth (the staleness delay,
which changes the search path but keeps it valid) are measured on a
representative batch; the fastest setting is cached per
(dtype, d, R, tier, L bucket, nq bucket) in a JSON file.

    best = autotune.tune(index, queries, k=10, L=192)
    fa.search(index, queries, k=10, L=192, **best["params"])
"""
from __future__ import annotations

import itertools
import json
import os

SPACE = {
    "delay": (0, 1),
    "waves_per_block": (1, 2, 4),
    "hash_bits": (8, 9, 10, 11, 12),
    "persistent": (False, True),
}

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "flashann", "autotune.json")


def _bucket(x: int) -> int:
    b = 1
    while b < x:
        b *= 2
    return b


def cache_key(index, L: int, nq: int) -> str:
    info = index.info()
    return "dt%d-d%d-R%d-tier%d-L%d-nq%d" % (info["dtype"], info["d"], info["R"], info["tier"],
                                            _bucket(L), _bucket(nq))


def measure(index, queries, k, L, params, reps=3, **extra):
    """Mean milliseconds per launch over `reps` launches (HIP events)."""
    import torch

    import paper_2507_10070_amd as fa

    st = torch.cuda.current_stream(queries.device)
    fa.search(index, queries, k=k, L=L, stream=st, **params, **extra)  # warm-up
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        fa.search(index, queries, k=k, L=L, stream=st, **params, **extra)
    e1.record(st)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(index, queries, k, L, space=None, reps=3, cache_path=DEFAULT_CACHE, use_cache=True,
         **extra):
    """Try every combination of `space`; return {"params", "ms", "table", "key"}."""
    key = cache_key(index, L, queries.shape[0])
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            with open(cache_path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        return cache[key]
    space = space or SPACE
    names = sorted(space)
    table = []
    for combo in itertools.product(*(space[n] for n in names)):
        params = dict(zip(names, combo))
        try:
            ms = measure(index, queries, k, L, params, reps=reps, **extra)
        except Exception as e:  # e.g. a tile whose LDS need exceeds the CU
            table.append({"params": params, "ms": None, "error": str(e)})
            continue
        table.append({"params": params, "ms": round(ms, 4)})
    ok = [r for r in table if r["ms"] is not None]
    best = min(ok, key=lambda r: r["ms"])
    res = {"params": best["params"], "ms": best["ms"], "key": key, "table": table}
    if cache_path:
        cache[key] = res
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        tmp = cache_path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(cache, f)
        os.replace(tmp, cache_path)
    return res
