"""Autotuner for search launches.

Two kinds of parameters are tuned on a representative batch:

* tiles that do not change results -- threads per query (a whole wave64,
  or half a wave with two queries per wave), waves per workgroup,
  visited-hash size, persistent or one-shot grid, with compressed navigation
  the way PQ distances are formed (`pq_scoring`: LDS table or centroids from
  the cache),
  and for uneven batches (per-query L) the processing order: as given, or
  longest list first (`longest_first`);
* schedule parameters that change the search path but keep it valid -- the
  staleness delay (prefetch depth, paper section 4.1.2) and the beam width W.
  These can move recall a little either way, so a setting is admissible only
  if its quality score (e.g. recall@10) is at least the default setting's
  minus `score_slack`.

The search is coordinate descent from the default setting (each parameter in
turn over its values, others fixed, `passes` times), which needs a few dozen
launches instead of the full product.  The fastest admissible setting is cached
per (dtype, d, R, tier, L bucket, nq bucket, uneven) in a JSON file.

    best = autotune.tune(index, queries, k=10, L=192)
    fa.search(index, queries, k=10, L=192, **autotune.search_kwargs(best["params"], {}))
"""
from __future__ import annotations

import json
import os

SPACE = {
    "delay": (0, 1, 2, 3),
    "beam_width": (1, 2, 4),
    "waves_per_block": (1, 2, 4),
    "hash_bits": (8, 9, 10, 11, 12),
    "persistent": (False, True),
    "query_lanes": (64, 32),
}
DEFAULT = {"delay": 1, "beam_width": 1, "waves_per_block": 4, "hash_bits": 10,
           "persistent": False, "query_lanes": 64}
SEMANTIC = ("delay", "beam_width")
MAX_IN_FLIGHT = 8   # (delay + 1) * beam_width limit of the kernels

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "flashann", "autotune.json")


def _bucket(x: int) -> int:
    b = 1
    while b < x:
        b *= 2
    return b


def cache_key(index, L: int, nq: int, uneven: bool = False, pq: bool = False) -> str:
    info = index.info()
    return "dt%d-d%d-R%d-tier%d-L%d-nq%d%s%s" % (
        info["dtype"], info["d"], info["R"], info["tier"], _bucket(L), _bucket(nq),
        "-uneven" if uneven else "", "-pq%d" % info["pq_m"] if pq else "")


def valid(params) -> bool:
    delay, beam = params.get("delay", 1), params.get("beam_width", 1)
    if params.get("query_lanes", 64) == 32 and (delay > 1 or beam != 1):
        return False  # two queries per wave: strict or one-step-stale, beam 1
    return (delay + 1) * beam <= MAX_IN_FLIGHT


def search_kwargs(params, extra):
    """fa.search keyword arguments of a tuned setting: `longest_first` turns
    into a processing order sorted by decreasing per-query L."""
    import torch

    p = dict(params)
    kw = dict(extra)
    if p.pop("longest_first", False) and kw.get("L_per_query") is not None:
        kw["order"] = torch.argsort(kw["L_per_query"], descending=True, stable=True).to(torch.int32)
    kw.update(p)
    return kw


def measure(index, queries, k, L, params, reps=3, score=None, **extra):
    """Mean milliseconds per launch over `reps` launches (HIP events on the
    launch stream) and, if `score` is given, score(ids, dists, steps) of the
    warm-up launch."""
    import torch

    import paper_2507_10070_amd as fa

    kw = search_kwargs(params, extra)
    params, extra = {}, kw
    st = torch.cuda.current_stream(queries.device)
    out = fa.search(index, queries, k=k, L=L, stream=st, **params, **extra)  # warm-up
    q = score(*out) if score is not None else None
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        fa.search(index, queries, k=k, L=L, stream=st, **params, **extra)
    e1.record(st)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps, q


def tune(index, queries, k, L, space=None, reps=3, cache_path=DEFAULT_CACHE, use_cache=True,
         score=None, score_slack=0.001, passes=2, start=None, progress=None, **extra):
    """Coordinate descent over `space` from `start` (default DEFAULT).
    Returns {"params", "ms", "score", "key", "table"}; `table` lists every
    setting tried with its time and score (None where the launch failed,
    e.g. a tile whose LDS need exceeds the CU).  `progress`, if given, is
    called with each new table row."""
    uneven = extra.get("L_per_query") is not None or extra.get("k_per_query") is not None
    key = cache_key(index, L, queries.shape[0], uneven, extra.get("navigation", 0) == 1)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            with open(cache_path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        return cache[key]
    space = dict(space or SPACE)
    if uneven and extra.get("order") is None:
        space.setdefault("longest_first", (False, True))
    if extra.get("navigation", 0) == 1 and extra.get("pq_scoring") is None:
        space.setdefault("pq_scoring", (2, 1))  # cache, table
    # two queries per wave: direct transport (not a file tier), full navigation
    if extra.get("navigation", 0) == 1 or extra.get("transport", 0) == 2 or \
            index.info()["tier"] == 2:
        space.pop("query_lanes", None)
    cur = dict(start or DEFAULT)
    cur = {n: cur.get(n, DEFAULT.get(n, space[n][0])) for n in space}
    if score is None:  # no quality measure: results-neutral parameters only
        for n in SEMANTIC:
            if n in space:
                space[n] = (cur[n],)
    seen = {}

    def run(p):
        t = tuple(sorted(p.items()))
        if t not in seen:
            try:
                ms, q = measure(index, queries, k, L, p, reps=reps, score=score, **extra)
                seen[t] = {"params": dict(p), "ms": round(ms, 4), "score": q}
            except Exception as e:  # noqa: BLE001 -- recorded, setting skipped
                seen[t] = {"params": dict(p), "ms": None, "score": None, "error": str(e)}
            if progress is not None:
                progress(seen[t])
        return seen[t]

    base = run(cur)
    if base["ms"] is None:
        raise RuntimeError("the starting setting failed: %s" % base.get("error"))
    floor = None if score is None else base["score"] - score_slack

    def admissible(r):
        return r["ms"] is not None and (floor is None or r["score"] >= floor)

    best = base
    for _ in range(passes):
        changed = False
        for name in sorted(space):
            for v in space[name]:
                p = dict(best["params"])
                p[name] = v
                if not valid(p):
                    continue
                r = run(p)
                if admissible(r) and r["ms"] < best["ms"]:
                    best, changed = r, True
        if not changed:
            break
    res = {"params": best["params"], "ms": best["ms"], "score": best["score"], "key": key,
           "default": {"params": base["params"], "ms": base["ms"], "score": base["score"]},
           "table": list(seen.values())}
    if cache_path:
        cache[key] = res
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        tmp = cache_path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(cache, f)
        os.replace(tmp, cache_path)
    return res
