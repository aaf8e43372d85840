"""Computation/I-O balanced graph-degree selection (paper section 4.3, Eq. 6).

For each candidate degree R, a sample index of random links over synthetic
vectors of the target dtype and dimension is searched with the strict
schedule under the production concurrency, and the kernel's own phase stamps
give the per-expansion record-fetch time T_f(R) and compute time T_c(R)
(medians of interleaved repeats).  The selected degree is
argmin_R |T_c(R) - T_f(R)|: with the two stages equal, a one-step-stale
pipeline overlaps them fully (section 4.1.4).  The choice is made on straight
models of T_f(R) and T_c(R) (a line for T_c; a constant for T_f when its
variation over the sweep is within its repeat noise, else a line), so that
noise in the dominant stage cannot decide it; the argmin over the raw medians
is reported beside it.

Optionally each R is validated on a real graph: QPS of the relaxed search at
the smallest L with recall@10 >= 0.95.

    python -m paper_2507_10070_amd.degree_selector --tier host --dtype f32 --d 96 \\
        --R 32 48 64 96 --slot 4096
"""
from __future__ import annotations

import argparse
import json
import os
import shutil
import sys
import tempfile
import time

import numpy as np


def _index(fa, base, adj, entry, slot, tier, tmp):
    if tier == "file":
        d = tempfile.mkdtemp(prefix="degsel_", dir=tmp)
        fa.save_index(d, base, adj, entry, slot)
        return fa.Index.load(d, fa.TIER_FILE), d
    t = {"host": fa.TIER_HOST, "hbm": fa.TIER_HBM}[tier]
    return fa.Index(base, adj, entry, slot, t), None


def profile_degrees(R_values, n=100_000, d=96, dtype="f32", components=1024, slot=4096,
                    tier="host", nq=10_000, L=64, seed=7, tmp=None, reps=3):
    """T_f and T_c per expansion (microseconds) for each R on random-link
    sample indices: `reps` measurements per R, taken round-robin over the R
    values so that drift of the device hits all of them alike; medians are
    reported.  Returns a list of dicts."""
    import torch

    import synth
    import paper_2507_10070_amd as fa

    tmp = tmp or os.environ.get("TMPDIR", "/tmp")
    base = synth.make_base(n, d, dtype, components, seed)
    q = synth.make_queries(nq, d, dtype, components, seed, seed + 1)
    qd = torch.from_numpy(q).to("cuda:0")
    khz = fa.device_clock_khz()
    idx = {}
    samples = {R: [] for R in R_values}
    try:
        for R in R_values:
            adj = synth.random_graph(n, R, seed + 1000 * R)
            idx[R] = _index(fa, base, adj, 0, slot, tier, tmp)
            fa.search(idx[R][0], qd, k=10, L=L, delay=0)  # warm-up
        for _ in range(reps):
            for R in R_values:
                ix = idx[R][0]
                phases = torch.zeros((nq, 2), dtype=torch.int64, device="cuda:0")
                t = time.perf_counter()
                _, _, steps = fa.search(ix, qd, k=10, L=L, delay=0, phases=phases)
                torch.cuda.synchronize()
                el = time.perf_counter() - t
                ph = phases.cpu().numpy().sum(0).astype(np.float64)
                nsteps = float(steps.cpu().numpy().view(np.uint32).astype(np.int64).sum())
                samples[R].append((ph[0] / nsteps / khz * 1e3, ph[1] / nsteps / khz * 1e3,
                                   int(nsteps), el))
        rows = []
        for R in R_values:
            tf = float(np.median([x[0] for x in samples[R]]))
            tc = float(np.median([x[1] for x in samples[R]]))
            rows.append({"R": R, "T_f_us": round(tf, 3), "T_c_us": round(tc, 3),
                         "io_to_compute": round(tf / tc, 3),
                         "T_f_spread_us": round(float(np.ptp([x[0] for x in samples[R]])), 3),
                         "expansions": samples[R][0][2],
                         "batch_s": round(float(np.median([x[3] for x in samples[R]])), 3),
                         "record_bytes": idx[R][0].info()["rec_bytes"]})
        return rows
    finally:
        for ix, path in idx.values():
            ix.close()
            if path:
                shutil.rmtree(path, ignore_errors=True)


def select(rows):
    """Eq. 6 on the measured medians: the degree whose compute and fetch
    times are closest."""
    return min(rows, key=lambda r: abs(r["T_c_us"] - r["T_f_us"]))["R"]


def select_fitted(rows):
    """Eq. 6 on fitted stage times, so that run-to-run noise cannot decide
    the choice (when reads dominate, their spread can exceed the whole range
    of the compute time over the sweep).  T_c(R) is a least-squares line.
    T_f(R) is a constant (its mean) when its variation across the sweep is
    within twice the spread of its own repeats -- record reads of a fixed
    slot do not depend on R -- and a least-squares line otherwise.
    Returns (R*, model)."""
    R = np.array([r["R"] for r in rows], np.float64)
    tf = np.array([r["T_f_us"] for r in rows])
    tc = np.array([r["T_c_us"] for r in rows])
    if len(R) < 2:
        return int(R[0]), None
    noise = max(float(r.get("T_f_spread_us", 0.0)) for r in rows)
    flat = float(np.ptp(tf)) <= 2.0 * noise
    bf = np.array([0.0, float(np.mean(tf))]) if flat else np.polyfit(R, tf, 1)
    bc = np.polyfit(R, tc, 1)
    gap = np.abs(np.polyval(bc, R) - np.polyval(bf, R))
    model = {"T_f_us": [round(float(x), 5) for x in bf], "T_f_constant": flat,
             "T_c_us": [round(float(x), 5) for x in bc]}
    return int(R[int(np.argmin(gap))]), model


def validate(R_values, n, d, dtype, components, slot, tier, nq, seed=11,
             L_sweep=(10, 12, 16, 20, 24, 32, 48, 64, 96, 128, 192, 256), tmp=None):
    """QPS at recall@10 >= 0.95 (relaxed) on real graphs of each degree."""
    import torch

    import synth
    import paper_2507_10070_amd as fa

    tmp = tmp or os.environ.get("TMPDIR", "/tmp")
    base = synth.make_base(n, d, dtype, components, seed)
    q = synth.make_queries(nq, d, dtype, components, seed, seed + 1)
    qd = torch.from_numpy(q).to("cuda:0")
    from .recall import exact_kth

    kth = exact_kth(base, q, 10, "cuda:0")
    out = []
    for R in R_values:
        t = time.time()
        adj, entry = synth.build_graph(base, R, seed + R, threads=min(16, os.cpu_count() or 1))
        tb = time.time() - t
        ix, path = _index(fa, base, adj, entry, slot, tier, tmp)
        try:
            best = None
            for L in L_sweep:
                _, dist, _ = fa.search(ix, qd, k=10, L=L, delay=1)
                torch.cuda.synchronize()
                dv = dist.cpu().numpy()
                dv = dv.astype(np.float64) if dv.dtype == np.float32 else \
                    dv.view(np.uint32).astype(np.float64)
                rec = float(np.minimum((dv <= kth[:, None] * (1 + 1e-6)).sum(1), 10).mean() / 10)
                if rec >= 0.95:
                    t = time.perf_counter()
                    for _ in range(3):
                        fa.search(ix, qd, k=10, L=L, delay=1)
                    torch.cuda.synchronize()
                    qps = 3 * nq / (time.perf_counter() - t)
                    best = {"R": R, "L": L, "recall@10": round(rec, 4), "qps": round(qps, 1),
                            "graph_build_s": round(tb, 1)}
                    break
            out.append(best or {"R": R, "L": None, "qps": 0.0, "graph_build_s": round(tb, 1)})
        finally:
            ix.close()
            if path:
                shutil.rmtree(path, ignore_errors=True)
        print("validate", out[-1], file=sys.stderr, flush=True)
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description="graph-degree selector (FlashANNS section 4.3)")
    ap.add_argument("--R", type=int, nargs="+", default=[32, 48, 64, 96])
    ap.add_argument("--n", type=int, default=100_000, help="sample index size")
    ap.add_argument("--d", type=int, default=96)
    ap.add_argument("--dtype", default="f32", choices=("u8", "i8", "f32"))
    ap.add_argument("--components", type=int, default=1024)
    ap.add_argument("--slot", type=int, default=4096)
    ap.add_argument("--tier", default="host", choices=("host", "file", "hbm"))
    ap.add_argument("--nq", type=int, default=10_000)
    ap.add_argument("--L", type=int, default=64)
    ap.add_argument("--reps", type=int, default=3, help="measurements per degree (median)")
    ap.add_argument("--validate-n", type=int, default=0,
                    help="also build real graphs of this size and measure QPS at recall>=0.95")
    ap.add_argument("--validate-nq", type=int, default=10_000)
    args = ap.parse_args(argv)
    rows = profile_degrees(args.R, args.n, args.d, args.dtype, args.components, args.slot,
                           args.tier, args.nq, args.L, reps=args.reps)
    for r in rows:
        print("profile", r, file=sys.stderr, flush=True)
    fitted, fit = select_fitted(rows)
    res = {"tier": args.tier, "dtype": args.dtype, "d": args.d, "slot": args.slot,
           "sample_n": args.n, "queries": args.nq, "L": args.L, "reps": args.reps,
           "profile": rows, "selected_R": fitted, "selected_R_raw": select(rows), "fit": fit}
    if args.validate_n:
        res["validation"] = validate(args.R, args.validate_n, args.d, args.dtype,
                                     args.components, args.slot, args.tier, args.validate_nq)
    print(json.dumps(res), flush=True)
    return res


if __name__ == "__main__":
    main()
