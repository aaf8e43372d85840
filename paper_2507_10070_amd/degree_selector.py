"""Computation/I-O balanced graph-degree selection (paper section 4.3, Eq. 6).

For each candidate degree R, a sample index of random links over synthetic
vectors of the target dtype and dimension is searched with the strict
schedule under the production concurrency, and the kernel's own phase stamps
give the per-expansion record-fetch time T_f(R) and compute time T_c(R).  The
selected degree is argmin_R |T_c(R) - T_f(R)|: with the two stages equal, a
one-step-stale pipeline overlaps them fully (section 4.1.4).

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
                    tier="host", nq=10_000, L=64, seed=7, tmp=None):
    """T_f and T_c per expansion (microseconds) for each R on random-link
    sample indices.  Returns a list of dicts."""
    import torch

    import synth
    import paper_2507_10070_amd as fa

    tmp = tmp or os.environ.get("TMPDIR", "/tmp")
    base = synth.make_base(n, d, dtype, components, seed)
    q = synth.make_queries(nq, d, dtype, components, seed, seed + 1)
    qd = torch.from_numpy(q).to("cuda:0")
    khz = fa.device_clock_khz()
    rows = []
    for R in R_values:
        adj = synth.random_graph(n, R, seed + 1000 * R)
        ix, path = _index(fa, base, adj, 0, slot, tier, tmp)
        try:
            fa.search(ix, qd, k=10, L=L, delay=0)  # warm-up
            phases = torch.zeros((nq, 2), dtype=torch.int64, device="cuda:0")
            t = time.perf_counter()
            _, _, steps = fa.search(ix, qd, k=10, L=L, delay=0, phases=phases)
            torch.cuda.synchronize()
            el = time.perf_counter() - t
            ph = phases.cpu().numpy().sum(0).astype(np.float64)
            nsteps = float(steps.cpu().numpy().view(np.uint32).astype(np.int64).sum())
            tf = ph[0] / nsteps / khz * 1e3
            tc = ph[1] / nsteps / khz * 1e3
            rows.append({"R": R, "T_f_us": round(tf, 3), "T_c_us": round(tc, 3),
                         "io_to_compute": round(tf / tc, 3), "expansions": int(nsteps),
                         "batch_s": round(el, 3),
                         "record_bytes": ix.info()["rec_bytes"]})
        finally:
            ix.close()
            if path:
                shutil.rmtree(path, ignore_errors=True)
    return rows


def select(rows):
    """Eq. 6: the degree whose compute and fetch times are closest."""
    return min(rows, key=lambda r: abs(r["T_c_us"] - r["T_f_us"]))["R"]


def validate(R_values, n, d, dtype, components, slot, tier, nq, seed=11,
             L_sweep=(32, 48, 64, 96, 128, 192, 256), tmp=None):
    """QPS at recall@10 >= 0.95 (relaxed) on real graphs of each degree."""
    import torch

    import synth
    import paper_2507_10070_amd as fa

    tmp = tmp or os.environ.get("TMPDIR", "/tmp")
    base = synth.make_base(n, d, dtype, components, seed)
    q = synth.make_queries(nq, d, dtype, components, seed, seed + 1)
    qd = torch.from_numpy(q).to("cuda:0")
    torch.backends.cuda.matmul.allow_tf32 = False
    x = torch.from_numpy(base).to("cuda:0").float()
    xx = (x * x).sum(1)
    kth = []
    for s in range(0, nq, 1000):
        qq = qd[s:s + 1000].float()
        dd = (qq * qq).sum(1, keepdim=True) + xx[None] - 2.0 * (qq @ x.T)
        kth.append(torch.topk(dd, 10, dim=1, largest=False).values[:, 9])
    kth = torch.cat(kth).cpu().numpy().astype(np.float64)
    del x, xx
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
    ap.add_argument("--validate-n", type=int, default=0,
                    help="also build real graphs of this size and measure QPS at recall>=0.95")
    ap.add_argument("--validate-nq", type=int, default=10_000)
    args = ap.parse_args(argv)
    rows = profile_degrees(args.R, args.n, args.d, args.dtype, args.components, args.slot,
                           args.tier, args.nq, args.L)
    for r in rows:
        print("profile", r, file=sys.stderr, flush=True)
    res = {"tier": args.tier, "dtype": args.dtype, "d": args.d, "slot": args.slot,
           "sample_n": args.n, "queries": args.nq, "L": args.L, "profile": rows,
           "selected_R": select(rows)}
    if args.validate_n:
        res["validation"] = validate(args.R, args.validate_n, args.d, args.dtype,
                                     args.components, args.slot, args.tier, args.validate_nq)
    print(json.dumps(res), flush=True)
    return res


if __name__ == "__main__":
    main()
