"""Sampled oracle parity of the f32/96 file-tier search at full size (GPU).

Not collected by pytest: the index it checks (tens of GB of records) is the
one `bench.py --f32-only --f32-file-n N --f32-keep DIR` leaves behind, so it
runs right after that leg:

    python tests/fullsize_f32_parity.py DIR [--sample 32] [--L 128]

A seeded sample of the queries is searched on the GPU with records read from
the file by the host agents (strict and relaxed, with traces) and by the
oracle over the same vectors and graph; the fp32 rule of tests/parity.py is
applied to every sampled query.  Prints one JSON summary line.
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from parity import assert_f32_parity  # noqa: E402


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("dir")
    ap.add_argument("--sample", type=int, default=32)
    ap.add_argument("--L", type=int, default=128)
    ap.add_argument("--seed", type=int, default=41)
    args = ap.parse_args(argv)

    import torch

    import paper_2507_10070_amd as fa

    with open(os.path.join(args.dir, "meta.json")) as f:
        meta = json.load(f)
    n, d, entry = meta["n"], meta["d"], meta["entry"]
    assert meta["dtype"] == "f32"
    base = np.fromfile(os.path.join(args.dir, "vectors.bin"), dtype=np.float32).reshape(n, d)
    adj = np.load(os.path.join(args.dir, "adj.npy"))
    queries = np.load(os.path.join(args.dir, "queries.npy"))
    rows = np.sort(np.random.default_rng(args.seed).choice(len(queries), args.sample,
                                                          replace=False))
    q = np.ascontiguousarray(queries[rows])
    out = {"n": n, "R": int(adj.shape[1]), "L": args.L, "sample": int(args.sample),
           "query_rows": rows.tolist()[:8] + (["..."] if len(rows) > 8 else [])}
    with fa.Index.load(args.dir, fa.TIER_FILE) as ix:
        qd = torch.from_numpy(q).to("cuda:0")
        for delay in (0, 1):
            trace = torch.full((len(q), 1200), -1, dtype=torch.int32, device="cuda:0")
            ids, dists, steps = fa.search(ix, qd, k=10, L=args.L, delay=delay, trace=trace)
            torch.cuda.synchronize()
            g = {"ids": ids.cpu().numpy(), "dists": dists.cpu().numpy(),
                 "steps": steps.cpu().numpy().view(np.uint32), "trace": trace.cpu().numpy()}
            t = time.time()
            ref = oracle.search(base, adj, entry, q, 10, args.L, delay=delay, trace_cap=1200)
            t_oracle = time.time() - t
            diverged = assert_f32_parity(base, q, g, ref)
            same_ids = int((g["ids"] == ref["ids"]).all(1).sum())
            out["delay%d" % delay] = {"queries_checked": len(q), "near_tie_divergences": diverged,
                                     "identical_ids": same_ids,
                                     "identical_steps": int((g["steps"] == ref["steps"]).sum()),
                                     "oracle_s": round(t_oracle, 1)}
            print("delay %d: %s" % (delay, out["delay%d" % delay]), flush=True)
    out["result"] = "pass"
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
