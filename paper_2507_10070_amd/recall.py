"""Recall measurement: exact k-th neighbour distances by a full scan.

Harness code for the benchmark and the degree selector's validation, not
part of the search.  The scan runs on the GPU as a plain fp32 GEMM expansion
|q|^2 + |x|^2 - 2 q.x, which is exact for u8/i8 data (every partial sum is an
integer below 2^24) and within fp32 rounding for unit f32 vectors.

The distance block of one chunk of queries is kept below 2^31 elements:
library top-k kernels index a block with 32-bit integers, and a larger block
(1,000 queries against 10M vectors is 10^10 elements) silently gave wrong
k-th distances.  A few sampled queries are recomputed exactly on the CPU
(numpy, integer arithmetic for u8/i8, float64 for f32) and must agree.
"""
from __future__ import annotations

import numpy as np

MAX_BLOCK = (1 << 31) - 1


def _cpu_kth(base: np.ndarray, q: np.ndarray, k: int, rows: int = 1 << 20) -> float:
    """k-th smallest squared distance of q to the rows of base (exact)."""
    parts = []
    if base.dtype == np.float32:
        qq = q.astype(np.float64)
        for s in range(0, base.shape[0], rows):
            diff = base[s:s + rows].astype(np.float64) - qq
            parts.append(np.einsum("ij,ij->i", diff, diff))
    else:
        qq = q.astype(np.int32)
        for s in range(0, base.shape[0], rows):
            diff = base[s:s + rows].astype(np.int32) - qq
            parts.append(np.einsum("ij,ij->i", diff, diff, dtype=np.int64))
    d = np.concatenate(parts)
    return float(np.partition(d, k - 1)[k - 1])


def exact_kth(base: np.ndarray, queries: np.ndarray, k: int, dev, check: int = 3,
              seed: int = 0) -> np.ndarray:
    """k-th nearest squared distance of every query (float64 array)."""
    import torch

    torch.backends.cuda.matmul.allow_tf32 = False
    n = base.shape[0]
    x = torch.from_numpy(np.ascontiguousarray(base)).to(dev).float()
    xx = (x * x).sum(1)
    chunk = max(1, min(1000, MAX_BLOCK // max(1, n)))
    out = []
    for s in range(0, queries.shape[0], chunk):
        q = torch.from_numpy(np.ascontiguousarray(queries[s:s + chunk])).to(dev).float()
        d = (q * q).sum(1, keepdim=True) + xx[None, :] - 2.0 * (q @ x.T)
        out.append(torch.topk(d, k, dim=1, largest=False).values[:, k - 1].cpu())
        del d
    del x, xx
    torch.cuda.empty_cache()
    kth = torch.cat(out).numpy().astype(np.float64)
    if check and queries.shape[0]:
        rows = np.random.default_rng(seed).choice(queries.shape[0],
                                                  min(check, queries.shape[0]), replace=False)
        for r in rows:
            want = _cpu_kth(base, queries[r], k)
            if base.dtype == np.float32:
                ok = abs(kth[r] - want) <= 1e-5 * max(want, 1e-30) + 1e-6
            else:
                ok = kth[r] == want
            if not ok:
                raise RuntimeError("ground truth of query %d: GPU scan %r, CPU %r" % (r, kth[r], want))
    return kth


def recall_at(dists, kth, k: int = 10, rel: float = 0.0) -> float:
    """Tie-aware recall@k: a returned distance counts as a hit when it is at
    most the exact k-th distance (times 1 + rel, for fp32 rounding); hits per
    query are capped at k."""
    d = np.asarray(dists, dtype=np.float64)[:, :k]
    hits = np.minimum((d <= kth[:, None] * (1.0 + rel)).sum(1), k)
    return float(hits.mean() / k)
