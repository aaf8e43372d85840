"""Product-quantisation codebooks for compressed navigation.

Codebook training is index construction, like the proximity graph: its output
is an input that the search library and the oracle both consume.  Nothing of
the search itself (encoding, distance tables, PQ distances) lives here.

train_codebooks(base, M) -> float32 [M, 256, d / M]: per subspace of d / M
consecutive dimensions, Lloyd's k-means with 256 centroids on a seeded sample
of the rows, initialised from distinct sample rows; a centroid left without
members is moved to the sample row farthest from its own centroid.
"""
from __future__ import annotations

import numpy as np

KSUB = 256


def train_codebooks(base: np.ndarray, M: int, iters: int = 10, sample: int = 20000,
                    seed: int = 0) -> np.ndarray:
    n, d = base.shape
    if M < 1 or d % M:
        raise ValueError("M=%d must divide d=%d" % (M, d))
    dsub = d // M
    rng = np.random.default_rng(seed)
    rows = rng.choice(n, size=min(n, sample), replace=False)
    X = base[np.sort(rows)].astype(np.float64)
    cb = np.empty((M, KSUB, dsub), dtype=np.float32)
    for m in range(M):
        Xm = X[:, m * dsub:(m + 1) * dsub]
        uniq = np.unique(Xm, axis=0)
        pick = rng.permutation(len(uniq))[:KSUB]
        C = uniq[pick]
        if len(C) < KSUB:  # fewer distinct points than centroids: repeat them
            C = C[np.arange(KSUB) % len(C)]
        C = C.astype(np.float64)
        xx = (Xm * Xm).sum(1)
        for _ in range(iters):
            d2 = xx[:, None] - 2.0 * Xm @ C.T + (C * C).sum(1)[None, :]
            a = np.argmin(d2, axis=1)
            cnt = np.bincount(a, minlength=KSUB)
            S = np.stack([np.bincount(a, weights=Xm[:, j], minlength=KSUB)
                          for j in range(dsub)], axis=1)
            live = cnt > 0
            C[live] = S[live] / cnt[live, None]
            if (~live).any() and len(uniq) >= KSUB:
                far = np.argsort(-d2[np.arange(len(a)), a])[: int((~live).sum())]
                C[~live] = Xm[far]
        cb[m] = C.astype(np.float32)
    return cb
