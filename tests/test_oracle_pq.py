"""Pins of the oracle's compressed (PQ) navigation, CPU only.

What fixes the answer independently of the oracle's own code:
* identity codebooks (one dimension per subspace, one centroid per integer
  value) make the code the vector itself and the PQ distance the exact
  distance, so the PQ search must reproduce the exact search (pinned on its
  own) step for step;
* a distance table entry is the squared distance of a query part to a
  centroid, and the sum over a code is the squared distance to the decoded
  vector (fp64 in numpy, within fp32 rounding);
* a code names the nearest centroid (fp64 within fp32 rounding) and the
  lowest index among equal ones;
* the answer is the first k of the expanded nodes (the trace) by exact
  distance, and with L covering a connected graph it is the exact top-k.
"""
import numpy as np
import pytest

import oracle
import synth


def identity_codebooks(d, dtype):
    cb = np.zeros((d, 256, 1), np.float32)
    cb[:, :, 0] = np.arange(256) - (128 if dtype == np.int8 else 0)
    return cb


@pytest.fixture(scope="module")
def small():
    base = synth.make_base(2000, 16, "u8", 8, 901)
    q = synth.make_queries(12, 16, "u8", 8, 901, 902)
    adj, entry = synth.build_graph(base, 8, 903, threads=4)
    return base, q, adj, entry


@pytest.mark.parametrize("dt", [np.uint8, np.int8])
def test_identity_codebook_codes_are_the_vectors(dt):
    rng = np.random.default_rng(1)
    base = rng.integers(-128 if dt == np.int8 else 0, 128 if dt == np.int8 else 256,
                        (300, 12)).astype(dt)
    codes = oracle.pq_encode(base, identity_codebooks(12, dt))
    want = base.astype(np.int64) + (128 if dt == np.int8 else 0)
    np.testing.assert_array_equal(codes, want.astype(np.uint8))


@pytest.mark.parametrize("dt", ["u8", "i8"])
@pytest.mark.parametrize("delay,beam", [(0, 1), (1, 1), (2, 2)])
def test_identity_codebook_search_equals_exact_search(dt, delay, beam):
    base = synth.make_base(1500, 16, dt, 6, 911)
    q = synth.make_queries(10, 16, dt, 6, 911, 912)
    adj, entry = synth.build_graph(base, 8, 913, threads=4)
    cb = identity_codebooks(16, base.dtype.type)
    ex = oracle.search(base, adj, entry, q, 10, 24, delay=delay, beam=beam, trace_cap=400)
    pq = oracle.search(base, adj, entry, q, 10, 24, delay=delay, beam=beam, trace_cap=400,
                       codebooks=cb)
    for key in ("ids", "dists", "steps", "trace"):
        np.testing.assert_array_equal(pq[key], ex[key])
    np.testing.assert_array_equal(pq["theta"], ex["theta"])


@pytest.mark.parametrize("dt,M", [(np.float32, 4), (np.uint8, 8), (np.int8, 3)])
def test_table_is_squared_distance_to_decoded_vector(dt, M):
    rng = np.random.default_rng(2)
    d = 24
    cb = rng.normal(0, 20, (M, 256, d // M)).astype(np.float32)
    if dt == np.float32:
        qv = rng.normal(0, 20, d).astype(np.float32)
    else:
        qv = rng.integers(-100 if dt == np.int8 else 0, 100 if dt == np.int8 else 200, d).astype(dt)
    tab = oracle.pq_table(qv, cb)
    parts = qv.astype(np.float64).reshape(M, 1, d // M)
    want = ((parts - cb.astype(np.float64)) ** 2).sum(-1)
    np.testing.assert_allclose(tab, want, rtol=2e-6, atol=1e-4)
    codes = rng.integers(0, 256, (50, M))
    got = tab[np.arange(M)[None, :], codes].astype(np.float64).sum(1)
    dec = cb[np.arange(M)[None, :], codes].reshape(50, d).astype(np.float64)
    np.testing.assert_allclose(got, ((dec - qv.astype(np.float64)) ** 2).sum(1), rtol=1e-5)


@pytest.mark.parametrize("dt", [np.uint8, np.float32])
def test_codes_name_the_nearest_centroid(dt):
    rng = np.random.default_rng(3)
    d, M = 16, 4
    base = (rng.integers(0, 256, (400, d)) if dt == np.uint8
            else rng.normal(0, 30, (400, d))).astype(dt)
    cb = rng.normal(120 if dt == np.uint8 else 0, 40, (M, 256, d // M)).astype(np.float32)
    codes = oracle.pq_encode(base, cb)
    parts = base.astype(np.float64).reshape(400, M, 1, d // M)
    d2 = ((parts - cb.astype(np.float64)[None]) ** 2).sum(-1)  # [n, M, 256]
    chosen = np.take_along_axis(d2, codes[..., None].astype(np.int64), 2)[..., 0]
    assert (chosen <= d2.min(-1) * (1 + 1e-5) + 1e-6).all()
    # exact ties go to the lowest index
    cb2 = cb.copy()
    cb2[:, 200] = base[0].reshape(M, d // M)
    cb2[:, 37] = base[0].reshape(M, d // M)
    assert (oracle.pq_encode(base[:1], cb2)[0] == 37).all()


def _check_rerank(base, q, ref, k):
    for i in range(len(q)):
        steps = int(ref["steps"][i])
        expanded = ref["trace"][i][:steps]
        assert (expanded >= 0).all() and len(set(expanded.tolist())) == steps
        full = oracle.distances(base, q[i])
        order = np.lexsort((expanded, full[expanded]))[:k]
        want = expanded[order]
        n_out = min(k, steps)
        np.testing.assert_array_equal(ref["ids"][i][:n_out], want)
        np.testing.assert_array_equal(ref["dists"][i][:n_out], full[want])
        assert (ref["ids"][i][n_out:] == -1).all()


@pytest.mark.parametrize("delay,beam", [(0, 1), (1, 1), (3, 2)])
def test_answer_is_exact_topk_of_expanded(small, delay, beam):
    base, q, adj, entry = small
    cb = synth.train_codebooks(base, 4, iters=4, sample=2000, seed=5)
    ref = oracle.search(base, adj, entry, q, 10, 32, delay=delay, beam=beam, trace_cap=2000,
                        codebooks=cb)
    _check_rerank(base, q, ref, 10)
    # the list is ordered by PQ distance: the L-th entry never grows
    for th in ref["theta"]:
        t = th[~np.isnan(th)]
        t = np.where(np.isinf(t), np.finfo(np.float64).max, t)  # +inf: list not yet full
        assert (np.diff(t) <= 0).all()


def test_degenerate_codebook_still_reranks(small):
    base, q, adj, entry = small
    cb = np.zeros((2, 256, 8), np.float32)  # every code 0, every PQ distance equal
    ref = oracle.search(base, adj, entry, q, 5, 16, delay=1, trace_cap=2000, codebooks=cb)
    _check_rerank(base, q, ref, 5)


def test_L_covering_graph_gives_exact_topk():
    base = synth.make_base(300, 8, "u8", 3, 921)
    q = synth.make_queries(6, 8, "u8", 3, 921, 922)
    adj, entry = synth.build_graph(base, 6, 923, threads=2)
    seen = {entry}
    todo = [entry]
    while todo:
        for x in adj[todo.pop()]:
            if 0 <= x < len(base) and x not in seen:
                seen.add(int(x))
                todo.append(int(x))
    reach = np.array(sorted(seen))
    cb = synth.train_codebooks(base, 2, iters=3, sample=300, seed=6)
    ref = oracle.search(base, adj, entry, q, 7, 512, delay=1, codebooks=cb)
    for i in range(len(q)):
        full = oracle.distances(base, q[i])[reach]
        want = reach[np.lexsort((reach, full))[:7]]
        np.testing.assert_array_equal(ref["ids"][i], want)


def test_invalid_codebooks_rejected(small):
    base, q, adj, entry = small
    with pytest.raises(ValueError):
        oracle.search(base, adj, entry, q, 5, 16, codebooks=np.zeros((3, 256, 5), np.float32))
    with pytest.raises(ValueError):
        oracle.pq_encode(base, np.zeros((4, 128, 4), np.float32))


def _heap_pq_search(x, codes, cb, adj, entry, q, k, L, R):
    """Textbook strict best-first search (min-heap of candidates, bounded
    max-heap of the L best seen) keyed by the squared distance to the decoded
    vector, then the expanded nodes re-ranked by exact distance."""
    import heapq

    M = cb.shape[0]

    def key(i):
        dec = cb[np.arange(M), codes[i]].reshape(-1).astype(np.float64)
        return (float(((dec - q.astype(np.float64)) ** 2).sum()), int(i))

    visited = {entry}
    cand = [key(entry)]
    best = [(-key(entry)[0], -entry)]
    trace = []
    while cand:
        c = heapq.heappop(cand)
        if c > (-best[0][0], -best[0][1]):
            break
        trace.append(c[1])
        for nb in adj[c[1]][:R]:
            nb = int(nb)
            if nb < 0 or nb >= len(x) or nb in visited:
                continue
            visited.add(nb)
            kn = key(nb)
            if len(best) < L or kn < (-best[0][0], -best[0][1]):
                heapq.heappush(cand, kn)
                heapq.heappush(best, (-kn[0], -kn[1]))
                if len(best) > L:
                    heapq.heappop(best)
    exact = ((x[trace].astype(np.float64) - q.astype(np.float64)) ** 2).sum(1)
    order = np.lexsort((np.array(trace), exact))[:k]
    return [trace[i] for i in order], trace


@pytest.mark.parametrize("L,R", [(1, 6), (4, 6), (10, 6), (25, 3)])
def test_strict_pq_equals_heap_formulation(L, R):
    # small integers everywhere: every fp32 table entry and sum is exact, so
    # numpy's fp64 decoded distances take the same decisions
    rng = np.random.default_rng(L * 7 + R)
    n, d, M = 400, 12, 4
    x = rng.integers(0, 16, (n, d)).astype(np.uint8)
    qs = rng.integers(0, 16, (40, d)).astype(np.uint8)
    cb = rng.integers(0, 16, (M, 256, d // M)).astype(np.float32)
    # nearest centroid in exact integer arithmetic, first (lowest) index on ties
    parts = x.astype(np.int64).reshape(n, M, 1, d // M)
    codes = np.argmin(((parts - cb.astype(np.int64)[None]) ** 2).sum(-1), axis=2)
    np.testing.assert_array_equal(oracle.pq_encode(x, cb), codes)
    adj = np.stack([rng.permutation(n)[:6] for _ in range(n)]).astype(np.int32)
    adj[:, 0] = (np.arange(n) + 1) % n  # a ring keeps the graph connected
    k = min(4, L)
    r = oracle.search(x, adj, 3, qs, k=k, L=L, R=R, delay=0, trace_cap=n, codebooks=cb)
    for i in range(len(qs)):
        ids, trace = _heap_pq_search(x, codes, cb, adj, 3, qs[i], k, L, R)
        assert r["trace"][i][: int(r["steps"][i])].tolist() == trace
        assert r["ids"][i].tolist()[: len(ids)] == ids
