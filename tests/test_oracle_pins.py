"""Pins of the CPU oracle against things other than itself.

* a hand-derived worked example (tests/golden/worked_example.json);
* a second hand-derived example for beam width W > 1 and staleness 2
  (tests/golden/beam_schedule_example.json), built so that the drain rule and
  the delay*W processing threshold change the selection order;
* exhaustive search: with L >= N on a connected graph every reachable node is
  expanded, so the result must be the exact top-k of a full scan computed
  with numpy's lexsort (paper section 4.1.1 search + the definition of k-NN);
* a textbook heap formulation of strict best-first search (candidate
  min-heap plus a bounded result set), written independently below;
* library distances (scipy) for every dtype;
* tie-breaking fixtures and argument validation.
"""
import heapq
import json
import os

import numpy as np
import pytest
from scipy.spatial.distance import cdist

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_example.json")
BEAM_GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "beam_schedule_example.json")


def _example():
    with open(GOLDEN) as f:
        g = json.load(f)
    x = np.array(g["points_1d_u8"], dtype=np.uint8).reshape(-1, 1)
    adj = np.array(g["adjacency"], dtype=np.int32)
    q = np.array([[g["query_1d_u8"]]], dtype=np.uint8)
    return g, x, adj, q


@pytest.mark.parametrize("case", range(3))
def test_worked_example(case):
    g, x, adj, q = _example()
    c = g["cases"][case]
    r = oracle.search(x, adj, g["entry"], q, g["k"], c["L"], delay=c["delay"], trace_cap=16)
    assert r["ids"][0].tolist() == c["ids"]
    assert r["dists"][0].tolist() == c["dists"]
    assert int(r["steps"][0]) == c["steps"]
    tr = r["trace"][0]
    assert tr[tr >= 0].tolist() == c["trace"]
    if c["theta"] is not None:
        th = r["theta"][0]
        assert th[~np.isnan(th)].tolist() == c["theta"]


@pytest.mark.parametrize("case", range(5))
def test_beam_schedule_example(case):
    """(delay, W) in {(0,1), (1,1), (0,2), (1,2), (2,1)}: traces, step counts,
    L-th key after each processed node (null = fewer than L candidates) and
    answers derived by hand from the schedule of paper section 4.1.2 with the
    beam-width reading R6."""
    with open(BEAM_GOLDEN) as f:
        g = json.load(f)
    x = np.array(g["points_1d_u8"], dtype=np.uint8).reshape(-1, 1)
    adj = np.array(g["adjacency"], dtype=np.int32)
    q = np.array([[g["query_1d_u8"]]], dtype=np.uint8)
    c = g["cases"][case]
    r = oracle.search(x, adj, g["entry"], q, g["k"], g["L"], delay=c["delay"], beam=c["beam"],
                      trace_cap=32)
    assert r["ids"][0].tolist() == c["ids"]
    assert r["dists"][0].tolist() == c["dists"]
    assert int(r["steps"][0]) == c["steps"]
    tr = r["trace"][0]
    assert tr[tr >= 0].tolist() == c["trace"]
    th = r["theta"][0]
    want = [np.inf if t is None else float(t) for t in c["theta"]]
    assert th[~np.isnan(th)].tolist() == want


def _rand(dtype, n, d, rng):
    if dtype == np.uint8:
        return rng.integers(0, 256, size=(n, d)).astype(np.uint8)
    if dtype == np.int8:
        return rng.integers(-128, 128, size=(n, d)).astype(np.int8)
    return rng.standard_normal(size=(n, d)).astype(np.float32)


def _ring_graph(n, R, rng):
    """Connected graph: a ring plus random edges (ids may include -1 padding)."""
    adj = np.full((n, R), -1, dtype=np.int32)
    for i in range(n):
        adj[i, 0] = (i + 1) % n
        others = rng.permutation(n)
        others = others[others != i][: R - 1]
        adj[i, 1:1 + len(others)] = others
    return adj


@pytest.mark.parametrize("dtype", [np.uint8, np.int8, np.float32])
def test_distances_match_scipy(dtype):
    rng = np.random.default_rng(7)
    x = _rand(dtype, 50, 37, rng)
    q = _rand(dtype, 1, 37, rng)
    got = oracle.distances(x, q[0])
    ref = cdist(q.astype(np.float64), x.astype(np.float64), "sqeuclidean")[0]
    if dtype == np.float32:
        np.testing.assert_allclose(got, ref, rtol=1e-13)
    else:
        np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("dtype", [np.uint8, np.int8, np.float32])
def test_bruteforce_matches_lexsort(dtype):
    rng = np.random.default_rng(11)
    x = _rand(dtype, 300, 16, rng)
    q = _rand(dtype, 9, 16, rng)
    ids, dists = oracle.bruteforce(x, q, 12, threads=3)
    ref = cdist(q.astype(np.float64), x.astype(np.float64), "sqeuclidean")
    for i in range(len(q)):
        order = np.lexsort((np.arange(len(x)), ref[i]))[:12]
        assert ids[i].tolist() == order.tolist()
        np.testing.assert_allclose(dists[i], ref[i][order], rtol=1e-12)


@pytest.mark.parametrize("dtype", [np.uint8, np.int8, np.float32])
@pytest.mark.parametrize("delay", [0, 1, 2])
@pytest.mark.parametrize("beam", [1, 3])
def test_exhaustive_when_L_covers_graph(dtype, delay, beam):
    """L >= N on a connected graph: every node is expanded exactly once and
    the output is the exact top-k (section 4.1.1 search over the whole graph)."""
    rng = np.random.default_rng(100 + delay + 10 * beam)
    n = 120
    x = _rand(dtype, n, 8, rng)
    q = _rand(dtype, 6, 8, rng)
    adj = _ring_graph(n, 5, rng)
    r = oracle.search(x, adj, 17, q, k=10, L=n, delay=delay, beam=beam, trace_cap=n + 5)
    ref = cdist(q.astype(np.float64), x.astype(np.float64), "sqeuclidean")
    for i in range(len(q)):
        order = np.lexsort((np.arange(n), ref[i]))[:10]
        assert r["ids"][i].tolist() == order.tolist()
        assert int(r["steps"][i]) == n
        tr = r["trace"][i]
        assert sorted(tr[tr >= 0].tolist()) == list(range(n))


def _heap_search(x, adj, entry, q, k, L, R):
    """Textbook strict best-first search: a min-heap of candidates and a
    bounded max-heap of the L best nodes seen; stop when the closest
    candidate is worse than the worst kept node."""
    def key(i):
        return (float(((x[i].astype(np.float64) - q.astype(np.float64)) ** 2).sum()), int(i))

    visited = {entry}
    cand = [key(entry)]
    best = [(-key(entry)[0], -entry)]  # max-heap via negation
    trace = []
    while cand:
        c = heapq.heappop(cand)
        worst = (-best[0][0], -best[0][1])
        if c > worst:
            break
        trace.append(c[1])
        for nb in adj[c[1]][:R]:
            nb = int(nb)
            if nb < 0 or nb >= len(x) or nb in visited:
                continue
            visited.add(nb)
            kn = key(nb)
            worst = (-best[0][0], -best[0][1])
            if len(best) < L or kn < worst:
                heapq.heappush(cand, kn)
                heapq.heappush(best, (-kn[0], -kn[1]))
                if len(best) > L:
                    heapq.heappop(best)
    res = sorted((-a, -b) for a, b in best)[:k]
    return [b for _, b in res], [a for a, _ in res], trace


@pytest.mark.parametrize("dtype", [np.uint8, np.int8, np.float32])
@pytest.mark.parametrize("L,R", [(4, 6), (10, 6), (25, 3)])
def test_strict_equals_heap_formulation(dtype, L, R):
    rng = np.random.default_rng(L * 31 + R)
    n = 400
    x = _rand(dtype, n, 12, rng)
    qs = _rand(dtype, 8, 12, rng)
    adj = _ring_graph(n, 6, rng)
    r = oracle.search(x, adj, 3, qs, k=min(4, L), L=L, R=R, delay=0, trace_cap=n)
    for i in range(len(qs)):
        ids, dists, trace = _heap_search(x, adj, 3, qs[i], min(4, L), L, R)
        assert r["ids"][i].tolist() == ids
        np.testing.assert_allclose(r["dists"][i], dists, rtol=1e-12)
        tr = r["trace"][i]
        assert tr[tr >= 0].tolist() == trace
        assert int(r["steps"][i]) == len(trace)


def test_tie_break_smaller_id_first():
    # query 50; ids 1 and 4 at 40 and 60 (both distance 100), id 2 at 50
    x = np.array([[0], [40], [50], [90], [60]], dtype=np.uint8)
    q = np.array([[50]], dtype=np.uint8)
    ids, d = oracle.bruteforce(x, q, 3)
    assert ids[0].tolist() == [2, 1, 4]
    adj = np.array([[4, 1], [0, 2], [1, 3], [2, 4], [3, 0]], dtype=np.int32)
    for delay in (0, 1):
        r = oracle.search(x, adj, 3, q, k=3, L=3, delay=delay)
        assert r["ids"][0].tolist() == [2, 1, 4]
        assert r["dists"][0].tolist() == [0, 100, 100]


def test_padding_and_short_results():
    x = np.array([[1], [2], [3]], dtype=np.uint8)
    adj = np.array([[1, -1], [-1, 0], [0, 1]], dtype=np.int32)  # node 2 unreachable
    r = oracle.search(x, adj, 0, np.array([[0]], np.uint8), k=4, L=4, delay=1)
    assert r["ids"][0].tolist() == [0, 1, -1, -1]
    assert np.isinf(r["dists"][0][2:]).all()
    assert int(r["steps"][0]) == 2


@pytest.mark.parametrize("kw", [dict(k=5, L=4), dict(k=0, L=4), dict(k=1, L=4, R=3),
                                dict(k=1, L=4, delay=-1), dict(k=1, L=4, beam=0)])
def test_validation(kw):
    x = np.zeros((4, 2), np.uint8)
    adj = np.zeros((4, 2), np.int32)
    with pytest.raises(ValueError):
        oracle.search(x, adj, 0, x[:1], **kw)
