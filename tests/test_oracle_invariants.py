"""Invariants of the search that hold on any input (paper sections 4.1.1-4.1.3):
each node is expanded at most once, the L-th key never increases, outputs
are sorted and duplicate-free and agree with the distance definition, and
the relaxed path length stays within the (delay+1) x strict bound of
section 4.1.3 (checked on every query of a seeded mixture workload)."""
import numpy as np
import pytest

import oracle
import synth


@pytest.fixture(scope="module")
def workload():
    base = synth.make_base(3000, 32, "u8", 8, 901)
    q = synth.make_queries(40, 32, "u8", 8, 901, 902)
    adj, entry = synth.build_graph(base, 16, 903, threads=4)
    return base, q, adj, entry


@pytest.mark.parametrize("delay", [0, 1, 2, 3])
@pytest.mark.parametrize("L", [8, 32])
def test_invariants(workload, delay, L):
    base, q, adj, entry = workload
    cap = 3000
    r = oracle.search(base, adj, entry, q, k=8, L=L, delay=delay, trace_cap=cap)
    for i in range(len(q)):
        tr = r["trace"][i]
        tr = tr[tr >= 0]
        assert len(tr) == int(r["steps"][i]) <= len(base)
        assert len(set(tr.tolist())) == len(tr)            # expanded at most once
        th = r["theta"][i]
        th = th[~np.isnan(th)]
        assert len(th) == len(tr)                           # every selected node is processed
        assert np.all(th[1:] <= th[:-1])                    # L-th key monotone
        ids, ds = r["ids"][i], r["dists"][i]
        assert len(set(ids.tolist())) == len(ids)
        keys = list(zip(ds.tolist(), ids.tolist()))
        assert keys == sorted(keys)
        full = oracle.distances(base, q[i])
        np.testing.assert_array_equal(ds, full[ids])


def test_relaxed_step_bound(workload):
    """|P_relax| <= (delay + 1) * |P_strict| (section 4.1.3, Eq. 5)."""
    base, q, adj, entry = workload
    for L in (8, 32, 64):
        s0 = oracle.search(base, adj, entry, q, k=8, L=L, delay=0)["steps"].astype(np.int64)
        for delay in (1, 2, 3):
            sd = oracle.search(base, adj, entry, q, k=8, L=L, delay=delay)["steps"]
            assert np.all(sd <= (delay + 1) * s0)


def test_threads_do_not_change_results(workload):
    base, q, adj, entry = workload
    a = oracle.search(base, adj, entry, q, k=8, L=32, delay=1, threads=1)
    b = oracle.search(base, adj, entry, q, k=8, L=32, delay=1, threads=5)
    for key in ("ids", "dists", "steps"):
        np.testing.assert_array_equal(a[key], b[key])


def test_beam_one_is_default(workload):
    base, q, adj, entry = workload
    a = oracle.search(base, adj, entry, q, k=8, L=32, delay=1)
    b = oracle.search(base, adj, entry, q, k=8, L=32, delay=1, beam=1)
    np.testing.assert_array_equal(a["ids"], b["ids"])
