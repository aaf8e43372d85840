"""Continuous-batching service: results are the same for a query served
alone and inside a concurrent stream of arrivals with differing k and L
(bit-exact for u8), equal the oracle, stay within the HBM budget, and the
kernel is started again after it leaves when idle."""
import time

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
fa = pytest.importorskip("paper_2507_10070_amd")


@pytest.fixture(scope="module")
def cfg1():
    cfg = synth.WORKLOADS["10k-u8-128"]
    base, q = synth.make_dataset(cfg)
    adj, entry = synth.build_graph(base, cfg.R, 3001, threads=8)
    return base, q, adj, entry


def plan(nq, seed):
    rng = np.random.default_rng(seed)
    ks = rng.choice([10, 100], nq)
    Ls = np.array([rng.choice([L for L in (32, 64, 128, 256) if L >= k]) for k in ks])
    return ks, Ls


def collect(srv, n, timeout_s=60):
    got = {}
    t_end = time.time() + timeout_s
    while len(got) < n and time.time() < t_end:
        for r in srv.poll(timeout_us=2000):
            got[r["tag"]] = r
    assert len(got) == n, "only %d of %d results" % (len(got), n)
    return got


def test_alone_vs_mix(cfg1):
    base, q, adj, entry = cfg1
    ks, Ls = plan(len(q), 1)
    with fa.Index(base, adj, entry, 256, fa.TIER_HOST) as ix:
        with fa.Server(ix, hbm_budget_bytes=64 << 20) as srv:
            alone = {}
            for i in range(len(q)):          # one at a time
                srv.submit(q[i], int(ks[i]), int(Ls[i]), i)
                alone.update(collect(srv, 1))
            rng = np.random.default_rng(2)
            for i in rng.permutation(len(q)):  # a stream with Poisson gaps
                srv.submit(q[i], int(ks[i]), int(Ls[i]), 1000 + i)
                time.sleep(rng.exponential(20e-6))
            mix = {t - 1000: r for t, r in collect(srv, len(q)).items()}
            st = srv.stats()
    assert st["completed"] == 2 * len(q)
    for i in range(len(q)):
        a, m = alone[i], mix[i]
        np.testing.assert_array_equal(a["ids"], m["ids"])
        np.testing.assert_array_equal(a["dists"], m["dists"])
        assert a["steps"] == m["steps"]
        ref = oracle.search(base, adj, entry, q[i:i + 1], int(ks[i]), int(Ls[i]), delay=1)
        np.testing.assert_array_equal(m["ids"], ref["ids"][0])
        np.testing.assert_array_equal(m["dists"].astype(np.float64), ref["dists"][0])
        assert m["steps"] == ref["steps"][0]


def test_budget_bounds_admission(cfg1):
    base, q, adj, entry = cfg1
    with fa.Index(base, adj, entry, 256, fa.TIER_HBM) as ix:
        probe = fa.Server(ix, hbm_budget_bytes=64 << 20)
        resident = probe.stats()["resident_waves"]
        probe.close()
        entry_bytes = 16 + 128
        with fa.Server(ix, hbm_budget_bytes=(resident + 3) * entry_bytes) as srv:
            assert srv.stats()["slots"] == 3
            for i in range(len(q)):
                srv.submit(q[i], 10, 64, i)
            got = collect(srv, len(q))
            st = srv.stats()
    assert st["max_inflight"] <= 3
    ref = oracle.search(base, adj, entry, q, 10, 64, delay=1)
    for i in range(len(q)):
        np.testing.assert_array_equal(got[i]["ids"], ref["ids"][i])


def test_idle_exit_and_relaunch(cfg1):
    base, q, adj, entry = cfg1
    with fa.Index(base, adj, entry, 256, fa.TIER_HBM) as ix:
        with fa.Server(ix, hbm_budget_bytes=64 << 20, idle_polls=300) as srv:
            srv.submit(q[0], 10, 64, 0)
            r0 = collect(srv, 1)[0]
            time.sleep(0.5)                   # the kernel leaves while idle
            srv.submit(q[1], 10, 64, 1)
            r1 = collect(srv, 1)[1]
            st = srv.stats()
    assert st["relaunches"] >= 1
    ref = oracle.search(base, adj, entry, q[:2], 10, 64, delay=1)
    np.testing.assert_array_equal(r0["ids"], ref["ids"][0])
    np.testing.assert_array_equal(r1["ids"], ref["ids"][1])


def test_server_rejects_bad_requests(cfg1):
    base, q, adj, entry = cfg1
    with fa.Index(base, adj, entry, 256, fa.TIER_HBM) as ix:
        with fa.Server(ix, hbm_budget_bytes=64 << 20, k_max=20, L_max=64) as srv:
            for k, L in ((0, 10), (21, 64), (10, 65), (30, 20)):
                with pytest.raises(fa.AnnError) as e:
                    srv.submit(q[0], k, L, 0)
                assert e.value.code == -22
        with pytest.raises(fa.AnnError) as e:
            fa.Server(ix, hbm_budget_bytes=1000)
        assert e.value.code == -12


@pytest.mark.parametrize("delay,beam", [(2, 2), (0, 4), (3, 1)])
def test_server_generic_schedules(cfg1, delay, beam):
    """The server runs any (delay, beam width) the batch search runs; every
    result equals the oracle's at its own k and L."""
    base, q, adj, entry = cfg1
    ks, Ls = plan(len(q), 7)
    with fa.Index(base, adj, entry, 256, fa.TIER_HOST) as ix:
        with fa.Server(ix, hbm_budget_bytes=64 << 20, delay=delay, beam_width=beam) as srv:
            for i in range(len(q)):
                srv.submit(q[i], int(ks[i]), int(Ls[i]), i)
            got = collect(srv, len(q))
    for i in range(len(q)):
        ref = oracle.search(base, adj, entry, q[i:i + 1], int(ks[i]), int(Ls[i]), delay=delay,
                            beam=beam)
        np.testing.assert_array_equal(got[i]["ids"], ref["ids"][0])
        np.testing.assert_array_equal(got[i]["dists"].astype(np.float64), ref["dists"][0])
        assert got[i]["steps"] == ref["steps"][0]


def test_server_rejects_too_deep_a_pipeline(cfg1):
    base, q, adj, entry = cfg1
    with fa.Index(base, adj, entry, 256, fa.TIER_HOST) as ix:
        with pytest.raises(fa.AnnError) as e:
            fa.Server(ix, hbm_budget_bytes=64 << 20, delay=2, beam_width=3)
        assert e.value.code == -95


# Serving through the agent transport: records in a file (or host DRAM) read
# by the server's own host agents, one request line per resident wave.
def _file_index(tmp_path, base, adj, entry):
    d = str(tmp_path / "ix")
    fa.save_index(d, base, adj, entry, 512)
    return fa.Index.load(d, fa.TIER_FILE)


@pytest.mark.parametrize("delay,beam", [(1, 1), (2, 2)])
def test_server_file_tier_matches_oracle(cfg1, tmp_path, delay, beam):
    base, q, adj, entry = cfg1
    ks, Ls = plan(len(q), 11)
    with _file_index(tmp_path, base, adj, entry) as ix:
        with fa.Server(ix, hbm_budget_bytes=64 << 20, delay=delay, beam_width=beam) as srv:
            for i in range(len(q)):
                srv.submit(q[i], int(ks[i]), int(Ls[i]), i)
            got = collect(srv, len(q))
    for i in range(len(q)):
        assert got[i]["status"] == 0
        ref = oracle.search(base, adj, entry, q[i:i + 1], int(ks[i]), int(Ls[i]), delay=delay,
                            beam=beam)
        np.testing.assert_array_equal(got[i]["ids"], ref["ids"][0])
        np.testing.assert_array_equal(got[i]["dists"].astype(np.float64), ref["dists"][0])
        assert got[i]["steps"] == ref["steps"][0]


def test_server_agent_host_tier_and_relaunch(cfg1):
    """AGENT over host DRAM; the kernel leaves between two bursts (short idle
    limit) and the relaunched waves continue their lines' request numbers."""
    base, q, adj, entry = cfg1
    ref = oracle.search(base, adj, entry, q, 10, 64, delay=1)
    with fa.Index(base, adj, entry, 256, fa.TIER_HOST) as ix:
        with fa.Server(ix, hbm_budget_bytes=64 << 20, transport=fa.TRANSPORT_AGENT,
                       idle_polls=200) as srv:
            for burst in range(3):
                for i in range(len(q)):
                    srv.submit(q[i], 10, 64, 1000 * burst + i)
                got = collect(srv, len(q))
                for i in range(len(q)):
                    r = got[1000 * burst + i]
                    assert r["status"] == 0
                    np.testing.assert_array_equal(r["ids"], ref["ids"][i])
                    np.testing.assert_array_equal(r["dists"].astype(np.float64), ref["dists"][i])
                time.sleep(0.3)  # long enough for the idle waves to leave
            st = srv.stats()
    assert st["relaunches"] >= 1


def test_server_agent_read_failure_is_per_query(cfg1, tmp_path):
    base, q, adj, entry = cfg1
    ref = oracle.search(base, adj, entry, q, 10, 64, delay=1, trace_cap=400)
    ids, cnt = np.unique(ref["trace"][ref["trace"] >= 0], return_counts=True)
    cand = ids[(cnt >= 2) & (cnt < len(q)) & (ids != entry)]
    bad = int(cand[0])
    hit = np.array([(row == bad).any() for row in ref["trace"]])
    assert 0 < hit.sum() < len(q)
    with _file_index(tmp_path, base, adj, entry) as ix:
        ix.configure_agent(threads=4, fail_node=bad)
        with fa.Server(ix, hbm_budget_bytes=64 << 20) as srv:
            for i in range(len(q)):
                srv.submit(q[i], 10, 64, i)
            got = collect(srv, len(q))
    for i in range(len(q)):
        if hit[i]:
            assert got[i]["status"] == -5
            assert (got[i]["ids"] == -1).all()
        else:
            assert got[i]["status"] == 0
            np.testing.assert_array_equal(got[i]["ids"], ref["ids"][i])


@pytest.mark.parametrize("tier,scoring,delay,beam", [("host", fa.PQ_CACHE, 1, 1),
                                                     ("host", fa.PQ_TABLE, 0, 1),
                                                     ("file", fa.PQ_AUTO, 2, 2)])
def test_server_pq_navigation_matches_oracle(cfg1, tmp_path, tier, scoring, delay, beam):
    """Compressed navigation in the server: every result equals the oracle's
    PQ search with re-rank, across the k / L mix, for both scorings and the
    file tier (served through the server's own agents)."""
    base, q, adj, entry = cfg1
    cb = synth.train_codebooks(base, 16, iters=4, sample=5000, seed=61)
    ks, Ls = plan(len(q), 21)
    ix = (fa.Index(base, adj, entry, 256, fa.TIER_HOST) if tier == "host"
          else _file_index(tmp_path, base, adj, entry))
    with ix:
        ix.set_pq(cb)
        with fa.Server(ix, hbm_budget_bytes=64 << 20, delay=delay, beam_width=beam,
                       navigation=fa.NAV_PQ, pq_scoring=scoring) as srv:
            for i in range(len(q)):
                srv.submit(q[i], int(ks[i]), int(Ls[i]), i)
            got = collect(srv, len(q))
    for i in range(len(q)):
        assert got[i]["status"] == 0
        ref = oracle.search(base, adj, entry, q[i:i + 1], int(ks[i]), int(Ls[i]), delay=delay,
                            beam=beam, codebooks=cb)
        np.testing.assert_array_equal(got[i]["ids"], ref["ids"][0])
        np.testing.assert_array_equal(got[i]["dists"].astype(np.float64), ref["dists"][0])
        assert got[i]["steps"] == ref["steps"][0]


def test_server_navigation_needs_its_data(cfg1):
    base, q, adj, entry = cfg1
    with fa.Index(base, adj, entry, 256, fa.TIER_HOST) as ix:
        with pytest.raises(fa.AnnError) as e:  # no codes yet
            fa.Server(ix, hbm_budget_bytes=64 << 20, navigation=fa.NAV_PQ)
        assert e.value.code == -22
        cb8 = synth.train_codebooks(base, 8, iters=2, sample=2000, seed=62)
        with fa.Server(ix, hbm_budget_bytes=64 << 20) as srv:
            with pytest.raises(fa.AnnError) as e:  # a running server reads the index
                ix.set_pq(cb8)
            assert e.value.code == -16
            srv.submit(q[0], 10, 64, 0)
            assert (collect(srv, 1)[0]["ids"] >= 0).all()
        ix.set_pq(cb8, drop_nav=True)  # allowed again once the server closed
        with pytest.raises(fa.AnnError) as e:  # the full-precision copy is gone
            fa.Server(ix, hbm_budget_bytes=64 << 20)
        assert e.value.code == -22
        with fa.Server(ix, hbm_budget_bytes=64 << 20, navigation=fa.NAV_PQ) as srv:
            srv.submit(q[0], 10, 64, 0)
            r = collect(srv, 1)[0]
        assert r["status"] == 0 and (r["ids"] >= 0).all()


@pytest.mark.parametrize("transport", ["direct", "agent"])
def test_tickets_past_two_to_the_32(cfg1, transport):
    """Admission tickets start just below 2^32 and run past it: a ticket cut
    to 32 bits anywhere would name the wrong ring entry or stop the claims.
    A small budget keeps the ring short, so its index wraps as well."""
    base, q, adj, entry = cfg1
    ref = oracle.search(base, adj, entry, q, 10, 64, delay=1)
    tr = fa.TRANSPORT_AGENT if transport == "agent" else fa.TRANSPORT_DIRECT
    with fa.Index(base, adj, entry, 256, fa.TIER_HOST) as ix:
        probe = fa.Server(ix, hbm_budget_bytes=64 << 20, transport=tr)
        resident = probe.stats()["resident_waves"]
        probe.close()
        with fa.Server(ix, hbm_budget_bytes=(resident + 5) * (16 + 128), transport=tr,
                       first_ticket=(1 << 32) - 37) as srv:
            for rep in range(3):
                for i in range(len(q)):
                    srv.submit(q[i], 10, 64, 1000 * rep + i)
                got = collect(srv, len(q))
                for i in range(len(q)):
                    r = got[1000 * rep + i]
                    assert r["status"] == 0
                    np.testing.assert_array_equal(r["ids"], ref["ids"][i])
                    np.testing.assert_array_equal(r["dists"].astype(np.float64), ref["dists"][i])
                    assert r["steps"] == ref["steps"][i]
            st = srv.stats()
    assert st["completed"] == 3 * len(q)


def test_index_free_refused_while_a_server_is_open(cfg1):
    base, q, adj, entry = cfg1
    ix = fa.Index(base, adj, entry, 256, fa.TIER_HBM)
    srv = fa.Server(ix, hbm_budget_bytes=64 << 20)
    with pytest.raises(fa.AnnError) as e:
        ix.close()
    assert e.value.code == -16
    srv.submit(q[0], 10, 64, 0)           # the index is intact and still served
    r = collect(srv, 1)[0]
    ref = oracle.search(base, adj, entry, q[:1], 10, 64, delay=1)
    np.testing.assert_array_equal(r["ids"], ref["ids"][0])
    srv.close()
    ix.close()                            # allowed once the server closed
