"""GPU parity with the hot-record cache: part of the records copied into
device memory, the rest read from host memory (direct loads or the agents)
or from record files (the agents).

The cache changes where bytes come from, never which bytes: every search
must still equal the oracle bit for bit (ids, distances, step counts,
expansion traces), the records' own vectors must agree with the navigation
copy (the kernel's record check counts zero mismatches, so no cached copy is
misplaced), and the cache must reach every schedule (strict, one-step-stale,
the generic FIFO that looks slots up at fetch time), both tiles, persistent
and graph launches, the agent transport, which must post requests for the
uncached nodes only, and the server.
"""
import numpy as np
import pytest

import oracle
import synth
from parity import assert_int_parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
fa = pytest.importorskip("paper_2507_10070_amd")


def dev():
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def cfg1():
    cfg = synth.WORKLOADS["10k-u8-128"]
    base, q = synth.make_dataset(cfg)
    adj, entry = synth.build_graph(base, cfg.R, 3001, threads=8)
    return base, q, adj, entry


def gpu_search(ix, q, k, L, trace_cap=0, stats=None, **kw):
    qd = torch.from_numpy(np.ascontiguousarray(q)).to(dev())
    trace = None
    if trace_cap:
        trace = torch.full((q.shape[0], trace_cap), -1, dtype=torch.int32, device=dev())
    ids, dists, steps = fa.search(ix, qd, k=k, L=L, trace=trace, stats=stats, **kw)
    torch.cuda.synchronize()
    out = {"ids": ids.cpu().numpy(), "dists": dists.cpu().numpy().view(np.uint32),
           "steps": steps.cpu().numpy().view(np.uint32)}
    if trace is not None:
        out["trace"] = trace.cpu().numpy()
    return out


def cache_sets(n, entry):
    rng = np.random.default_rng(17)
    return {"entry_only": np.array([entry]),
            "random_tenth": rng.choice(n, n // 10, replace=False),
            "all": rng.permutation(n),
            "none": np.array([], np.int64)}


@pytest.mark.parametrize("which", ["entry_only", "random_tenth", "all", "none"])
@pytest.mark.parametrize("delay,beam", [(0, 1), (1, 1), (2, 1), (1, 2)])
def test_cache_parity(cfg1, which, delay, beam):
    base, q, adj, entry = cfg1
    ids = cache_sets(base.shape[0], entry)[which]
    with fa.Index(base, adj, entry, 256, fa.TIER_HOST) as ix:
        ix.set_record_cache(ids)
        assert ix.info()["cached_records"] == len(ids)
        stats = torch.zeros(3, dtype=torch.int64, device=dev())
        g = gpu_search(ix, q, 10, 64, delay=delay, beam_width=beam, trace_cap=400, stats=stats)
        assert int(stats[2].item()) == 0  # every record read matches its node
    ref = oracle.search(base, adj, entry, q, 10, 64, delay=delay, beam=beam, trace_cap=400)
    assert_int_parity(g, ref, check_trace=True)


def test_cache_with_tiles_persistent_and_graphs(cfg1):
    """Half-wave queries, persistent waves and a captured graph read the same
    cache; a replaced or released cache takes effect in later searches."""
    base, q, adj, entry = cfg1
    n = base.shape[0]
    rng = np.random.default_rng(3)
    ref = oracle.search(base, adj, entry, q, 10, 44, delay=1)
    with fa.Index(base, adj, entry, 256, fa.TIER_HOST) as ix:
        ix.set_record_cache(rng.choice(n, n // 4, replace=False))
        for kw in (dict(query_lanes=32), dict(persistent=True), dict(query_lanes=32, persistent=True)):
            assert_int_parity(gpu_search(ix, q, 10, 44, delay=1, **kw), ref)
        side = torch.cuda.Stream()
        qbuf = torch.from_numpy(q).to(dev())
        with torch.cuda.stream(side):
            gr = fa.SearchGraph(ix, qbuf, k=10, L=44, stream=side, delay=1)
        try:
            for _ in range(3):
                out = gr.launch()
                side.synchronize()
                got = {"ids": out[0].cpu().numpy(), "dists": out[1].cpu().numpy().view(np.uint32),
                       "steps": out[2].cpu().numpy().view(np.uint32)}
                fa.search(ix, qbuf[:9].contiguous(), k=3, L=20, delay=0)  # eager work between
                torch.cuda.synchronize()
                assert_int_parity(got, ref)
        finally:
            gr.close()
        ix.set_record_cache(rng.choice(n, n // 2, replace=False))   # replaced
        assert_int_parity(gpu_search(ix, q, 10, 44, delay=1), ref)
        ix.set_record_cache([])                                    # released
        assert ix.info()["cached_records"] == 0
        assert_int_parity(gpu_search(ix, q, 10, 44, delay=1), ref)


def requests_of(ix):
    return ix.agent_stats()["requests"] if ix.info()["tier"] != fa.TIER_HBM else 0


@pytest.mark.parametrize("tier", ["host", "file"])
@pytest.mark.parametrize("delay,beam", [(0, 1), (1, 1), (2, 1), (1, 2)])
def test_cache_through_the_agents(cfg1, tmp_path, tier, delay, beam):
    """The agent transport posts no request for a cached node and reads its
    copy in device memory: results equal the oracle, and the agents serve
    exactly the expansions of nodes outside the cache (counted from the
    traces)."""
    base, q, adj, entry = cfg1
    n = base.shape[0]
    ids = np.random.default_rng(41).choice(n, n // 5, replace=False)
    cached = np.zeros(n, bool)
    cached[ids] = True
    if tier == "file":
        fa.save_index(str(tmp_path), base, adj, entry, 512)
        ix = fa.Index.load(str(tmp_path), fa.TIER_FILE)
    else:
        ix = fa.Index(base, adj, entry, 256, fa.TIER_HOST)
    with ix:
        ix.set_record_cache(ids)
        r0 = requests_of(ix)
        g = gpu_search(ix, q, 10, 64, delay=delay, beam_width=beam, trace_cap=400,
                       transport=fa.TRANSPORT_AGENT)
        served = requests_of(ix) - r0
    ref = oracle.search(base, adj, entry, q, 10, 64, delay=delay, beam=beam, trace_cap=400)
    assert_int_parity(g, ref, check_trace=True)
    tr = g["trace"][g["trace"] >= 0]
    assert served == int((~cached[tr]).sum())
    assert 0 < served < len(tr)


@pytest.mark.parametrize("transport", ["direct", "agent"])
def test_cache_serves_the_server(cfg1, transport):
    """A server on a cached index: a burst of 500 requests (the 100 queries
    five times over) returns the oracle's result for each."""
    base, q, adj, entry = cfg1
    n = base.shape[0]
    m = 5 * len(q)
    qq = np.tile(q, (5, 1))
    tr = fa.TRANSPORT_DIRECT if transport == "direct" else fa.TRANSPORT_AGENT
    with fa.Index(base, adj, entry, 256, fa.TIER_HOST) as ix:
        ix.set_record_cache(np.arange(0, n, 3))
        with fa.Server(ix, hbm_budget_bytes=64 << 20, transport=tr) as srv:
            srv.submit_batch(qq, np.full(m, 10, np.int32), np.full(m, 48, np.int32),
                             np.arange(m, dtype=np.uint64))
            res = srv.drain(m, timeout_s=60)
        assert (res["status"] == 0).all()
        order = np.argsort(res["tags"])
        got = {"ids": res["ids"][order][:, :10], "dists": res["dists"][order][:, :10],
               "steps": res["steps"][order]}
    ref = oracle.search(base, adj, entry, q, 10, 48, delay=1)
    ref = {key: np.concatenate([ref[key]] * 5) for key in ("ids", "dists", "steps")}
    assert_int_parity(got, ref)


def test_cache_validation(cfg1):
    base, q, adj, entry = cfg1
    n = base.shape[0]
    with fa.Index(base, adj, entry, 256, fa.TIER_HOST) as ix:
        for bad in ([n], [-1], [5, 5]):
            with pytest.raises(fa.AnnError) as e:
                ix.set_record_cache(bad)
            assert e.value.code == -22
        assert ix.info()["cached_records"] == 0
        with fa.Server(ix, hbm_budget_bytes=16 << 20) as srv:
            with pytest.raises(fa.AnnError) as e:
                ix.set_record_cache([1, 2])
            assert e.value.code == -16
    with fa.Index(base, adj, entry, 256, fa.TIER_HBM) as ix:
        with pytest.raises(fa.AnnError) as e:
            ix.set_record_cache([1, 2])
        assert e.value.code == -95
