"""GPU parity of the query-grained record transport (paper section 4.2) and
of the index files, through the C ABI.

The agent transport must give bit-exact results (ids, distances, steps,
traces) for records in pinned host DRAM and in a file; host-forced faults
must affect exactly the queries that expand the faulty node.
"""
import os

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


def run(ix, q, k, L, trace_cap=0, **kw):
    qd = torch.from_numpy(np.ascontiguousarray(q)).to("cuda:0")
    trace = None
    if trace_cap:
        trace = torch.full((q.shape[0], trace_cap), -1, dtype=torch.int32, device="cuda:0")
    ids, dists, steps = fa.search(ix, qd, k=k, L=L, trace=trace, **kw)
    torch.cuda.synchronize()
    out = {"ids": ids.cpu().numpy(), "dists": dists.cpu().numpy().view(np.uint32),
           "steps": steps.cpu().numpy().view(np.uint32)}
    if trace is not None:
        out["trace"] = trace.cpu().numpy()
    return out


def assert_same(g, ref, rows=None):
    rows = slice(None) if rows is None else rows
    np.testing.assert_array_equal(g["ids"][rows], ref["ids"][rows])
    gd = g["dists"][rows].astype(np.float64)
    gd[g["dists"][rows] == 0xFFFFFFFF] = np.inf
    np.testing.assert_array_equal(gd, ref["dists"][rows])
    np.testing.assert_array_equal(g["steps"][rows], ref["steps"][rows])


@pytest.mark.parametrize("delay", [0, 1])
@pytest.mark.parametrize("L", [32, 100])
def test_agent_transport_host_parity(cfg1, delay, L):
    base, q, adj, entry = cfg1
    with fa.Index(base, adj, entry, 256, fa.TIER_HOST) as ix:
        ix.configure_agent(threads=4)
        g = run(ix, q, 10, L, delay=delay, transport=fa.TRANSPORT_AGENT, trace_cap=400)
        st = ix.agent_stats()
    ref = oracle.search(base, adj, entry, q, 10, L, delay=delay, trace_cap=400)
    assert_same(g, ref)
    np.testing.assert_array_equal(g["trace"], ref["trace"])
    assert st["requests"] == int(ref["steps"].sum())   # one request per expansion
    assert st["errors"] == 0


@pytest.mark.parametrize("slot", [256, 512])
@pytest.mark.parametrize("tier", ["hbm", "host", "file"])
def test_index_files_all_tiers(cfg1, tmp_path, slot, tier):
    base, q, adj, entry = cfg1
    d = str(tmp_path / "ix")
    fa.save_index(d, base, adj, entry, slot)
    t = {"hbm": fa.TIER_HBM, "host": fa.TIER_HOST, "file": fa.TIER_FILE}[tier]
    ix = fa.Index.load(d, t)
    try:
        info = ix.info()
        assert info["n"] == base.shape[0] and info["R"] == adj.shape[1]
        assert info["entry"] == entry and info["slot_bytes"] == slot
        if tier == "file":
            print("direct_io", info["direct_io"])
        for delay in (0, 1):
            g = run(ix, q, 10, 64, delay=delay)
            ref = oracle.search(base, adj, entry, q, 10, 64, delay=delay)
            assert_same(g, ref)
    finally:
        ix.close()


def _node_in_some_traces(ref, want_min=2):
    """A node expanded by some queries but not all (not the entry)."""
    tr = ref["trace"]
    counts = {}
    for row in tr:
        for v in set(row[row >= 0].tolist()):
            counts[v] = counts.get(v, 0) + 1
    nq = tr.shape[0]
    cands = sorted((c, v) for v, c in counts.items() if want_min <= c <= nq // 4)
    return cands[len(cands) // 2][1]


@pytest.mark.parametrize("delay", [0, 1])
def test_agent_faults(cfg1, delay):
    base, q, adj, entry = cfg1
    ref = oracle.search(base, adj, entry, q, 10, 64, delay=delay, trace_cap=400)
    bad_node = _node_in_some_traces(ref)
    hit = np.array([(row == bad_node).any() for row in ref["trace"]])
    assert 0 < hit.sum() < len(q)
    with fa.Index(base, adj, entry, 256, fa.TIER_HOST) as ix:
        # a straggler changes nothing
        ix.configure_agent(threads=3, delay_node=bad_node, delay_us=2000)
        assert_same(run(ix, q, 10, 64, delay=delay, transport=fa.TRANSPORT_AGENT), ref)
        # a failed read: those queries report ANN_EIO with ids -1, the others are exact
        ix.configure_agent(threads=3, fail_node=bad_node)
        qd = torch.from_numpy(q).to("cuda:0")
        ids = torch.empty((len(q), 10), dtype=torch.int32, device="cuda:0")
        dists = torch.empty((len(q), 10), dtype=torch.int32, device="cuda:0")
        steps = torch.empty((len(q),), dtype=torch.int32, device="cuda:0")
        with pytest.raises(fa.AnnError) as e:
            fa.search(ix, qd, k=10, L=64, delay=delay, transport=fa.TRANSPORT_AGENT,
                      out=(ids, dists, steps))
        assert e.value.code == -5
        g = {"ids": ids.cpu().numpy(), "dists": dists.cpu().numpy().view(np.uint32),
             "steps": steps.cpu().numpy().view(np.uint32)}
        assert (g["ids"][hit] == -1).all()
        assert_same(g, ref, rows=~hit)
        # a read that never completes: those queries time out (bounded poll)
        ix.configure_agent(threads=3, drop_node=bad_node)
        with pytest.raises(fa.AnnError) as e:
            fa.search(ix, qd, k=10, L=64, delay=delay, transport=fa.TRANSPORT_AGENT,
                      spin_limit=2000, out=(ids, dists, steps))
        assert e.value.code == -110
        g["ids"] = ids.cpu().numpy()
        assert (g["ids"][hit] == -1).all()
        np.testing.assert_array_equal(g["ids"][~hit], ref["ids"][~hit])


def test_transport_validation(cfg1):
    base, q, adj, entry = cfg1
    qd = torch.from_numpy(q[:4]).to("cuda:0")
    with fa.Index(base, adj, entry, 256, fa.TIER_HBM) as ix:
        with pytest.raises(fa.AnnError) as e:
            fa.search(ix, qd, k=10, L=64, transport=fa.TRANSPORT_AGENT)
        assert e.value.code == -22
        with pytest.raises(fa.AnnError) as e:
            fa.search(ix, qd, k=10, L=64, transport=7)
        assert e.value.code == -22


@pytest.mark.parametrize("delay,beam", [(2, 1), (3, 1), (1, 2), (0, 4), (3, 2), (7, 1)])
def test_agent_deep_pipeline_parity(cfg1, tmp_path, delay, beam):
    """Up to (delay + 1) * W requests of one query in flight through the
    agent: host DRAM and file tiers give the oracle's results bit-exactly."""
    base, q, adj, entry = cfg1
    ref = oracle.search(base, adj, entry, q, 10, 64, delay=delay, beam=beam, trace_cap=600)
    with fa.Index(base, adj, entry, 256, fa.TIER_HOST) as ix:
        ix.configure_agent(threads=4)
        g = run(ix, q, 10, 64, delay=delay, beam_width=beam, transport=fa.TRANSPORT_AGENT,
                trace_cap=600)
        assert_same(g, ref)
        np.testing.assert_array_equal(g["trace"], ref["trace"])
        assert ix.agent_stats()["requests"] == int(ref["steps"].sum())
    d = str(tmp_path / "ix")
    fa.save_index(d, base, adj, entry, 512)
    with fa.Index.load(d, fa.TIER_FILE) as fix:
        assert_same(run(fix, q, 10, 64, delay=delay, beam_width=beam), ref)


def test_agent_deep_pipeline_faults(cfg1):
    base, q, adj, entry = cfg1
    ref = oracle.search(base, adj, entry, q, 10, 64, delay=2, beam=2, trace_cap=400)
    bad_node = _node_in_some_traces(ref)
    hit = np.array([(row == bad_node).any() for row in ref["trace"]])
    qd = torch.from_numpy(q).to("cuda:0")
    ids = torch.empty((len(q), 10), dtype=torch.int32, device="cuda:0")
    dists = torch.empty((len(q), 10), dtype=torch.int32, device="cuda:0")
    steps = torch.empty((len(q),), dtype=torch.int32, device="cuda:0")
    with fa.Index(base, adj, entry, 256, fa.TIER_HOST) as ix:
        ix.configure_agent(threads=3, delay_node=bad_node, delay_us=2000)
        assert_same(run(ix, q, 10, 64, delay=2, beam_width=2, transport=fa.TRANSPORT_AGENT), ref)
        ix.configure_agent(threads=3, fail_node=bad_node)
        with pytest.raises(fa.AnnError) as e:
            fa.search(ix, qd, k=10, L=64, delay=2, beam_width=2, transport=fa.TRANSPORT_AGENT,
                      out=(ids, dists, steps))
        assert e.value.code == -5
        g = {"ids": ids.cpu().numpy(), "dists": dists.cpu().numpy().view(np.uint32),
             "steps": steps.cpu().numpy().view(np.uint32)}
        assert (g["ids"][hit] == -1).all()
        assert_same(g, ref, rows=~hit)
        ix.configure_agent(threads=3, drop_node=bad_node)
        with pytest.raises(fa.AnnError) as e:
            fa.search(ix, qd, k=10, L=64, delay=2, beam_width=2, transport=fa.TRANSPORT_AGENT,
                      spin_limit=2000, out=(ids, dists, steps))
        assert e.value.code == -110
        g["ids"] = ids.cpu().numpy()
        assert (g["ids"][hit] == -1).all()
        np.testing.assert_array_equal(g["ids"][~hit], ref["ids"][~hit])


def test_kernel_grained_agent_parity(cfg1, tmp_path):
    """Kernel-grained rounds over the agent transport (host DRAM and file):
    each round's requests all complete before any query computes; results
    equal the strict search."""
    base, q, adj, entry = cfg1
    ref = oracle.search(base, adj, entry, q, 10, 64, delay=0, trace_cap=400)
    with fa.Index(base, adj, entry, 256, fa.TIER_HOST) as ix:
        ix.configure_agent(threads=4)
        g = run(ix, q, 10, 64, delay=0, transport=fa.TRANSPORT_AGENT,
                sync_grain=fa.SYNC_KERNEL, spin_limit=1 << 22, trace_cap=400)
        assert_same(g, ref)
        np.testing.assert_array_equal(g["trace"], ref["trace"])
    d = str(tmp_path / "ix")
    fa.save_index(d, base, adj, entry, 512)
    with fa.Index.load(d, fa.TIER_FILE) as fix:
        assert_same(run(fix, q, 10, 64, delay=0, sync_grain=fa.SYNC_KERNEL,
                        spin_limit=1 << 22), ref)


@pytest.mark.parametrize("stripes", [1, 2, 4])
def test_striped_records_parity(cfg1, tmp_path, stripes):
    """Records striped over S files (record v in file v % S, as over S
    storage devices): the file tier read by the agents' asynchronous reads,
    and the host tier loaded from the stripes, give the oracle's results
    bit-exactly; every stripe serves its share of the reads."""
    base, q, adj, entry = cfg1
    d = str(tmp_path / "ix")
    fa.save_index(d, base, adj, entry, 512)
    paths = [str(tmp_path / ("stripe%d.bin" % s)) for s in range(stripes)]
    fa.save_records_striped(base, adj, 512, paths)
    ref = {delay: oracle.search(base, adj, entry, q, 10, 64, delay=delay, trace_cap=400)
           for delay in (0, 1)}
    with fa.Index.load_striped(d, paths, fa.TIER_FILE) as ix:
        info = ix.info()
        assert info["stripes"] == stripes
        for delay in (0, 1):
            g = run(ix, q, 10, 64, delay=delay, trace_cap=400)
            assert_same(g, ref[delay])
            np.testing.assert_array_equal(g["trace"], ref[delay]["trace"])
        prof = ix.agent_profile()
        print("agent profile", prof)
        assert prof["stripes"] == stripes and prof["errors"] == 0
        assert sum(prof["stripe_requests"]) == prof["requests"]
        assert prof["requests"] == int(ref[0]["steps"].sum() + ref[1]["steps"].sum())
        if stripes > 1:
            assert min(prof["stripe_requests"]) > 0
        if info["direct_io"]:
            assert prof["async_io"] == 1
    with fa.Index.load_striped(d, paths, fa.TIER_HOST) as hix:
        assert_same(run(hix, q, 10, 64, delay=1), ref[1])
        assert_same(run(hix, q, 10, 64, delay=1, transport=fa.TRANSPORT_AGENT), ref[1])


def test_striped_records_faults_and_validation(cfg1, tmp_path):
    base, q, adj, entry = cfg1
    d = str(tmp_path / "ix")
    fa.save_index(d, base, adj, entry, 512)
    paths = [str(tmp_path / ("s%d.bin" % s)) for s in range(3)]
    fa.save_records_striped(base, adj, 512, paths)
    ref = oracle.search(base, adj, entry, q, 10, 64, delay=1, trace_cap=400)
    bad_node = _node_in_some_traces(ref)
    hit = np.array([(row == bad_node).any() for row in ref["trace"]])
    with fa.Index.load_striped(d, paths, fa.TIER_FILE) as ix:
        ix.configure_agent(threads=2, fail_node=bad_node)
        qd = torch.from_numpy(q).to("cuda:0")
        ids = torch.empty((len(q), 10), dtype=torch.int32, device="cuda:0")
        dists = torch.empty((len(q), 10), dtype=torch.int32, device="cuda:0")
        steps = torch.empty((len(q),), dtype=torch.int32, device="cuda:0")
        with pytest.raises(fa.AnnError) as e:
            fa.search(ix, qd, k=10, L=64, delay=1, out=(ids, dists, steps))
        assert e.value.code == -5
        g = {"ids": ids.cpu().numpy(), "dists": dists.cpu().numpy().view(np.uint32),
             "steps": steps.cpu().numpy().view(np.uint32)}
        assert (g["ids"][hit] == -1).all()
        assert_same(g, ref, rows=~hit)
    with pytest.raises(fa.AnnError) as e:      # a stripe too short for its records
        fa.Index.load_striped(d, paths[:2], fa.TIER_FILE)
    assert e.value.code == -5
    with pytest.raises(fa.AnnError) as e:
        fa.save_records_striped(base, adj, 512, [str(tmp_path / ("x%d" % s)) for s in range(17)])
    assert e.value.code == -22
