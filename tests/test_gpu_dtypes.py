"""GPU parity of the int8 and fp32 kernels on every record path, through the
C ABI, against the oracle.

* The shape of the f32/96 workload with 4 KB record slots: degrees 48, 64
  and 96 (more than 64 neighbours take two gather blocks), list size 128,
  staleness 0 and 1, records in host DRAM (direct loads and the host agents)
  and in a file (host agents, O_DIRECT).
* int8/100 (ids at a 112 B offset, degree 48) and fp32/96 through the agent
  transport, from host DRAM and from a file, for strict, relaxed and the
  generic FIFO schedules.
* int8 and fp32 continuous-batching servers (direct loads from HBM, and the
  server's own agents over a file) across a mix of k and L.

int8 results are bit-exact; fp32 results follow the positional rule of
tests/parity.py.
"""
import time

import numpy as np
import pytest

import oracle
import synth
from parity import assert_f32_parity, assert_f32_query, assert_int_parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
fa = pytest.importorskip("paper_2507_10070_amd")


def run(ix, q, k, L, trace_cap=0, **kw):
    qd = torch.from_numpy(np.ascontiguousarray(q)).to("cuda:0")
    trace = None
    if trace_cap:
        trace = torch.full((q.shape[0], trace_cap), -1, dtype=torch.int32, device="cuda:0")
    ids, dists, steps = fa.search(ix, qd, k=k, L=L, trace=trace, **kw)
    torch.cuda.synchronize()
    d = dists.cpu().numpy()
    out = {"ids": ids.cpu().numpy(), "steps": steps.cpu().numpy().view(np.uint32),
           "dists": d if d.dtype == np.float32 else d.view(np.uint32)}
    if trace is not None:
        out["trace"] = trace.cpu().numpy()
    return out


def min_slot(d, elem, R):
    return (((d * elem + 15) // 16) * 16 + 4 * R + 15) // 16 * 16


# ----------------------------------------------------- f32/96, 4 KB slots
@pytest.fixture(scope="module")
def f32_4k():
    base = synth.make_base(6000, 96, "f32", 64, 1003)
    q = synth.make_queries(64, 96, "f32", 64, 1003, 2003)
    graphs = {R: synth.build_graph(base, R, 3003, threads=8) for R in (48, 64, 96)}
    return base, q, graphs


@pytest.mark.parametrize("R", [48, 64, 96])
@pytest.mark.parametrize("path", ["host-direct", "host-agent", "file"])
def test_f32_4k_slot_shape(f32_4k, tmp_path, R, path):
    base, q, graphs = f32_4k
    adj, entry = graphs[R]
    if path == "file":
        d = str(tmp_path / "ix")
        fa.save_index(d, base, adj, entry, 4096)
        ix = fa.Index.load(d, fa.TIER_FILE)
    else:
        ix = fa.Index(base, adj, entry, 4096, fa.TIER_HOST)
    kw = {"transport": fa.TRANSPORT_AGENT} if path == "host-agent" else {}
    with ix:
        assert ix.info()["slot_bytes"] == 4096
        for delay in (0, 1):
            g = run(ix, q, 10, 128, delay=delay, trace_cap=700, **kw)
            ref = oracle.search(base, adj, entry, q, 10, 128, delay=delay, trace_cap=700)
            assert_f32_parity(base, q, g, ref)


# ------------------------------------ int8 / fp32 through the host agents
@pytest.fixture(scope="module")
def i8w():
    base = synth.make_base(6000, 100, "i8", 32, 1004)
    q = synth.make_queries(80, 100, "i8", 32, 1004, 2004)
    adj, entry = synth.build_graph(base, 48, 3004, threads=8)
    return base, q, adj, entry


@pytest.fixture(scope="module")
def f32w():
    base = synth.make_base(5000, 96, "f32", 64, 1005)
    q = synth.make_queries(80, 96, "f32", 64, 1005, 2005)
    adj, entry = synth.build_graph(base, 32, 3005, threads=8)
    return base, q, adj, entry


SCHEDULES = [(0, 1), (1, 1), (2, 1), (1, 2)]


@pytest.mark.parametrize("tier", ["host", "file"])
def test_i8_agent_transport(i8w, tmp_path, tier):
    base, q, adj, entry = i8w
    if tier == "file":
        d = str(tmp_path / "ix")
        fa.save_index(d, base, adj, entry, 512)
        ix = fa.Index.load(d, fa.TIER_FILE)
    else:
        ix = fa.Index(base, adj, entry, 512, fa.TIER_HOST)
    with ix:
        ix.configure_agent(threads=4)
        for delay, beam in SCHEDULES:
            g = run(ix, q, 10, 72, delay=delay, beam_width=beam, transport=fa.TRANSPORT_AGENT,
                    trace_cap=500)
            ref = oracle.search(base, adj, entry, q, 10, 72, delay=delay, beam=beam, trace_cap=500)
            assert_int_parity(g, ref, check_trace=True)
        assert ix.agent_stats()["errors"] == 0


@pytest.mark.parametrize("tier", ["host", "file"])
def test_f32_agent_transport(f32w, tmp_path, tier):
    base, q, adj, entry = f32w
    slot = min_slot(96, 4, 32)
    if tier == "file":
        d = str(tmp_path / "ix")
        fa.save_index(d, base, adj, entry, 1024)
        ix = fa.Index.load(d, fa.TIER_FILE)
    else:
        ix = fa.Index(base, adj, entry, slot, fa.TIER_HOST)
    with ix:
        ix.configure_agent(threads=4)
        for delay, beam in SCHEDULES:
            g = run(ix, q, 10, 96, delay=delay, beam_width=beam, transport=fa.TRANSPORT_AGENT,
                    trace_cap=600)
            ref = oracle.search(base, adj, entry, q, 10, 96, delay=delay, beam=beam, trace_cap=600)
            assert_f32_parity(base, q, g, ref)


# -------------------------------------------------- int8 / fp32 servers
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


def _serve(ix, q, ks, Ls, delay, beam):
    """Each query alone, then all of them as one stream: returns both."""
    with fa.Server(ix, hbm_budget_bytes=64 << 20, delay=delay, beam_width=beam) as srv:
        alone = {}
        for i in range(len(q)):
            srv.submit(q[i], int(ks[i]), int(Ls[i]), i)
            alone.update(collect(srv, 1))
        rng = np.random.default_rng(9)
        for i in rng.permutation(len(q)):
            srv.submit(q[i], int(ks[i]), int(Ls[i]), 1000 + i)
            time.sleep(rng.exponential(20e-6))
        mix = {t - 1000: r for t, r in collect(srv, len(q)).items()}
    for i in range(len(q)):
        assert alone[i]["status"] == 0 and mix[i]["status"] == 0
        np.testing.assert_array_equal(alone[i]["ids"], mix[i]["ids"])
        np.testing.assert_array_equal(alone[i]["dists"], mix[i]["dists"])
        assert alone[i]["steps"] == mix[i]["steps"]
    return mix


@pytest.mark.parametrize("tier,delay,beam", [("hbm", 1, 1), ("file", 0, 1), ("file", 2, 2)])
def test_i8_server(i8w, tmp_path, tier, delay, beam):
    base, q, adj, entry = i8w
    ks, Ls = plan(len(q), 31)
    if tier == "file":
        d = str(tmp_path / "ix")
        fa.save_index(d, base, adj, entry, 512)
        ix = fa.Index.load(d, fa.TIER_FILE)
    else:
        ix = fa.Index(base, adj, entry, 512, fa.TIER_HBM)
    with ix:
        got = _serve(ix, q, ks, Ls, delay, beam)
    for i in range(len(q)):
        ref = oracle.search(base, adj, entry, q[i:i + 1], int(ks[i]), int(Ls[i]), delay=delay,
                            beam=beam)
        np.testing.assert_array_equal(got[i]["ids"], ref["ids"][0])
        np.testing.assert_array_equal(got[i]["dists"].astype(np.float64), ref["dists"][0])
        assert got[i]["steps"] == ref["steps"][0]


@pytest.mark.parametrize("tier,delay,beam", [("hbm", 1, 1), ("file", 0, 1), ("host", 1, 2)])
def test_f32_server(f32w, tmp_path, tier, delay, beam):
    base, q, adj, entry = f32w
    ks, Ls = plan(len(q), 32)
    if tier == "file":
        d = str(tmp_path / "ix")
        fa.save_index(d, base, adj, entry, 1024)
        ix = fa.Index.load(d, fa.TIER_FILE)
    else:
        ix = fa.Index(base, adj, entry, min_slot(96, 4, 32),
                      fa.TIER_HBM if tier == "hbm" else fa.TIER_HOST)
    with ix:
        got = _serve(ix, q, ks, Ls, delay, beam)
    for i in range(len(q)):
        ref = oracle.search(base, adj, entry, q[i:i + 1], int(ks[i]), int(Ls[i]), delay=delay,
                            beam=beam)
        full = oracle.distances(base, q[i])
        assert_f32_query(full, got[i]["ids"], got[i]["dists"], ref["ids"][0], ref["dists"][0])
