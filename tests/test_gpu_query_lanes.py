"""GPU parity of the threads-per-query tile: two queries per wave
(query_lanes = 32), each on one half of the wave.

Every search must equal the oracle exactly as the one-query-per-wave kernel
does (integer vectors: ids, distances, step counts and expansion traces
bit-exact; fp32: the positional rule of tests/parity.py), across the three
merge forms a 32-lane query uses (list of at most 32 entries in registers,
up to 64 entries two per lane, longer lists in LDS), odd batch sizes that
leave a half idle, persistent waves whose halves take queries on their own,
uneven per-query L and k, and graph replays.  The tile's limits are refused
with ANN_ENOTSUP.
"""
import numpy as np
import pytest

import oracle
import synth
from parity import assert_f32_parity, assert_int_parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
fa = pytest.importorskip("paper_2507_10070_amd")

PAIR = dict(query_lanes=32)


def dev():
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def cfg1():
    cfg = synth.WORKLOADS["10k-u8-128"]
    base, q = synth.make_dataset(cfg)
    adj, entry = synth.build_graph(base, cfg.R, 3001, threads=8)
    return base, q, adj, entry


def gpu_search(ix, q, k, L, trace_cap=0, **kw):
    qd = torch.from_numpy(np.ascontiguousarray(q)).to(dev())
    trace = None
    if trace_cap:
        trace = torch.full((q.shape[0], trace_cap), -1, dtype=torch.int32, device=dev())
    ids, dists, steps = fa.search(ix, qd, k=k, L=L, trace=trace, **kw)
    torch.cuda.synchronize()
    out = {"ids": ids.cpu().numpy(), "steps": steps.cpu().numpy().view(np.uint32)}
    d = dists.cpu().numpy()
    out["dists"] = d if d.dtype == np.float32 else d.view(np.uint32)
    if trace is not None:
        out["trace"] = trace.cpu().numpy()
    return out


def min_slot(d, elem, R):
    return (((d * elem + 15) // 16) * 16 + 4 * R + 15) // 16 * 16


@pytest.mark.parametrize("tier", ["hbm", "host"])
@pytest.mark.parametrize("delay", [0, 1])
@pytest.mark.parametrize("L", [16, 32, 44, 64, 100, 200])
def test_pair_parity(cfg1, tier, delay, L):
    base, q, adj, entry = cfg1
    t = fa.TIER_HBM if tier == "hbm" else fa.TIER_HOST
    with fa.Index(base, adj, entry, 256, t) as ix:
        g = gpu_search(ix, q, 10, L, delay=delay, trace_cap=600, **PAIR)
    ref = oracle.search(base, adj, entry, q, 10, L, delay=delay, trace_cap=600)
    assert_int_parity(g, ref, check_trace=True)


@pytest.mark.parametrize("persistent", [False, True])
@pytest.mark.parametrize("wpb", [1, 2, 3, 4])
def test_pair_ragged_batches(cfg1, persistent, wpb):
    """Batch sizes that leave the second half of the last wave idle, or a
    wave with one query only."""
    base, q, adj, entry = cfg1
    with fa.Index(base, adj, entry, 256) as ix:
        for nq in (1, 2, 3, 7, 99):
            for delay in (0, 1):
                g = gpu_search(ix, q[:nq], 10, 44, delay=delay, waves_per_block=wpb,
                               persistent=persistent, **PAIR)
                ref = oracle.search(base, adj, entry, q[:nq], 10, 44, delay=delay)
                assert_int_parity(g, ref)


@pytest.mark.parametrize("k,L", [(1, 1), (1, 8), (32, 32), (33, 33), (64, 64), (100, 128),
                                 (10, 1024)])
def test_pair_k_and_L_edges(cfg1, k, L):
    base, q, adj, entry = cfg1
    with fa.Index(base, adj, entry, 256) as ix:
        for delay in (0, 1):
            g = gpu_search(ix, q[:37], k, L, delay=delay, **PAIR)
            ref = oracle.search(base, adj, entry, q[:37], k, L, delay=delay)
            assert_int_parity(g, ref)


@pytest.mark.parametrize("hash_bits", [6, 8])
def test_pair_forgetful_visited_set(cfg1, hash_bits):
    base, q, adj, entry = cfg1
    with fa.Index(base, adj, entry, 256) as ix:
        for L in (44, 128):
            g = gpu_search(ix, q, 10, L, delay=1, hash_bits=hash_bits, trace_cap=300, **PAIR)
            ref = oracle.search(base, adj, entry, q, 10, L, delay=1, trace_cap=300)
            assert_int_parity(g, ref, check_trace=True)


def test_pair_equals_wave_per_query_with_counters(cfg1):
    """The same steps and rows scored as one query per wave (counters)."""
    base, q, adj, entry = cfg1
    with fa.Index(base, adj, entry, 256, fa.TIER_HOST) as ix:
        out = []
        for lanes in (64, 32):
            stats = torch.zeros(3, dtype=torch.int64, device=dev())
            g = gpu_search(ix, q, 10, 44, delay=1, stats=stats, query_lanes=lanes)
            out.append((g, stats.cpu().numpy()))
    (g64, s64), (g32, s32) = out
    for key in ("ids", "dists", "steps"):
        np.testing.assert_array_equal(g64[key], g32[key])
    np.testing.assert_array_equal(s64, s32)
    assert s32[2] == 0


@pytest.mark.parametrize("dtype,d,R", [("i8", 100, 48), ("u8", 128, 96), ("i8", 17, 5),
                                       ("u8", 3, 2)])
def test_pair_integer_shapes(dtype, d, R):
    base = synth.make_base(4000, d, dtype, 8, 501)
    q = synth.make_queries(64, d, dtype, 8, 501, 502)
    adj, entry = synth.build_graph(base, R, 503, threads=8)
    with fa.Index(base, adj, entry, min_slot(d, 1, R)) as ix:
        for delay in (0, 1):
            g = gpu_search(ix, q, 10, 80, delay=delay, trace_cap=400, **PAIR)
            ref = oracle.search(base, adj, entry, q, 10, 80, delay=delay, trace_cap=400)
            assert_int_parity(g, ref, check_trace=True)


@pytest.mark.parametrize("d,R", [(96, 32), (33, 10)])
def test_pair_f32_parity(d, R):
    base = synth.make_base(5000, d, "f32", 64, 601)
    q = synth.make_queries(100, d, "f32", 64, 601, 602)
    adj, entry = synth.build_graph(base, R, 603, threads=8)
    with fa.Index(base, adj, entry, min_slot(d, 4, R)) as ix:
        for delay in (0, 1):
            for L in (40, 96):
                g = gpu_search(ix, q, 10, L, delay=delay, trace_cap=600, **PAIR)
                ref = oracle.search(base, adj, entry, q, 10, L, delay=delay, trace_cap=600)
                assert_f32_parity(base, q, g, ref)


def test_pair_uneven_batch_and_graph_replays(cfg1):
    """Per-query L and k in one persistent launch with a longest-first order,
    then the same search captured in a HIP graph: every replay equals the
    eager search and the oracle."""
    base, q, adj, entry = cfg1
    rng = np.random.default_rng(77)
    Ls = rng.choice(np.array([8, 20, 44, 64, 100, 256], np.int32), len(q))
    ks = np.minimum(rng.choice(np.array([1, 5, 10], np.int32), len(q)), Ls).astype(np.int32)
    ref_ids = np.full((len(q), 10), -1, np.int32)
    ref_d = np.full((len(q), 10), np.inf)
    ref_s = np.zeros(len(q), np.uint32)
    for k in np.unique(ks):
        for L in np.unique(Ls):
            sel = np.where((ks == k) & (Ls == L))[0]
            if len(sel):
                r = oracle.search(base, adj, entry, q[sel], int(k), int(L), delay=1)
                ref_ids[sel, :k] = r["ids"]
                ref_d[sel, :k] = r["dists"]
                ref_s[sel] = r["steps"]
    d = dev()
    Lt, kt = torch.from_numpy(Ls).to(d), torch.from_numpy(ks).to(d)
    order = torch.from_numpy(np.argsort(-Ls, kind="stable").astype(np.int32)).to(d)
    qbuf = torch.from_numpy(q).to(d)

    def same(ids, dists, steps):
        np.testing.assert_array_equal(ids.cpu().numpy(), ref_ids)
        dd = dists.cpu().numpy().view(np.uint32).astype(np.float64)
        dd[dd == 0xFFFFFFFF] = np.inf
        np.testing.assert_array_equal(dd, ref_d)
        np.testing.assert_array_equal(steps.cpu().numpy().view(np.uint32), ref_s)

    with fa.Index(base, adj, entry, 256, fa.TIER_HBM) as ix:
        out = fa.search(ix, qbuf, k=10, L=256, delay=1, persistent=True, L_per_query=Lt,
                        k_per_query=kt, order=order, **PAIR)
        torch.cuda.synchronize()
        same(*out)
        side = torch.cuda.Stream()
        with torch.cuda.stream(side):
            g = fa.SearchGraph(ix, qbuf, k=10, L=256, stream=side, delay=1, L_per_query=Lt,
                               k_per_query=kt, **PAIR)
        try:
            for rep in range(3):
                ids, dists, steps = g.launch()
                side.synchronize()
                got = (ids.clone(), dists.clone(), steps.clone())
                fa.search(ix, qbuf[:17].contiguous(), k=3, L=40, delay=0)  # eager work between
                torch.cuda.synchronize()
                same(*got)
        finally:
            g.close()


def test_pair_limits_refused(cfg1, tmp_path):
    base, q, adj, entry = cfg1
    qd = torch.from_numpy(q[:4]).to(dev())
    with fa.Index(base, adj, entry, 256, fa.TIER_HOST) as ix:
        for kw in (dict(delay=2), dict(beam_width=2), dict(delay=0, beam_width=2),
                   dict(transport=fa.TRANSPORT_AGENT), dict(sync_grain=fa.SYNC_KERNEL, delay=0)):
            with pytest.raises(fa.AnnError) as e:
                fa.search(ix, qd, k=5, L=20, query_lanes=32, **kw)
            assert e.value.code == -95, kw
        for lanes in (16, 48, 128):
            with pytest.raises(fa.AnnError) as e:
                fa.search(ix, qd, k=5, L=20, query_lanes=lanes)
            assert e.value.code == -22
    # records above 512 B (128 B vector + 128 ids = 640 B)
    b2 = synth.make_base(600, 128, "u8", 4, 11)
    a2, e2 = synth.build_graph(b2, 128, 12, threads=4)
    with fa.Index(b2, a2, e2, 640) as ix:
        with pytest.raises(fa.AnnError) as e:
            fa.search(ix, torch.from_numpy(b2[:3]).to(dev()), k=5, L=20, query_lanes=32)
        assert e.value.code == -95
        g = gpu_search(ix, b2[:3], 5, 20, delay=1)           # one query per wave still serves it
        ref = oracle.search(b2, a2, e2, b2[:3], 5, 20, delay=1)
        assert_int_parity(g, ref)
    # a file tier is read through the agents only
    fa.save_index(str(tmp_path), base, adj, entry, 256)
    with fa.Index.load(str(tmp_path), fa.TIER_FILE) as ix:
        with pytest.raises(fa.AnnError) as e:
            fa.search(ix, qd, k=5, L=20, query_lanes=32)
        assert e.value.code == -95
