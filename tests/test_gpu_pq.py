"""GPU parity of compressed (PQ) navigation through the C ABI.

The PQ arithmetic is fp32 in one fixed order on both sides, so codes, the
search path (traces and step counts) and, for u8/i8, the re-ranked ids and
exact distances are bit-exact against the oracle.  For f32 vectors the traces
are bit-exact too; the exact re-rank distances are fp32 sums on the GPU and
fp64 in the oracle, so the positional rule of tests/parity.py applies: each
distance within 1e-5 relative of the oracle's at the same position and of its
own id's fp64 distance, a different id only at a tie inside the tolerance.
"""
import numpy as np
import pytest

import oracle
import synth
from parity import assert_f32_query

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
fa = pytest.importorskip("paper_2507_10070_amd")

def slot_for(d, elem, R):
    return (((d * elem + 15) // 16) * 16 + 4 * R + 15) // 16 * 16


@pytest.fixture(scope="module")
def u8w():
    cfg = synth.WORKLOADS["10k-u8-128"]
    base, q = synth.make_dataset(cfg)
    q = q[:300]
    adj, entry = synth.build_graph(base, cfg.R, 3001, threads=8)
    cbs = {M: synth.train_codebooks(base, M, iters=6, sample=5000, seed=40 + M)
           for M in (8, 16, 32)}
    return base, q, adj, entry, cbs


def run(ix, q, k, L, trace_cap=0, **kw):
    qd = torch.from_numpy(np.ascontiguousarray(q)).to("cuda:0")
    trace = None
    if trace_cap:
        trace = torch.full((q.shape[0], trace_cap), -1, dtype=torch.int32, device="cuda:0")
    ids, dists, steps = fa.search(ix, qd, k=k, L=L, trace=trace, navigation=fa.NAV_PQ, **kw)
    torch.cuda.synchronize()
    d = dists.cpu().numpy()
    out = {"ids": ids.cpu().numpy(), "steps": steps.cpu().numpy().view(np.uint32),
           "dists": d if d.dtype == np.float32 else d.view(np.uint32)}
    if trace is not None:
        out["trace"] = trace.cpu().numpy()
    return out


def assert_int_parity(g, ref):
    np.testing.assert_array_equal(g["steps"], ref["steps"])
    if "trace" in g:
        cap = g["trace"].shape[1]
        np.testing.assert_array_equal(g["trace"], ref["trace"][:, :cap])
    np.testing.assert_array_equal(g["ids"], ref["ids"])
    gd = g["dists"].astype(np.float64)
    gd[g["dists"] == 0xFFFFFFFF] = np.inf
    np.testing.assert_array_equal(gd, ref["dists"])


@pytest.mark.parametrize("M", [8, 16, 32])
def test_codes_bit_exact(u8w, M):
    base, q, adj, entry, cbs = u8w
    with fa.Index(base, adj, entry, 512) as ix:
        ix.set_pq(cbs[M])
        got = ix.pq_codes()
        assert ix.info()["pq_m"] == M and ix.info()["nav_full"] == 1
    np.testing.assert_array_equal(got, oracle.pq_encode(base, cbs[M]))


SCORINGS = ["table", "cache"]


def scoring(name):
    return {"table": fa.PQ_TABLE, "cache": fa.PQ_CACHE}[name]


@pytest.mark.parametrize("sc", SCORINGS)
@pytest.mark.parametrize("tier", ["hbm", "host"])
@pytest.mark.parametrize("delay,beam", [(0, 1), (1, 1), (2, 2), (1, 4)])
@pytest.mark.parametrize("L", [16, 64, 200])
def test_u8_parity(u8w, sc, tier, delay, beam, L):
    base, q, adj, entry, cbs = u8w
    t = fa.TIER_HBM if tier == "hbm" else fa.TIER_HOST
    with fa.Index(base, adj, entry, 512, t) as ix:
        ix.set_pq(cbs[16])
        g = run(ix, q, 10, L, delay=delay, beam_width=beam, trace_cap=800,
                pq_scoring=scoring(sc))
    ref = oracle.search(base, adj, entry, q, 10, L, delay=delay, beam=beam, trace_cap=800,
                        codebooks=cbs[16])
    assert_int_parity(g, ref)


@pytest.mark.parametrize("sc", SCORINGS)
@pytest.mark.parametrize("M", [8, 32])
@pytest.mark.parametrize("persistent", [False, True])
def test_u8_subspaces_and_persistent(u8w, sc, M, persistent):
    base, q, adj, entry, cbs = u8w
    with fa.Index(base, adj, entry, 512) as ix:
        ix.set_pq(cbs[M])
        g = run(ix, q, 10, 48, delay=1, persistent=persistent, trace_cap=500,
                pq_scoring=scoring(sc))
    ref = oracle.search(base, adj, entry, q, 10, 48, delay=1, trace_cap=500, codebooks=cbs[M])
    assert_int_parity(g, ref)


@pytest.mark.parametrize("k,L", [(1, 1), (1, 8), (64, 64), (100, 128), (10, 1024)])
def test_k_and_L_edges(u8w, k, L):
    base, q, adj, entry, cbs = u8w
    with fa.Index(base, adj, entry, 512) as ix:
        ix.set_pq(cbs[16])
        for delay, sc in ((0, "table"), (1, "table"), (1, "cache")):
            g = run(ix, q[:37], k, L, delay=delay, pq_scoring=scoring(sc))
            ref = oracle.search(base, adj, entry, q[:37], k, L, delay=delay, codebooks=cbs[16])
            assert_int_parity(g, ref)


def test_uneven_batch(u8w):
    base, q, adj, entry, cbs = u8w
    rng = np.random.default_rng(17)
    Ls = rng.choice([16, 40, 96, 200], len(q)).astype(np.int32)
    ks = np.minimum(rng.choice([1, 10, 50], len(q)), Ls).astype(np.int32)
    with fa.Index(base, adj, entry, 512) as ix:
        ix.set_pq(cbs[16])
        g = run(ix, q, 50, 200, delay=1, persistent=True,
                L_per_query=torch.from_numpy(Ls).cuda(), k_per_query=torch.from_numpy(ks).cuda())
    for L in np.unique(Ls):
        for k in np.unique(ks[Ls == L]):
            rows = np.where((Ls == L) & (ks == k))[0]
            ref = oracle.search(base, adj, entry, q[rows], int(k), int(L), delay=1,
                                codebooks=cbs[16])
            np.testing.assert_array_equal(g["ids"][rows, :k], ref["ids"])
            np.testing.assert_array_equal(g["steps"][rows], ref["steps"])
            assert (g["ids"][rows, k:] == -1).all()


def test_agent_transport_file_tier(u8w, tmp_path):
    base, q, adj, entry, cbs = u8w
    d = str(tmp_path / "ix")
    fa.save_index(d, base, adj, entry, 512)
    with fa.Index.load(d, fa.TIER_FILE) as ix:
        ix.configure_agent(threads=8)
        ix.set_pq(cbs[16])
        for delay, beam, sc in ((0, 1, "table"), (1, 1, "cache"), (1, 2, "table")):
            g = run(ix, q[:120], 10, 64, delay=delay, beam_width=beam, trace_cap=500,
                    pq_scoring=scoring(sc))
            ref = oracle.search(base, adj, entry, q[:120], 10, 64, delay=delay, beam=beam,
                                trace_cap=500, codebooks=cbs[16])
            assert_int_parity(g, ref)


def test_graph_replay_matches_eager(u8w):
    base, q, adj, entry, cbs = u8w
    qd = torch.from_numpy(np.ascontiguousarray(q)).to("cuda:0")
    st = torch.cuda.Stream()
    with fa.Index(base, adj, entry, 512) as ix:
        ix.set_pq(cbs[16])
        eager = run(ix, q, 10, 64, delay=1)
        g = fa.SearchGraph(ix, qd, 10, 64, st, navigation=fa.NAV_PQ)
        for _ in range(3):
            g.ids.fill_(-7)
            g.launch()
            st.synchronize()
            np.testing.assert_array_equal(g.ids.cpu().numpy(), eager["ids"])
            run(ix, q[:5], 10, 64, delay=0)  # eager work between replays
        g.close()


@pytest.mark.parametrize("dt,d,M,R", [("i8", 100, 25, 48), ("i8", 100, 20, 48)])
def test_i8_parity(dt, d, M, R):
    base = synth.make_base(6000, d, dt, 48, 701)
    q = synth.make_queries(120, d, dt, 48, 701, 702)
    adj, entry = synth.build_graph(base, R, 703, threads=8)
    cb = synth.train_codebooks(base, M, iters=5, sample=4000, seed=704)
    with fa.Index(base, adj, entry, slot_for(d, 1, R)) as ix:
        ix.set_pq(cb)
        np.testing.assert_array_equal(ix.pq_codes(), oracle.pq_encode(base, cb))
        for delay, sc in ((0, "table"), (1, "table"), (1, "cache")):
            g = run(ix, q, 10, 80, delay=delay, trace_cap=600, pq_scoring=scoring(sc))
            ref = oracle.search(base, adj, entry, q, 10, 80, delay=delay, trace_cap=600,
                                codebooks=cb)
            assert_int_parity(g, ref)


@pytest.mark.parametrize("d,M", [(96, 16), (96, 32), (33, 11)])
def test_f32_parity(d, M):
    base = synth.make_base(5000, d, "f32", 64, 601)
    q = synth.make_queries(100, d, "f32", 64, 601, 602)
    adj, entry = synth.build_graph(base, 32, 603, threads=8)
    cb = synth.train_codebooks(base, M, iters=5, sample=4000, seed=605)
    with fa.Index(base, adj, entry, slot_for(d, 4, 32)) as ix:
        ix.set_pq(cb)
        np.testing.assert_array_equal(ix.pq_codes(), oracle.pq_encode(base, cb))
        for delay, sc in ((0, "table"), (1, "table"), (1, "cache")):
            g = run(ix, q, 10, 96, delay=delay, trace_cap=600, pq_scoring=scoring(sc))
            ref = oracle.search(base, adj, entry, q, 10, 96, delay=delay, trace_cap=600,
                                codebooks=cb)
            np.testing.assert_array_equal(g["trace"], ref["trace"])
            np.testing.assert_array_equal(g["steps"], ref["steps"])
            for i in range(len(q)):
                full = oracle.distances(base, q[i])
                assert (g["ids"][i] >= 0).all()
                assert_f32_query(full, g["ids"][i], g["dists"][i], ref["ids"][i], ref["dists"][i])


def test_drop_nav_and_errors(u8w):
    base, q, adj, entry, cbs = u8w
    with fa.Index(base, adj, entry, 512) as ix:
        with pytest.raises(fa.AnnError) as e:  # no codes yet
            run(ix, q[:4], 10, 32)
        assert e.value.code == -22
        with pytest.raises(fa.AnnError):
            ix.pq_codes()
        bad = np.zeros((3, 256, 42), np.float32)  # 3 does not divide 128 evenly into <= 32
        with pytest.raises(ValueError):
            ix.set_pq(bad)
        with pytest.raises(fa.AnnError) as e:  # 128 / 2 = 64 dimensions per subspace
            ix.set_pq(np.zeros((2, 256, 64), np.float32))
        assert e.value.code == -22
        h0 = ix.info()["hbm_bytes"]
        ix.set_pq(cbs[16], drop_nav=True)
        info = ix.info()
        assert info["nav_full"] == 0 and info["pq_m"] == 16
        assert info["hbm_bytes"] == h0 - len(base) * info["nav_stride"] + len(base) * 32 + 16 * 256 * 8 * 4
        g = run(ix, q, 10, 64, delay=1)
        ref = oracle.search(base, adj, entry, q, 10, 64, delay=1, codebooks=cbs[16])
        assert_int_parity(g, ref)
        qd = torch.from_numpy(np.ascontiguousarray(q[:4])).to("cuda:0")
        with pytest.raises(fa.AnnError) as e:  # full navigation needs the copy
            fa.search(ix, qd, k=10, L=32)
        assert e.value.code == -22
        with pytest.raises(fa.AnnError) as e:  # re-encoding needs the copy
            ix.set_pq(cbs[8])
        assert e.value.code == -22
        with pytest.raises(fa.AnnError) as e:
            fa.search(ix, qd, k=10, L=32, delay=0, navigation=fa.NAV_PQ, sync_grain=fa.SYNC_KERNEL)
        assert e.value.code == -95
        with pytest.raises(fa.AnnError) as e:
            fa.Server(ix, hbm_budget_bytes=64 << 20)
        assert e.value.code == -22
        with pytest.raises(fa.AnnError) as e:
            fa.search(ix, qd, k=10, L=32, navigation=fa.NAV_PQ, pq_scoring=3)
        assert e.value.code == -22


@pytest.mark.parametrize("M", [12, 6, 3])  # d/M = 4, 8 (partial last groups) and 16
def test_partial_subspace_groups(M):
    d = 48
    base = synth.make_base(4000, d, "u8", 16, 801)
    q = synth.make_queries(80, d, "u8", 16, 801, 802)
    adj, entry = synth.build_graph(base, 24, 803, threads=8)
    cb = synth.train_codebooks(base, M, iters=4, sample=3000, seed=804)
    with fa.Index(base, adj, entry, slot_for(d, 1, 24)) as ix:
        ix.set_pq(cb)
        ref = oracle.search(base, adj, entry, q, 10, 48, delay=1, trace_cap=400, codebooks=cb)
        for sc in SCORINGS:
            g = run(ix, q, 10, 48, delay=1, trace_cap=400, pq_scoring=scoring(sc))
            assert_int_parity(g, ref)


def test_autotune_picks_a_scoring(u8w):
    from paper_2507_10070_amd import autotune

    base, q, adj, entry, cbs = u8w
    qd = torch.from_numpy(np.ascontiguousarray(q)).to("cuda:0")
    with fa.Index(base, adj, entry, 512) as ix:
        ix.set_pq(cbs[32])
        best = autotune.tune(ix, qd, 10, 64, cache_path=None, reps=1, passes=1,
                             navigation=fa.NAV_PQ)
        assert best["params"]["pq_scoring"] in (fa.PQ_TABLE, fa.PQ_CACHE)
        kw = autotune.search_kwargs(best["params"], {"navigation": fa.NAV_PQ})
        ids, dists, steps = fa.search(ix, qd, k=10, L=64, **kw)
        torch.cuda.synchronize()
    ref = oracle.search(base, adj, entry, q, 10, 64, delay=1, codebooks=cbs[32])
    np.testing.assert_array_equal(ids.cpu().numpy(), ref["ids"])
