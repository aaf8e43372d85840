"""Batches of uneven searches in one kernel: per-query L and k, persistent
waves taking queries from a work counter, a processing order, and the same
search captured in a HIP graph and replayed.  Every query must equal the
oracle at its own (k, L), bit-exactly for integer vectors."""
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


def oracle_uneven(base, adj, entry, q, ks, Ls, kmax, delay):
    """Per-query oracle results laid out like the GPU output (stride kmax)."""
    nq = len(q)
    ids = np.full((nq, kmax), -1, np.int32)
    dists = np.full((nq, kmax), np.inf)
    steps = np.zeros(nq, np.uint32)
    for k in np.unique(ks):
        for L in np.unique(Ls):
            sel = np.where((ks == k) & (Ls == L))[0]
            if len(sel) == 0:
                continue
            r = oracle.search(base, adj, entry, q[sel], int(k), int(L), delay=delay)
            ids[sel, :k] = r["ids"]
            dists[sel, :k] = r["dists"]
            steps[sel] = r["steps"]
    return ids, dists, steps


def check(ids, dists, steps, ref):
    rid, rd, rs = ref
    np.testing.assert_array_equal(ids.cpu().numpy(), rid)
    d = dists.cpu().numpy().view(np.uint32).astype(np.float64)
    d[d == 0xFFFFFFFF] = np.inf
    np.testing.assert_array_equal(d, rd)
    np.testing.assert_array_equal(steps.cpu().numpy().view(np.uint32), rs)


def uneven(nq, seed, Ls=(16, 32, 64, 100, 128), ks=(1, 5, 10)):
    rng = np.random.default_rng(seed)
    L = rng.choice(np.array(Ls, np.int32), nq)
    k = np.minimum(rng.choice(np.array(ks, np.int32), nq), L)
    return k.astype(np.int32), L.astype(np.int32)


@pytest.mark.parametrize("persistent", [False, True])
@pytest.mark.parametrize("delay", [0, 1])
@pytest.mark.parametrize("ordered", [False, True])
def test_uneven_batch_parity(cfg1, persistent, delay, ordered):
    base, q, adj, entry = cfg1
    ks, Ls = uneven(len(q), 5 + delay)
    kmax, Lmax = int(ks.max()), int(Ls.max())
    dev = "cuda:0"
    order = torch.from_numpy(np.argsort(-Ls, kind="stable").astype(np.int32)).to(dev) \
        if ordered else None
    with fa.Index(base, adj, entry, 256, fa.TIER_HOST) as ix:
        ids, dists, steps = fa.search(ix, torch.from_numpy(q).to(dev), k=kmax, L=Lmax,
                                      delay=delay, persistent=persistent,
                                      L_per_query=torch.from_numpy(Ls).to(dev),
                                      k_per_query=torch.from_numpy(ks).to(dev), order=order)
        torch.cuda.synchronize()
    check(ids, dists, steps, oracle_uneven(base, adj, entry, q, ks, Ls, kmax, delay))


def test_uneven_batch_i8_d100_r48():
    """i8, d = 100, R = 48, 512 B records, L uniform over {32, 64, 128, 256} in
    one persistent kernel (the batched workload's shape at a reduced N)."""
    base = synth.make_base(30000, 100, "i8", 64, 1004)
    q = synth.make_queries(400, 100, "i8", 64, 1004, 2004)
    adj, entry = synth.build_graph(base, 48, 3004, threads=16)
    ks, Ls = uneven(len(q), 9, Ls=(32, 64, 128, 256), ks=(10,))
    dev = "cuda:0"
    order = torch.from_numpy(np.argsort(-Ls, kind="stable").astype(np.int32)).to(dev)
    with fa.Index(base, adj, entry, 512, fa.TIER_HOST) as ix:
        for delay in (0, 1):
            ids, dists, steps = fa.search(ix, torch.from_numpy(q).to(dev), k=10, L=256,
                                          delay=delay, persistent=True,
                                          L_per_query=torch.from_numpy(Ls).to(dev), order=order)
            torch.cuda.synchronize()
            check(ids, dists, steps, oracle_uneven(base, adj, entry, q, ks, Ls, 10, delay))


def test_graph_replays_match_eager(cfg1):
    base, q, adj, entry = cfg1
    dev = "cuda:0"
    side = torch.cuda.Stream()
    qbuf = torch.from_numpy(q).to(dev)
    ks, Ls = uneven(len(q), 21)
    Lt, kt = torch.from_numpy(Ls).to(dev), torch.from_numpy(ks).to(dev)
    rng = np.random.default_rng(0)
    with fa.Index(base, adj, entry, 256, fa.TIER_HBM) as ix:
        with torch.cuda.stream(side):
            g = fa.SearchGraph(ix, qbuf, k=10, L=128, stream=side, delay=1, L_per_query=Lt,
                               k_per_query=kt)
        try:
            for rep in range(4):
                perm = rng.permutation(len(q))
                qbuf.copy_(torch.from_numpy(q[perm]).to(dev))   # new contents, same buffer
                torch.cuda.synchronize()
                ids, dists, steps = g.launch()
                side.synchronize()
                got = (ids.clone(), dists.clone(), steps.clone())
                # eager work between replays, on the default stream
                e_ids, e_d, e_s = fa.search(ix, qbuf, k=10, L=128, delay=1, L_per_query=Lt,
                                            k_per_query=kt)
                fa.search(ix, qbuf[:17].contiguous(), k=3, L=40, delay=0)
                torch.cuda.synchronize()
                for a, b in zip(got, (e_ids, e_d, e_s)):
                    assert torch.equal(a, b), "replay %d differs from the eager search" % rep
                check(*got, oracle_uneven(base, adj, entry, q[perm], ks, Ls, 10, 1))
        finally:
            g.close()


def test_autotuner_picks_a_valid_setting(cfg1):
    """The tuner's choice runs, stays within the in-flight limit, and its
    results-neutral parameters leave the results unchanged."""
    from paper_2507_10070_amd import autotune

    base, q, adj, entry = cfg1
    dev = "cuda:0"
    qd = torch.from_numpy(q).to(dev)
    ks, Ls = uneven(len(q), 31)
    Lt = torch.from_numpy(Ls).to(dev)
    ref = oracle_uneven(base, adj, entry, q, np.full(len(q), 10, np.int32), Ls, 10, 1)
    kth = ref[1][:, 9]

    def score(ids, dists, steps):
        d = dists.cpu().numpy().view(np.uint32).astype(np.float64)
        return float(np.minimum((d <= kth[:, None]).sum(1), 10).mean() / 10)

    with fa.Index(base, adj, entry, 256, fa.TIER_HOST) as ix:
        res = autotune.tune(ix, qd, 10, 128, cache_path=None, reps=1, passes=1, score=score,
                            space={"delay": (0, 1, 2), "beam_width": (1, 2),
                                   "waves_per_block": (1, 4), "persistent": (False, True)},
                            L_per_query=Lt)
        p = res["params"]
        assert autotune.valid(p)
        assert res["score"] >= res["default"]["score"] - 0.001
        assert all(r["ms"] is not None for r in res["table"])
        # tiles that do not change results: the same search with other tiles
        kw = autotune.search_kwargs(p, {"L_per_query": Lt})
        a = fa.search(ix, qd, k=10, L=128, **kw)
        kw2 = dict(kw, waves_per_block=3, persistent=not p.get("persistent", False))
        kw2.pop("order", None)
        b = fa.search(ix, qd, k=10, L=128, **kw2)
        torch.cuda.synchronize()
        for x, y in zip(a, b):
            assert torch.equal(x, y)
