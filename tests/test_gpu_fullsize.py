"""Parity at full size: 1M u8/128 vectors, degree-64 graph, 512 B records in
pinned host DRAM, 10,000 queries, k = 10, L = 192 -- the workload and launch
configuration the benchmark times.  The GPU runs every query; the oracle
recomputes a seeded sample of them one by one; sampled rows must match
bit-exactly (ids, distances, steps), for both schedules and both record
transports."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
fa = pytest.importorskip("paper_2507_10070_amd")

L_BENCH = 192
SAMPLE = 256


@pytest.fixture(scope="module")
def w1m():
    cfg = synth.WORKLOADS["1m-u8-128"]
    base, q = synth.make_dataset(cfg)
    adj, entry = synth.build_graph(base, cfg.R, 3000 + cfg.seed_offset, threads=16)
    sample = np.sort(np.random.default_rng(12345).choice(cfg.nq, SAMPLE, replace=False))
    return cfg, base, q, adj, entry, sample


@pytest.mark.parametrize("transport", ["direct", "agent"])
def test_1m_sampled_parity(w1m, transport):
    cfg, base, q, adj, entry, sample = w1m
    tr = fa.TRANSPORT_DIRECT if transport == "direct" else fa.TRANSPORT_AGENT
    qd = torch.from_numpy(q).to("cuda:0")
    with fa.Index(base, adj, entry, cfg.slot, fa.TIER_HOST) as ix:
        for delay in (0, 1):
            ids, dists, steps = fa.search(ix, qd, k=cfg.k, L=L_BENCH, delay=delay, transport=tr)
            torch.cuda.synchronize()
            ids = ids.cpu().numpy()[sample]
            dists = dists.cpu().numpy().view(np.uint32)[sample].astype(np.float64)
            steps = steps.cpu().numpy().view(np.uint32)[sample]
            ref = oracle.search(base, adj, entry, q[sample], cfg.k, L_BENCH, delay=delay,
                                threads=16)
            np.testing.assert_array_equal(ids, ref["ids"])
            np.testing.assert_array_equal(dists, ref["dists"])
            np.testing.assert_array_equal(steps, ref["steps"])
