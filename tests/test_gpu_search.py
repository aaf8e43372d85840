"""GPU parity: the HIP search (through the C ABI) against the CPU oracle.

Integer vectors: ids, distances, step counts and expansion traces bit-exact.
fp32 vectors: the positional rule of tests/parity.py for every query (each
distance within 1e-5 relative of the oracle's at the same position; a
different id only at a tie inside the tolerance), with trace divergences
explained by a near-tie at the first divergent selection and bounded in
number.
"""
import numpy as np
import pytest

import oracle
import synth
from parity import assert_f32_parity, assert_int_parity

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


@pytest.mark.parametrize("tier", ["hbm", "host"])
@pytest.mark.parametrize("delay", [0, 1])
@pytest.mark.parametrize("L", [16, 64, 100, 200])
def test_10k_u8_parity(cfg1, tier, delay, L):
    base, q, adj, entry = cfg1
    t = fa.TIER_HBM if tier == "hbm" else fa.TIER_HOST
    with fa.Index(base, adj, entry, 256, t) as ix:
        g = gpu_search(ix, q, 10, L, delay=delay, trace_cap=600)
    ref = oracle.search(base, adj, entry, q, 10, L, delay=delay, trace_cap=600)
    assert_int_parity(g, ref, check_trace=True)


@pytest.mark.parametrize("k,L", [(1, 1), (1, 8), (64, 64), (100, 128), (10, 1024)])
def test_k_and_L_edges(cfg1, k, L):
    base, q, adj, entry = cfg1
    with fa.Index(base, adj, entry, 256) as ix:
        for delay in (0, 1):
            g = gpu_search(ix, q[:37], k, L, delay=delay)
            ref = oracle.search(base, adj, entry, q[:37], k, L, delay=delay)
            assert_int_parity(g, ref)


@pytest.mark.parametrize("R", [1, 7, 20])
def test_fewer_neighbours_than_index(cfg1, R):
    base, q, adj, entry = cfg1
    with fa.Index(base, adj, entry, 256) as ix:
        g = gpu_search(ix, q, 10, 48, R=R, delay=1)
    ref = oracle.search(base, adj, entry, q, 10, 48, R=R, delay=1)
    assert_int_parity(g, ref)


@pytest.mark.parametrize("hash_bits", [6, 8, 12])
def test_forgetful_visited_set_is_result_neutral(cfg1, hash_bits):
    """A small visited hash forgets ids; results must not change."""
    base, q, adj, entry = cfg1
    with fa.Index(base, adj, entry, 256) as ix:
        for delay in (0, 1):
            g = gpu_search(ix, q, 10, 128, delay=delay, hash_bits=hash_bits, trace_cap=300)
            ref = oracle.search(base, adj, entry, q, 10, 128, delay=delay, trace_cap=300)
            assert_int_parity(g, ref, check_trace=True)


@pytest.mark.parametrize("wpb", [1, 2, 3, 4])
def test_ragged_batches(cfg1, wpb):
    base, q, adj, entry = cfg1
    with fa.Index(base, adj, entry, 256) as ix:
        for nq in (1, 5, 99):
            g = gpu_search(ix, q[:nq], 10, 64, delay=1, waves_per_block=wpb)
            ref = oracle.search(base, adj, entry, q[:nq], 10, 64, delay=1)
            assert_int_parity(g, ref)


def test_empty_batch(cfg1):
    base, q, adj, entry = cfg1
    with fa.Index(base, adj, entry, 256) as ix:
        g = gpu_search(ix, q[:0], 10, 64)
        assert g["ids"].shape == (0, 10)


def test_stats_counters(cfg1):
    base, q, adj, entry = cfg1
    stats = torch.zeros(3, dtype=torch.int64, device=dev())
    with fa.Index(base, adj, entry, 256, fa.TIER_HOST) as ix:
        g = gpu_search(ix, q, 10, 64, delay=1, stats=stats)
    s = stats.cpu().numpy()
    assert s[0] == int(g["steps"].sum())
    assert s[1] > 0
    assert s[2] == 0  # every record's vector agrees with the navigation copy


def min_slot(d, elem, R):
    """Smallest record slot: vector padded to 16 B, then R int32 ids, 16 B multiple."""
    return (((d * elem + 15) // 16) * 16 + 4 * R + 15) // 16 * 16


@pytest.mark.parametrize("dtype,d,R,extra", [("i8", 100, 48, 208), ("u8", 128, 96, 0),
                                             ("u8", 512, 32, 384), ("i8", 17, 5, 0),
                                             ("u8", 3, 2, 0)])
def test_integer_shapes(dtype, d, R, extra):
    slot = min_slot(d, 1, R) + extra
    base = synth.make_base(4000, d, dtype, 8, 501)
    q = synth.make_queries(64, d, dtype, 8, 501, 502)
    adj, entry = synth.build_graph(base, R, 503, threads=8)
    with fa.Index(base, adj, entry, slot) as ix:
        for delay in (0, 1):
            g = gpu_search(ix, q, 10, 80, delay=delay, trace_cap=400)
            ref = oracle.search(base, adj, entry, q, 10, 80, delay=delay, trace_cap=400)
            assert_int_parity(g, ref, check_trace=True)


def test_ties_broken_by_id():
    rng = np.random.default_rng(5)
    uniq = rng.integers(0, 256, size=(300, 16)).astype(np.uint8)
    base = np.concatenate([uniq, uniq, uniq[:100]])  # duplicates: equal distances
    q = rng.integers(0, 256, size=(20, 16)).astype(np.uint8)
    q[:5] = uniq[:5]  # distance-0 duplicates
    adj, entry = synth.build_graph(base, 12, 7, threads=4)
    with fa.Index(base, adj, entry, 64) as ix:
        for delay in (0, 1):
            g = gpu_search(ix, q, 8, 40, delay=delay)
            ref = oracle.search(base, adj, entry, q, 8, 40, delay=delay)
            assert_int_parity(g, ref)


def test_padding_and_unreachable():
    base = np.array([[1], [2], [3], [9], [200]], dtype=np.uint8)
    adj = np.array([[1, -1], [-1, 0], [0, 1], [4, 2], [3, 3]], dtype=np.int32)
    q = np.array([[0], [250]], dtype=np.uint8)
    with fa.Index(base, adj, 0, min_slot(1, 1, 2)) as ix:
        for delay in (0, 1):
            g = gpu_search(ix, q, 4, 4, delay=delay)
            ref = oracle.search(base, adj, 0, q, 4, 4, delay=delay)
            assert_int_parity(g, ref)
            assert g["ids"][0].tolist() == [0, 1, -1, -1]


@pytest.mark.parametrize("d,R", [(96, 32), (128, 24), (33, 10)])
def test_f32_parity(d, R):
    base = synth.make_base(5000, d, "f32", 64, 601)
    q = synth.make_queries(100, d, "f32", 64, 601, 602)
    adj, entry = synth.build_graph(base, R, 603, threads=8)
    slot = min_slot(d, 4, R)
    with fa.Index(base, adj, entry, slot) as ix:
        for delay in (0, 1):
            g = gpu_search(ix, q, 10, 96, delay=delay, trace_cap=600)
            ref = oracle.search(base, adj, entry, q, 10, 96, delay=delay, trace_cap=600)
            assert_f32_parity(base, q, g, ref)


def test_invalid_arguments(cfg1):
    base, q, adj, entry = cfg1
    qd = torch.from_numpy(q[:4]).to(dev())
    with fa.Index(base, adj, entry, 256) as ix:
        for kw, code in [(dict(k=0, L=8), -22), (dict(k=9, L=8), -22), (dict(k=1, L=8, R=33), -22),
                         (dict(k=1, L=2000), -22), (dict(k=1, L=8, delay=-1), -22),
                         (dict(k=1, L=8, delay=8), -95), (dict(k=1, L=8, beam_width=9), -95),
                         (dict(k=1, L=8, delay=2, beam_width=3), -95),
                         (dict(k=1, L=8, beam_width=0), -22),
                         (dict(k=1, L=8, hash_bits=3), -22),
                         (dict(k=1, L=8, waves_per_block=5), -22)]:
            with pytest.raises(fa.flashann.AnnError) as e:
                fa.search(ix, qd, **kw)
            assert e.value.code == code
    with pytest.raises(fa.flashann.AnnError) as e:
        fa.Index(base, adj, entry, 200)  # slot too small for 128 + 32*4
    assert e.value.code == -22
    with pytest.raises(fa.flashann.AnnError) as e:
        fa.Index(base, adj, base.shape[0], 256)  # entry out of range
    assert e.value.code == -22


def test_phase_stamps_do_not_change_results(cfg1):
    base, q, adj, entry = cfg1
    phases = torch.zeros((q.shape[0], 2), dtype=torch.int64, device=dev())
    with fa.Index(base, adj, entry, 256, fa.TIER_HOST) as ix:
        g = gpu_search(ix, q, 10, 64, delay=0, phases=phases)
        with pytest.raises(fa.AnnError):
            gpu_search(ix, q, 10, 64, delay=1, phases=phases)   # strict schedule only
    ref = oracle.search(base, adj, entry, q, 10, 64, delay=0)
    assert_int_parity(g, ref)
    ph = phases.cpu().numpy()
    assert (ph > 0).all()


def test_degree_selector_small():
    from paper_2507_10070_amd import degree_selector

    rows = degree_selector.profile_degrees([8, 24], n=4000, d=32, dtype="u8", components=8,
                                           slot=256, tier="host", nq=300, L=32)
    assert [r["R"] for r in rows] == [8, 24]
    for r in rows:
        assert r["T_f_us"] > 0 and r["T_c_us"] > 0 and r["expansions"] > 0
    assert degree_selector.select(rows) in (8, 24)


def test_beam_schedule_example_hand_derived():
    """The hand-derived example of tests/golden/beam_schedule_example.json
    (staleness 0..2, beam width 1..2) run on the GPU: every schedule's trace,
    step count and answer as derived by hand."""
    import json
    import os

    path = os.path.join(os.path.dirname(__file__), "golden", "beam_schedule_example.json")
    with open(path) as f:
        gold = json.load(f)
    x = np.array(gold["points_1d_u8"], dtype=np.uint8).reshape(-1, 1)
    adj = np.array(gold["adjacency"], dtype=np.int32)
    q = np.array([[gold["query_1d_u8"]]], dtype=np.uint8)
    with fa.Index(x, adj, gold["entry"], min_slot(1, 1, 2)) as ix:
        for c in gold["cases"]:
            for hbits in (0, 6):
                g = gpu_search(ix, q, gold["k"], gold["L"], delay=c["delay"],
                               beam_width=c["beam"], hash_bits=hbits, trace_cap=16)
                assert g["ids"][0].tolist() == c["ids"], c
                assert g["dists"][0].tolist() == c["dists"], c
                assert int(g["steps"][0]) == c["steps"], c
                tr = g["trace"][0]
                assert tr[tr >= 0].tolist() == c["trace"], c


# Any staleness and beam width: the generic FIFO kernel (delta * W nodes may
# stay in flight after each iteration, up to (delta + 1) * W = 8 in all).
GENERIC = [(2, 1), (3, 1), (7, 1), (0, 2), (1, 2), (2, 2), (3, 2), (0, 4), (1, 4), (0, 8)]


@pytest.mark.parametrize("tier", ["hbm", "host"])
@pytest.mark.parametrize("delay,beam", GENERIC)
def test_generic_schedule_parity(cfg1, tier, delay, beam):
    base, q, adj, entry = cfg1
    t = fa.TIER_HBM if tier == "hbm" else fa.TIER_HOST
    with fa.Index(base, adj, entry, 256, t) as ix:
        for L in (16, 100):
            g = gpu_search(ix, q, 10, L, delay=delay, beam_width=beam, trace_cap=800)
            ref = oracle.search(base, adj, entry, q, 10, L, delay=delay, beam=beam,
                                trace_cap=800)
            assert_int_parity(g, ref, check_trace=True)


@pytest.mark.parametrize("delay,beam", [(2, 1), (1, 3), (0, 4)])
def test_generic_schedule_shapes(delay, beam):
    """i8/100 with R = 48 (two gather blocks per record, ids at a 112 B
    offset), ragged batch, persistent grid."""
    base = synth.make_base(6000, 100, "i8", 32, 701)
    q = synth.make_queries(77, 100, "i8", 32, 701, 702)
    adj, entry = synth.build_graph(base, 48, 703, threads=8)
    with fa.Index(base, adj, entry, 512) as ix:
        for persistent in (False, True):
            g = gpu_search(ix, q, 7, 72, delay=delay, beam_width=beam, persistent=persistent,
                           trace_cap=500)
            ref = oracle.search(base, adj, entry, q, 7, 72, delay=delay, beam=beam, trace_cap=500)
            assert_int_parity(g, ref, check_trace=True)


@pytest.mark.parametrize("delay,beam", [(2, 1), (1, 2), (0, 4)])
def test_generic_schedule_f32(delay, beam):
    base = synth.make_base(5000, 96, "f32", 64, 611)
    q = synth.make_queries(100, 96, "f32", 64, 611, 612)
    adj, entry = synth.build_graph(base, 32, 613, threads=8)
    with fa.Index(base, adj, entry, min_slot(96, 4, 32)) as ix:
        g = gpu_search(ix, q, 10, 96, delay=delay, beam_width=beam, trace_cap=800)
    ref = oracle.search(base, adj, entry, q, 10, 96, delay=delay, beam=beam, trace_cap=800)
    assert_f32_parity(base, q, g, ref)


def test_generic_exhaustive_equals_bruteforce():
    """L >= N on a connected graph expands every node: any schedule returns
    the exact top-k."""
    base = synth.make_base(200, 128, "u8", 4, 721)
    q = synth.make_queries(40, 128, "u8", 4, 721, 722)
    adj, entry = synth.build_graph(base, 16, 723, threads=4)
    bf_ids, bf_d = oracle.bruteforce(base, q, 10)
    with fa.Index(base, adj, entry, 256) as ix:
        for delay, beam in ((2, 1), (1, 4), (0, 8)):
            g = gpu_search(ix, q, 10, 256, delay=delay, beam_width=beam)
            np.testing.assert_array_equal(g["ids"], bf_ids)
            np.testing.assert_array_equal(g["dists"].astype(np.float64), bf_d)
            assert (g["steps"] == 200).all()


# Kernel-grained synchronisation (lockstep rounds with grid barriers): the
# strict search's results, for one partial group of queries and for several
# groups of co-resident queries.
@pytest.mark.parametrize("tier", ["hbm", "host"])
def test_kernel_grained_parity(cfg1, tier):
    base, q, adj, entry = cfg1
    t = fa.TIER_HBM if tier == "hbm" else fa.TIER_HOST
    ref = oracle.search(base, adj, entry, q, 10, 64, delay=0, trace_cap=400)
    with fa.Index(base, adj, entry, 256, t) as ix:
        g = gpu_search(ix, q, 10, 64, delay=0, sync_grain=fa.SYNC_KERNEL, spin_limit=1 << 22,
                       trace_cap=400)
    assert_int_parity(g, ref, check_trace=True)


def test_kernel_grained_many_groups(cfg1):
    base, q, adj, entry = cfg1
    rows = np.random.default_rng(3).integers(0, len(q), 20000)
    qq = q[rows]
    Ls = np.random.default_rng(4).choice(np.array([16, 40, 64], np.int32), len(qq))
    ref = {L: oracle.search(base, adj, entry, q, 10, int(L), delay=0) for L in (16, 40, 64)}
    with fa.Index(base, adj, entry, 256, fa.TIER_HOST) as ix:
        for wpb in (1, 4):
            g = gpu_search(ix, qq, 10, 64, delay=0, sync_grain=fa.SYNC_KERNEL, spin_limit=1 << 22,
                           waves_per_block=wpb, L_per_query=torch.from_numpy(Ls).to(dev()))
            for L in (16, 40, 64):
                sel = Ls == L
                sub = {key: ref[L][key][rows[sel]] for key in ("ids", "dists", "steps")}
                assert_int_parity({key: g[key][sel] for key in ("ids", "dists", "steps")}, sub)


def test_kernel_grained_validation(cfg1):
    base, q, adj, entry = cfg1
    qd = torch.from_numpy(q[:4]).to(dev())
    with fa.Index(base, adj, entry, 256) as ix:
        for kw in (dict(delay=1), dict(delay=0, beam_width=2), dict(delay=0, persistent=True)):
            with pytest.raises(fa.flashann.AnnError) as e:
                fa.search(ix, qd, k=5, L=16, sync_grain=fa.SYNC_KERNEL, **kw)
            assert e.value.code == -22
        with pytest.raises(fa.flashann.AnnError) as e:
            fa.search(ix, qd, k=5, L=16, delay=0, sync_grain=2)
        assert e.value.code == -22
