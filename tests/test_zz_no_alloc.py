"""The allocation-free search (ann_search_noalloc, through the C ABI) gives
ann_search's results, bit-exact for integer vectors and within the fp32 rule
for float vectors, on two calls in a row (the second smaller, so stale
scratch from the first would show), for one-shot and persistent grids and
kernel-grained synchronisation; it refuses what it cannot serve."""
import numpy as np
import pytest

import synth
from parity import assert_int_parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
fa = pytest.importorskip("paper_2507_10070_amd")
flashann = fa.flashann


@pytest.fixture(scope="module")
def cfg1():
    cfg = synth.WORKLOADS["10k-u8-128"]
    base, q = synth.make_dataset(cfg)
    adj, entry = synth.build_graph(base, cfg.R, 3001, threads=8)
    return base, q, adj, entry


def _out(nq, k, dist_dtype=torch.int32):
    dev = "cuda:0"
    return (torch.full((nq, k), -7, dtype=torch.int32, device=dev),
            torch.full((nq, k), -7, dtype=dist_dtype, device=dev),
            torch.full((nq,), -7, dtype=torch.int32, device=dev))


def _np(out, f32=False):
    ids, dists, steps = (t.cpu().numpy() for t in out)
    return {"ids": ids, "dists": dists if f32 else dists.view(np.uint32),
            "steps": steps.view(np.uint32)}


def _as_ref(g):
    """A GPU result in the oracle's layout (float64 distances, +inf padding)."""
    d = g["dists"].astype(np.float64)
    d[g["dists"] == 0xFFFFFFFF] = np.inf
    return {"ids": g["ids"], "dists": d, "steps": g["steps"]}


MODES = [dict(delay=1), dict(delay=0, persistent=True), dict(delay=2, beam_width=2, persistent=True),
         dict(delay=0, sync_grain=fa.SYNC_KERNEL, spin_limit=1 << 22)]


@pytest.mark.parametrize("tier", ["hbm", "host"])
@pytest.mark.parametrize("mode", range(len(MODES)))
def test_noalloc_matches_search(cfg1, tier, mode):
    base, q, adj, entry = cfg1
    kw = MODES[mode]
    t = fa.TIER_HBM if tier == "hbm" else fa.TIER_HOST
    with fa.Index(base, adj, entry, 256, t) as ix:
        for nq, k, L in ((len(q), 10, 64), (37, 5, 40)):   # second call smaller
            qd = torch.from_numpy(q[:nq]).to("cuda:0")
            ref = _np(fa.search(ix, qd, k=k, L=L, out=_out(nq, k), **kw))
            got = _out(nq, k)
            flashann.search_noalloc(ix, qd, k=k, L=L, out=got, **kw)
            torch.cuda.synchronize()
            assert_int_parity(_np(got), _as_ref(ref))


def test_noalloc_f32_and_pq(cfg1):
    base = synth.make_base(3000, 96, "f32", 32, 611)
    q = synth.make_queries(50, 96, "f32", 32, 611, 612)
    adj, entry = synth.build_graph(base, 24, 613, threads=8)
    with fa.Index(base, adj, entry, 512, fa.TIER_HOST) as ix:
        for nq in (50, 9):
            qd = torch.from_numpy(q[:nq]).to("cuda:0")
            ref = _np(fa.search(ix, qd, k=10, L=64, persistent=True,
                                out=_out(nq, 10, torch.float32)), f32=True)
            got = _out(nq, 10, torch.float32)
            flashann.search_noalloc(ix, qd, k=10, L=64, out=got, persistent=True)
            torch.cuda.synchronize()
            g = _np(got, f32=True)
            # the same kernel on the same inputs: identical bits
            np.testing.assert_array_equal(g["ids"], ref["ids"])
            np.testing.assert_array_equal(g["dists"].view(np.uint32), ref["dists"].view(np.uint32))
            np.testing.assert_array_equal(g["steps"], ref["steps"])
    base, q, adj, entry = cfg1
    cb = synth.train_codebooks(base, 16, iters=3, sample=3000, seed=7)
    with fa.Index(base, adj, entry, 256, fa.TIER_HBM) as ix:
        ix.set_pq(cb)
        for nq in (len(q), 11):
            qd = torch.from_numpy(q[:nq]).to("cuda:0")
            ref = _np(fa.search(ix, qd, k=10, L=48, navigation=fa.NAV_PQ, out=_out(nq, 10)))
            got = _out(nq, 10)
            flashann.search_noalloc(ix, qd, k=10, L=48, out=got, navigation=fa.NAV_PQ)
            torch.cuda.synchronize()
            assert_int_parity(_np(got), _as_ref(ref))


def test_noalloc_refusals(cfg1, tmp_path):
    import ctypes

    base, q, adj, entry = cfg1
    qd = torch.from_numpy(q[:4]).to("cuda:0")
    lib = fa.load_library()
    with fa.Index(base, adj, entry, 256, fa.TIER_HOST) as ix:
        # the agent transport needs host request lines the library allocates
        opts = fa.SearchOptions(delay=1, beam_width=1, transport=fa.TRANSPORT_AGENT)
        o = _out(4, 5)
        rc = lib.ann_search_noalloc(ix.handle, qd.data_ptr(), 4, 5, 16, 0, ctypes.byref(opts),
                                    o[0].data_ptr(), o[1].data_ptr(), o[2].data_ptr(), None)
        assert rc == -22
        with pytest.raises(ValueError):
            flashann.search_noalloc(ix, qd, k=5, L=16, out=None)
    d = str(tmp_path / "ix")
    fa.save_index(d, base, adj, entry, 512)
    with fa.Index.load(d, fa.TIER_FILE) as fix:
        with pytest.raises(fa.AnnError) as e:
            flashann.search_noalloc(fix, qd, k=5, L=16, out=_out(4, 5))
        assert e.value.code == -22
