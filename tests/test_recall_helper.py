"""The recall helper's exact k-th distances (a full scan in chunks whose
distance blocks stay below 2^31 elements) against the oracle's brute force,
on the CPU; chunking is forced by lowering the block limit."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
recall = pytest.importorskip("paper_2507_10070_amd.recall")


@pytest.mark.parametrize("dtype,d", [("u8", 128), ("i8", 100), ("f32", 96)])
def test_exact_kth_matches_bruteforce(monkeypatch, dtype, d):
    base = synth.make_base(3000, d, dtype, 8, 41)
    q = synth.make_queries(37, d, dtype, 8, 41, 42)
    _, bd = oracle.bruteforce(base, q, 10)
    monkeypatch.setattr(recall, "MAX_BLOCK", 5 * 3000)   # 5 queries per block
    kth = recall.exact_kth(base, q, 10, "cpu", check=2)
    if dtype == "f32":
        np.testing.assert_allclose(kth, bd[:, 9], rtol=1e-5)
    else:
        np.testing.assert_array_equal(kth, bd[:, 9])


def test_recall_at_is_tie_aware():
    kth = np.array([4.0, 9.0])
    d = np.array([[1, 2, 4, 4, 4, 4, 4, 4, 4, 4, 4], [1, 9, 10, 10, 10, 10, 10, 10, 10, 10, 10]],
                 dtype=np.float64)
    assert recall.recall_at(d, kth) == pytest.approx((10 + 2) / 20)
