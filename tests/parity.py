"""Comparison rules of the GPU parity tests (imported by the test modules;
not collected by pytest).

Integer vectors: ids, distances and step counts bit-exact (traces too where
recorded).

fp32 vectors (reading R10, tolerance 1e-5 relative), for every query and
every result position j, with gamma the GPU's distances and omega the
oracle's fp64 ones:
  * padding (id -1) at the same positions;
  * |gamma_j - omega_j| <= 1e-5 * omega_j;
  * gamma_j within 1e-5 of the fp64 distance of the GPU's own id;
  * where the ids differ, the fp64 distance of the GPU's id within 1e-5 of
    omega_j (a tie inside the tolerance);
  * where traces are available and equal, ids and step counts equal; where
    they differ, the first divergent selection is between two candidates
    whose fp64 distances lie within 1e-5 of each other (a near-tie the fp32
    arithmetic may order either way).  Unexplained divergences: none; the
    number of explained ones is returned and bounded by the caller.
"""
import numpy as np

import oracle

TOL = 1e-5


def assert_int_parity(g, ref, check_trace=False, rows=None):
    rows = slice(None) if rows is None else rows
    np.testing.assert_array_equal(g["ids"][rows], ref["ids"][rows])
    gd = g["dists"][rows].astype(np.float64)
    gd[g["dists"][rows] == 0xFFFFFFFF] = np.inf
    np.testing.assert_array_equal(gd, ref["dists"][rows])
    np.testing.assert_array_equal(g["steps"][rows], ref["steps"][rows])
    if check_trace:
        cap = g["trace"].shape[1]
        np.testing.assert_array_equal(g["trace"][rows], ref["trace"][rows][:, :cap])


def assert_f32_query(full, ids, gd, rids, rd):
    """The positional rule for one query; `full` holds the fp64 distances of
    every base row to the query."""
    ids = np.asarray(ids)
    rids = np.asarray(rids)
    gd = np.asarray(gd, dtype=np.float64)
    rd = np.asarray(rd, dtype=np.float64)
    np.testing.assert_array_equal(ids < 0, rids < 0)
    ok = ids >= 0
    np.testing.assert_allclose(gd[ok], full[ids[ok]], rtol=TOL, atol=0)
    assert np.all(np.abs(gd[ok] - rd[ok]) <= TOL * rd[ok]), (gd[ok], rd[ok])
    diff = ok & (ids != rids)
    assert np.all(np.abs(full[ids[diff]] - rd[diff]) <= TOL * rd[diff]), (ids, rids)
    return int(diff.any())


def assert_f32_parity(base, q, g, ref, max_diverged=None):
    """The fp32 rule over a batch with traces; returns the number of queries
    whose traces diverged at a near-tie (asserted <= max_diverged, default
    5 % of the batch, at least 1)."""
    diverged = unexplained = 0
    for i in range(len(q)):
        full = oracle.distances(base, q[i])
        assert_f32_query(full, g["ids"][i], g["dists"][i], ref["ids"][i], ref["dists"][i])
        gt, rt = g["trace"][i], ref["trace"][i][: g["trace"].shape[1]]
        if np.array_equal(gt, rt):
            np.testing.assert_array_equal(g["ids"][i], ref["ids"][i])
            assert g["steps"][i] == ref["steps"][i]
            continue
        diverged += 1
        t = int(np.argmax(gt != rt))
        a, b = int(gt[t]), int(rt[t])
        if not (a >= 0 and b >= 0 and abs(full[a] - full[b]) <= TOL * max(full[a], full[b])):
            unexplained += 1
    assert unexplained == 0, "%d divergent queries without a near-tie" % unexplained
    bound = max(1, len(q) // 20) if max_diverged is None else max_diverged
    print("fp32 parity: %d of %d queries diverged at a near-tie" % (diverged, len(q)))
    assert diverged <= bound, "%d near-tie divergences (bound %d)" % (diverged, bound)
    return diverged
