"""Host-side logic that needs no GPU: the degree selector's choice rule
(paper section 4.3, Eq. 6) and the autotuner's admissibility rule."""
import numpy as np

from paper_2507_10070_amd import autotune, degree_selector


def rows(R, tf, tc, spread=0.0):
    return [{"R": r, "T_f_us": f, "T_c_us": c, "T_f_spread_us": spread}
            for r, f, c in zip(R, tf, tc)]


def test_balanced_degree_at_the_crossing():
    R = [32, 48, 64, 96]
    tc = [10.0 + 0.5 * r for r in R]          # compute grows with the degree
    tf = [45.0] * 4                            # fixed-size reads
    assert degree_selector.select(rows(R, tf, tc)) == 64   # |42-45| is the smallest gap
    assert degree_selector.select_fitted(rows(R, tf, tc))[0] == 64


def test_io_bound_noise_does_not_decide():
    """Reads dominate at every degree and their time is noisy: the raw argmin
    follows the noise, the fitted choice takes the degree with the most
    compute per read."""
    R = [32, 48, 64, 96]
    tc = [25.0, 35.0, 45.6, 68.8]
    tf = [9342.4, 9869.3, 9661.7, 9782.0]     # I/O-bound, +-3 % noise
    assert degree_selector.select(rows(R, tf, tc, 600.0)) == 32
    assert degree_selector.select_fitted(rows(R, tf, tc, 600.0))[0] == 96


def test_compute_bound_takes_the_smallest_degree():
    R = [32, 48, 64, 96]
    tc = [21.3, 28.9, 30.0, 41.0]
    tf = [11.9, 13.4, 12.2, 11.6]
    assert degree_selector.select_fitted(rows(R, tf, tc, 1.0))[0] == 32


def test_reads_growing_with_the_degree():
    """Reads that grow with the record (beyond their noise) are fitted as a
    line; the balance is where the lines cross."""
    R = [32, 48, 64, 96]
    tf = [20.0 + 0.25 * r for r in R]   # 28, 32, 36, 44
    tc = [4.0 + 0.5 * r for r in R]     # 20, 28, 36, 52
    R_star, model = degree_selector.select_fitted(rows(R, tf, tc, 0.5))
    assert R_star == 64 and not model["T_f_constant"]


def test_autotune_in_flight_limit():
    assert autotune.valid({"delay": 3, "beam_width": 2})
    assert not autotune.valid({"delay": 2, "beam_width": 3})
    assert autotune.valid({"delay": 7, "beam_width": 1})


def test_autotune_two_queries_per_wave_schedules():
    """Half-wave queries run the strict and one-step-stale schedules with
    beam width 1 only; the tuner never proposes another combination."""
    for delay in (0, 1):
        assert autotune.valid({"delay": delay, "beam_width": 1, "query_lanes": 32})
    for delay, beam in ((2, 1), (0, 2), (1, 2), (3, 1)):
        assert not autotune.valid({"delay": delay, "beam_width": beam, "query_lanes": 32})
        assert autotune.valid({"delay": delay, "beam_width": beam, "query_lanes": 64})
    assert autotune.DEFAULT["query_lanes"] == 64 and 32 in autotune.SPACE["query_lanes"]


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs on one GPU; any other count exits with a message
    before touching a device."""
    import os
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_kernel_hash_ignores_comments_only():
    """The stored memory-counter figures stay valid across comment edits of the
    kernel source, and not across code edits."""
    import bench

    src = b"int a; // one\n\n// two\nint b;  \n"
    assert bench._code_only(src) == bench._code_only(b"int a;\nint b; // three\n")
    assert bench._code_only(src) != bench._code_only(b"int a;\nint c;\n")
