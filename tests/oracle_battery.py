"""Pin battery run against one oracle library (used by the mutation test).

Usage: python oracle_battery.py LIBRARY.so  -> exit 0 if every pin holds.
Not collected by pytest (no test_ prefix)."""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)

import oracle  # noqa: E402


def main(path):
    oracle.use_library(path)
    import numpy as np
    import test_oracle_pins as P
    import test_oracle_invariants as I
    import synth

    for case in range(3):
        P.test_worked_example(case)
    for dt in (np.uint8, np.int8, np.float32):
        P.test_distances_match_scipy(dt)
        P.test_bruteforce_matches_lexsort(dt)
        for delay in (0, 1):
            P.test_exhaustive_when_L_covers_graph(dt, delay, 1)
    for L, R in ((4, 6), (10, 6), (25, 3)):
        P.test_strict_equals_heap_formulation(np.uint8, L, R)
    P.test_tie_break_smaller_id_first()
    P.test_padding_and_short_results()
    base = synth.make_base(1500, 16, "u8", 4, 77)
    q = synth.make_queries(10, 16, "u8", 4, 77, 78)
    adj, entry = synth.build_graph(base, 8, 79, threads=2)
    wl = (base, q, adj, entry)
    for delay in (0, 1, 2):
        I.test_invariants(wl, delay, 16)
    I.test_relaxed_step_bound(wl)
    print("ALL PINS HOLD")


if __name__ == "__main__":
    main(sys.argv[1])
