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
    for case in range(5):
        P.test_beam_schedule_example(case)
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

    import test_oracle_pq as Q
    for dt in (np.uint8, np.int8):
        Q.test_identity_codebook_codes_are_the_vectors(dt)
    for dt in ("u8", "i8"):
        for delay, beam in ((0, 1), (1, 1), (2, 2)):
            Q.test_identity_codebook_search_equals_exact_search(dt, delay, beam)
    for dt, M in ((np.float32, 4), (np.uint8, 8), (np.int8, 3)):
        Q.test_table_is_squared_distance_to_decoded_vector(dt, M)
    for dt in (np.uint8, np.float32):
        Q.test_codes_name_the_nearest_centroid(dt)
    for L, R in ((1, 6), (4, 6), (10, 6), (25, 3)):
        Q.test_strict_pq_equals_heap_formulation(L, R)
    sbase = synth.make_base(2000, 16, "u8", 8, 901)
    sq = synth.make_queries(12, 16, "u8", 8, 901, 902)
    sadj, sentry = synth.build_graph(sbase, 8, 903, threads=2)
    sm = (sbase, sq, sadj, sentry)
    for delay, beam in ((0, 1), (1, 1), (3, 2)):
        Q.test_answer_is_exact_topk_of_expanded(sm, delay, beam)
    Q.test_degenerate_codebook_still_reranks(sm)
    Q.test_L_covering_graph_gives_exact_topk()
    print("ALL PINS HOLD")


if __name__ == "__main__":
    main(sys.argv[1])
