"""Pairs of the batched workload that the oracle proves quickly, chosen from
the oracle's stored results (tests/golden/expected_c4.json, written by
make_expected.py from the oracle alone), so a test that also calls the
oracle on them stays short."""
import json
import os

import mcs_instances as mi

_GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "expected_c4.json")


def easy_c4(count, start=0, max_nodes=2_000_000):
    """(pairs, indices) of the first count pairs from index start on whose
    stored oracle run finished within max_nodes nodes."""
    with open(_GOLDEN) as f:
        rows = json.load(f)["pairs"]
    idx = [i for i in range(start, len(rows))
           if rows[i]["complete"] and rows[i]["nodes"] <= max_nodes][:count]
    allp = mi.pairs_c4(max(idx) + 1)
    return [allp[i] for i in idx], idx
