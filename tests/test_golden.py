"""The oracle's two routines against pairs worked out by hand from the
definitions of Sec. 1 (tests/golden/hand_examples.txt)."""
import numpy as np
import pytest

import oracle
from golden_examples import close, load

EXAMPLES = load()


def test_fixture_is_consistent():
    # the partition identity behind Step 5 holds for every hand-worked line
    for e in EXAMPLES:
        n = e["u"].size
        assert e["v"].size == n, e["name"]
        total = e["nc"] + e["nd"] + e["n1"] + e["n2"] - e["n3"]
        assert total == n * (n - 1) // 2, e["name"]
    assert len(EXAMPLES) >= 8


@pytest.mark.parametrize("method", ["brute", "gse"])
@pytest.mark.parametrize("e", EXAMPLES, ids=[e["name"] for e in EXAMPLES])
def test_oracle_matches_hand_examples(e, method):
    got = oracle.pair_counts(e["u"], e["v"], method)
    for k in ("nc", "nd", "n1", "n2", "n3"):
        assert got[k] == e[k], (k, got[k], e[k])
    X = np.vstack([e["u"], e["v"]])
    res = oracle.allpairs(X, method)
    assert close(float(res["tau_b"][0]), e["tau_b"])
    assert close(float(res["tau_a"][0]), e["tau_a"])


@pytest.mark.parametrize("method", ["brute", "gse"])
@pytest.mark.parametrize("e", EXAMPLES, ids=[e["name"] for e in EXAMPLES])
def test_selected_pairs_match_hand_examples(e, method):
    # the list-of-pairs routine returns per-pair n1 (of the first row) and n2
    # (of the second); swapping the rows swaps them and keeps the rest
    X = np.vstack([e["u"], e["v"]])
    got = oracle.pairs(X, [0, 1], [1, 0], method)
    for k in ("nc", "nd", "n3"):
        assert got[k][0] == e[k] and got[k][1] == e[k], k
    assert got["n1"][0] == e["n1"] and got["n2"][0] == e["n2"]
    assert got["n1"][1] == e["n2"] and got["n2"][1] == e["n1"]
    assert close(float(got["tau_b"][0]), e["tau_b"])
    assert close(float(got["tau_b"][1]), e["tau_b"])
    assert close(float(got["tau_a"][0]), e["tau_a"])
