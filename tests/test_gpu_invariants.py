"""The HIP path against facts that do not come from any implementation here:
hand-worked pairs, closed forms and invariants of the definitions (Sec. 1).

These complement the element-by-element parity tests against the oracle: a
mistake shared by the oracle and the kernels would still fail here.
"""
import math

import numpy as np
import pytest
import torch

from golden_examples import close, load
from paper_1704_03767_amd import ktau as K

pytestmark = pytest.mark.gpu


def _run(X, **kw):
    Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda()
    out = K.ktau_allpairs(Xd, tau_a=True, **kw)
    return {k: v.cpu().numpy() for k, v in out.items() if v is not None}


def _schemes_for(n):
    names = K.ktau_scheme_names()
    return [s for s in range(len(names)) if K.ktau_scheme_capacity(s) >= n]


@pytest.mark.parametrize("e", load(), ids=[e["name"] for e in load()])
def test_hand_examples_every_scheme(e):
    X = np.vstack([e["u"], e["v"]])
    for s in _schemes_for(X.shape[1]):
        got = _run(X, scheme=s)
        assert int(got["nc"][0]) == e["nc"] and int(got["nd"][0]) == e["nd"], s
        assert int(got["n3"][0]) == e["n3"], s
        assert int(got["n1"][0]) == e["n1"] and int(got["n1"][1]) == e["n2"], s
        assert close(float(got["tau_b"][0]), e["tau_b"]), s
        assert close(float(got["tau_a"][0]), e["tau_a"]), s
        # the same pair with the rows swapped: n1 and n2 trade places
        got = _run(X[::-1].copy(), scheme=s)
        assert int(got["nc"][0]) == e["nc"] and int(got["nd"][0]) == e["nd"], s
        assert close(float(got["tau_b"][0]), e["tau_b"]), s


def _lehmer_perm(rng, n):
    """A random permutation of 0..n-1 and its inversion count (sum of its
    Lehmer code digits)."""
    code = np.array([rng.integers(0, n - i) for i in range(n)])
    pool = list(range(n))
    perm = np.array([pool.pop(c) for c in code])
    return perm, int(code.sum())


@pytest.mark.parametrize("n", [2, 3, 64, 129, 1024, 1025, 4096, 8193, 16384, 17941, 32768])
def test_permutation_inversions_closed_form(n):
    rng = np.random.default_rng(n)
    rows, want = [np.arange(n, dtype=np.float32)], []
    for _ in range(5):
        perm, inv = _lehmer_perm(rng, n)
        rows.append(perm.astype(np.float32))
        want.append(inv)
    rows.append(np.arange(n, dtype=np.float32)[::-1].copy())
    want.append(n * (n - 1) // 2)
    X = np.vstack(rows)
    n0 = n * (n - 1) // 2
    for s in _schemes_for(n):
        got = _run(X, scheme=s)
        # pairs (0, x) are slots x - 1: u = identity, v = the permutation
        nd = got["nd"][: len(want)]
        assert np.array_equal(nd, np.array(want)), (s, nd, want)
        assert np.array_equal(got["nc"][: len(want)], n0 - np.array(want)), s
        assert (got["n3"] == 0).all() and (got["n1"] == 0).all()
        assert np.array_equal(got["tau_a"], got["tau_b"])


@pytest.mark.parametrize("n", [128, 1000, 4096])
def test_self_negation_constant_and_monotone_maps(n):
    rng = np.random.default_rng(100 + n)
    u = np.round(rng.standard_normal(n), 1).astype(np.float32)   # ties
    ranks = np.unique(u, return_inverse=True)[1].astype(np.float32)
    X = np.vstack([u, u, -u, np.full(n, 2.5, np.float32), ranks, u * np.float32(8.0),
                   np.ldexp(u, -20).astype(np.float32)])
    got = _run(X)
    m = X.shape[0]
    J = lambda y, x: K.ktau_pair_to_job(m, y, x)
    assert got["tau_b"][J(0, 1)] == 1.0
    assert got["tau_b"][J(0, 2)] == -1.0
    assert got["tau_b"][J(1, 2)] == -1.0
    for y in range(m):
        if y != 3:
            a, b = (y, 3) if y < 3 else (3, y)
            assert math.isnan(got["tau_b"][J(a, b)])
    assert got["n1"][3] == n * (n - 1) // 2
    # rank replacement and exact scalings give the counts of u itself
    for x in (4, 5, 6):
        assert got["tau_b"][J(0, x)] == 1.0
        assert got["nd"][J(0, x)] == 0
        assert got["n1"][x] == got["n1"][0]
    # negation swaps concordant and discordant pairs
    v = np.round(rng.standard_normal(n), 1).astype(np.float32)
    Y = np.vstack([u, v, -v])
    g = _run(Y)
    assert g["nc"][0] == g["nd"][1] and g["nd"][0] == g["nc"][1]
    assert g["tau_b"][0] == -g["tau_b"][1]


def test_shared_sample_permutation_and_partition_identity():
    rng = np.random.default_rng(5)
    m, n = 96, 700
    X = np.round(rng.standard_normal((m, n)), 1).astype(np.float32)
    X[3, : n // 3] = 0.0
    X[4, : n // 3] = -0.0
    a = _run(X)
    b = _run(X[:, rng.permutation(n)].copy())
    for k in ("nc", "nd", "n3", "n1"):
        assert np.array_equal(a[k], b[k]), k
    assert np.array_equal(a["tau_b"], b["tau_b"])
    ys, xs = np.triu_indices(m, 1)
    n0 = n * (n - 1) // 2
    total = a["nc"] + a["nd"] + a["n1"][ys] + a["n1"][xs] - a["n3"]
    assert (total == n0).all()
    # reversing the row order maps pair (y, x) to (m-1-x, m-1-y)
    r = _run(X[::-1].copy())
    J = np.array([K.ktau_pair_to_job(m, m - 1 - x, m - 1 - y) for y, x in zip(ys, xs)])
    for k in ("nc", "nd", "n3"):
        assert np.array_equal(a[k], r[k][J]), k
    assert np.array_equal(a["tau_b"], r["tau_b"][J])
