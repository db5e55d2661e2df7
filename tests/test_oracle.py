"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each check is chosen so that a plausible slip in the oracle (a dropped tie
term, a '<=' for '<', a wrong sign, a swapped operand, a missing tail copy in
the merge) fails at least one of them:

* brute force on tiny inputs: the sorting routine (Sec. 3.2) equals the
  definition (Sec. 1) on every pair of two exhaustive tiny domains;
* closed forms: a permutation built from a Lehmer code has exactly the sum of
  its digits as inversions; reversal gives n0; one adjacent swap gives 1;
  tie groups of chosen sizes give sum t(t-1)/2 (Table 1 definitions);
* library routines: scipy.stats.kendalltau (tau-b) and numpy.unique
  tie-group counts recover nc - nd, n1, n2, n3 independently;
* invariants stated by the paper or forced by the mathematics: self and
  negation, commutativity (Sec. 1), rank transform and exact monotone maps
  (Sec. 3), a shared sample permutation, the partition identity behind Step 5,
  tau_A = tau_B without ties (Sec. 1).
"""
import itertools
import math

import numpy as np
import pytest
from scipy import stats

import oracle

KEYS = ("nc", "nd", "n1", "n2", "n3")


def n0(n):
    return n * (n - 1) // 2


# ---------------------------------------------------------------- brute force


def _exhaustive_rows(alphabet, length):
    return np.array(list(itertools.product(range(alphabet), repeat=length)), np.float32)


@pytest.mark.parametrize("alphabet,length", [(3, 6), (2, 8)])
def test_routines_agree_on_exhaustive_domain(alphabet, length):
    X = _exhaustive_rows(alphabet, length)          # 729 x 6 or 256 x 8
    a = oracle.allpairs(X, "brute")
    b = oracle.allpairs(X, "gse")
    for k in ("nc", "nd", "n3", "n1"):
        assert np.array_equal(a[k], b[k]), k
    assert np.array_equal(a["tau_b"], b["tau_b"], equal_nan=True)


def test_routines_agree_on_random_tie_heavy_vectors():
    rng = np.random.default_rng(11)
    for n in list(range(2, 40)) + [63, 64, 65, 127, 128, 129, 200, 255, 256, 257, 300]:
        for _ in range(3):
            A = int(rng.integers(1, n + 1))
            u = rng.integers(0, A, n).astype(np.float32)
            v = rng.integers(0, int(rng.integers(1, n + 1)), n).astype(np.float32)
            assert oracle.pair_counts(u, v, "brute") == oracle.pair_counts(u, v, "gse"), (n, A)


# ---------------------------------------------------------------- closed forms


def _perm_from_lehmer(code):
    """Permutation whose element i has code[i] smaller elements after it."""
    avail = list(range(len(code)))
    return np.array([avail.pop(c) for c in code], np.float32)


@pytest.mark.parametrize("method", ["brute", "gse"])
def test_lehmer_code_inversions(method):
    rng = np.random.default_rng(5)
    for n in (2, 3, 7, 16, 33, 100, 257, 1000):
        code = [int(rng.integers(0, n - i)) for i in range(n)]
        v = _perm_from_lehmer(code)
        u = np.arange(n, dtype=np.float32)
        c = oracle.pair_counts(u, v, method)
        assert c["nd"] == sum(code)
        assert c["nc"] == n0(n) - sum(code)
        assert c["n1"] == c["n2"] == c["n3"] == 0


@pytest.mark.parametrize("method", ["brute", "gse"])
def test_reversal_and_adjacent_swap(method):
    for n in (2, 5, 64, 513):
        u = np.arange(n, dtype=np.float32)
        c = oracle.pair_counts(u, u[::-1].copy(), method)
        assert (c["nd"], c["nc"]) == (n0(n), 0)
        for i in sorted({0, max(0, n // 2 - 1), n - 2}):
            v = u.copy()
            v[i], v[i + 1] = v[i + 1], v[i]
            c = oracle.pair_counts(u, v, method)
            assert (c["nd"], c["nc"]) == (1, n0(n) - 1)


@pytest.mark.parametrize("method", ["brute", "gse"])
def test_tie_group_sizes(method):
    rng = np.random.default_rng(9)
    for _ in range(20):
        sizes_u = rng.integers(1, 9, rng.integers(1, 12))
        u = np.repeat(np.arange(sizes_u.size), sizes_u).astype(np.float32)
        n = u.size
        # v: each u-group split into joint sub-groups of chosen sizes, with
        # fresh values so that no two sub-groups share a v value
        v = np.empty(n, np.float32)
        joint = []
        pos, val = 0, 0
        for t in sizes_u:
            left = int(t)
            while left:
                w = int(rng.integers(1, left + 1))
                v[pos:pos + w] = val
                joint.append(w)
                pos += w
                left -= w
                val += 1
        perm = rng.permutation(n)
        c = oracle.pair_counts(u[perm], v[perm], method)
        assert c["n1"] == sum(t * (t - 1) // 2 for t in sizes_u)
        assert c["n3"] == sum(w * (w - 1) // 2 for w in joint)
        assert c["n2"] == c["n3"]          # every v group lies inside one u group


# ------------------------------------------------------------ library routines


def _library_counts(u, v):
    n = u.size

    def tie_pairs(*cols):
        if len(cols) == 1:
            _, cnt = np.unique(cols[0], return_counts=True)
        else:
            _, cnt = np.unique(np.stack(cols, 1), axis=0, return_counts=True)
        return int(sum(int(t) * (int(t) - 1) // 2 for t in cnt))

    n1, n2, n3 = tie_pairs(u), tie_pairs(v), tie_pairs(u, v)
    den = math.sqrt((n0(n) - n1) * (n0(n) - n2))
    tau_b = stats.kendalltau(u.astype(np.float64), v.astype(np.float64), variant="b").statistic
    s = int(round(tau_b * den))                      # nc - nd, exact while den < 1e12
    tot = n0(n) - n1 - n2 + n3                       # nc + nd
    assert (tot + s) % 2 == 0
    return {"nc": (tot + s) // 2, "nd": (tot - s) // 2, "n1": n1, "n2": n2, "n3": n3}, tau_b


@pytest.mark.parametrize("method", ["brute", "gse"])
def test_against_scipy_and_numpy_unique(method):
    rng = np.random.default_rng(3)
    for n in (5, 17, 64, 128, 333, 512):
        for scale in (1, 4, 30, None):
            if scale is None:
                u = rng.standard_normal(n).astype(np.float32)
                v = (0.5 * u + rng.standard_normal(n)).astype(np.float32)
            else:
                u = np.round(rng.standard_normal(n) * scale).astype(np.float32)
                v = np.round((0.5 * u / scale + rng.standard_normal(n)) * scale).astype(np.float32)
            if np.unique(u).size < 2 or np.unique(v).size < 2:
                continue
            lib, tau_lib = _library_counts(u, v)
            c = oracle.pair_counts(u, v, method)
            assert c == lib
            tb, _ = oracle.tau(c, n)
            assert abs(tb - tau_lib) <= 1e-14


# ------------------------------------------------------------------ invariants


def test_self_and_negation_are_exact():
    rng = np.random.default_rng(4)
    for n in (2, 3, 50, 1024, 4096):
        u = np.round(rng.standard_normal(n), 1).astype(np.float32)
        if np.unique(u).size < 2:
            continue
        c = oracle.pair_counts(u, u)
        assert oracle.tau(c, n)[0] == 1.0
        c = oracle.pair_counts(u, -u)
        assert oracle.tau(c, n)[0] == -1.0


def test_constant_row_gives_nan_with_exact_counts():
    n = 40
    u = np.full(n, 2.5, np.float32)
    v = np.round(np.random.default_rng(1).standard_normal(n), 1).astype(np.float32)
    c = oracle.pair_counts(u, v)
    assert c["n1"] == n0(n) and c["nc"] == 0 and c["nd"] == 0 and c["n3"] == c["n2"]
    tb, ta = oracle.tau(c, n)
    assert math.isnan(tb) and ta == 0.0


def test_symmetry_and_partition_identity():
    rng = np.random.default_rng(8)
    X = np.round(rng.standard_normal((12, 90)) * 2).astype(np.float32)
    for y in range(12):
        for x in range(12):
            a = oracle.pair_counts(X[y], X[x])
            b = oracle.pair_counts(X[x], X[y])
            assert (a["nc"], a["nd"], a["n3"]) == (b["nc"], b["nd"], b["n3"])
            assert (a["n1"], a["n2"]) == (b["n2"], b["n1"])
            assert a["nc"] + a["nd"] + a["n1"] + a["n2"] - a["n3"] == n0(90)
            assert oracle.tau(a, 90)[0] == oracle.tau(b, 90)[0] or y == x


def test_monotone_maps_and_sample_permutation():
    rng = np.random.default_rng(12)
    n = 257
    u = np.round(rng.standard_normal(n), 1).astype(np.float32)
    v = np.round(rng.standard_normal(n) + 0.3 * u, 1).astype(np.float32)
    base = oracle.pair_counts(u, v)
    # exact order-preserving maps: scaling by a power of two, shifting into a
    # range where the sum is exact, replacing values by their ranks
    ranks_u = np.unique(u, return_inverse=True)[1].astype(np.float32)
    for uu in (u * np.float32(8.0), u * np.float32(2.0 ** -20), ranks_u):
        assert oracle.pair_counts(uu, v) == base
    # negating v swaps concordant and discordant
    neg = oracle.pair_counts(u, -v)
    assert (neg["nc"], neg["nd"]) == (base["nd"], base["nc"])
    # -0.0 ties with +0.0
    z = np.array([0.0, -0.0, 1.0, -0.0], np.float32)
    w = np.array([1.0, 2.0, 3.0, 4.0], np.float32)
    assert oracle.pair_counts(z, w)["n1"] == 3
    # one permutation of the samples applied to both rows
    p = rng.permutation(n)
    assert oracle.pair_counts(u[p], v[p]) == base


def test_no_ties_tau_a_equals_tau_b():
    rng = np.random.default_rng(13)
    u = rng.permutation(200).astype(np.float32)
    v = rng.permutation(200).astype(np.float32)
    c = oracle.pair_counts(u, v)
    assert c["nc"] + c["nd"] == n0(200)
    tb, ta = oracle.tau(c, 200)
    assert tb == ta


# ------------------------------------------------------ rank transform, top-k


def test_rank_rows_against_numpy():
    rng = np.random.default_rng(14)
    X = np.round(rng.standard_normal((30, 301)), 1).astype(np.float32)
    X[3, :50] = -0.0
    X[3, 50:90] = 0.0
    r = oracle.rank_rows(X)
    for i in range(X.shape[0]):
        assert np.array_equal(r["order"][i], np.argsort(X[i], kind="stable"))
        _, inv, cnt = np.unique(X[i], return_inverse=True, return_counts=True)
        assert np.array_equal(r["rank"][i], inv)
        assert r["n1"][i] == sum(int(t) * (int(t) - 1) // 2 for t in cnt)


def test_query_topk_selection_rule():
    rng = np.random.default_rng(15)
    m, n, k = 300, 64, 25
    db = np.round(rng.standard_normal((m, n)), 1).astype(np.float32)
    db[7] = 1.0                                       # constant row -> NaN, excluded
    db[20] = db[10]                                   # equal |tau| -> smaller index first
    Q = np.round(rng.standard_normal((3, n)), 1).astype(np.float32)
    Q[1] = db[10]
    got = oracle.query_topk(db, Q, k)
    for qi in range(3):
        res = oracle.pairs(np.vstack([Q[qi:qi + 1], db]), np.zeros(m, np.int64),
                           np.arange(1, m + 1))
        tb = res["tau_b"]
        ok = ~np.isnan(tb)
        idx = np.arange(m)[ok]
        order = idx[np.lexsort((idx, -np.abs(tb[ok])))][:k]
        assert np.array_equal(got["idx"][qi], order)
        assert np.array_equal(got["tau"][qi], tb[order])
    assert got["idx"][1][0] in (10, 20) and got["idx"][1][0] == 10
    small = oracle.query_topk(db[:5], Q[:1], 8)
    assert (small["idx"][0][5:] == -1).all() and np.isnan(small["tau"][0][5:]).all()
    assert (small["idx"][0][:5] >= 0).all()


def test_enumeration_is_row_major():
    ys, xs = oracle.enumerate_pairs(6)
    assert list(zip(ys, xs))[:6] == [(0, 1), (0, 2), (0, 3), (0, 4), (0, 5), (1, 2)]
    assert len(ys) == 15 and (ys < xs).all()


def test_nan_is_refused():
    X = np.zeros((3, 4), np.float32)
    X[1, 2] = np.nan
    with pytest.raises(oracle.OracleError):
        oracle.allpairs(X)


# ------------------------------------------------------------ permutation test


def _mahonian(n):
    """Number of permutations of n elements with k inversions, k = 0..n(n-1)/2
    (the textbook recurrence: inserting the n-th element adds 0..n-1)."""
    row = [1]
    for size in range(2, n + 1):
        nxt = [0] * (len(row) + size - 1)
        for k, c in enumerate(row):
            for j in range(size):
                nxt[k + j] += c
        row = nxt
    return row


def _s_by_definition(u, v):
    u, v = [float(t) for t in u], [float(t) for t in v]
    s = 0
    for a in range(len(u)):
        for b in range(a + 1, len(u)):
            du = (u[a] > u[b]) - (u[a] < u[b])
            dv = (v[a] > v[b]) - (v[a] < v[b])
            s += du * dv
    return s


def test_perm_test_identity_permutations():
    rng = np.random.default_rng(8)
    X = np.round(rng.standard_normal((4, 30)), 1).astype(np.float32)
    perms = np.tile(np.arange(30, dtype=np.uint16), (5, 1))
    ys, xs = oracle.enumerate_pairs(4)
    got = oracle.perm_test(X, perms, ys, xs)
    assert (got["count"] == 5).all() and (got["p"] == 1.0).all()


def test_perm_test_all_permutations_give_the_mahonian_tail():
    # u in increasing order, v with distinct values: over all n! permutations
    # of v's samples, S = n0 - 2 (inversions of the permuted v), and the
    # number of permutations with k inversions is the Mahonian number M(n, k)
    n = 6
    n0 = n * (n - 1) // 2
    M = _mahonian(n)
    assert sum(M) == math.factorial(n)
    perms = np.array(list(itertools.permutations(range(n))), dtype=np.uint16)
    rng = np.random.default_rng(9)
    for _ in range(6):
        v = rng.permutation(n).astype(np.float32) + 0.5
        X = np.vstack([np.arange(n, dtype=np.float32), v])
        s_obs = abs(_s_by_definition(X[0], X[1]))
        want = sum(c for k, c in enumerate(M) if abs(n0 - 2 * k) >= s_obs)
        for method in ("gse", "brute"):
            got = oracle.perm_test(X, perms, [0], [1], method)
            assert got["count"][0] == want
            assert got["p"][0] == (1 + want) / (len(perms) + 1)


def test_perm_test_matches_the_definition_with_ties():
    rng = np.random.default_rng(10)
    n, B = 9, 40
    X = rng.integers(0, 4, (5, n)).astype(np.float32)
    X[4] = 1.0                                        # constant row: S = 0 always
    perms = np.array([rng.permutation(n) for _ in range(B)], dtype=np.uint16)
    ys, xs = oracle.enumerate_pairs(5)
    got = oracle.perm_test(X, perms, ys, xs)
    for i, (y, x) in enumerate(zip(ys, xs)):
        s_obs = abs(_s_by_definition(X[y], X[x]))
        want = sum(abs(_s_by_definition(X[y], X[x][p])) >= s_obs for p in perms)
        assert got["count"][i] == want, (y, x)
    assert (got["count"][xs == 4] == B).all()


def test_perm_test_rejects_a_non_permutation():
    X = np.arange(12, dtype=np.float32).reshape(2, 6)
    bad = np.array([[0, 1, 2, 3, 4, 4]], dtype=np.uint16)
    with pytest.raises(oracle.OracleError):
        oracle.perm_test(X, bad, [0], [1])
