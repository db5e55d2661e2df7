"""Permutation test on the GPU against the oracle: for every pair, the number
of permutations of the second row's samples whose |n_c - n_d| is at least
the observed one (bit-exact) and the P-value (1 + count) / (B + 1)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1704_03767_amd import ktau as K
from paper_1704_03767_amd import synth

pytestmark = pytest.mark.gpu


def _run(X, perms, J_begin=-1, J_end=-1):
    Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda()
    Pd = torch.from_numpy(perms.astype(np.int16)).cuda()
    out = K.ktau_perm_test(Xd, Pd, J_begin, J_end)
    return {k: v.cpu().numpy() for k, v in out.items()}


def _want(X, perms, J=None):
    ys, xs = oracle.enumerate_pairs(X.shape[0])
    if J is not None:
        ys, xs = ys[J], xs[J]
    return oracle.perm_test(X, perms, ys, xs)


def _tied_matrix(m, n, seed):
    rng = np.random.default_rng(seed)
    X = np.round(rng.standard_normal((m, n)), 1).astype(np.float32)
    X[0] = rng.integers(0, 3, n)                    # heavy ties
    X[1] = X[2] + np.float32(0.0)                   # equal rows: S_obs is the maximum
    X[3] = np.where(rng.random(n) < 0.1, 0.0, X[3]).astype(np.float32)
    return X


def test_small_matrix_against_the_oracle():
    X = _tied_matrix(24, 300, 61)
    perms = synth.permutations(64, 300, 62)
    got = _run(X, perms)
    want = _want(X, perms)
    assert np.array_equal(got["count"], want["count"])
    assert np.array_equal(got["p"], want["p"])
    # equal rows: no permutation reaches |S_obs| unless it keeps the order
    assert got["count"][K.ktau_pair_to_job(24, 1, 2)] <= 1


@pytest.mark.parametrize("n", [2, 65, 128, 200, 512, 1000, 2048, 3000, 4096, 5000, 17941])
def test_every_scheme_class(n):
    m = 6 if n < 10000 else 4
    X = _tied_matrix(m, n, 70 + n) if n > 4 else np.array(
        [[1, 2], [2, 1], [3, 3], [0, 5], [1, 1], [2, 2]], np.float32)[:m, :n]
    perms = synth.permutations(12, n, 71 + n)
    got = _run(X, perms)
    want = _want(X, perms)
    assert np.array_equal(got["count"], want["count"]), (got["count"], want["count"])
    assert np.array_equal(got["p"], want["p"])


def test_identity_permutations_and_ranges():
    X = _tied_matrix(20, 700, 63)
    ident = np.tile(np.arange(700, dtype=np.uint16), (7, 1))
    got = _run(X, ident)
    assert (got["count"] == 7).all() and (got["p"] == 1.0).all()
    perms = synth.permutations(20, 700, 64)
    full = _run(X, perms)
    part = _run(X, perms, 17, 150)
    assert np.array_equal(part["count"], full["count"][17:150])
    assert np.array_equal(full["count"][17:150], _want(X, perms, np.arange(17, 150))["count"])


def test_tied_and_constant_rows_take_the_lighter_order():
    # heavily tied second rows make the kernel permute the first row by the
    # inverse permutations instead; two constant rows give count = B at once
    rng = np.random.default_rng(68)
    n = 900
    X = np.round(rng.standard_normal((10, n)), 2).astype(np.float32)
    X[1::3] = rng.integers(0, 2, (3, n))            # binary rows after lighter ones
    X[8] = 4.0
    X[9] = -1.0
    perms = synth.permutations(16, n, 69)
    got = _run(X, perms)
    want = _want(X, perms)
    assert np.array_equal(got["count"], want["count"])
    assert got["count"][K.ktau_pair_to_job(10, 8, 9)] == 16


def test_nan_is_reported():
    X = _tied_matrix(6, 200, 72)
    X[4, 17] = np.nan
    with pytest.raises(K.KtauError) as e:
        _run(X, synth.permutations(3, 200, 73))
    assert e.value.status == K.KTAU_ENAN


def test_a_bad_permutation_is_reported():
    X = _tied_matrix(8, 100, 65)
    perms = synth.permutations(3, 100, 66)
    perms[1, 5] = perms[1, 6]
    with pytest.raises(K.KtauError) as e:
        _run(X, perms)
    assert e.value.status == K.KTAU_EINVAL
    perms[1, 5] = 100                              # out of range
    with pytest.raises(K.KtauError):
        _run(X, perms)
    # a good call on a fresh workspace afterwards
    good = synth.permutations(3, 100, 67)
    assert np.array_equal(_run(X, good)["count"], _want(X, good)["count"])

