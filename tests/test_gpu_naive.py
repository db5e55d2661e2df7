"""The naive bit-set count (every sample pair compared, stored per row as bit
sets) against the CPU oracle and against the network schemes, through the C
ABI.  Bar: n_c, n_d, n3, n1 bit-exact; tau_B and tau_A within 1e-15 (the same
integers and the same formula give the same doubles)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1704_03767_amd import ktau as K
from paper_1704_03767_amd import synth

pytestmark = pytest.mark.gpu
TAU_TOL = 1e-15
NAIVE = K.NAIVE_SCHEME_NAME


def _np(d):
    return {k: v.cpu().numpy() for k, v in d.items() if v is not None}


def _run(X, **kw):
    Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda()
    return _np(K.ktau_allpairs(Xd, tau_a=True, **kw))


def _assert_tau(got, want, what):
    assert np.array_equal(np.isnan(got), np.isnan(want)), what
    ok = ~np.isnan(want)
    if ok.any():
        assert np.abs(got[ok] - want[ok]).max() <= TAU_TOL, what


def _assert_same(got, want, slots=None):
    sel = (lambda a: a) if slots is None else (lambda a: a[slots])
    for k in ("nc", "nd", "n3"):
        g, w = sel(got[k]), want[k]
        if not np.array_equal(g, w):
            bad = np.nonzero(g != w)[0]
            raise AssertionError(f"{k} differs at {bad.size} slots, first {bad[:5]}: "
                                 f"got {g[bad[:5]]} want {w[bad[:5]]}")
    _assert_tau(sel(got["tau_b"]), want["tau_b"], "tau_b")
    if "tau_a" in want:
        _assert_tau(sel(got["tau_a"]), want["tau_a"], "tau_a")


def _planted(m, n, seed):
    """Rounded normals (ties) with planted rows: constant, binary, a
    permutation (no ties), its negation and a copy, signed zeros, three
    levels."""
    rng = np.random.default_rng(seed)
    X = np.round(rng.standard_normal((m, n)), 1).astype(np.float32)
    X[0] = 1.0
    X[1] = rng.integers(0, 2, n).astype(np.float32)
    X[2] = rng.permutation(n).astype(np.float32)
    X[3] = -X[2]
    X[4] = X[2]
    X[5] = np.where(rng.random(n) < 0.5, -0.0, 0.0).astype(np.float32)
    X[5, ::7] = 1.0
    X[6] = rng.integers(0, 3, n).astype(np.float32)
    return X


# Every word count (1, 2, 4, 8 words per set) with full, ragged and
# single-bit last words; 37 rows are few pairs, so the job-order kernel runs
# (the tile kernel is checked on 1460-1500 rows below).
NAIVE_N = [2, 3, 31, 32, 33, 63, 64, 65, 100, 127, 128, 129, 200, 255, 256]


@pytest.mark.parametrize("n", NAIVE_N)
def test_naive_matches_oracle(n):
    m = 37
    X = _planted(m, n, 300 + n)
    got = _run(X, scheme=NAIVE)
    want = oracle.allpairs(X, "gse")
    _assert_same(got, want)
    assert np.array_equal(got["n1"], want["n1"])
    if n > 2:
        assert got["tau_b"][K.ktau_pair_to_job(m, 2, 4)] == 1.0
        assert got["tau_b"][K.ktau_pair_to_job(m, 2, 3)] == -1.0
    for x in range(1, m):
        assert np.isnan(got["tau_b"][K.ktau_pair_to_job(m, 0, x)])


@pytest.mark.parametrize("n", [64, 128, 200, 256])
def test_naive_equals_network_bit_for_bit(n):
    X = synth.gaussian_rounded(150, n, 40 + n)
    a = _run(X, scheme=NAIVE)
    b = _run(X, scheme=K.ktau_default_scheme(n))   # the network's default scheme
    for k in ("nc", "nd", "n3", "tau_b", "tau_a", "n1"):
        assert np.array_equal(a[k], b[k], equal_nan=True), k


def test_naive_tile_edges():
    # 1500 rows (1,124,250 pairs): above the job-order cut-off of 2^20 pairs,
    # so the tile kernel runs; a ragged last tile for every edge
    X = synth.gaussian_rounded(1500, 100, 8)
    want = oracle.allpairs(X, "gse")
    for q in (1, 5, 16, 64):
        _assert_same(_run(X, scheme=NAIVE, q=q), want)


@pytest.mark.parametrize("n", [32, 64, 128, 256])
def test_naive_tiles_every_width(n):
    # the tile kernel at each set width (1, 2, 4, 8 words), full oracle check
    X = _planted(1460, n, 900 + n)
    _assert_same(_run(X, scheme=NAIVE), oracle.allpairs(X, "gse"))


@pytest.mark.parametrize("m", [2, 3, 17, 33])
def test_naive_row_counts(m):
    X = synth.gaussian_rounded(m, 77, m)
    _assert_same(_run(X, scheme=NAIVE), oracle.allpairs(X, "gse"))


def test_naive_heavy_ties():
    # joint ties at every level count, including rows tied almost everywhere
    rng = np.random.default_rng(22)
    for n in (40, 128, 256):
        rows = [rng.integers(0, lv, n).astype(np.float32) for lv in (2, 3, 4, 8, 30)]
        rows.append(np.where(rng.random(n) < 0.9, 0.0, rng.standard_normal(n)).astype(np.float32))
        rows.append(rng.standard_normal(n).astype(np.float32))
        X = np.stack(rows)
        _assert_same(_run(X, scheme=NAIVE), oracle.allpairs(X, "gse"))


def test_naive_ranges_equal_full_slices():
    X = synth.config_matrix(1)
    m = X.shape[0]
    Xd = torch.from_numpy(X).cuda()
    full = _np(K.ktau_allpairs(Xd, scheme=NAIVE))
    P = m * (m - 1) // 2
    for a, b in [(0, P), (0, 1), (5, 6), (100, 1000), (P - 7, P), (1000, 1000)]:
        part = _np(K.ktau_allpairs_range(Xd, a, b, scheme=NAIVE))
        for k in ("nc", "nd", "n3", "tau_b"):
            assert np.array_equal(part[k], full[k][a:b], equal_nan=True), (a, b, k)


def test_naive_prepare_then_pairs():
    # the two halves: one pre-pass, then the naive pass and a network pass
    X = synth.gaussian_rounded(90, 160, 5)
    m, n = X.shape
    Xd = torch.from_numpy(X).cuda()
    ws = K.alloc_workspace(m, n, Xd.device)
    K.ktau_prepare(Xd, ws)
    P = m * (m - 1) // 2
    outs = []
    for scheme in (NAIVE, K.ktau_default_scheme(n)):
        out = K.alloc_outputs(P, m, Xd.device, tau_a=True)
        K.ktau_pairs(m, n, out, ws, scheme=scheme)
        outs.append(_np(out))
    assert K.ktau_status(ws) == K.KTAU_OK
    want = oracle.allpairs(X, "gse")
    _assert_same(outs[0], want)
    for k in ("nc", "nd", "n3", "tau_b"):
        assert np.array_equal(outs[0][k], outs[1][k], equal_nan=True), k


def test_naive_sampled_at_scale():
    # 4096 rows of 256 log-normal samples (blocks of 64 rows, 2% zeros):
    # 8,386,560 pairs, 20,000 of them checked one by one
    X = synth.lognormal_blocks(4096, 256, 12)
    m = X.shape[0]
    got = _run(X, scheme=NAIVE)
    rng = np.random.default_rng(13)
    J = np.unique(rng.integers(0, m * (m - 1) // 2, 20000))
    yx = np.array([K.ktau_job_to_pair(m, int(j)) for j in J])
    want = oracle.pairs(X, yx[:, 0], yx[:, 1], "gse")
    _assert_same(got, want, slots=J)


def test_naive_nan_is_reported():
    X = synth.config_matrix(1).copy()
    X[10, 20] = np.nan
    with pytest.raises(K.KtauError) as e:
        _run(X, scheme=NAIVE)
    assert e.value.status == K.KTAU_ENAN
    _assert_same(_run(synth.config_matrix(1), scheme=NAIVE),
                 oracle.allpairs(synth.config_matrix(1), "gse"))


def test_naive_random_shapes_equal_network():
    # seeded shapes across both kernels (job order below 2^20 pairs, tiles
    # above) and every set width, with a mix of tie structures per row;
    # every output compared with a network scheme, 500 pairs with the oracle
    rng = np.random.default_rng(77)
    for t in range(12):
        m = int(rng.integers(2, 2200))
        n = int(rng.integers(2, 257))
        X = rng.standard_normal((m, n)).astype(np.float32)
        kind = rng.integers(0, 4, m)
        X[kind == 1] = np.round(X[kind == 1], 1)
        X[kind == 2] = rng.integers(0, 3, (int((kind == 2).sum()), n)).astype(np.float32)
        X[kind == 3] = np.where(rng.random((int((kind == 3).sum()), n)) < 0.1, 0.0,
                                X[kind == 3]).astype(np.float32)
        a = _run(X, scheme=NAIVE)
        b = _run(X, scheme=K.ktau_default_scheme(n))
        for k in ("nc", "nd", "n3", "tau_b", "tau_a", "n1"):
            assert np.array_equal(a[k], b[k], equal_nan=True), (t, m, n, k)
        P = m * (m - 1) // 2
        J = np.unique(rng.integers(0, P, min(P, 500)))
        yx = np.array([K.ktau_job_to_pair(m, int(j)) for j in J])
        _assert_same(a, oracle.pairs(X, yx[:, 0], yx[:, 1], "gse"), slots=J)


@pytest.mark.parametrize("scheme", [NAIVE, "network"])
def test_tau_a_only_outputs(scheme):
    # tau_A alone (every other output NULL), as the naive kernel of the paper
    # computes it; the kernels skip the NULL arrays
    X = synth.gaussian_rounded(200, 128, 31)
    m, n = X.shape
    P = m * (m - 1) // 2
    Xd = torch.from_numpy(X).cuda()
    out = {"tau_a": torch.full((P,), -7.0, dtype=torch.float64, device=Xd.device)}
    ws = K.alloc_workspace(m, n, Xd.device)
    s = NAIVE if scheme == NAIVE else K.ktau_default_scheme(n)
    K.ktau_allpairs_ex(Xd, -1, -1, out, ws, s, 0)
    assert K.ktau_status(ws) == K.KTAU_OK
    want = oracle.allpairs(X, "gse")
    _assert_tau(out["tau_a"].cpu().numpy(), want["tau_a"], "tau_a")
