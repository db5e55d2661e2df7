"""HIP path vs the CPU oracle, element by element, through the C ABI.

Bar: n_c, n_d, n3, n1 bit-exact; tau_B within 1e-15 absolute (identical
integers and the same IEEE formula, so it is expected to be equal); rank
pre-pass outputs bit-exact.  Full-size workloads are checked on seeded samples
of pairs the oracle computes one by one.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1704_03767_amd import ktau as K
from paper_1704_03767_amd import synth

pytestmark = pytest.mark.gpu
TAU_TOL = 1e-15
ALL_SCHEMES = list(range(len(K.ktau_scheme_names())))


def _np(d):
    return {k: v.cpu().numpy() for k, v in d.items() if v is not None}


def _gpu_allpairs(X, **kw):
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    return _np(K.ktau_allpairs(Xd, tau_a=True, **kw))


def _assert_tau(got, want, what="tau_b"):
    assert np.array_equal(np.isnan(got), np.isnan(want)), what
    ok = ~np.isnan(want)
    if ok.any():
        err = np.abs(got[ok] - want[ok]).max()
        assert err <= TAU_TOL, (what, err)


def _assert_same(got, want, slots=None):
    sel = (lambda a: a) if slots is None else (lambda a: a[slots])
    for k in ("nc", "nd", "n3"):
        g, w = sel(got[k]), want[k]
        if not np.array_equal(g, w):
            bad = np.nonzero(g != w)[0]
            raise AssertionError(f"{k} differs at {bad.size} slots, first {bad[:5]}: "
                                 f"got {g[bad[:5]]} want {w[bad[:5]]}")
    _assert_tau(sel(got["tau_b"]), want["tau_b"])
    if "tau_a" in want and "tau_a" in got:
        _assert_tau(sel(got["tau_a"]), want["tau_a"], "tau_a")


def _check_full(X, **kw):
    got = _gpu_allpairs(X, **kw)
    want = oracle.allpairs(X, "gse")
    _assert_same(got, want)
    assert np.array_equal(got["n1"], want["n1"])
    return got


# ------------------------------------------------------------- rank pre-pass


def _oracle_rstart(order, rank):
    srt = np.take_along_axis(rank, order, axis=1)          # dense rank at sorted position
    out = np.empty_like(srt)
    for r in range(srt.shape[0]):
        out[r] = np.searchsorted(srt[r], srt[r], side="left")
    return out


@pytest.mark.parametrize("shape_seed", [(64, 128, 1), (33, 1000, 2), (17, 4096, 3), (5, 2, 4),
                                        (6, 8193, 6), (5, 16384, 7), (4, 16385, 8),
                                        (6, 17941, 9), (3, 32768, 10),
                                        (3, 32769, 11), (4, 40000, 12), (4, 65536, 13),
                                        (9, 65, 5)])
def test_prepass_matches_oracle(shape_seed):
    m, n, seed = shape_seed
    rng = np.random.default_rng(seed)
    X = np.round(rng.standard_normal((m, n)), 1).astype(np.float32)
    X[0, : n // 2] = -0.0
    X[0, n // 2:] = 0.0
    X[1] = 3.0                                             # constant row
    if m > 3:
        X[2] = np.float32(np.inf)
        X[2, ::3] = -np.inf
    got = K.ktau_rank(torch.from_numpy(X).cuda())
    want = oracle.rank_rows(X)
    assert np.array_equal(got["perm"].cpu().numpy(), want["order"])
    assert np.array_equal(got["rank"].cpu().numpy(), want["rank"])
    assert np.array_equal(got["n1"].cpu().numpy(), want["n1"])
    assert np.array_equal(got["rstart"].cpu().numpy(), _oracle_rstart(want["order"], want["rank"]))


# ------------------------------------------------------------ small workload


@pytest.mark.parametrize("scheme", ALL_SCHEMES)
def test_small_workload_every_scheme(scheme):
    X = synth.config_matrix(1)                              # 64 x 128, ties from rounding
    _check_full(X, scheme=scheme)


@pytest.mark.parametrize("q", [1, 3, 8, 16, 64])
def test_small_workload_tile_edges(q):
    X = synth.config_matrix(1)
    _check_full(X, q=q)


def test_small_workload_twice_is_identical():
    X = synth.config_matrix(1)
    a = _gpu_allpairs(X)
    b = _gpu_allpairs(X)
    for k in ("nc", "nd", "n3", "tau_b", "n1"):
        assert np.array_equal(a[k], b[k], equal_nan=True)


# ------------------------------------------------------------ edge shapes


EDGE_N = [2, 3, 63, 64, 65, 127, 128, 129, 255, 256, 257, 511, 512, 513, 1023, 1024, 1025,
          2047, 2048, 2049, 4095, 4096]


def _edge_matrix(m, n, seed):
    rng = np.random.default_rng(seed)
    X = np.round(rng.standard_normal((m, n)), 1).astype(np.float32)
    X[0] = 1.0                                               # constant
    X[1] = rng.integers(0, 2, n).astype(np.float32)          # binary: very many ties
    X[2] = rng.permutation(n).astype(np.float32)             # no ties
    X[3] = -X[2]
    X[4] = X[2]
    X[5] = np.where(rng.random(n) < 0.5, -0.0, 0.0).astype(np.float32)
    X[5, :: 7] = 1.0
    X[6] = rng.integers(0, 3, n).astype(np.float32)
    return X


@pytest.mark.parametrize("n", EDGE_N)
def test_edge_sample_counts(n):
    m = 9
    X = _edge_matrix(m, n, n)
    got = _check_full(X)
    # closed forms on the planted rows (self, negation)
    j = K.ktau_pair_to_job(m, 2, 4)
    assert got["tau_b"][j] == 1.0
    j = K.ktau_pair_to_job(m, 2, 3)
    assert got["tau_b"][j] == -1.0
    for x in range(1, m):
        assert np.isnan(got["tau_b"][K.ktau_pair_to_job(m, 0, x)])


@pytest.mark.parametrize("n", [100, 700, 1024, 1500, 3000, 4096])
def test_block_schemes_on_edges(n):
    X = _edge_matrix(9, n, 7 + n)
    for scheme in ALL_SCHEMES:
        if K.ktau_scheme_capacity(scheme) >= n:
            _check_full(X, scheme=scheme)


def _planted_ties(n, seed):
    """Rows with 0, 1, 2 or 3 tie groups at chosen dense ranks: a short group
    (2 samples), a long one (70, listed after the short runs of its row) and
    one longer than any listed-long run (600), at the minimum, the middle and
    the maximum of the row; pairs of groups in both orders of rank."""
    rng = np.random.default_rng(seed)
    rows = []

    def row(groups):
        x = rng.permutation(n).astype(np.float32) + 1.0      # distinct values 1..n
        idx = rng.permutation(n)
        k = 0
        for size, where in groups:
            size = min(size, n - k)
            if size < 2:
                continue
            val = {"min": 0.0, "mid": n / 2 + 0.5, "max": n + 1.0}[where]
            x[idx[k:k + size]] = val
            k += size
        return x

    rows.append(row([]))
    for size in (2, 70, 600):
        for where in ("min", "mid", "max"):
            rows.append(row([(size, where)]))
    rows.append(row([(2, "max"), (70, "min")]))    # long run first in rank, listed last
    rows.append(row([(70, "max"), (2, "min")]))
    rows.append(row([(600, "mid"), (70, "max")]))
    rows.append(row([(3, "min"), (5, "mid"), (70, "max")]))   # three groups
    z = rng.lognormal(0.0, 1.0, n).astype(np.float32)
    z[rng.random(n) < 0.02] = 0.0                              # a run of zeros
    rows.append(z)
    u = np.round(rng.standard_normal(n), 1).astype(np.float32)  # u-rows with ties
    rows.append(u)
    return np.stack(rows)


@pytest.mark.parametrize("n", [33, 300, 513, 800, 1000, 1024, 2000, 4096])
def test_top_level_from_global_ranks(n):
    """The last merge's count is taken from global ranks when v has at most
    two tie groups (and is empty when the second half is padding): every
    scheme whose network fits, against the oracle."""
    X = _planted_ties(n, 40 + n)
    for scheme in ALL_SCHEMES:
        if K.ktau_scheme_capacity(scheme) >= n and K.scheme_name(scheme).startswith(("sub", "wave", "block")):
            _check_full(X, scheme=scheme)


@pytest.mark.parametrize("n", [4097, 8192, 12289, 17941, 32768])
def test_merge_top_level_from_global_ranks(n):
    """The merge scheme's top merge is taken from global ranks too (rows of v
    with at most two tie groups): planted groups at both merge schemes."""
    X = _planted_ties(n, 70 + n)
    for name in ("merge_k32", "merge_k64"):
        _check_full(X, scheme=K.scheme_id(name))


# Samples beyond 4096 run on 256-lane blocks with 32, 64 or 128 keys per lane;
# beyond 16384 the pre-pass merges in global scratch and every pair counts its
# ties directly.
LARGE_N = [4097, 5000, 8191, 8192, 8193, 12289, 16383, 16384, 16385, 17941, 24000, 32767, 32768]


@pytest.mark.parametrize("n", LARGE_N)
def test_large_sample_counts(n):
    m = 9
    X = _edge_matrix(m, n, 1000 + n)
    got = _check_full(X)
    assert got["tau_b"][K.ktau_pair_to_job(m, 2, 4)] == 1.0
    assert got["tau_b"][K.ktau_pair_to_job(m, 2, 3)] == -1.0
    for scheme in ALL_SCHEMES:
        if K.ktau_scheme_capacity(scheme) >= n:
            _check_full(X, scheme=scheme, q=2)


# Rows longer than 32768 samples: plain 16-bit ranks in the workspace and the
# merge scheme's two passes over the halves of the rank range.
WIDE_N = [32769, 40000, 65535, 65536]


@pytest.mark.parametrize("n", WIDE_N)
def test_wide_sample_counts(n):
    m = 10
    X = _edge_matrix(m, n, 2000 + n)
    X[7] = 5.0                                               # a second constant row
    X[8] = np.round(np.random.default_rng(n).standard_normal(n), 2).astype(np.float32)
    got = _check_full(X)
    assert got["tau_b"][K.ktau_pair_to_job(m, 2, 4)] == 1.0
    assert got["tau_b"][K.ktau_pair_to_job(m, 2, 3)] == -1.0
    j = K.ktau_pair_to_job(m, 0, 7)                          # two constant rows
    assert got["nd"][j] == 0 and got["n3"][j] == n * (n - 1) // 2
    # a job sub-range through the same kernel
    part = _np(K.ktau_allpairs_range(torch.from_numpy(X).cuda(), 5, 31))
    for k in ("nc", "nd", "n3", "tau_b"):
        assert np.array_equal(part[k], got[k][5:31], equal_nan=True), k


@pytest.mark.parametrize("n", [32769, 65536])
def test_wide_rank_halves_closed_forms(n):
    # the counting passes split ranks at 32767 | 32768: pairs of samples on
    # either side of the split, in both orders, against closed forms (a
    # permutation pi of the samples against the identity has n_d = inv(pi))
    base = np.arange(n, dtype=np.float32)
    rows = [base]
    swap = base.copy()
    swap[[32767, 32768]] = swap[[32768, 32767]]              # one inversion at the split
    rows.append(swap)
    rows.append(base[::-1].copy())                            # n0 inversions
    rot = np.roll(base, 1)                                    # n - 1 inversions
    rows.append(rot)
    blk = base.copy()                                         # upper half moved first
    blk = np.concatenate([base[32768:], base[:32768]])
    rows.append(blk)
    X = np.stack(rows)
    got = _gpu_allpairs(X)
    n0 = n * (n - 1) // 2
    hi = n - 32768
    expect = {(0, 1): 1, (0, 2): n0, (0, 3): n - 1, (0, 4): 32768 * hi}
    for (y, x), nd in expect.items():
        j = K.ktau_pair_to_job(len(rows), y, x)
        assert got["nd"][j] == nd, (y, x, got["nd"][j], nd)
        assert got["nc"][j] == n0 - nd and got["n3"][j] == 0
    want = oracle.allpairs(X, "gse")
    _assert_same(got, want)


@pytest.mark.parametrize("scheme", ["merge_k32", "merge_k64"])
@pytest.mark.parametrize("n", [2, 100, 2048, 2049, 4096, 4097, 6143, 8192, 12289, 20000])
def test_merge_schemes_every_chunk_count(scheme, n):
    # one chunk (network only) up to many, each with a ragged last chunk
    cap = K.ktau_scheme_capacity(K.scheme_id(scheme))
    if n > cap:
        pytest.skip("beyond the scheme's capacity")
    X = _edge_matrix(9, n, 3000 + n)
    _check_full(X, scheme=scheme)
    Y = synth.lognormal_blocks(11, n, 70 + n % 5)
    _check_full(Y, scheme=scheme)


@pytest.mark.parametrize("n", [5000, 17941, 32768])
def test_merge_long_tie_runs(n):
    # tie runs around the lengths the merge scheme counts by networks
    # (64 < length <= 512) and by the pairwise walk, in both rows of a pair
    rng = np.random.default_rng(n)
    rows = []
    for lens in ((65, 100, 512, 513, 63, 2, 1000), (64, 300, 65, 7), (511, 512, 128)):
        x = rng.standard_normal(n).astype(np.float32) * 100 + 1000
        pos = rng.permutation(n)
        at = 0
        for lv, ln in enumerate(lens):
            x[pos[at:at + ln]] = np.float32(lv)            # a tie run of length ln
            at += ln
        rows.append(x)
    rows.append(np.round(rng.standard_normal(n), 1).astype(np.float32))   # many long runs
    rows.append(rng.integers(0, 40, n).astype(np.float32))
    rows.append(rng.standard_normal(n).astype(np.float32))
    X = np.stack(rows)
    for scheme in ("merge_k32", "merge_k64"):
        if K.ktau_scheme_capacity(K.scheme_id(scheme)) >= n:
            _check_full(X, scheme=scheme)


@pytest.mark.parametrize("n", [6000, 16384, 17941])
def test_large_gene_expression_tiles(n):
    # several tiles and a ragged tail of rows, rows with 2% exact zeros
    X = synth.lognormal_blocks(37, n, 60 + n % 7)
    _check_full(X)
    _check_full(X, q=5)


def test_large_heavy_tie_paths():
    rng = np.random.default_rng(23)
    for n in (5000, 16384, 20000):
        rows = [rng.integers(0, lv, n).astype(np.float32) for lv in (2, 3, 8, 200, 3000)]
        rows.append(np.where(rng.random(n) < 0.9, 0.0, rng.standard_normal(n)).astype(np.float32))
        rows.append(rng.standard_normal(n).astype(np.float32))
        X = np.stack(rows)
        for scheme in ALL_SCHEMES:
            if K.ktau_scheme_capacity(scheme) >= n:
                _check_full(X, scheme=scheme)


@pytest.mark.parametrize("m", [2, 3, 7, 8, 9, 17])
def test_edge_row_counts(m):
    rng = np.random.default_rng(m)
    X = np.round(rng.standard_normal((m, 300)), 1).astype(np.float32)
    _check_full(X)
    _check_full(X, q=4)


def test_heavy_tie_paths():
    # Pairs where both rows carry ties: a few (direct in-run count) and very
    # many (the literal (u, v) sort), at several n.
    rng = np.random.default_rng(21)
    for n in (128, 300, 1024, 2500):
        rows = []
        for levels in (2, 3, 4, 8, 30, 200):
            rows.append(rng.integers(0, levels, n).astype(np.float32))
        rows.append(np.where(rng.random(n) < 0.9, 0.0, rng.standard_normal(n)).astype(np.float32))
        rows.append(np.where(rng.random(n) < 0.05, 0.0, rng.standard_normal(n)).astype(np.float32))
        X = np.stack(rows)
        for scheme in ALL_SCHEMES:
            if K.ktau_scheme_capacity(scheme) >= n:
                _check_full(X, scheme=scheme)


# ------------------------------------------------------------ job sub-ranges


def test_ranges_equal_full_slices():
    X = synth.config_matrix(1)
    m, n = X.shape
    Xd = torch.from_numpy(X).cuda()
    full = _np(K.ktau_allpairs(Xd))
    P = m * (m - 1) // 2
    for a, b in [(0, P), (0, 1), (5, 6), (100, 1000), (P - 7, P), (1000, 1000)]:
        part = _np(K.ktau_allpairs_range(Xd, a, b))
        for k in ("nc", "nd", "n3", "tau_b"):
            assert np.array_equal(part[k], full[k][a:b], equal_nan=True), (a, b, k)
    for scheme in ALL_SCHEMES:
        part = _np(K.ktau_allpairs_range(Xd, 7, 1500, scheme=scheme))
        for k in ("nc", "nd", "n3", "tau_b"):
            assert np.array_equal(part[k], full[k][7:1500], equal_nan=True)


# ------------------------------------------------------------ errors


def test_nan_input_is_reported():
    X = synth.config_matrix(1).copy()
    X[10, 20] = np.nan
    with pytest.raises(K.KtauError) as e:
        _gpu_allpairs(X)
    assert e.value.status == K.KTAU_ENAN
    # the workspace status is cleared and the next call succeeds
    _check_full(synth.config_matrix(1))


@pytest.mark.parametrize("col", [3, 16384, 19999])
def test_nan_in_a_long_row_is_reported(col):
    # rows over 16384 samples are sorted in two halves: a NaN in either half
    X = synth.samples_matrix(4, 20000, 6)
    X[2, col] = np.nan
    with pytest.raises(K.KtauError) as e:
        _gpu_allpairs(X)
    assert e.value.status == K.KTAU_ENAN


# ------------------------------------------------------------ full-size workloads


def _sampled(cfg, count, seed):
    X = synth.config_matrix(cfg)
    m, n = X.shape
    Xd = torch.from_numpy(X).cuda()
    got = _np(K.ktau_allpairs(Xd))
    del Xd
    P = m * (m - 1) // 2
    rng = np.random.default_rng(seed)
    J = np.unique(np.concatenate([rng.integers(0, P, count), [0, P - 1]]))
    yx = np.array([K.ktau_job_to_pair(m, int(j)) for j in J])
    want = oracle.pairs(X, yx[:, 0], yx[:, 1], "gse")
    _assert_same(got, want, slots=J)
    assert np.array_equal(got["n1"], oracle.rank_rows(X)["n1"])
    # properties at every pair: partition identity and |tau| <= 1
    n0 = n * (n - 1) // 2
    n1 = got["n1"]
    ys, xs = yx[:, 0], yx[:, 1]
    assert np.all(got["nc"][J] + got["nd"][J] + n1[ys] + n1[xs] - got["n3"][J] == n0)
    tb = got["tau_b"]
    assert np.all(np.abs(tb[~np.isnan(tb)]) <= 1.0)
    assert (got["nd"] >= 0).all() and (got["nc"] >= 0).all() and (got["n3"] >= 0).all()
    return got


@pytest.mark.slow
def test_medium_workload_sampled():
    _sampled(2, 20000, 22)


@pytest.mark.slow
def test_gene_expression_scale_sampled():
    _sampled(3, 20000, 33)


@pytest.mark.slow
@pytest.mark.parametrize("shape", ["gene_vs_gene", "sample_vs_sample"])
def test_paper_orientations_sampled(shape):
    # the paper's data in both orientations, as bench.py times them:
    # m = 17941 genes x n = 353 samples, and m = 353 samples x n = 17941 genes
    if shape == "gene_vs_gene":
        X = synth.lognormal_blocks(17941, 353, 7)
    else:
        X = synth.samples_matrix(353, 17941, 6)
    m, n = X.shape
    Xd = torch.from_numpy(X).cuda()
    out = K.ktau_allpairs(Xd)
    P = m * (m - 1) // 2
    rng = np.random.default_rng(44)
    J = np.unique(np.concatenate([rng.integers(0, P, 3000), [0, P - 1]]))
    Jd = torch.from_numpy(J).cuda()
    got = {k: out[k][Jd].cpu().numpy() for k in ("nc", "nd", "n3", "tau_b")}
    yx = np.array([K.ktau_job_to_pair(m, int(j)) for j in J])
    want = oracle.pairs(X, yx[:, 0], yx[:, 1], "gse")
    _assert_same(got, want)
    assert np.array_equal(out["n1"].cpu().numpy(), oracle.rank_rows(X)["n1"])
    tb = out["tau_b"]
    assert bool((tb.abs() <= 1.0).all()) and not bool(tb.isnan().any())


@pytest.mark.slow
def test_gene_expression_scale_batched_equals_plain():
    # the launch configuration bench.py reports as its value: a one-matrix
    # batched plan (autotuned scheme, the tile launch of a matrix of 8192 rows
    # or more, hipGraph), replayed
    # twice; every output equals the plain call's (itself checked against the
    # oracle on samples above)
    X = synth.config_matrix(3)
    Xd = torch.from_numpy(X).cuda()
    plain = K.ktau_allpairs(Xd)
    b = K.KtauBatch([Xd])
    for _ in range(2):
        b.run()
        assert b.status() == K.KTAU_OK
        got = b.outs[0]
        for k in ("nc", "nd", "n3", "n1"):
            assert torch.equal(got[k], plain[k]), k
        assert torch.equal(got["tau_b"].isnan(), plain["tau_b"].isnan())
        ok = ~plain["tau_b"].isnan()
        assert torch.equal(got["tau_b"][ok], plain["tau_b"][ok])
    b.close()
