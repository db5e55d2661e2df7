"""Query-vs-database search and the continuous-batching server.

Top-k results must equal the oracle's full sort under the tie rule (|tau|
descending, row ascending, NaN excluded, -1 padding); every request's results
must be identical alone and in a mix of concurrent requests; admission under a
tiny memory budget must still serve everything correctly; a forced launch
failure and a cancellation affect only their own request."""
import numpy as np
import pytest
import torch

import oracle
from paper_1704_03767_amd import ktau as K
from paper_1704_03767_amd import serve as S
from paper_1704_03767_amd import synth

pytestmark = pytest.mark.gpu


def _db(m=600, n=800, seed=51):
    d = synth.database(m, n, seed)
    X = d.X.copy()
    X[7] = 2.0                                  # constant row: NaN tau, never returned
    X[20] = X[10]                               # equal |tau| -> smaller row first
    X[30] = np.round(X[30] * 2) / 2             # tied rows
    X[31] = np.where(np.arange(n) % 3 == 0, 1.0, X[31]).astype(np.float32)
    d.X = X
    return d


def _queries(db, count, seed):
    Q = synth.queries(db, count, seed)
    Q[0] = db.X[10]
    if count > 2:
        Q[2] = np.round(Q[2] * 4) / 4               # a heavily tied query row
    return Q


def _check_topk(got, want):
    assert np.array_equal(got["idx"], want["idx"])
    gt, wt = got["tau"], want["tau"]
    assert np.array_equal(np.isnan(gt), np.isnan(wt))
    ok = ~np.isnan(wt)
    assert np.abs(gt[ok] - wt[ok]).max(initial=0) <= 1e-15
    assert np.array_equal(got["nd"], want["nd"])


@pytest.mark.parametrize("k", [1, 17, 100])
def test_query_matches_oracle(k):
    db = _db()
    Q = _queries(db, 5, 52)
    kdb = S.KtauDb(torch.from_numpy(db.X).cuda())
    got = {a: b.cpu().numpy() for a, b in S.ktau_query(kdb, torch.from_numpy(Q).cuda(), k).items()}
    _check_topk(got, oracle.query_topk(db.X, Q, k))
    kdb.close()


def test_query_every_scheme():
    db = _db(m=500, n=300, seed=56)
    Q = _queries(db, 3, 57)
    Q[0, :40] = 0.0                                          # ties on the query side
    want = oracle.query_topk(db.X, Q, 20)
    for s, name in enumerate(K.ktau_scheme_names()):
        if K.ktau_scheme_capacity(s) < db.X.shape[1] or name.startswith("merge"):
            continue
        kdb = S.KtauDb(torch.from_numpy(db.X).cuda(), scheme=s)
        got = {a: b.cpu().numpy()
               for a, b in S.ktau_query(kdb, torch.from_numpy(Q).cuda(), 20).items()}
        _check_topk(got, want)
        kdb.close()


@pytest.mark.parametrize("n,forced", [(64, None), (100, None), (128, "naive_bits"),
                                      (200, "naive_bits"), (256, "naive_bits")])
def test_query_naive_bits_scheme(n, forced):
    # short rows: the database's bit sets (the default up to 128 samples)
    db = _db(m=700, n=n, seed=60 + n)
    Q = _queries(db, 5, 61)
    Q[1, : n // 3] = 0.0                                     # ties on the query side
    Q[2] = np.round(Q[2], 1)
    kdb = S.KtauDb(torch.from_numpy(db.X).cuda(), scheme=forced)
    got = {a: b.cpu().numpy() for a, b in S.ktau_query(kdb, torch.from_numpy(Q).cuda(), 40).items()}
    _check_topk(got, oracle.query_topk(db.X, Q, 40))
    kdb.close()
    # heavily tied rows on both sides
    rng = np.random.default_rng(n)
    X = rng.integers(0, 3, (300, n)).astype(np.float32)
    X[::5] = rng.standard_normal((60, n)).astype(np.float32)
    Qt = rng.integers(0, 2, (4, n)).astype(np.float32)
    kdb = S.KtauDb(torch.from_numpy(X).cuda(), scheme=forced)
    got = {a: b.cpu().numpy() for a, b in S.ktau_query(kdb, torch.from_numpy(Qt).cuda(), 50).items()}
    _check_topk(got, oracle.query_topk(X, Qt, 50))
    kdb.close()


@pytest.mark.parametrize("n", [8192, 16384, 24000])
def test_query_large_samples(n):
    db = _db(m=120, n=n, seed=58)
    Q = _queries(db, 3, 59)
    kdb = S.KtauDb(torch.from_numpy(db.X).cuda())
    got = {a: b.cpu().numpy() for a, b in S.ktau_query(kdb, torch.from_numpy(Q).cuda(), 30).items()}
    _check_topk(got, oracle.query_topk(db.X, Q, 30))
    kdb.close()


def test_query_pads_when_k_exceeds_rows():
    db = _db(m=40, n=300, seed=53)
    Q = _queries(db, 3, 54)
    kdb = S.KtauDb(torch.from_numpy(db.X).cuda())
    got = {a: b.cpu().numpy() for a, b in S.ktau_query(kdb, torch.from_numpy(Q).cuda(), 64).items()}
    want = oracle.query_topk(db.X, Q, 64)
    _check_topk(got, want)
    assert (got["idx"][:, 39:] == -1).all()
    kdb.close()


def test_query_heavy_ties_both_sides():
    rng = np.random.default_rng(55)
    n = 256
    X = rng.integers(0, 3, (300, n)).astype(np.float32)        # every row heavily tied
    X[::5] = rng.standard_normal((60, n)).astype(np.float32)
    Q = rng.integers(0, 2, (4, n)).astype(np.float32)
    kdb = S.KtauDb(torch.from_numpy(X).cuda())
    got = {a: b.cpu().numpy() for a, b in S.ktau_query(kdb, torch.from_numpy(Q).cuda(), 50).items()}
    _check_topk(got, oracle.query_topk(X, Q, 50))
    kdb.close()


def _serve_requests(db, Q, sizes, k, concurrent, **cfg):
    kdb = S.KtauDb(torch.from_numpy(db.X).cuda())
    srv = S.KtauServer(kdb, **cfg)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    out = []
    if concurrent:
        # queued together while admission is paused, so that they merge
        srv.pause(True)
        tickets = [srv.submit(Q[offs[i]:offs[i + 1]], k) for i in range(len(sizes))]
        srv.pause(False)
        for t in tickets:
            st, res, lat = srv.wait(t)
            assert st == K.KTAU_OK
            out.append(res)
    else:
        for i in range(len(sizes)):
            st, res, lat = srv.wait(srv.submit(Q[offs[i]:offs[i + 1]], k))
            assert st == K.KTAU_OK and lat["batch_requests"] == 1
            out.append(res)
    stats = srv.stats()
    srv.close()
    kdb.close()
    return out, stats


@pytest.mark.parametrize("k", [1, 29, 45, 250, 400])
def test_topk_cut_inside_equal_keys(k):
    """Selection where the k-th result falls inside a group of equal |tau|:
    10 distinct rows, each repeated 30 times (equal tau for every copy), 20
    constant rows (NaN, never returned), so that the first k in row order of
    the boundary group are taken and k = 400 leaves padding."""
    rng = np.random.default_rng(81)
    n = 300
    base = rng.standard_normal((10, n)).astype(np.float32)
    X = np.repeat(base, 30, axis=0)[rng.permutation(300)]
    X = np.concatenate([X, np.full((20, n), 3.0, np.float32)])[rng.permutation(320)]
    X = np.ascontiguousarray(X)
    Q = np.ascontiguousarray(rng.standard_normal((6, n)).astype(np.float32))
    Q[1] = base[3]
    kdb = S.KtauDb(torch.from_numpy(X).cuda())
    got = {a: b.cpu().numpy() for a, b in S.ktau_query(kdb, torch.from_numpy(Q).cuda(), k).items()}
    _check_topk(got, oracle.query_topk(X, Q, k))


def test_server_merges_different_k():
    # requests with different k merge into one launch of the largest k; each
    # keeps the first k of its rows (a prefix of the longer list)
    db = _db(m=700, n=500, seed=62)
    Q = _queries(db, 9, 63)
    kdb = S.KtauDb(torch.from_numpy(db.X).cuda())
    srv = S.KtauServer(kdb)
    ks = [(Q[0:2], 10), (Q[2:5], 100), (Q[5:6], 1), (Q[6:9], 37)]
    srv.pause(True)
    tickets = [srv.submit(q, k) for q, k in ks]
    srv.pause(False)
    merged = 0
    for t, (q, k) in zip(tickets, ks):
        st, res, lat = srv.wait(t)
        assert st == K.KTAU_OK
        merged = max(merged, lat["batch_requests"])
        assert res["idx"].shape == (q.shape[0], k)
        _check_topk(res, oracle.query_topk(db.X, q, k))
    assert merged == len(ks)
    srv.close()
    kdb.close()


def test_server_alone_equals_mix_equals_oracle():
    db = _db(m=900, n=800, seed=56)
    sizes = [1, 5, 3, 12, 1, 7, 2, 30, 4, 1, 9, 2]
    Q = _queries(db, sum(sizes), 57)
    alone, _ = _serve_requests(db, Q, sizes, 100, False)
    mix, stats = _serve_requests(db, Q, sizes, 100, True, max_batch_queries=24)
    assert stats["merged_requests"] > 0                        # requests were batched
    offs = np.concatenate([[0], np.cumsum(sizes)])
    for i in range(len(sizes)):
        for key in ("idx", "tau", "nd"):
            assert np.array_equal(alone[i][key], mix[i][key], equal_nan=True), (i, key)
    want = oracle.query_topk(db.X, Q, 100)
    for i in range(len(sizes)):
        sl = slice(offs[i], offs[i + 1])
        _check_topk(mix[i], {a: b[sl] for a, b in want.items()})


def test_server_tiny_budget_queues_and_serves():
    db = _db(m=300, n=200, seed=58)
    Q = _queries(db, 30, 59)
    kdb = S.KtauDb(torch.from_numpy(db.X).cuda())
    probe = S.KtauServer(kdb, mem_budget_bytes=1 << 24)
    one = probe.launch_bytes(3, 10)
    probe.close()
    budget = 2 * one + 256                   # room for two 3-row launches, never three
    srv = S.KtauServer(kdb, slots=4, max_batch_queries=3, mem_budget_bytes=budget)
    tickets = [srv.submit(Q[3 * i:3 * i + 3], 10) for i in range(10)]
    res = [srv.wait(t) for t in tickets]
    st = srv.stats()
    srv.close()
    assert all(r[0] == K.KTAU_OK for r in res)
    assert st["peak_pool_bytes"] <= budget
    assert st["peak_running"] <= 2           # memory, not the 4 slots, bounded concurrency
    want = oracle.query_topk(db.X, Q, 10)
    for i, (_, got, _) in enumerate(res):
        _check_topk(got, {a: b[3 * i:3 * i + 3] for a, b in want.items()})
    # a request that can never fit is refused at submission
    srv = S.KtauServer(kdb, mem_budget_bytes=budget)
    with pytest.raises(K.KtauError) as e:
        srv.submit(Q[:30], 10)
    assert e.value.status == K.KTAU_ENOMEM
    srv.close()
    kdb.close()


def test_server_failure_and_cancel_are_isolated():
    db = _db(m=500, n=400, seed=60)
    Q = _queries(db, 40, 61)
    kdb = S.KtauDb(torch.from_numpy(db.X).cuda())
    srv = S.KtauServer(kdb, slots=1, max_batch_queries=8)
    tickets = [srv.submit(Q[4 * i:4 * i + 4], 20) for i in range(10)]
    # later requests are still queued behind the single slot
    fail_rc = srv.inject_failure(tickets[6])
    cancel_rc = srv.cancel(tickets[8])
    results = [srv.wait(t) for t in tickets]
    srv.close()
    want = oracle.query_topk(db.X, Q, 20)
    for i, (st, got, _) in enumerate(results):
        if i == 6 and fail_rc == K.KTAU_OK:
            assert st == K.KTAU_ECANCELED
        elif i == 8 and cancel_rc == K.KTAU_OK:
            assert st == K.KTAU_ECANCELED
        else:
            assert st == K.KTAU_OK
            _check_topk(got, {a: b[4 * i:4 * i + 4] for a, b in want.items()})
    assert fail_rc == K.KTAU_OK or cancel_rc == K.KTAU_OK
    kdb.close()


def test_server_rejects_nan_and_bad_k():
    db = _db(m=100, n=64, seed=62)
    kdb = S.KtauDb(torch.from_numpy(db.X).cuda())
    srv = S.KtauServer(kdb, k_max=50)
    q = db.X[:2].copy()
    q[1, 3] = np.nan
    with pytest.raises(K.KtauError) as e:
        srv.submit(q, 5)
    assert e.value.status == K.KTAU_ENAN
    with pytest.raises(K.KtauError) as e:
        srv.submit(db.X[:1], 51)
    assert e.value.status == K.KTAU_ERANGE
    srv.close()
    kdb.close()


@pytest.mark.slow
def test_query_full_size_database():
    # the serving workload's database (20000 x 800) and k = 100, against the
    # oracle's full sort for a few queries
    db = synth.database(20000, 800, 5)
    Q = synth.queries(db, 4, 61)
    kdb = S.KtauDb(torch.from_numpy(db.X).cuda())
    got = {a: b.cpu().numpy() for a, b in S.ktau_query(kdb, torch.from_numpy(Q).cuda(), 100).items()}
    _check_topk(got, oracle.query_topk(db.X, Q, 100))
    kdb.close()


@pytest.mark.slow
def test_server_full_size_200_requests():
    # the serving workload's database (20000 x 800): 200 seeded requests of one
    # query row each (half near a database row), k = 100, queued together so
    # that they merge, each against the oracle's full sort of its 20000 taus
    db = synth.database(20000, 800, 5)
    Q = synth.queries(db, 200, 64)
    kdb = S.KtauDb(torch.from_numpy(db.X).cuda())
    srv = S.KtauServer(kdb)
    srv.pause(True)
    tickets = [srv.submit(Q[i:i + 1], 100) for i in range(200)]
    srv.pause(False)
    got = {"idx": [], "tau": [], "nd": []}
    for t in tickets:
        st, res, _ = srv.wait(t)
        assert st == K.KTAU_OK
        for key in got:
            got[key].append(res[key])
    stats = srv.stats()
    srv.close()
    kdb.close()
    assert stats["merged_requests"] > 0
    _check_topk({k: np.concatenate(v) for k, v in got.items()}, oracle.query_topk(db.X, Q, 100))
