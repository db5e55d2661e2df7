"""Batched form: one plan over many uneven matrices, captured in a hipGraph.

Every matrix's results must equal the plain per-matrix call bit for bit, and
the oracle on each small matrix; graph replays must repeat them exactly."""
import numpy as np
import pytest
import torch

import oracle
from paper_1704_03767_amd import ktau as K
from paper_1704_03767_amd import synth

pytestmark = pytest.mark.gpu
KEYS = ("nc", "nd", "n3", "tau_b", "n1")


def _np(d):
    return {k: v.cpu().numpy() for k, v in d.items() if v is not None}


def _small_batch(count=24, seed=41):
    shapes = synth.batch_shapes(count, seed, m_range=(2, 90), n_range=(2, 700))
    shapes[0] = (2, 2)
    shapes[1] = (90, 4096)
    shapes[2] = (33, 1025)
    return [synth.batch_matrix(s, seed, i) for i, s in enumerate(shapes)]


@pytest.mark.parametrize("use_graph", [True, False])
def test_batch_matches_oracle_and_plain(use_graph, tmp_path):
    mats = _small_batch()
    dev = [torch.from_numpy(X).cuda() for X in mats]
    b = K.KtauBatch(dev, use_graph=use_graph, tune_cache=str(tmp_path / "tune.txt"))
    for rep in range(3):
        b.run()
        assert b.status() == K.KTAU_OK
        got = [_np(o) for o in b.outs]
        for i, X in enumerate(mats):
            want = oracle.allpairs(X, "gse")
            for k in ("nc", "nd", "n3", "n1"):
                assert np.array_equal(got[i][k], want[k]), (rep, i, k, X.shape, b.plan(i))
            assert np.array_equal(got[i]["tau_b"], want["tau_b"], equal_nan=True), (rep, i)
            plain = _np(K.ktau_allpairs(dev[i]))
            for k in KEYS:
                assert np.array_equal(got[i][k], plain[k], equal_nan=True)
    b.close()


def test_batch_with_large_samples():
    # classes of 256-lane schemes next to small ones; the pre-pass and the
    # composite pass are sized by the largest n of the batch
    shapes = [(21, 16384), (3, 9000), (40, 300), (2, 8192), (17, 4097), (9, 17941), (2, 32768),
              (3, 40000), (2, 65536)]
    mats = [synth.batch_matrix(s, 47, i) for i, s in enumerate(shapes)]
    mats[1][1] = np.floor(mats[1][1])                 # a heavily tied row
    mats[1][2] = np.round(mats[1][2])
    dev = [torch.from_numpy(X).cuda() for X in mats]
    b = K.KtauBatch(dev)
    for _ in range(2):
        b.run()
        assert b.status() == K.KTAU_OK
        for i, X in enumerate(mats):
            got = _np(b.outs[i])
            want = oracle.allpairs(X, "gse")
            for k in ("nc", "nd", "n3", "n1"):
                assert np.array_equal(got[k], want[k]), (i, k, X.shape, b.plan(i))
            assert np.array_equal(got["tau_b"], want["tau_b"], equal_nan=True), i
    b.close()


def test_batch_forced_schemes():
    mats = _small_batch(10, 43)
    dev = [torch.from_numpy(X).cuda() for X in mats]
    want = [oracle.allpairs(X, "gse") for X in mats]
    for scheme in ("block_k16", "block_k8", "wave_k64", "sub16_k64", "sub8_k16", "merge_k32",
                   "merge_k64", K.NAIVE_SCHEME_NAME):
        cap = 256 if scheme == K.NAIVE_SCHEME_NAME else K.ktau_scheme_capacity(K.scheme_id(scheme))
        small = [i for i, X in enumerate(mats) if X.shape[1] <= cap]
        b = K.KtauBatch([dev[i] for i in small], force_scheme=scheme, force_q=3)
        b.run()
        assert b.status() == K.KTAU_OK
        for j, i in enumerate(small):
            got = _np(b.outs[j])
            for k in ("nc", "nd", "n3"):
                assert np.array_equal(got[k], want[i][k])
        b.close()


def test_batch_nan_is_reported():
    mats = _small_batch(5, 44)
    mats[3] = mats[3].copy()
    mats[3][0, 0] = np.nan
    b = K.KtauBatch([torch.from_numpy(X).cuda() for X in mats], autotune=False)
    b.run()
    assert b.status() == K.KTAU_ENAN
    b.close()


def test_naive_class_in_batch_and_autotuner(tmp_path):
    # short rows: the autotuner times the naive bit-set count among the
    # candidates of classes up to 256 samples; a batch whose small matrices
    # take it still equals the oracle and the plain calls, graph replays too
    plans = K.ktau_autotune([32, 64, 128], str(tmp_path / "c.txt"))
    assert any(name == K.NAIVE_SCHEME_NAME for name, _ in plans), plans
    rng = np.random.default_rng(48)
    mats = [np.round(rng.standard_normal((m, n)), 1).astype(np.float32)
            for m, n in ((40, 32), (300, 64), (90, 100), (7, 128), (2, 2), (60, 256), (33, 700))]
    mats[1][3] = 1.0                                   # a constant row
    dev = [torch.from_numpy(X).cuda() for X in mats]
    for force in (K.NAIVE_SCHEME_NAME, None):
        keep = [i for i, X in enumerate(mats) if force is None or X.shape[1] <= 256]
        b = K.KtauBatch([dev[i] for i in keep], force_scheme=force,
                        tune_cache=str(tmp_path / "c.txt"))
        for _ in range(2):
            b.run()
            assert b.status() == K.KTAU_OK
            for j, i in enumerate(keep):
                got = _np(b.outs[j])
                want = oracle.allpairs(mats[i], "gse")
                for k in ("nc", "nd", "n3", "n1"):
                    assert np.array_equal(got[k], want[k]), (force, i, k, b.plan(j))
                assert np.array_equal(got["tau_b"], want["tau_b"], equal_nan=True)
        if force is not None:
            assert all(b.plan(j)[0] == K.NAIVE_SCHEME_NAME for j in range(len(keep)))
        b.close()


def test_autotune_cache_roundtrip(tmp_path):
    path = str(tmp_path / "cache.txt")
    plans = K.ktau_autotune([100, 700, 1000, 3000], path)
    for (name, q), n in zip(plans, [100, 700, 1000, 3000]):
        cap = 256 if name == K.NAIVE_SCHEME_NAME else K.ktau_scheme_capacity(K.scheme_id(name))
        assert cap >= n and 1 <= q <= 64
    text = open(path).read().split()
    assert len(text) >= 4 * 4
    assert K.ktau_autotune([100, 700, 1000, 3000], path) == plans


@pytest.mark.slow
def test_uneven_batch_sampled():
    # the full uneven workload (256 matrices), checked on seeded samples
    mats = synth.batch(256, 4)
    dev = [torch.from_numpy(X).cuda() for X in mats]
    b = K.KtauBatch(dev)
    b.run()
    assert b.status() == K.KTAU_OK
    rng = np.random.default_rng(45)
    for i in rng.choice(len(mats), 12, replace=False):
        X = mats[i]
        m = X.shape[0]
        P = m * (m - 1) // 2
        got = _np(b.outs[i])
        J = np.unique(rng.integers(0, P, 300))
        yx = np.array([K.ktau_job_to_pair(m, int(j)) for j in J])
        want = oracle.pairs(X, yx[:, 0], yx[:, 1], "gse")
        for k in ("nc", "nd", "n3"):
            assert np.array_equal(got[k][J], want[k]), (i, k)
        assert np.array_equal(got["tau_b"][J], want["tau_b"], equal_nan=True)
    b.close()


def test_large_matrix_takes_the_tile_launch(tmp_path):
    # a matrix of 8192 rows or more on a network scheme runs as a plain tile
    # launch inside the batch (16 x 16 tiles); its neighbours of the same
    # scheme keep the persistent kernel; all equal the plain calls bit for bit
    shapes = [(8300, 300), (700, 300), (40, 280), (9000, 1000)]
    mats = [synth.batch_matrix(sh, 43, i) for i, sh in enumerate(shapes)]
    dev = [torch.from_numpy(X).cuda() for X in mats]
    b = K.KtauBatch(dev, tune_cache=str(tmp_path / "tune.txt"))
    for _ in range(2):
        b.run()
        assert b.status() == K.KTAU_OK
        for i, Xd in enumerate(dev):
            want = K.ktau_allpairs(Xd)
            got = b.outs[i]
            for k in ("nc", "nd", "n3", "n1"):
                assert torch.equal(got[k], want[k]), (i, k, b.plan(i))
            assert torch.equal(got["tau_b"].isnan(), want["tau_b"].isnan())
            ok = ~want["tau_b"].isnan()
            assert torch.equal(got["tau_b"][ok], want["tau_b"][ok]), (i, b.plan(i))
    b.close()

