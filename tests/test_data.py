"""Sanity of the seeded input generators against what their recipes imply.

These are statistical checks of the stand-ins for the paper's gene-expression
matrices, not bit pins: the tau values are computed by the oracle and compared
with closed forms for Gaussian data.
"""
import math

import numpy as np

import oracle
from paper_1704_03767_amd import synth


def _null_sd(n):
    # standard deviation of tau for independent continuous rows of length n
    return math.sqrt(2 * (2 * n + 5) / (9 * n * (n - 1)))


def test_shapes_seeds_and_determinism():
    for cfg, (m, n) in synth.SHAPES.items():
        if cfg == 3:
            X = synth.lognormal_blocks(128, n, synth.DEFAULT_SEEDS[3])
            assert X.shape == (128, n)
        else:
            X = synth.config_matrix(cfg)
            assert X.shape == (m, n)
        assert X.dtype == np.float32 and np.isfinite(X).all()
    a = synth.config_matrix(1)
    assert synth.sha256(a) == synth.sha256(synth.config_matrix(1))
    assert synth.sha256(a) != synth.sha256(synth.config_matrix(1, seed=7))
    # the first rows of the big matrix do not depend on how many rows are drawn
    assert np.array_equal(synth.lognormal_blocks(128, 64, 3), synth.lognormal_blocks(256, 64, 3)[:128])


def test_gene_expression_blocks_have_the_stated_correlation():
    n, block, rho, p = 1024, 64, 0.6, 0.02
    X = synth.lognormal_blocks(8 * block, n, 3, block=block, rho=rho, zero_frac=p)
    assert abs((X == 0).mean() - p) < 0.002
    assert (X >= 0).all()
    res = oracle.allpairs(X)
    ys, xs = oracle.enumerate_pairs(X.shape[0])
    same = ys // block == xs // block
    tau = res["tau_b"]
    # Gaussian copula: tau = (2/pi) asin(rho); exp() keeps it; a zero in either
    # sample of a pair makes its sign independent of the other row, so the
    # expected numerator shrinks by (1 - p)^4
    want = (2 / math.pi) * math.asin(rho) * (1 - p) ** 4
    assert abs(tau[same].mean() - want) < 0.01, (tau[same].mean(), want)
    assert abs(tau[~same].mean()) < 0.005
    assert 0.85 < tau[~same].std() / _null_sd(n) < 1.1


def test_sample_orientation_correlations():
    # rows = samples over shared genes: log-expression correlation is
    # (gene + group variance) / total within a group and gene / total across
    # groups; the Gaussian-copula closed form and the zero shrinkage as above
    X = synth.samples_matrix(24, 17941, 6)
    assert X.shape == (24, 17941) and abs((X == 0).mean() - 0.02) < 0.001
    res = oracle.allpairs(X)
    ys, xs = oracle.enumerate_pairs(24)
    same = ys % 4 == xs % 4
    g2, c2, e2 = 1.5 ** 2, 0.5 ** 2, 0.5 ** 2
    shrink = (1 - 0.02) ** 4
    for sel, rho in ((same, (g2 + c2) / (g2 + c2 + e2)), (~same, g2 / (g2 + c2 + e2))):
        want = (2 / math.pi) * math.asin(rho) * shrink
        assert abs(res["tau_b"][sel].mean() - want) < 0.01, (res["tau_b"][sel].mean(), want)


def test_medium_workload_quantised_rows():
    X = synth.config_matrix(2)
    m, n = X.shape
    distinct = np.array([np.unique(r).size for r in X])
    quant = distinct <= 16
    assert quant.sum() == round(0.10 * m)
    q = X[quant]
    assert (q == np.round(q)).all() and q.min() == 0 and q.max() == 15
    assert (distinct[~quant] > n // 2).all()


def test_small_workload_is_rounded_to_tenths():
    X = synth.config_matrix(1).astype(np.float64)
    assert np.allclose(X * 10, np.round(X * 10), atol=1e-4)
    assert np.array([np.unique(r).size for r in X]).max() < X.shape[1]


def test_uneven_batch_shapes_and_grid():
    shapes = synth.batch_shapes()
    assert len(shapes) == 256
    ms = np.array([s[0] for s in shapes])
    ns = np.array([s[1] for s in shapes])
    assert ms.min() >= 32 and ms.max() <= 2048 and ns.min() >= 64 and ns.max() <= 4096
    assert abs(ms.mean() - 1040) < 120 and abs(ns.mean() - 2080) < 240
    A = synth.batch_matrix(shapes[0], 4, 0).astype(np.float64)
    on_grid = np.isclose(A * 4, np.round(A * 4))
    assert abs(on_grid.mean() - 0.2) < 0.02


def test_queries_hit_the_database_about_half_the_time():
    db = synth.database(m=2000, n=800, seed=5)
    Q = synth.queries(db, 40, seed=6)
    top = oracle.query_topk(db.X, Q, 1)["tau"][:, 0]
    # a query built from a database row's latent normal plus N(0, 0.25) noise
    # correlates with it at rho = 1/sqrt(1.25): tau = (2/pi) asin(rho) ~ 0.70
    hits = np.abs(top) > 0.5
    assert 10 <= hits.sum() <= 30
    want = (2 / math.pi) * math.asin(1 / math.sqrt(1.25))
    assert abs(np.abs(top[hits]).mean() - want) < 0.03
    assert np.abs(top[~hits]).max() < 0.2


def test_poisson_arrivals():
    t, nq = synth.poisson_requests(4000, rate=500.0, seed=7)
    gaps = np.diff(t)
    assert abs(gaps.mean() - 1 / 500.0) < 0.1 / 500.0
    assert nq.min() >= 1 and nq.max() <= 64
    assert t[0] == 0 and (gaps >= 0).all()
