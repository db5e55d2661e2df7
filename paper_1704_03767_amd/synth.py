"""Seeded synthetic inputs shaped like the paper's gene-expression workloads.

This module only draws random numbers; it holds none of the tau arithmetic.
The HIP library and the CPU oracle both consume what it returns.  The paper
measured four GPL570 expression matrices (17,941 genes x 310-353 samples, log
scale, with ties); those datasets are not available here, so these generators
stand in for them with the same character: log-normal values, correlated gene
blocks, exact-zero and quantised ties.

All draws use numpy's PCG64 ``default_rng(seed)`` in float64 and are cast to
float32 at the end.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass

import numpy as np

# (m, n) of the single-matrix workloads.
SHAPES = {1: (64, 128), 2: (4096, 512), 3: (16384, 1024)}
DEFAULT_SEEDS = {1: 1, 2: 2, 3: 3, 4: 4, 5: 5}


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def gaussian_rounded(m: int, n: int, seed: int, decimals: int = 1) -> np.ndarray:
    """N(0,1) rounded to ``decimals`` places so that ties occur (small case)."""
    rng = np.random.default_rng(seed)
    return np.round(rng.standard_normal((m, n)), decimals).astype(np.float32)


def latent_factor(m: int, n: int, seed: int, factors: int = 8, noise_sd: float = 0.5,
                  quant_frac: float = 0.10, levels: int = 16) -> np.ndarray:
    """X = L F + E with L (m x f), F (f x n) ~ N(0,1), E ~ N(0, sd^2).

    A seeded ``quant_frac`` of the rows is replaced by its level index on
    ``levels`` equal-width bins over that row's [min, max] (heavy ties)."""
    rng = np.random.default_rng(seed)
    L = rng.standard_normal((m, factors))
    F = rng.standard_normal((factors, n))
    X = L @ F + noise_sd * rng.standard_normal((m, n))
    nq = int(round(quant_frac * m))
    rows = np.sort(rng.choice(m, size=nq, replace=False))
    for r in rows:
        x = X[r]
        lo, hi = x.min(), x.max()
        lvl = np.floor(levels * (x - lo) / (hi - lo))
        X[r] = np.minimum(levels - 1, lvl)
    return X.astype(np.float32)


def lognormal_blocks(m: int, n: int, seed: int, block: int = 64, rho: float = 0.6,
                     zero_frac: float = 0.02) -> np.ndarray:
    """Log-normal (mu 0, sigma 1) rows in blocks of ``block`` rows whose
    normal-scale correlation is ``rho``; a Bernoulli(``zero_frac``) mask sets
    entries to an exact 0.0 (a tie run at the bottom of every row)."""
    rng = np.random.default_rng(seed)
    X = np.empty((m, n), np.float32)
    a, b = np.sqrt(rho), np.sqrt(1.0 - rho)
    for r0 in range(0, m, block):
        r1 = min(m, r0 + block)
        G = rng.standard_normal(n)
        E = rng.standard_normal((r1 - r0, n))
        Z = a * G[None, :] + b * E
        blk = np.exp(Z)
        mask = rng.random((r1 - r0, n)) < zero_frac
        blk[mask] = 0.0
        X[r0:r1] = blk.astype(np.float32)
    return X


def samples_matrix(m: int = 353, n: int = 17941, seed: int = 6, groups: int = 4,
                   gene_sd: float = 1.5, group_sd: float = 0.5, noise_sd: float = 0.5,
                   zero_frac: float = 0.02) -> np.ndarray:
    """Sample-vs-sample orientation (rows = samples, columns = genes): log
    expression = a per-gene level shared by every sample, N(0, gene_sd^2),
    plus a per-(group, gene) offset, N(0, group_sd^2), for the sample's group
    (sample s is in group s mod groups), plus noise, N(0, noise_sd^2); X is its
    exponential with a Bernoulli(zero_frac) subset of entries set to exactly 0
    (dropouts).  Rows are strongly and unevenly correlated, as samples over
    shared genes are."""
    rng = np.random.default_rng(seed)
    level = rng.standard_normal(n) * gene_sd
    offset = rng.standard_normal((groups, n)) * group_sd
    Z = level + offset[np.arange(m) % groups] + rng.standard_normal((m, n)) * noise_sd
    X = np.exp(Z)
    X[rng.random((m, n)) < zero_frac] = 0.0
    return X.astype(np.float32)


def permutations(B: int, n: int, seed: int) -> np.ndarray:
    """B independent uniform permutations of 0..n-1 (rows, uint16) for the
    permutation test."""
    rng = np.random.default_rng(seed)
    return np.stack([rng.permutation(n) for _ in range(B)]).astype(np.uint16)


def config_matrix(cfg: int, seed: int | None = None) -> np.ndarray:
    """The single-matrix workloads 1-3."""
    seed = DEFAULT_SEEDS[cfg] if seed is None else seed
    m, n = SHAPES[cfg]
    if cfg == 1:
        return gaussian_rounded(m, n, seed)
    if cfg == 2:
        return latent_factor(m, n, seed)
    if cfg == 3:
        return lognormal_blocks(m, n, seed)
    raise ValueError(cfg)


def batch_shapes(count: int = 256, seed: int = 4, m_range=(32, 2048),
                 n_range=(64, 4096)) -> list[tuple[int, int]]:
    """Uneven (m, n) per matrix, m and n uniform on the inclusive ranges."""
    rng = np.random.default_rng(seed)
    ms = rng.integers(m_range[0], m_range[1] + 1, size=count)
    ns = rng.integers(n_range[0], n_range[1] + 1, size=count)
    return [(int(a), int(b)) for a, b in zip(ms, ns)]


def batch_matrix(shape: tuple[int, int], seed: int, index: int,
                 round_frac: float = 0.2, step: float = 0.25) -> np.ndarray:
    """One matrix of the uneven batch: N(0,1), a Bernoulli(``round_frac``)
    subset of entries rounded to multiples of ``step``."""
    rng = np.random.default_rng([seed, index])
    m, n = shape
    X = rng.standard_normal((m, n))
    mask = rng.random((m, n)) < round_frac
    X[mask] = np.round(X[mask] / step) * step
    return X.astype(np.float32)


def batch(count: int = 256, seed: int = 4, m_range=(32, 2048), n_range=(64, 4096),
          round_frac: float = 0.2):
    """The uneven batch: a list of ``count`` float32 matrices."""
    shapes = batch_shapes(count, seed, m_range, n_range)
    return [batch_matrix(s, seed, i, round_frac) for i, s in enumerate(shapes)]


@dataclass
class Database:
    X: np.ndarray        # (m, n) float32 log-normal subject rows
    Z: np.ndarray        # (m, n) float64 latent normals of the rows


def database(m: int = 20000, n: int = 800, seed: int = 5) -> Database:
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((m, n))
    return Database(X=np.exp(Z).astype(np.float32), Z=Z)


def queries(db: Database, count: int, seed: int, noise_sd: float = 0.5,
            hit_frac: float = 0.5) -> np.ndarray:
    """Query rows: ``hit_frac`` of them are a random database row's latent
    normal plus N(0, sd^2) noise, then exp (so true co-expressed hits exist);
    the rest are fresh log-normal rows."""
    rng = np.random.default_rng(seed)
    m, n = db.Z.shape
    out = np.empty((count, n), np.float32)
    for i in range(count):
        if rng.random() < hit_frac:
            j = int(rng.integers(0, m))
            z = db.Z[j] + noise_sd * rng.standard_normal(n)
        else:
            z = rng.standard_normal(n)
        out[i] = np.exp(z).astype(np.float32)
    return out


def poisson_requests(count: int, rate: float, seed: int, nq_range=(1, 64)):
    """Arrival times (s) of a Poisson stream at ``rate`` requests/s and the
    number of query rows of each request (uniform on the inclusive range)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    sizes = rng.integers(nq_range[0], nq_range[1] + 1, size=count)
    return arrivals, sizes
